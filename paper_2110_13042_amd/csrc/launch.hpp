// Host-side launchers of the library's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "plan.hpp"

namespace ata {

// All leaf products of a plan (one grouped launch, one workgroup per tile).
// tile_cfg selects the output tile of the split-BF16 kernel (0: 128 x 128,
// 1: 256 x 128); the other modes have one tile shape.
hipError_t launch_leaves(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks,
                         int64_t ntiles, const void* A, void* C, void* arena, const uint8_t* flags,
                         int chunk, hipStream_t stream);

// FP64 fallback of flagged SYRK leaves (FP32 inputs and output); the tasks
// are the plan's fallback-capable SYRK leaves, unflagged ones exit at once.
hipError_t launch_fallback_leaves(const LeafDesc* d_tasks, int ntasks, int64_t ntiles, const void* A,
                                  void* C, void* arena, const uint8_t* flags, int chunk,
                                  hipStream_t stream);

// One Strassen level of pre-sums (S1..S5 / T1..T5 for every node of the level).
hipError_t launch_presum(int32_t mode, const PresumDesc* d_tasks, int ntasks, int64_t items,
                         const void* A, void* arena, const uint8_t* flags, hipStream_t stream);

// Split-BF16 packing of the leaf operands (one launch for the whole plan).
hipError_t launch_pack(const PackDesc* d_tasks, int ntasks, int64_t items, const void* A,
                       void* arena, const uint8_t* flags, hipStream_t stream);

// One height of Strassen combines (seven products -> four quadrants).
hipError_t launch_combine(int32_t mode, const CombineDesc* d_tasks, int ntasks, int64_t items,
                          void* C, void* arena, const uint8_t* flags, hipStream_t stream);

// Squared column norms (FP64) of a float matrix, deterministic two-pass sum:
// partial[chunk][j] over row chunks, then nu[j] = sum over chunks in order.
hipError_t launch_colnorms(const float* A, int64_t m, int64_t n, int64_t lda, double* partial,
                           int64_t nchunks, double* nu, hipStream_t stream);
int64_t colnorm_chunks(int64_t m, int64_t n);

// flags[i] = spread of nu over node i's columns > tau^2 (1/0); count in *count.
hipError_t launch_flags(const double* nu, const NodeDesc* d_nodes, int nnodes, double tau2,
                        uint8_t* flags, hipStream_t stream);

// Freivalds residual ||C x - A^T (A x)|| / (||A||_F^2 ||x||), x_j = +-1 from
// SplitMix64(seed, j).  `work` must hold residual_work_elems(m, n) doubles.
int64_t residual_work_elems(int64_t m, int64_t n);
hipError_t launch_residual(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda,
                           const void* C, uint64_t seed, double* work, double* out,
                           hipStream_t stream);

}  // namespace ata
