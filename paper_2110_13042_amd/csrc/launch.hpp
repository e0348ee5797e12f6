// Host-side launchers of the library's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "plan.hpp"

namespace ata {

// Device arrays of a batch: A and C pointer of problem i at A[i], C[i]; the
// persistent leaf launch's queue head and grid size.
struct BatchPtrs {
    const void* const* A;
    void* const* C;
    unsigned long long* counter;   // eight queue heads; null: one workgroup per tile
    int64_t persistent_blocks;
};

// Resident workgroups per CU of the mode's persistent leaf kernel (occupancy query).
int leaf_blocks_per_cu(int32_t mode, int32_t tile_cfg);

// All leaf products of a plan (one grouped launch, one workgroup per tile).
// tile_cfg selects the output tile of the split-BF16 kernel (0: 128 x 128,
// 1: 256 x 128, 2: 256 x 256); the other modes have one tile shape.  Tile
// order: every window of 8 x chunk consecutive tiles gives each XCD chunk
// consecutive tiles; GEMM leaves number their tiles in bands of `band` tile
// rows, column by column.
// tile_base: the launch covers tiles [tile_base, tile_base + ntiles) of the
// plan's tile order (a plan's leaves may be split over two launches).
hipError_t launch_leaves(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks,
                         int64_t ntiles, const void* A, void* C, void* arena, const uint8_t* flags,
                         int chunk, int band, hipStream_t stream, const BatchPtrs* bp = nullptr,
                         const void* B = nullptr, int64_t tile_base = 0);

// The leaf launch of a plan with Strassen combines in the leaf epilogues
// (Plan::fuse_combine): the same kernels, built to add a leaf's product into
// its one or two node quadrants (LeafDesc::nq); leaves with nq = 0 store as
// usual.  One call per launch round.
hipError_t launch_leaves_epi(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks, int64_t ntiles,
                             const void* A, void* C, void* arena, const uint8_t* flags, int chunk, int band,
                             hipStream_t stream, const BatchPtrs* bp = nullptr, const void* B = nullptr,
                             int64_t tile_base = 0);

// FP64 fallback of flagged SYRK leaves (FP32 inputs and output); the tasks
// are the plan's fallback-capable SYRK leaves, unflagged ones exit at once.
hipError_t launch_fallback_leaves(const LeafDesc* d_tasks, int ntasks, int64_t ntiles, const void* A,
                                  void* C, void* arena, const uint8_t* flags, int chunk, int band,
                                  hipStream_t stream, const BatchPtrs* bp = nullptr);

// One Strassen level of pre-sums (S1..S5 / T1..T5 for every node of the level).
hipError_t launch_presum(int32_t mode, const PresumDesc* d_tasks, int ntasks, int64_t items,
                         const void* A, void* arena, const uint8_t* flags, hipStream_t stream,
                         const BatchPtrs* bp = nullptr, const void* B = nullptr);

// Split-BF16 packing of the leaf operands (one launch for the whole plan).
hipError_t launch_pack(const PackDesc* d_tasks, int ntasks, int64_t items, const void* A,
                       void* arena, const uint8_t* flags, hipStream_t stream,
                       const BatchPtrs* bp = nullptr, const void* B = nullptr);

// FP8 quantisation of the leaf operands (one workgroup per 128 x 128 block).
hipError_t launch_quant8(const Pack8Desc* d_tasks, int ntasks, int64_t blocks, const void* A,
                         void* arena, const uint8_t* flags, hipStream_t stream,
                         const BatchPtrs* bp = nullptr, const void* B = nullptr, double* partial = nullptr);

// Partial sums of the split-K leaves (after both leaf launches).
hipError_t launch_reduce(int32_t mode, const ReduceDesc* d_tasks, int ntasks, int64_t items, void* C,
                         void* arena, const uint8_t* flags, hipStream_t stream,
                         const BatchPtrs* bp = nullptr);

// c = alpha t + beta c over len elements (beta = 0: c is not read).
hipError_t launch_axpby(int32_t mode, const void* t, void* c, int64_t len, double alpha, double beta,
                        hipStream_t stream);
// At (n x m dense) = transpose of A (m x n, row stride lda).
hipError_t launch_transpose(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda, void* At,
                            hipStream_t stream);
// Full symmetric n x n matrix (row stride ldf) from packed lower storage.
hipError_t launch_unpack(int32_t mode, const void* Cp, int64_t n, void* F, int64_t ldf, hipStream_t stream);

// Column equilibration: Ap (m x n dense) = A diag(2^-e) with e_j the binary
// exponent of column j's norm (from nu = squared norms); and packed
// C_ij *= 2^(e_i + e_j) afterwards.
hipError_t launch_eq_scale(const float* A, int64_t m, int64_t n, int64_t lda, const double* nu, float* Ap,
                           int* e, hipStream_t stream);
hipError_t launch_eq_unscale(float* Cp, int64_t n, const int* e, hipStream_t stream);

// Bounded workspace: single pre-sums (Sum2Desc) and the adding of one
// product into its quadrants (AccumDesc).
hipError_t launch_sum2(int32_t mode, const Sum2Desc* d_tasks, int ntasks, int64_t items, const void* A,
                       void* arena, const uint8_t* flags, hipStream_t stream);
hipError_t launch_accum(int32_t mode, const AccumDesc* d_tasks, int ntasks, int64_t items, void* C, void* arena,
                        const uint8_t* flags, hipStream_t stream);

// One height of Strassen combines (seven products -> four quadrants).
hipError_t launch_combine(int32_t mode, const CombineDesc* d_tasks, int ntasks, int64_t items,
                          void* C, void* arena, const uint8_t* flags, hipStream_t stream,
                          const BatchPtrs* bp = nullptr);

// Squared column norms (FP64) of every problem of the task lists (pass 1
// over row chunks into `partial`, pass 2 sums each column's chunks in order
// into `nu`).  A: the matrix when Aptrs is null, else Aptrs[prob].
hipError_t launch_colnorms(const ColDesc* d_pass1, int n1, int64_t items1, const ColDesc* d_pass2,
                           int n2, int64_t items2, const float* A, const void* const* Aptrs,
                           double* partial, double* nu, hipStream_t stream, void* arena = nullptr,
                           bool pack = false);

// flags[i] = spread of nu over node i's columns > tau^2 (1/0); count in *count.
hipError_t launch_flags(const double* nu, const NodeDesc* d_nodes, int nnodes, double tau2,
                        uint8_t* flags, hipStream_t stream);

// Freivalds residual ||C x - A^T (A x)|| / (||A||_F^2 ||x||), x_j = +-1 from
// SplitMix64(seed, j).  `work` must hold residual_work_elems(m, n) doubles.
int64_t residual_work_elems(int64_t m, int64_t n);

// Sampled-column check: FP64 columns (A^T A)[:, cols[k]] against the packed
// C.  d_cols: device array of `count` column indices; `work` must hold
// column_check_work_elems(m, n, count) doubles; on return the last
// 2 * ceil(n / 64) * ceil(count / 16) of them hold per-workgroup
// (sum (C - ref)^2, sum ref^2) pairs.
int64_t column_check_work_elems(int64_t m, int64_t n, int64_t count);
hipError_t launch_column_check(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda, const void* C,
                               const int64_t* d_cols, int64_t count, double* work, hipStream_t stream);
hipError_t launch_residual(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda,
                           const void* C, uint64_t seed, double* work, double* out,
                           hipStream_t stream);

}  // namespace ata
