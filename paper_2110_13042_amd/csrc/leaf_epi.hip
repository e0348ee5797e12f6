// Leaf launches of plans with Strassen combines in the leaf epilogues: the
// same kernels as leaf.hip, built so that a leaf adds its product into one
// or two quadrants of its node's target (a translation unit of its own, so
// the two builds compile side by side).
#include "leaf_kernels.hpp"

namespace ata {

hipError_t launch_leaves_epi(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks, int64_t ntiles,
                             const void* A, void* C, void* arena, const uint8_t* flags, int chunk, int band,
                             hipStream_t stream, const BatchPtrs* bp, const void* B, int64_t tile_base) {
    return launch_leaves_t<true>(mode, tile_cfg, d_tasks, ntasks, ntiles, A, C, arena, flags, chunk, band, stream,
                                 bp, B, tile_base);
}

}  // namespace ata
