// Leaf launches of plans whose leaves store their products: the grouped
// leaf launch, the FP64 fallback launch of flagged SYRK leaves, and the
// occupancy query of the persistent launch.  The kernels themselves are in
// leaf_kernels.hpp.
#include "leaf_kernels.hpp"

namespace ata {

hipError_t launch_leaves(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks,
                         int64_t ntiles, const void* A, void* C, void* arena, const uint8_t* flags,
                         int chunk, int band, hipStream_t stream, const BatchPtrs* bp, const void* B,
                         int64_t tile_base) {
    return launch_leaves_t<false>(mode, tile_cfg, d_tasks, ntasks, ntiles, A, C, arena, flags, chunk, band, stream,
                                  bp, B, tile_base);
}

hipError_t launch_fallback_leaves(const LeafDesc* d_tasks, int ntasks, int64_t ntiles, const void* A,
                                  void* C, void* arena, const uint8_t* flags, int chunk, int band,
                                  hipStream_t stream, const BatchPtrs* bp) {
    if (ntiles <= 0) return hipSuccess;
    LeafArgs a{d_tasks, ntasks, chunk, band, ntiles, A, C, arena, flags,
               bp ? bp->A : nullptr, bp ? bp->C : nullptr, nullptr, nullptr};
    hipLaunchKernelGGL((leaf_kernel<MODE_FALLBACK, false>), dim3((unsigned)ntiles), dim3(LEAF_THREADS), 0, stream, a);
    return hipGetLastError();
}

int leaf_blocks_per_cu(int32_t mode, int32_t tile_cfg) {
    // cached per (mode, tile): the answer depends on the compiled kernels only
    static std::atomic<int> cache[8][8];
    const bool cacheable = mode >= 0 && mode < 8 && tile_cfg >= 0 && tile_cfg < 8;
    if (cacheable) {
        const int c = cache[mode][tile_cfg].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int nb = 0;
    hipError_t e = hipSuccess;
    if (mode == MODE_BF16X3 && tile_cfg == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_BF16X3_LARGE, false>, LEAF_THREADS, 0);
    else if (mode == MODE_BF16X3 && tile_cfg == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_BF16X3_HUGE, false>, 512, 0);
    else if (mode == MODE_BF16X3 && tile_cfg == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_BF16X3_WIDE, false>, LEAF_THREADS, 0);
    else if (mode == MODE_BF16X3 && tile_cfg == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_BF16X3_WIDE8, false>, 512, 0);
    else if (mode == MODE_BF16X3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_BF16X3, false>, LEAF_THREADS, 0);
    else if (mode == MODE_F32 && tile_cfg == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_F32_WIDE, false>, LEAF_THREADS, 0);
    else if (mode == MODE_F32 && tile_cfg == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_F32_WIDE8, false>, 512, 0);
    else if (mode == MODE_FP8 && tile_cfg == 3)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_FP8_WIDE, false>, 512, 0);
    else if (mode == MODE_FP8)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_FP8, false>, LEAF_THREADS, 0);
    else if (mode == MODE_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_F32, false>, LEAF_THREADS, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, leaf_kernel_persistent<MODE_F64, false>, LEAF_THREADS, 0);
    if (e != hipSuccess || nb <= 0) return 1;
    if (cacheable) cache[mode][tile_cfg].store(nb, std::memory_order_relaxed);
    return nb;
}

}  // namespace ata
