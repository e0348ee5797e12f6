// Device-side helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "plan.hpp"

namespace ata {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int LEAF_THREADS = 256;

// Row-major lower packed index of (i, j), j <= i.
__device__ __forceinline__ int64_t packed_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Consecutive workgroup ids go round-robin to the 8 XCDs.  Remap so that, in
// every window of 8 * chunk ids, XCD x works on the consecutive tile range
// [x * chunk, (x + 1) * chunk) of that window: tiles that share operand
// panels then share one XCD's L2.  The last partial window keeps identity.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t total, int64_t chunk) {
    const int64_t win = 8 * chunk;
    const int64_t full = (total / win) * win;
    if (bid >= full) return bid;
    const int64_t w0 = (bid / win) * win;
    const int64_t r = bid - w0;
    return w0 + (r % 8) * chunk + r / 8;
}

template <class D>
__device__ __forceinline__ int find_task(const D* tasks, int ntasks, int64_t x) {
    // largest t with tasks[t].begin <= x (begin fields ascending)
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].elem_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Task of the calling workgroup in a streaming launch whose tasks begin at
// multiples of ITEM_BLOCK items: the lookup is the same for every lane, so it
// runs once per wave on the scalar unit instead of once per thread.
template <class D>
__device__ __forceinline__ int block_task(const D* tasks, int ntasks) {
    return find_task(tasks, ntasks, (int64_t)blockIdx.x * ITEM_BLOCK);
}
// The same for virtual block vb of a launch whose workgroups loop over blocks.
template <class D>
__device__ __forceinline__ int block_task(const D* tasks, int ntasks, int64_t vb) {
    return find_task(tasks, ntasks, vb * ITEM_BLOCK);
}

// a / b for 0 <= a, 0 < b; 32-bit division when both operands fit.
__device__ __forceinline__ int64_t udiv(int64_t a, int64_t b) {
    if (((uint64_t)a | (uint64_t)b) >> 32 == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}

}  // namespace ata
