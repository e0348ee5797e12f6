// Leaf products of the AtA plan on MFMA: SYRK leaves (lower(X^T X), the
// paper's ?syrk base case, Sec. 3.1) and GEMM leaves (X^T Y, the ?gemm base
// case of Strassen), all leaves of a plan in one grouped launch.
//
// Each workgroup (4 waves) computes one 128 x 128 output tile.  The
// contraction runs over rows of A (the K loop): a 16-row slab of X's and Y's
// tile columns is staged through LDS (double-buffered, one barrier per slab),
// each wave owns a 64 x 64 sub-tile.  Rows of A are contiguous along the
// output dimensions, so global loads are 16-byte vectors along columns and
// the slab is stored k-major in LDS, which is exactly the operand order the
// FP32 and FP64 MFMAs read (one element per lane per operand).
//
// MFMA lane layouts used (checked on gfx950):
//   v_mfma_f32_32x32x2f32:  A lane l -> (i = l%32, k = l/32), B likewise with
//     j; result register v of lane l -> (i = 8(v/4) + 4(l/32) + v%4, j = l%32)
//   v_mfma_f64_16x16x4f64:  A lane l -> (i = l%16, k = l/16), B likewise;
//     result register v of lane l -> (i = 4v + l/16, j = l%16)
//   v_mfma_f32_32x32x16_bf16: A lane l element e -> (i = l%32, k = 8(l/32) + e),
//     B likewise; result layout as v_mfma_f32_32x32x2f32
//
// Split-BF16 (three products): each FP32 operand element a is split (by the
// packing pass) into hi = bf16_RNE(a) and lo = bf16_RNE(a - hi) (a - hi is
// exact in FP32); the tile accumulates Xh^T Yh + Xh^T Yl + Xl^T Yh in FP32.
// The BF16 MFMA wants each lane's eight consecutive k values of one row i
// together, so the slab is stored i-major in LDS ([i][k], k contiguous).
#include "kernels_common.hpp"
#include "launch.hpp"

namespace ata {

namespace {

constexpr int BK = 16;          // rows of A per K step
constexpr int PAD32 = 4;        // LDS row padding (floats)
constexpr int PAD64 = 2;        // LDS row padding (doubles)
constexpr int LD32 = TILE_M + PAD32;
constexpr int LD64 = TILE_M + PAD64;
constexpr size_t LDS32_BYTES = 2 * 2 * BK * LD32 * sizeof(float);
constexpr size_t LDS64_BYTES = 2 * 2 * BK * LD64 * sizeof(double);
constexpr size_t LEAF_LDS_BYTES = LDS64_BYTES > LDS32_BYTES ? LDS64_BYTES : LDS32_BYTES;
constexpr int BKB = 32;         // rows of A per K step, split-BF16 path
constexpr int LDB = 40;         // bf16 per LDS row: 32 k values + 8 pad (80-byte stride)
constexpr size_t LDSB_BYTES = 2 * 4 * TILE_M * LDB * 2;   // 2 stages x {Xh, Xl, Yh, Yl}
// Kernel variant of the FP64 fallback: FP32 inputs, FP64 MFMA, FP32 output.
constexpr int MODE_FALLBACK = 100;
constexpr size_t lds_bytes(int mode) {
    return mode == MODE_BF16X3 ? LDSB_BYTES : mode == MODE_F32 ? LDS32_BYTES : LDS64_BYTES;
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

struct LeafArgs {
    const LeafDesc* tasks;
    int ntasks;
    int chunk;
    int64_t ntiles;
    const void* A;
    void* C;
    void* arena;
    const uint8_t* flags;
};

__device__ __forceinline__ int find_leaf(const LeafDesc* t, int n, int64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (t[mid].tile_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Four consecutive elements (r, c..c+3) of a zero-padded float operand.
__device__ __forceinline__ float4 load4f(const float* p, int64_t ld, int64_t r, int64_t c,
                                         int64_t K, int64_t pc, bool vec) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < K) {
        const float* q = p + r * ld + c;
        if (vec && c + 3 < pc) {
            v = *reinterpret_cast<const float4*>(q);
        } else {
            if (c < pc) v.x = q[0];
            if (c + 1 < pc) v.y = q[1];
            if (c + 2 < pc) v.z = q[2];
            if (c + 3 < pc) v.w = q[3];
        }
    }
    return v;
}

__device__ __forceinline__ double2 load2d(const double* p, int64_t ld, int64_t r, int64_t c,
                                          int64_t K, int64_t pc, bool vec) {
    double2 v = make_double2(0.0, 0.0);
    if (r < K) {
        const double* q = p + r * ld + c;
        if (vec && c + 1 < pc) {
            v = *reinterpret_cast<const double2*>(q);
        } else {
            if (c < pc) v.x = q[0];
            if (c + 1 < pc) v.y = q[1];
        }
    }
    return v;
}

template <class T>
__device__ __forceinline__ const T* view_ptr(const View& v, const void* A, const void* arena) {
    return (v.base == BASE_A ? static_cast<const T*>(A) : static_cast<const T*>(arena)) + v.off;
}

template <class T>
__device__ __forceinline__ bool vec_ok(const T* p, int64_t ld, int width) {
    return ((reinterpret_cast<uintptr_t>(p) & 15) == 0) && (ld % width == 0);
}

// Store one accumulator element of tile (ti, tj) at tile-local (r, c).
template <class OutT>
__device__ __forceinline__ void store_elem(const LeafDesc& d, int ti, int tj, int r, int c,
                                           OutT v, OutT* C, OutT* arena) {
    const int64_t gi = (int64_t)ti * TILE_M + r, gj = (int64_t)tj * TILE_N + c;
    if (gi >= d.rows || gj >= d.cols) return;
    if (d.kind == LEAF_SYRK && gj > gi) return;
    if (d.out_kind == OUT_PACKED)
        C[packed_index(d.out_row0 + gi, d.out_col0 + gj)] = v;
    else
        arena[d.out_off + gi * d.out_ld + gj] = v;
}

// ---------------------------------------------------------------- FP32 MFMA
__device__ void tile_f32(const LeafDesc& d, const float* Xp, const float* Yp, int ti, int tj,
                         float* C, float* arena, unsigned char* smem) {
    float* Xs = reinterpret_cast<float*>(smem);          // [2][BK][LD32]
    float* Ys = Xs + 2 * BK * LD32;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int lr = t >> 5, lc = (t & 31) << 2;
    const int64_t xc = (int64_t)ti * TILE_M + lc, yc = (int64_t)tj * TILE_N + lc;
    const bool xv = vec_ok(Xp, d.X.ld, 4), yv = vec_ok(Yp, d.Y.ld, 4);
    const int64_t K = d.K;
    const int64_t nk = (K + BK - 1) / BK;

    v16f acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    float4 rx0, rx1, ry0, ry1;
    auto gload = [&](int64_t k0) {
        rx0 = load4f(Xp, d.X.ld, k0 + lr, xc, K, d.X.pcols, xv);
        rx1 = load4f(Xp, d.X.ld, k0 + lr + 8, xc, K, d.X.pcols, xv);
        ry0 = load4f(Yp, d.Y.ld, k0 + lr, yc, K, d.Y.pcols, yv);
        ry1 = load4f(Yp, d.Y.ld, k0 + lr + 8, yc, K, d.Y.pcols, yv);
    };
    auto sstore = [&](int buf) {
        float* xs = Xs + buf * BK * LD32;
        float* ys = Ys + buf * BK * LD32;
        *reinterpret_cast<float4*>(xs + lr * LD32 + lc) = rx0;
        *reinterpret_cast<float4*>(xs + (lr + 8) * LD32 + lc) = rx1;
        *reinterpret_cast<float4*>(ys + lr * LD32 + lc) = ry0;
        *reinterpret_cast<float4*>(ys + (lr + 8) * LD32 + lc) = ry1;
    };

    if (nk > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int ko = lane >> 5, io = lane & 31;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const float* xs = Xs + cur * BK * LD32 + wm * 64 + io;
        const float* ys = Ys + cur * BK * LD32 + wn * 64 + io;
#pragma unroll
        for (int kk = 0; kk < BK / 2; ++kk) {
            const int row = (2 * kk + ko) * LD32;
            const float a0 = xs[row], a1 = xs[row + 32];
            const float b0 = ys[row], b1 = ys[row + 32];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 16; ++v) {
                const int r = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int c = wn * 64 + b * 32 + (lane & 31);
                store_elem<float>(d, ti, tj, r, c, acc[a][b][v], C, arena);
            }
}

// ------------------------------------------------------------ split-BF16 x3
// Operands come pre-split and packed (see Packed): each 16-byte chunk is the
// eight consecutive k values of one column, so a slab load is a plain
// 16-byte load per chunk and an LDS store at [column][k]; no conversion work
// is left in the K loop.  Loads go through buffer resources bounded by the
// packed array, so reads past its end return zero instead of faulting.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t packed_rsrc(const float* arena, const Packed& P, bool lo) {
    const float* b = arena + P.off + (lo ? P.lo_delta : 0);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(b), (short)0,
                                             (int)(uint32_t)((P.end - P.off) * 4), 0x00020000);
}

__device__ void tile_bf16x3(const LeafDesc& d, const float* arena_in, int ti, int tj,
                            float* C, float* arena, unsigned char* smem) {
    unsigned short* lds = reinterpret_cast<unsigned short*>(smem);
    // stage s, array a (0 = Xh, 1 = Xl, 2 = Yh, 3 = Yl): TILE_M rows of LDB bf16
    auto arr = [&](int s, int a) { return lds + (s * 4 + a) * TILE_M * LDB; };
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int c = t & 127, side = t >> 7;          // chunk column; 0 = X, 1 = Y (wave-uniform)
    const Packed& P = side ? d.PY : d.PX;
    const __amdgpu_buffer_rsrc_t rh = packed_rsrc(arena_in, P, false), rl = packed_rsrc(arena_in, P, true);
    const uint32_t colb = (uint32_t)(((side ? tj : ti) * TILE_M + c) * 16);
    const uint32_t gsb = (uint32_t)(P.gstride * 4);
    const int64_t K = d.K;
    const int64_t nk = (K + BKB - 1) / BKB;

    v16f acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    v4u rh4[4], rl4[4];
    auto gload = [&](int64_t kt) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int64_t grow = kt * 4 + g;
            if (grow * 8 < K) {
                const uint32_t off = (uint32_t)grow * gsb + colb;
                rh4[g] = __builtin_amdgcn_raw_buffer_load_b128(rh, (int)off, 0, 0);
                rl4[g] = __builtin_amdgcn_raw_buffer_load_b128(rl, (int)off, 0, 0);
            } else {
                rh4[g] = v4u{0u, 0u, 0u, 0u};
                rl4[g] = v4u{0u, 0u, 0u, 0u};
            }
        }
    };
    auto sstore = [&](int s) {
        unsigned short* hi = arr(s, 2 * side) + c * LDB;
        unsigned short* lo = arr(s, 2 * side + 1) + c * LDB;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            *reinterpret_cast<v4u*>(hi + 8 * g) = rh4[g];
            *reinterpret_cast<v4u*>(lo + 8 * g) = rl4[g];
        }
    };

    if (nk > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int io = lane & 31, ko = 8 * (lane >> 5);
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload(kt + 1);
        const unsigned short* xh = arr(cur, 0) + (wm * 64 + io) * LDB + ko;
        const unsigned short* xl = arr(cur, 1) + (wm * 64 + io) * LDB + ko;
        const unsigned short* yh = arr(cur, 2) + (wn * 64 + io) * LDB + ko;
        const unsigned short* yl = arr(cur, 3) + (wn * 64 + io) * LDB + ko;
#pragma unroll
        for (int ks = 0; ks < BKB / 16; ++ks) {
            v8bf ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                ah[s2] = *reinterpret_cast<const v8bf*>(xh + s2 * 32 * LDB + ks * 16);
                al[s2] = *reinterpret_cast<const v8bf*>(xl + s2 * 32 * LDB + ks * 16);
                bh[s2] = *reinterpret_cast<const v8bf*>(yh + s2 * 32 * LDB + ks * 16);
                bl[s2] = *reinterpret_cast<const v8bf*>(yl + s2 * 32 * LDB + ks * 16);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 16; ++v) {
                const int r = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int cc = wn * 64 + b * 32 + (lane & 31);
                store_elem<float>(d, ti, tj, r, cc, acc[a][b][v], C, arena);
            }
}

// ---------------------------------------------------------------- FP64 MFMA
// InT = double (FP64 mode) or float (FP64 fallback of the FP32 family: the
// inputs are promoted exactly, the result is rounded to OutT on store).
template <class InT, class OutT>
__device__ void tile_f64(const LeafDesc& d, const InT* Xp, const InT* Yp, int ti, int tj,
                         OutT* C, OutT* arena, unsigned char* smem) {
    double* Xs = reinterpret_cast<double*>(smem);        // [2][BK][LD64]
    double* Ys = Xs + 2 * BK * LD64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int64_t K = d.K;
    const int64_t nk = (K + BK - 1) / BK;

    v4d acc[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;

    // staging registers: 8 elements of X and 8 of Y per thread per slab
    double rx[8], ry[8];
    int lr, lc, rstep;
    if constexpr (sizeof(InT) == 8) { lr = t >> 6; lc = (t & 63) << 1; rstep = 4; }
    else { lr = t >> 5; lc = (t & 31) << 2; rstep = 8; }
    const int64_t xc = (int64_t)ti * TILE_M + lc, yc = (int64_t)tj * TILE_N + lc;
    const bool xv = vec_ok(Xp, d.X.ld, 16 / (int)sizeof(InT));
    const bool yv = vec_ok(Yp, d.Y.ld, 16 / (int)sizeof(InT));

    auto gload = [&](int64_t k0) {
        if constexpr (sizeof(InT) == 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 x = load2d(Xp, d.X.ld, k0 + lr + q * rstep, xc, K, d.X.pcols, xv);
                const double2 y = load2d(Yp, d.Y.ld, k0 + lr + q * rstep, yc, K, d.Y.pcols, yv);
                rx[2 * q] = x.x; rx[2 * q + 1] = x.y;
                ry[2 * q] = y.x; ry[2 * q + 1] = y.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float4 x = load4f(Xp, d.X.ld, k0 + lr + q * rstep, xc, K, d.X.pcols, xv);
                const float4 y = load4f(Yp, d.Y.ld, k0 + lr + q * rstep, yc, K, d.Y.pcols, yv);
                rx[4 * q] = x.x; rx[4 * q + 1] = x.y; rx[4 * q + 2] = x.z; rx[4 * q + 3] = x.w;
                ry[4 * q] = y.x; ry[4 * q + 1] = y.y; ry[4 * q + 2] = y.z; ry[4 * q + 3] = y.w;
            }
        }
    };
    auto sstore = [&](int buf) {
        double* xs = Xs + buf * BK * LD64;
        double* ys = Ys + buf * BK * LD64;
        if constexpr (sizeof(InT) == 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *reinterpret_cast<double2*>(xs + (lr + q * rstep) * LD64 + lc) = make_double2(rx[2 * q], rx[2 * q + 1]);
                *reinterpret_cast<double2*>(ys + (lr + q * rstep) * LD64 + lc) = make_double2(ry[2 * q], ry[2 * q + 1]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double* xr = xs + (lr + q * rstep) * LD64 + lc;
                double* yr = ys + (lr + q * rstep) * LD64 + lc;
                *reinterpret_cast<double2*>(xr) = make_double2(rx[4 * q], rx[4 * q + 1]);
                *reinterpret_cast<double2*>(xr + 2) = make_double2(rx[4 * q + 2], rx[4 * q + 3]);
                *reinterpret_cast<double2*>(yr) = make_double2(ry[4 * q], ry[4 * q + 1]);
                *reinterpret_cast<double2*>(yr + 2) = make_double2(ry[4 * q + 2], ry[4 * q + 3]);
            }
        }
    };

    if (nk > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int ko = lane >> 4, io = lane & 15;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const double* xs = Xs + cur * BK * LD64 + wm * 64 + io;
        const double* ys = Ys + cur * BK * LD64 + wn * 64 + io;
#pragma unroll
        for (int kq = 0; kq < BK / 4; ++kq) {
            const int row = (4 * kq + ko) * LD64;
            double a[4], b[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) { a[s] = xs[row + 16 * s]; b[s] = ys[row + 16 * s]; }
#pragma unroll
            for (int sa = 0; sa < 4; ++sa)
#pragma unroll
                for (int sb = 0; sb < 4; ++sb)
                    acc[sa][sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[sa], b[sb], acc[sa][sb], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int v = 0; v < 4; ++v) {
                const int r = wm * 64 + a * 16 + 4 * v + (lane >> 4);
                const int c = wn * 64 + b * 16 + (lane & 15);
                store_elem<OutT>(d, ti, tj, r, c, (OutT)acc[a][b][v], C, arena);
            }
}

template <int MODE>
__global__ __launch_bounds__(LEAF_THREADS) void leaf_kernel(LeafArgs args) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[lds_bytes(MODE)];
    const int64_t bid = xcd_remap(blockIdx.x, args.ntiles, args.chunk);
    const LeafDesc& d = args.tasks[find_leaf(args.tasks, args.ntasks, bid)];
    if (d.pred_node >= 0 && (int32_t)args.flags[d.pred_node] != d.pred_value) return;
    const int64_t q = bid - d.tile_begin;
    int ti, tj;
    if (d.kind == LEAF_SYRK) {
        tri_tile(q, ti, tj);
    } else {
        ti = (int)(q / d.tiles_n);
        tj = (int)(q % d.tiles_n);
    }
    // SYRK leaves under the spread check run in exactly one of the two
    // launches: the FP64 fallback kernel when their node is flagged, the
    // mode's own kernel otherwise.
    const bool flagged = d.fb_node >= 0 && args.flags[d.fb_node];
    if constexpr (MODE == MODE_F64) {
        tile_f64<double, double>(d, view_ptr<double>(d.X, args.A, args.arena),
                                 view_ptr<double>(d.Y, args.A, args.arena), ti, tj,
                                 static_cast<double*>(args.C), static_cast<double*>(args.arena), smem);
    } else if constexpr (MODE == MODE_FALLBACK) {
        if (!flagged) return;
        tile_f64<float, float>(d, view_ptr<float>(d.X, args.A, args.arena),
                               view_ptr<float>(d.Y, args.A, args.arena), ti, tj,
                               static_cast<float*>(args.C), static_cast<float*>(args.arena), smem);
    } else if constexpr (MODE == MODE_BF16X3) {
        if (flagged) return;
        tile_bf16x3(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(args.C),
                    static_cast<float*>(args.arena), smem);
    } else {
        if (flagged) return;
        tile_f32(d, view_ptr<float>(d.X, args.A, args.arena), view_ptr<float>(d.Y, args.A, args.arena),
                 ti, tj, static_cast<float*>(args.C), static_cast<float*>(args.arena), smem);
    }
}

}  // namespace

hipError_t launch_leaves(int32_t mode, const LeafDesc* d_tasks, int ntasks, int64_t ntiles,
                         const void* A, void* C, void* arena, const uint8_t* flags, int chunk,
                         hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    LeafArgs a{d_tasks, ntasks, chunk, ntiles, A, C, arena, flags};
    dim3 grid((unsigned)ntiles), block(LEAF_THREADS);
    switch (mode) {
        case MODE_F64: hipLaunchKernelGGL(leaf_kernel<MODE_F64>, grid, block, 0, stream, a); break;
        case MODE_F32: hipLaunchKernelGGL(leaf_kernel<MODE_F32>, grid, block, 0, stream, a); break;
        case MODE_BF16X3: hipLaunchKernelGGL(leaf_kernel<MODE_BF16X3>, grid, block, 0, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fallback_leaves(const LeafDesc* d_tasks, int ntasks, int64_t ntiles, const void* A,
                                  void* C, void* arena, const uint8_t* flags, int chunk,
                                  hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    LeafArgs a{d_tasks, ntasks, chunk, ntiles, A, C, arena, flags};
    hipLaunchKernelGGL(leaf_kernel<MODE_FALLBACK>, dim3((unsigned)ntiles), dim3(LEAF_THREADS), 0, stream, a);
    return hipGetLastError();
}

}  // namespace ata
