// Leaf products of the AtA plan on MFMA: SYRK leaves (lower(X^T X), the
// paper's ?syrk base case, Sec. 3.1) and GEMM leaves (X^T Y, the ?gemm base
// case of Strassen), all leaves of a plan in one grouped launch (or in the
// five launch rounds of a plan that combines its last Strassen level in the
// leaf epilogues).  The kernels are templates on EPI: leaf.hip builds them
// with plain stores, leaf_epi.hip with the epilogue that adds a product into
// its one or two node quadrants (TileStore).
//
// The 128 x 128 engines: each workgroup (4 waves) computes one output tile.  The
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
#pragma once

#include <atomic>

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
// Kernel variant of the FP64 fallback: FP32 inputs, FP64 MFMA, FP32 output.
constexpr int MODE_FALLBACK = 100;
// Split-BF16 with the 256 x 128 and 256 x 256 tiles.
constexpr int MODE_BF16X3_LARGE = 101;
constexpr int MODE_BF16X3_HUGE = 102;
constexpr int MODE_BF16X3_WIDE = 103;
constexpr int MODE_FP8_WIDE = 104;
constexpr int MODE_F32_WIDE = 105;
constexpr int MODE_F32_WIDE8 = 106;
constexpr int MODE_BF16X3_WIDE8 = 107;
constexpr int WIDE_STAGES = 4;  // LDS ring depth of the 256 x 256 split-BF16 engines (32 KB each)
constexpr int F32W8_SK = 32;    // rows per slab of the eight-wave FP32 engine
constexpr int F32W8_ST = 2;     // its LDS stages (72 KB each)
// Geometry of the FP32 256 x 256 engine (tile_f32_wide).
namespace wide32 {
constexpr int TM = 256, TN = 256;
constexpr int SK = 16;                        // rows per slab
constexpr int RS = 288;                       // LDS row stride in floats
constexpr int HALF = SK * RS * 4;             // one operand's slab: 18 KB
constexpr int STAGE = 2 * HALF;
constexpr int STAGES = 3;                     // slabs kt .. kt + STAGES - 2 are in flight
// s_waitcnt immediate: vmcnt(v) with lgkmcnt(l) (expcnt unconstrained)
constexpr int waitcnt_imm(int v, int l) { return (v & 15) | ((v >> 4) << 14) | 0x70 | (l << 8); }
// loads a wave may still have in flight once slab kt + 1 has landed
constexpr int LATER = 32 * (STAGES - 2) < 63 ? 32 * (STAGES - 2) : 63;
}  // namespace wide32

constexpr size_t lds_bytes(int mode) {
    return mode == MODE_BF16X3 ? 2 * (2 * 128 + 2 * 128) * 24 * 2
           : mode == MODE_BF16X3_LARGE ? 2 * (2 * 256 + 2 * 128) * 24 * 2
           : mode == MODE_BF16X3_HUGE ? 2 * (2 * 256 + 2 * 256) * 24 * 2
           : mode == MODE_BF16X3_WIDE ? 2 * (2 * 256 + 2 * 256) * 24 * 2
           : mode == MODE_FP8_WIDE ? (size_t)2 * 2 * 8 * 256 * 16
           : mode == MODE_F32_WIDE ? (size_t)(wide32::STAGES * wide32::STAGE > 8 * wide32::HALF ? wide32::STAGES * wide32::STAGE : 8 * wide32::HALF)
           : mode == MODE_F32_WIDE8 ? (size_t)F32W8_ST * 2 * F32W8_SK * wide32::RS * 4
           : mode == MODE_BF16X3_WIDE8 ? (size_t)WIDE_STAGES * 4 * 2 * 256 * 16
           : mode == MODE_F32 ? LDS32_BYTES : mode == MODE_FP8 ? 2 * 2 * 128 * 144 : LDS64_BYTES;
}
constexpr int threads_for(int mode) {
    return mode == MODE_BF16X3_HUGE || mode == MODE_F32_WIDE8 || mode == MODE_BF16X3_WIDE8 || mode == MODE_FP8_WIDE
               ? 512 : LEAF_THREADS;
}
// Resident workgroups per CU the one-tile-per-workgroup kernel is compiled
// for: the 128 x 128 FP32 engine keeps four (64 VGPRs + 64 accumulators per
// lane) with its fused pre-sum loads included.
// Minimum waves per SIMD the register allocation must allow: four for the
// 128 x 128 FP32 engine, two for the FP64 engines (their 66.5 KB of LDS
// allow two workgroups per CU), so that one wave's MFMAs cover the other's
// waits.
constexpr int min_blocks_for(int mode) {
    return mode == MODE_F32 ? 4 : mode == MODE_F64 || mode == MODE_FALLBACK ? 2 : 1;
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

struct LeafArgs {
    const LeafDesc* tasks;
    int ntasks;
    int chunk;                    // consecutive tiles per XCD in each window of 8 chunks
    int band;                     // GEMM tile rows per band
    int64_t ntiles;
    const void* A;
    void* C;
    void* arena;
    const uint8_t* flags;
    const void* const* Aptrs;     // batches: A and C of problem d.prob (else A, C)
    void* const* Cptrs;
    unsigned long long* counter;  // persistent mode: eight tile queue heads (else null)
    const void* B;                // second input of a general product (else null)
    int64_t tile_base;            // first tile of this launch in the plan's tile order
};

__device__ __forceinline__ int find_leaf(const LeafDesc* t, int n, int64_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (t[mid].tile_begin <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A load through the global address space.  Operand pointers reach the
// kernels as generic pointers, and a generic (flat) load also counts against
// the LDS wait counter: every wait for an LDS read in the K loop would then
// wait for the next slab's prefetch as well, exposing its latency.
template <class T>
__device__ __forceinline__ T gld(const T* p) {
    typedef const __attribute__((address_space(1))) T GT;
    return *(GT*)p;
}
// HIP's vector structs would be copied through a generic reference: load the
// native vector type instead.
__device__ __forceinline__ float4 gld(const float4* p) {
    typedef float nv4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) nv4 GT;
    const nv4 v = *(GT*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gld(const double2* p) {
    typedef double nv2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) nv2 GT;
    const nv2 v = *(GT*)p;
    return make_double2(v.x, v.y);
}

// Four consecutive elements (r, c..c+3) of a zero-padded float operand.
__device__ __forceinline__ float4 load4f(const float* p, int64_t ld, int64_t r, int64_t c,
                                         int64_t K, int64_t pc, bool vec) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < K) {
        const float* q = p + r * ld + c;
        if (vec && c + 3 < pc) {
            v = gld(reinterpret_cast<const float4*>(q));
        } else {
            if (c < pc) v.x = gld(q);
            if (c + 1 < pc) v.y = gld(q + 1);
            if (c + 2 < pc) v.z = gld(q + 2);
            if (c + 3 < pc) v.w = gld(q + 3);
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
            v = gld(reinterpret_cast<const double2*>(q));
        } else {
            if (c < pc) v.x = gld(q);
            if (c + 1 < pc) v.y = gld(q + 1);
        }
    }
    return v;
}

// Tile coordinates of the q-th tile of a leaf.  SYRK: lower-triangular rows,
// row ti holding min(rho (ti + 1), tiles_n) tiles.  GEMM: bands of B tile
// rows, column by column inside a band.
template <int RHO>
__device__ __forceinline__ void leaf_tile(const LeafDesc& d, int64_t q, int64_t B, int& ti, int& tj) {
    const int64_t tn = d.tiles_n;
    if (d.kind == LEAF_SYRK && RHO == 1) {
        // the lower triangle in bands of B tile rows, each band column by
        // column (as the general leaves), so consecutive tiles share row and
        // column panels; band k (rows r0 = k B .. r0 + h - 1, h = min(B,
        // tn - r0)) holds r0 h rectangle tiles, then h (h + 1) / 2 triangle
        // tiles (column r0 + c has h - c of them)
        int64_t k = 0, start = 0;
        for (;;) {
            const int64_t r0 = k * B, h = tn - r0 < B ? tn - r0 : B;
            const int64_t cnt = r0 * h + h * (h + 1) / 2;
            if (q < start + cnt || r0 + h >= tn) {
                int64_t u = q - start;
                if (u < r0 * h) {
                    tj = (int)(u / h);
                    ti = (int)(r0 + u % h);
                } else {
                    u -= r0 * h;
                    int64_t c = 0;
                    while (u >= h - c) { u -= h - c; ++c; }
                    tj = (int)(r0 + c);
                    ti = (int)(r0 + c + u);
                }
                return;
            }
            start += cnt;
            ++k;
        }
    }
    if (d.kind == LEAF_SYRK) {
        const int64_t L = tn / RHO;
        const int64_t full = RHO * L * (L + 1) / 2;
        if (q < full) {
            int64_t i = (int64_t)((__builtin_sqrt(8.0 * (double)q / RHO + 1.0) - 1.0) * 0.5);
            while (i > 0 && RHO * i * (i + 1) / 2 > q) --i;
            while (RHO * (i + 1) * (i + 2) / 2 <= q) ++i;
            ti = (int)i;
            tj = (int)(q - RHO * i * (i + 1) / 2);
        } else {
            const int64_t r = q - full;
            ti = (int)(L + r / tn);
            tj = (int)(r % tn);
        }
    } else {
        const int64_t bnd = q / (B * tn);
        const int64_t rows = d.tiles_m - bnd * B < B ? d.tiles_m - bnd * B : B;
        const int64_t local = q - bnd * B * tn;
        ti = (int)(bnd * B + local % rows);
        tj = (int)(local / rows);
    }
}

template <class T>
__device__ __forceinline__ const T* view_ptr(const View& v, const void* A, const void* B, const void* arena) {
    return (v.base == BASE_A ? static_cast<const T*>(A)
            : v.base == BASE_B ? static_cast<const T*>(B) : static_cast<const T*>(arena)) + v.off;
}

template <class T>
__device__ __forceinline__ bool vec_ok(const T* p, int64_t ld, int width) {
    return ((reinterpret_cast<uintptr_t>(p) & 15) == 0) && (ld % width == 0);
}

// Contraction rows [kb, ke) of one tile and its K chunk (split-K leaves).
struct KRange {
    int64_t kb, ke;
    int split;
};

// Where one epilogue pass stores a tile's elements.  Element (i, j) of the
// leaf's product (i < rows, j < cols; SYRK: j <= i) goes to base + i * ld +
// j, or to base + packed_index(row0 + i, col0 + j) for the packed C; the
// pass stores sign * v, or adds it to what is there (accum).
template <class OutT>
struct Dest {
    OutT* base;
    int64_t ld, row0, col0;
    int64_t rows, cols;
    OutT sign;
    int32_t packed, syrk, accum;
};

// Epilogue passes of a leaf: one, or one per quadrant when the leaf adds its
// product into a Strassen node's quadrants (the combine in the epilogue).
__device__ __forceinline__ int store_passes(const LeafDesc& d) {
    return d.ksplit > 1 || d.nq <= 0 ? 1 : d.nq;
}

// Pass `pass` of a leaf: its K chunk's partial sums (split leaf), its
// target, or quadrant d.quad[pass] of the node's target (quadrant q starts
// at row q >= 2 ? qn1 : 0 and column q odd ? qk1 : 0; the first contribution
// to a quadrant overwrites it, the later ones add or subtract, the combine's
// own IEEE operations in the combine's order).
template <class OutT>
__device__ __forceinline__ Dest<OutT> make_dest(const LeafDesc& d, int pass, int split, OutT* C, OutT* arena) {
    Dest<OutT> o{};
    o.rows = d.rows;
    o.cols = d.cols;
    o.sign = (OutT)1;
    o.syrk = d.kind == LEAF_SYRK;
    if (d.ksplit > 1) {
        o.base = arena + d.part_off + (int64_t)split * d.rows * d.cols;
        o.ld = d.cols;
        return o;
    }
    int64_t r0 = 0, c0 = 0;
    if (d.nq > 0) {
        const int q = d.quad[pass];
        if (q < 2) o.rows = d.qn1;
        else r0 = d.qn1;
        if ((q & 1) == 0) o.cols = d.qk1;
        else c0 = d.qk1;
        o.sign = d.qsign[pass] < 0 ? (OutT)-1 : (OutT)1;
        o.accum = d.qfirst[pass] ? 0 : 1;
        o.syrk = 0;
    }
    if (d.out_kind == OUT_PACKED) {
        o.base = C;
        o.packed = 1;
        o.row0 = d.out_row0 + r0;
        o.col0 = d.out_col0 + c0;
    } else if (d.out_kind == OUT_CDENSE) {
        o.base = C + (d.out_row0 + r0) * d.out_ld + d.out_col0 + c0;
        o.ld = d.out_ld;
    } else {
        o.base = arena + d.out_off + r0 * d.out_ld + c0;
        o.ld = d.out_ld;
    }
    return o;
}

// Store product element (gi, gj) at one destination.
template <class OutT>
__device__ __forceinline__ void store_at(const Dest<OutT>& o, int64_t gi, int64_t gj, OutT v) {
    if (gi >= o.rows || gj >= o.cols) return;
    if (o.syrk && gj > gi) return;
    OutT* p = o.packed ? o.base + packed_index(o.row0 + gi, o.col0 + gj) : o.base + gi * o.ld + gj;
    const OutT x = o.sign * v;
    *p = o.accum ? *p + x : x;
}

// The epilogue stores of one tile, a row at a time: row(ti, r) takes tile
// row r of tile (ti, .) once, put(row, tj, c, v) stores its accumulator
// element in column c of tile (., tj).  Kernels built without combines in the
// epilogue (EPI false) store into the leaf's target or its K chunk's partial
// sums: the destination's base, row stride and form (packed or strided) are
// fixed per tile, so a row costs one address and one column limit and an
// element a compare and a store.  The others send each element to one or two
// destinations (make_dest).
template <bool EPI, class OutT, int TM, int TN>
struct TileStore;

template <class OutT, int TM, int TN>
struct TileStore<false, OutT, TM, TN> {
    struct Row {
        OutT* p;          // element (gi, 0) of the leaf's output
        int64_t lim;      // columns gj < lim are stored (0 past the leaf's rows)
    };
    OutT* base;
    int64_t ld, row0, rows, cols;
    bool packed, syrk;
    __device__ __forceinline__ TileStore(const LeafDesc& d, int split, OutT* C, OutT* arena) {
        rows = d.rows;
        cols = d.cols;
        syrk = d.kind == LEAF_SYRK;
        packed = false;
        row0 = 0;
        if (d.ksplit > 1) {
            base = arena + d.part_off + (int64_t)split * d.rows * d.cols;
            ld = d.cols;
        } else if (d.out_kind == OUT_CDENSE) {
            base = C + d.out_row0 * d.out_ld + d.out_col0;
            ld = d.out_ld;
        } else if (d.out_kind == OUT_PACKED) {
            base = C + d.out_col0;        // row i of C starts at packed_index(i, 0)
            ld = 0;
            row0 = d.out_row0;
            packed = true;
        } else {
            base = arena + d.out_off;
            ld = d.out_ld;
        }
    }
    __device__ __forceinline__ Row row(int ti, int r) const {
        const int64_t gi = (int64_t)ti * TM + r;
        const int64_t lim = gi >= rows ? 0 : syrk && gi + 1 < cols ? gi + 1 : cols;
        const int64_t off = packed ? packed_index(row0 + gi, 0) : gi * ld;
        return Row{base + off, lim};
    }
    __device__ __forceinline__ void put(const Row& w, int tj, int c, OutT v) const {
        const int64_t gj = (int64_t)tj * TN + c;
        // C and the arena are device memory: a global store, not a flat one
        if (gj < w.lim) *(__attribute__((address_space(1))) OutT*)(w.p + gj) = v;
    }
};

template <class OutT, int TM, int TN>
struct TileStore<true, OutT, TM, TN> {
    struct Row {
        int64_t gi;
    };
    Dest<OutT> d0, d1;
    bool second;
    __device__ __forceinline__ TileStore(const LeafDesc& d, int split, OutT* C, OutT* arena)
        : d0(make_dest<OutT>(d, 0, split, C, arena)), d1(make_dest<OutT>(d, store_passes(d) - 1, split, C, arena)),
          second(store_passes(d) > 1) {}
    __device__ __forceinline__ Row row(int ti, int r) const { return Row{(int64_t)ti * TM + r}; }
    __device__ __forceinline__ void put(const Row& w, int tj, int c, OutT v) const {
        const int64_t gj = (int64_t)tj * TN + c;
        store_at(d0, w.gi, gj, v);
        if (second) store_at(d1, w.gi, gj, v);
    }
};

// Rows of a view inside its physical extent, counted from the K chunk's
// first row and clipped to the chunk.
__device__ __forceinline__ int64_t rows_in(const View& v, const KRange& kr) {
    const int64_t r = v.prows - kr.kb, K = kr.ke - kr.kb;
    return r < 0 ? 0 : r < K ? r : K;
}

// a + s b for a fused pre-sum (s = +1 or -1: the exact product, one rounding,
// i.e. the IEEE sum or difference the pre-sum pass stores).
__device__ __forceinline__ float4 add_term(float4 a, float4 b, float s) {
    return make_float4(fmaf(s, b.x, a.x), fmaf(s, b.y, a.y), fmaf(s, b.z, a.z), fmaf(s, b.w, a.w));
}
__device__ __forceinline__ double2 add_term(double2 a, double2 b, double s) {
    return make_double2(fma(s, b.x, a.x), fma(s, b.y, a.y));
}

// LDS destination of a buffer load that writes LDS directly.
#define ATA_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// ---------------------------------------------------------------- FP32 MFMA
template <bool EPI>
__device__ void tile_f32(const LeafDesc& d, const float* Xp, const float* Yp, const float* X2p, const float* Y2p,
                         int ti, int tj, float* C, float* arena, unsigned char* smem, const KRange& kr) {
    Xp += kr.kb * d.X.ld;
    Yp += kr.kb * d.Y.ld;
    X2p += kr.kb * d.X2.ld;
    Y2p += kr.kb * d.Y2.ld;
    const int64_t xl = rows_in(d.X, kr), yl = rows_in(d.Y, kr);
    const int64_t x2l = d.sx2 ? rows_in(d.X2, kr) : 0, y2l = d.sy2 ? rows_in(d.Y2, kr) : 0;
    const float sx = (float)d.sx2, sy = (float)d.sy2;
    float* Xs = reinterpret_cast<float*>(smem);          // [2][BK][LD32]
    float* Ys = Xs + 2 * BK * LD32;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int lr = t >> 5, lc = (t & 31) << 2;
    const int64_t xc = (int64_t)ti * TILE_M + lc, yc = (int64_t)tj * TILE_N + lc;
    const bool xv = vec_ok(Xp, d.X.ld, 4), yv = vec_ok(Yp, d.Y.ld, 4);
    const bool x2v = vec_ok(X2p, d.X2.ld, 4), y2v = vec_ok(Y2p, d.Y2.ld, 4);
    const int64_t K = kr.ke - kr.kb;
    const int64_t nk = (K + BK - 1) / BK;

    v16f acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    float4 rx0, rx1, ry0, ry1;
    auto gload = [&](int64_t k0) {
        rx0 = load4f(Xp, d.X.ld, k0 + lr, xc, xl, d.X.pcols, xv);
        rx1 = load4f(Xp, d.X.ld, k0 + lr + 8, xc, xl, d.X.pcols, xv);
        ry0 = load4f(Yp, d.Y.ld, k0 + lr, yc, yl, d.Y.pcols, yv);
        ry1 = load4f(Yp, d.Y.ld, k0 + lr + 8, yc, yl, d.Y.pcols, yv);
        if (d.sx2) {
            rx0 = add_term(rx0, load4f(X2p, d.X2.ld, k0 + lr, xc, x2l, d.X2.pcols, x2v), sx);
            rx1 = add_term(rx1, load4f(X2p, d.X2.ld, k0 + lr + 8, xc, x2l, d.X2.pcols, x2v), sx);
        }
        if (d.sy2) {
            ry0 = add_term(ry0, load4f(Y2p, d.Y2.ld, k0 + lr, yc, y2l, d.Y2.pcols, y2v), sy);
            ry1 = add_term(ry1, load4f(Y2p, d.Y2.ld, k0 + lr + 8, yc, y2l, d.Y2.pcols, y2v), sy);
        }
    };
    auto sstore = [&](int buf) {
        float* xs = Xs + buf * BK * LD32;
        float* ys = Ys + buf * BK * LD32;
        *reinterpret_cast<float4*>(xs + lr * LD32 + lc) = rx0;
        *reinterpret_cast<float4*>(xs + (lr + 8) * LD32 + lc) = rx1;
        *reinterpret_cast<float4*>(ys + lr * LD32 + lc) = ry0;
        *reinterpret_cast<float4*>(ys + (lr + 8) * LD32 + lc) = ry1;
    };

    // two slabs in flight (see the split-BF16 engine)
    if (nk > 0) {
        gload(0);
        sstore(0);
    }
    if (nk > 1) gload(BK);
    __syncthreads();
    const int ko = lane >> 5, io = lane & 31;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) sstore(cur ^ 1);
        if (kt + 2 < nk) gload((kt + 2) * BK);
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
        __syncthreads();
    }
    const TileStore<EPI, float, TILE_M, TILE_N> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                sink.put(row, tj, wn * 64 + b * 32 + (lane & 31), acc[a][b][v]);
        }
}

// FP32 with a 256 x 256 tile: four waves of 128 x 128 (4 x 4 blocks of
// 32 x 32 on v_mfma_f32_32x32x2f32), one wave per SIMD: 16 independent MFMAs
// (1024 cycles) per pair of k rows against 8 LDS reads.  Slabs of 16 rows
// stream into three 36 KB LDS stages, X[16][288] then Y[16][288] (rows
// padded so that the two k rows one read serves fall in opposite bank
// halves), through 4-byte buffer loads that write LDS directly.  Each load
// covers 64 columns of one row through a buffer resource based at that row
// and sized to the view's physical columns, or to nothing for rows past K:
// the hardware's range check supplies the zero padding, with no offsets
// that grow with the matrix.  The schedule is fixed by hand: the operands of
// pair kk + 1 are read and one slab row of slab kt + 2 is issued under the
// MFMAs of pair kk, and the one barrier per slab sits inside the last pair,
// after which the first operands of slab kt + 1 are read, so the matrix
// cores do not wait on LDS latency at the slab boundary.

template <bool EPI>
__device__ __forceinline__ void tile_f32_wide(const LeafDesc& d, const float* Xp, const float* Yp, int ti, int tj,
                                              float* C, float* arena, unsigned char* smem, const KRange& kr) {
    using namespace wide32;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 1, wn = w & 1;
    const int64_t K = kr.ke - kr.kb;
    const int64_t nk = (K + SK - 1) / SK;
    // wave w streams operand (w < 2 ? X : Y), slab rows 8 (w % 2) .. + 7
    const bool isx = w < 2;
    const int64_t ld = isx ? d.X.ld : d.Y.ld;
    const float* P = (isx ? Xp : Yp) + kr.kb * ld;
    const int prow = (int)((isx ? d.X.pcols : d.Y.pcols) * 4);      // bytes of one physical row
    const uint32_t cbyte = (uint32_t)(((isx ? (int64_t)ti * TM : (int64_t)tj * TN) + lane) * 4);
    const int r0 = (w & 1) * 8;
    // 64 columns (segment seg) of this wave's slab row `part` of slab kt into stage st
    auto issue = [&](int64_t kt, int st, int part, int seg) {
        const int rr = r0 + part;
        const int64_t row = kt * SK + rr;
        const __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(P + row * ld), (short)0, row < K ? prow : 0, 0x00020000);
        unsigned char* base = smem + st * STAGE + (isx ? 0 : HALF) + rr * RS * 4;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base + seg * 256), 4, (int)(cbyte + seg * 256),
                                                 0, 0, 0);
    };
    auto issue_row = [&](int64_t kt, int st, int part) {
#pragma unroll
        for (int seg = 0; seg < 4; ++seg) issue(kt, st, part, seg);
    };

    v16f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    const int ko = lane >> 5, io = lane & 31;
    float a[2][4], b[2][4];
    auto read = [&](int st, int kk, int buf) {
        const float* xs = reinterpret_cast<const float*>(smem + st * STAGE) + wm * 128 + io + (2 * kk + ko) * RS;
        const float* ys = reinterpret_cast<const float*>(smem + st * STAGE + HALF) + wn * 128 + io + (2 * kk + ko) * RS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[buf][q] = xs[q * 32];
            b[buf][q] = ys[q * 32];
        }
    };
    auto mfma = [&](int buf, int i0, int i1) {
#pragma unroll
        for (int i = i0; i < i1; ++i)
            acc[i >> 2][i & 3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i >> 2], b[buf][i & 3],
                                                                      acc[i >> 2][i & 3], 0, 0, 0);
    };

    // Slabs past the end read as zeros, so every step issues the same 32
    // loads per wave and one wait count serves every step.
#pragma unroll
    for (int part = 0; part < 8; ++part) issue_row(0, 0, part);
#pragma unroll
    for (int sl = 1; sl < STAGES - 1; ++sl)
#pragma unroll
        for (int part = 0; part < 8; ++part) issue_row(sl, sl, part);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(LATER, 15));   // slab 0 has landed
    __builtin_amdgcn_s_barrier();
    read(0, 0, 0);
    int cur = 0, nxt = 1, fill = STAGES - 1;      // stages of slabs kt, kt + 1, kt + STAGES - 1
    for (int64_t kt = 0; kt < nk; ++kt) {
#pragma unroll
        for (int kk = 0; kk < SK / 2 - 1; ++kk) {
            const int buf = kk & 1;
            mfma(buf, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
            read(cur, kk + 1, buf ^ 1);
            __builtin_amdgcn_sched_barrier(0);
            // one load between consecutive MFMAs: a load that holds up issue
            // then delays no MFMA
            const int nl = kk == SK / 2 - 2 ? 8 : 4;
#pragma unroll
            for (int l = 0; l < nl; ++l) {
                mfma(buf, 1 + l, 2 + l);
                __builtin_amdgcn_sched_barrier(0);
                issue(kt + STAGES - 1, fill, kk + (l >> 2), l & 3);
                __builtin_amdgcn_sched_barrier(0);
            }
            mfma(buf, 1 + nl, 16);
            __builtin_amdgcn_sched_barrier(0);
        }
        mfma(1, 0, 4);
        __builtin_amdgcn_sched_barrier(0);
        // slab kt + 1 has landed (only later slabs' loads may be pending) and
        // this wave's reads of slab kt are done, so after the barrier slab
        // kt + 1 is visible and slab kt's stage free
        __builtin_amdgcn_s_waitcnt(waitcnt_imm(LATER, 0));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        read(nxt, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        mfma(1, 4, 16);
        __builtin_amdgcn_sched_barrier(0);
        cur = nxt;
        nxt = nxt == STAGES - 1 ? 0 : nxt + 1;
        fill = fill == STAGES - 1 ? 0 : fill + 1;
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);           // the zero slabs past the end have landed
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * 128 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sink.put(row, tj, wn * 128 + b * 32 + (lane & 31), acc[a][b][v]);
        }
}

// The 256 x 256 FP32 tile on eight waves of 128 x 64 (4 x 2 blocks of 32 x 32,
// 128 accumulators per lane), two waves per SIMD: while one wave waits on a
// load's issue or an LDS read, the other's MFMAs keep the matrix core busy.
// Same per-row buffer resources and fixed schedule as the four-wave form,
// with slabs of 32 rows in two stages (half the barriers; a slab's loads are
// issued in the first eight of its sixteen k-row pairs); each wave streams
// eight rows of X (waves 0-3) or Y (4-7).
template <bool EPI, int SK8, int ST8>
__device__ __forceinline__ void tile_f32_wide8(const LeafDesc& d, const float* Xp, const float* Yp, int ti, int tj,
                                               float* C, float* arena, unsigned char* smem, const KRange& kr) {
    using wide32::TM;
    using wide32::TN;
    using wide32::RS;
    using wide32::waitcnt_imm;
    constexpr int SK = SK8;                       // rows per slab
    constexpr int STAGES = ST8;
    constexpr int HALF = SK * RS * 4;
    constexpr int STAGE = 2 * HALF;
    constexpr int RPW = SK / 4;                   // slab rows per wave
    constexpr int NL = RPW * 4;                   // loads per wave per slab
    constexpr int LATER8 = NL * (STAGES - 2) < 63 ? NL * (STAGES - 2) : 63;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 2, wn = w & 3;
    const int64_t K = kr.ke - kr.kb;
    const int64_t nk = (K + SK - 1) / SK;
    const bool isx = w < 4;
    const int64_t ld = isx ? d.X.ld : d.Y.ld;
    const float* P = (isx ? Xp : Yp) + kr.kb * ld;
    const int64_t lim = isx ? rows_in(d.X, kr) : rows_in(d.Y, kr);
    const int prow = (int)((isx ? d.X.pcols : d.Y.pcols) * 4);
    const uint32_t cbyte = (uint32_t)(((isx ? (int64_t)ti * TM : (int64_t)tj * TN) + lane) * 4);
    const int r0 = (w & 3) * RPW;
    // load l (0..NL-1) of this wave's share of slab kt: row r0 + l / 4, segment l % 4
    auto issue = [&](int64_t kt, int st, int l) {
        const int rr = r0 + (l >> 2), seg = l & 3;
        const int64_t row = kt * SK + rr;
        const __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(P + row * ld), (short)0, row < lim ? prow : 0, 0x00020000);
        unsigned char* base = smem + st * STAGE + (isx ? 0 : HALF) + rr * RS * 4;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base + seg * 256), 4, (int)(cbyte + seg * 256),
                                                 0, 0, 0);
    };

    v16f acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    const int ko = lane >> 5, io = lane & 31;
    float a[2][4], b[2][2];
    auto read = [&](int st, int kk, int buf) {
        const float* xs = reinterpret_cast<const float*>(smem + st * STAGE) + wm * 128 + io + (2 * kk + ko) * RS;
        const float* ys = reinterpret_cast<const float*>(smem + st * STAGE + HALF) + wn * 64 + io + (2 * kk + ko) * RS;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[buf][q] = xs[q * 32];
#pragma unroll
        for (int q = 0; q < 2; ++q) b[buf][q] = ys[q * 32];
    };
    auto mfma = [&](int buf, int i0, int i1) {
#pragma unroll
        for (int i = i0; i < i1; ++i)
            acc[i >> 1][i & 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i >> 1], b[buf][i & 1],
                                                                      acc[i >> 1][i & 1], 0, 0, 0);
    };

#pragma unroll
    for (int l = 0; l < NL; ++l) issue(0, 0, l);
#pragma unroll
    for (int sl = 1; sl < STAGES - 1; ++sl)
#pragma unroll
        for (int l = 0; l < NL; ++l) issue(sl, sl, l);
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(LATER8, 15));  // slab 0 has landed
    __builtin_amdgcn_s_barrier();
    read(0, 0, 0);
    int cur = 0, nxt = 1, fill = STAGES - 1;
    for (int64_t kt = 0; kt < nk; ++kt) {
#pragma unroll
        for (int kk = 0; kk < SK / 2 - 1; ++kk) {
            const int buf = kk & 1;
            mfma(buf, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
            read(cur, kk + 1, buf ^ 1);
            __builtin_amdgcn_sched_barrier(0);
            if (kk < NL / 4) {
                // four of slab kt + STAGES - 1's loads, one per MFMA
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    mfma(buf, 1 + l, 2 + l);
                    __builtin_amdgcn_sched_barrier(0);
                    issue(kt + STAGES - 1, fill, kk * 4 + l);
                    __builtin_amdgcn_sched_barrier(0);
                }
                mfma(buf, 5, 8);
            } else {
                mfma(buf, 1, 8);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        mfma(1, 0, 2);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(waitcnt_imm(LATER8, 0));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        read(nxt, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        mfma(1, 2, 8);
        __builtin_amdgcn_sched_barrier(0);
        cur = nxt;
        nxt = nxt == STAGES - 1 ? 0 : nxt + 1;
        fill = fill == STAGES - 1 ? 0 : fill + 1;
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * 128 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                sink.put(row, tj, wn * 64 + b * 32 + (lane & 31), acc[a][b][v]);
        }
}

// The same engine for leaves with fused pre-sums: a side whose operand is
// the sum or difference of two views streams both into LDS and combines them
// as the MFMA operands are read (the IEEE sum or difference the pre-sum pass
// would have stored; a plain side skips the combine).  Two 72 KB stages of
// X, X2, Y and Y2 slabs; slab kt + 1 is loaded under the first k-row pairs
// of slab kt, one load between consecutive MFMAs.  V16: every term's rows
// start 16-byte aligned and hold a multiple of four physical columns, so one
// 16-byte load per lane moves a whole 256-column row (16 loads per wave per
// slab); otherwise 4-byte loads (64 per wave per slab).
template <bool EPI, bool V16>
__device__ __forceinline__ void tile_f32_wide_sum(const LeafDesc& d, const float* Xp, const float* Yp,
                                                  const float* X2p, const float* Y2p, int ti, int tj,
                                                  float* C, float* arena, unsigned char* smem, const KRange& kr) {
    using namespace wide32;
    constexpr int QS = 4 * HALF;                  // one stage: X, X2, Y, Y2
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 1, wn = w & 1;
    const int64_t K = kr.ke - kr.kb;
    const int64_t nk = (K + SK - 1) / SK;
    // wave w streams both terms of side (w < 2 ? X : Y), slab rows 8 (w % 2) .. + 7
    // every descriptor field the loop needs, read once (the loads that
    // write LDS are opaque memory operations, so the compiler would re-read
    // the descriptor after each one)
    const bool isx = w < 2;
    const int64_t lda_ = isx ? d.X.ld : d.Y.ld, ldb_ = isx ? d.X2.ld : d.Y2.ld;
    const bool two = (isx ? d.sx2 : d.sy2) != 0;
    const float* Pa = (isx ? Xp : Yp) + kr.kb * lda_;
    const float* Pb = (isx ? X2p : Y2p) + kr.kb * ldb_;
    const int64_t la = isx ? rows_in(d.X, kr) : rows_in(d.Y, kr);
    const int64_t lb = !two ? 0 : isx ? rows_in(d.X2, kr) : rows_in(d.Y2, kr);
    const int pa = (int)((isx ? d.X.pcols : d.Y.pcols) * 4), pb = (int)((isx ? d.X2.pcols : d.Y2.pcols) * 4);
    const int64_t col0 = isx ? (int64_t)ti * TM : (int64_t)tj * TN;
    const uint32_t cbyte = (uint32_t)((col0 + (V16 ? 4 : 1) * lane) * 4);
    const int r0 = (w & 1) * 8;
    constexpr int NL = V16 ? 16 : 64;             // loads per wave per slab
    // load l of this wave's share of slab kt: term, row and (4-byte form) 64-column segment
    auto issue = [&](int64_t kt, int st, int l) {
        const int term = V16 ? l >> 3 : l >> 5;
        const int rr = r0 + (V16 ? l & 7 : (l >> 2) & 7), seg = V16 ? 0 : l & 3;
        const int64_t row = kt * SK + rr;
        const float* rp = term ? Pb + row * ldb_ : Pa + row * lda_;
        const int nrec = row < (term ? lb : la) ? (term ? pb : pa) : 0;
        const __amdgpu_buffer_rsrc_t src =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(rp), (short)0, nrec, 0x00020000);
        unsigned char* base = smem + st * QS + (isx ? 0 : 2 * HALF) + term * HALF + rr * RS * 4;
        if constexpr (V16)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base), 16, (int)cbyte, 0, 0, 0);
        else
            __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base + seg * 256), 4, (int)(cbyte + seg * 256),
                                                     0, 0, 0);
    };

    v16f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    const int ko = lane >> 5, io = lane & 31;
    const int sx2 = __builtin_amdgcn_readfirstlane(d.sx2), sy2 = __builtin_amdgcn_readfirstlane(d.sy2);
    const bool fx = sx2 != 0, fy = sy2 != 0;
    const float sx = (float)sx2, sy = (float)sy2;
    float a[2][4], b[2][4];
    auto read = [&](int st, int kk, int buf) {
        const float* xs = reinterpret_cast<const float*>(smem + st * QS) + wm * 128 + io + (2 * kk + ko) * RS;
        const float* ys = reinterpret_cast<const float*>(smem + st * QS + 2 * HALF) + wn * 128 + io +
                          (2 * kk + ko) * RS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x1 = xs[q * 32], x2 = xs[HALF / 4 + q * 32];
            const float y1 = ys[q * 32], y2 = ys[HALF / 4 + q * 32];
            a[buf][q] = fx ? fmaf(sx, x2, x1) : x1;
            b[buf][q] = fy ? fmaf(sy, y2, y1) : y1;
        }
    };
    auto mfma = [&](int buf, int i0, int i1) {
#pragma unroll
        for (int i = i0; i < i1; ++i)
            acc[i >> 2][i & 3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[buf][i >> 2], b[buf][i & 3],
                                                                      acc[i >> 2][i & 3], 0, 0, 0);
    };

#pragma unroll
    for (int l = 0; l < NL; ++l) issue(0, 0, l);
    __builtin_amdgcn_s_waitcnt(0x0F70);           // vmcnt(0): slab 0 has landed
    __builtin_amdgcn_s_barrier();
    read(0, 0, 0);
    int cur = 0;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int nxt = cur ^ 1;
#pragma unroll
        for (int kk = 0; kk < SK / 2 - 1; ++kk) {
            const int buf = kk & 1;
            mfma(buf, 0, 1);
            __builtin_amdgcn_sched_barrier(0);
            read(cur, kk + 1, buf ^ 1);
            __builtin_amdgcn_sched_barrier(0);
            if (kk < NL / 16) {
                // slab kt + 1 (zeros past the end) into the stage slab kt - 1 left
#pragma unroll
                for (int l = 0; l < 15; ++l) {
                    mfma(buf, 1 + l, 2 + l);
                    __builtin_amdgcn_sched_barrier(0);
                    issue(kt + 1, nxt, kk * 16 + l);
                    __builtin_amdgcn_sched_barrier(0);
                }
                issue(kt + 1, nxt, kk * 16 + 15);
            } else {
                mfma(buf, 1, 16);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        mfma(1, 0, 4);
        __builtin_amdgcn_sched_barrier(0);
        // slab kt + 1 has landed and this wave's reads of slab kt are done:
        // after the barrier slab kt + 1 is visible and slab kt's stage free
        __builtin_amdgcn_s_waitcnt(0x0070);       // vmcnt(0) lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        read(nxt, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        mfma(1, 4, 16);
        __builtin_amdgcn_sched_barrier(0);
        cur = nxt;
    }
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * 128 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sink.put(row, tj, wn * 128 + b * 32 + (lane & 31), acc[a][b][v]);
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

// Split-BF16 x3 tile engine: WM x WN waves, each owning BMB x BNB blocks of
// 32 x 32 (tile TM x TN = 32 WM BMB x 32 WN BNB).  Each 16-row slab is one
// MFMA k step.  The K loop is software-pipelined so that the matrix pipe
// never waits on LDS after the per-slab barrier:
//   - the fragments of slab kt + 1 are read while slab kt's MFMAs run, each
//     fragment register being refilled as soon as the pass that reads it has
//     been issued (pass 1: lo(X) hi(Y); pass 2: hi(X) hi(Y); pass 3: hi(X)
//     lo(Y)), so one set of fragment registers suffices;
//   - global loads run two slabs ahead into two staging sets; slab kt + 2 is
//     written to the LDS stage slab kt has left, in the middle of the
//     iteration, and one barrier at its end publishes it;
//   - loads go through buffer resources bounded to the K chunk's row groups,
//     so groups past the chunk read as zeros and the loop needs no selects.
// Instances: 128 x 128 on four waves (tile 0), 256 x 128 on four waves
// (tile 1), 256 x 256 on eight waves of 128 x 64 (tile 2, two waves per SIMD)
// and on four waves of 128 x 128 (tile 3, one wave per SIMD, a third fewer
// LDS reads per MFMA).
namespace pipe {
constexpr int LDR = 24;                       // bf16 per LDS column row: 16 k + 8 pad (48 bytes)
// s_waitcnt immediates: lgkmcnt(0) (vmcnt and expcnt unconstrained); vmcnt(n)
// (lgkmcnt and expcnt unconstrained)
constexpr int WAIT_LGKM0 = 0xC07F;
constexpr int wait_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0F70; }
template <int WM, int WN, int BMB, int BNB>
struct Geo {
    static constexpr int TM = 32 * WM * BMB, TN = 32 * WN * BNB, NT = 64 * WM * WN;
    static constexpr int PX = 2 * TM / NT, PY = 2 * TN / NT;    // chunks per thread per slab
    static constexpr int STAGE = (2 * TM + 2 * TN) * LDR;      // bf16 elements
    static constexpr size_t LDS = (size_t)2 * STAGE * 2;       // two stages, bytes
    static_assert(PX >= 1 && PY >= 1 && PX * NT == 2 * TM && PY * NT == 2 * TN, "loader layout");
};
}  // namespace pipe

__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const float* arena, const Packed& P, bool lo,
                                                             int64_t gb, int64_t ngk) {
    const float* b = arena + P.off + (lo ? P.lo_delta : 0) + gb * P.gstride;
    const int64_t avail = (P.end - P.off - gb * P.gstride) * 4;
    const int64_t want = ngk * P.gstride * 4;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(b), (short)0,
                                             (int)(uint32_t)(want < avail ? want : avail), 0x00020000);
}

template <bool EPI, int WM, int WN, int BMB, int BNB>
__device__ __forceinline__ void tile_bf16x3(const LeafDesc& d, const float* arena_in, int ti, int tj,
                                            float* C, float* arena, unsigned char* smem, const KRange& kr) {
    using G = pipe::Geo<WM, WN, BMB, BNB>;
    constexpr int TM = G::TM, TN = G::TN, NT = G::NT, PX = G::PX, PY = G::PY, LDR = pipe::LDR;
    constexpr int STAGE = G::STAGE;
    constexpr int XH = 0, XL = TM * LDR, YH = 2 * TM * LDR, YL = (2 * TM + TN) * LDR;
    unsigned short* lds = reinterpret_cast<unsigned short*>(smem);
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w / WN, wn = w % WN;
    const int64_t K = kr.ke - kr.kb;
    const int64_t gb = kr.kb / 8;                 // first 8-row group of the K chunk
    const int64_t ngk = (K + 7) / 8;              // row groups of the chunk
    const int64_t nk = ((K + 15) / 16 + 1) & ~int64_t(1);   // slabs, rounded up to even (zeros past K)

    // loader: chunk t + NT i of the slab's X (or Y) chunks = (group g, column col)
    const __amdgpu_buffer_rsrc_t rxh = chunk_rsrc(arena_in, d.PX, false, gb, ngk);
    const __amdgpu_buffer_rsrc_t rxl = chunk_rsrc(arena_in, d.PX, true, gb, ngk);
    const __amdgpu_buffer_rsrc_t ryh = chunk_rsrc(arena_in, d.PY, false, gb, ngk);
    const __amdgpu_buffer_rsrc_t ryl = chunk_rsrc(arena_in, d.PY, true, gb, ngk);
    const uint32_t xgs = (uint32_t)(d.PX.gstride * 4), ygs = (uint32_t)(d.PY.gstride * 4);
    uint32_t xo0[PX], yo0[PY];
    int xso[PX], yso[PY];
#pragma unroll
    for (int i = 0; i < PX; ++i) {
        const int ci = t + NT * i, g = ci / TM, col = ci % TM;
        xo0[i] = (uint32_t)g * xgs + (uint32_t)((ti * TM + col) * 16);
        xso[i] = col * LDR + 8 * g;
    }
#pragma unroll
    for (int i = 0; i < PY; ++i) {
        const int ci = t + NT * i, g = ci / TN, col = ci % TN;
        yo0[i] = (uint32_t)g * ygs + (uint32_t)((tj * TN + col) * 16);
        yso[i] = col * LDR + 8 * g;
    }
    v4u sxh[2][PX], sxl[2][PX], syh[2][PY], syl[2][PY];
    auto gload = [&](int set, int64_t s) {
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            const uint32_t o = xo0[i] + (uint32_t)s * 2u * xgs;
            sxh[set][i] = __builtin_amdgcn_raw_buffer_load_b128(rxh, (int)o, 0, 0);
            sxl[set][i] = __builtin_amdgcn_raw_buffer_load_b128(rxl, (int)o, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            const uint32_t o = yo0[i] + (uint32_t)s * 2u * ygs;
            syh[set][i] = __builtin_amdgcn_raw_buffer_load_b128(ryh, (int)o, 0, 0);
            syl[set][i] = __builtin_amdgcn_raw_buffer_load_b128(ryl, (int)o, 0, 0);
        }
    };
    auto sstore = [&](int set, int stage) {
        unsigned short* st = lds + stage * STAGE;
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            *reinterpret_cast<v4u*>(st + XH + xso[i]) = sxh[set][i];
            *reinterpret_cast<v4u*>(st + XL + xso[i]) = sxl[set][i];
        }
#pragma unroll
        for (int i = 0; i < PY; ++i) {
            *reinterpret_cast<v4u*>(st + YH + yso[i]) = syh[set][i];
            *reinterpret_cast<v4u*>(st + YL + yso[i]) = syl[set][i];
        }
    };

    // fragment of lane l: column (l % 32) of its block, k = 8 (l / 32) .. + 7
    const int ao = (wm * BMB * 32 + (lane & 31)) * LDR + 8 * (lane >> 5);
    const int bo = (wn * BNB * 32 + (lane & 31)) * LDR + 8 * (lane >> 5);
    auto frag = [&](int stage, int half, int off) {
        return *reinterpret_cast<const v8bf*>(lds + stage * STAGE + half + off);
    };
    v8bf ah[BMB], al[BMB], bh[BNB], bl[BNB];

    v16f acc[BMB][BNB];
#pragma unroll
    for (int a = 0; a < BMB; ++a)
#pragma unroll
        for (int b = 0; b < BNB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    auto barrier = [] {
        __builtin_amdgcn_s_waitcnt(pipe::WAIT_LGKM0);
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
    };

    // iteration kt (par = kt & 1): the fragment registers hold slab kt; LDS
    // stage par ^ 1 holds slab kt + 1; staging set par holds slab kt + 2 and
    // set par ^ 1 slab kt + 3 (in flight)
    auto iter = [&](int64_t kt, int par) {
        const int nx = par ^ 1;
#pragma unroll
        for (int a = 0; a < BMB; ++a)
#pragma unroll
            for (int b = 0; b < BNB; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < BMB; ++a) al[a] = frag(nx, XL, ao + a * 32 * LDR);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < BMB; ++a)
#pragma unroll
            for (int b = 0; b < BNB; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < BNB; ++b) bh[b] = frag(nx, YH, bo + b * 32 * LDR);
        // slab kt + 2 into the stage slab kt has left: its loads are the
        // older half of those this thread has in flight
        __builtin_amdgcn_s_waitcnt(pipe::wait_vm(2 * (PX + PY)));
        sstore(par, par);
        gload(par, kt + 4);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < BMB; ++a) {
#pragma unroll
            for (int b = 0; b < BNB; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            ah[a] = frag(nx, XH, ao + a * 32 * LDR);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int b = 0; b < BNB; ++b) bl[b] = frag(nx, YL, bo + b * 32 * LDR);
        barrier();
    };

    // the two staging sets are issued one after the other (never
    // interleaved), so that waiting for the older set leaves the newer in flight
    gload(0, 0);
    gload(1, 1);
    sstore(0, 0);
    sstore(1, 1);
    __builtin_amdgcn_sched_barrier(0);
    gload(0, 2);
    __builtin_amdgcn_sched_barrier(0);
    gload(1, 3);
    __builtin_amdgcn_sched_barrier(0);
    barrier();
#pragma unroll
    for (int a = 0; a < BMB; ++a) {
        ah[a] = frag(0, XH, ao + a * 32 * LDR);
        al[a] = frag(0, XL, ao + a * 32 * LDR);
    }
#pragma unroll
    for (int b = 0; b < BNB; ++b) {
        bh[b] = frag(0, YH, bo + b * 32 * LDR);
        bl[b] = frag(0, YL, bo + b * 32 * LDR);
    }
    barrier();                                     // stage 0 is free for slab 2
    for (int64_t kt = 0; kt < nk; kt += 2) {
        iter(kt, 0);
        iter(kt + 1, 1);
    }
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < BMB; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * BMB * 32 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < BNB; ++b)
                sink.put(row, tj, wn * BNB * 32 + b * 32 + (lane & 31), acc[a][b][v]);
        }
}

// LDS ring of the streamed split-BF16 engine (tile 4): slabs of 16 k (two
// 8-k groups) stream into four LDS stages through buffer loads that write LDS
// directly; stage s holds Xh, Xl, Yh, Yl, each [group][256 columns] of
// 16-byte chunks, and lane l of a load lands at 16 l bytes past the
// instruction's LDS base.
namespace wide {
constexpr int TM = 256, TN = 256;
constexpr int STAGES = WIDE_STAGES;
constexpr int ARR = 2 * 256 * 16;             // bytes of one operand half in a stage
constexpr int STAGE = 4 * ARR;                // 32 KB
constexpr size_t LDS = (size_t)STAGES * STAGE;
}  // namespace wide

// Split-BF16 256 x 256 tile on eight waves of 128 x 64 (4 x 2 blocks, 128
// accumulators per lane), two waves per SIMD, operands streamed through the
// LDS ring above; each operand half is streamed by two waves, one 8-row group
// each, and the fragments of slab kt + 1 are read under slab kt's MFMAs.
template <bool EPI>
__device__ __forceinline__ void tile_bf16x3_wide8(const LeafDesc& d, const float* arena_in, int ti, int tj, float* C,
                                                  float* arena, unsigned char* smem, const KRange& kr) {
    using namespace wide;
    constexpr int L8 = 4;                          // buffer->LDS loads per wave per slab
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 2, wn = w & 3;
    const int64_t K = kr.ke - kr.kb;
    const int64_t gb = kr.kb / 8;
    const int64_t nk = ((K + 15) / 16 + 1) & ~int64_t(1);

    // waves 2h and 2h + 1 stream operand half h (0 Xh, 1 Xl, 2 Yh, 3 Yl), group w % 2 of every slab
    const int half = w >> 1, g = w & 1;
    const bool isx = half < 2;
    const __amdgpu_buffer_rsrc_t src = packed_rsrc(arena_in, isx ? d.PX : d.PY, (half & 1) != 0);
    const uint32_t gs = (uint32_t)((isx ? d.PX.gstride : d.PY.gstride) * 4);
    const uint32_t col0 = (uint32_t)((isx ? ti * TM : tj * TN) + lane) * 16u;
    const uint32_t past = (uint32_t)(((isx ? d.PX.end - d.PX.off : d.PY.end - d.PY.off)) * 4);
    auto issue = [&](int64_t kt) {
        unsigned char* base = smem + (kt % STAGES) * STAGE + half * ARR + g * 4096;
        const int64_t lrow = kt * 2 + g;
        const bool in = lrow * 8 < K;
#pragma unroll
        for (int seg = 0; seg < L8; ++seg) {
            const uint32_t off = in ? (uint32_t)(gb + lrow) * gs + col0 + (uint32_t)(seg * 64 * 16) : past;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base + seg * 1024), 16, (int)off, 0, 0, 0);
        }
    };
    // at most 4 n loads of this wave outstanding
    auto wait_n = [](int64_t n) {
        if (n <= 0) __builtin_amdgcn_s_waitcnt(0x0F70);        // vmcnt(0)
        else if (n == 1) __builtin_amdgcn_s_waitcnt(0x0F74);   // vmcnt(4)
        else if (n == 2) __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8)
        else __builtin_amdgcn_s_waitcnt(0x0F7C);               // vmcnt(12)
    };

    v16f acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    const int fo = (lane >> 5) * 4096 + (lane & 31) * 16;
    v8bf xh[2][4], xl[2][4], yh[2][2], yl[2][2];
    auto frags = [&](int buf, int64_t kt) {
        const unsigned char* st = smem + (kt % STAGES) * STAGE + fo;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int xo = (wm * 128 + a * 32) * 16;
            xh[buf][a] = *reinterpret_cast<const v8bf*>(st + 0 * ARR + xo);
            xl[buf][a] = *reinterpret_cast<const v8bf*>(st + 1 * ARR + xo);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int yo = (wn * 64 + b * 32) * 16;
            yh[buf][b] = *reinterpret_cast<const v8bf*>(st + 2 * ARR + yo);
            yl[buf][b] = *reinterpret_cast<const v8bf*>(st + 3 * ARR + yo);
        }
    };
    auto mfmas = [&](int buf) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[buf][a], yh[buf][b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[buf][a], yl[buf][b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[buf][a], yh[buf][b], acc[a][b], 0, 0, 0);
    };
    constexpr int AHEAD = STAGES - 1;
    auto step = [&](int64_t kt, int cur) {
        if (kt + 1 < nk) wait_n((kt + AHEAD - 1 < nk ? kt + AHEAD - 1 : nk - 1) - kt - 1);
        __builtin_amdgcn_s_barrier();
        if (kt + AHEAD < nk) issue(kt + AHEAD);
        if (kt + 1 < nk) frags(cur ^ 1, kt + 1);
        mfmas(cur);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // two MFMAs
        }
    };

    for (int64_t j = 0; j < AHEAD && j < nk; ++j) issue(j);
    if (nk > 0) {
        wait_n((nk < AHEAD ? nk : AHEAD) - 1);
        __builtin_amdgcn_s_barrier();
        frags(0, 0);
    }
    for (int64_t kt = 0; kt < nk; kt += 2) {
        step(kt, 0);
        step(kt + 1, 1);
    }
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const auto row = sink.row(ti, wm * 128 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3));
#pragma unroll
            for (int b = 0; b < 2; ++b)
                sink.put(row, tj, wn * 64 + b * 32 + (lane & 31), acc[a][b][v]);
        }
}

// ------------------------------------------------------------ FP8 e4m3
// 128 x 128 tile, four waves (2 x 2), each 64 x 64 = 4 x 4 blocks of 16 x 16
// on v_mfma_scale_f32_16x16x128_f8f6f4.  A slab is 128 rows, i.e. exactly one
// 128-row scale block of each operand, and a tile column range is one
// 128-column scale block, so both E8M0 scales (127 + e) are uniform per slab.
// MFMA lane layout: lane l holds row/column l%16 and k = 32(l/16) .. +31; the
// result register v of lane l is (i = 4(l/16) + v, j = l%16).
typedef int v8i __attribute__((ext_vector_type(8)));
constexpr int LD8 = 144;                         // bytes per LDS row: 128 k + 16 pad
constexpr size_t LDS8_BYTES = 2 * 2 * 128 * LD8;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t q8_rsrc(const float* arena, const Packed8& Q) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(arena + Q.off), (short)0,
                                             (int)(uint32_t)((Q.end - Q.off) * 4), 0x00020000);
}

template <bool EPI>
__device__ void tile_fp8(const LeafDesc& d, const float* arena_in, int ti, int tj,
                         float* C, float* arena, unsigned char* smem, const KRange& kr) {
    auto xq_ = [&](int s) { return smem + s * 2 * 128 * LD8; };
    auto yq_ = [&](int s) { return smem + s * 2 * 128 * LD8 + 128 * LD8; };
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const __amdgpu_buffer_rsrc_t rx = q8_rsrc(arena_in, d.QX), ry = q8_rsrc(arena_in, d.QY);
    const int* sx = reinterpret_cast<const int*>(arena_in + d.QX.scales);
    const int* sy = reinterpret_cast<const int*>(arena_in + d.QY.scales);
    const int64_t sxs = d.QX.ld / 128, sys = d.QY.ld / 128;     // scale rows
    const int64_t K = kr.ke - kr.kb;
    const int64_t sb0 = kr.kb / 128;              // first 128-row slab of the K chunk
    const int64_t nk = (K + 127) / 128;
    const int wave_base = __builtin_amdgcn_readfirstlane(t & ~63);

    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.f;

    // chunks: X [0, 1024) then Y [0, 1024); chunk (g, col): rows 16g..16g+15 of the slab
    v4u st[8];
    auto gload = [&](int64_t kt) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int trw = wave_base + 256 * i;
            const bool isx = trw < 1024;
            const int trw2 = isx ? trw : trw - 1024;
            const int g = trw2 >> 7, col = (trw2 & 127) + lane;
            const int64_t ld = isx ? d.QX.ld : d.QY.ld;
            const uint32_t off = (uint32_t)((((sb0 + kt) * 8 + g) * ld + (isx ? ti : tj) * 128 + col) * 16);
            st[i] = __builtin_amdgcn_raw_buffer_load_b128(isx ? rx : ry, (int)off, 0, 0);
        }
    };
    auto sstore = [&](int s) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int trw = wave_base + 256 * i;
            const bool isx = trw < 1024;
            const int trw2 = isx ? trw : trw - 1024;
            const int g = trw2 >> 7, col = (trw2 & 127) + lane;
            *reinterpret_cast<v4u*>((isx ? xq_(s) : yq_(s)) + col * LD8 + 16 * g) = st[i];
        }
    };

    // two slabs in flight (see the split-BF16 engine); the block scales of
    // the next slab are read one iteration ahead
    if (nk > 0) {
        gload(0);
        sstore(0);
    }
    if (nk > 1) gload(1);
    __syncthreads();
    const int io = lane & 15, ko = 32 * (lane >> 4);
    // block scales: the exponents of slab kt + 1 are loaded in iteration kt
    // ahead of the slab loads and biased in iteration kt + 1 (vector memory
    // counts complete in order: a use right after them would also wait for
    // slab kt + 2's loads)
    int ex = nk > 0 ? sx[sb0 * sxs + ti] : 0, ey = nk > 0 ? sy[sb0 * sys + tj] : 0;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) sstore(cur ^ 1);
        const int sa = 127 + ex, sb = 127 + ey;
        if (kt + 1 < nk) {
            ex = sx[(sb0 + kt + 1) * sxs + ti];
            ey = sy[(sb0 + kt + 1) * sys + tj];
        }
        if (kt + 2 < nk) gload(kt + 2);
        v8i fa[4], fb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const unsigned char* p = xq_(cur) + (wm * 64 + a * 16 + io) * LD8 + ko;
            const v4u lo = *reinterpret_cast<const v4u*>(p), hi = *reinterpret_cast<const v4u*>(p + 16);
            fa[a] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const unsigned char* p = yq_(cur) + (wn * 64 + b * 16 + io) * LD8 + ko;
            const v4u lo = *reinterpret_cast<const v4u*>(p), hi = *reinterpret_cast<const v4u*>(p + 16);
            fb[b] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa[a], fb[b], acc[a][b],
                                                                             0, 0, 0, sa, 0, sb);
        __syncthreads();
    }
    const TileStore<EPI, float, TILE_M, TILE_N> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const auto row = sink.row(ti, wm * 64 + a * 16 + 4 * (lane >> 4) + v);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sink.put(row, tj, wn * 64 + b * 16 + (lane & 15), acc[a][b][v]);
        }
}

// FP8 e4m3 with a 256 x 256 tile: four waves of 128 x 128 (8 x 8 blocks of
// 16 x 16 on v_mfma_scale_f32_16x16x128_f8f6f4), one wave per SIMD.  A slab
// is 128 rows, one scale block deep; each wave's 128 tile rows (columns) are
// exactly one 128-column scale block of X (of Y), so both E8M0 scales stay
// uniform per wave and slab.  Slabs stream into two 64 KB LDS stages by
// buffer loads that write LDS directly: stage layout X[group 0..7][256
// columns], then Y, of 16-byte chunks (16 consecutive rows of one column);
// wave w streams X (w < 2) or Y groups 4 (w % 2) .. + 3.  The next slab's
// loads run under the current slab's 64 MFMAs.
namespace wide8 {
constexpr int TM = 256, TN = 256;
constexpr int HALF = 8 * 256 * 16;            // one operand's slab: 32 KB
constexpr int STAGE = 2 * HALF;
}  // namespace wide8

// FP8 256 x 256 tile on eight waves (2 x 4) of 128 x 64 (8 x 4 blocks of
// 16 x 16 on the scaled 16 x 16 x 128 MFMA, 128 accumulators per lane), two
// waves per SIMD, so that one wave's MFMAs cover the other's load waits,
// barrier and fragment reads.  A slab is 128 rows, one scale block of each
// operand: waves 0-3 stream X's eight 16-row groups (two each), waves 4-7
// Y's, through buffer loads that write LDS directly ([group][256 columns] of
// 16-byte chunks; lane l of a load lands at 16 l bytes past its base).  Two
// stages: slab kt + 1 streams in while slab kt is multiplied.
template <bool EPI>
__device__ __forceinline__ void tile_fp8_wide(const LeafDesc& d, const float* arena_in, int ti, int tj, float* C,
                                              float* arena, unsigned char* smem, const KRange& kr) {
    using namespace wide8;
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wm = w >> 2, wn = w & 3;
    const int64_t K = kr.ke - kr.kb;
    const int64_t nk = (K + 127) / 128;
    const int64_t sb0 = kr.kb / 128;              // first 128-row slab of the K chunk
    const bool isx = w < 4;
    const Packed8& Q = isx ? d.QX : d.QY;
    const __amdgpu_buffer_rsrc_t src = q8_rsrc(arena_in, Q);
    const uint32_t past = (uint32_t)((Q.end - Q.off) * 4);
    const int64_t cp = Q.cols_p, ld = Q.ld;
    const int64_t col0 = (isx ? (int64_t)ti * TM : (int64_t)tj * TN) + lane;
    const int gbase = (w & 3) * 2;                // this wave's two row-groups of the slab
    // byte offsets of this lane's four column segments in row-group gbase of
    // the K chunk's first slab; a lane past the padded width keeps the offset
    // past the end of the array (keep = 0), where the range check reads zeros
    uint32_t o0[4], keep[4];
#pragma unroll
    for (int seg = 0; seg < 4; ++seg) {
        const int64_t col = col0 + seg * 64;
        o0[seg] = col < cp ? (uint32_t)(((sb0 * 8 + gbase) * ld + col) * 16) : past;
        keep[seg] = col < cp ? 0xFFFFFFFFu : 0u;
    }
    const uint32_t group_bytes = (uint32_t)(ld * 16), slab_bytes = 8 * group_bytes;
    auto issue = [&](int64_t kt, int stage) {
        unsigned char* base = smem + stage * STAGE + (isx ? 0 : HALF);
        const uint32_t step = (uint32_t)kt * slab_bytes;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int g = gbase + (i >> 2), seg = i & 3;
            const uint32_t off = o0[seg] + ((step + (uint32_t)(i >> 2) * group_bytes) & keep[seg]);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(src, ATA_LDS_PTR(base + (g * 256 + seg * 64) * 16), 16,
                                                     (int)off, 0, 0, 0);
        }
    };
    // scales: this wave's X and Y column blocks (clamped: a tile column past
    // the padded width only feeds outputs that are never stored)
    const int* sx = reinterpret_cast<const int*>(arena_in + d.QX.scales);
    const int* sy = reinterpret_cast<const int*>(arena_in + d.QY.scales);
    const int64_t sxs = d.QX.ld / 128, sys = d.QY.ld / 128;     // scale rows
    const int64_t nbx = d.QX.cols_p / 128, nby = d.QY.cols_p / 128;
    const int64_t bx = (int64_t)ti * 2 + wm < nbx ? (int64_t)ti * 2 + wm : nbx - 1;
    const int64_t by = (int64_t)tj * 2 + (wn >> 1) < nby ? (int64_t)tj * 2 + (wn >> 1) : nby - 1;

    v4f acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.f;

    // fragment of lane l: column (l % 16) of its block, rows 32 (l / 16) ..
    // + 31 of the slab = groups 2 (l / 16) and 2 (l / 16) + 1
    const int fo = (2 * (lane >> 4)) * 256 * 16 + (lane & 15) * 16;
    auto frag = [](const unsigned char* p) {
        const v4u lo = *reinterpret_cast<const v4u*>(p);
        const v4u hi = *reinterpret_cast<const v4u*>(p + 256 * 16);
        return v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    };
    // block scales: the exponents of slab kt + 1 are loaded at the start of
    // step kt, ahead of that step's slab loads, and biased at step kt + 1
    // (vector memory counts complete in order, so a use in step kt would also
    // wait for the slab loads issued before it)
    int ex = nk > 0 ? sx[sb0 * sxs + bx] : 0, ey = nk > 0 ? sy[sb0 * sys + by] : 0;
    auto step = [&](int64_t kt) {
        const int cur = (int)(kt & 1);
        __builtin_amdgcn_s_waitcnt(0x0F70);       // this wave's loads of slab kt are done
        __builtin_amdgcn_s_barrier();             // every wave's loads of slab kt are visible,
                                                  // and slab kt - 1's stage is free
        const int sa = 127 + ex, sb = 127 + ey;
        if (kt + 1 < nk) {
            ex = sx[(sb0 + kt + 1) * sxs + bx];
            ey = sy[(sb0 + kt + 1) * sys + by];
            issue(kt + 1, cur ^ 1);
        }
        const unsigned char* xs = smem + cur * STAGE + fo + (wm * 128) * 16;
        const unsigned char* ys = smem + cur * STAGE + HALF + fo + (wn * 64) * 16;
        v8i fb[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) fb[b] = frag(ys + b * 16 * 16);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const v8i fa = frag(xs + a * 16 * 16);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa, fb[b], acc[a][b], 0, 0, 0, sa, 0, sb);
        }
    };
    if (nk > 0) issue(0, 0);
    for (int64_t kt = 0; kt < nk; ++kt) step(kt);
    const TileStore<EPI, float, TM, TN> sink(d, kr.split, C, arena);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const auto row = sink.row(ti, wm * 128 + a * 16 + 4 * (lane >> 4) + v);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sink.put(row, tj, wn * 64 + b * 16 + (lane & 15), acc[a][b][v]);
        }
}

// ---------------------------------------------------------------- FP64 MFMA
// InT = double (FP64 mode) or float (FP64 fallback of the FP32 family: the
// inputs are promoted exactly, the result is rounded to OutT on store).
template <bool EPI, class InT, class OutT>
__device__ __forceinline__ void tile_f64(const LeafDesc& d, const InT* Xp, const InT* Yp, const InT* X2p, const InT* Y2p,
                         int ti, int tj, OutT* C, OutT* arena, unsigned char* smem, const KRange& kr) {
    Xp += kr.kb * d.X.ld;
    Yp += kr.kb * d.Y.ld;
    X2p += kr.kb * d.X2.ld;
    Y2p += kr.kb * d.Y2.ld;
    const int64_t xl = rows_in(d.X, kr), yl = rows_in(d.Y, kr);
    const int64_t x2l = d.sx2 ? rows_in(d.X2, kr) : 0, y2l = d.sy2 ? rows_in(d.Y2, kr) : 0;
    double* Xs = reinterpret_cast<double*>(smem);        // [2][BK][LD64]
    double* Ys = Xs + 2 * BK * LD64;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int64_t K = kr.ke - kr.kb;
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
    // descriptor fields in registers: read through the reference, they are
    // reloaded after every LDS store of the K loop
    const int64_t xld = d.X.ld, yld = d.Y.ld, xpc = d.X.pcols, ypc = d.Y.pcols;
    const int64_t x2ld = d.X2.ld, y2ld = d.Y2.ld, x2pc = d.X2.pcols, y2pc = d.Y2.pcols;
    const int32_t sx2 = d.sx2, sy2 = d.sy2;
    const bool xv = vec_ok(Xp, xld, 16 / (int)sizeof(InT));
    const bool yv = vec_ok(Yp, yld, 16 / (int)sizeof(InT));
    const bool x2v = vec_ok(X2p, x2ld, 16 / (int)sizeof(InT));
    const bool y2v = vec_ok(Y2p, y2ld, 16 / (int)sizeof(InT));

    auto gload = [&](int64_t k0) {
        if constexpr (sizeof(InT) == 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double2 x = load2d(Xp, xld, k0 + lr + q * rstep, xc, xl, xpc, xv);
                double2 y = load2d(Yp, yld, k0 + lr + q * rstep, yc, yl, ypc, yv);
                if (sx2)
                    x = add_term(x, load2d(X2p, x2ld, k0 + lr + q * rstep, xc, x2l, x2pc, x2v), (double)sx2);
                if (sy2)
                    y = add_term(y, load2d(Y2p, y2ld, k0 + lr + q * rstep, yc, y2l, y2pc, y2v), (double)sy2);
                rx[2 * q] = x.x; rx[2 * q + 1] = x.y;
                ry[2 * q] = y.x; ry[2 * q + 1] = y.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                // the FP64 fallback's SYRK leaves have no fused pre-sums
                const float4 x = load4f(Xp, xld, k0 + lr + q * rstep, xc, xl, xpc, xv);
                const float4 y = load4f(Yp, yld, k0 + lr + q * rstep, yc, yl, ypc, yv);
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
    // a wave whose 64 x 64 block of a SYRK tile lies wholly above the
    // diagonal (nothing it computes is stored) skips its MFMAs, leaving the
    // matrix pipe to the other workgroup's wave on its SIMD; it still loads,
    // stores and waits
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const bool idle = d.kind == LEAF_SYRK &&
                      (int64_t)tj * TILE_N + (wu & 1) * 64 >= (int64_t)ti * TILE_M + ((wu >> 1) + 1) * 64;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const double* xs = Xs + cur * BK * LD64 + wm * 64 + io;
        const double* ys = Ys + cur * BK * LD64 + wn * 64 + io;
#pragma unroll
        for (int kq = 0; kq < BK / 4; ++kq) {
            if (idle) break;
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
    const TileStore<EPI, OutT, TILE_M, TILE_N> sink(d, kr.split, C, arena);
    if constexpr (EPI) {
        // (the wider epilogue needs the explicit unroll to keep acc in registers;
        // the FP64 fallback never combines in its epilogue)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const auto row = sink.row(ti, wm * 64 + a * 16 + 4 * v + (lane >> 4));
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    sink.put(row, tj, wn * 64 + b * 16 + (lane & 15), (OutT)acc[a][b][v]);
            }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wm * 64 + a * 16 + 4 * v + (lane >> 4);
                const int c = wn * 64 + b * 16 + (lane & 15);
                if (d.ksplit > 1 && sizeof(OutT) == 4) {
                    // FP64 fallback of a split leaf: its partial sums stay FP64
                    const int64_t gi = (int64_t)ti * TILE_M + r, gj = (int64_t)tj * TILE_N + c;
                    if (gi < d.rows && gj < d.cols && !(d.kind == LEAF_SYRK && gj > gi))
                        reinterpret_cast<double*>(arena + d.part64_off)[((int64_t)kr.split * d.rows + gi) * d.cols + gj] =
                            acc[a][b][v];
                } else {
                    sink.put(sink.row(ti, r), tj, c, (OutT)acc[a][b][v]);
                }
            }
}

static_assert(lds_bytes(MODE_BF16X3) == pipe::Geo<2, 2, 2, 2>::LDS, "tile 0 LDS");
static_assert(lds_bytes(MODE_BF16X3_LARGE) == pipe::Geo<2, 2, 4, 2>::LDS, "tile 1 LDS");
static_assert(lds_bytes(MODE_BF16X3_HUGE) == pipe::Geo<2, 4, 4, 2>::LDS, "tile 2 LDS");
static_assert(lds_bytes(MODE_BF16X3_WIDE) == pipe::Geo<2, 2, 4, 4>::LDS, "tile 3 LDS");
static_assert(threads_for(MODE_BF16X3) == pipe::Geo<2, 2, 2, 2>::NT && threads_for(MODE_BF16X3_LARGE) ==
              pipe::Geo<2, 2, 4, 2>::NT && threads_for(MODE_BF16X3_HUGE) == pipe::Geo<2, 4, 4, 2>::NT,
              "split-BF16 workgroup sizes");

template <int MODE, bool EPI>
__device__ __forceinline__ void run_tile(const LeafArgs& args, int64_t bid, unsigned char* smem) {
    const LeafDesc& d = args.tasks[find_leaf(args.tasks, args.ntasks, bid)];
    const void* Aptr = args.Aptrs ? args.Aptrs[d.prob] : args.A;
    void* Cptr = args.Cptrs ? args.Cptrs[d.prob] : args.C;
    if (d.pred_node >= 0 && (int32_t)args.flags[d.pred_node] != d.pred_value) return;
    int64_t q = bid - d.tile_begin;
    KRange kr{0, d.K, 0};
    if (d.ksplit > 1) {
        kr.split = (int)(q / d.tiles_split);
        q -= (int64_t)kr.split * d.tiles_split;
        kr.kb = (int64_t)kr.split * d.kchunk;
        kr.ke = kr.kb + d.kchunk < d.K ? kr.kb + d.kchunk : d.K;
    }
    int ti, tj;
    leaf_tile<MODE == MODE_BF16X3_LARGE ? 2 : 1>(d, q, args.band, ti, tj);
    // SYRK leaves under the spread check run in exactly one of the two
    // launches: the FP64 fallback kernel when their node is flagged, the
    // mode's own kernel otherwise.
    const bool flagged = d.fb_node >= 0 && args.flags[d.fb_node];
    if constexpr (MODE == MODE_F64) {
        tile_f64<EPI, double, double>(d, view_ptr<double>(d.X, Aptr, args.B, args.arena),
                                 view_ptr<double>(d.Y, Aptr, args.B, args.arena),
                                 view_ptr<double>(d.X2, Aptr, args.B, args.arena),
                                 view_ptr<double>(d.Y2, Aptr, args.B, args.arena), ti, tj,
                                 static_cast<double*>(Cptr), static_cast<double*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_FALLBACK) {
        if (!flagged) return;
        const float* Xf = view_ptr<float>(d.X, Aptr, args.B, args.arena);
        const float* Yf = view_ptr<float>(d.Y, Aptr, args.B, args.arena);
        tile_f64<false, float, float>(d, Xf, Yf, Xf, Yf, ti, tj, static_cast<float*>(Cptr),
                               static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_BF16X3) {
        if (flagged) return;
        tile_bf16x3<EPI, 2, 2, 2, 2>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                                static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_BF16X3_LARGE) {
        if (flagged) return;
        tile_bf16x3<EPI, 2, 2, 4, 2>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                                static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_F32_WIDE) {
        if (flagged) return;
        if (d.sx2 | d.sy2) {
            const float* X1 = view_ptr<float>(d.X, Aptr, args.B, args.arena);
            const float* Y1 = view_ptr<float>(d.Y, Aptr, args.B, args.arena);
            const float* X2 = view_ptr<float>(d.X2, Aptr, args.B, args.arena);
            const float* Y2 = view_ptr<float>(d.Y2, Aptr, args.B, args.arena);
            // 16-byte rows: aligned bases and strides, whole 16-byte column groups
            auto v16 = [](const float* p, const View& v) {
                return ((reinterpret_cast<uintptr_t>(p) & 15) | ((v.ld | v.pcols) & 3)) == 0;
            };
            if (v16(X1, d.X) && v16(Y1, d.Y) && (!d.sx2 || v16(X2, d.X2)) && (!d.sy2 || v16(Y2, d.Y2)))
                tile_f32_wide_sum<EPI, true>(d, X1, Y1, X2, Y2, ti, tj, static_cast<float*>(Cptr),
                                        static_cast<float*>(args.arena), smem, kr);
            else
                tile_f32_wide_sum<EPI, false>(d, X1, Y1, X2, Y2, ti, tj, static_cast<float*>(Cptr),
                                         static_cast<float*>(args.arena), smem, kr);
        } else
            tile_f32_wide<EPI>(d, view_ptr<float>(d.X, Aptr, args.B, args.arena),
                          view_ptr<float>(d.Y, Aptr, args.B, args.arena), ti, tj, static_cast<float*>(Cptr),
                          static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_F32_WIDE8) {
        if (flagged) return;
        tile_f32_wide8<EPI, F32W8_SK, F32W8_ST>(d, view_ptr<float>(d.X, Aptr, args.B, args.arena),
                                                  view_ptr<float>(d.Y, Aptr, args.B, args.arena), ti, tj,
                                                  static_cast<float*>(Cptr), static_cast<float*>(args.arena), smem,
                                                  kr);
    } else if constexpr (MODE == MODE_FP8_WIDE) {
        if (flagged) return;
        tile_fp8_wide<EPI>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                      static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_FP8) {
        if (flagged) return;
        tile_fp8<EPI>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                 static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_BF16X3_WIDE8) {
        if (flagged) return;
        tile_bf16x3_wide8<EPI>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                          static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_BF16X3_WIDE) {
        if (flagged) return;
        tile_bf16x3<EPI, 2, 2, 4, 4>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                                static_cast<float*>(args.arena), smem, kr);
    } else if constexpr (MODE == MODE_BF16X3_HUGE) {
        if (flagged) return;
        tile_bf16x3<EPI, 2, 4, 4, 2>(d, static_cast<const float*>(args.arena), ti, tj, static_cast<float*>(Cptr),
                                static_cast<float*>(args.arena), smem, kr);
    } else {
        if (flagged) return;
        tile_f32<EPI>(d, view_ptr<float>(d.X, Aptr, args.B, args.arena), view_ptr<float>(d.Y, Aptr, args.B, args.arena),
                 view_ptr<float>(d.X2, Aptr, args.B, args.arena), view_ptr<float>(d.Y2, Aptr, args.B, args.arena),
                 ti, tj, static_cast<float*>(Cptr), static_cast<float*>(args.arena), smem, kr);
    }
}

// One workgroup per tile (XCD-aware order).
template <int MODE, bool EPI>
__global__ __launch_bounds__(threads_for(MODE), min_blocks_for(MODE)) void leaf_kernel(LeafArgs args) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[lds_bytes(MODE)];
    run_tile<MODE, EPI>(args, args.tile_base + xcd_remap(blockIdx.x, args.ntiles, args.chunk), smem);
}

// Persistent form (its own kernel, so that the queue logic does not change
// the register allocation of the one-tile-per-workgroup form): eight tile
// queues, one per XCD (workgroup ids go round-robin to the XCDs).  Queue q
// owns the chunk-sized runs q, q + 8, q + 16, ... of the longest-first tile
// order, so the tiles one XCD runs share operand panels in its L2.  A
// workgroup drains its own XCD's queue, then the others; a queue's tile index
// grows with its ticket, so the first ticket past the end means the queue is
// empty for good.
template <int MODE, bool EPI>
__global__ __launch_bounds__(threads_for(MODE), MODE == MODE_F64 || MODE == MODE_FALLBACK ? 2 : 1)
void leaf_kernel_persistent(LeafArgs args) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[lds_bytes(MODE)];
    // the ticket is passed through the first bytes of the tile's LDS, which
    // no tile touches between the two barriers around it
    int64_t* next = reinterpret_cast<int64_t*>(smem);
    const uint32_t chunk = (uint32_t)args.chunk;
    const int home = (int)(blockIdx.x & 7);
    for (int probe = 0; probe < 8;) {
        const int q = (home + probe) & 7;
        __syncthreads();                          // the previous tile is done with LDS
        if (threadIdx.x == 0) {
            const uint64_t k = atomicAdd(args.counter + q, 1ull);
            const uint64_t run = k / chunk;
            *next = (int64_t)((run * 8 + (uint64_t)q) * chunk + (k - run * chunk));
        }
        __syncthreads();
        const int64_t tile = *next;
        __syncthreads();
        if (tile >= args.ntiles) {
            ++probe;
            continue;
        }
        run_tile<MODE, EPI>(args, args.tile_base + tile, smem);
    }
}

// Resets the eight queue heads of a persistent launch (a kernel, not a
// memset, so that the reset is safe inside a captured graph).
__global__ void zero_counter(unsigned long long* c) { c[threadIdx.x] = 0ull; }

// The leaf launch of a plan, with the kernels built for plain stores (EPI
// false) or for combines in the epilogue (EPI true).
template <bool EPI>
hipError_t launch_leaves_t(int32_t mode, int32_t tile_cfg, const LeafDesc* d_tasks, int ntasks, int64_t ntiles,
                           const void* A, void* C, void* arena, const uint8_t* flags, int chunk, int band,
                           hipStream_t stream, const BatchPtrs* bp, const void* B, int64_t tile_base) {
    if (ntiles <= 0) return hipSuccess;
    // a dispatch counts its work-items in 32 bits: refuse a grid that would wrap
    if (!(bp && bp->counter) && ntiles > (int64_t)(0xFFFFFFFFu / 512u)) return hipErrorInvalidConfiguration;
    LeafArgs a{d_tasks, ntasks, chunk, band, ntiles, A, C, arena, flags, nullptr, nullptr, nullptr, B, tile_base};
    dim3 grid((unsigned)ntiles);
    if (bp) {
        a.Aptrs = bp->A;
        a.Cptrs = bp->C;
        if (bp->counter) {
            a.counter = bp->counter;
            hipLaunchKernelGGL(zero_counter, dim3(1), dim3(8), 0, stream, bp->counter);
            const int64_t g = ntiles < bp->persistent_blocks ? ntiles : bp->persistent_blocks;
            grid = dim3((unsigned)g);
        }
    }
#define ATA_LAUNCH_LEAF(M, threads)                                                          \
    do {                                                                                 \
        if (a.counter)                                                                   \
            hipLaunchKernelGGL((leaf_kernel_persistent<M, EPI>), grid, dim3(threads), 0, stream, a); \
        else                                                                             \
            hipLaunchKernelGGL((leaf_kernel<M, EPI>), grid, dim3(threads), 0, stream, a);       \
    } while (0)
    if (mode == MODE_BF16X3 && tile_cfg == 1) {
        ATA_LAUNCH_LEAF(MODE_BF16X3_LARGE, LEAF_THREADS);
        return hipGetLastError();
    }
    if (mode == MODE_BF16X3 && tile_cfg == 2) {
        ATA_LAUNCH_LEAF(MODE_BF16X3_HUGE, 512);
        return hipGetLastError();
    }
    if (mode == MODE_BF16X3 && tile_cfg == 3) {
        if constexpr (EPI) return hipErrorInvalidValue;    // (not built with epilogue combines)
        else ATA_LAUNCH_LEAF(MODE_BF16X3_WIDE, LEAF_THREADS);
        return hipGetLastError();
    }
    if (mode == MODE_BF16X3 && tile_cfg == 4) {
        ATA_LAUNCH_LEAF(MODE_BF16X3_WIDE8, 512);
        return hipGetLastError();
    }
    if (mode == MODE_FP8 && tile_cfg == 3) {
        ATA_LAUNCH_LEAF(MODE_FP8_WIDE, 512);
        return hipGetLastError();
    }
    if (mode == MODE_F32 && tile_cfg == 3) {
        if constexpr (EPI) return hipErrorInvalidValue;    // (not built with epilogue combines)
        else ATA_LAUNCH_LEAF(MODE_F32_WIDE, LEAF_THREADS);
        return hipGetLastError();
    }
    if (mode == MODE_F32 && tile_cfg == 2) {
        ATA_LAUNCH_LEAF(MODE_F32_WIDE8, 512);
        return hipGetLastError();
    }
    switch (mode) {
        case MODE_F64: ATA_LAUNCH_LEAF(MODE_F64, LEAF_THREADS); break;
        case MODE_F32: ATA_LAUNCH_LEAF(MODE_F32, LEAF_THREADS); break;
        case MODE_BF16X3: ATA_LAUNCH_LEAF(MODE_BF16X3, LEAF_THREADS); break;
        case MODE_FP8: ATA_LAUNCH_LEAF(MODE_FP8, LEAF_THREADS); break;
        default: return hipErrorInvalidValue;
    }
#undef ATA_LAUNCH_LEAF
    return hipGetLastError();
}

}  // namespace
}  // namespace ata
