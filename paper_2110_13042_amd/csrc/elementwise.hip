// Memory-bound kernels of the AtA plan: Strassen pre-sums and combines
// (the block additions of Sec. 3.1 / 3.2, done as fused streaming passes
// instead of one ?axpy per block pair), column norms and spread flags for the
// FP64 fallback, and the FP64 Freivalds residual probe.
#include "kernels_common.hpp"
#include "launch.hpp"

namespace ata {

namespace {

constexpr int EW_THREADS = 256;
static_assert(EW_THREADS == ITEM_BLOCK, "one workgroup per aligned item block");

// --------------------------------------------------------------- pre-sums
// Work item = one row r and four consecutive columns c..c+3 of the m2 x n2
// sums.  Reads the four quadrant values of the parent operand (zero outside
// its physical extent and outside the quadrant's real size) and writes the
// five sums (Winograd: four, the chained ones from the rounded earlier sums),
// including the zero padding of the ceil-sized buffers.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    const v2bf p = {(__bf16)a, (__bf16)b};          // round to nearest even
    return __builtin_bit_cast(uint32_t, p);
}

// Split eight consecutive k values into packed hi and lo chunks.
__device__ __forceinline__ void split8(const float* v, uint4& hi, uint4& lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = pk_bf16(v[2 * q], v[2 * q + 1]);
        const float h0 = __builtin_bit_cast(float, h[q] << 16);
        const float h1 = __builtin_bit_cast(float, h[q] & 0xFFFF0000u);
        l[q] = pk_bf16(v[2 * q] - h0, v[2 * q + 1] - h1);
    }
    hi = make_uint4(h[0], h[1], h[2], h[3]);
    lo = make_uint4(l[0], l[1], l[2], l[3]);
}

// Pre-sums of a node whose products are all leaves, written straight into the
// split-BF16 packed layout.  Work item = one chunk (row-group g, column c):
// eight rows of the four quadrant values, the five (Winograd: four) sums
// formed in FP32, then split.
__device__ void presum_packed(const PresumDesc& d, int64_t e, const float* A, const float* B, float* arena) {
    const int64_t g = udiv(e, d.n2), c = e - g * d.n2;
    const float* V = (d.V.base == BASE_A ? A : d.V.base == BASE_B ? B : arena) + d.V.off;
    const int64_t ld = d.V.ld, pr = d.V.prows, pc = d.V.pcols;
    const int64_t m1 = d.m1, m2 = d.m2, n1 = d.n1, n2 = d.n2;
    float sum[5][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t r = 8 * g + q;
        auto get = [&](int qr, int qc) -> float {
            const int64_t rr = qr ? m1 + r : r, cc = qc ? n1 + c : c;
            const bool in = r < (qr ? m2 : m1) && c < (qc ? n2 : n1) && rr < pr && cc < pc;
            return in ? V[rr * ld + cc] : 0.f;
        };
        const float a11 = get(0, 0), a12 = get(0, 1), a21 = get(1, 0), a22 = get(1, 1);
        if (d.variant == 1) {
            if (d.side == 0) {
                sum[0][q] = a12 + a22; sum[1][q] = sum[0][q] - a11;
                sum[2][q] = a11 - a12; sum[3][q] = a21 - sum[1][q];
            } else {
                sum[0][q] = a12 - a11; sum[1][q] = a22 - sum[0][q];
                sum[2][q] = a22 - a12; sum[3][q] = sum[1][q] - a21;
            }
            sum[4][q] = 0.f;
        } else if (d.side == 0) {
            sum[0][q] = a11 + a22; sum[1][q] = a12 + a22; sum[2][q] = a11 + a21;
            sum[3][q] = a12 - a11; sum[4][q] = a21 - a22;
        } else {
            sum[0][q] = a11 + a22; sum[1][q] = a12 - a22; sum[2][q] = a21 - a11;
            sum[3][q] = a11 + a12; sum[4][q] = a21 + a22;
        }
    }
    const int64_t groups = (m2 + 7) / 8, each = groups * n2 * 8, lo_delta = groups * n2 * 4;
    const int nsums = d.variant == 1 ? 4 : 5;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (i >= nsums) break;
        uint4 hi, lo;
        split8(sum[i], hi, lo);
        float* base = arena + d.out_off + i * each;
        reinterpret_cast<uint4*>(base)[g * n2 + c] = hi;
        reinterpret_cast<uint4*>(base + lo_delta)[g * n2 + c] = lo;
    }
}

template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { struct type { double x, y, z, w; }; };

template <class T>
__device__ __forceinline__ typename Vec4<T>::type ld4(const T* p) {
    if constexpr (sizeof(T) == 4) {
        return *reinterpret_cast<const float4*>(p);
    } else {
        const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
        return {a.x, a.y, b.x, b.y};
    }
}
template <class T>
__device__ __forceinline__ void st4(T* p, const typename Vec4<T>::type& v) {
    if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = v;
    } else {
        reinterpret_cast<double2*>(p)[0] = make_double2(v.x, v.y);
        reinterpret_cast<double2*>(p)[1] = make_double2(v.z, v.w);
    }
}
#define V4OP(a, op, b) {a.x op b.x, a.y op b.y, a.z op b.z, a.w op b.w}

template <class T>
__device__ __forceinline__ void presum_kernel_block(const PresumDesc* tasks, int ntasks,
                                                            int64_t items, const T* A0, T* arena,
                                                            const uint8_t* flags, const void* const* Aptrs,
                                                            const T* B, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= items) return;
    const PresumDesc& d = tasks[block_task(tasks, ntasks, vb)];
    const int64_t e = x - d.elem_begin;
    if (e >= d.elems) return;
    if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) return;
    const T* A = Aptrs ? static_cast<const T*>(Aptrs[d.prob]) : A0;
    if constexpr (sizeof(T) == 4) {
        if (d.packed_out) {
            presum_packed(d, e, A, B, arena);
            return;
        }
    }
    const T* V = (d.V.base == BASE_A ? A : d.V.base == BASE_B ? B : arena) + d.V.off;
    const int64_t ld = d.V.ld, pr = d.V.prows, pc = d.V.pcols;
    const int64_t m1 = d.m1, m2 = d.m2, n1 = d.n1, n2 = d.n2;
    const int64_t plane = m2 * n2;
    if (d.unit == 1) {
        // one column per work item: rows whose starts are not 16-byte
        // aligned, read and written by consecutive lanes at consecutive
        // addresses
        const int64_t r = udiv(e, n2), c = e - r * n2;
        auto get1 = [&](int qr, int qc) -> T {
            const int64_t rr = qr ? m1 + r : r, cc = qc ? n1 + c : c;
            const bool in = r < (qr ? m2 : m1) && c < (qc ? n2 : n1) && rr < pr && cc < pc;
            return in ? V[rr * ld + cc] : T(0);
        };
        const T a11 = get1(0, 0), a12 = get1(0, 1), a21 = get1(1, 0), a22 = get1(1, 1);
        T* o = arena + d.out_off + r * n2 + c;
        if (d.variant == 1) {
            if (d.side == 0) {
                const T s1 = a12 + a22, s2 = s1 - a11;
                o[0] = s1; o[plane] = s2; o[2 * plane] = a11 - a12; o[3 * plane] = a21 - s2;
            } else {
                const T t1 = a12 - a11, t2 = a22 - t1;
                o[0] = t1; o[plane] = t2; o[2 * plane] = a22 - a12; o[3 * plane] = t2 - a21;
            }
        } else if (d.side == 0) {
            o[0] = a11 + a22; o[plane] = a12 + a22; o[2 * plane] = a11 + a21;
            o[3 * plane] = a12 - a11; o[4 * plane] = a21 - a22;
        } else {
            o[0] = a11 + a22; o[plane] = a12 - a22; o[2 * plane] = a21 - a11;
            o[3 * plane] = a11 + a12; o[4 * plane] = a21 + a22;
        }
        return;
    }
    const int64_t groups = (d.n2 + 3) >> 2;
    const int64_t r = udiv(e, groups), c0 = (e - r * groups) << 2;
    T* out = arena + d.out_off + r * n2;
    // fast path: four full columns in every quadrant, 16-byte aligned rows
    const bool inside = r < m1 && m1 + r < pr && c0 + 4 <= n1 && n1 + c0 + 4 <= pc;
    const bool aligned = ((reinterpret_cast<uintptr_t>(V) | (uintptr_t)(ld * sizeof(T)) |
                           (uintptr_t)(n1 * sizeof(T)) | (uintptr_t)(n2 * sizeof(T))) & 15) == 0;
    if (inside && aligned) {
        typedef typename Vec4<T>::type V4;
        const V4 a11 = ld4(V + r * ld + c0), a12 = ld4(V + r * ld + n1 + c0);
        const V4 a21 = ld4(V + (m1 + r) * ld + c0), a22 = ld4(V + (m1 + r) * ld + n1 + c0);
        if (d.variant == 1) {
            if (d.side == 0) {
                const V4 s1 = V4OP(a12, +, a22), s2 = V4OP(s1, -, a11);
                st4(out + 0 * plane + c0, s1);                     // S1 = X12 + X22
                st4(out + 1 * plane + c0, s2);                     // S2 = S1 - X11
                st4(out + 2 * plane + c0, V4 V4OP(a11, -, a12));   // S3 = X11 - X12
                st4(out + 3 * plane + c0, V4 V4OP(a21, -, s2));    // S4 = X21 - S2
            } else {
                const V4 t1 = V4OP(a12, -, a11), t2 = V4OP(a22, -, t1);
                st4(out + 0 * plane + c0, t1);                     // T1 = Y12 - Y11
                st4(out + 1 * plane + c0, t2);                     // T2 = Y22 - T1
                st4(out + 2 * plane + c0, V4 V4OP(a22, -, a12));   // T3 = Y22 - Y12
                st4(out + 3 * plane + c0, V4 V4OP(t2, -, a21));    // T4 = T2 - Y21
            }
            return;
        }
        if (d.side == 0) {
            st4(out + 0 * plane + c0, V4 V4OP(a11, +, a22));   // S1 = X11 + X22
            st4(out + 1 * plane + c0, V4 V4OP(a12, +, a22));   // S2 = X12 + X22
            st4(out + 2 * plane + c0, V4 V4OP(a11, +, a21));   // S3 = X11 + X21
            st4(out + 3 * plane + c0, V4 V4OP(a12, -, a11));   // S4 = X12 - X11
            st4(out + 4 * plane + c0, V4 V4OP(a21, -, a22));   // S5 = X21 - X22
        } else {
            st4(out + 0 * plane + c0, V4 V4OP(a11, +, a22));   // T1 = Y11 + Y22
            st4(out + 1 * plane + c0, V4 V4OP(a12, -, a22));   // T2 = Y12 - Y22
            st4(out + 2 * plane + c0, V4 V4OP(a21, -, a11));   // T3 = Y21 - Y11
            st4(out + 3 * plane + c0, V4 V4OP(a11, +, a12));   // T4 = Y11 + Y12
            st4(out + 4 * plane + c0, V4 V4OP(a21, +, a22));   // T5 = Y21 + Y22
        }
        return;
    }
    auto get = [&](int qr, int qc, int64_t c) -> T {
        const int64_t rr = qr ? m1 + r : r, cc = qc ? n1 + c : c;
        const bool in = r < (qr ? m2 : m1) && c < (qc ? n2 : n1) && rr < pr && cc < pc;
        return in ? V[rr * ld + cc] : T(0);
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t c = c0 + q;
        if (c >= n2) break;
        const T a11 = get(0, 0, c), a12 = get(0, 1, c), a21 = get(1, 0, c), a22 = get(1, 1, c);
        if (d.variant == 1) {
            if (d.side == 0) {
                const T s1 = a12 + a22, s2 = s1 - a11;
                out[0 * plane + c] = s1;
                out[1 * plane + c] = s2;
                out[2 * plane + c] = a11 - a12;
                out[3 * plane + c] = a21 - s2;
            } else {
                const T t1 = a12 - a11, t2 = a22 - t1;
                out[0 * plane + c] = t1;
                out[1 * plane + c] = t2;
                out[2 * plane + c] = a22 - a12;
                out[3 * plane + c] = t2 - a21;
            }
        } else if (d.side == 0) {
            out[0 * plane + c] = a11 + a22;
            out[1 * plane + c] = a12 + a22;
            out[2 * plane + c] = a11 + a21;
            out[3 * plane + c] = a12 - a11;
            out[4 * plane + c] = a21 - a22;
        } else {
            out[0 * plane + c] = a11 + a22;
            out[1 * plane + c] = a12 - a22;
            out[2 * plane + c] = a21 - a11;
            out[3 * plane + c] = a11 + a12;
            out[4 * plane + c] = a21 + a22;
        }
    }
}

template <class T>
__global__ __launch_bounds__(EW_THREADS) void presum_kernel(const PresumDesc* tasks, int ntasks,
                                                            int64_t items, const T* A0, T* arena,
                                                            const uint8_t* flags, const void* const* Aptrs,
                                                            const T* B) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x)
        presum_kernel_block(tasks, ntasks, items, A0, arena, flags, Aptrs, B, vb);
}

// ------------------------------------------------------ split-BF16 packing

// Work item = one 16-byte chunk (row-group g, column c): rows 8g..8g+7 of
// column c split into hi = bf16(a) and lo = bf16(a - hi).
__device__ __forceinline__ void pack_kernel_block(const PackDesc* tasks, int ntasks,
                                                          int64_t items, const float* A0,
                                                          float* arena, const uint8_t* flags,
                                                          const void* const* Aptrs, const float* B, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= items) return;
    const PackDesc& d = tasks[block_task(tasks, ntasks, vb)];
    const int64_t e = x - d.elem_begin;
    if (e >= d.elems) return;
    if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) return;
    const float* A = Aptrs ? static_cast<const float*>(Aptrs[d.prob]) : A0;
    const int64_t g = udiv(e, d.cols), c = e - g * d.cols;
    const float* src = (d.src.base == BASE_A ? A : d.src.base == BASE_B ? B : arena) + d.src.off;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t r = 8 * g + q;
        v[q] = (r < d.src.prows && c < d.src.pcols) ? src[r * d.src.ld + c] : 0.f;
    }
    uint4 hi, lo;
    split8(v, hi, lo);
    reinterpret_cast<uint4*>(arena + d.dst)[g * d.cols + c] = hi;
    reinterpret_cast<uint4*>(arena + d.dst + d.lo_delta)[g * d.cols + c] = lo;
}

__global__ __launch_bounds__(EW_THREADS) void pack_kernel(const PackDesc* tasks, int ntasks,
                                                          int64_t items, const float* A0,
                                                          float* arena, const uint8_t* flags,
                                                          const void* const* Aptrs, const float* B) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x)
        pack_kernel_block(tasks, ntasks, items, A0, arena, flags, Aptrs, B, vb);
}

// ------------------------------------------------------------ FP8 quantising
// One workgroup per 128 x 128 block of an operand view: block amax, the
// power-of-two exponent e (smallest e with amax <= 448 * 2^e; 448 = 0.875 * 2^9,
// so with amax = f 2^E, f in [0.5, 1): e = E - 9 if f <= 0.875 else E - 8,
// exact), then q = e4m3_RNE(a * 2^-e) packed in 16-row chunks.  A task with
// `norm` set (a full-height column slice of A) also writes, per column, the
// FP64 sum of squares of the block's 128 rows in row order:
// partial[part_off + bi * part_ld + col].
__global__ __launch_bounds__(EW_THREADS) void quant8_kernel(const Pack8Desc* tasks, int ntasks,
                                                            const float* A0, float* arena,
                                                            const uint8_t* flags,
                                                            const void* const* Aptrs, const float* B,
                                                            double* partial) {
    __shared__ float wmax[EW_THREADS / 64];
    __shared__ double lower[128];
    const int64_t x = blockIdx.x;
    const Pack8Desc& d = tasks[find_task(tasks, ntasks, x)];
    if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) return;
    const float* A = Aptrs ? static_cast<const float*>(Aptrs[d.prob]) : A0;
    const int64_t blk = x - d.elem_begin;
    const int64_t nbc = d.cols_p / 128;
    const int64_t bi = blk / nbc, bj = blk - bi * nbc;
    const float* src = (d.src.base == BASE_A ? A : d.src.base == BASE_B ? B : arena) + d.src.off;
    const int t = threadIdx.x, c = t & 127, h = t >> 7;
    const int64_t col = bj * 128 + c, row0 = bi * 128 + h * 64;
    float v[64];
    float amax = 0.f;
#pragma unroll
    for (int q = 0; q < 64; ++q) {
        const int64_t r = row0 + q;
        v[q] = (r < d.src.prows && col < d.src.pcols) ? src[r * d.src.ld + col] : 0.f;
        amax = fmaxf(amax, fabsf(v[q]));
    }
    double ss = 0.0;
    if (d.norm) {
#pragma unroll
        for (int q = 0; q < 64; ++q) ss += (double)v[q] * (double)v[q];
        if (h == 1) lower[c] = ss;
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    if ((t & 63) == 0) wmax[t >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    if (d.norm && h == 0 && col < d.src.pcols) partial[d.part_off + bi * d.part_ld + col] = ss + lower[c];
    int e = 0;
    if (amax > 0.f) {
        int E;
        const float f = frexpf(amax, &E);
        e = f <= 0.875f ? E - 9 : E - 8;
    }
    if (t == 0) reinterpret_cast<int*>(arena + d.scales)[blk] = e;
    unsigned char* data = reinterpret_cast<unsigned char*>(arena + d.dst);
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        uint32_t wds[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float* p4 = v + ch * 16 + q * 4;
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(p4[0], -e), ldexpf(p4[1], -e), 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(p4[2], -e), ldexpf(p4[3], -e), w, true);
            wds[q] = (uint32_t)w;
        }
        const int64_t g = row0 / 16 + ch;
        reinterpret_cast<uint4*>(data)[g * d.cols_p + col] = make_uint4(wds[0], wds[1], wds[2], wds[3]);
    }
}

// ------------------------------------------------------------- split-K sums
// Work item = one output element of a split leaf: its K-chunk partials are
// summed in chunk order in FP64 and rounded once into the leaf's target.
// Partials come from the FP64 fallback (FP64 array) when the leaf's node is
// flagged, else from the mode's leaf kernel (arrays of the mode's type).
template <class T>
__device__ __forceinline__ void reduce_kernel_block(const ReduceDesc* tasks, int ntasks,
                                                            int64_t items, T* C0, T* arena,
                                                            const uint8_t* flags, void* const* Cptrs, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= items) return;
    const ReduceDesc& d = tasks[block_task(tasks, ntasks, vb)];
    const int64_t e = x - d.elem_begin;
    if (e >= d.elems) return;
    if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) return;
    const int64_t i = udiv(e, d.cols), j = e - i * d.cols;
    if (d.kind == LEAF_SYRK && j > i) return;
    const int64_t plane = d.rows * d.cols;
    double s = 0.0;
    if (d.fb_node >= 0 && flags[d.fb_node]) {
        if (d.ksplit_fb <= 1) return;          // the unsplit fallback wrote the target
        const double* p = reinterpret_cast<const double*>(arena + d.part64_off) + e;
        for (int k = 0; k < d.ksplit_fb; ++k) s += p[k * plane];
    } else {
        if (d.ksplit <= 1) return;             // the unsplit leaf wrote the target
        const T* p = arena + d.part_off + e;
        for (int k = 0; k < d.ksplit; ++k) s += (double)p[k * plane];
    }
    if (d.out_kind == OUT_PACKED) {
        T* C = Cptrs ? static_cast<T*>(Cptrs[d.prob]) : C0;
        C[packed_index(d.out_row0 + i, d.out_col0 + j)] = (T)s;
    } else if (d.out_kind == OUT_CDENSE) {
        C0[(d.out_row0 + i) * d.out_ld + d.out_col0 + j] = (T)s;
    } else {
        arena[d.out_off + i * d.out_ld + j] = (T)s;
    }
}

template <class T>
__global__ __launch_bounds__(EW_THREADS) void reduce_kernel(const ReduceDesc* tasks, int ntasks,
                                                            int64_t items, T* C0, T* arena,
                                                            const uint8_t* flags, void* const* Cptrs) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x)
        reduce_kernel_block(tasks, ntasks, items, C0, arena, flags, Cptrs, vb);
}

// ------------------------------------------------- BLAS-style conveniences
// C = alpha T + beta C over packed arrays (beta = 0: C is not read).
template <class T>
__device__ __forceinline__ void axpby_kernel_block(const T* t, T* c, int64_t len, T alpha, T beta, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= len) return;
    c[x] = beta == T(0) ? alpha * t[x] : alpha * t[x] + beta * c[x];
}

template <class T>
__global__ __launch_bounds__(EW_THREADS) void axpby_kernel(const T* t, T* c, int64_t len, T alpha, T beta) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < len; vb += gridDim.x)
        axpby_kernel_block(t, c, len, alpha, beta, vb);
}

// At[j][i] = A[i][j] (A m x n with row stride lda, At n x m dense), through
// 32 x 33 LDS tiles so both sides are coalesced.
template <class T>
__global__ __launch_bounds__(EW_THREADS) void transpose_kernel(const T* A, int64_t m, int64_t n, int64_t lda,
                                                               T* At) {
    __shared__ T tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;          // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r, j = j0 + tx;
        if (i < m && j < n) tile[r][tx] = A[i * lda + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + r, i = i0 + tx;
        if (j < n && i < m) At[j * m + i] = tile[tx][r];
    }
}

// Full symmetric n x n matrix (row stride ldf) from packed lower storage.
template <class T>
__device__ __forceinline__ void unpack_kernel_block(const T* Cp, int64_t n, T* F, int64_t ldf, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= n * n) return;
    const int64_t i = x / n, j = x - i * n;
    const int64_t r = i > j ? i : j, c = i > j ? j : i;
    F[i * ldf + j] = Cp[packed_index(r, c)];
}

template <class T>
__global__ __launch_bounds__(EW_THREADS) void unpack_kernel(const T* Cp, int64_t n, T* F, int64_t ldf) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < n * n; vb += gridDim.x)
        unpack_kernel_block(Cp, n, F, ldf, vb);
}

// ------------------------------------------------- column equilibration
// e_j = the binary exponent of the column norm (sqrt(nu_j) = f 2^e_j, f in
// [0.5, 1)), 0 for a zero column.  Scaling a column by 2^-e_j is exact.
__device__ __forceinline__ int eq_exponent(double nu) {
    if (!(nu > 0.0)) return 0;
    int e;
    (void)frexp(sqrt(nu), &e);
    return e;
}

// Ap (m x n dense) = A diag(2^-e); e_j stored by the threads of row 0.
__device__ __forceinline__ void eq_scale_kernel_block(const float* A, int64_t m, int64_t n, int64_t lda,
                                                              const double* nu, float* Ap, int* e, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= m * n) return;
    const int64_t r = udiv(x, n), j = x - r * n;
    const int ej = eq_exponent(nu[j]);
    Ap[x] = ldexpf(A[r * lda + j], -ej);
    if (r == 0) e[j] = ej;
}

__global__ __launch_bounds__(EW_THREADS) void eq_scale_kernel(const float* A, int64_t m, int64_t n, int64_t lda,
                                                              const double* nu, float* Ap, int* e) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < m * n; vb += gridDim.x)
        eq_scale_kernel_block(A, m, n, lda, nu, Ap, e, vb);
}

// Packed C_ij *= 2^(e_i + e_j): the Gram product of the scaled columns back
// to the original scale (exact).
__device__ __forceinline__ void eq_unscale_kernel_block(float* Cp, int64_t n, const int* e, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= n * (n + 1) / 2) return;
    int64_t i = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while (i > 0 && i * (i + 1) / 2 > x) --i;
    while ((i + 1) * (i + 2) / 2 <= x) ++i;
    const int64_t j = x - i * (i + 1) / 2;
    Cp[x] = ldexpf(Cp[x], e[i] + e[j]);
}

__global__ __launch_bounds__(EW_THREADS) void eq_unscale_kernel(float* Cp, int64_t n, const int* e) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < n * (n + 1) / 2; vb += gridDim.x)
        eq_unscale_kernel_block(Cp, n, e, vb);
}

// ---------------------------------------------------------------- combine
// Work item = one row i and four columns j..j+3 of the n2 x k2 products (one
// column when k2 is not a multiple of four).
// C11 = M1 + M4 - M5 + M7, C12 = M3 + M5, C21 = M2 + M4,
// C22 = M1 - M2 + M3 + M6, each summed left to right; only the leading part
// of a product reaches a floor-sized quadrant.  Winograd's form shares partial
// sums: U2 = M1 + M6, U3 = U2 + M7, C11 = M1 + M2, C12 = (U2 + M5) + M3,
// C21 = U3 - M4, C22 = U3 + M5.
template <class T>
__device__ __forceinline__ void combine_kernel_block(const CombineDesc* tasks, int ntasks,
                                                             int64_t items, T* C0, T* arena,
                                                             const uint8_t* flags, void* const* Cptrs, int64_t vb) {
    const int64_t x = vb * EW_THREADS + threadIdx.x;
    if (x >= items) return;
    const CombineDesc& d = tasks[block_task(tasks, ntasks, vb)];
    const int64_t e = x - d.elem_begin;
    if (e >= d.elems) return;
    if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) return;
    T* C = Cptrs ? static_cast<T*>(Cptrs[d.prob]) : C0;
    // four columns per work item, or one when k2 is not a multiple of four
    const int w = d.unit == 1 ? 1 : 4;
    const int64_t groups = w == 1 ? d.k2 : (d.k2 + 3) >> 2;
    const int64_t i = udiv(e, groups), j0 = w == 1 ? e - i * groups : (e - i * groups) << 2;
    const int64_t n1 = d.n1, k1 = d.k1, k2 = d.k2, plane = d.n2 * d.k2;
    const T* M = arena + d.m_off + i * k2;
    auto dst = [&](int64_t ii, int64_t jj) -> T* {
        return d.out_kind == OUT_PACKED ? C + packed_index(d.out_row0 + ii, d.out_col0 + jj)
               : d.out_kind == OUT_CDENSE ? C + (d.out_row0 + ii) * d.out_ld + d.out_col0 + jj
                                          : arena + d.out_off + ii * d.out_ld + jj;
    };
    if (w == 4 && i < n1 && j0 + 4 <= k1 && (k2 & 3) == 0) {
        typedef typename Vec4<T>::type V4;
        const V4 m1 = ld4(M + j0), m2 = ld4(M + plane + j0), m3 = ld4(M + 2 * plane + j0);
        const V4 m4 = ld4(M + 3 * plane + j0), m5 = ld4(M + 4 * plane + j0);
        const V4 m6 = ld4(M + 5 * plane + j0), m7 = ld4(M + 6 * plane + j0);
        V4 c11, c12, c21, c22;
        if (d.variant == 1) {
            const V4 u2 = V4OP(m1, +, m6);
            const V4 u3 = V4OP(u2, +, m7);
            const V4 u4 = V4OP(u2, +, m5);
            c11 = V4 V4OP(m1, +, m2);
            c12 = V4 V4OP(u4, +, m3);
            c21 = V4 V4OP(u3, -, m4);
            c22 = V4 V4OP(u3, +, m5);
        } else {
            const V4 t14 = V4OP(m1, +, m4);
            const V4 t145 = V4OP(t14, -, m5);
            c11 = V4 V4OP(t145, +, m7);
            c12 = V4 V4OP(m3, +, m5);
            c21 = V4 V4OP(m2, +, m4);
            const V4 t12 = V4OP(m1, -, m2);
            const V4 t123 = V4OP(t12, +, m3);
            c22 = V4 V4OP(t123, +, m6);
        }
        T* p11 = dst(i, j0);
        T* p12 = dst(i, k1 + j0);
        T* p21 = dst(n1 + i, j0);
        T* p22 = dst(n1 + i, k1 + j0);
        const V4* vs[4] = {&c11, &c12, &c21, &c22};
        T* ps[4] = {p11, p12, p21, p22};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if ((reinterpret_cast<uintptr_t>(ps[q]) & 15) == 0) {
                st4(ps[q], *vs[q]);
            } else {
                ps[q][0] = vs[q]->x; ps[q][1] = vs[q]->y; ps[q][2] = vs[q]->z; ps[q][3] = vs[q]->w;
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t j = j0 + q;
        if (q >= w || j >= k2) break;
        const T m1 = M[j], m2 = M[plane + j], m3 = M[2 * plane + j], m4 = M[3 * plane + j];
        const T m5 = M[4 * plane + j], m6 = M[5 * plane + j], m7 = M[6 * plane + j];
        if (d.variant == 1) {
            const T u2 = m1 + m6, u3 = u2 + m7;
            if (i < n1) {
                if (j < k1) *dst(i, j) = m1 + m2;
                *dst(i, k1 + j) = (u2 + m5) + m3;
            }
            if (j < k1) *dst(n1 + i, j) = u3 - m4;
            *dst(n1 + i, k1 + j) = u3 + m5;
            continue;
        }
        if (i < n1) {
            if (j < k1) *dst(i, j) = ((m1 + m4) - m5) + m7;
            *dst(i, k1 + j) = m3 + m5;
        }
        if (j < k1) *dst(n1 + i, j) = m2 + m4;
        *dst(n1 + i, k1 + j) = ((m1 - m2) + m3) + m6;
    }
}

template <class T>
__global__ __launch_bounds__(EW_THREADS) void combine_kernel(const CombineDesc* tasks, int ntasks,
                                                             int64_t items, T* C0, T* arena,
                                                             const uint8_t* flags, void* const* Cptrs) {
    // the grid (at most ew_grid() workgroups) walks the virtual blocks
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x)
        combine_kernel_block(tasks, ntasks, items, C0, arena, flags, Cptrs, vb);
}

// ------------------------------------------------------------ column norms
constexpr int64_t NORM_ROWS = 256;   // residual passes

// Sum of squares of rows [r0, r1) of four columns starting at p (row stride
// ld floats), each column summed in ascending row order.  `vec`: 16-byte
// aligned rows and all four columns present; else `cols` columns, scalar.
__device__ __forceinline__ void sumsq4(const float* p, int64_t ld, int64_t r0, int64_t r1, bool vec,
                                       int cols, double s[4]) {
    int64_t r = r0;
    if (vec) {
        constexpr int U = 8;
        for (; r + U <= r1; r += U) {
            float4 a[U];
#pragma unroll
            for (int q = 0; q < U; ++q) a[q] = *reinterpret_cast<const float4*>(p + (r + q) * ld);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                s[0] += (double)a[q].x * (double)a[q].x;
                s[1] += (double)a[q].y * (double)a[q].y;
                s[2] += (double)a[q].z * (double)a[q].z;
                s[3] += (double)a[q].w * (double)a[q].w;
            }
        }
        for (; r < r1; ++r) {
            const float4 a = *reinterpret_cast<const float4*>(p + r * ld);
            s[0] += (double)a.x * (double)a.x;
            s[1] += (double)a.y * (double)a.y;
            s[2] += (double)a.z * (double)a.z;
            s[3] += (double)a.w * (double)a.w;
        }
        return;
    }
    for (; r < r1; ++r) {
        const float* row = p + r * ld;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < cols) { const double a = (double)row[q]; s[q] += a * a; }
    }
}

// Sums of squares of columns jb + lane + 64 c (c = 0..3) over rows [r0, r1)
// (r0 a multiple of 8) that also writes their split-BF16 packing: chunk
// (g, j) = rows 8g..8g+7 of column j, zero past the matrix's last row (r1 is
// a multiple of 8 or the row count).  Columns 64 apart per lane keep both the
// loads (a row segment of 64 columns per instruction) and the 16-byte chunk
// stores contiguous across the wave.  Rows are summed in order, as in sumsq4.
__device__ __forceinline__ void sumsq_pack(const float* A, int64_t ld, int64_t r0, int64_t r1, int64_t jb,
                                           int lane, int64_t n, double s[4], float* hi_base, int64_t lo_delta) {
    for (int64_t r = r0; r < r1; r += 8) {
        float v[4][8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t j = jb + lane + 64 * c;
                v[c][q] = (r + q < r1 && j < n) ? A[(r + q) * ld + j] : 0.f;
            }
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += (double)v[c][q] * (double)v[c][q];
        const int64_t g = r >> 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = jb + lane + 64 * c;
            if (j < n) {
                uint4 h, l;
                split8(v[c], h, l);
                reinterpret_cast<uint4*>(hi_base)[g * n + j] = h;
                reinterpret_cast<uint4*>(hi_base + lo_delta)[g * n + j] = l;
            }
        }
    }
}

// Column norms, pass 1: a workgroup covers 256 columns (four per lane) of one
// row chunk; its four waves take consecutive quarters of the chunk's rows and
// their sums are added in wave order through LDS (deterministic).
// partial[part_off + chunk * n + j] = sum of a_rj^2 over the chunk's rows.
// PACK: the launch has tasks that also write the split-BF16 packing (a
// separate instantiation, so that the plain form keeps its occupancy).
template <bool PACK>
__global__ __launch_bounds__(EW_THREADS) void colnorm_pass1(const ColDesc* tasks, int ntasks,
                                                            int64_t items, const float* A0,
                                                            const void* const* Aptrs, double* partial,
                                                            float* arena) {
    __shared__ double red[3][64][4];
    const int64_t x0 = (int64_t)blockIdx.x * EW_THREADS;
    if (x0 >= items) return;
    const ColDesc& d = tasks[block_task(tasks, ntasks)];
    const int64_t blk = (x0 - d.elem_begin) / EW_THREADS;      // workgroup-uniform
    if (x0 - d.elem_begin >= d.elems) return;
    const float* A = Aptrs ? static_cast<const float*>(Aptrs[d.prob]) : A0;
    const int64_t xblocks = (d.n + 255) / 256;
    const int64_t chunk = blk / xblocks, xb = blk - chunk * xblocks;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j0 = xb * 256 + lane * 4;
    const int64_t q = d.rows / 4;
    const int64_t rb = chunk * d.rows + wave * q;
    const int64_t r0 = rb < d.m ? rb : d.m, r1 = rb + q < d.m ? rb + q : d.m;
    const int cols = j0 >= d.n ? 0 : (d.n - j0 < 4 ? (int)(d.n - j0) : 4);
    const bool vec = cols == 4 && ((reinterpret_cast<uintptr_t>(A) | (uintptr_t)(d.lda * 4)) & 15) == 0;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const bool pack = PACK && d.pack;
    if (pack)
        sumsq_pack(A, d.lda, r0, r1, xb * 256, lane, d.n, s, arena + d.pack_dst, d.pack_lo);
    else if (cols > 0)
        sumsq4(A + j0, d.lda, r0, r1, vec, cols, s);
    if (wave > 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) red[wave - 1][lane][c] = s[c];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += red[w][lane][c];
        double* p = partial + d.part_off + chunk * d.n;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            // this lane's columns: j0 + c, or xb * 256 + lane + 64 c with the packing
            const int64_t j = pack ? xb * 256 + lane + 64 * c : j0 + c;
            if (j < d.n) p[j] = s[c];
        }
    }
}

// Column norms, pass 2: item = one column of one problem; the chunks are
// summed in order (eight loads in flight).
__global__ __launch_bounds__(EW_THREADS) void colnorm_pass2(const ColDesc* tasks, int ntasks,
                                                            int64_t items, const double* partial,
                                                            double* nu) {
    const int64_t x = (int64_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (x >= items) return;
    const ColDesc& d = tasks[block_task(tasks, ntasks)];
    const int64_t j = x - d.elem_begin;
    if (j >= d.elems) return;
    const double* p = partial + d.part_off + j;
    const int64_t n = d.n, nc = d.nchunks;
    double s = 0.0;
    int64_t c = 0;
    for (; c + 8 <= nc; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(c + u) * n];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nc; ++c) s += p[c * n];
    nu[d.nu_off + j] = s;
}

__global__ __launch_bounds__(EW_THREADS) void sum_partials(const double* partial, int64_t nchunks,
                                                           int64_t n, double* out) {
    const int64_t j = (int64_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) s += partial[c * n + j];
    out[j] = s;
}

// spread flag per AtA node: max/min of the nonzero squared norms > tau^2
__global__ __launch_bounds__(EW_THREADS) void flags_kernel(const double* nu, const NodeDesc* nodes,
                                                           double tau2, uint8_t* flags) {
    __shared__ double smax[EW_THREADS], smin[EW_THREADS];
    __shared__ int scnt[EW_THREADS];
    const NodeDesc nd = nodes[blockIdx.x];
    double mx = 0.0, mn = 0.0;
    int cnt = 0;
    for (int64_t j = nd.c0 + threadIdx.x; j < nd.c0 + nd.w; j += EW_THREADS) {
        const double v = nu[j];
        if (v > 0.0) {
            mx = cnt ? fmax(mx, v) : v;
            mn = cnt ? fmin(mn, v) : v;
            ++cnt;
        }
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    scnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = EW_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const int o = threadIdx.x + s;
            if (scnt[o]) {
                if (scnt[threadIdx.x]) {
                    smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[o]);
                    smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[o]);
                } else {
                    smax[threadIdx.x] = smax[o];
                    smin[threadIdx.x] = smin[o];
                }
                scnt[threadIdx.x] += scnt[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double spread = scnt[0] >= 2 ? smax[0] / smin[0] : 1.0;
        flags[blockIdx.x] = spread > tau2 ? 1 : 0;
    }
}

// ------------------------------------------------------- Freivalds residual
__device__ __forceinline__ double probe_sign(uint64_t seed, int64_t j) {
    // SplitMix64 output at counter j: state = seed + (j + 1) * gamma, then mix
    uint64_t z = seed + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (z >> 63) ? -1.0 : 1.0;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// y[r] = sum_j A[r][j] x_j : one wave per row, lanes stride over j
template <class T>
__global__ __launch_bounds__(EW_THREADS) void res_ax(const T* A, int64_t m, int64_t n, int64_t lda,
                                                     uint64_t seed, double* y) {
    const int64_t r = (int64_t)blockIdx.x * (EW_THREADS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= m) return;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) s += (double)A[r * lda + j] * probe_sign(seed, j);
    s = wave_sum(s);
    if (lane == 0) y[r] = s;
}

// zpart[chunk][j] = sum_{r in chunk} A[r][j] y[r];  fpart[chunk][j] = sum a^2
template <class T>
__global__ __launch_bounds__(EW_THREADS) void res_aty(const T* A, int64_t m, int64_t n, int64_t lda,
                                                      const double* y, double* zpart, double* fpart) {
    const int64_t j = (int64_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (j >= n) return;
    const int64_t r0 = chunk * NORM_ROWS, r1 = r0 + NORM_ROWS < m ? r0 + NORM_ROWS : m;
    double s = 0.0, f = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double a = (double)A[r * lda + j];
        s += a * y[r];
        f += a * a;
    }
    zpart[chunk * n + j] = s;
    fpart[chunk * n + j] = f;
}

// wrow[i] = sum_{j <= i} C[i][j] x_j : one wave per packed row
template <class T>
__global__ __launch_bounds__(EW_THREADS) void res_crow(const T* Cp, int64_t n, uint64_t seed, double* wrow) {
    const int64_t i = (int64_t)blockIdx.x * (EW_THREADS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const T* row = Cp + i * (i + 1) / 2;
    double s = 0.0;
    for (int64_t j = lane; j <= i; j += 64) s += (double)row[j] * probe_sign(seed, j);
    s = wave_sum(s);
    if (lane == 0) wrow[i] = s;
}

// wpart[band][j] = sum_{i in band, i > j} C[i][j] x_i  (the strictly-upper part of C x)
constexpr int64_t BAND = 256;
template <class T>
__global__ __launch_bounds__(EW_THREADS) void res_ccol(const T* Cp, int64_t n, uint64_t seed, double* wpart) {
    const int64_t j = (int64_t)blockIdx.x * EW_THREADS + threadIdx.x;
    const int64_t band = blockIdx.y;
    if (j >= n) return;
    const int64_t i0 = band * BAND, i1 = i0 + BAND < n ? i0 + BAND : n;
    double s = 0.0;
    for (int64_t i = (i0 > j + 1 ? i0 : j + 1); i < i1; ++i)
        s += (double)Cp[i * (i + 1) / 2 + j] * probe_sign(seed, i);
    wpart[band * n + j] = s;
}

// one block: residual = ||wrow + wcol - z|| / (||A||_F^2 sqrt(n))
__global__ __launch_bounds__(EW_THREADS) void res_final(const double* wrow, const double* wcol,
                                                        const double* z, const double* fro,
                                                        int64_t n, double* out) {
    __shared__ double s1[EW_THREADS], s2[EW_THREADS];
    double a = 0.0, f = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += EW_THREADS) {
        const double d = wrow[j] + wcol[j] - z[j];
        a += d * d;
        f += fro[j];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = f;
    __syncthreads();
    for (int s = EW_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double denom = s2[0] * sqrt((double)n);
        *out = denom > 0.0 ? sqrt(s1[0]) / denom : 0.0;
    }
}

unsigned blocks_for(int64_t items) { return (unsigned)((items + EW_THREADS - 1) / EW_THREADS); }

// Grid of the streaming kernels that walk virtual blocks.  A dispatch holds
// its size in work-items as a 32-bit count, so a launch of more than 2^32
// work-items would wrap; 2^20 workgroups of 256 fill the GPU many times over.
unsigned ew_grid(int64_t items) {
    const unsigned b = blocks_for(items);
    return b < (1u << 20) ? (b > 0 ? b : 1u) : (1u << 20);
}

// ------------------------------------------------- sampled-column check
// G[r][k] = A[r][cols[k]] in FP64 (the sampled columns, gathered once).
template <class T>
__global__ __launch_bounds__(EW_THREADS) void cc_gather(const T* A, int64_t m, int64_t lda, const int64_t* cols,
                                                        int64_t count, double* G) {
    const int64_t x = (int64_t)blockIdx.x * EW_THREADS + threadIdx.x;
    if (x >= m * count) return;
    const int64_t r = udiv(x, count), k = x - r * count;
    G[x] = (double)A[r * lda + cols[k]];
}

// Exact-as-FP64 reference columns (A^T A)[:, cols[s0 .. s0 + 15]] for the 64
// output rows i0 .. i0 + 63 of a workgroup: lane l takes row i0 + l, wave w a
// quarter of A's rows, products and sums in FP64 (a product of two FP32
// values is exact in FP64); the quarters are added in wave order.  Then
// per-workgroup sums of (C - ref)^2 and ref^2 over its outputs, C read from
// the packed lower triangle.  out[2 b], out[2 b + 1] for workgroup b.
template <class T>
__global__ __launch_bounds__(EW_THREADS) void cc_check(const T* A, int64_t m, int64_t n, int64_t lda,
                                                       const double* G, const int64_t* cols, int64_t count,
                                                       const T* Cp, double* out) {
    __shared__ double red[3][64][16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const int64_t s0 = (int64_t)blockIdx.y * 16;
    const int ns = count - s0 < 16 ? (int)(count - s0) : 16;
    const int64_t q = (m + 3) / 4;
    const int64_t r0 = wave * q < m ? wave * q : m, r1 = (wave + 1) * q < m ? (wave + 1) * q : m;
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    if (i < n) {
        for (int64_t r = r0; r < r1; ++r) {
            const double a = (double)A[r * lda + i];
            const double* g = G + r * count + s0;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < ns) acc[k] = fma(a, g[k], acc[k]);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) red[wave - 1][lane][k] = acc[k];
    }
    __syncthreads();
    double d2 = 0.0, r2 = 0.0;
    if (wave == 0 && i < n) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k >= ns) continue;
            const double ref = acc[k] + red[0][lane][k] + red[1][lane][k] + red[2][lane][k];
            const int64_t j = cols[s0 + k];
            const double c = (double)(i >= j ? Cp[packed_index(i, j)] : Cp[packed_index(j, i)]);
            d2 += (c - ref) * (c - ref);
            r2 += ref * ref;
        }
    }
    // wave 0 sums its lanes in a fixed tree order
    if (wave == 0) {
        for (int off = 32; off > 0; off >>= 1) {
            d2 += __shfl_down(d2, off, 64);
            r2 += __shfl_down(r2, off, 64);
        }
        if (lane == 0) {
            const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            out[2 * b] = d2;
            out[2 * b + 1] = r2;
        }
    }
}

}  // namespace

hipError_t launch_presum(int32_t mode, const PresumDesc* d_tasks, int ntasks, int64_t items,
                         const void* A, void* arena, const uint8_t* flags, hipStream_t stream,
                         const BatchPtrs* bp, const void* B) {
    if (items <= 0) return hipSuccess;
    const void* const* Ap = bp ? bp->A : nullptr;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(presum_kernel<double>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<const double*>(A),
                           static_cast<double*>(arena), flags, Ap, static_cast<const double*>(B));
    else
        hipLaunchKernelGGL(presum_kernel<float>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<const float*>(A),
                           static_cast<float*>(arena), flags, Ap, static_cast<const float*>(B));
    return hipGetLastError();
}

hipError_t launch_pack(const PackDesc* d_tasks, int ntasks, int64_t items, const void* A,
                       void* arena, const uint8_t* flags, hipStream_t stream, const BatchPtrs* bp,
                       const void* B) {
    if (items <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream, d_tasks,
                       ntasks, items, static_cast<const float*>(A), static_cast<float*>(arena), flags,
                       bp ? bp->A : nullptr, static_cast<const float*>(B));
    return hipGetLastError();
}

hipError_t launch_quant8(const Pack8Desc* d_tasks, int ntasks, int64_t blocks, const void* A,
                         void* arena, const uint8_t* flags, hipStream_t stream, const BatchPtrs* bp,
                         const void* B, double* partial) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(quant8_kernel, dim3((unsigned)blocks), dim3(EW_THREADS), 0, stream, d_tasks,
                       ntasks, static_cast<const float*>(A), static_cast<float*>(arena), flags,
                       bp ? bp->A : nullptr, static_cast<const float*>(B), partial);
    return hipGetLastError();
}

hipError_t launch_reduce(int32_t mode, const ReduceDesc* d_tasks, int ntasks, int64_t items, void* C,
                         void* arena, const uint8_t* flags, hipStream_t stream, const BatchPtrs* bp) {
    if (items <= 0) return hipSuccess;
    void* const* Cp = bp ? bp->C : nullptr;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(reduce_kernel<double>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<double*>(C), static_cast<double*>(arena), flags, Cp);
    else
        hipLaunchKernelGGL(reduce_kernel<float>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<float*>(C), static_cast<float*>(arena), flags, Cp);
    return hipGetLastError();
}

hipError_t launch_axpby(int32_t mode, const void* t, void* c, int64_t len, double alpha, double beta,
                        hipStream_t stream) {
    if (len <= 0) return hipSuccess;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(axpby_kernel<double>, dim3(ew_grid(len)), dim3(EW_THREADS), 0, stream,
                           static_cast<const double*>(t), static_cast<double*>(c), len, alpha, beta);
    else
        hipLaunchKernelGGL(axpby_kernel<float>, dim3(ew_grid(len)), dim3(EW_THREADS), 0, stream,
                           static_cast<const float*>(t), static_cast<float*>(c), len, (float)alpha, (float)beta);
    return hipGetLastError();
}

hipError_t launch_transpose(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda, void* At,
                            hipStream_t stream) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
    if (mode == MODE_F64)
        hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(EW_THREADS), 0, stream,
                           static_cast<const double*>(A), m, n, lda, static_cast<double*>(At));
    else
        hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(EW_THREADS), 0, stream,
                           static_cast<const float*>(A), m, n, lda, static_cast<float*>(At));
    return hipGetLastError();
}

hipError_t launch_unpack(int32_t mode, const void* Cp, int64_t n, void* F, int64_t ldf, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(unpack_kernel<double>, dim3(ew_grid(n * n)), dim3(EW_THREADS), 0, stream,
                           static_cast<const double*>(Cp), n, static_cast<double*>(F), ldf);
    else
        hipLaunchKernelGGL(unpack_kernel<float>, dim3(ew_grid(n * n)), dim3(EW_THREADS), 0, stream,
                           static_cast<const float*>(Cp), n, static_cast<float*>(F), ldf);
    return hipGetLastError();
}

hipError_t launch_eq_scale(const float* A, int64_t m, int64_t n, int64_t lda, const double* nu, float* Ap,
                           int* e, hipStream_t stream) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eq_scale_kernel, dim3(ew_grid(m * n)), dim3(EW_THREADS), 0, stream, A, m, n, lda, nu,
                       Ap, e);
    return hipGetLastError();
}

hipError_t launch_eq_unscale(float* Cp, int64_t n, const int* e, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eq_unscale_kernel, dim3(ew_grid(n * (n + 1) / 2)), dim3(EW_THREADS), 0, stream, Cp, n, e);
    return hipGetLastError();
}

namespace {

// Bounded workspace: one pre-sum on its own, one element per work item
// (consecutive items are consecutive columns of a row).
template <class T>
__global__ __launch_bounds__(EW_THREADS) void sum2_kernel(const Sum2Desc* tasks, int ntasks, int64_t items,
                                                          const T* A, T* arena, const uint8_t* flags) {
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x) {
        const int64_t x = vb * EW_THREADS + threadIdx.x;
        if (x >= items) continue;
        const Sum2Desc& d = tasks[block_task(tasks, ntasks, vb)];
        const int64_t e = x - d.elem_begin;
        if (e >= d.elems) continue;
        if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) continue;
        const int64_t r = udiv(e, d.cols), c = e - r * d.cols;
        auto get = [&](const View& v) -> T {
            const T* base = (v.base == BASE_A ? A : arena) + v.off;
            return r < v.prows && c < v.pcols ? base[r * v.ld + c] : T(0);
        };
        const T a = get(d.a), b = get(d.b);
        arena[d.out_off + e] = d.sign > 0 ? a + b : a - b;
    }
}

// Bounded workspace: product i of a root into its one or two quadrants (the
// first contribution overwrites), one product element per work item.
template <class T>
__global__ __launch_bounds__(EW_THREADS) void accum_kernel(const AccumDesc* tasks, int ntasks, int64_t items,
                                                           T* C, T* arena, const uint8_t* flags) {
    for (int64_t vb = blockIdx.x; vb * EW_THREADS < items; vb += gridDim.x) {
        const int64_t x = vb * EW_THREADS + threadIdx.x;
        if (x >= items) continue;
        const AccumDesc& d = tasks[block_task(tasks, ntasks, vb)];
        const int64_t e = x - d.elem_begin;
        if (e >= d.elems) continue;
        if (d.pred_node >= 0 && (int32_t)flags[d.pred_node] != d.pred_value) continue;
        const int64_t i = udiv(e, d.k2), j = e - i * d.k2;
        const T m = arena[d.m_off + e];
        for (int q = 0; q < d.nq; ++q) {
            const int quad = d.quad[q];
            const int64_t ro = quad >= 2 ? d.n1 : 0, co = (quad & 1) ? d.k1 : 0;
            const int64_t rl = quad >= 2 ? d.n2 : d.n1, cl = (quad & 1) ? d.k2 : d.k1;
            if (i >= rl || j >= cl) continue;
            const int64_t ii = ro + i, jj = co + j;
            T* p = d.out_kind == OUT_PACKED ? C + packed_index(d.out_row0 + ii, d.out_col0 + jj)
                   : d.out_kind == OUT_CDENSE ? C + (d.out_row0 + ii) * d.out_ld + d.out_col0 + jj
                                              : arena + d.out_off + ii * d.out_ld + jj;
            *p = d.first[q] ? m : d.sign[q] > 0 ? *p + m : *p - m;
        }
    }
}

}  // namespace

hipError_t launch_sum2(int32_t mode, const Sum2Desc* d_tasks, int ntasks, int64_t items, const void* A,
                       void* arena, const uint8_t* flags, hipStream_t stream) {
    if (items <= 0) return hipSuccess;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(sum2_kernel<double>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream, d_tasks, ntasks,
                           items, static_cast<const double*>(A), static_cast<double*>(arena), flags);
    else
        hipLaunchKernelGGL(sum2_kernel<float>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream, d_tasks, ntasks,
                           items, static_cast<const float*>(A), static_cast<float*>(arena), flags);
    return hipGetLastError();
}

hipError_t launch_accum(int32_t mode, const AccumDesc* d_tasks, int ntasks, int64_t items, void* C, void* arena,
                        const uint8_t* flags, hipStream_t stream) {
    if (items <= 0) return hipSuccess;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(accum_kernel<double>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream, d_tasks, ntasks,
                           items, static_cast<double*>(C), static_cast<double*>(arena), flags);
    else
        hipLaunchKernelGGL(accum_kernel<float>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream, d_tasks, ntasks,
                           items, static_cast<float*>(C), static_cast<float*>(arena), flags);
    return hipGetLastError();
}

hipError_t launch_combine(int32_t mode, const CombineDesc* d_tasks, int ntasks, int64_t items,
                          void* C, void* arena, const uint8_t* flags, hipStream_t stream,
                          const BatchPtrs* bp) {
    if (items <= 0) return hipSuccess;
    void* const* Cp = bp ? bp->C : nullptr;
    if (mode == MODE_F64)
        hipLaunchKernelGGL(combine_kernel<double>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<double*>(C),
                           static_cast<double*>(arena), flags, Cp);
    else
        hipLaunchKernelGGL(combine_kernel<float>, dim3(ew_grid(items)), dim3(EW_THREADS), 0, stream,
                           d_tasks, ntasks, items, static_cast<float*>(C),
                           static_cast<float*>(arena), flags, Cp);
    return hipGetLastError();
}

int64_t residual_chunks(int64_t m) { return m <= 0 ? 1 : (m + NORM_ROWS - 1) / NORM_ROWS; }

hipError_t launch_colnorms(const ColDesc* d_pass1, int n1, int64_t items1, const ColDesc* d_pass2,
                           int n2, int64_t items2, const float* A, const void* const* Aptrs,
                           double* partial, double* nu, hipStream_t stream, void* arena, bool pack) {
    if (items1 > 0 && pack)
        hipLaunchKernelGGL(colnorm_pass1<true>, dim3(blocks_for(items1)), dim3(EW_THREADS), 0, stream,
                           d_pass1, n1, items1, A, Aptrs, partial, static_cast<float*>(arena));
    else if (items1 > 0)
        hipLaunchKernelGGL(colnorm_pass1<false>, dim3(blocks_for(items1)), dim3(EW_THREADS), 0, stream,
                           d_pass1, n1, items1, A, Aptrs, partial, static_cast<float*>(arena));
    if (items2 > 0)
        hipLaunchKernelGGL(colnorm_pass2, dim3(blocks_for(items2)), dim3(EW_THREADS), 0, stream,
                           d_pass2, n2, items2, partial, nu);
    return hipGetLastError();
}

hipError_t launch_flags(const double* nu, const NodeDesc* d_nodes, int nnodes, double tau2,
                        uint8_t* flags, hipStream_t stream) {
    if (nnodes <= 0) return hipSuccess;
    hipLaunchKernelGGL(flags_kernel, dim3(nnodes), dim3(EW_THREADS), 0, stream, nu, d_nodes, tau2, flags);
    return hipGetLastError();
}

int64_t residual_work_elems(int64_t m, int64_t n) {
    const int64_t chunks = residual_chunks(m), bands = (n + BAND - 1) / BAND;
    // y | zpart | fpart | z | fro | wrow | wpart | wcol
    return m + 2 * chunks * n + 2 * n + n + bands * n + n;
}

hipError_t launch_residual(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda,
                           const void* C, uint64_t seed, double* work, double* out,
                           hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t chunks = residual_chunks(m), bands = (n + BAND - 1) / BAND;
    double* y = work;
    double* zpart = y + m;
    double* fpart = zpart + chunks * n;
    double* z = fpart + chunks * n;
    double* fro = z + n;
    double* wrow = fro + n;
    double* wpart = wrow + n;
    double* wcol = wpart + bands * n;
    const dim3 blk(EW_THREADS);
    const unsigned rows_blocks = (unsigned)((m + 3) / 4), crow_blocks = (unsigned)((n + 3) / 4);
    if (mode == MODE_F64) {
        const double* a = static_cast<const double*>(A);
        const double* c = static_cast<const double*>(C);
        if (m > 0) hipLaunchKernelGGL(res_ax<double>, dim3(rows_blocks), blk, 0, stream, a, m, n, lda, seed, y);
        hipLaunchKernelGGL(res_aty<double>, dim3(blocks_for(n), (unsigned)chunks), blk, 0, stream, a, m, n, lda, y, zpart, fpart);
        hipLaunchKernelGGL(res_crow<double>, dim3(crow_blocks), blk, 0, stream, c, n, seed, wrow);
        hipLaunchKernelGGL(res_ccol<double>, dim3(blocks_for(n), (unsigned)bands), blk, 0, stream, c, n, seed, wpart);
    } else {
        const float* a = static_cast<const float*>(A);
        const float* c = static_cast<const float*>(C);
        if (m > 0) hipLaunchKernelGGL(res_ax<float>, dim3(rows_blocks), blk, 0, stream, a, m, n, lda, seed, y);
        hipLaunchKernelGGL(res_aty<float>, dim3(blocks_for(n), (unsigned)chunks), blk, 0, stream, a, m, n, lda, y, zpart, fpart);
        hipLaunchKernelGGL(res_crow<float>, dim3(crow_blocks), blk, 0, stream, c, n, seed, wrow);
        hipLaunchKernelGGL(res_ccol<float>, dim3(blocks_for(n), (unsigned)bands), blk, 0, stream, c, n, seed, wpart);
    }
    hipLaunchKernelGGL(sum_partials, dim3(blocks_for(n)), blk, 0, stream, zpart, chunks, n, z);
    hipLaunchKernelGGL(sum_partials, dim3(blocks_for(n)), blk, 0, stream, fpart, chunks, n, fro);
    hipLaunchKernelGGL(sum_partials, dim3(blocks_for(n)), blk, 0, stream, wpart, bands, n, wcol);
    hipLaunchKernelGGL(res_final, dim3(1), blk, 0, stream, wrow, wcol, z, fro, n, out);
    return hipGetLastError();
}

int64_t column_check_work_elems(int64_t m, int64_t n, int64_t count) {
    return m * count + 2 * ((n + 63) / 64) * ((count + 15) / 16);
}

hipError_t launch_column_check(int32_t mode, const void* A, int64_t m, int64_t n, int64_t lda, const void* C,
                               const int64_t* d_cols, int64_t count, double* work, hipStream_t stream) {
    if (n <= 0 || count <= 0) return hipSuccess;
    double* G = work;
    double* out = work + m * count;
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((count + 15) / 16));
    if (mode == MODE_F64) {
        const double* a = static_cast<const double*>(A);
        if (m > 0)
            hipLaunchKernelGGL(cc_gather<double>, dim3(blocks_for(m * count)), dim3(EW_THREADS), 0, stream, a, m, lda,
                               d_cols, count, G);
        hipLaunchKernelGGL(cc_check<double>, grid, dim3(EW_THREADS), 0, stream, a, m, n, lda, G, d_cols, count,
                           static_cast<const double*>(C), out);
    } else {
        const float* a = static_cast<const float*>(A);
        if (m > 0)
            hipLaunchKernelGGL(cc_gather<float>, dim3(blocks_for(m * count)), dim3(EW_THREADS), 0, stream, a, m, lda,
                               d_cols, count, G);
        hipLaunchKernelGGL(cc_check<float>, grid, dim3(EW_THREADS), 0, stream, a, m, n, lda, G, d_cols, count,
                           static_cast<const float*>(C), out);
    }
    return hipGetLastError();
}

}  // namespace ata
