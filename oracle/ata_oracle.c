/*
 * Plain FP64 oracle for the Gram product C = A^T A (lower triangle, packed).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links or calls this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes is the plain definition the AtA method reaches exactly in
 * exact arithmetic (Sec. 3.1, Eq. "Cij": every block of C is a sum of block
 * products of A, and only the lower triangle is kept because C is symmetric):
 *
 *     C[i][j] = sum_{r = 0}^{m-1} A[r][i] * A[r][j],      0 <= j <= i < n,
 *
 * with every entry summed in ascending r, each product rounded to double and
 * then added (built with -ffp-contract=off, so no fused multiply-add).  Input
 * elements are promoted exactly to double (float -> double is exact).
 *
 * Storage conventions:
 *   A is row-major, element (r, c) at A[r * lda + c], lda >= n.
 *   Packed lower C: element (i, j), j <= i, at Cp[i * (i + 1) / 2 + j]
 *   (row-major lower packed; Sec. 4.3.1 packs the lower triangle of A^T A
 *   partial results but does not fix an element order).
 *
 * The loop order (r outside j) only changes which independent entry is
 * visited when; the per-entry sum is still the ascending-r sum above, so the
 * bits do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

static inline double elem(const void* A, int is_f32, int64_t idx) {
    return is_f32 ? (double)((const float*)A)[idx] : ((const double*)A)[idx];
}

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int oracle_threads_used(int nthreads) {
    set_threads(nthreads);
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
}

/* O1: lower(C) = A^T A, packed, plain definition.  Returns 0 on success. */
int oracle_gram_plain(const void* A, int is_f32, int64_t m, int64_t n, int64_t lda,
                      double* Cp, int nthreads) {
    if (m < 0 || n < 0 || lda < n || (n > 0 && !Cp)) return 1;
    set_threads(nthreads);
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < n; ++i) {
        double* Ci = Cp + i * (i + 1) / 2;
        for (int64_t j = 0; j <= i; ++j) Ci[j] = 0.0;
        for (int64_t r = 0; r < m; ++r) {
            const int64_t row = r * lda;
            const double ari = elem(A, is_f32, row + i);
            if (is_f32) {
                const float* Ar = (const float*)A + row;
                for (int64_t j = 0; j <= i; ++j) Ci[j] += ari * (double)Ar[j];
            } else {
                const double* Ar = (const double*)A + row;
                for (int64_t j = 0; j <= i; ++j) Ci[j] += ari * Ar[j];
            }
        }
    }
    return 0;
}

/*
 * Sampled full columns of C: out[s * n + i] = C[i][S[s]] for all i in [0, n)
 * (both triangles, by symmetry C[i][j] = C[j][i]).  Same per-entry ascending-r
 * sum, hence bit-identical to the packed O1 entries.  Threads split i.
 */
int oracle_gram_cols(const void* A, int is_f32, int64_t m, int64_t n, int64_t lda,
                     const int64_t* S, int64_t ns, double* out, int nthreads) {
    if (m < 0 || n < 0 || lda < n || ns < 0 || (ns > 0 && (!S || !out))) return 1;
    for (int64_t s = 0; s < ns; ++s)
        if (S[s] < 0 || S[s] >= n) return 1;
    set_threads(nthreads);
    memset(out, 0, sizeof(double) * (size_t)(ns * n));
#pragma omp parallel
    {
        const int nt = omp_get_num_threads();
        const int t = omp_get_thread_num();
        const int64_t i0 = n * t / nt, i1 = n * (t + 1) / nt;
        for (int64_t r = 0; r < m; ++r) {
            const int64_t row = r * lda;
            for (int64_t s = 0; s < ns; ++s) {
                const double ars = elem(A, is_f32, row + S[s]);
                double* o = out + s * n;
                if (is_f32) {
                    const float* Ar = (const float*)A + row;
                    for (int64_t i = i0; i < i1; ++i) o[i] += (double)Ar[i] * ars;
                } else {
                    const double* Ar = (const double*)A + row;
                    for (int64_t i = i0; i < i1; ++i) o[i] += Ar[i] * ars;
                }
            }
        }
    }
    return 0;
}

/* Squared column norms nu[j] = sum_r A[r][j]^2, ascending r, FP64. */
int oracle_colnorms(const void* A, int is_f32, int64_t m, int64_t n, int64_t lda,
                    double* nu, int nthreads) {
    if (m < 0 || n < 0 || lda < n || (n > 0 && !nu)) return 1;
    set_threads(nthreads);
    for (int64_t j = 0; j < n; ++j) nu[j] = 0.0;
#pragma omp parallel
    {
        const int nt = omp_get_num_threads();
        const int t = omp_get_thread_num();
        const int64_t j0 = n * t / nt, j1 = n * (t + 1) / nt;
        for (int64_t r = 0; r < m; ++r)
            for (int64_t j = j0; j < j1; ++j) {
                const double a = elem(A, is_f32, r * lda + j);
                nu[j] += a * a;
            }
    }
    return 0;
}

/* General product of the Strassen step (Sec. 3.1, Eq. "Cij": the off-diagonal
 * block of AtA is a product X^T Y of two column blocks), written out plainly:
 *
 *     C[i][j] = sum_{r = 0}^{m-1} A[r][i] * B[r][j],   0 <= i < n, 0 <= j < k,
 *
 * ascending r, FP64, no fused multiply-add.  A is m x n (lda), B is m x k
 * (ldb), both of the same element type; C is n x k dense row-major (ldc).
 * Threads split the rows i of C; each entry's sum keeps the ascending-r
 * order, so the bits do not depend on the thread count. */
int oracle_gemm_tn(const void* A, const void* B, int is_f32, int64_t m, int64_t n, int64_t k,
                   int64_t lda, int64_t ldb, double* C, int64_t ldc, int nthreads) {
    if (m < 0 || n < 0 || k < 0 || lda < n || ldb < k || ldc < k || (n > 0 && k > 0 && !C)) return 1;
    set_threads(nthreads);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) C[i * ldc + j] = 0.0;
#pragma omp parallel
    {
        const int nt = omp_get_num_threads();
        const int t = omp_get_thread_num();
        const int64_t i0 = n * t / nt, i1 = n * (t + 1) / nt;
        for (int64_t r = 0; r < m; ++r) {
            for (int64_t i = i0; i < i1; ++i) {
                const double ari = elem(A, is_f32, r * lda + i);
                double* Ci = C + i * ldc;
                for (int64_t j = 0; j < k; ++j) Ci[j] += ari * elem(B, is_f32, r * ldb + j);
            }
        }
    }
    return 0;
}
