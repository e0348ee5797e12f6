"""O1: ctypes wrapper over the plain FP64 C oracle (test infrastructure only).

The arithmetic lives in ``ata_oracle.c``: C[i][j] = sum_r A[r][i] A[r][j] in
ascending r, FP64, no fused multiply-add (Sec. 3.1, Eq. "Cij").  Pinned in
``tests/test_oracle_plain.py`` by hand-computed tiny cases, closed forms
(identity, orthonormal columns, rank one, all ones), symmetry / PSD /
diagonal invariants, the Freivalds identity x^T C x = ||A x||^2, and an
independent library product (numpy float64 matmul).  ``gemm_tn`` is the
plain general product A^T B of the Strassen step, pinned the same way.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.OUT
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i64, vp, dp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
        lib.oracle_gram_plain.argtypes = [vp, ctypes.c_int, i64, i64, i64, dp, ctypes.c_int]
        lib.oracle_gram_cols.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, i64, dp, ctypes.c_int]
        lib.oracle_colnorms.argtypes = [vp, ctypes.c_int, i64, i64, i64, dp, ctypes.c_int]
        lib.oracle_threads_used.argtypes = [ctypes.c_int]
        lib.oracle_gemm_tn.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i64, i64, dp, i64, ctypes.c_int]
        for f in (lib.oracle_gram_plain, lib.oracle_gram_cols, lib.oracle_colnorms,
                  lib.oracle_threads_used, lib.oracle_gemm_tn):
            f.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _as_input(A):
    A = np.asarray(A)
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    if A.dtype not in (np.float32, np.float64):
        A = A.astype(np.float64)
    if A.strides[1] != A.itemsize or A.strides[0] % A.itemsize:
        A = np.ascontiguousarray(A)
    lda = A.strides[0] // A.itemsize if A.shape[0] > 1 else A.shape[1]
    return A, int(A.dtype == np.float32), A.shape[0], A.shape[1], max(lda, A.shape[1])


def gemm_tn(A, B, nthreads: int = 0) -> np.ndarray:
    """Dense C = A^T B (n x k, FP64), A m x n and B m x k of one element type."""
    A, f32, m, n, lda = _as_input(A)
    B = np.asarray(B, dtype=A.dtype)
    B, f32b, mb, k, ldb = _as_input(B)
    if mb != m or f32b != f32:
        raise ValueError("A and B need the same rows and element type")
    C = np.empty((n, k), dtype=np.float64)
    rc = _lib().oracle_gemm_tn(A.ctypes.data, B.ctypes.data, f32, m, n, k, lda, ldb, C.ctypes.data,
                               max(k, 1), nthreads)
    if rc:
        raise ValueError("oracle_gemm_tn rejected its arguments")
    return C


def threads_used(nthreads: int = 0) -> int:
    return _lib().oracle_threads_used(nthreads)


def gram_packed(A, nthreads: int = 0) -> np.ndarray:
    """Packed lower C (length n(n+1)/2, FP64): Cp[i(i+1)/2 + j] = C[i][j]."""
    A, f32, m, n, lda = _as_input(A)
    Cp = np.empty(n * (n + 1) // 2, dtype=np.float64)
    rc = _lib().oracle_gram_plain(A.ctypes.data, f32, m, n, lda, Cp.ctypes.data, nthreads)
    if rc:
        raise ValueError("oracle_gram_plain rejected its arguments")
    return Cp


def gram_cols(A, S, nthreads: int = 0) -> np.ndarray:
    """Full columns C[:, S] as an (n, len(S)) FP64 array."""
    A, f32, m, n, lda = _as_input(A)
    S = np.ascontiguousarray(np.asarray(S, dtype=np.int64))
    out = np.empty((len(S), n), dtype=np.float64)
    rc = _lib().oracle_gram_cols(A.ctypes.data, f32, m, n, lda, S.ctypes.data, len(S),
                                 out.ctypes.data, nthreads)
    if rc:
        raise ValueError("oracle_gram_cols rejected its arguments")
    return out.T.copy()


def colnorms(A, nthreads: int = 0) -> np.ndarray:
    """Squared column norms nu_j = sum_r A[r][j]^2 (FP64)."""
    A, f32, m, n, lda = _as_input(A)
    nu = np.empty(n, dtype=np.float64)
    rc = _lib().oracle_colnorms(A.ctypes.data, f32, m, n, lda, nu.ctypes.data, nthreads)
    if rc:
        raise ValueError("oracle_colnorms rejected its arguments")
    return nu


def unpack(Cp, n: int) -> np.ndarray:
    """Full symmetric n x n matrix from row-major lower packed storage."""
    Cp = np.asarray(Cp)
    if Cp.shape != (n * (n + 1) // 2,):
        raise ValueError("packed length does not match n")
    C = np.zeros((n, n), dtype=Cp.dtype)
    rows, cols = np.tril_indices(n)
    C[rows, cols] = Cp
    C[cols, rows] = Cp
    return C
