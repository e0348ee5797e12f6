"""O2: the recursive AtA algorithm of Sec. 3, step by step, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This follows Alg. 1 ("AtA - Serial") and the Strassen description of Sec. 3.1
and Sec. 3.2 in the paper's order and notation, with counters for the
operations it performs.  Library matrix products stand in for the BLAS leaves
(``?syrk`` for AtA leaves, ``?gemm`` for Strassen leaves), as in the paper.

Readings of the paper used here:

* Partition (Eq. "submatA"): m1 = floor(m/2), m2 = ceil(m/2), n1 = floor(n/2),
  n2 = ceil(n/2); the leading blocks are the floor-sized ones; the fourth
  block, printed with the same label as the third, is A22 = A[m1:m, n1:n].
* Leaf rule: the paper stops when the block fits in a cache whose size it
  never states.  Here an AtA call is a leaf iff n <= b (or m <= 1, or n <= 1)
  and a Strassen call is a leaf iff max(n, k) <= b (or min(m, n, k) <= 1),
  or when an optional Strassen depth cap is reached.
* Strassen's formulas are not printed; the original seven-product scheme of
  Strassen (1969) is applied to the 2x2 blocks of X^T and Y, which for
  C = X^T Y gives the sums S1..S5 of X blocks and T1..T5 of Y blocks below.
* Odd sizes: no peeling and no padding of A; operands of a sum that are one
  row or column short count as if padded with a trailing zero row/column, so
  every temporary has the ceil dimensions and only the leading part of a
  product reaches a floor-sized block of C.  The oracle materialises those
  zero-padded operands (a copy, not counted as workspace).
* ``split_m=True`` is Alg. 1 literally (four AtA calls, two Strassen calls per
  level).  ``split_m=False`` keeps all m rows in every call (two AtA calls and
  one Strassen call per level); it performs the same multiplications and is
  the form the GPU plan mirrors.
* Workspace follows Sec. 3.3: one product buffer M plus one A-side sum buffer
  (P) and one B-side sum buffer (Q) live per Strassen level; each product is
  accumulated into its C quadrants as soon as it is formed, so a level holds
  at most one S, one T and one M at a time.  Counted in elements.

Pins (tests/test_oracle_recursive.py): bit-exact equality with O1 on
small-integer inputs for both forms; the multiplication count against the
closed form 2/3 n^log2(7) + 1/3 n^2 printed in Sec. 1 (leaf size 1) and its
leaf-size-b generalisation; 10 pre-sums, 7 products and 18 block sums per
Strassen level (Sec. 3.2); the Strassen-alone addition count 6(7^L - 4^L);
the workspace bound 3/2 n^2 of Sec. 3.3; FP64 agreement with O1 on random
inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Counters:
    mults: int = 0              # scalar multiplications in leaves
    leaf_adds: int = 0          # scalar additions inside leaves (one per multiply-accumulate)
    presum_blocks: int = 0      # block sums forming S1..S5, T1..T5
    presum_adds: int = 0        # element additions in those sums (real, unpadded operands)
    postsum_blocks: int = 0     # Strassen post-sums (8 per level, Sec. 3.2's 18 = 10 + 8)
    accum_blocks: int = 0       # block accumulations of products into C (12 per level)
    accum_adds: int = 0         # element additions of those accumulations
    syrk_leaves: int = 0
    gemm_leaves: int = 0
    ata_nodes: int = 0
    strassen_nodes: int = 0
    ws_live: int = 0            # live Strassen workspace (elements)
    ws_peak: int = 0
    ata_list: list = field(default_factory=list)      # (col0, w, is_leaf) of every AtA call
    syrk_list: list = field(default_factory=list)     # (row0, col0, m, w) of AtA leaves
    strassen_roots: list = field(default_factory=list)  # (xcol0, ycol0, m, n, k, levels, mults)

    def alloc(self, elems: int) -> None:
        self.ws_live += elems
        self.ws_peak = max(self.ws_peak, self.ws_live)

    def free(self, elems: int) -> None:
        self.ws_live -= elems


def _halves(x: int):
    return x // 2, x - x // 2


def _padded(B: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """B with trailing zero rows/columns up to rows x cols (simulated padding)."""
    if B.shape == (rows, cols):
        return B
    if B.strides == (0, 0):                      # dry run: shape only
        return np.broadcast_to(np.float64(0), (rows, cols))
    out = np.zeros((rows, cols), dtype=np.float64)
    out[: B.shape[0], : B.shape[1]] = B
    return out


class _Recursion:
    def __init__(self, b: int, split_m: bool, max_strassen_depth: int | None,
                 ctr: Counters, leaf_product=None, round_sum=None, dry: bool = False):
        self.dry = dry          # walk the recursion for its counts only, no arithmetic
        self.b = b
        self.split_m = split_m
        self.max_depth = max_strassen_depth
        self.ctr = ctr
        # leaf arithmetic: X^T Y of the leaf operands (FP64 by default; the
        # reduced-precision emulations in ``emulate`` substitute their own)
        self.leaf_product = leaf_product or (lambda X, Y: X.T @ Y)
        # rounding applied to every Strassen pre-sum (identity in FP64)
        self.round_sum = round_sum or (lambda S: S)

    # --- Alg. 1, procedure AtA: lower(C) += A^T A ---------------------------
    def ata(self, A: np.ndarray, C: np.ndarray, row0: int, col0: int) -> None:
        ctr = self.ctr
        ctr.ata_nodes += 1
        m, n = A.shape
        is_leaf = n <= self.b or m <= 1 or n <= 1
        ctr.ata_list.append((col0, n, is_leaf))
        if is_leaf:
            # base case: ?syrk on the lower triangle of this diagonal block
            ctr.syrk_leaves += 1
            ctr.syrk_list.append((row0, col0, m, n))
            ctr.mults += m * n * (n + 1) // 2
            ctr.leaf_adds += m * n * (n + 1) // 2
            if not self.dry:
                C += np.tril(self.leaf_product(A, A))
            return
        m1, m2 = _halves(m)
        n1, n2 = _halves(n)
        C11 = C[:n1, :n1]
        C21 = C[n1:, :n1]
        C22 = C[n1:, n1:]
        if self.split_m:
            A11, A12 = A[:m1, :n1], A[:m1, n1:]
            A21, A22 = A[m1:, :n1], A[m1:, n1:]
            self.ata(A11, C11, row0, col0)
            self.ata(A21, C11, row0 + m1, col0)
            self.ata(A12, C22, row0, col0 + n1)
            self.ata(A22, C22, row0 + m1, col0 + n1)
            self.fast_strassen(A12, A11, C21, col0 + n1, col0)
            self.fast_strassen(A22, A21, C21, col0 + n1, col0)
        else:
            self.ata(A[:, :n1], C11, row0, col0)
            self.ata(A[:, n1:], C22, row0, col0 + n1)
            self.fast_strassen(A[:, n1:], A[:, :n1], C21, col0 + n1, col0)

    # --- Alg. 1, procedure FastStrassen: C += X^T Y ---------------------------
    def fast_strassen(self, X, Y, C, xcol0: int, ycol0: int) -> None:
        before = self.ctr.mults
        levels = self.strassen(X, Y, C, 0)
        m, n = X.shape
        k = Y.shape[1]
        self.ctr.strassen_roots.append((xcol0, ycol0, m, n, k, levels,
                                        self.ctr.mults - before))

    def strassen(self, X: np.ndarray, Y: np.ndarray, C: np.ndarray, depth: int) -> int:
        """C += X^T Y by Strassen's scheme; returns the number of levels below."""
        ctr = self.ctr
        m, n = X.shape
        k = Y.shape[1]
        assert Y.shape[0] == m and C.shape == (n, k)
        capped = self.max_depth is not None and depth >= self.max_depth
        if max(n, k) <= self.b or min(m, n, k) <= 1 or capped:
            # base case: ?gemm
            ctr.gemm_leaves += 1
            ctr.mults += m * n * k
            ctr.leaf_adds += m * n * k
            if not self.dry:
                C += self.leaf_product(X, Y)
            return 0
        ctr.strassen_nodes += 1
        m1, m2 = _halves(m)
        n1, n2 = _halves(n)
        k1, k2 = _halves(k)
        # 2x2 blocks of X (m x n) and Y (m x k), leading blocks floor-sized
        X11, X12 = X[:m1, :n1], X[:m1, n1:]
        X21, X22 = X[m1:, :n1], X[m1:, n1:]
        Y11, Y12 = Y[:m1, :k1], Y[:m1, k1:]
        Y21, Y22 = Y[m1:, :k1], Y[m1:, k1:]
        # quadrants of C (n x k)
        C11, C12 = C[:n1, :k1], C[:n1, k1:]
        C21, C22 = C[n1:, :k1], C[n1:, k1:]

        def P(B):  # operand of X-side shape, simulated padding to m2 x n2
            return _padded(B, m2, n2)

        def Q(B):  # operand of Y-side shape, simulated padding to m2 x k2
            return _padded(B, m2, k2)

        def presum(a, b_, sign, shape_fn):
            ctr.presum_blocks += 1
            ctr.presum_adds += min(a.shape[0], b_.shape[0]) * min(a.shape[1], b_.shape[1])
            if self.dry:
                return np.broadcast_to(np.float64(0), shape_fn(a).shape)
            return self.round_sum(shape_fn(a) + sign * shape_fn(b_))

        def accumulate(dst, Mi, sign):
            ctr.accum_blocks += 1
            ctr.accum_adds += dst.size
            if not self.dry:
                dst += sign * Mi[: dst.shape[0], : dst.shape[1]]

        levels = 0

        def product(S, T, need_s: bool, need_t: bool):
            nonlocal levels
            if need_s:
                ctr.alloc(m2 * n2)
            if need_t:
                ctr.alloc(m2 * k2)
            ctr.alloc(n2 * k2)
            if self.dry:
                Mi = np.broadcast_to(np.float64(0), (n2, k2))
            else:
                Mi = np.zeros((n2, k2), dtype=np.float64)
            levels = max(levels, 1 + self.strassen(S, T, Mi, depth + 1))
            return Mi

        def release(need_s: bool, need_t: bool):
            ctr.free(n2 * k2)
            if need_t:
                ctr.free(m2 * k2)
            if need_s:
                ctr.free(m2 * n2)

        # M1 = (X11 + X22)^T (Y11 + Y22)
        S1 = presum(X11, X22, +1, P)
        T1 = presum(Y11, Y22, +1, Q)
        M1 = product(S1, T1, True, True)
        accumulate(C11, M1, +1)
        accumulate(C22, M1, +1)
        release(True, True)
        # M2 = (X12 + X22)^T Y11
        S2 = presum(X12, X22, +1, P)
        M2 = product(S2, Q(Y11), True, False)
        accumulate(C21, M2, +1)
        accumulate(C22, M2, -1)
        release(True, False)
        # M3 = X11^T (Y12 - Y22)
        T2 = presum(Y12, Y22, -1, Q)
        M3 = product(P(X11), T2, False, True)
        accumulate(C12, M3, +1)
        accumulate(C22, M3, +1)
        release(False, True)
        # M4 = X22^T (Y21 - Y11)
        T3 = presum(Y21, Y11, -1, Q)
        M4 = product(P(X22), T3, False, True)
        accumulate(C11, M4, +1)
        accumulate(C21, M4, +1)
        release(False, True)
        # M5 = (X11 + X21)^T Y22
        S3 = presum(X11, X21, +1, P)
        M5 = product(S3, Q(Y22), True, False)
        accumulate(C11, M5, -1)
        accumulate(C12, M5, +1)
        release(True, False)
        # M6 = (X12 - X11)^T (Y11 + Y12)
        S4 = presum(X12, X11, -1, P)
        T4 = presum(Y11, Y12, +1, Q)
        M6 = product(S4, T4, True, True)
        accumulate(C22, M6, +1)
        release(True, True)
        # M7 = (X21 - X22)^T (Y21 + Y22)
        S5 = presum(X21, X22, -1, P)
        T5 = presum(Y21, Y22, +1, Q)
        M7 = product(S5, T5, True, True)
        accumulate(C11, M7, +1)
        release(True, True)
        # the 12 accumulations are Strassen's 8 post-sums plus the 4 updates
        # C_ij += (sum), i.e. C11 = M1+M4-M5+M7, C12 = M3+M5, C21 = M2+M4,
        # C22 = M1-M2+M3+M6
        ctr.postsum_blocks += 8
        return levels


def ata(A, b: int, split_m: bool = True, max_strassen_depth: int | None = None,
        leaf_product=None, round_sum=None):
    """Packed lower C (FP64) and the counters of the recursive AtA.

    ``b`` is the leaf cutoff (Sec. 3.1 base case), ``split_m`` picks Alg. 1's
    literal four-way AtA recursion or the rows-kept form, and
    ``max_strassen_depth`` caps the Strassen levels under each AtA node.
    ``leaf_product(X, Y)`` replaces the FP64 leaf product X^T Y and
    ``round_sum`` rounds each Strassen pre-sum (used by the reduced-precision
    emulations; both default to exact FP64).
    """
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    if b < 1:
        raise ValueError("leaf cutoff b must be >= 1")
    m, n = A.shape
    ctr = Counters()
    C = np.zeros((n, n), dtype=np.float64)
    if n > 0 and m > 0:
        _Recursion(b, split_m, max_strassen_depth, ctr, leaf_product,
                   round_sum).ata(A, C, 0, 0)
    rows, cols = np.tril_indices(n)
    return C[rows, cols].copy(), ctr


def strassen_product(X, Y, b: int, max_depth: int | None = None):
    """FastStrassen alone: X^T Y (FP64, full n x k) and its counters."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    ctr = Counters()
    C = np.zeros((X.shape[1], Y.shape[1]), dtype=np.float64)
    _Recursion(b, False, max_depth, ctr).strassen(X, Y, C, 0)
    return C, ctr


def mults_closed_form(n: int, b: int) -> int:
    """Multiplications of AtA on a square n = b * 2^L matrix down to leaf b.

    From the recurrence AtA(n) = 4 AtA(n/2) + 2 S(n/2), S(n) = 7 S(n/2),
    AtA(b) = b^2 (b+1)/2, S(b) = b^3: (2 b^3 / 3) 7^L + (b^2 (3 - b) / 6) 4^L.
    For b = 1 this is the 2/3 n^log2(7) + 1/3 n^2 stated in Sec. 1.
    """
    L = 0
    while b << L < n:
        L += 1
    if b << L != n:
        raise ValueError("n must be b times a power of two")
    num = 4 * b ** 3 * 7 ** L + b * b * (3 - b) * 4 ** L
    assert num % 6 == 0
    return num // 6


def count(m: int, n: int, b: int, split_m: bool = False,
          max_strassen_depth: int | None = None) -> Counters:
    """Counters of the recursion on an m x n input without doing arithmetic.

    Walks exactly the code path of ``ata`` on shape-only (zero-stride) arrays.
    """
    ctr = Counters()
    if m > 0 and n > 0:
        A = np.broadcast_to(np.float64(0), (m, n))
        C = np.broadcast_to(np.float64(0), (n, n))
        _Recursion(b, split_m, max_strassen_depth, ctr, dry=True).ata(A, C, 0, 0)
    return ctr
