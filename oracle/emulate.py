"""CPU emulation of the reduced-precision modes, spread flags and the residual.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes in one IEEE precision throughout and says nothing about
mixed precision; the definitions below are this project's readings, each
written from the format definitions rather than from any library:

* split-BF16: hi = bf16_RNE(a), lo = bf16_RNE(a - hi) (a - hi is exact in
  FP32); a leaf product X^T Y becomes Xh^T Yh + Xh^T Yl + Xl^T Yh (the
  lo * lo term is dropped).
* block-scaled FP8: the OCP e4m3 ("fn") format -- 4 exponent bits with bias 7,
  3 mantissa bits, subnormals, no infinities, largest finite 448.  Every leaf
  operand is cut into 128 x 128 blocks aligned to its own first row and
  column; each block gets the power-of-two scale s = 2^e with the smallest e
  such that amax <= 448 * 2^e (s = 1 for an all-zero block), and its elements
  become q = e4m3_RNE(a / s).  The dequantised value q * s is exact in FP64.
* spread flag of an AtA node (a set of columns): with nu_j the squared column
  norms, spread = max nu / min nu over the node's nonzero columns (1 if fewer
  than two are nonzero); the node is flagged when spread > tau^2, tau being a
  bound on the ratio of column norms.
* Freivalds probe: x in {-1, +1}^n with x_j = +1 iff the top bit of
  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) at counter j of stream
  ``seed`` is 0; residual = ||C x - A^T (A x)||_2 / (||A||_F^2 ||x||_2).

Pins live in tests/test_oracle_emulate.py: RNE to bf16 against an integer
rounding of the bit pattern; the e4m3 rounding against torch's
``float8_e4m3fn`` cast and against hand-listed codes; the scale rule at and
around powers of two; the emulated products against exact FP64 on operands
that are already representable; SplitMix64 against the published first
outputs for seed 0 (fixture ``tests/golden/splitmix64.txt``); the residual's
value and normalisation on hand-computed cases
(``tests/golden/freivalds_hand.txt``); the recursion with Strassen levels
bit-exact against the plain FP64 product on small integers in both modes, and
the FP32 rounding of the pre-sums on a hand-derived two-level case
(``tests/golden/emulated_presum_rounding.txt``).
"""
from __future__ import annotations

import numpy as np

from . import recursive

# ----------------------------------------------------------------- split-BF16


def bf16_rne(a) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); float32 out.

    bfloat16 keeps the top 16 bits of the float32 pattern, so RNE is: add
    0x7FFF plus the lowest kept bit to the pattern, then clear the low 16
    bits.  NaN is not produced by the inputs used here.
    """
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + keep_lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def split_bf16(a):
    """(hi, lo) as float32 arrays holding bfloat16 values."""
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_rne(a)
    lo = bf16_rne(a - hi)          # a - hi is exact in float32
    return hi, lo


def bf16x3_product(X, Y) -> np.ndarray:
    """Xh^T Yh + Xh^T Yl + Xl^T Yh in FP64 (operands are rounded to float32 first)."""
    Xh, Xl = split_bf16(np.asarray(X, dtype=np.float32))
    Yh, Yl = split_bf16(np.asarray(Y, dtype=np.float32))
    Xh, Xl, Yh, Yl = (t.astype(np.float64) for t in (Xh, Xl, Yh, Yl))
    return Xh.T @ Yh + Xh.T @ Yl + Xl.T @ Yh


# ------------------------------------------------------------------ FP8 e4m3

E4M3_MAX = 448.0


def e4m3_values() -> np.ndarray:
    """All non-negative finite e4m3fn values, indexed by their 7-bit code."""
    vals = []
    for code in range(128):
        e, mant = code >> 3, code & 7
        if e == 15 and mant == 7:
            vals.append(np.nan)          # S.1111.111 is NaN; no infinities
        elif e == 0:
            vals.append(mant / 8.0 * 2.0 ** -6)
        else:
            vals.append((1.0 + mant / 8.0) * 2.0 ** (e - 7))
    return np.array(vals, dtype=np.float64)


_E4M3 = e4m3_values()[:127]              # finite magnitudes, ascending with the code


def e4m3_rne(x) -> np.ndarray:
    """Nearest e4m3fn value (ties to the even code), |x| must be <= 448."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    if np.any(ax > E4M3_MAX):
        raise ValueError("value outside the e4m3 range")
    hi_idx = np.searchsorted(_E4M3, ax, side="left")       # first value >= ax
    hi_idx = np.minimum(hi_idx, len(_E4M3) - 1)
    lo_idx = np.maximum(hi_idx - 1, 0)
    lo, hi = _E4M3[lo_idx], _E4M3[hi_idx]
    exact = hi == ax
    d_lo, d_hi = ax - lo, hi - ax
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (hi_idx % 2 == 0))
    code = np.where(exact, hi_idx, np.where(pick_hi, hi_idx, lo_idx))
    return np.sign(x) * _E4M3[code]


def pow2_scale_exponent(amax: float) -> int:
    """Smallest e with amax <= 448 * 2^e, computed exactly (amax > 0).

    448 = 0.875 * 2^9.  With amax = f * 2^E, f in [0.5, 1): e = E - 9 when
    f <= 0.875, else E - 8.
    """
    f, E = np.frexp(amax)
    return int(E - 9) if f <= 0.875 else int(E - 8)


def quantize_fp8(X, block: int = 128):
    """Block-quantise one leaf operand; returns (dequantised FP64, exponents)."""
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    out = np.zeros_like(X)
    exps = np.zeros(((m + block - 1) // block, (n + block - 1) // block), dtype=np.int64)
    for bi, r0 in enumerate(range(0, m, block)):
        for bj, c0 in enumerate(range(0, n, block)):
            blk = X[r0:r0 + block, c0:c0 + block]
            amax = float(np.max(np.abs(blk))) if blk.size else 0.0
            e = pow2_scale_exponent(amax) if amax > 0 else 0
            exps[bi, bj] = e
            out[r0:r0 + block, c0:c0 + block] = e4m3_rne(np.ldexp(blk, -e)) * 2.0 ** e
    return out, exps


def fp8_product(X, Y) -> np.ndarray:
    """deq(q(X))^T deq(q(Y)) in FP64 with per-operand 128 x 128 block scales."""
    Xd, _ = quantize_fp8(np.asarray(X, dtype=np.float32))
    Yd, _ = quantize_fp8(np.asarray(Y, dtype=np.float32))
    return Xd.T @ Yd


def _round_f32(S):
    return S.astype(np.float32).astype(np.float64)


def ata_emulated(A, mode: str, b: int, max_strassen_depth: int | None = None):
    """Packed lower C of the GPU plan's recursion with the mode's leaf arithmetic.

    The recursion is O2's rows-kept form; pre-sums are rounded to float32
    (the precision the reduced-precision modes form them in) and every leaf
    product uses the mode's operand transform.  FP64 accumulation.
    """
    leaf = {"bf16x3": bf16x3_product, "fp8": fp8_product}[mode]
    Cp, _ = recursive.ata(np.asarray(A, dtype=np.float32), b, split_m=False,
                          max_strassen_depth=max_strassen_depth,
                          leaf_product=leaf, round_sum=_round_f32)
    return Cp


# --------------------------------------------------------------- spread flags


def spread(nu) -> float:
    nz = np.asarray(nu, dtype=np.float64)
    nz = nz[nz > 0]
    if nz.size < 2:
        return 1.0
    return float(nz.max() / nz.min())


def spread_flags(nu, nodes, tau: float):
    """Flag per AtA node (col0, w, ...): spread of nu over its columns > tau^2."""
    return [spread(nu[c0:c0 + w]) > tau * tau for (c0, w, *_rest) in nodes]


# ------------------------------------------------------------ Freivalds probe

_MASK = (1 << 64) - 1


def splitmix64(state: int) -> tuple[int, int]:
    """One SplitMix64 step: returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & _MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return state, z ^ (z >> 31)


def probe_signs(n: int, seed: int) -> np.ndarray:
    """x_j = +1 iff the top bit of the SplitMix64 output at counter j is 0.

    Counter form: output j is the step taken from state seed + j * gamma.
    """
    x = np.empty(n, dtype=np.float64)
    gamma = 0x9E3779B97F4A7C15
    for j in range(n):
        _, z = splitmix64((seed + j * gamma) & _MASK)
        x[j] = -1.0 if (z >> 63) else 1.0
    return x


def freivalds_residual(A, Cp, seed: int) -> float:
    """||C x - A^T (A x)|| / (||A||_F^2 ||x||), C given in packed lower form."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    x = probe_signs(n, seed)
    Cp = np.asarray(Cp, dtype=np.float64)
    C = np.zeros((n, n))
    rows, cols = np.tril_indices(n)
    C[rows, cols] = Cp
    C[cols, rows] = Cp
    r = C @ x - A.T @ (A @ x)
    denom = float(np.sum(A * A)) * float(np.linalg.norm(x))
    return float(np.linalg.norm(r) / denom) if denom > 0 else 0.0
