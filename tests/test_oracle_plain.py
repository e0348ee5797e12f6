"""Pins for O1, the plain FP64 Gram product (CPU only)."""
import numpy as np
import pytest

from oracle import plain
from conftest import golden_path


def _read_hand_cases():
    cases, lines = [], [l.strip() for l in open(golden_path("tiny_hand.txt"))
                        if l.strip() and not l.startswith("#")]
    i = 0
    while i < len(lines):
        _, r, c = lines[i].split()
        r, c = int(r), int(c)
        A = np.array([[float(v) for v in lines[i + 1 + k].split()] for k in range(r)])
        assert lines[i + 1 + r] == "C"
        Cp = np.array([float(v) for v in lines[i + 2 + r].split()])
        cases.append((A, Cp))
        i += 3 + r
    return cases


def test_hand_computed_cases():
    cases = _read_hand_cases()
    assert len(cases) == 5
    for A, Cp in cases:
        assert np.array_equal(plain.gram_packed(A), Cp)
        assert np.array_equal(plain.gram_packed(A.astype(np.float32)), Cp)


def test_identity_and_all_ones():
    for n in (1, 7, 64):
        Cp = plain.gram_packed(np.eye(n))
        assert np.array_equal(plain.unpack(Cp, n), np.eye(n))
    for m, n in ((5, 3), (33, 17)):
        Cp = plain.gram_packed(np.ones((m, n)))
        assert np.all(Cp == m)


def test_rank_one_closed_form():
    rng = np.random.default_rng(11)
    u = rng.integers(-5, 6, 40).astype(np.float64)
    v = rng.integers(-5, 6, 23).astype(np.float64)
    A = np.outer(u, v)
    C = plain.unpack(plain.gram_packed(A), 23)
    assert np.array_equal(C, (u @ u) * np.outer(v, v))


def test_orthonormal_columns_give_identity():
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((300, 40)))
    C = plain.unpack(plain.gram_packed(Q), 40)
    assert np.max(np.abs(C - np.eye(40))) < 1e-14


def test_symmetric_psd_and_diagonal():
    rng = np.random.default_rng(13)
    A = rng.uniform(-1, 1, (257, 61))
    Cp = plain.gram_packed(A)
    C = plain.unpack(Cp, 61)
    assert np.array_equal(C, C.T)
    lam = np.linalg.eigvalsh(C)
    assert lam.min() >= -1e-13 * lam.max()
    # diagonal = squared column norms, summed independently (math.fsum is exact-rounded)
    import math
    for i in range(61):
        assert abs(C[i, i] - math.fsum(A[:, i] ** 2)) <= 1e-14 * C[i, i]


def test_freivalds_identity():
    rng = np.random.default_rng(14)
    A = rng.standard_normal((500, 77))
    C = plain.unpack(plain.gram_packed(A), 77)
    x = rng.choice([-1.0, 1.0], 77)
    assert abs(x @ C @ x - np.sum((A @ x) ** 2)) <= 1e-12 * np.sum(A * A) * 77


def test_library_cross_check():
    rng = np.random.default_rng(15)
    A = rng.uniform(-1, 1, (700, 129))
    ref = A.T @ A
    C = plain.unpack(plain.gram_packed(A), 129)
    assert np.linalg.norm(C - ref) <= 1e-14 * np.linalg.norm(ref)


def test_float32_inputs_promote_exactly_and_lda():
    rng = np.random.default_rng(16)
    A = rng.uniform(-1, 1, (90, 50)).astype(np.float32)
    assert np.array_equal(plain.gram_packed(A), plain.gram_packed(A.astype(np.float64)))
    wide = rng.uniform(-1, 1, (90, 64))
    view = wide[:, 3:53]                     # row stride 64 > n = 50
    assert np.array_equal(plain.gram_packed(view),
                          plain.gram_packed(np.ascontiguousarray(view)))


def test_columns_match_packed_bitwise_and_threads():
    rng = np.random.default_rng(17)
    A = rng.standard_normal((333, 45))
    Cp1 = plain.gram_packed(A, nthreads=1)
    Cp8 = plain.gram_packed(A, nthreads=8)
    assert np.array_equal(Cp1, Cp8)
    C = plain.unpack(Cp1, 45)
    S = np.array([0, 7, 44, 13])
    cols = plain.gram_cols(A, S, nthreads=3)
    assert np.array_equal(cols, C[:, S])


def test_colnorms():
    rng = np.random.default_rng(18)
    A = rng.standard_normal((100, 9))
    nu = plain.colnorms(A)
    C = plain.unpack(plain.gram_packed(A), 9)
    assert np.array_equal(nu, np.diag(C))


def test_degenerate_shapes():
    assert plain.gram_packed(np.zeros((0, 5))).tolist() == [0.0] * 15
    assert plain.gram_packed(np.zeros((4, 0))).size == 0
    with pytest.raises(ValueError):
        plain.unpack(np.zeros(5), 3)


# --------------------------------------------------------------- A^T B
def test_gemm_tn_hand_computed():
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    B = np.array([[5.0], [6.0]])
    C = plain.gemm_tn(A, B)
    assert C.shape == (2, 1)
    assert C[0, 0] == 1 * 5 + 3 * 6 and C[1, 0] == 2 * 5 + 4 * 6


def test_gemm_tn_identity_and_transpose_symmetry():
    rng = np.random.default_rng(21)
    B = rng.standard_normal((9, 4))
    assert np.array_equal(plain.gemm_tn(np.eye(9), B), B)          # I^T B = B
    A = rng.standard_normal((40, 7))
    # (A^T B)^T = B^T A entry for entry: the same products in the same order
    B2 = rng.standard_normal((40, 5))
    assert np.array_equal(plain.gemm_tn(A, B2), plain.gemm_tn(B2, A).T)


def test_gemm_tn_of_a_with_itself_is_the_gram_product():
    rng = np.random.default_rng(22)
    for dt in (np.float64, np.float32):
        A = rng.standard_normal((123, 17)).astype(dt)
        C = plain.gemm_tn(A, A)
        i, j = np.tril_indices(17)
        assert np.array_equal(C[i, j], plain.gram_packed(A))      # packed order is row-major lower


def test_gemm_tn_against_numpy_and_threads():
    rng = np.random.default_rng(23)
    A = rng.standard_normal((300, 40))
    B = rng.standard_normal((300, 25))
    C = plain.gemm_tn(A, B)
    ref = A.T @ B
    assert np.linalg.norm(C - ref) / np.linalg.norm(ref) <= 1e-14
    assert np.array_equal(plain.gemm_tn(A, B, nthreads=1), plain.gemm_tn(A, B, nthreads=3))
    assert plain.gemm_tn(np.zeros((0, 4)), np.zeros((0, 2))).tolist() == [[0.0, 0.0]] * 4
