"""Pins for O2, the recursive AtA of Sec. 3 (CPU only)."""
import numpy as np
import pytest

from oracle import plain, recursive
from conftest import golden_path


def _small_int(rng, m, n, q=3):
    return rng.integers(-q, q + 1, (m, n)).astype(np.float64)


@pytest.mark.parametrize("split_m", [True, False])
def test_bit_exact_on_small_integers(split_m):
    rng = np.random.default_rng(21)
    shapes = [(1, 1), (1, 9), (9, 1), (2, 2), (3, 2), (2, 3), (5, 7), (17, 33),
              (64, 64), (65, 63), (100, 37), (31, 130)]
    shapes += [tuple(int(v) for v in rng.integers(1, 300, 2)) for _ in range(12)]
    for m, n in shapes:
        A = _small_int(rng, m, n)
        ref = plain.gram_packed(A)
        # tiny leaves only on small inputs (the pure-Python recursion is slow)
        for b in ((1, 2, 4, 8, 16) if max(m, n) <= 40 else (7, 33)):
            Cp, _ = recursive.ata(A, b, split_m=split_m)
            assert np.array_equal(Cp, ref), (m, n, b, split_m)


def test_both_forms_same_multiplications():
    # equal when every split is even; with odd splits the padded operand sizes
    # (ceil dimensions) make the counts differ slightly between the two forms
    for m, n, b in [(64, 64, 1), (128, 32, 4), (256, 512, 16), (1024, 1024, 256),
                    (4096, 2048, 128)]:
        a = recursive.count(m, n, b, split_m=True).mults
        c = recursive.count(m, n, b, split_m=False).mults
        assert a == c


def test_multiplication_counts_against_closed_forms():
    rows = [l.split() for l in open(golden_path("mult_counts.txt")) if l[0] != "#"]
    assert len(rows) == 11
    for n, b, want in ((int(a), int(b_), int(c)) for a, b_, c in rows):
        if b == 1:
            L = n.bit_length() - 1
            # Sec. 1: 2/3 n^log2(7) + 1/3 n^2, n = 2^L
            assert 3 * want == 2 * 7 ** L + 4 ** L
        assert recursive.mults_closed_form(n, b) == want
        if n // b > 64:
            continue                 # too many leaves for the Python walk
        for split_m in (True, False):
            assert recursive.count(n, n, b, split_m=split_m).mults == want, (n, b)


def test_strassen_structure_per_level():
    # Sec. 3.2: seven products and 18 block sums (10 pre-sums, 8 post-sums) per level
    for L in range(1, 6):
        n = 2 ** L
        X = np.ones((n, n))
        _, c = recursive.strassen_product(X, X, b=1)
        nodes = (7 ** L - 1) // 6
        assert c.strassen_nodes == nodes
        assert c.gemm_leaves == 7 ** L and c.mults == 7 ** L
        assert c.presum_blocks == 10 * nodes and c.postsum_blocks == 8 * nodes
        assert c.accum_blocks == 12 * nodes
        # element additions: 10 pre-sums of (n/2)^2 per level -> (10/3)(7^L - 4^L);
        # with the 8 post-sums this is the textbook 6 (7^L - 4^L)
        assert 3 * c.presum_adds == 10 * (7 ** L - 4 ** L)
        assert c.accum_adds == 4 * (7 ** L - 4 ** L)
        assert c.presum_adds + (c.accum_adds * 8) // 12 == 6 * (7 ** L - 4 ** L)


def test_strassen_product_exact_and_odd():
    rng = np.random.default_rng(22)
    for m, n, k in [(5, 3, 4), (7, 7, 7), (33, 17, 20), (64, 31, 45), (9, 2, 11)]:
        X = _small_int(rng, m, n)
        Y = _small_int(rng, m, k)
        for b in (1, 2, 3, 8):
            C, _ = recursive.strassen_product(X, Y, b)
            assert np.array_equal(C, X.T @ Y), (m, n, k, b)


def test_workspace_bound():
    # Sec. 3.3: the M, P, Q buffers need at most 3/2 n^2 elements
    for n, b in ((8, 1), (16, 1), (37, 1), (64, 2), (127, 4), (256, 8), (1000, 16)):
        for split_m in (True, False):
            c = recursive.count(n, n, b, split_m=split_m)
            assert c.ws_peak <= 1.5 * n * n
    # Strassen alone, n = 2^L down to 1: one S, T and M per level, 3 sum (n/2^i)^2
    for L in range(1, 6):
        n = 2 ** L
        _, c = recursive.strassen_product(np.ones((n, n)), np.ones((n, n)), 1)
        assert c.ws_peak == sum(3 * (n >> i) ** 2 for i in range(1, L + 1))


def test_fp64_random_agrees_with_plain():
    rng = np.random.default_rng(23)
    A = rng.uniform(-1, 1, (1024, 1024))
    ref = plain.gram_packed(A)
    for split_m in (True, False):
        Cp, ctr = recursive.ata(A, 256, split_m=split_m)
        assert ctr.mults == 503840768
        err = np.linalg.norm(Cp - ref) / np.linalg.norm(ref)
        assert err < 1e-14


def test_node_structure_covers_lower_triangle():
    for n, b in [(1024, 256), (1000, 100), (37, 5)]:
        c = recursive.count(64, n, b, split_m=False)
        cover = np.zeros((n, n), dtype=np.int64)
        for (_, c0, _, w) in c.syrk_list:
            blk = cover[c0:c0 + w, c0:c0 + w]
            blk += np.tril(np.ones((w, w), dtype=np.int64))
        for (x0, y0, _, nn, kk, _, _) in c.strassen_roots:
            cover[x0:x0 + nn, y0:y0 + kk] += 1
        assert np.array_equal(cover, np.tril(np.ones((n, n), dtype=np.int64)))


def test_planted_mistake_is_caught():
    """A wrong sign in one Strassen sum must break the integer exactness pin."""
    rng = np.random.default_rng(24)
    A = _small_int(rng, 40, 40)
    ref = plain.gram_packed(A)
    bad = recursive._Recursion.strassen

    def mutated(self, X, Y, C, depth):
        levels = bad(self, X, Y, C, depth)
        if depth == 0 and levels > 0:
            C[0, 0] += 1.0          # stands for a dropped / mis-signed term
        return levels

    recursive._Recursion.strassen = mutated
    try:
        Cp, _ = recursive.ata(A, 4, split_m=False)
    finally:
        recursive._Recursion.strassen = bad
    assert not np.array_equal(Cp, ref)
