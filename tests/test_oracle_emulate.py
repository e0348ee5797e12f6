"""Pins for the reduced-precision emulation, spread flags and residual (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import emulate, plain, recursive
from conftest import golden_path


def test_bf16_rne_against_library_and_hand_cases():
    rng = np.random.default_rng(31)
    x = (rng.standard_normal(200000) * 10.0 ** rng.uniform(-8, 8, 200000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(emulate.bf16_rne(x), ref)
    # ties go to the even bf16 mantissa: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    t = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0], dtype=np.float32)
    assert emulate.bf16_rne(t).tolist() == [1.0, 1 + 2 ** -6, -1.0, 0.0]


def test_split_bf16_accuracy():
    rng = np.random.default_rng(32)
    a = rng.standard_normal(100000).astype(np.float32)
    hi, lo = emulate.split_bf16(a)
    assert np.array_equal(emulate.bf16_rne(hi), hi) and np.array_equal(emulate.bf16_rne(lo), lo)
    err = np.abs(a.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -17 * np.abs(a))
    b = emulate.bf16_rne(a)
    hb, lb = emulate.split_bf16(b)
    assert np.array_equal(hb, b) and np.all(lb == 0)


def test_bf16x3_exact_on_representable_operands():
    rng = np.random.default_rng(33)
    X = emulate.bf16_rne(rng.standard_normal((64, 20)).astype(np.float32))
    Y = emulate.bf16_rne(rng.standard_normal((64, 9)).astype(np.float32))
    got = emulate.bf16x3_product(X, Y)
    assert np.array_equal(got, X.astype(np.float64).T @ Y.astype(np.float64))


def test_e4m3_value_set_and_rounding():
    v = emulate.e4m3_values()
    assert v[127 - 1] == 448.0 and np.isnan(v[127])
    assert v[1] == 2.0 ** -9 and v[8] == 2.0 ** -6 and v[56] == 1.0
    # hand cases: ties to even code, smallest subnormal halfway rounds to 0
    cases = {1.0625: 1.0, 1.1875: 1.25, 2.0 ** -10: 0.0, 3 * 2.0 ** -10: 2.0 ** -8,
             440.0: 448.0, 17.0: 16.0, 19.0: 20.0, -1.0625: -1.0}
    for x, want in cases.items():
        assert emulate.e4m3_rne(np.array([x]))[0] == want, x
    rng = np.random.default_rng(34)
    x = np.clip(rng.standard_normal(200000) * 40, -448, 448).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).float().numpy()
    assert np.array_equal(emulate.e4m3_rne(x.astype(np.float64)), ref)


def test_scale_exponent_rule():
    assert emulate.pow2_scale_exponent(448.0) == 0
    assert emulate.pow2_scale_exponent(np.nextafter(448.0, 1e9)) == 1
    assert emulate.pow2_scale_exponent(224.0) == -1
    assert emulate.pow2_scale_exponent(896.0) == 1
    assert emulate.pow2_scale_exponent(1.0) == -8      # 1 <= 448 * 2^-8 = 1.75
    for amax in 10.0 ** np.linspace(-30, 30, 301):
        e = emulate.pow2_scale_exponent(amax)
        assert amax <= 448.0 * 2.0 ** e and amax > 448.0 * 2.0 ** (e - 1)


def test_fp8_quantisation_blocks_and_exactness():
    rng = np.random.default_rng(35)
    X = rng.integers(-16, 17, (300, 200)).astype(np.float64)   # all exact in e4m3
    X[:128, :128] = 0.0
    Xd, exps = emulate.quantize_fp8(X)
    assert exps.shape == (3, 2) and exps[0, 0] == 0
    assert np.array_equal(Xd, X)
    Y = rng.integers(-16, 17, (300, 7)).astype(np.float64)
    assert np.array_equal(emulate.fp8_product(X, Y), X.T @ Y)
    # a block's scale is a power of two with amax / s <= 448
    Z = rng.standard_normal((256, 256)) * 1e3
    Zd, e = emulate.quantize_fp8(Z)
    for bi in range(2):
        for bj in range(2):
            blk = Z[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]
            assert np.abs(blk).max() <= 448 * 2.0 ** e[bi, bj]
    assert np.max(np.abs(Zd - Z) / np.abs(Z).max()) <= 2.0 ** -4


def test_emulated_ata_depth0_structure():
    rng = np.random.default_rng(36)
    A = rng.standard_normal((200, 96)).astype(np.float32)
    got = emulate.ata_emulated(A, "bf16x3", b=32, max_strassen_depth=0)
    # at Strassen depth 0 every entry is one leaf product of whole columns
    hi, lo = emulate.split_bf16(A)
    hi, lo = hi.astype(np.float64), lo.astype(np.float64)
    full = hi.T @ hi + hi.T @ lo + lo.T @ hi
    r, c = np.tril_indices(96)
    assert np.allclose(got, full[r, c], rtol=0, atol=1e-12)
    ref = plain.gram_packed(A)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 2e-5


def test_splitmix64_published_outputs():
    want = [int(l, 16) for l in open(golden_path("splitmix64.txt")) if l[0] != "#"]
    s, got = 0, []
    for _ in range(4):
        s, z = emulate.splitmix64(s)
        got.append(z)
    assert got == want
    x = emulate.probe_signs(4, 0)
    assert x.tolist() == [-1.0 if w >> 63 else 1.0 for w in want]


def test_freivalds_residual():
    rng = np.random.default_rng(37)
    A = rng.standard_normal((400, 50))
    Cp = plain.gram_packed(A)
    assert emulate.freivalds_residual(A, Cp, 7) < 1e-15
    bad = Cp.copy()
    bad[3] += 1e-3 * np.abs(Cp).max()
    assert emulate.freivalds_residual(A, bad, 7) > 1e-7


def test_spread_flags():
    A = np.ones((10, 8))
    A[:, 1] *= 1e3                     # squared-norm ratio 1e6 inside [0, 4)
    A[:, 6] = 0.0                      # zero columns are ignored
    nu = plain.colnorms(A)
    nodes = [(0, 4), (4, 4), (0, 8), (6, 1)]
    assert emulate.spread_flags(nu, nodes, tau=100.0) == [True, False, True, False]
    assert emulate.spread_flags(nu, nodes, tau=1e3) == [False, False, False, False]
    c = recursive.count(10, 8, 2)
    assert len(emulate.spread_flags(nu, c.ata_list, 10.0)) == c.ata_nodes


def _read_freivalds_cases():
    cases = []
    for line in open(golden_path("freivalds_hand.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        name, mn, a, c, seed, res, _why = [f.strip() for f in line.split("|", 6)]
        m, n = (int(v) for v in mn.split())
        A = np.array([float(v) for v in a.split()]).reshape(m, n)
        Cp = np.array([float(v) for v in c.split()])
        cases.append((name, A, Cp, int(seed), float(res)))
    return cases


def test_freivalds_residual_hand_cases():
    """The residual's value, normalisation included, on hand-computed cases
    (tests/golden/freivalds_hand.txt): ||E x|| / (||A||_F^2 ||x||)."""
    cases = _read_freivalds_cases()
    assert len(cases) == 6
    for name, A, Cp, seed, want in cases:
        got = emulate.freivalds_residual(A, Cp, seed)
        if want == 0:
            assert got == 0, name
        else:
            assert abs(got - want) <= 1e-15 * want, (name, got, want)
    # the sign-dependent pair: the same E under two seeds gives 1 vs sqrt(5)
    by = {c[0]: c[4] for c in cases}
    assert abs(by["off_sg"] / by["off_s0"] - np.sqrt(5)) < 1e-15


def test_freivalds_residual_planted_normalisations_fail():
    """Plausible normalisation mistakes give values the hand cases reject."""
    A, Cp, seed, want = None, None, None, None
    for name, A_, Cp_, seed_, want_ in _read_freivalds_cases():
        if name == "sq3":
            A, Cp, seed, want = A_, Cp_, seed_, want_
    n = A.shape[1]
    x = emulate.probe_signs(n, seed)
    C = plain.unpack(Cp, n)
    num = np.linalg.norm(C @ x - A.T @ (A @ x))
    fro2 = float(np.sum(A * A))
    wrong = [num / (fro2 * float(x @ x)),               # ||x||^2 for ||x||
             num / (np.sqrt(fro2) * np.linalg.norm(x)),  # ||A||_F for ||A||_F^2
             num / fro2]                                 # no ||x||
    for w in wrong:
        assert abs(w - want) > 1e-3 * want


def _read_rounding_case():
    A = None
    deltas = []
    b = depth = None
    for line in open(golden_path("emulated_presum_rounding.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "shape":
            A = np.zeros((int(f[1]), int(f[2])), dtype=np.float32)
        elif f[0] == "cutoff":
            b = int(f[1])
        elif f[0] == "depth":
            depth = int(f[1])
        elif f[0] == "a":
            A[int(f[1]), int(f[2])] = float.fromhex(f[3])
        elif f[0] == "d":
            deltas.append((int(f[1]), int(f[2]), float.fromhex(f[3])))
    return A, b, depth, deltas


def test_emulated_presum_rounding_hand_case():
    """Two Strassen levels: each pre-sum is rounded to FP32 before it is split
    (hand-derived in tests/golden/emulated_presum_rounding.txt)."""
    A, b, depth, deltas = _read_rounding_case()
    n = A.shape[1]
    want = plain.unpack(plain.gram_packed(A), n)
    for r, c, d in deltas:
        want[r, c] += d
    rr, cc = np.tril_indices(n)
    got = emulate.ata_emulated(A, "bf16x3", b=b, max_strassen_depth=depth)
    assert np.array_equal(got, want[rr, cc])
    # planted mistake: the same recursion without the FP32 rounding of the
    # pre-sums (only the final leaf operand is rounded) misses the fixture
    unrounded, _ = recursive.ata(A, b, split_m=False, max_strassen_depth=depth,
                                 leaf_product=emulate.bf16x3_product)
    assert not np.array_equal(unrounded, want[rr, cc])


@pytest.mark.parametrize("mode,lim", [("bf16x3", 8), ("fp8", 4)])
@pytest.mark.parametrize("m,n,b,depth", [(37, 29, 4, 1), (37, 29, 4, 2), (64, 48, 8, 2),
                                         (130, 67, 16, 2), (9, 40, 5, 2)])
def test_emulated_integers_exact_with_strassen(mode, lim, m, n, b, depth):
    """Small integers whose pre-sums stay exact in the mode's operand format
    (|sum| <= 4 lim: <= 32 for bf16, <= 16 for e4m3 after the power-of-two
    block scale) give exactly the plain FP64 Gram product at Strassen depth
    1 and 2, odd splits included."""
    rng = np.random.default_rng(1000 + m + n + b + depth)
    A = rng.integers(-lim, lim + 1, (m, n)).astype(np.float32)
    got = emulate.ata_emulated(A, mode, b=b, max_strassen_depth=depth)
    c = recursive.count(m, n, b, split_m=False, max_strassen_depth=depth)
    assert c.strassen_nodes > 0
    assert np.array_equal(got, plain.gram_packed(A))
