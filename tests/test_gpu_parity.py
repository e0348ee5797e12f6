"""Parity of the HIP path (through the C ABI) against the CPU oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import emulate, plain, recursive
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, mode_input, packed_columns, run_gram

pytestmark = pytest.mark.gpu

TOL = {ata.F64: 1e-12, ata.F32: 2e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    device()
    hd = ata.Handle()
    yield hd
    hd.close()


def test_square_f64_1024_leaf256_one_strassen_level(h):
    """1024 x 1024 uniform FP64, leaf cutoff 256: <= 1e-12 and the paper's count."""
    _say("case: square_f64_1024 b=256")
    A = workloads.make("square_f64_1024")
    h.set("leaf_cutoff", 256)
    h.set("max_depth", -1)
    Cp = run_gram(A, ata.F64, h)
    rep = h.report()
    assert rep["multiplications"] == 503840768
    assert rep["strassen_levels"] == 1
    err = full_error(Cp, plain.gram_packed(A))
    _say("e_F", err)
    assert err <= 1e-12


@pytest.mark.parametrize("mode", [ata.F64, ata.F32])
def test_small_integers_bit_exact(h, mode):
    """Exact arithmetic: Strassen levels and odd splits reproduce O1 bit for bit."""
    rng = np.random.default_rng(41)
    shapes = [(1, 1), (1, 7), (7, 1), (3, 2), (2, 3), (129, 130), (257, 255), (300, 513),
              (1000, 777), (64, 1500), (513, 1025)]
    for (m, n) in shapes:
        for b, depth in [(64, 3), (100, 1), (128, 64)]:
            if mode == ata.F32 and depth > 2:
                depth = 2
            _say("case: int", m, n, b, depth, mode)
            A = rng.integers(-2, 3, (m, n)).astype(np.float64)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            h.set("spread_tau", 0)
            Cp = run_gram(A, mode, h)
            assert np.array_equal(Cp, plain.gram_packed(A)), (m, n, b, depth, mode)
    h.set("spread_tau", 4096)


@pytest.mark.parametrize("mode", [ata.F64, ata.F32])
def test_random_ragged_shapes(h, mode):
    rng = np.random.default_rng(42)
    for (m, n, b, depth) in [(700, 333, 96, 2), (1031, 1029, 128, 3), (2000, 640, 160, 2),
                             (129, 1100, 256, 2), (4096, 1536, 512, 2)]:
        _say("case: random", m, n, b, depth, mode)
        A = rng.uniform(-1, 1, (m, n))
        if mode == ata.F32:
            A = A.astype(np.float32)
        h.set("leaf_cutoff", b)
        h.set("max_depth", depth)
        Cp = run_gram(A, mode, h)
        err = full_error(Cp, plain.gram_packed(A))
        _say("  e_F", err)
        assert err <= TOL[mode]


def test_leading_dimension_and_degenerate(h):
    rng = np.random.default_rng(43)
    A = rng.integers(-3, 4, (300, 257)).astype(np.float64)
    h.set("leaf_cutoff", 64)
    h.set("max_depth", 2)
    _say("case: lda 320")
    Cp = run_gram(A, ata.F64, h, lda=320)
    assert np.array_equal(Cp, plain.gram_packed(A))
    _say("case: m = 0")
    dev = device()
    C = torch.full((10 * 11 // 2,), 7.0, dtype=torch.float32, device=dev)
    Z = torch.zeros((0, 10), dtype=torch.float32, device=dev)
    ata.gram(Z, ata.F32, handle=h, out=C)
    torch.cuda.synchronize()
    assert torch.all(C == 0).item()
    _say("case: n = 0")
    E = torch.zeros((5, 0), dtype=torch.float32, device=dev)
    out = ata.gram(E, ata.F32, handle=h)
    assert out.numel() == 0


def test_deterministic_runs(h):
    rng = np.random.default_rng(44)
    A = rng.standard_normal((2048, 1500)).astype(np.float32)
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 2)
    _say("case: determinism")
    C1 = run_gram(A, ata.F32, h)
    C2 = run_gram(A, ata.F32, h)
    assert np.array_equal(C1, C2)


def test_argument_errors_leave_c_untouched(h):
    dev = device()
    A = torch.ones((8, 8), dtype=torch.float32, device=dev)
    C = torch.full((36,), 5.0, dtype=torch.float32, device=dev)
    L = ata.lib()
    assert L.ata_gram(h.h, A.data_ptr(), 8, 8, 4, ata.F32, C.data_ptr(), None) == 1   # lda < n
    assert L.ata_gram(h.h, A.data_ptr(), -1, 8, 8, ata.F32, C.data_ptr(), None) == 1
    assert L.ata_gram(h.h, A.data_ptr(), 8, 8, 8, 7, C.data_ptr(), None) == 1
    assert L.ata_gram(h.h, A.data_ptr(), 8, 8, 8, ata.F32, A.data_ptr(), None) == 1  # overlap
    h.set("workspace_limit", 1024)
    h.set("leaf_cutoff", 2)
    h.set("max_depth", 2)
    assert L.ata_gram(h.h, A.data_ptr(), 8, 8, 8, ata.F32, C.data_ptr(), None) == 3
    h.set("workspace_limit", 0)
    torch.cuda.synchronize()
    assert torch.all(C == 5.0).item()


@pytest.mark.parametrize("mode", [ata.F64, ata.F32])
def test_residual_probe_matches_oracle(h, mode):
    """ata_residual on the oracle's C plus a seeded perturbation."""
    rng = np.random.default_rng(45)
    m, n = 1500, 700
    A = rng.standard_normal((m, n))
    if mode == ata.F32:
        A = A.astype(np.float32)
    Cp = plain.gram_packed(A)
    Cp = Cp + rng.standard_normal(Cp.size) * 1e-4 * np.abs(Cp).max()
    if mode == ata.F32:
        Cp = Cp.astype(np.float32)
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    Ad = torch.from_numpy(np.ascontiguousarray(A)).to(dev, dt)
    Cd = torch.from_numpy(np.ascontiguousarray(Cp)).to(dev, dt)
    _say("case: residual", mode)
    r_gpu = ata.ata_residual(h.h, Ad.data_ptr(), m, n, n, mode, Cd.data_ptr(), 12345)
    r_ref = emulate.freivalds_residual(A, Cp, 12345)
    _say("  residual", r_gpu, r_ref)
    assert r_ref > 1e-8
    assert abs(r_gpu - r_ref) <= 1e-9 * r_ref


def test_residual_option_after_gram(h):
    rng = np.random.default_rng(47)
    A = rng.standard_normal((1000, 600))
    h.set("leaf_cutoff", 128)
    h.set("max_depth", 2)
    h.set("residual", 1)
    _say("case: residual option")
    run_gram(A, ata.F64, h)
    r = h.report()["residual"]
    h.set("residual", 0)
    _say("  residual", r)
    assert 0 <= r < 1e-15


def test_fallback_flags_match_oracle(h):
    rng = np.random.default_rng(46)
    m, n, b = 3000, 1200, 150
    A = workloads.scaled_normal(m, n, seed=46, dtype=np.float32, span=1.0)
    h.set("leaf_cutoff", b)
    h.set("max_depth", 2)
    # squared-norm spreads of this input's 15 nodes lie in [8150, 9528]:
    # tau^2 = 9025 flags 9 of them, 0.66% or more away from the threshold
    tau = 95.0
    h.set("spread_tau", tau)
    _say("case: fallback flags")
    Cp = run_gram(A, ata.F32, h)
    rep = h.report()
    nu_gpu, nodes = h.spread(n)
    c = recursive.count(m, n, b, split_m=False, max_strassen_depth=2)
    nu = plain.colnorms(A)
    # nu: FP64 sums of exact products of the FP32 inputs, in another order
    assert np.allclose(nu_gpu, nu, rtol=1e-13, atol=0)
    # the same AtA nodes, in the recursion's order
    assert [(c0, w) for c0, w, _f in nodes] == [(c0, w) for c0, w, _leaf in c.ata_list]
    got = [bool(f) for _c0, _w, f in nodes]
    # the decision rule on the GPU's own norms is exact ...
    assert got == emulate.spread_flags(np.asarray(nu_gpu), c.ata_list, tau)
    # ... and the oracle's norms give the same flags (no node sits within
    # rounding of the threshold here)
    spreads = [emulate.spread(nu[c0:c0 + w]) for c0, w, _leaf in c.ata_list]
    assert min(abs(sp / tau ** 2 - 1) for sp in spreads) > 1e-9
    want = emulate.spread_flags(nu, c.ata_list, tau)
    assert got == want
    assert rep["flagged_nodes"] == sum(want) and 0 < sum(want) < len(want)
    err = full_error(Cp, plain.gram_packed(A))
    _say("  e_F", err, "flagged", want)
    assert err <= 2e-5
    h.set("spread_tau", 4096)


@pytest.mark.parametrize("b,depth", [(2048, 0), (150, 1)])
def test_fp8_norms_from_quantisation_match_oracle(h, b, depth):
    """FP8: the quantisations of A's column slices also sum the column
    squares (no separate norm pass over A).  The norms must match the oracle's
    and the flags must follow from them, for one leaf over all columns and
    for the recursion's diagonal slices."""
    m, n = 3000, 1200
    A = workloads.scaled_normal(m, n, seed=46, dtype=np.float32, span=1.0)
    h.set("leaf_cutoff", b)
    h.set("max_depth", depth)
    tau = 95.0              # the spreads of this input: see test_fallback_flags_match_oracle
    h.set("spread_tau", tau)
    _say("case: fp8 norms from the quantisation", b, depth)
    Cp = run_gram(A, ata.F32_FP8E4M3, h)
    rep = h.report()
    nu_gpu, nodes = h.spread(n)
    nu = plain.colnorms(A)
    assert np.allclose(nu_gpu, nu, rtol=1e-13, atol=0)
    c = recursive.count(m, n, b, split_m=False, max_strassen_depth=depth)
    assert [(c0, w) for c0, w, _f in nodes] == [(c0, w) for c0, w, _leaf in c.ata_list]
    got = [bool(f) for _c0, _w, f in nodes]
    spreads = [emulate.spread(nu[c0:c0 + w]) for c0, w, _leaf in c.ata_list]
    assert min(abs(sp / tau ** 2 - 1) for sp in spreads) > 1e-9
    want = emulate.spread_flags(nu, c.ata_list, tau)
    assert got == want and rep["flagged_nodes"] == sum(want) > 0
    err = full_error(Cp, plain.gram_packed(A))
    _say("  flagged", sum(want), "of", len(want), "e_F", err, "launches", rep["kernel_launches"])
    assert err < 0.1
    if depth == 0:
        # the one node is flagged: the whole product in FP64, rounded once to
        # the FP32 output
        assert err <= 2.0 ** -24
    h.set("spread_tau", 4096)


def test_full_size_square_f32_8192_sampled(h):
    """The benchmark's workload at full size, default plan, 64 sampled columns."""
    _say("case: square_f32_8192 full size")
    A = workloads.make("square_f32_8192")
    h.set("leaf_cutoff", 0)
    h.set("max_depth", -1)
    Cp = run_gram(A, ata.F32, h)
    S = workloads.sampled_columns(8192, 64, seed=99)
    got = packed_columns(Cp, 8192, S)
    ref = plain.gram_cols(A, S)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say("  e_S", err, h.report())
    assert err <= 2e-5


@pytest.mark.parametrize("tile", [3, 2])
def test_f32_wide_tile(h, tile):
    """FP32 leaves on the 256 x 256 tiles (four and eight waves): exact on
    integers (Strassen levels, odd splits, a leading dimension that is not a
    multiple of four, split-K on a tall input) and within 2e-5 of the oracle
    on random data."""
    rng = np.random.default_rng(44)
    h.set("leaf_tile", tile)
    h.set("spread_tau", 0)
    try:
        for (m, n, b, depth, lda) in [(1, 1, 64, 0, 1), (3, 2, 64, 0, 2), (257, 255, 64, 2, 255),
                                      (300, 513, 100, 1, 515), (1000, 777, 128, 2, 777),
                                      (64, 1500, 256, 1, 1501), (20000, 300, 300, 0, 301),
                                      (513, 1025, 512, 1, 1025)]:
            _say("case: f32 wide int", m, n, b, depth, "lda", lda)
            A = rng.integers(-2, 3, (m, n)).astype(np.float32)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            Cp = run_gram(A, ata.F32, h, lda=lda)
            assert np.array_equal(Cp, plain.gram_packed(A)), (m, n, b, depth, lda)
        for (m, n, b, depth) in [(1031, 1029, 256, 2), (4096, 1536, 512, 1), (129, 1100, 256, 2)]:
            _say("case: f32 wide random", m, n, b, depth)
            A = rng.uniform(-1, 1, (m, n)).astype(np.float32)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            Cp = run_gram(A, ata.F32, h)
            err = full_error(Cp, plain.gram_packed(A))
            _say("  e_F", err)
            assert err <= TOL[ata.F32]
    finally:
        h.set("leaf_tile", 0)
        h.set("spread_tau", 4096)


@pytest.mark.parametrize("mode,tile", [(ata.F32, 3), (ata.F32, 2), (ata.F32, 0), (ata.F64, 0)])
def test_persistent_leaf_launch_matches_grid(h, mode, tile):
    """The persistent leaf launch (per-XCD tile queues) and the one-workgroup-
    per-tile launch give bit-identical results, on a plan with unequal
    contractions (Strassen levels) and on a split-K plan."""
    rng = np.random.default_rng(45)
    h.set("leaf_tile", tile)
    try:
        for (m, n, b, depth) in [(3000, 1100, 256, 2), (40000, 300, 300, 0)]:
            _say("case: persistent vs grid", mode, "tile", tile, m, n, b, depth)
            A = mode_input(rng.uniform(-1, 1, (m, n)), mode)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            outs = []
            for pers in (0, 1):
                h.set("leaf_persistent", pers)
                outs.append(run_gram(A, mode, h))
            assert np.array_equal(outs[0], outs[1])
            err = full_error(outs[1], plain.gram_packed(A))
            _say("  e_F", err)
            assert err <= TOL[mode]
    finally:
        h.set("leaf_persistent", -1)
        h.set("leaf_tile", 0)
