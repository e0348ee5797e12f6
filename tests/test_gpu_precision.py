"""Reduced-precision modes (split-BF16 x3, block-scaled FP8) against the oracle.

Two references: the plain FP64 oracle (the normwise error the mode reaches)
and the CPU emulation of the mode's operand transform with FP64 products
(pins the split / quantisation itself: the GPU may differ from it only by
FP32 accumulation order)."""
import sys

import numpy as np
import pytest
import torch

from oracle import emulate, plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, packed_columns, run_gram

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    device()
    hd = ata.Handle(spread_tau=0)
    yield hd
    hd.close()


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4])
def test_bf16x3_small_integers_bit_exact(h, tile):
    rng = np.random.default_rng(51)
    h.set("leaf_tile", tile)
    for (m, n, b, depth) in [(300, 513, 64, 2), (1000, 777, 100, 1), (64, 1500, 128, 2), (5, 3, 64, 0),
                             (77, 300, 300, 0)]:
        _say("case: bf16x3 int", m, n, b, depth, "tile", tile)
        A = rng.integers(-2, 3, (m, n)).astype(np.float32)
        h.set("leaf_cutoff", b)
        h.set("max_depth", depth)
        Cp = run_gram(A, ata.F32_BF16X3, h)
        assert np.array_equal(Cp, plain.gram_packed(A)), (m, n, b, depth)


@pytest.mark.parametrize("depth,tile", [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2), (2, 2), (0, 3), (1, 3),
                                        (0, 4), (1, 4)])
def test_bf16x3_matches_emulation(h, depth, tile):
    rng = np.random.default_rng(52 + depth)
    m, n, b = 1536, 1100, 256
    A = rng.standard_normal((m, n)).astype(np.float32)
    h.set("leaf_cutoff", b)
    h.set("max_depth", depth)
    h.set("leaf_tile", tile)
    _say("case: bf16x3 emulation depth", depth, "tile", tile)
    Cp = run_gram(A, ata.F32_BF16X3, h)
    emul = emulate.ata_emulated(A, "bf16x3", b, max_strassen_depth=depth)
    exact = plain.gram_packed(A)
    d_emul = full_error(Cp, emul)
    e_exact = full_error(Cp, exact)
    _say("  vs emulation", d_emul, " vs FP64 oracle", e_exact, " emulation vs oracle",
         full_error(emul, exact))
    assert d_emul <= 1e-6
    assert e_exact <= 2e-5


def test_precision_forms_16384_sampled(h):
    """16384 x 16384 N(0,1) on 256 sampled columns: FP32 and split-BF16 within
    2e-5; block-scaled FP8 reported."""
    _say("case: normal_f32_16384 full size")
    A = workloads.make("normal_f32_16384")
    S = workloads.sampled_columns(16384, 256, seed=4, after_rows=16384, after_cols=16384)
    ref = plain.gram_cols(A, S)
    h.set("leaf_cutoff", 0)
    h.set("max_depth", -1)
    h.set("leaf_tile", 0)
    for mode, tol in [(ata.F32, 2e-5), (ata.F32_BF16X3, 2e-5), (ata.F32_FP8E4M3, None)]:
        Cp = run_gram(A, mode, h)
        got = packed_columns(Cp, 16384, S)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("  mode", mode, "e_S", err, h.report()["strassen_levels"])
        if tol is not None:
            assert err <= tol
        else:                       # FP8: reported, not bounded; sanity only
            assert err < 0.1


@pytest.mark.parametrize("tile", [0, 3])
def test_fp8_small_integers_bit_exact(h, tile):
    rng = np.random.default_rng(61)
    h.set("leaf_tile", tile)
    # (the last two: long contractions with an odd number of 128-row slabs,
    # cut into K chunks because their launches have few tiles)
    # (1024 and 2048 columns: the leaves' column slices of A are whole 128-column
    # blocks and read one shared quantisation of A)
    for (m, n, b, depth) in [(300, 513, 128, 1), (1000, 777, 256, 0), (64, 700, 128, 1), (5, 3, 64, 0),
                             (2000, 900, 1024, 0), (4000, 700, 1024, 0), (9000, 300, 512, 0),
                             (700, 1024, 256, 0), (1000, 2048, 512, 1)]:
        _say("case: fp8 int", m, n, b, depth, "tile", tile)
        A = rng.integers(-2, 3, (m, n)).astype(np.float32)
        h.set("leaf_cutoff", b)
        h.set("max_depth", depth)
        Cp = run_gram(A, ata.F32_FP8E4M3, h)
        assert np.array_equal(Cp, plain.gram_packed(A)), (m, n, b, depth)


@pytest.mark.parametrize("n", [1100, 1024])
@pytest.mark.parametrize("depth,tile", [(0, 0), (1, 0), (0, 3), (1, 3)])
def test_fp8_matches_emulation(h, depth, tile, n):
    """Block-scaled e4m3 leaves against the CPU emulation of the same
    quantisation (each leaf operand quantised on its own).  With 1024 columns
    the leaves' column slices of A are whole 128-column blocks and read one
    shared quantisation of A, which must give the same blocks."""
    rng = np.random.default_rng(62 + depth)
    m, b = 1536, 256
    A = (rng.standard_normal((m, n)) * np.exp(rng.uniform(-2, 2, n))).astype(np.float32)
    h.set("leaf_cutoff", b)
    h.set("max_depth", depth)
    h.set("leaf_tile", tile)
    _say("case: fp8 emulation depth", depth, "tile", tile)
    Cp = run_gram(A, ata.F32_FP8E4M3, h)
    emul = emulate.ata_emulated(A, "fp8", b, max_strassen_depth=depth)
    exact = plain.gram_packed(A)
    d_emul = full_error(Cp, emul)
    e_q = full_error(emul, exact)
    _say("  vs emulation", d_emul, " vs FP64 oracle", full_error(Cp, exact),
         " emulation vs oracle", e_q)
    # The FP8 MFMA's internal 128-deep reduction is not FP32-exact (measured
    # ~1e-5 normwise against an emulation with FP32-exact sums), so the bound
    # is 5e-5: still ~300x below the quantisation error e_q, so a wrong scale,
    # a wrong rounding or a misplaced block would fail it.
    assert d_emul <= 5e-5
    assert d_emul <= 1e-2 * e_q


@pytest.mark.parametrize("tile", [0, 2, 4])
def test_bf16x3_packing_in_norm_pass_matches_pack_kernel(tile):
    """With the spread check on, the column-norm pass also writes A's split
    packing; with it off, the pack kernel does.  On well-scaled data no node
    is flagged, so both must give the same bits (ragged m, n and padded lda;
    single problems and a batch).  Split-K and tail balancing are off: the
    spread check changes how the planner splits the fallback-capable leaves,
    and with it the summation order."""
    rng = np.random.default_rng(53)
    dev = device()
    outs = {}
    for tau in (0.0, 4096.0):
        hd = ata.Handle(spread_tau=tau)
        hd.set("leaf_tile", tile)
        hd.set("split_target", 0)
        hd.set("balance_tail", 0)
        res = []
        for (m, n, b, depth, lda) in [(1000, 777, 128, 1, 779), (37, 300, 64, 0, 300), (4099, 1030, 256, 1, 1032),
                                      (8, 5, 64, 0, 5)]:
            _say("case: bf16x3 norm-pass packing", tau, tile, m, n, b, depth, lda)
            A = rng.uniform(-1, 1, (m, n)).astype(np.float32) if tau == 0.0 else outs[(m, n)][0]
            hd.set("leaf_cutoff", b)
            hd.set("max_depth", depth)
            res.append(run_gram(A, ata.F32_BF16X3, hd, lda=lda))
            if tau == 0.0:
                outs[(m, n)] = (A, res[-1])
        As = [outs[k][0] for k in outs]
        Ts = [torch.from_numpy(a).to(dev) for a in As]
        hd.set("leaf_cutoff", 128)
        hd.set("max_depth", 1)
        batch = [c.double().cpu().numpy() for c in ata.gram_batched(Ts, ata.F32_BF16X3, handle=hd)]
        torch.cuda.synchronize()
        if tau == 0.0:
            ref_single, ref_batch = res, batch
        else:
            rep = hd.report()
            assert rep["flagged_nodes"] in (0, -1)
            for a, b_ in zip(ref_single, res):
                assert np.array_equal(a, b_)
            for a, b_ in zip(ref_batch, batch):
                assert np.array_equal(a, b_)
        hd.close()
