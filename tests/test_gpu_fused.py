"""Fused Strassen pre-sums (FP32 and FP64): the leaves of a node whose seven
products are all leaves form S1..S5, T1..T5 (Sec. 3.2) while loading their
operands.  Each operand element is the same single IEEE sum or difference the
pre-sum pass stores, so the fused plan must reproduce the materialised plan
exactly, and both must match the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import plain
from paper_2110_13042_amd import ata
from gpu_helpers import device, full_error, mode_input, run_gram

pytestmark = pytest.mark.gpu

TOL = {ata.F64: 1e-12, ata.F32: 2e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    device()
    hd = ata.Handle(spread_tau=0)
    yield hd
    hd.close()


# ragged shapes (4-byte operand loads in the 256 x 256 FP32 engine) and
# shapes whose every view is 16-byte aligned (16-byte loads)
CASES = [(1000, 777, 128, 2), (1031, 1029, 256, 1), (2047, 1500, 256, 3), (4096, 1536, 512, 1),
         (300, 513, 64, 2), (5000, 900, 256, 2), (3000, 2048, 512, 2), (20000, 1024, 256, 1)]


@pytest.mark.parametrize("mode,tile", [(ata.F64, 0), (ata.F32, 0), (ata.F32, 3)])
def test_fused_presums_reproduce_materialised(h, mode, tile):
    rng = np.random.default_rng(71)
    h.set("leaf_tile", tile)
    try:
        for (m, n, b, depth) in CASES:
            A = mode_input(rng.uniform(-1, 1, (m, n)), mode)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            outs = []
            for fuse in (0, 1):
                h.set("fuse_presum", fuse)
                outs.append(run_gram(A, mode, h))
                rep = h.report()
            _say("case: fused vs materialised", mode, "tile", tile, m, n, b, depth,
                 "levels", rep["strassen_levels"])
            assert rep["strassen_levels"] >= 1
            assert np.array_equal(outs[0], outs[1]), (m, n, b, depth)
            err = full_error(outs[1], plain.gram_packed(A))
            _say("  e_F", err)
            assert err <= TOL[mode]
    finally:
        h.set("fuse_presum", 0)
        h.set("leaf_tile", 0)


@pytest.mark.parametrize("mode,tile", [(ata.F64, 0), (ata.F32, 0), (ata.F32, 3)])
def test_fused_presums_integers_exact(h, mode, tile):
    """Small integers: every sum and product is exact, so the fused plan equals
    the plain product bit for bit (odd splits, lda > n)."""
    rng = np.random.default_rng(72)
    h.set("leaf_tile", tile)
    h.set("fuse_presum", 1)
    try:
        for (m, n, b, depth, lda) in [(257, 255, 64, 2, 255), (1000, 777, 100, 2, 781), (513, 1025, 256, 1, 1025),
                                      (64, 1500, 128, 3, 1500)]:
            _say("case: fused int", mode, "tile", tile, m, n, b, depth, lda)
            A = rng.integers(-2, 3, (m, n)).astype(np.float64)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            Cp = run_gram(A, mode, h, lda=lda)
            assert np.array_equal(Cp, plain.gram_packed(A)), (m, n, b, depth)
    finally:
        h.set("fuse_presum", 0)
        h.set("leaf_tile", 0)


def test_fused_presums_shrink_the_workspace(h):
    """The fused plan skips the last level's ten pre-sum buffers."""
    A = np.random.default_rng(73).uniform(-1, 1, (2048, 2048)).astype(np.float32)
    h.set("leaf_cutoff", 512)
    h.set("max_depth", 1)
    ws = []
    for fuse in (0, 1):
        h.set("fuse_presum", fuse)
        run_gram(A, ata.F32, h)
        ws.append(h.report()["workspace_bytes"])
    h.set("fuse_presum", 0)
    _say("workspace materialised / fused", ws)
    # one Strassen node per AtA level above the leaves; each drops 10 m2 x n2 sums
    assert ws[1] < ws[0]
