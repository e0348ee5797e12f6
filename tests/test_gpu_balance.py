"""Tail balancing of the leaf launch (ATA_OPT_BALANCE_TAIL): leaves of an
underfilled last round are cut into K chunks whose partial sums the split-K
reduce adds.  Without the spread check, 8192 columns on 256 x 256 tiles give
528 equal tiles: two full rounds on 256 resident workgroups and a last round
of 16.  Integer inputs must stay bit-exact; random inputs must match the
uncut plan up to rounding and the oracle within the mode's tolerance."""
import sys

import numpy as np
import pytest

from oracle import plain
from paper_2110_13042_amd import ata
from gpu_helpers import device, full_error, run_gram

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def h():
    device()
    hd = ata.Handle(spread_tau=0)
    yield hd
    hd.set("balance_tail", 1)
    hd.close()


@pytest.fixture(scope="module")
def ints():
    A = np.random.default_rng(111).integers(-2, 3, (1024, 8192)).astype(np.float64)
    return A, plain.gram_packed(A)


@pytest.mark.parametrize("mode,tile,expect_cut", [(ata.F32_BF16X3, 2, True), (ata.F32, 2, True),
                                                  (ata.F64, 0, False)])
def test_balanced_tail_integers_exact(h, ints, mode, tile, expect_cut):
    A, ref = ints
    h.set("leaf_tile", tile)
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 0)
    try:
        for bal in (1, 0):
            h.set("balance_tail", bal)
            _say("case: tail balance ints mode", mode, "tile", tile, "balance", bal)
            Cp = run_gram(A, mode, h)
            rep = h.report()
            _say("  cut leaves", rep["tail_split_leaves"], "chunks", rep["tail_split_chunks"])
            if bal == 0:
                assert rep["tail_split_leaves"] == 0
            elif expect_cut:
                assert rep["tail_split_leaves"] > 0 and rep["tail_split_chunks"] >= 2
            assert np.array_equal(Cp, ref), (mode, tile, bal)
    finally:
        h.set("balance_tail", 1)
        h.set("leaf_tile", 0)


def test_balanced_tail_random_matches_uncut(h):
    rng = np.random.default_rng(112)
    A = rng.uniform(-1, 1, (2048, 8192)).astype(np.float32)
    ref = plain.gram_packed(A)
    h.set("leaf_tile", 2)
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 0)
    try:
        out = {}
        for bal in (0, 1):
            h.set("balance_tail", bal)
            out[bal] = run_gram(A, ata.F32_BF16X3, h)
            rep = h.report()
            _say("case: tail balance random, balance", bal, "cut", rep["tail_split_leaves"],
                 "x", rep["tail_split_chunks"], "e_F", full_error(out[bal], ref))
        scale = np.abs(ref).max()
        assert np.abs(out[1] - out[0]).max() <= 1e-5 * scale
        assert full_error(out[1], ref) <= 2e-5
    finally:
        h.set("balance_tail", 1)
        h.set("leaf_tile", 0)
