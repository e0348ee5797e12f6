"""Split-K leaves (long contractions with few output tiles): the K-chunk
partial sums and their reduce pass against the oracle, in every dtype, with
the FP64 fallback, and inside a batch."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, run_gram

pytestmark = pytest.mark.gpu

BIG = 1_000_000          # split target larger than any test's tile count: always split


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _leaves_split(m, n, mode, b, depth):
    _, leaves = ata.ata_plan_query(m, n, mode, b, depth)
    return max(L["ksplit"] for L in leaves)


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3, ata.F32_FP8E4M3])
def test_split_k_small_integers_bit_exact(mode):
    rng = np.random.default_rng(91)
    h = ata.Handle(spread_tau=0)
    try:
        for (m, n, b, depth) in [(20000, 300, 128, 1), (33000, 130, 256, 0), (17000, 513, 256, 1)]:
            A = rng.integers(-2, 3, (m, n)).astype(np.float64 if mode == ata.F64 else np.float32)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            h.set("split_target", BIG)
            _say("case: split int mode", mode, m, n, b, depth)
            Cs = run_gram(A, mode, h)
            ref = plain.gram_packed(A)
            assert np.array_equal(Cs, ref), (m, n, b, depth)
    finally:
        h.close()


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3])
def test_split_k_random_matches_oracle_and_unsplit(mode):
    rng = np.random.default_rng(92)
    m, n = 40000, 700
    A = rng.uniform(-1, 1, (m, n)).astype(np.float32)
    ref = plain.gram_packed(A)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 256)
        h.set("max_depth", 1)
        out = {}
        for target in (BIG, 0):
            h.set("split_target", target)
            _say("case: split random mode", mode, "target", target)
            out[target] = run_gram(A, mode, h)
        e_split, e_plain = full_error(out[BIG], ref), full_error(out[0], ref)
        _say("  split", e_split, "unsplit", e_plain)
        assert e_split <= 2e-5 and e_plain <= 2e-5
        assert full_error(out[BIG], out[0]) <= 2e-5
    finally:
        h.close()


def test_split_k_with_fp64_fallback():
    """Ill-scaled columns: the flagged SYRK leaves run in the FP64 fallback and
    keep FP64 partial sums; unflagged ones take the FP32 kernel's partials."""
    A = workloads.scaled_normal(24000, 600, seed=93, span=2.0)
    ref = plain.gram_packed(A)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 128)
        h.set("max_depth", 1)
        h.set("spread_tau", 30.0)
        h.set("split_target", BIG)
        _say("case: split with fallback")
        Cs = run_gram(A, ata.F32, h)
        rep = h.report()
        _say("  flagged", rep["flagged_nodes"], "error", full_error(Cs, ref))
        assert rep["flagged_nodes"] > 0
        assert full_error(Cs, ref) <= 2e-5
        # diagonal of the flagged leaves: FP64 accumulation, one rounding
        n = A.shape[1]
        idx = np.arange(n)
        diag = Cs[idx * (idx + 1) // 2 + idx]
        rdiag = ref[idx * (idx + 1) // 2 + idx]
        assert np.max(np.abs(diag - rdiag) / rdiag) <= 2 ** -23
    finally:
        h.close()


def test_fallback_split_alone():
    """The FP64 fallback launch is split on its own: with a split target of
    100 tiles, the FP32 launch (136 tiles of 128 x 128) stays whole while the
    fallback's (8 diagonal leaves, 24 tiles) is cut into 4 K chunks.  Flagged
    leaves then take the reduce of the FP64 partials, unflagged ones were
    written by the FP32 kernel directly."""
    A = workloads.scaled_normal(4096, 2048, seed=94, span=2.0)
    ref = plain.gram_packed(A)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 256)
        h.set("max_depth", 0)
        h.set("leaf_tile", 0)
        h.set("spread_tau", 30.0)
        h.set("split_target", 100)
        h.set("balance_tail", 0)
        _say("case: fallback split alone")
        Cs = run_gram(A, ata.F32, h)
        rep = h.report()
        _say("  flagged", rep["flagged_nodes"], "error", full_error(Cs, ref))
        assert rep["flagged_nodes"] > 0
        assert full_error(Cs, ref) <= 2e-5
        n = A.shape[1]
        idx = np.arange(n)
        diag = Cs[idx * (idx + 1) // 2 + idx]
        rdiag = ref[idx * (idx + 1) // 2 + idx]
        assert np.max(np.abs(diag - rdiag) / rdiag) <= 2 ** -23
    finally:
        h.close()


def test_split_k_in_batch():
    rng = np.random.default_rng(94)
    shapes = [(20000, 200), (300, 100), (17000, 64), (1000, 900), (40000, 33)]
    mats = [rng.integers(-2, 3, s).astype(np.float32) for s in shapes]
    dev = device()
    As = [torch.from_numpy(M).to(dev) for M in mats]
    h = ata.Handle(spread_tau=0)
    try:
        h.set("leaf_cutoff", 256)
        h.set("max_depth", 1)
        h.set("split_target", BIG)
        for graph in (0, 1):
            h.set("batch_graph", graph)
            _say("case: split batch graph", graph)
            Cs = ata.gram_batched(As, ata.F32, handle=h)
            torch.cuda.synchronize()
            for M, C in zip(mats, Cs):
                assert np.array_equal(C.double().cpu().numpy(), plain.gram_packed(M)), M.shape
    finally:
        h.close()
