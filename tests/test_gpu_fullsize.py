"""The benchmark's own plans at full size against the plain FP64 oracle.

The 16384 x 16384 precision workload and the 8192 x 8192 square workload run
with the packaged tune table and the library's default spread check, exactly
as the benchmark runs them; errors are on sampled columns.  The 512-problem
batch runs with the batch plans the batch autotuner picks for it (FP32: leaf
cutoff 2048, one Strassen level, the 256 x 256 tile, persistent; split-BF16:
cutoff 2048, no Strassen level, the 128 x 128 tile), with lda = n and with lda
rounded up to a multiple of 64, through captured-graph replays, against the
oracle on every problem.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, packed_columns

pytestmark = pytest.mark.gpu

TUNE_TABLE = os.path.join(os.path.dirname(ata.__file__), "tune_table.json")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bench_handle():
    h = ata.Handle()
    h.tune_load(TUNE_TABLE)
    return h


def _sampled(A_t, mode, S, ref, h):
    C = ata.gram(A_t, mode, handle=h)
    torch.cuda.synchronize()
    rep = h.report()
    got = packed_columns(C.double().cpu().numpy(), A_t.shape[1], S)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), rep


def test_precision_16384_benchmark_plans():
    _say("case: normal_f32_16384, tune-table plans, 256 sampled columns")
    A = workloads.make("normal_f32_16384")
    n = A.shape[1]
    S = workloads.sampled_columns(n, 256, seed=4, after_rows=A.shape[0], after_cols=n)
    ref = plain.gram_cols(A, S)
    A_t = torch.from_numpy(A).to(device())
    h = _bench_handle()
    try:
        for mode, tol in [(ata.F32_BF16X3, 2e-5), (ata.F32, 2e-5), (ata.F32_FP8E4M3, None)]:
            err, rep = _sampled(A_t, mode, S, ref, h)
            _say(f"  mode {mode}: e_S {err:.3e}  b {rep['leaf_cutoff']} levels {rep['strassen_levels']} "
                 f"tile {rep['leaf_tile']} persistent {rep['leaf_persistent']} "
                 f"tail {rep['tail_split_leaves']}/{rep['tail_split_chunks']}")
            if tol is not None:
                assert err <= tol
            else:
                assert err < 0.1
    finally:
        h.close()


def test_square_8192_benchmark_plans():
    _say("case: square_f32_8192, tune-table plans, 128 sampled columns")
    A = workloads.make("square_f32_8192")
    n = A.shape[1]
    S = workloads.sampled_columns(n, 128, seed=1234)
    ref = plain.gram_cols(A, S)
    A_t = torch.from_numpy(A).to(device())
    h = _bench_handle()
    try:
        for mode in (ata.F32_BF16X3, ata.F32):
            err, rep = _sampled(A_t, mode, S, ref, h)
            _say(f"  mode {mode}: e_S {err:.3e}  b {rep['leaf_cutoff']} levels {rep['strassen_levels']} "
                 f"tile {rep['leaf_tile']} tail {rep['tail_split_leaves']}/{rep['tail_split_chunks']}")
            assert err <= 2e-5
            if mode == ata.F32_BF16X3:
                # the tuned split-BF16 plan cuts its last round of tiles into K chunks
                assert rep["tail_split_leaves"] > 0
    finally:
        h.close()


@pytest.fixture(scope="module")
def batch512():
    mats = workloads.batch(seed=5)
    assert len(mats) == 512
    refs = [plain.gram_packed(M) for M in mats]
    return mats, refs


def _batch_tensors(mats, pad64):
    dev = device()
    As = []
    for M in mats:
        t = torch.from_numpy(M).to(dev)
        if pad64:
            lda = -(-M.shape[1] // 64) * 64
            big = torch.zeros((M.shape[0], lda), dtype=torch.float32, device=dev)
            big[:, : M.shape[1]] = t
            t = big[:, : M.shape[1]]
        As.append(t)
    return As


@pytest.mark.parametrize("mode,opts", [
    (ata.F32, dict(leaf_cutoff=2048, max_depth=1, leaf_tile=2)),
    (ata.F32_BF16X3, dict(leaf_cutoff=2048, max_depth=0, leaf_tile=0)),
])
@pytest.mark.parametrize("pad64", [False, True])
def test_batch_512_full(batch512, mode, opts, pad64):
    mats, refs = batch512
    _say(f"case: batch_512_uneven_f32 full, mode {mode}, lda padded to 64: {pad64}")
    As = _batch_tensors(mats, pad64)
    with ata.Handle(**opts) as h:
        h.set("batch_graph", 1)
        outs = [torch.full((M.shape[1] * (M.shape[1] + 1) // 2,), np.nan, dtype=torch.float32,
                           device=device()) for M in mats]
        worst = 0.0
        for rep in range(3):
            for C in outs:
                C.fill_(float(rep) - 5.0)          # eager work between replays
            ata.gram_batched(As, mode, handle=h, outs=outs)
            torch.cuda.synchronize()
            got = [C.double().cpu().numpy() for C in outs]
            if rep == 0:
                first = got
                r = h.report()
                _say(f"  plan: mults {r['multiplications']} leaves {r['syrk_leaves'] + r['gemm_leaves']} "
                     f"strassen nodes {r['strassen_nodes']} tile {r['leaf_tile']} persistent {r['leaf_persistent']}")
                for i, (G, R) in enumerate(zip(got, refs)):
                    err = full_error(G, R)
                    worst = max(worst, err)
                    assert err <= 2e-5, (i, mats[i].shape, err)
            else:
                for i, (G, F) in enumerate(zip(got, first)):
                    assert np.array_equal(G, F), (rep, i)
        _say(f"  worst e_F over 512 problems {worst:.3e}")
