"""Autotuner: the tuned plan is chosen for its shape bucket, its result still
matches the oracle, and the table survives a save / load round trip."""
import json
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, run_gram

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3])
def test_autotune_choice_used_and_correct(tmp_path, mode):
    dev = device()
    rng = np.random.default_rng(81)
    m, n = 900, 700
    A = rng.standard_normal((m, n)).astype(np.float32)
    h = ata.Handle()
    try:
        At = torch.from_numpy(A).to(dev)
        C = torch.empty(n * (n + 1) // 2, dtype=torch.float32, device=dev)
        _say("case: autotune mode", mode, m, n)
        best = ata.ata_autotune(h.h, At.data_ptr(), m, n, n, mode, C.data_ptr(), 0)
        _say("  best", best)
        assert best["leaf_cutoff"] >= 128 and best["ms"] > 0
        h.set("leaf_cutoff", 0)
        h.set("max_depth", -1)
        Cp = run_gram(A, mode, h)
        rep = h.report()
        assert rep["leaf_cutoff"] == best["leaf_cutoff"]
        assert rep["strassen_levels"] <= best["max_depth"]
        assert full_error(Cp, plain.gram_packed(A)) <= 2e-5
        # a shape in another bucket keeps the defaults
        B = rng.standard_normal((64, 40)).astype(np.float32)
        assert full_error(run_gram(B, mode, h), plain.gram_packed(B)) <= 2e-5
        # save / load into a fresh handle
        path = str(tmp_path / "tune.json")
        ata.ata_tune_save(h.h, path)
        rows = json.load(open(path))
        assert len(rows) == 1 and rows[0]["leaf_cutoff"] == best["leaf_cutoff"]
        h2 = ata.Handle()
        try:
            ata.ata_tune_load(h2.h, path)
            run_gram(A, mode, h2)
            assert h2.report()["leaf_cutoff"] == best["leaf_cutoff"]
        finally:
            h2.close()
    finally:
        h.close()


def test_batch_autotune_choice_used_and_correct():
    dev = device()
    rng, ms, ns = workloads.batch_shapes(24, 83, (64, 3000), (16, 900))
    mats = [rng.uniform(-1, 1, (int(m), int(n))).astype(np.float32) for m, n in zip(ms, ns)]
    As = [torch.from_numpy(M).to(dev) for M in mats]
    Cs = [torch.empty(M.shape[1] * (M.shape[1] + 1) // 2, dtype=torch.float32, device=dev) for M in mats]
    h = ata.Handle()
    try:
        args = ([A.data_ptr() for A in As], [M.shape[0] for M in mats], [M.shape[1] for M in mats],
                [M.shape[1] for M in mats])
        _say("case: batch autotune bf16x3, 24 problems")
        best = ata.ata_autotune_batched(h.h, *args, ata.F32_BF16X3, [C.data_ptr() for C in Cs], 0)
        _say("  best", best)
        assert best["leaf_cutoff"] >= 128 and best["ms"] > 0
        out = ata.gram_batched(As, ata.F32_BF16X3, handle=h)
        torch.cuda.synchronize()
        assert h.report()["leaf_cutoff"] == best["leaf_cutoff"] or \
            all(M.shape[1] <= best["leaf_cutoff"] for M in mats)
        for M, C in zip(mats, out):
            assert full_error(C.double().cpu().numpy(), plain.gram_packed(M)) <= 2e-5
    finally:
        h.close()
