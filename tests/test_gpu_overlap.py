"""Overlap of the Strassen pre-sums with the leaves that read only A
(ATA_OPT_OVERLAP): those leaves run in their own launch on a second stream,
beside the pre-sums and the other leaves.  The same tiles are computed either
way, so the result must equal the single-launch schedule bit for bit."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, mode_input

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gram(A_np, mode, overlap, **opts):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev, dt)
    with ata.Handle(overlap=overlap, **opts) as h:
        outs = []
        for _ in range(2):                       # the second call reuses plan, stream and events
            outs.append(ata.gram(A, mode, handle=h).double().cpu().numpy())
        torch.cuda.synchronize()
        rep = h.report()
    assert np.array_equal(outs[0], outs[1])
    return outs[0], rep


@pytest.mark.parametrize("mode,opts,shape", [
    (ata.F64, dict(leaf_cutoff=128, max_depth=2), (1500, 1300)),
    (ata.F32, dict(leaf_cutoff=256, max_depth=2), (2048, 1800)),
    (ata.F32, dict(leaf_cutoff=512, max_depth=2, leaf_tile=2), (3000, 2600)),
    # split-BF16: quadrants of A that get packings of their own (odd column
    # splits, row splits off the 8-row groups) are packed before the fork
    (ata.F32_BF16X3, dict(leaf_cutoff=256, max_depth=2), (2048, 1500)),
    (ata.F32_BF16X3, dict(leaf_cutoff=256, max_depth=2, spread_tau=0), (1999, 1501)),
    # FP8: the quantisations of views of A run before the fork
    (ata.F32_FP8E4M3, dict(leaf_cutoff=256, max_depth=1), (1536, 1100)),
    (ata.F32_BF16X3, dict(leaf_cutoff=1024, max_depth=1, leaf_tile=2), (4096, 4096)),
    # split-K: a tall input with few tiles
    (ata.F32, dict(leaf_cutoff=256, max_depth=1), (40000, 700)),
    # flagged nodes: their diagonal leaves run in FP64 on the side stream
    (ata.F32, dict(leaf_cutoff=128, max_depth=2, spread_tau=20.0), "scaled"),
])
def test_overlap_matches_single_launch(mode, opts, shape):
    if shape == "scaled":
        A = workloads.scaled_normal(1500, 1200, seed=41, span=1.5)
    else:
        A = mode_input(workloads.uniform(*shape, seed=42, dtype=np.float64), mode)
    _say("case: overlap", mode, A.shape, opts)
    got, ro = _gram(A, mode, 1, **opts)
    ref_gpu, rs = _gram(A, mode, 0, **opts)
    _say(f"  overlapped {ro['overlapped']} levels {ro['strassen_levels']} launches {ro['kernel_launches']} vs "
         f"{rs['kernel_launches']} flagged {ro['flagged_nodes']}")
    assert ro["overlapped"] == 1 and rs["overlapped"] == 0
    assert ro["multiplications"] == rs["multiplications"] and ro["strassen_levels"] >= 1
    if opts.get("spread_tau"):
        assert ro["flagged_nodes"] == rs["flagged_nodes"] > 0
    assert np.array_equal(got, ref_gpu)
    err = full_error(got, plain.gram_packed(A))
    _say("  e_F", err)
    if mode != ata.F32_FP8E4M3:                  # FP8: reported, not bounded
        assert err <= (1e-12 if mode == ata.F64 else 2e-5)


def test_overlap_not_applied_without_presums():
    A = workloads.uniform(1000, 900, seed=43, dtype=np.float32)
    for mode in (ata.F32, ata.F32_BF16X3, ata.F32_FP8E4M3):
        _, rep = _gram(A, mode, 1, leaf_cutoff=256, max_depth=0)
        assert rep["overlapped"] == 0


def test_overlap_integers_exact():
    rng = np.random.default_rng(44)
    for mode in (ata.F64, ata.F32, ata.F32_BF16X3):
        A = rng.integers(-3, 4, (1300, 1100)).astype(np.float64 if mode == ata.F64 else np.float32)
        got, rep = _gram(A, mode, 1, leaf_cutoff=128, max_depth=3)
        assert rep["overlapped"] == 1
        assert np.array_equal(got, plain.gram_packed(A)), mode
