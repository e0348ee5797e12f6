"""Bounded workspace (ATA_OPT_BOUNDED_WORKSPACE): every Strassen root runs its
top levels product by product, reusing one set of buffers per level (the
buffer reuse of Sec. 3.3).  Checked against the resident schedule (bit for
bit, with split-K and tail cuts off so that both run the same leaves), on
integers (exact), under the spread check with flagged nodes, and at FP64
30000 x 30000 with the default leaf cutoff and depth, whose workspace must
stay within Sec. 3.3's 3/2 n^2 elements."""
import sys
import time

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, mode_input, packed_columns

pytestmark = pytest.mark.gpu

TOL = {ata.F64: 1e-12, ata.F32: 2e-5, ata.F32_BF16X3: 2e-5, ata.F32_FP8E4M3: None}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gram(A_np, mode, bounded, lda=None, **opts):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev, dt)
    if lda is not None and lda > A.shape[1]:
        big = torch.zeros((A.shape[0], lda), dtype=dt, device=dev)
        big[:, : A.shape[1]] = A
        A = big[:, : A_np.shape[1]]
    with ata.Handle(split_target=0, balance_tail=0, bounded_workspace=int(bounded), **opts) as h:
        C = ata.gram(A, mode, handle=h)
        torch.cuda.synchronize()
        rep = h.report()
    return C.double().cpu().numpy(), rep


@pytest.mark.parametrize("mode,opts,shape", [
    (ata.F64, dict(leaf_cutoff=128, max_depth=3), (1500, 1300)),
    (ata.F32, dict(leaf_cutoff=256, max_depth=2), (2048, 1800)),
    (ata.F32, dict(leaf_cutoff=512, max_depth=2, leaf_tile=2), (3000, 2600)),
    (ata.F32_BF16X3, dict(leaf_cutoff=256, max_depth=2), (2000, 1500)),
    (ata.F32_BF16X3, dict(leaf_cutoff=512, max_depth=1, leaf_tile=2), (3000, 2600)),
    (ata.F32_FP8E4M3, dict(leaf_cutoff=256, max_depth=1), (1536, 1100)),
])
def test_bounded_matches_resident(mode, opts, shape):
    m, n = shape
    A = mode_input(workloads.uniform(m, n, seed=31, dtype=np.float64), mode)
    _say("case: bounded vs resident", mode, shape, opts)
    got, rb = _gram(A, mode, True, **opts)
    ref_gpu, rr = _gram(A, mode, False, **opts)
    _say(f"  levels {rb['strassen_levels']} workspace bounded {rb['workspace_bytes']} resident {rr['workspace_bytes']}"
         f" launches {rb['kernel_launches']} vs {rr['kernel_launches']}")
    assert rb["multiplications"] == rr["multiplications"]
    assert rb["strassen_levels"] == rr["strassen_levels"] >= 1
    assert rb["workspace_bytes"] < rr["workspace_bytes"]
    assert np.array_equal(got, ref_gpu)
    err = full_error(got, plain.gram_packed(A))
    _say("  e_F", err)
    if TOL[mode] is not None:
        assert err <= TOL[mode]


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3])
def test_bounded_integers_exact(mode):
    rng = np.random.default_rng(33)
    for (m, n, b, depth, lda) in [(777, 1001, 64, 3, None), (1200, 700, 100, 2, 707), (64, 900, 128, 2, None)]:
        A = rng.integers(-3, 4, (m, n)).astype(np.float64 if mode == ata.F64 else np.float32)
        _say("case: bounded ints", mode, m, n, b, depth, lda)
        got, rep = _gram(A, mode, True, lda=lda, leaf_cutoff=b, max_depth=depth)
        assert rep["strassen_levels"] >= 1
        assert np.array_equal(got, plain.gram_packed(A)), (m, n, b, depth)


def test_bounded_spread_check_flagged_nodes():
    """Ill-scaled column blocks flag some AtA nodes: their C21 then comes from
    the plain product of stage 0 and the Strassen stages skip them."""
    A = workloads.scaled_normal(1500, 1200, seed=34, span=1.5)
    opts = dict(leaf_cutoff=128, max_depth=2, spread_tau=20.0)
    _say("case: bounded with flagged nodes")
    got, rb = _gram(A, ata.F32, True, **opts)
    ref_gpu, rr = _gram(A, ata.F32, False, **opts)
    _say("  flagged", rb["flagged_nodes"], rr["flagged_nodes"])
    assert rb["flagged_nodes"] == rr["flagged_nodes"] > 0
    assert np.array_equal(got, ref_gpu)
    assert full_error(got, plain.gram_packed(A)) <= 2e-5


def test_bounded_f64_30000_default_depth_within_sec33():
    """FP64 30000^2, default leaf cutoff (512) and depth: all five Strassen
    levels kept (resident they would need 460 GB), workspace within 3/2 n^2."""
    n = 30000
    free, _ = torch.cuda.mem_get_info()
    if free < 40e9:
        pytest.skip("needs 40 GB of free device memory")
    _say("case: FP64 30000^2 bounded, default depth")
    t0 = time.perf_counter()
    A = workloads.uniform(n, n, seed=1, dtype=np.float64)
    S = workloads.sampled_columns(n, 16, seed=35)
    ref = plain.gram_cols(A, S)
    _say(f"  host input and oracle columns {time.perf_counter() - t0:.1f} s")
    dev = device()
    At = torch.from_numpy(A).to(dev)
    del A
    with ata.Handle(bounded_workspace=1) as h:
        C = ata.gram(At, ata.F64, handle=h)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        C = ata.gram(At, ata.F64, handle=h, out=C)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        rep = h.report()
    got = packed_columns(C.double().cpu().numpy(), n, S)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    _say(f"  {dt:.3f} s ({n ** 3 / dt / 1e12:.1f} TF), levels {rep['strassen_levels']}, workspace "
         f"{rep['workspace_bytes'] / 1e9:.2f} GB (3/2 n^2: {1.5 * n * n * 8 / 1e9:.2f} GB), e_S {err:.2e}")
    assert rep["strassen_levels"] == 5
    assert rep["workspace_bytes"] <= 1.5 * n * n * 8
    assert err <= 1e-12
