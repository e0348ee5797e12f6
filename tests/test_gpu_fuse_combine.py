"""Strassen combine in the leaf epilogues (ATA_OPT_FUSE_COMBINE): a node whose
seven products are leaves has no product buffers and no combine pass; each
product's leaf adds itself into its quadrants in five launch rounds, in the
combine's own order.  With split-K and tail cuts off both schedules run the
same leaves and the same additions, so the result must equal the default
schedule's bit for bit; on small integers it must equal the plain FP64
oracle exactly, and on random data it must be within the mode's tolerance.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error, mode_input

pytestmark = pytest.mark.gpu

TOL = {ata.F64: 1e-12, ata.F32: 2e-5, ata.F32_BF16X3: 2e-5, ata.F32_FP8E4M3: None}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tensor(A_np, mode, lda=None):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev, dt)
    if lda is not None and lda > A.shape[1]:
        big = torch.zeros((A.shape[0], lda), dtype=dt, device=dev)
        big[:, : A.shape[1]] = A
        A = big[:, : A_np.shape[1]]
    return A


def _gram(A_np, mode, fuse, lda=None, calls=1, **opts):
    A = _tensor(A_np, mode, lda)
    with ata.Handle(split_target=0, balance_tail=0, fuse_combine=int(fuse), **opts) as h:
        outs = []
        for _ in range(calls):
            outs.append(ata.gram(A, mode, handle=h).double().cpu().numpy())
        torch.cuda.synchronize()
        rep = h.report()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])            # a second call reuses the plan
    return outs[0], rep


@pytest.mark.parametrize("mode,opts,shape", [
    (ata.F64, dict(leaf_cutoff=128, max_depth=1), (1000, 1000)),
    (ata.F64, dict(leaf_cutoff=128, max_depth=3), (1501, 1299)),
    (ata.F32, dict(leaf_cutoff=256, max_depth=2), (2048, 1800)),
    (ata.F32, dict(leaf_cutoff=512, max_depth=2, leaf_tile=2), (3000, 2600)),
    (ata.F32, dict(leaf_cutoff=256, max_depth=1, leaf_persistent=1), (1999, 1501)),
    (ata.F32_BF16X3, dict(leaf_cutoff=256, max_depth=2), (2047, 1500)),
    (ata.F32_BF16X3, dict(leaf_cutoff=512, max_depth=1, leaf_tile=2), (3000, 2600)),
    (ata.F32_BF16X3, dict(leaf_cutoff=256, max_depth=1, leaf_tile=1), (1800, 1700)),
    (ata.F32_BF16X3, dict(leaf_cutoff=512, max_depth=1, leaf_tile=4), (2600, 2300)),
    (ata.F32_FP8E4M3, dict(leaf_cutoff=256, max_depth=1), (1536, 1100)),
    (ata.F32_FP8E4M3, dict(leaf_cutoff=512, max_depth=1, leaf_tile=3), (2048, 2048)),
    # FP32 with the fused pre-sums as well: both ends of the products fused
    (ata.F32, dict(leaf_cutoff=256, max_depth=2, fuse_presum=1), (1700, 1500)),
])
def test_epilogue_combine_matches_default_schedule(mode, opts, shape):
    A = mode_input(workloads.uniform(*shape, seed=51, dtype=np.float64), mode)
    _say("case: epilogue combine", mode, shape, opts)
    got, rf = _gram(A, mode, True, calls=2, **opts)
    ref_gpu, rd = _gram(A, mode, False, **opts)
    _say(f"  rounds {rf['leaf_rounds']} launches {rf['kernel_launches']} vs {rd['kernel_launches']} "
         f"workspace {rf['workspace_bytes']} vs {rd['workspace_bytes']} levels {rf['strassen_levels']}")
    assert rf["leaf_rounds"] == 5 and rd["leaf_rounds"] == 1
    assert rf["multiplications"] == rd["multiplications"] and rf["strassen_levels"] >= 1
    assert rf["workspace_bytes"] < rd["workspace_bytes"]
    assert np.array_equal(got, ref_gpu)
    err = full_error(got, plain.gram_packed(A))
    _say("  e_F", err)
    if TOL[mode] is not None:
        assert err <= TOL[mode]


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3])
def test_epilogue_combine_integers_exact(mode):
    rng = np.random.default_rng(52)
    for (m, n, b, depth, lda) in [(777, 1001, 64, 3, None), (1200, 700, 100, 2, 707), (64, 900, 128, 2, None)]:
        A = rng.integers(-3, 4, (m, n)).astype(np.float64 if mode == ata.F64 else np.float32)
        _say("case: epilogue combine ints", mode, m, n, b, depth, lda)
        got, rep = _gram(A, mode, True, lda=lda, leaf_cutoff=b, max_depth=depth)
        assert rep["leaf_rounds"] == 5
        assert np.array_equal(got, plain.gram_packed(A)), (m, n, b, depth)


def test_epilogue_combine_flagged_nodes():
    """Ill-scaled column blocks flag AtA nodes: their C21 comes from the plain
    product, and the fused Strassen leaves of those nodes skip themselves."""
    A = workloads.scaled_normal(1500, 1200, seed=53, span=1.5)
    opts = dict(leaf_cutoff=128, max_depth=2, spread_tau=20.0)
    _say("case: epilogue combine with flagged nodes")
    got, rf = _gram(A, ata.F32, True, **opts)
    ref_gpu, rd = _gram(A, ata.F32, False, **opts)
    assert rf["flagged_nodes"] == rd["flagged_nodes"] > 0
    assert np.array_equal(got, ref_gpu)
    assert full_error(got, plain.gram_packed(A)) <= 2e-5


def test_epilogue_combine_default_splits_within_tolerance():
    """With the default split-K target and tail balancing, leaves that do not
    combine in their epilogue may be cut differently: rounding only."""
    A = mode_input(workloads.uniform(4000, 1500, seed=54, dtype=np.float64), ata.F32)
    dev_A = _tensor(A, ata.F32)
    outs = {}
    for fuse in (1, 0):
        with ata.Handle(leaf_cutoff=256, max_depth=2, fuse_combine=fuse) as h:
            outs[fuse] = ata.gram(dev_A, ata.F32, handle=h).double().cpu().numpy()
            rep = h.report()
        if fuse:
            assert rep["leaf_rounds"] == 5
    ref = plain.gram_packed(A)
    assert full_error(outs[1], ref) <= 2e-5
    assert full_error(outs[1], outs[0]) <= 1e-6


def test_epilogue_combine_not_with_four_wave_256_tiles():
    """The 256 x 256 four-wave FP32 and split-BF16 tiles are not built with
    epilogue combines: such plans run the combine pass as usual."""
    A = mode_input(workloads.uniform(2100, 2048, seed=55, dtype=np.float64), ata.F32)
    for mode in (ata.F32, ata.F32_BF16X3):
        got, rep = _gram(A, mode, True, leaf_cutoff=512, max_depth=1, leaf_tile=3)
        assert rep["leaf_rounds"] == 1 and rep["strassen_levels"] == 1
        assert full_error(got, plain.gram_packed(A)) <= 2e-5


def test_epilogue_combine_gemm_tn():
    """General product C = A^T B: the same plan with and without epilogue
    combines, bit for bit, and exact on integers."""
    rng = np.random.default_rng(56)
    dev = device()
    for mode in (ata.F64, ata.F32):
        dt = torch.float64 if mode == ata.F64 else torch.float32
        npdt = np.float64 if mode == ata.F64 else np.float32
        for integer in (True, False):
            m, n, k = 1300, 900, 1100
            if integer:
                A = rng.integers(-3, 4, (m, n)).astype(npdt)
                B = rng.integers(-3, 4, (m, k)).astype(npdt)
            else:
                A = rng.uniform(-1, 1, (m, n)).astype(npdt)
                B = rng.uniform(-1, 1, (m, k)).astype(npdt)
            At = torch.from_numpy(A).to(dev, dt)
            Bt = torch.from_numpy(B).to(dev, dt)
            outs = {}
            for fuse in (1, 0):
                with ata.Handle(split_target=0, balance_tail=0, leaf_cutoff=128, max_depth=2,
                                fuse_combine=fuse) as h:
                    C = torch.full((n, k), 7.0, dtype=dt, device=dev)
                    ata.ata_gemm_tn(h.h, At.data_ptr(), Bt.data_ptr(), m, n, k, n, k, mode, C.data_ptr(), k,
                                    torch.cuda.current_stream().cuda_stream)
                    torch.cuda.synchronize()
                    outs[fuse] = C.double().cpu().numpy()
                    if fuse:
                        assert h.report()["leaf_rounds"] == 5
            assert np.array_equal(outs[1], outs[0]), (mode, integer)
            ref = A.astype(np.float64).T @ B.astype(np.float64)
            if integer:
                assert np.array_equal(outs[1], ref)
            else:
                tol = 1e-12 if mode == ata.F64 else 2e-5
                assert np.linalg.norm(outs[1] - ref) / np.linalg.norm(ref) <= tol


def test_epilogue_combine_noalloc():
    """ata_gram_noalloc with epilogue combines equals ata_gram's result."""
    A = mode_input(workloads.uniform(1500, 1100, seed=57, dtype=np.float64), ata.F32)
    At = _tensor(A, ata.F32)
    n = A.shape[1]
    with ata.Handle(leaf_cutoff=128, max_depth=2, fuse_combine=1, split_target=0) as h:
        C1 = torch.full((n * (n + 1) // 2,), np.nan, dtype=torch.float32, device=device())
        ata.ata_gram_noalloc(h.h, At.data_ptr(), A.shape[0], n, At.stride(0), ata.F32, C1.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
        C2 = ata.gram(At, ata.F32, handle=h)
        torch.cuda.synchronize()
        assert h.report()["leaf_rounds"] == 5
    assert torch.equal(C1, C2)
    assert full_error(C1.double().cpu().numpy(), plain.gram_packed(A)) <= 2e-5
