"""General product C = A^T B (ata_gemm_tn: the Strassen recursion on its own)
against the plain FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata
from gpu_helpers import device

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _padded(M, pad, dt, dev):
    t = torch.zeros((M.shape[0], M.shape[1] + pad), dtype=dt, device=dev)
    t[:, : M.shape[1]] = torch.from_numpy(np.ascontiguousarray(M)).to(dev, dt)
    return t


def _run(h, A, B, mode, pads=(0, 0, 0)):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    m, n = A.shape
    k = B.shape[1]
    At, Bt = _padded(A, pads[0], dt, dev), _padded(B, pads[1], dt, dev)
    C = torch.full((n, k + pads[2]), 7.0, dtype=dt, device=dev)
    ata.ata_gemm_tn(h.h, At.data_ptr(), Bt.data_ptr(), m, n, k, n + pads[0], k + pads[1], mode,
                    C.data_ptr(), k + pads[2], torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = C.double().cpu().numpy()
    if pads[2]:
        assert np.all(out[:, k:] == 7.0)            # the padding columns of C are untouched
    return out[:, :k]


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3, ata.F32_FP8E4M3])
def test_gemm_tn_small_integers_bit_exact(mode):
    rng = np.random.default_rng(101)
    h = ata.Handle()
    try:
        for (m, n, k, b, depth, pads) in [(300, 257, 190, 64, 2, (3, 0, 5)), (129, 65, 400, 128, 1, (0, 1, 0)),
                                          (1000, 300, 300, 128, 1, (0, 0, 0)), (5, 3, 7, 64, 0, (1, 1, 1)),
                                          (20000, 200, 150, 128, 0, (0, 0, 0))]:
            if mode == ata.F32_FP8E4M3 and depth > 1:
                depth = 1
            A = rng.integers(-2, 3, (m, n)).astype(np.float64)
            B = rng.integers(-2, 3, (m, k)).astype(np.float64)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            _say("case: gemm_tn int mode", mode, m, n, k, b, depth, pads)
            got = _run(h, A, B, mode, pads)
            assert np.array_equal(got, plain.gemm_tn(A, B)), (m, n, k, b, depth)
    finally:
        h.close()


@pytest.mark.parametrize("mode,tol", [(ata.F64, 1e-12), (ata.F32, 2e-5), (ata.F32_BF16X3, 2e-5),
                                      (ata.F32_FP8E4M3, None)])
def test_gemm_tn_random_against_oracle(mode, tol):
    rng = np.random.default_rng(102)
    m, n, k = 3000, 1100, 900
    A = rng.uniform(-1, 1, (m, n))
    B = rng.uniform(-1, 1, (m, k))
    if mode != ata.F64:
        A, B = A.astype(np.float32), B.astype(np.float32)
    ref = plain.gemm_tn(A, B)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 256)
        h.set("max_depth", 2 if mode != ata.F32_FP8E4M3 else 1)
        _say("case: gemm_tn random mode", mode)
        got = _run(h, A, B, mode)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("  error", err, "levels", h.report()["strassen_levels"])
        assert h.report()["strassen_levels"] >= 1
        if tol is not None:
            assert err <= tol
        else:
            assert err < 0.1
    finally:
        h.close()


def test_gemm_tn_degenerate_and_errors():
    dev = device()
    h = ata.Handle()
    try:
        A = torch.zeros((0, 5), device=dev)
        B = torch.zeros((0, 3), device=dev)
        C = ata.gemm_tn(A, B, handle=h)                    # m = 0: zeros
        torch.cuda.synchronize()
        assert C.shape == (5, 3) and float(C.abs().max()) == 0.0
        A = torch.ones((4, 4), device=dev)
        with pytest.raises(ata.AtaError):                  # C overlapping B
            ata.ata_gemm_tn(h.h, A.data_ptr(), A.data_ptr(), 4, 4, 4, 4, 4, ata.F32, A.data_ptr(), 4)
        with pytest.raises(ata.AtaError):                  # ldb < k
            ata.ata_gemm_tn(h.h, A.data_ptr(), A.data_ptr(), 4, 4, 4, 4, 3, ata.F32, A.data_ptr(), 4)
    finally:
        h.close()
