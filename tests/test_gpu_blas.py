"""BLAS-style forms around the AtA product: alpha/beta scaling, A A^T, and
unpacking to a full symmetric matrix, against the plain FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata
from gpu_helpers import device, full_error

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3])
def test_gram_scaled_integers_bit_exact(mode):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    rng = np.random.default_rng(111)
    m, n = 700, 301
    A = rng.integers(-2, 3, (m, n)).astype(np.float64)
    C0 = rng.integers(-50, 50, n * (n + 1) // 2).astype(np.float64)
    At = torch.from_numpy(A).to(dev, dt)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 64)
        h.set("max_depth", 2)
        for alpha, beta in [(2.0, -3.0), (-1.0, 0.0), (1.0, 1.0), (0.5, 0.25)]:
            _say("case: gram_scaled mode", mode, alpha, beta)
            C = torch.from_numpy(C0).to(dev, dt)
            ata.ata_gram_scaled(h.h, At.data_ptr(), m, n, n, mode, alpha, beta, C.data_ptr())
            torch.cuda.synchronize()
            ref = alpha * plain.gram_packed(A) + beta * C0
            assert np.array_equal(C.double().cpu().numpy(), ref), (alpha, beta)
    finally:
        h.close()


def test_gram_scaled_beta_zero_ignores_nan_in_c():
    dev = device()
    A = torch.ones((10, 4), device=dev)
    C = torch.full((10,), float("nan"), device=dev)
    h = ata.Handle()
    try:
        ata.ata_gram_scaled(h.h, A.data_ptr(), 10, 4, 4, ata.F32, 3.0, 0.0, C.data_ptr())
        torch.cuda.synchronize()
        assert torch.equal(C, torch.full((10,), 30.0, device=dev))
        with pytest.raises(ata.AtaError):
            ata.ata_gram_scaled(h.h, A.data_ptr(), 10, 4, 4, ata.F32, float("inf"), 0.0, C.data_ptr())
    finally:
        h.close()


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3, ata.F32_FP8E4M3])
def test_gram_aat(mode):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    rng = np.random.default_rng(112)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 128)
        h.set("max_depth", 1)
        for (m, n, lda) in [(333, 1000, 1000), (129, 77, 80), (1, 5, 5)]:
            A = rng.integers(-2, 3, (m, n)).astype(np.float64)
            big = np.zeros((m, lda))
            big[:, :n] = A
            At = torch.from_numpy(big).to(dev, dt)
            C = torch.empty(m * (m + 1) // 2, dtype=dt, device=dev)
            _say("case: gram_aat mode", mode, m, n, lda)
            ata.ata_gram_aat(h.h, At.data_ptr(), m, n, lda, mode, C.data_ptr())
            torch.cuda.synchronize()
            assert np.array_equal(C.double().cpu().numpy(), plain.gram_packed(np.ascontiguousarray(A.T)))
        A = rng.uniform(-1, 1, (500, 2000))
        At = torch.from_numpy(A).to(dev, dt)
        C = torch.empty(500 * 501 // 2, dtype=dt, device=dev)
        ata.ata_gram_aat(h.h, At.data_ptr(), 500, 2000, 2000, mode, C.data_ptr())
        torch.cuda.synchronize()
        err = full_error(C.double().cpu().numpy(), plain.gram_packed(np.ascontiguousarray(A.T).astype(
            np.float64 if mode == ata.F64 else np.float32)))
        _say("  random error", err)
        assert err <= (1e-12 if mode == ata.F64 else 2e-5 if mode != ata.F32_FP8E4M3 else 0.1)
    finally:
        h.close()


def test_unpack_full_symmetric():
    dev = device()
    rng = np.random.default_rng(113)
    for n, ldf in [(1, 1), (300, 300), (257, 260)]:
        Cp = rng.standard_normal(n * (n + 1) // 2).astype(np.float32)
        F = torch.full((n, ldf), -9.0, device=dev)
        h = ata.Handle()
        try:
            ata.ata_unpack(h.h, torch.from_numpy(Cp).to(dev).data_ptr(), n, ata.F32, F.data_ptr(), ldf)
            torch.cuda.synchronize()
        finally:
            h.close()
        got = F.cpu().numpy()
        i, j = np.tril_indices(n)
        full = np.zeros((n, n), np.float32)
        full[i, j] = Cp
        full[j, i] = Cp
        assert np.array_equal(got[:, :n], full)
        assert np.all(got[:, n:] == -9.0)
