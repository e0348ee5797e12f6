"""The FP64 sampled-column check on the GPU (ata_check_columns) against the
same measure computed on the host from the FP64 oracle's columns."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, packed_columns

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host_measure(Cp_host, A, S):
    n = A.shape[1]
    got = packed_columns(Cp_host, n, S)
    ref = plain.gram_cols(A, S)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("mode", [ata.F64, ata.F32, ata.F32_BF16X3])
def test_check_columns_matches_host_measure(mode):
    dev = device()
    h = ata.Handle()
    rng = np.random.default_rng(81)
    dt = torch.float64 if mode == ata.F64 else torch.float32
    try:
        for (m, n, count, lda) in [(1000, 777, 37, 777), (3001, 1500, 64, 1503), (17, 5, 5, 5)]:
            _say("case: check columns", mode, m, n, count, lda)
            A = rng.uniform(-1, 1, (m, n))
            if mode != ata.F64:
                A = A.astype(np.float32)
            At = torch.zeros((m, lda), dtype=dt, device=dev)
            At[:, :n] = torch.from_numpy(A).to(dev, dt)
            C = torch.empty(n * (n + 1) // 2, dtype=dt, device=dev)
            sp = torch.cuda.current_stream(dev).cuda_stream
            ata.ata_gram(h.h, At.data_ptr(), m, n, lda, mode, C.data_ptr(), sp)
            S = rng.choice(n, size=count, replace=False)
            r_gpu = ata.ata_check_columns(h.h, At.data_ptr(), m, n, lda, mode, C.data_ptr(), S, sp)
            r_host = _host_measure(C.double().cpu().numpy(), A.astype(np.float64), S)
            _say("  gpu", r_gpu, "host", r_host)
            assert abs(r_gpu - r_host) <= 1e-6 * r_host + 1e-15
    finally:
        h.close()


def test_check_columns_exact_and_planted_error():
    """Integers: the product is exact, so the measure is 0; one entry moved by
    delta in a sampled column gives exactly delta / ||ref_S||."""
    dev = device()
    rng = np.random.default_rng(82)
    m, n = 500, 300
    A = rng.integers(-3, 4, (m, n)).astype(np.float32)
    At = torch.from_numpy(A).to(dev)
    h = ata.Handle()
    try:
        C = ata.gram(At, ata.F32, handle=h)
        sp = torch.cuda.current_stream(dev).cuda_stream
        S = [0, 7, 150, 299, 7]
        assert ata.ata_check_columns(h.h, At.data_ptr(), m, n, n, ata.F32, C.data_ptr(), S, sp) == 0.0
        # plant: C[200][150] += 64 (lower entry of sampled column 150)
        p = 200 * 201 // 2 + 150
        C[p] += 64.0
        torch.cuda.synchronize()
        r = ata.ata_check_columns(h.h, At.data_ptr(), m, n, n, ata.F32, C.data_ptr(), S, sp)
        ref = plain.gram_cols(A.astype(np.float64), np.array(S))
        want = 64.0 / np.linalg.norm(ref)
        _say("planted", r, want)
        assert abs(r - want) <= 1e-12 * want
        # an index out of range is refused before any device work
        with pytest.raises(ata.AtaError):
            ata.ata_check_columns(h.h, At.data_ptr(), m, n, n, ata.F32, C.data_ptr(), [0, n], sp)
    finally:
        h.close()
