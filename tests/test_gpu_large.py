"""Launches of more than 2^32 work-items.  A dispatch holds its grid size in
work-items as a 32-bit count, so the streaming kernels walk virtual blocks
on a capped grid.  A 50000^2 FP32 product with two Strassen levels has a
second-level pre-sum launch of about 4.4e9 items (one column per item: the
level-1 sums' rows are not 16-byte aligned); every sampled column must match
the FP64 oracle.  Needs about 200 GB of free device memory."""
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


def test_presum_launch_beyond_32_bit_work_items():
    dev = device()
    n = 50000
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(dev)
    if free < 200e9:
        pytest.skip(f"needs about 200 GB of free device memory, {free / 1e9:.0f} GB free")
    A_np = workloads.uniform(n, n, seed=50, dtype=np.float32)
    S = workloads.sampled_columns(n, 8, seed=51)
    ref = plain.gram_cols(A_np, S)
    A = torch.from_numpy(A_np).to(dev)
    del A_np
    C = torch.empty(n * (n + 1) // 2, dtype=torch.float32, device=dev)
    h = ata.Handle(spread_tau=0)
    try:
        h.set("leaf_cutoff", 1024)
        h.set("max_depth", 2)
        _say("case: 50000^2 FP32, b 1024, depth 2")
        ata.ata_gram(h.h, A.data_ptr(), n, n, n, ata.F32, C.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert h.report()["strassen_levels"] == 2
        got = packed_columns(C.double().cpu().numpy(), n, S)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("  e_S", err)
        assert err <= 2e-5
    finally:
        h.close()


def test_split_bf16_beyond_the_whole_a_packing():
    """50000^2 split-BF16: A's whole hi/lo packing would pass the 4 GiB reach
    of a buffer resource, so every leaf operand gets a packing of its own.
    Small integers make every product and sum exact: sampled columns must
    equal the oracle's bit for bit."""
    dev = device()
    n = 50000
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(dev)
    if free < 200e9:
        pytest.skip(f"needs about 200 GB of free device memory, {free / 1e9:.0f} GB free")
    rng = np.random.default_rng(52)
    A_np = np.empty((n, n), dtype=np.float32)
    for r0 in range(0, n, 5000):
        A_np[r0:r0 + 5000] = rng.integers(-2, 3, (min(n, r0 + 5000) - r0, n))
    S = workloads.sampled_columns(n, 8, seed=53)
    ref = plain.gram_cols(A_np, S)
    A = torch.from_numpy(A_np).to(dev)
    del A_np
    C = torch.empty(n * (n + 1) // 2, dtype=torch.float32, device=dev)
    h = ata.Handle()
    try:
        h.set("leaf_cutoff", 2048)
        h.set("max_depth", 1)
        h.set("leaf_tile", 2)
        _say("case: 50000^2 split-BF16 integers, b 2048, depth 1")
        ata.ata_gram(h.h, A.data_ptr(), n, n, n, ata.F32_BF16X3, C.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert h.report()["strassen_levels"] == 1
        got = packed_columns(C.double().cpu().numpy(), n, S)
        assert np.array_equal(got, ref)
    finally:
        h.close()
