"""ata_gram captured in a caller's HIP graph (torch.cuda.CUDAGraph): once
the plan is cached and the workspace reserved by a first call, the call
enqueues kernels only (no allocation, no memset node, no host sync), so its
replays must reproduce eager calls.  The graph reads A in place: A is
rewritten between replays, with eager work and synchronisations in between,
and every replay is compared with an eager call on the same data."""
import sys

import numpy as np
import pytest
import torch

from paper_2110_13042_amd import ata
from gpu_helpers import device

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode,tile,b,depth", [(ata.F32, 3, 512, 1), (ata.F32_BF16X3, 2, 256, 0),
                                               (ata.F64, 0, 256, 1), (ata.F32, 0, 256, 2)])
def test_gram_graph_replays_match_eager(mode, tile, b, depth):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    m, n = 1500, 1300
    rng = np.random.default_rng(91)
    h = ata.Handle()
    h.set("leaf_tile", tile)
    h.set("leaf_cutoff", b)
    h.set("max_depth", depth)
    A = torch.from_numpy(rng.uniform(-1, 1, (m, n))).to(dev, dt)
    C = torch.empty(n * (n + 1) // 2, dtype=dt, device=dev)
    s = torch.cuda.Stream(device=dev)
    try:
        with torch.cuda.stream(s):
            ata.ata_gram(h.h, A.data_ptr(), m, n, n, mode, C.data_ptr(), s.cuda_stream)   # plan + workspace
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ata.ata_gram(h.h, A.data_ptr(), m, n, n, mode, C.data_ptr(), s.cuda_stream)
        torch.cuda.synchronize()
        for rep in range(3):
            _say("case: graph replay", mode, tile, b, depth, "replay", rep)
            A.copy_(torch.from_numpy(rng.uniform(-1, 1, (m, n))).to(dev, dt))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = C.clone()
            C.fill_(float("nan"))
            ref = ata.gram(A, mode, handle=h)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), rep
        del g
    finally:
        torch.cuda.synchronize()
        h.close()
