"""Batched Gram products (one merged plan, persistent leaf launch, hipGraph)
against the oracle, and graph replays against the eager result."""
import sys

import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import device, full_error

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(seed, count, m_range, n_range, integer=False):
    rng, ms, ns = workloads.batch_shapes(count, seed, m_range, n_range)
    out = []
    for m, n in zip(ms, ns):
        if integer:
            out.append(rng.integers(-2, 3, (int(m), int(n))).astype(np.float32))
        else:
            out.append(rng.uniform(-1, 1, (int(m), int(n))).astype(np.float32))
    return out


def _run(h, mats, mode, lda_pad=0):
    dev = device()
    dt = torch.float64 if mode == ata.F64 else torch.float32
    As = []
    for M in mats:
        t = torch.from_numpy(np.ascontiguousarray(M)).to(dev, dt)
        if lda_pad:
            big = torch.zeros((M.shape[0], M.shape[1] + lda_pad), dtype=dt, device=dev)
            big[:, : M.shape[1]] = t
            t = big[:, : M.shape[1]]
        As.append(t)
    Cs = ata.gram_batched(As, mode, handle=h)
    torch.cuda.synchronize()
    return [C.double().cpu().numpy() for C in Cs], As, Cs


@pytest.fixture(scope="module")
def h():
    device()
    hd = ata.Handle()
    yield hd
    hd.close()


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3, ata.F64])
def test_batch_integer_bit_exact(h, mode):
    mats = _batch(71, 24, (1, 700), (1, 600), integer=True)
    mats += [np.zeros((0, 5), np.float32), np.ones((3, 1), np.float32)]
    if mode == ata.F64:
        mats = [M.astype(np.float64) for M in mats]
    h.set("leaf_cutoff", 128)
    h.set("max_depth", 2)
    _say("case: batch ints mode", mode, "problems", len(mats))
    got, _, _ = _run(h, mats, mode, lda_pad=3)
    for i, (G, M) in enumerate(zip(got, mats)):
        assert np.array_equal(G, plain.gram_packed(M)), (i, M.shape)


def test_batch_random_against_oracle_and_separate_calls(h):
    mats = _batch(72, 40, (64, 2048), (32, 1100))
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 2)
    _say("case: batch random fp32")
    got, As, _ = _run(h, mats, ata.F32)
    for i, (G, M) in enumerate(zip(got, mats)):
        err = full_error(G, plain.gram_packed(M))
        assert err <= 2e-5, (i, M.shape, err)
    # the same problems one call at a time agree to rounding
    for i, A in enumerate(As[:8]):
        one = ata.gram(A, ata.F32, handle=h).double().cpu().numpy()
        assert full_error(got[i], one) <= 1e-6


def test_graph_replays_match_eager(h):
    """Several replays of the captured graph, with eager work and syncs between."""
    mats = _batch(73, 30, (100, 1500), (16, 700))
    dev = device()
    As = [torch.from_numpy(M).to(dev) for M in mats]
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 1)
    h.set("batch_graph", 0)
    eager = [C.clone() for C in ata.gram_batched(As, ata.F32, handle=h)]
    torch.cuda.synchronize()
    h.set("batch_graph", 1)
    outs = [torch.full_like(C, -7.0) for C in eager]
    for rep in range(4):
        _say("case: graph replay", rep)
        for C in outs:
            C.fill_(float(rep))                 # eager work between replays
        ata.gram_batched(As, ata.F32, handle=h, outs=outs)
        torch.cuda.synchronize()
        for i, (C, E) in enumerate(zip(outs, eager)):
            assert torch.equal(C, E), (rep, i)
    # new output pointers with the same shapes reuse the graph
    outs2 = [torch.empty_like(C) for C in eager]
    ata.gram_batched(As, ata.F32, handle=h, outs=outs2)
    torch.cuda.synchronize()
    for C, E in zip(outs2, eager):
        assert torch.equal(C, E)


def test_batch_bad_member_reports_index(h):
    dev = device()
    A = torch.ones((4, 4), dtype=torch.float32, device=dev)
    C = torch.zeros(10, dtype=torch.float32, device=dev)
    with pytest.raises(ata.AtaError):
        ata.ata_gram_batched(h.h, [A.data_ptr(), A.data_ptr()], [4, 4], [4, 4], [4, 2], ata.F32,
                             [C.data_ptr(), C.data_ptr()])
    assert h.report()["m"] == -2


def test_batch_fallback_flags(h):
    """Ill-scaled members take the FP64 fallback inside the batch."""
    mats = [workloads.scaled_normal(600, 300, seed=s, span=1.0) for s in range(4)]
    mats += _batch(74, 6, (100, 800), (50, 400))
    h.set("leaf_cutoff", 64)
    h.set("max_depth", 2)
    h.set("spread_tau", 20.0)
    _say("case: batch fallback")
    got, _, _ = _run(h, mats, ata.F32)
    h.set("spread_tau", 4096)
    for i, (G, M) in enumerate(zip(got, mats)):
        assert full_error(G, plain.gram_packed(M)) <= 2e-5, i


def test_batch_fp8_fallback_matches_single_calls(h):
    """FP8 batch with ill-scaled members: the column norms come from the
    quantisations of each member's column slices, so every member must take
    the same flags as its own ata_gram call (a flag taken differently would
    put FP64 against FP8 results, about 1e-2 apart)."""
    mats = [workloads.scaled_normal(600, 300, seed=s, dtype=np.float32, span=1.0) for s in range(4)]
    mats += _batch(76, 6, (100, 800), (50, 400))
    mats.insert(2, np.zeros((0, 120), dtype=np.float32))      # no rows: its norm pass 1 task stays
    h.set("leaf_cutoff", 64)
    h.set("max_depth", 1)
    h.set("spread_tau", 20.0)
    _say("case: fp8 batch fallback")
    got, _, _ = _run(h, mats, ata.F32_FP8E4M3)
    dev = device()
    flagged = 0
    for i, (G, M) in enumerate(zip(got, mats)):
        if M.shape[0] == 0:
            assert not np.any(G), i
            continue
        one = ata.gram(torch.from_numpy(M).to(dev), ata.F32_FP8E4M3, handle=h).double().cpu().numpy()
        flagged += h.report()["flagged_nodes"]
        assert full_error(G, one) <= 1e-6, i
        assert full_error(G, plain.gram_packed(M)) < 0.1, i
    h.set("spread_tau", 4096)
    assert flagged > 0


def test_batch_fp8_shared_quantisation_matches_single_calls():
    """FP8 members whose leaves are column slices of A made of whole
    128-column blocks (1024 and 2048 columns) read one quantisation of their
    A; merged into a batch, their offsets move with the arena.  With split-K
    and tail cuts off the batch runs each member's own plan, so every member
    must equal its own ata_gram call bit for bit."""
    rng = np.random.default_rng(77)
    shapes = [(700, 1024), (900, 2048), (300, 1100), (1200, 1024), (64, 2048)]
    mats = [(rng.standard_normal((m, n)) * np.exp(rng.uniform(-1, 1, n))).astype(np.float32) for m, n in shapes]
    dev = device()
    with ata.Handle(leaf_cutoff=256, max_depth=0, split_target=0, balance_tail=0) as h2:
        _say("case: fp8 batch, shared quantisations")
        As = [torch.from_numpy(M).to(dev) for M in mats]
        got = [C.double().cpu().numpy() for C in ata.gram_batched(As, ata.F32_FP8E4M3, handle=h2)]
        for i, (A, G) in enumerate(zip(As, got)):
            one = ata.gram(A, ata.F32_FP8E4M3, handle=h2).double().cpu().numpy()
            assert np.array_equal(G, one), (i, shapes[i])
            assert full_error(G, plain.gram_packed(mats[i])) < 0.1, i


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3, ata.F32_FP8E4M3])
def test_persistent_and_grid_launch_agree(h, mode):
    """The persistent leaf launch (per-XCD queues) and the one-workgroup-per-tile
    launch run the same tiles, so the results are bit-identical."""
    mats = _batch(75, 60, (64, 3000), (16, 1300))
    h.set("leaf_cutoff", 256)
    h.set("max_depth", 1)
    dev = device()
    As = [torch.from_numpy(M).to(dev) for M in mats]
    outs = {}
    for pers in (1, 0):
        for graph in (0, 1):
            _say("case: batch launch persistent", pers, "graph", graph, "mode", mode)
            h.set("batch_persistent", pers)
            h.set("batch_graph", graph)
            outs[(pers, graph)] = [C.clone() for C in ata.gram_batched(As, mode, handle=h)]
            torch.cuda.synchronize()
    h.set("batch_persistent", 1)
    h.set("batch_graph", 1)
    ref = outs[(1, 0)]
    for key, got in outs.items():
        for i, (G, R) in enumerate(zip(got, ref)):
            assert torch.equal(G, R), (key, i)
    if mode != ata.F32_FP8E4M3:
        for i in range(0, len(mats), 7):
            assert full_error(ref[i].double().cpu().numpy(), plain.gram_packed(mats[i])) <= 2e-5
