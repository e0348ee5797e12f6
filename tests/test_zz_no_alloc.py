"""ata_gram_noalloc (the entry point that allocates nothing: every workspace
buffer lives in the GPU's static array) against ata_gram, through the C ABI.

Each case runs two calls in a row on one stream, the second on a smaller
input, and checks both against ata_gram's output for the same handle options
(bit for bit: the plans agree) and against the plain FP64 oracle within the
mode's tolerance.
"""
import numpy as np
import pytest
import torch

from oracle import plain
from paper_2110_13042_amd import ata, workloads

from gpu_helpers import device, full_error, mode_input

pytestmark = pytest.mark.gpu

TOL = {ata.F64: 1e-12, ata.F32: 2e-5, ata.F32_BF16X3: 2e-5, ata.F32_FP8E4M3: None}


def _tensor(A_np, mode):
    dt = torch.float64 if mode == ata.F64 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(A_np)).to(device(), dt)


def _empty(n, mode, fill=np.nan):
    dt = torch.float64 if mode == ata.F64 else torch.float32
    return torch.full((n * (n + 1) // 2,), fill, dtype=dt, device=device())


def _call(fn, h, A, mode, C):
    m, n = A.shape
    fn(h.h, A.data_ptr(), m, n, A.stride(0), mode, C.data_ptr(),
       torch.cuda.current_stream(A.device).cuda_stream)


@pytest.mark.parametrize("mode,opts,shapes", [
    (ata.F32, dict(leaf_cutoff=128, max_depth=2), [(1500, 1100), (700, 517)]),
    (ata.F32_BF16X3, dict(leaf_cutoff=128, max_depth=2), [(1300, 1030), (611, 333)]),
    (ata.F64, dict(leaf_cutoff=128, max_depth=3), [(900, 777), (400, 301)]),
    (ata.F32_FP8E4M3, dict(leaf_cutoff=256, max_depth=1), [(1024, 1000), (512, 300)]),
    # 256 x 256 FP32 tile: persistent leaf launch with its queue heads in the
    # array (no split-K: its partials would pass the array and change the plan)
    (ata.F32, dict(leaf_cutoff=1024, max_depth=1, leaf_tile=2, split_target=0), [(2304, 2200), (1200, 1100)]),
    # split-BF16 256 x 256 tile, split-K on a tall input
    (ata.F32_BF16X3, dict(leaf_tile=2, max_depth=0), [(12000, 600), (5000, 300)]),
])
def test_noalloc_matches_gram_two_calls(mode, opts, shapes):
    rng_seeds = [11, 12]
    inputs = [mode_input(workloads.uniform(m, n, seed=s, dtype=np.float64), mode)
              for (m, n), s in zip(shapes, rng_seeds)]
    As = [_tensor(a, mode) for a in inputs]
    with ata.Handle(**opts) as h:
        # the static-workspace calls, back to back on one stream, then one sync
        outs = [_empty(a.shape[1], mode) for a in inputs]
        reps = []
        for A, C in zip(As, outs):
            _call(ata.ata_gram_noalloc, h, A, mode, C)
            reps.append(h.report())
        torch.cuda.synchronize()
        got = [C.double().cpu().numpy() for C in outs]
    with ata.Handle(**opts) as h:
        refs_gpu = []
        for A, rep in zip(As, reps):
            C = _empty(A.shape[1], mode)
            _call(ata.ata_gram, h, A, mode, C)
            torch.cuda.synchronize()
            r2 = h.report()
            # same plan, hence the same arithmetic (ata_gram may split the leaf
            # launch in two to overlap the pre-sums: same tiles, one more launch)
            for k in ("multiplications", "strassen_levels", "leaf_tile", "leaf_cutoff",
                      "tail_split_leaves", "tail_split_chunks", "workspace_bytes", "leaf_persistent"):
                assert rep[k] == r2[k], (k, rep[k], r2[k])
            refs_gpu.append(C.double().cpu().numpy())
    for a, g, r in zip(inputs, got, refs_gpu):
        assert np.array_equal(g, r), "ata_gram_noalloc differs from ata_gram"
        ref = plain.gram_packed(a)
        err = full_error(g, ref)
        print(f"mode {mode} {a.shape}: rel err {err:.3e}")
        if TOL[mode] is not None:
            assert err <= TOL[mode]
    if mode != ata.F32_FP8E4M3 and opts.get("max_depth", 0) > 0:
        assert reps[0]["strassen_levels"] >= 1


def test_noalloc_integers_bit_exact_and_depth_lowered():
    """A plan whose default workspace passes the array gets fewer Strassen
    levels; the result equals ata_gram's with the depth it used, and integer
    inputs are exact."""
    m, n = 4096, 4096
    rng = np.random.default_rng(5)
    a = rng.integers(-3, 4, size=(m, n)).astype(np.float32)
    A = _tensor(a, ata.F32)
    with ata.Handle(leaf_cutoff=512, max_depth=3, leaf_tile=0) as h:
        C = _empty(n, ata.F32)
        _call(ata.ata_gram_noalloc, h, A, ata.F32, C)
        torch.cuda.synchronize()
        rep = h.report()
        assert rep["workspace_bytes"] <= ata.NOALLOC_SCRATCH_BYTES
        full = ata.ata_plan_query(m, n, ata.F32, 512, 3)[0]
        assert full["workspace_bytes"] > ata.NOALLOC_SCRATCH_BYTES
        assert rep["strassen_levels"] < 3
        got = C.double().cpu().numpy()
    with ata.Handle(leaf_cutoff=512, max_depth=rep["strassen_levels"], leaf_tile=0) as h:
        C2 = _empty(n, ata.F32)
        _call(ata.ata_gram, h, A, ata.F32, C2)
        torch.cuda.synchronize()
        assert np.array_equal(got, C2.double().cpu().numpy())
    ref = plain.gram_packed(a)
    assert np.array_equal(got, ref)


def test_noalloc_rejects_what_the_array_cannot_hold():
    """split-BF16 packs 4 bytes per element of A: 8192 x 8192 needs 256 MiB of
    packed operands plus the rest, above the array; the call fails with
    ATA_ERR_OUT_OF_MEMORY and leaves C untouched."""
    m = n = 8192
    A = torch.ones((m, n), dtype=torch.float32, device=device())
    C = _empty(n, ata.F32_BF16X3, fill=7.0)
    with ata.Handle() as h:
        with pytest.raises(ata.AtaError) as ei:
            _call(ata.ata_gram_noalloc, h, A, ata.F32_BF16X3, C)
        assert ei.value.status == 3
        h.set("residual", 1)
        small = _tensor(np.ones((64, 64), np.float32), ata.F32)
        Cs = _empty(64, ata.F32, fill=7.0)
        with pytest.raises(ata.AtaError) as ei:
            _call(ata.ata_gram_noalloc, h, small, ata.F32, Cs)
        assert ei.value.status == 2
    torch.cuda.synchronize()
    assert bool((C == 7.0).all()) and bool((Cs == 7.0).all())


def test_noalloc_degenerate_shapes():
    with ata.Handle() as h:
        C = _empty(5, ata.F32, fill=3.0)
        A = torch.empty((0, 5), dtype=torch.float32, device=device())
        ata.ata_gram_noalloc(h.h, A.data_ptr(), 0, 5, 5, ata.F32, C.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert bool((C == 0).all())
        ata.ata_gram_noalloc(h.h, 0, 7, 0, 1, ata.F32, 0, torch.cuda.current_stream().cuda_stream)
