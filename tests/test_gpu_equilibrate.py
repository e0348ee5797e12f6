"""Column equilibration (exact power-of-two column scaling) as the alternative
to the FP64 fallback for ill-scaled columns, against the FP64 oracle."""
import sys

import numpy as np
import pytest

from oracle import plain
from paper_2110_13042_amd import ata, workloads
from gpu_helpers import full_error, run_gram

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scaled_error(Cp, ref):
    n = int((np.sqrt(8 * len(ref) + 1) - 1) / 2)
    i, j = np.tril_indices(n)
    idx = np.arange(n)
    d = np.sqrt(ref[idx * (idx + 1) // 2 + idx])
    w = d[i] * d[j]
    return full_error(Cp / w, ref / w)


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3])
def test_equilibrate_power_of_two_scaled_integers_bit_exact(mode):
    rng = np.random.default_rng(121)
    h = ata.Handle(equilibrate=1)
    try:
        for (m, n, b, depth) in [(500, 300, 64, 2), (2000, 130, 128, 1), (20000, 200, 128, 0)]:
            A = rng.integers(-2, 3, (m, n)).astype(np.float64) * 2.0 ** rng.integers(-20, 21, n)
            A = A.astype(np.float32)
            h.set("leaf_cutoff", b)
            h.set("max_depth", depth)
            _say("case: equilibrate ints mode", mode, m, n, b, depth)
            assert np.array_equal(run_gram(A, mode, h), plain.gram_packed(A)), (m, n)
    finally:
        h.close()


@pytest.mark.parametrize("mode", [ata.F32, ata.F32_BF16X3])
def test_equilibrate_ill_scaled_columns(mode):
    A = workloads.scaled_normal(20000, 600, seed=122, span=3.0)
    ref = plain.gram_packed(A)
    out = {}
    for name, opts in [("equilibrate", dict(equilibrate=1)), ("fallback", {}), ("neither", dict(spread_tau=0))]:
        h = ata.Handle(**opts)
        try:
            h.set("leaf_cutoff", 128)
            h.set("max_depth", 2)
            Cp = run_gram(A, mode, h)
            out[name] = (full_error(Cp, ref), _scaled_error(Cp, ref), h.report()["flagged_nodes"])
            _say("  mode", mode, name, "e_F %.3e e_D %.3e flagged %d" % out[name])
        finally:
            h.close()
    e_f, e_d, flagged = out["equilibrate"]
    assert flagged == -1                 # no spread check on the scaled copy
    assert e_f <= 2e-5
    assert e_d <= 1e-5
    assert e_d <= out["neither"][1]      # scaling never hurts the column-relative error
