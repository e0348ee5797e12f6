"""Host-side checks of the C ABI: the library loads, exports what the header
declares, plans like the oracle's recursion, and rejects bad arguments before
touching a device (CPU only)."""
import ctypes
import os

import numpy as np
import pytest

from oracle import recursive
from paper_2110_13042_amd import ata

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    syms = ata.header_symbols()
    assert {"ata_create", "ata_gram", "ata_gram_batched", "ata_destroy"} <= set(syms)
    lib = ata.lib()
    for s in syms:
        assert hasattr(lib, s), s


def test_status_strings():
    for code, name in ata.STATUS.items():
        assert ata.status_string(code) == name


@pytest.mark.parametrize("m,n,b,depth", [(1024, 1024, 256, -1), (8192, 8192, 1024, 3),
                                         (8192, 8192, 512, 3), (262144, 4096, 1024, 3),
                                         (300, 257, 16, 2), (1000, 999, 100, 4), (50, 37, 5, 64)])
def test_plan_matches_oracle_recursion(m, n, b, depth):
    dtype = ata.F64 if depth == 64 or depth == -1 else ata.F32
    info, leaves = ata.ata_plan_query(m, n, dtype, b, depth)
    d = 64 if depth == -1 else depth
    c = recursive.count(m, n, b, split_m=False, max_strassen_depth=d)
    assert info["multiplications"] == c.mults
    assert info["syrk_leaves"] == c.syrk_leaves
    assert info["gemm_leaves"] == c.gemm_leaves
    assert info["strassen_nodes"] == c.strassen_nodes
    assert info["ata_nodes"] == c.ata_nodes
    assert len(leaves) == c.syrk_leaves + c.gemm_leaves
    # leaves written straight into C tile the lower triangle exactly once
    # (Strassen products land in the workspace, their roots cover the rest)
    cover = np.zeros((n, n), dtype=np.int32) if n <= 1200 else None
    if cover is not None:
        for L in leaves:
            if L["out_row0"] < 0:
                continue
            r0, c0, R, Cn = L["out_row0"], L["out_col0"], L["rows"], L["cols"]
            blk = cover[r0:r0 + R, c0:c0 + Cn]
            blk += np.tril(np.ones((R, Cn), np.int32)) if L["kind"] == 0 else 1
        for (x0, y0, _, nn, kk, levels, _) in c.strassen_roots:
            if levels > 0:
                cover[x0:x0 + nn, y0:y0 + kk] += 1
        assert np.array_equal(cover, np.tril(np.ones((n, n), np.int32)))


def test_plan_mult_count_pin():
    info, _ = ata.ata_plan_query(1024, 1024, ata.F64, 256, -1)
    assert info["multiplications"] == 503840768
    assert info["strassen_levels"] == 1


def test_plan_query_rejects_bad_arguments():
    with pytest.raises(ata.AtaError):
        ata.ata_plan_query(-1, 5, ata.F64)
    with pytest.raises(ata.AtaError):
        ata.ata_plan_query(5, 5, 9)


def test_gram_argument_errors_need_no_device():
    L = ata.lib()
    # NULL handle, negative sizes, lda < n: rejected synchronously
    assert L.ata_gram(None, None, 4, 4, 4, 1, None, None) == 1
    assert L.ata_set_option(None, 0, 1.0) == 1
    assert L.ata_get_report(None, None) == 1
    assert L.ata_destroy(None) == 0
    assert L.ata_gram_batched(None, 0, None, None, None, None, 1, None, None) == 1
    h = ctypes.c_void_p()
    assert L.ata_create(None) == 1
    r = ctypes.c_double()
    cols = (ctypes.c_int64 * 2)(0, 1)
    assert L.ata_check_columns(None, None, 4, 4, 4, 1, None, cols, 2, ctypes.byref(r), None) == 1


def test_plan_query_rejects_packed_operands_of_4_gib():
    """Split-BF16 and FP8 leaf operands are read with 32-bit buffer offsets:
    a plan whose packed array reaches 4 GiB is refused as not supported,
    while the same shape in FP32 (plain pointers) plans normally."""
    m = 1 << 21                       # 2^21 x 1024: 4 GiB of packed BF16 hi
    with pytest.raises(ata.AtaError) as e:
        ata.ata_plan_query(m, 1024, ata.F32_BF16X3, 2048, 0)
    assert e.value.status == 2
    info, _ = ata.ata_plan_query(m, 1024, ata.F32, 2048, 0)
    assert info["syrk_leaves"] == 1
    info, _ = ata.ata_plan_query(m // 2, 1024, ata.F32_BF16X3, 2048, 0)
    assert info["syrk_leaves"] == 1


def test_plan_splits_k_only_for_long_contractions_with_few_tiles():
    # tall-skinny: few output tiles, K = 262144 -> every leaf is split
    info, leaves = ata.ata_plan_query(262144, 4096, ata.F32, 1024, 1)
    assert all(L["ksplit"] >= 2 for L in leaves if L["contraction"] >= 16384)
    assert all(L["contraction"] // L["ksplit"] >= 8192 - 256 for L in leaves)
    # splitting changes neither the leaves nor the multiplication count
    assert info["multiplications"] == sum(
        L["rows"] * (L["rows"] + 1) // 2 * L["contraction"] if L["kind"] == 0
        else L["rows"] * L["cols"] * L["contraction"] for L in leaves)
    # square 8192: thousands of tiles already -> no split
    _, leaves = ata.ata_plan_query(8192, 8192, ata.F32, 1024, 2)
    assert all(L["ksplit"] == 1 for L in leaves)
    # a launch with very few tiles splits even moderate contractions, in
    # chunks of at least 128 rows (FP32; 256 for the packed split-BF16 operands)
    _, leaves = ata.ata_plan_query(8000, 300, ata.F32, 1024, 0)
    assert leaves[0]["ksplit"] >= 2 and 8000 / leaves[0]["ksplit"] >= 128
    _, leaves = ata.ata_plan_query(8000, 300, ata.F32_BF16X3, 1024, 0)
    assert leaves[0]["ksplit"] >= 2 and 8000 / leaves[0]["ksplit"] >= 256
    # contractions shorter than two chunks are never split
    _, leaves = ata.ata_plan_query(250, 300, ata.F32, 1024, 0)
    assert all(L["ksplit"] == 1 for L in leaves)
    _, leaves = ata.ata_plan_query(400, 300, ata.F32_BF16X3, 1024, 0)
    assert all(L["ksplit"] == 1 for L in leaves)


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes mirrors have the sizes and field offsets the C
    compiler gives the structs of include/ata.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"ata_report_t": ata.Report, "ata_leaf_t": ata.Leaf, "ata_tune_entry_t": ata.TuneEntry}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ata.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_split_bf16_plans_past_the_whole_a_packing_limit():
    """A 50000^2 split-BF16 plan: one hi/lo packing of all of A would pass the
    4 GiB reach of a buffer resource, so the planner packs each leaf operand
    on its own instead of rejecting the shape; the multiplication count is the
    same as for an FP32 plan of that shape."""
    info, leaves = ata.ata_plan_query(50000, 50000, ata.F32_BF16X3, 2048, 1)
    ref, _ = ata.ata_plan_query(50000, 50000, ata.F32, 2048, 1)
    assert info["strassen_levels"] == 1 and len(leaves) > 0
    assert info["multiplications"] == ref["multiplications"]
