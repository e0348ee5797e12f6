"""Host-side checks of the planner's scheduling decisions (CPU only): the
planner source is compiled with the host compiler into a small driver that
prints the plans' structure.  Covers the tail balancer, the FP64 fallback's
own K split, the K-chunk granule, the per-operand split-BF16 packing past the
4 GiB buffer reach, the pre-sum work-item width, Winograd's workspace, and
the bounded-workspace (staged) plans against the resident ones, the plans
that combine their last Strassen level in the leaf epilogues, and the FP8
quantisation that also sums the column squares."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_13042_amd", "csrc")

DRIVER = r"""
#include "plan.hpp"
#include <algorithm>
#include <cstdio>
#include <map>
#include <tuple>
#include <stdexcept>
#include <vector>
using namespace ata;

static void show(const char* tag, int32_t mode, int64_t m, int64_t n, int64_t b, int32_t d, int32_t tile,
                 double tau, int64_t slots, int32_t variant = 0) {
    PlanOptions o;
    o.leaf_cutoff = b; o.max_depth = d; o.tile_cfg = tile; o.spread_tau = tau;
    o.split_target = 2048; o.slots = slots; o.variant = variant;
    try {
        Plan p = make_plan(mode, m, n, n, o);
        int64_t mode_split = 0, fb_split = 0, max_ks = 0, max_fbks = 0, min_chunk = 1 << 30;
        for (const auto& L : p.leaves) {
            if (L.ksplit > 1) { ++mode_split; max_ks = std::max<int64_t>(max_ks, L.ksplit);
                                min_chunk = std::min<int64_t>(min_chunk, L.kchunk); }
            if (L.fb_ksplit > 1) { ++fb_split; max_fbks = std::max<int64_t>(max_fbks, L.fb_ksplit); }
        }
        int64_t unit1 = 0, unit4 = 0, presums = 0;
        for (const auto& lv : p.presum)
            for (const auto& t : lv) { ++presums; (t.unit == 1 ? unit1 : unit4) += 1; }
        printf("%s tiles=%lld fb_tiles=%lld tail=%d chunks=%d mode_split=%lld max_ks=%lld min_chunk=%lld "
               "fb_split=%lld max_fbks=%lld packs=%zu presums=%lld unit1=%lld unit4=%lld arena=%lld levels=%d\n",
               tag, (long long)p.total_tiles, (long long)p.fb_tiles, p.tail_leaves, p.tail_chunks,
               (long long)mode_split, (long long)max_ks, (long long)(mode_split ? min_chunk : 0),
               (long long)fb_split, (long long)max_fbks, p.pack.size(), (long long)presums,
               (long long)unit1, (long long)unit4, (long long)p.arena_elems, p.stats.max_levels);
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

// Bounded workspace: the staged plan against the resident one.
static void show_staged(const char* tag, int32_t mode, int64_t m, int64_t n, int64_t b, int32_t d,
                        double tau) {
    PlanOptions o;
    o.leaf_cutoff = b; o.max_depth = d; o.spread_tau = tau; o.split_target = 2048; o.slots = 0;
    try {
        Plan r = make_plan(mode, m, n, n, o);
        o.bounded = true;
        std::vector<Plan> st = make_staged_plan(mode, m, n, n, o);
        int64_t maxa = 0, sums = 0, acc = 0, leaves = 0;
        for (const auto& q : st) {
            maxa = std::max<int64_t>(maxa, q.arena_elems);
            for (const auto& v : q.sums) sums += (int64_t)v.size();
            for (const auto& v : q.accum) acc += (int64_t)v.size();
            leaves += (int64_t)q.leaves.size();
        }
        int64_t rleaves = (int64_t)r.leaves.size();
        printf("%s stages=%zu arena=%lld resident_arena=%lld mults=%lld resident_mults=%lld levels=%d "
               "resident_levels=%d nodes=%lld resident_nodes=%lld leaves=%lld resident_leaves=%lld sums=%lld "
               "accum=%lld\n", tag, st.size(), (long long)maxa, (long long)r.arena_elems,
               (long long)st[0].stats.mults, (long long)r.stats.mults, st[0].stats.max_levels, r.stats.max_levels,
               (long long)st[0].stats.strassen_nodes, (long long)r.stats.strassen_nodes, (long long)leaves,
               (long long)rleaves, (long long)sums, (long long)acc);
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

// Combines in the leaf epilogues against the materialised plan: same
// multiplications; per fused node, every quadrant's writers in increasing
// launch rounds with the combine's order of signs, the first one overwriting.
static void show_epi(const char* tag, int32_t mode, int64_t m, int64_t n, int64_t b, int32_t d, double tau,
                     bool gemm = false, int64_t k = 0) {
    PlanOptions o;
    o.leaf_cutoff = b; o.max_depth = d; o.spread_tau = tau; o.split_target = 2048; o.slots = 256;
    try {
        Plan r = gemm ? make_gemm_plan(mode, m, n, k, n, k, k, o) : make_plan(mode, m, n, n, o);
        o.fuse_combine = true;
        Plan f = gemm ? make_gemm_plan(mode, m, n, k, n, k, k, o) : make_plan(mode, m, n, n, o);
        int64_t rc = 0, fc = 0, fused = 0, split_fused = 0, bad_round = 0;
        for (const auto& v : r.combine) rc += (int64_t)v.size();
        for (const auto& v : f.combine) fc += (int64_t)v.size();
        struct W { int round, sign, first; };
        std::map<std::tuple<int32_t, int64_t, int64_t, int64_t, int32_t, int32_t, int>, std::vector<W>> q;
        for (const auto& L : f.leaves) {
            const int rr = L.round;
            if (!f.round_tiles.empty() &&
                (L.tile_begin < f.round_tiles.at(rr) || L.tile_begin + L.tiles > f.round_tiles.at(rr + 1)))
                ++bad_round;
            if (L.nq == 0) continue;
            ++fused;
            if (L.ksplit > 1) ++split_fused;
            for (int i = 0; i < L.nq; ++i)
                q[std::make_tuple(L.out_kind, L.out_off, L.out_row0, L.out_col0, L.pred_node, L.pred_value, L.quad[i])]
                    .push_back(W{L.round, L.qsign[i], L.qfirst[i]});
        }
        static const int want_n[4] = {4, 2, 2, 4};
        static const int want_sign[4][4] = {{1, 1, -1, 1}, {1, 1, 0, 0}, {1, 1, 0, 0}, {1, -1, 1, 1}};
        int64_t bad_quad = 0;
        for (auto& kv : q) {
            auto& w = kv.second;
            const int quad = std::get<6>(kv.first);
            std::stable_sort(w.begin(), w.end(), [](const W& a, const W& c) { return a.round < c.round; });
            bool ok = (int)w.size() == want_n[quad];
            for (size_t i = 0; ok && i < w.size(); ++i) {
                ok = w[i].sign == want_sign[quad][i] && w[i].first == (i == 0 ? 1 : 0) &&
                     (i == 0 || w[i].round > w[i - 1].round);
            }
            if (!ok) ++bad_quad;
        }
        printf("%s mults=%lld resident_mults=%lld levels=%d resident_levels=%d arena=%lld resident_arena=%lld "
               "combines=%lld resident_combines=%lld fused=%lld quads=%zu bad_quad=%lld split_fused=%lld "
               "bad_round=%lld rounds=%zu launches=%lld resident_launches=%lld\n", tag, (long long)f.stats.mults,
               (long long)r.stats.mults, f.stats.max_levels, r.stats.max_levels, (long long)f.arena_elems,
               (long long)r.arena_elems, (long long)fc, (long long)rc, (long long)fused, q.size(),
               (long long)bad_quad, (long long)split_fused, (long long)bad_round, f.round_tiles.size(),
               (long long)f.launches(), (long long)r.launches());
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

// FP8 with column norms: quantisations of column slices of A take over norm
// pass 1.  Prints the fused tasks (whether they tile the columns once, full
// height and unpredicated, with their partial offsets), the rebuilt partial
// layout, whether every quantisation launch numbers its work items from 0
// contiguously, and the launch counts before and after.
static void show_q8(const char* tag, int64_t m, int64_t n, int64_t b, int32_t d, bool overlap) {
    PlanOptions o;
    o.leaf_cutoff = b; o.max_depth = d; o.spread_tau = 4096.0; o.split_target = 2048; o.slots = 0;
    o.overlap = overlap;
    try {
        Plan p = make_plan(MODE_FP8, m, n, n, o);
        const int64_t before = p.launches(), partial_before = p.col_partial;
        const size_t tasks = p.pack8.size();
        fuse_norms_into_quant(p, p.col1, p.col2, p.col_partial);
        const int32_t pn = p.pack8_norm, q = std::max(p.pack8_split, pn);
        int numbering_ok = 1;
        int64_t e = 0;
        for (size_t i = 0; i < p.pack8.size(); ++i) {
            if ((int32_t)i == pn || (int32_t)i == q) e = 0;
            if (p.pack8[i].elem_begin != e) numbering_ok = 0;
            e += p.pack8[i].elems;
        }
        int fused_flags = 0, front = 1, tiles_once = 1, offsets_ok = 1;
        std::vector<std::pair<int64_t, int64_t>> cols;
        for (size_t i = 0; i < p.pack8.size(); ++i) {
            const Pack8Desc& t = p.pack8[i];
            fused_flags += t.norm;
            if (t.norm && (int32_t)i >= pn) front = 0;
            if (!t.norm) continue;
            if (t.src.base != BASE_A || t.src.prows != m || t.pred_node >= 0) tiles_once = 0;
            if (t.part_off != p.col2.at(0).part_off + t.src.off || t.part_ld != n) offsets_ok = 0;
            cols.push_back({t.src.off, t.src.pcols});
        }
        std::sort(cols.begin(), cols.end());
        int64_t pos = 0;
        for (auto& cw : cols) {
            if (cw.first != pos) tiles_once = 0;
            pos = cw.first + cw.second;
        }
        if (pos != n) tiles_once = 0;
        printf("%s pn=%d fused_flags=%d front=%d tiles_once=%d offsets_ok=%d nchunks=%lld partial=%lld "
               "partial_before=%lld pass1=%d col1=%zu col1_items=%lld numbering_ok=%d tasks=%zu tasks_before=%zu "
               "split=%d launches=%lld launches_before=%lld\n", tag, pn, fused_flags, front, tiles_once, offsets_ok,
               (long long)p.col2.at(0).nchunks, (long long)p.col_partial, (long long)partial_before,
               p.norm_pass1 ? 1 : 0, p.col1.size(), (long long)(p.col1.back().elem_begin + p.col1.back().elems),
               numbering_ok, p.pack8.size(), tasks, p.pack8_split, (long long)p.launches(), (long long)before);
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

// The same for a batch: one member with no rows (its pass 1 task stays and
// writes zero norms), one whose quantisations take over, one SYRK leaf each.
static void show_q8_batch(const char* tag) {
    PlanOptions o;
    o.leaf_cutoff = 512; o.max_depth = 0; o.spread_tau = 4096.0; o.split_target = 0; o.slots = 0;
    try {
        const int64_t m[3] = {0, 700, 300}, n[3] = {300, 400, 200}, lda[3] = {300, 400, 256};
        std::vector<Plan> parts;
        for (int i = 0; i < 3; ++i) parts.push_back(make_plan(MODE_FP8, m[i], n[i], lda[i], o));
        Plan p = merge_plans(parts);
        std::vector<ColDesc> col1, col2;
        int64_t part = 0;
        build_colnorm_tasks(m, n, lda, 3, col1, col2, &part);
        const int64_t before = part;
        fuse_norms_into_quant(p, col1, col2, part);
        // the partial regions of pass 2 tile [0, part) in problem order
        int64_t off = 0, regions_ok = 1, chunks[3] = {0, 0, 0};
        for (const auto& c2 : col2) {
            if (c2.part_off != off) regions_ok = 0;
            chunks[c2.prob] = c2.nchunks;
            off += c2.nchunks * c2.n;
        }
        if (off != part) regions_ok = 0;
        int64_t kept_prob = -1, kept_items = 0, fused_ok = 1;
        for (const auto& c1 : col1) {
            if (c1.elems > 0) { kept_prob = c1.prob; kept_items = c1.elems; }
            if (c1.part_off != col2.at(0).part_off) fused_ok = 0;    // the m = 0 member's region
        }
        int64_t fused_probs = 0;
        for (size_t i = 0; i < p.pack8.size(); ++i) {
            const Pack8Desc& t = p.pack8[i];
            if (!t.norm) continue;
            fused_probs |= 1 << t.prob;
            const ColDesc* c2 = nullptr;
            for (const auto& c : col2) if (c.prob == t.prob) c2 = &c;
            if (!c2 || t.part_off != c2->part_off + t.src.off || t.part_ld != c2->n || (int32_t)i >= p.pack8_norm)
                fused_ok = 0;
        }
        printf("%s col1=%zu kept_prob=%lld kept_items=%lld fused_probs=%lld fused_ok=%d regions_ok=%lld "
               "chunks0=%lld chunks1=%lld chunks2=%lld pass1=%d part=%lld before=%lld\n", tag, col1.size(),
               (long long)kept_prob, (long long)kept_items, (long long)fused_probs, (int)fused_ok,
               (long long)regions_ok, (long long)chunks[0], (long long)chunks[1], (long long)chunks[2],
               p.norm_pass1 ? 1 : 0, (long long)part, (long long)before);
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

// FP8 leaf operands that are column slices of A: quantised once as the whole
// of A when every slice is a run of whole 128-column blocks.  Prints the
// quantisation count and whether every leaf operand that is such a slice
// reads the whole's blocks at its own first column.
static void show_q8_shared(const char* tag, int64_t m, int64_t n, int64_t b) {
    PlanOptions o;
    o.leaf_cutoff = b; o.max_depth = 0; o.spread_tau = 4096.0; o.split_target = 2048; o.slots = 256;
    try {
        Plan p = make_plan(MODE_FP8, m, n, n, o);
        int whole = -1;
        for (size_t i = 0; i < p.pack8.size(); ++i) {
            const View& v = p.pack8[i].src;
            if (v.base == BASE_A && v.off == 0 && v.prows == m && v.pcols == n) whole = (int)i;
        }
        int64_t slice_ops = 0, slices_ok = 1, own_ok = 1;
        for (const auto& L : p.leaves)
            for (int side = 0; side < 2; ++side) {
                const View& v = side ? L.Y : L.X;
                const Packed8& q = side ? L.QY : L.QX;
                const bool slice = v.base == BASE_A && v.prows == m && v.off < n;
                if (!slice) continue;
                ++slice_ops;
                if (whole >= 0) {
                    const Pack8Desc& w = p.pack8[whole];
                    const int64_t wcols = w.cols_p;
                    if (q.ld != wcols || q.off != w.dst + v.off * 4 || q.scales != w.scales + v.off / 128 ||
                        q.cols_p != std::max<int64_t>(128, (v.cols + 127) / 128 * 128) ||
                        q.end != w.dst + w.rows_p * w.cols_p / 4)
                        slices_ok = 0;
                } else if (q.ld != q.cols_p) {
                    own_ok = 0;
                }
            }
        printf("%s tasks=%zu whole=%d slice_ops=%lld slices_ok=%lld own_ok=%lld leaves=%zu\n", tag, p.pack8.size(),
               whole >= 0 ? 1 : 0, (long long)slice_ops, (long long)slices_ok, (long long)own_ok, p.leaves.size());
    } catch (const std::exception& e) {
        printf("%s error=%s\n", tag, e.what());
    }
}

int main() {
    show_q8_shared("q8s_aligned", 4096, 16384, 2048);
    show_q8_shared("q8s_aligned_2560", 600, 2560, 1024);
    show_q8_shared("q8s_unaligned_2944", 600, 2944, 1024);
    show_q8_shared("q8s_unaligned", 3000, 3000, 512);
    show_q8_batch("q8_batch");
    show_q8("q8_leaf", 16384, 16384, 16384, 0, false);
    show_q8("q8_odd", 1999, 1501, 256, 1, false);
    show_q8("q8_overlap", 1536, 1100, 256, 1, true);
    show_epi("epi_f32_2lv", MODE_F32, 16384, 16384, 2048, 2, 4096.0);
    show_epi("epi_f64_odd", MODE_F64, 3001, 2999, 256, 3, 0.0);
    show_epi("epi_bf16_fb", MODE_BF16X3, 4095, 4097, 512, 2, 20.0);
    show_epi("epi_gemm", MODE_F32, 3000, 2500, 512, 2, 0.0, true, 2100);
    show_epi("epi_none", MODE_F32, 2048, 2048, 4096, 2, 0.0);
    show_staged("staged_f64_30k", MODE_F64, 30000, 30000, 0, -1, 0.0);
    show_staged("staged_f64_odd", MODE_F64, 3001, 2999, 256, 3, 0.0);
    show_staged("staged_f32_fb", MODE_F32, 4096, 4096, 512, 2, 4096.0);
    show_staged("staged_bf16", MODE_BF16X3, 4096, 4096, 512, 2, 4096.0);
    show("bf16_tail", MODE_BF16X3, 8192, 8192, 256, 0, 2, 4096.0, 256);
    show("bf16_nobal", MODE_BF16X3, 8192, 8192, 256, 0, 2, 4096.0, 0);
    show("f32_balanced", MODE_F32, 8192, 8192, 2048, 1, 2, 4096.0, 256);
    show("f64_small", MODE_F64, 1024, 1024, 256, 1, 0, 0.0, 512);
    show("bf16_big", MODE_BF16X3, 50000, 50000, 2048, 1, 2, 4096.0, 256);
    show("bf16_mid", MODE_BF16X3, 40000, 40000, 2048, 1, 2, 4096.0, 256);
    show("f64_odd", MODE_F64, 30000, 30000, 512, 2, 0, 0.0, 0);
    show("f32_pow2", MODE_F32, 16384, 16384, 2048, 2, 2, 0.0, 0);
    show("strassen", MODE_F32, 2048, 2048, 512, 1, 0, 0.0, 0, 0);
    show("winograd", MODE_F32, 2048, 2048, 512, 1, 0, 0.0, 0, 1);
    return 0;
}
"""


@pytest.fixture(scope="module")
def plans(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("plan")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, str(src), os.path.join(CSRC, "plan.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.strip().splitlines():
        tag, *kv = line.split()
        res[tag] = {k: (v if k == "error" else int(v)) for k, v in (x.split("=", 1) for x in kv)}
    return res


def test_tail_balancer_fills_the_last_round(plans):
    """8192^2 on 256^2 tiles: 528 equal tiles on 256 slots.  The balancer cuts
    16 one-tile leaves into 16 K chunks (768 tiles); without slots, nothing."""
    p, q = plans["bf16_tail"], plans["bf16_nobal"]
    assert q["tiles"] == 528 and q["tail"] == 0 and q["mode_split"] == 0
    assert p["tail"] == 16 and p["chunks"] == 16 and p["tiles"] == 528 - 16 + 16 * 16


def test_fallback_split_leaves_the_mode_launch_whole(plans):
    """The 32 diagonal leaves under the spread check get K chunks in the FP64
    fallback launch only; the mode launch keeps them whole."""
    p = plans["bf16_nobal"]
    assert p["fb_split"] == 32 and p["max_fbks"] >= 2
    assert p["mode_split"] == 0


def test_balanced_fp32_plan_is_left_alone(plans):
    p = plans["f32_balanced"]
    assert p["tail"] == 0 and p["levels"] == 1


def test_fp64_k_chunks_down_to_128_rows(plans):
    """A small FP64 launch cuts its 1024-row contractions into 128-row chunks."""
    p = plans["f64_small"]
    assert p["max_ks"] == 8 and p["min_chunk"] == 128


def test_split_bf16_packs_each_operand_past_the_buffer_reach(plans):
    """50000^2: one packing of A would pass 4 GiB, so each leaf operand gets its
    own; 40000^2 still shares one whole-A packing for its aligned views."""
    big, mid = plans["bf16_big"], plans["bf16_mid"]
    assert "error" not in big and big["packs"] > 1
    assert "error" not in mid and mid["packs"] == 1


def test_presum_work_item_width_follows_alignment(plans):
    """Rows whose starts are not 16-byte aligned (odd splits of 30000) take one
    column per work item; power-of-two shapes keep four."""
    odd, pow2 = plans["f64_odd"], plans["f32_pow2"]
    assert odd["unit1"] > 0
    assert pow2["unit1"] == 0 and pow2["unit4"] == pow2["presums"] > 0


def test_winograd_needs_less_workspace(plans):
    """Four pre-sum buffers per operand instead of five."""
    assert plans["winograd"]["arena"] < plans["strassen"]["arena"]
    assert plans["winograd"]["levels"] == plans["strassen"]["levels"] == 1


def test_staged_plan_performs_the_resident_plans_products(plans):
    """The bounded-workspace plan runs exactly the resident plan's
    multiplications, Strassen nodes and levels, as (for every root) seven
    single-sum stages; its workspace is the largest stage's."""
    for tag in ("staged_f64_30k", "staged_f64_odd", "staged_f32_fb", "staged_bf16"):
        p = plans[tag]
        assert "error" not in p, (tag, p)
        assert p["mults"] == p["resident_mults"], tag
        assert p["nodes"] == p["resident_nodes"] and p["levels"] == p["resident_levels"] >= 2, tag
        assert p["stages"] > 7 and p["accum"] % 7 == 0, tag
        assert p["arena"] < p["resident_arena"], tag


def test_staged_workspace_within_sec33_bound(plans):
    """FP64 30000^2 at the default leaf cutoff and depth: every level resident
    needs about 28 n^2 elements (224 GB); the staged plan's largest stage stays
    within Sec. 3.3's 3/2 n^2."""
    p = plans["staged_f64_30k"]
    n = 30000
    assert p["resident_arena"] > 20 * n * n
    assert p["arena"] <= 1.5 * n * n


def test_epilogue_combine_plans(plans):
    """Combines in the leaf epilogues: the same multiplications and levels as
    the materialised plan, one combine fewer per fused node (seven product
    buffers less workspace), no fused leaf cut into K chunks, every leaf inside
    its launch round, and every quadrant of every fused node written in the
    combine's order (C11: +M1 +M4 -M5 +M7, C12: +M3 +M5, C21: +M2 +M4, C22:
    +M1 -M2 +M3 +M6) in strictly increasing rounds, the first write
    overwriting.  Flagged-node alternatives and general products included."""
    for tag in ("epi_f32_2lv", "epi_f64_odd", "epi_bf16_fb", "epi_gemm"):
        p = plans[tag]
        assert "error" not in p, (tag, p)
        assert p["mults"] == p["resident_mults"] and p["levels"] == p["resident_levels"] >= 1, tag
        assert p["fused"] > 0 and p["fused"] % 7 == 0, tag
        nodes = p["fused"] // 7
        assert p["combines"] == p["resident_combines"] - nodes, tag
        assert p["quads"] == 4 * nodes and p["bad_quad"] == 0, tag
        assert p["split_fused"] == 0 and p["bad_round"] == 0 and p["rounds"] == 6, tag
        assert p["arena"] < p["resident_arena"], tag
    # no Strassen level: nothing to fuse, one leaf launch
    p = plans["epi_none"]
    assert p["fused"] == 0 and p["rounds"] == 0 and p["launches"] == p["resident_launches"]


def test_fp8_quantisation_takes_over_norm_pass1(plans):
    """FP8 with the spread check: the quantisations of full-height column
    slices of A that tile its columns once (the whole of A for a single leaf,
    the diagonal leaves' slices under the recursion), unpredicated and moved
    to the front, also write the column-norm partials, one row of n doubles
    per 128-row block row, and norm pass 1 has nothing left; every
    quantisation launch numbers its work items from 0.  The norm launch of
    the quantisations replaces pass 1, so the launch count does not grow."""
    dims = {"q8_leaf": (16384, 16384), "q8_odd": (1999, 1501), "q8_overlap": (1536, 1100)}
    for tag, (m, n) in dims.items():
        p = plans[tag]
        assert "error" not in p, (tag, p)
        assert p["pn"] >= 1 and p["fused_flags"] == p["pn"] and p["front"] == 1, tag
        assert p["tiles_once"] == 1 and p["offsets_ok"] == 1, tag
        assert p["nchunks"] == -(-m // 128) and p["partial"] == p["nchunks"] * n, tag
        assert p["pass1"] == 0 and p["col1"] == 1 and p["col1_items"] == 0, tag
        assert p["numbering_ok"] == 1 and p["tasks"] == p["tasks_before"], tag
    # a single SYRK leaf: its quantisation takes the norms, pass 1 goes
    assert plans["q8_leaf"]["tasks"] == 1 and plans["q8_leaf"]["pn"] == 1
    assert plans["q8_leaf"]["launches"] == plans["q8_leaf"]["launches_before"] - 1
    # the recursion: eight diagonal leaves; the pre-sum quantisations keep
    # their own launch
    assert plans["q8_odd"]["pn"] == 8 and plans["q8_odd"]["tasks"] > 8
    assert plans["q8_odd"]["launches"] == plans["q8_odd"]["launches_before"]
    # overlap: the other views of A still go before the pre-sums
    assert plans["q8_overlap"]["split"] > plans["q8_overlap"]["pn"] == 8


def test_fp8_batch_norms_partial_layout(plans):
    """A batch: the member without rows keeps its pass 1 task (zero norms,
    its own partial region), the members whose quantisations tile their
    columns drop out of pass 1 and sum ceil(m / 128) block rows in pass 2,
    and the regions of all members lie end to end."""
    p = plans["q8_batch"]
    assert "error" not in p, p
    assert p["col1"] == 1 and p["kept_prob"] == 0 and p["kept_items"] > 0 and p["pass1"] == 1
    assert p["fused_probs"] == 0b110 and p["fused_ok"] == 1 and p["regions_ok"] == 1
    assert p["chunks1"] == -(-700 // 128) and p["chunks2"] == -(-300 // 128)
    assert p["part"] == p["chunks0"] * 300 + p["chunks1"] * 400 + p["chunks2"] * 200


def test_fp8_slices_of_a_share_one_quantisation(plans):
    """FP8 leaves whose operands are column slices of A, each a run of whole
    128-column blocks (or ending at A's last column), read one quantisation
    of the whole of A at their own first column (data, block scales, the
    whole's group stride); unaligned slices keep one quantisation each."""
    p = plans["q8s_aligned"]
    assert "error" not in p, p
    assert p["tasks"] == 1 and p["whole"] == 1 and p["slices_ok"] == 1 and p["leaves"] > 8
    # 2560 = 20 x 128 halves into 1280 and 640 column slices, all aligned
    p = plans["q8s_aligned_2560"]
    assert "error" not in p, p
    assert p["tasks"] == 1 and p["whole"] == 1 and p["slices_ok"] == 1 and p["leaves"] > 4
    # 2944 = 23 x 128 halves into 1472 = 11.5 x 128: unaligned, as is 3000
    for tag in ("q8s_unaligned", "q8s_unaligned_2944"):
        p = plans[tag]
        assert "error" not in p, (tag, p)
        assert p["whole"] == 0 and p["tasks"] > 1 and p["own_ok"] == 1, tag
