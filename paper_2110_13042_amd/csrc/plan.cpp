// Planner: AtA recursion (Alg. 1, rows kept) -> flattened launch phases.
#include "plan.hpp"

#include <algorithm>
#include <functional>
#include <queue>
#include <map>
#include <stdexcept>
#include <tuple>

namespace ata {

int64_t default_leaf_cutoff(int32_t mode, int64_t m, int64_t n, int32_t tile_cfg) {
    (void)m;
    switch (mode) {
        case MODE_F64: return n <= 2048 ? 256 : 512;
        case MODE_F32: return tile_cfg >= 2 ? 2048 : 1024;
        case MODE_BF16X3: return 2048;
        default: return 2048;
    }
}

int32_t default_leaf_tile(int32_t mode, int64_t m, int64_t n) {
    if (mode == MODE_F32) return m >= 2048 && n >= 2048 ? 2 : 0;
    if (mode == MODE_BF16X3) return m >= 4096 && n >= 4096 ? 2 : 0;
    return 0;
}

int32_t default_max_depth(int32_t mode, int64_t m) {
    // Strassen's rounding error adds to the contraction's own, which grows
    // with m: long contractions get no Strassen level in the FP32 family
    // (measured on 262144 x 4096 FP32 with equilibrated columns: one level
    // reaches 2.1e-5 normwise on sampled columns, against 1.2e-5 without)
    const bool long_k = m >= 65536;
    switch (mode) {
        case MODE_F64: return 64;
        case MODE_F32: return long_k ? 0 : 3;
        case MODE_BF16X3: return long_k ? 0 : 2;
        default: return 1;
    }
}

int64_t syrk_tiles(int64_t tm, int64_t tn, int64_t rho) {
    const int64_t L = tn / rho;   // rows 0..L-1 are not clipped by tn
    if (tm <= L) return rho * tm * (tm + 1) / 2;
    return rho * L * (L + 1) / 2 + (tm - L) * tn;
}

int64_t Plan::alloc(int64_t elems) {
    const int64_t off = arena_elems;
    const int64_t align = 256 / elem_bytes();
    arena_elems += (elems + align - 1) / align * align;
    return off;
}

int64_t Plan::launches() const {
    int64_t l = leaves.empty() ? 0 : 1;
    if (!round_tiles.empty()) {
        l = 0;
        for (size_t r = 0; r + 1 < round_tiles.size(); ++r) l += round_tiles[r + 1] > round_tiles[r] ? 1 : 0;
    }
    for (const auto& v : presum) l += v.empty() ? 0 : 1;
    for (const auto& v : combine) l += v.empty() ? 0 : 1;
    if (pack_split > 0) l += 1;
    if ((int64_t)pack.size() > pack_split) l += 1;
    const int32_t q8 = std::max(pack8_split, pack8_norm);
    if (pack8_norm > 0) l += 1;
    if (q8 > pack8_norm) l += 1;
    if ((int64_t)pack8.size() > q8) l += 1;
    if (!fb_leaves.empty()) l += 1;
    if (!reduce.empty()) l += 1;
    if (fallback) l += norm_pass1 ? 3 : 2;  // column norm passes + flags
    for (const auto& v : sums) l += v.empty() ? 0 : 1;
    for (const auto& v : accum) l += v.empty() ? 0 : 1;
    return l;
}

namespace {

int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return std::max(lo, std::min(hi, v)); }

// Sub-block of v starting at (r0, c0) whose real extent is real_r x real_c
// and whose logical (zero-padded) extent is log_r x log_c.
View sub(const View& v, int64_t r0, int64_t real_r, int64_t log_r, int64_t c0,
         int64_t real_c, int64_t log_c) {
    View s = v;
    s.off = v.off + r0 * v.ld + c0;
    s.prows = clamp64(std::min(v.prows, r0 + real_r) - r0, 0, real_r);
    s.pcols = clamp64(std::min(v.pcols, c0 + real_c) - c0, 0, real_c);
    s.rows = log_r;
    s.cols = log_c;
    return s;
}

View arena_view(int64_t off, int64_t rows, int64_t cols) {
    View v{};
    v.base = BASE_ARENA;
    v.off = off;
    v.ld = cols;
    v.rows = v.prows = rows;
    v.cols = v.pcols = cols;
    return v;
}

struct Target {
    int32_t kind;
    int64_t off, ld;      // dense
    int64_t row0, col0;   // packed
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Packed and quantised operands are read through buffer resources with
// 32-bit byte offsets: one array must stay below 4 GiB.
void check_buffer_bytes(int64_t floats) {
    if (floats * 4 > (int64_t)0xFFFFFF00) throw std::length_error("leaf operand array exceeds 4 GiB");
}

struct Builder {
    Plan& p;
    int64_t b;
    int32_t maxd;
    bool fb;
    bool counting = true;   // false while planning a fallback alternative
    // bounded workspace: C21 blocks with Strassen levels are collected here
    // instead of being planned in place
    struct Root {
        View X, Y;
        Target t;
        int32_t pn, pv;
        int level;            // AtA depth of the node
    };
    bool collect = false;
    std::vector<Root> roots;
    int ata_level = 0;
    // combine in the epilogue: the target quadrants of the next leaf added
    // (null: the leaf stores its product)
    struct Epi {
        int32_t round, nq, quad[2], sign[2], first[2];
    };
    const Epi* epi = nullptr;
    int64_t epi_n1 = 0, epi_k1 = 0;

    explicit Builder(Plan& plan) : p(plan), b(plan.b), maxd(plan.max_depth), fb(plan.fallback) {}

    int64_t alloc(int64_t elems) { return p.alloc(elems); }

    View a_cols(int64_t c0, int64_t w) const {
        View v{};
        v.base = BASE_A;
        v.off = c0;
        v.ld = p.lda;
        v.rows = v.prows = p.m;
        v.cols = v.pcols = w;
        return v;
    }

    // One side of a leaf: a view, or the sum / difference of two views.
    struct Operand {
        View a, b{};
        int32_t sign = 0;     // operand = a + sign * b; 0: a alone
        // rows the leaf contracts over: a sum spans the logical rows, as the
        // pre-sum buffer it replaces does (rows past both terms' physical
        // extents read as zero), so K and the split-K chunks are the same
        int64_t prows() const { return sign ? a.rows : a.prows; }
    };

    void add_leaf(int32_t kind, const View& X, const View& Y, const Target& t, int depth,
                  int32_t pred_node, int32_t pred_value, int32_t fb_node) {
        add_leaf(kind, Operand{X}, Operand{Y}, t, depth, pred_node, pred_value, fb_node);
    }

    void add_leaf(int32_t kind, const Operand& OX, const Operand& OY, const Target& t, int depth,
                  int32_t pred_node, int32_t pred_value, int32_t fb_node) {
        const View& X = OX.a;
        const View& Y = OY.a;
        LeafDesc L{};
        L.kind = kind;
        L.out_kind = t.kind;
        L.X = X;
        L.Y = Y;
        L.X2 = OX.b;
        L.Y2 = OY.b;
        L.sx2 = OX.sign;
        L.sy2 = OY.sign;
        L.rows = X.cols;
        L.cols = Y.cols;
        L.K = std::min(OX.prows(), OY.prows());
        const int tmz = tile_m_for(p.mode, p.tile_cfg), tnz = tile_n_for(p.mode, p.tile_cfg);
        L.tiles_m = (int32_t)cdiv(L.rows, tmz);
        L.tiles_n = (int32_t)cdiv(L.cols, tnz);
        L.tiles = kind == LEAF_SYRK ? syrk_tiles(L.tiles_m, L.tiles_n, tmz / tnz)
                                    : (int64_t)L.tiles_m * L.tiles_n;
        L.out_off = t.off;
        L.out_ld = t.ld;
        L.out_row0 = t.row0;
        L.out_col0 = t.col0;
        L.pred_node = pred_node;
        L.pred_value = pred_value;
        L.fb_node = fb_node;
        L.depth = depth;
        if (epi) {
            L.round = epi->round;
            L.nq = epi->nq;
            for (int q = 0; q < 2; ++q) {
                L.quad[q] = epi->quad[q];
                L.qsign[q] = epi->sign[q];
                L.qfirst[q] = epi->first[q];
            }
            L.qn1 = epi_n1;
            L.qk1 = epi_k1;
        }
        if (counting) {
            if (kind == LEAF_SYRK) {
                ++p.stats.syrk_leaves;
                p.stats.mults += X.rows * X.cols * (X.cols + 1) / 2;
            } else {
                ++p.stats.gemm_leaves;
                p.stats.mults += X.rows * X.cols * Y.cols;
            }
        }
        p.leaves.push_back(L);
    }

    // Levels a Strassen call on (mm, n, k) would recurse (ignores predicates).
    int levels(int64_t mm, int64_t n, int64_t k, int depth) const {
        if (std::max(n, k) <= b || std::min(mm, std::min(n, k)) <= 1 || depth >= maxd) return 0;
        return 1 + levels(mm - mm / 2, n - n / 2, k - k / 2, depth + 1);
    }

    void ata(int64_t c0, int64_t w) {
        const int32_t node = (int32_t)p.nodes.size();
        p.nodes.push_back(NodeDesc{c0, w});
        ++p.stats.ata_nodes;
        if (w <= b || p.m <= 1 || w <= 1) {
            Target t{OUT_PACKED, 0, 0, c0, c0};
            View X = a_cols(c0, w);
            add_leaf(LEAF_SYRK, X, X, t, 0, -1, 0, fb ? node : -1);
            return;
        }
        const int64_t n1 = w / 2, n2 = w - n1;
        ++ata_level;
        ata(c0, n1);
        ata(c0 + n1, n2);
        --ata_level;
        const View X = a_cols(c0 + n1, n2), Y = a_cols(c0, n1);
        const Target t{OUT_PACKED, 0, 0, c0 + n1, c0};
        const bool deep = levels(p.m, n2, n1, 0) > 0;
        if (fb && deep) {
            // flagged node: plain product, no Strassen (predicated on the device)
            counting = false;
            add_leaf(LEAF_GEMM, X, Y, t, 0, node, 1, -1);
            counting = true;
            if (collect) roots.push_back(Root{X, Y, t, node, 0, ata_level});
            else strassen(X, Y, t, 0, node, 0);
        } else if (collect && deep) {
            roots.push_back(Root{X, Y, t, -1, 0, ata_level});
        } else {
            strassen(X, Y, t, 0, -1, 0);
        }
    }

    // C_target = X^T Y.  Returns the height of this node (0 = leaf).
    int strassen(const View& X, const View& Y, const Target& t, int depth, int32_t pn, int32_t pv) {
        const int64_t mm = X.rows, n = X.cols, k = Y.cols;
        if (std::max(n, k) <= b || std::min(mm, std::min(n, k)) <= 1 || depth >= maxd) {
            add_leaf(LEAF_GEMM, X, Y, t, depth, pn, pv, -1);
            return 0;
        }
        if (counting) ++p.stats.strassen_nodes;
        const int64_t m1 = mm / 2, m2 = mm - m1, n1 = n / 2, n2 = n - n1, k1 = k / 2, k2 = k - k1;
        // split-BF16: when all seven products are leaves, the sums are only
        // ever leaf operands, so the pre-sum writes them split and packed
        const bool children_leaf = std::max(n2, k2) <= b || std::min(m2, std::min(n2, k2)) <= 1 ||
                                   depth + 1 >= maxd;
        const bool packed = p.mode == MODE_BF16X3 && children_leaf;
        const View X11 = sub(X, 0, m1, m2, 0, n1, n2), X12 = sub(X, 0, m1, m2, n1, n2, n2);
        const View X21 = sub(X, m1, m2, m2, 0, n1, n2), X22 = sub(X, m1, m2, m2, n1, n2, n2);
        const View Y11 = sub(Y, 0, m1, m2, 0, k1, k2), Y12 = sub(Y, 0, m1, m2, k1, k2, k2);
        const View Y21 = sub(Y, m1, m2, m2, 0, k1, k2), Y22 = sub(Y, m1, m2, m2, k1, k2, k2);
        auto Mt = [&](int i, int64_t M) { return Target{OUT_DENSE, M + (i - 1) * n2 * k2, k2, 0, 0}; };
        // combine in the epilogue: the seven products are leaves that add
        // themselves into the quadrants of t in five launch rounds.  Each
        // quadrant gets its contributions in the combine's order (C11 =
        // ((M1 + M4) - M5) + M7, C12 = M3 + M5, C21 = M2 + M4, C22 = ((M1 -
        // M2) + M3) + M6), one writer per element per round.
        static const Epi kEpi[7] = {
            {0, 2, {0, 3}, {1, 1}, {1, 1}},      // M1 -> C11, C22
            {1, 2, {2, 3}, {1, -1}, {1, 0}},     // M2 -> C21, -C22
            {2, 2, {1, 3}, {1, 1}, {1, 0}},      // M3 -> C12, C22
            {2, 2, {0, 2}, {1, 1}, {0, 0}},      // M4 -> C11, C21
            {3, 2, {0, 1}, {-1, 1}, {0, 0}},     // M5 -> -C11, C12
            {3, 1, {3, 0}, {1, 0}, {0, 0}},      // M6 -> C22
            {4, 1, {0, 0}, {1, 0}, {0, 0}},      // M7 -> C11
        };
        const bool in_epilogue = p.fuse_combine && p.variant == 0 && children_leaf;
        auto product_leaf = [&](int i, const Operand& OX, const Operand& OY, int64_t M) {
            if (in_epilogue) {
                epi = &kEpi[i - 1];
                epi_n1 = n1;
                epi_k1 = k1;
            }
            add_leaf(LEAF_GEMM, OX, OY, in_epilogue ? t : Mt(i, M), depth + 1, pn, pv, -1);
            epi = nullptr;
        };
        auto push_combine = [&](int64_t M, int level) {
            if ((int)p.combine.size() < level + 1) p.combine.resize(level + 1);
            CombineDesc c{};
            c.m_off = M; c.n1 = n1; c.n2 = n2; c.k1 = k1; c.k2 = k2;
            c.out_kind = t.kind; c.out_off = t.off; c.out_ld = t.ld; c.out_row0 = t.row0; c.out_col0 = t.col0;
            c.unit = k2 % 4 == 0 ? 4 : 1;
            c.elems = n2 * cdiv(k2, c.unit); c.pred_node = pn; c.pred_value = pv; c.variant = p.variant;
            p.combine[level].push_back(c);
        };
        if (p.fuse && p.variant == 0 && children_leaf &&
            ((p.mode == MODE_F32 && p.tile_cfg != 2) || p.mode == MODE_F64)) {
            // the seven products are leaves: each forms its pre-sums while
            // loading its operands (same IEEE sums as the pre-sum pass)
            const int64_t M = in_epilogue ? 0 : alloc(7 * n2 * k2);
            auto op = [](const View& a, const View& b, int32_t sg) { return Operand{a, b, sg}; };
            const Operand S1 = op(X11, X22, 1), S2 = op(X12, X22, 1), S3 = op(X11, X21, 1);
            const Operand S4 = op(X12, X11, -1), S5 = op(X21, X22, -1);
            const Operand T1 = op(Y11, Y22, 1), T2 = op(Y12, Y22, -1), T3 = op(Y21, Y11, -1);
            const Operand T4 = op(Y11, Y12, 1), T5 = op(Y21, Y22, 1);
            product_leaf(1, S1, T1, M);                       // M1 = S1^T T1
            product_leaf(2, S2, Operand{Y11}, M);             // M2 = S2^T Y11
            product_leaf(3, Operand{X11}, T2, M);             // M3 = X11^T T2
            product_leaf(4, Operand{X22}, T3, M);             // M4 = X22^T T3
            product_leaf(5, S3, Operand{Y22}, M);             // M5 = S3^T Y22
            product_leaf(6, S4, T4, M);                       // M6 = S4^T T4
            product_leaf(7, S5, T5, M);                       // M7 = S5^T T5
            if (!in_epilogue) push_combine(M, 0);
            if (counting) p.stats.max_levels = std::max<int32_t>(p.stats.max_levels, depth + 1);
            return 1;
        }
        const bool wino = p.variant == 1;
        const int nsums = wino ? 4 : 5;
        const int64_t groups = cdiv(m2, 8);
        const int64_t s_each = packed ? groups * n2 * 8 : m2 * n2;
        const int64_t t_each = packed ? groups * k2 * 8 : m2 * k2;
        const int64_t S = alloc(nsums * s_each), T = alloc(nsums * t_each);
        const int64_t M = in_epilogue ? 0 : alloc(7 * n2 * k2);
        if ((int)p.presum.size() <= depth) p.presum.resize(depth + 1);
        PresumDesc ps{};
        ps.V = X; ps.m1 = m1; ps.m2 = m2; ps.n1 = n1; ps.n2 = n2; ps.out_off = S;
        // four columns per work item when every row of the quadrants and of
        // the sums starts 16-byte aligned (A itself is checked on the device),
        // else one: consecutive lanes then still read consecutive elements
        const int64_t es = p.elem_bytes();
        auto unit_of = [&](const View& V, int64_t c1, int64_t c2) {
            return ((V.off * es) | (V.ld * es) | (c1 * es) | (c2 * es)) % 16 == 0 ? 4 : 1;
        };
        ps.unit = unit_of(X, n1, n2);
        ps.elems = packed ? groups * n2 : m2 * cdiv(n2, ps.unit);
        ps.side = 0; ps.pred_node = pn; ps.pred_value = pv; ps.packed_out = packed ? 1 : 0;
        ps.variant = p.variant;
        p.presum[depth].push_back(ps);
        PresumDesc pt = ps;
        pt.V = Y; pt.n1 = k1; pt.n2 = k2; pt.out_off = T; pt.side = 1;
        pt.unit = unit_of(Y, k1, k2);
        pt.elems = packed ? groups * k2 : m2 * cdiv(k2, pt.unit);
        p.presum[depth].push_back(pt);

        auto Sv = [&](int i) {
            View v = arena_view(S + (i - 1) * s_each, m2, n2);
            if (packed) v.base = BASE_PACKED;
            return v;
        };
        auto Tv = [&](int i) {
            View v = arena_view(T + (i - 1) * t_each, m2, k2);
            if (packed) v.base = BASE_PACKED;
            return v;
        };
        int h = 0;
        if (wino) {
            // Winograd's form of C = X^T Y (Xt_ij = X_ji^T), with S1 = X12 + X22,
            // S2 = S1 - X11, S3 = X11 - X12, S4 = X21 - S2, T1 = Y12 - Y11,
            // T2 = Y22 - T1, T3 = Y22 - Y12, T4 = T2 - Y21
            h = std::max(h, strassen(X11, Y11, Mt(1, M), depth + 1, pn, pv));      // M1 = X11^T Y11
            h = std::max(h, strassen(X21, Y21, Mt(2, M), depth + 1, pn, pv));      // M2 = X21^T Y21
            h = std::max(h, strassen(Sv(4), Y22, Mt(3, M), depth + 1, pn, pv));    // M3 = S4^T Y22
            h = std::max(h, strassen(X22, Tv(4), Mt(4, M), depth + 1, pn, pv));    // M4 = X22^T T4
            h = std::max(h, strassen(Sv(1), Tv(1), Mt(5, M), depth + 1, pn, pv));  // M5 = S1^T T1
            h = std::max(h, strassen(Sv(2), Tv(2), Mt(6, M), depth + 1, pn, pv));  // M6 = S2^T T2
            h = std::max(h, strassen(Sv(3), Tv(3), Mt(7, M), depth + 1, pn, pv));  // M7 = S3^T T3
        } else if (in_epilogue) {
            product_leaf(1, Operand{Sv(1)}, Operand{Tv(1)}, M);   // M1 = S1^T T1
            product_leaf(2, Operand{Sv(2)}, Operand{Y11}, M);     // M2 = S2^T Y11
            product_leaf(3, Operand{X11}, Operand{Tv(2)}, M);     // M3 = X11^T T2
            product_leaf(4, Operand{X22}, Operand{Tv(3)}, M);     // M4 = X22^T T3
            product_leaf(5, Operand{Sv(3)}, Operand{Y22}, M);     // M5 = S3^T Y22
            product_leaf(6, Operand{Sv(4)}, Operand{Tv(4)}, M);   // M6 = S4^T T4
            product_leaf(7, Operand{Sv(5)}, Operand{Tv(5)}, M);   // M7 = S5^T T5
            if (counting) p.stats.max_levels = std::max<int32_t>(p.stats.max_levels, depth + 1);
            return 1;
        } else {
            h = std::max(h, strassen(Sv(1), Tv(1), Mt(1, M), depth + 1, pn, pv));  // M1 = S1^T T1
            h = std::max(h, strassen(Sv(2), Y11, Mt(2, M), depth + 1, pn, pv));    // M2 = S2^T Y11
            h = std::max(h, strassen(X11, Tv(2), Mt(3, M), depth + 1, pn, pv));    // M3 = X11^T T2
            h = std::max(h, strassen(X22, Tv(3), Mt(4, M), depth + 1, pn, pv));    // M4 = X22^T T3
            h = std::max(h, strassen(Sv(3), Y22, Mt(5, M), depth + 1, pn, pv));    // M5 = S3^T Y22
            h = std::max(h, strassen(Sv(4), Tv(4), Mt(6, M), depth + 1, pn, pv));  // M6 = S4^T T4
            h = std::max(h, strassen(Sv(5), Tv(5), Mt(7, M), depth + 1, pn, pv));  // M7 = S5^T T5
        }
        const int height = h + 1;
        push_combine(M, height - 1);
        if (counting) p.stats.max_levels = std::max<int32_t>(p.stats.max_levels, depth + 1);
        return height;
    }
};

// Split-BF16: give every leaf operand a packed hi/lo copy.  Views of A whose
// first row is a multiple of 8 share one packing of the whole of A (rows past
// the leaf's contraction length are masked by the kernel chunk-wise, which is
// exact when that length is a multiple of 8 or reaches the end of A); every
// other view is packed on its own, once per distinct view.
void assign_packed(Plan& p) {
    int64_t a_off = -1, a_groups = 0;
    auto packed_a = [&]() {
        if (a_off < 0) {
            a_groups = std::max<int64_t>(1, cdiv(p.m, 8));
            a_off = p.alloc(a_groups * p.n * 8);
            PackDesc d{};
            d.src.base = BASE_A;
            d.src.off = 0;
            d.src.ld = p.lda;
            d.src.rows = d.src.prows = p.m;
            d.src.cols = d.src.pcols = p.n;
            d.dst = a_off;
            d.lo_delta = a_groups * p.n * 4;
            d.groups = a_groups;
            d.cols = p.n;
            d.elems = a_groups * p.n;
            d.pred_node = -1;
            p.pack.push_back(d);
        }
        return a_off;
    };
    std::map<std::tuple<int32_t, int64_t, int64_t, int64_t, int64_t, int64_t>, Packed> memo;
    auto ref = [&](const View& V, int64_t K, int32_t pn, int32_t pv) {
        Packed P{};
        if (V.base == BASE_PACKED) {
            const int64_t groups = std::max<int64_t>(1, cdiv(V.prows, 8));
            P.off = V.off;
            P.lo_delta = groups * V.cols * 4;
            P.gstride = V.cols * 4;
            P.end = V.off + groups * V.cols * 4;
            check_buffer_bytes(P.end - P.off);
            return P;
        }
        const int64_t r0 = V.base == BASE_A ? V.off / p.lda : 0, c0 = V.base == BASE_A ? V.off % p.lda : 0;
        // (a whole-A packing past the 4 GiB reach of a buffer resource gives
        // way to packings of the views themselves)
        const bool a_fits = std::max<int64_t>(1, cdiv(p.m, 8)) * p.n * 16 <= (int64_t)0xFFFFFF00;
        if (V.base == BASE_A && a_fits && !p.own_packings && r0 % 8 == 0 && V.pcols == V.cols &&
            (K % 8 == 0 || r0 + K == p.m)) {
            const int64_t base = packed_a();
            P.off = base + (r0 / 8) * p.n * 4 + c0 * 4;
            P.lo_delta = a_groups * p.n * 4;
            P.gstride = p.n * 4;
            P.end = base + a_groups * p.n * 4;
            check_buffer_bytes(P.end - P.off);
            return P;
        }
        const auto key = std::make_tuple(V.base, V.off, V.ld, V.prows, V.pcols, V.cols);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        const int64_t groups = std::max<int64_t>(1, cdiv(V.prows, 8));
        const int64_t off = p.alloc(groups * V.cols * 8);
        PackDesc d{};
        d.src = V;
        d.dst = off;
        d.lo_delta = groups * V.cols * 4;
        d.groups = groups;
        d.cols = V.cols;
        d.elems = groups * V.cols;
        d.pred_node = pn;
        d.pred_value = pv;
        p.pack.push_back(d);
        P.off = off;
        P.lo_delta = groups * V.cols * 4;
        P.gstride = V.cols * 4;
        P.end = off + groups * V.cols * 4;
        check_buffer_bytes(P.end - P.off);
        memo.emplace(key, P);
        return P;
    };
    for (auto& L : p.leaves) {
        L.PX = ref(L.X, L.K, L.pred_node, L.pred_value);
        L.PY = L.kind == LEAF_SYRK ? L.PX : ref(L.Y, L.K, L.pred_node, L.pred_value);
    }
    int64_t e = 0;
    for (auto& d : p.pack) { d.elem_begin = e; e = item_align(e + d.elems); }
}

// FP8: every distinct leaf operand view is quantised on its own (blocks
// aligned to the view's first row and column), except the full-height column
// slices of A: when each of those is a run of whole 128-column blocks of A
// (its first column a multiple of 128, its width too unless it ends at A's
// last column), A is quantised once and they read its blocks (the same
// blocks, exponents and codes as quantising each slice on its own), so a
// plan whose leaves cover A in several slices reads and quantises A once.
void assign_quant(Plan& p) {
    std::map<std::tuple<int32_t, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t>, Packed8> memo;
    auto ref = [&](const View& V, int32_t pn, int32_t pv) {
        const auto key = std::make_tuple(V.base, V.off, V.ld, V.prows, V.pcols, V.rows, V.cols);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        const int64_t rows_p = std::max<int64_t>(128, cdiv(V.prows, 128) * 128);
        const int64_t cols_p = std::max<int64_t>(128, cdiv(V.cols, 128) * 128);
        Pack8Desc d{};
        d.src = V;
        d.dst = p.alloc(rows_p * cols_p / 4);
        d.scales = p.alloc((rows_p / 128) * (cols_p / 128));
        d.rows_p = rows_p;
        d.cols_p = cols_p;
        d.elems = (rows_p / 128) * (cols_p / 128);
        d.pred_node = pn;
        d.pred_value = pv;
        p.pack8.push_back(d);
        Packed8 Q{};
        Q.off = d.dst;
        Q.scales = d.scales;
        Q.cols_p = cols_p;
        Q.ld = cols_p;
        Q.end = d.dst + rows_p * cols_p / 4;
        check_buffer_bytes(Q.end - Q.off);
        memo.emplace(key, Q);
        return Q;
    };
    auto a_slice = [&](const View& V) {
        return V.base == BASE_A && V.off >= 0 && V.off < p.lda && V.ld == p.lda && V.rows == p.m &&
               V.prows == p.m && V.pcols == V.cols && V.off + V.cols <= p.n;
    };
    bool slices = false, aligned = true;
    for (const auto& L : p.leaves)
        for (const View* V : {&L.X, &L.Y})
            if (a_slice(*V)) {
                slices = true;
                aligned = aligned && V->off % 128 == 0 && (V->cols % 128 == 0 || V->off + V->cols == p.n);
            }
    Packed8 W{};
    const bool shared = slices && aligned;
    if (shared) {
        View A{};
        A.base = BASE_A;
        A.ld = p.lda;
        A.rows = A.prows = p.m;
        A.cols = A.pcols = p.n;
        W = ref(A, -1, 0);
    }
    auto quant = [&](const View& V, int32_t pn, int32_t pv) {
        if (!shared || !a_slice(V)) return ref(V, pn, pv);
        Packed8 Q = W;                       // column c of A is chunk column c
        Q.off = W.off + V.off * 4;           // 16 bytes (4 floats) per chunk column
        Q.scales = W.scales + V.off / 128;
        Q.cols_p = std::max<int64_t>(128, cdiv(V.cols, 128) * 128);
        return Q;
    };
    for (auto& L : p.leaves) {
        L.QX = quant(L.X, L.pred_node, L.pred_value);
        L.QY = L.kind == LEAF_SYRK ? L.QX : quant(L.Y, L.pred_node, L.pred_value);
    }
    int64_t e = 0;
    for (auto& d : p.pack8) { d.elem_begin = e; e += d.elems; }
}

}  // namespace

Plan make_plan(int32_t mode, int64_t m, int64_t n, int64_t lda, const PlanOptions& opt) {
    if (mode < MODE_F64 || mode > MODE_FP8) throw std::invalid_argument("mode");
    if (m < 0 || n < 0 || lda < std::max<int64_t>(1, n)) throw std::invalid_argument("sizes");
    Plan p;
    p.mode = mode;
    p.m = m;
    p.n = n;
    p.lda = lda;
    p.b = opt.leaf_cutoff > 0 ? opt.leaf_cutoff : default_leaf_cutoff(mode, m, n, opt.tile_cfg);
    p.max_depth = opt.max_depth >= 0 ? opt.max_depth : default_max_depth(mode, m);
    p.fallback = mode != MODE_F64 && opt.spread_tau > 0 && n > 0 && m > 0;
    p.tile_cfg = mode == MODE_BF16X3 ? opt.tile_cfg : (mode == MODE_FP8 || mode == MODE_F32) && opt.tile_cfg == 3 ? 3 : mode == MODE_F32 && opt.tile_cfg == 2 ? 2 : 0;
    p.fuse = opt.fuse_presum;
    p.variant = opt.variant;
    p.overlap = opt.overlap;
    p.fuse_combine = opt.fuse_combine;
    if (n == 0) return p;
    Builder bld(p);
    bld.ata(0, n);
    if (mode == MODE_BF16X3 && m > 0) assign_packed(p);
    if (mode == MODE_FP8 && m > 0) assign_quant(p);
    if (p.fallback) build_colnorm_tasks(&p.m, &p.n, &p.lda, 1, p.col1, p.col2, &p.col_partial);
    if (opt.split_target > 0) split_leaves(p, opt.split_target);
    if (opt.slots > 0) balance_tail(p, opt.slots);
    finalize_plan(p);
    return p;
}

std::vector<Plan> make_staged_plan(int32_t mode, int64_t m, int64_t n, int64_t lda, const PlanOptions& opt) {
    if (mode < MODE_F64 || mode > MODE_FP8) throw std::invalid_argument("mode");
    if (m < 0 || n < 0 || lda < std::max<int64_t>(1, n)) throw std::invalid_argument("sizes");
    std::vector<Plan> stages;
    Plan p;
    p.mode = mode;
    p.m = m;
    p.n = n;
    p.lda = lda;
    p.b = opt.leaf_cutoff > 0 ? opt.leaf_cutoff : default_leaf_cutoff(mode, m, n, opt.tile_cfg);
    p.max_depth = opt.max_depth >= 0 ? opt.max_depth : default_max_depth(mode, m);
    p.fallback = mode != MODE_F64 && opt.spread_tau > 0 && n > 0 && m > 0;
    p.tile_cfg = mode == MODE_BF16X3 ? opt.tile_cfg : (mode == MODE_FP8 || mode == MODE_F32) && opt.tile_cfg == 3 ? 3 : mode == MODE_F32 && opt.tile_cfg == 2 ? 2 : 0;
    if (n == 0) {
        stages.push_back(std::move(p));
        return stages;
    }
    Builder bld(p);
    bld.collect = true;
    bld.ata(0, n);
    std::vector<Builder::Root> roots = bld.roots;
    if (mode == MODE_BF16X3 && m > 0) assign_packed(p);
    if (mode == MODE_FP8 && m > 0) assign_quant(p);
    if (p.fallback) build_colnorm_tasks(&p.m, &p.n, &p.lda, 1, p.col1, p.col2, &p.col_partial);
    if (opt.split_target > 0) split_leaves(p, opt.split_target);
    if (opt.slots > 0) balance_tail(p, opt.slots);
    finalize_plan(p);

    // Strassen's seven products of a node C = X^T Y: which sums they take
    // (sx / sy: 0 = a quadrant, 1..5 = S_i / T_i) and where they go
    struct Prod { int sx, qx, sy, qy; int nq; int quad[2]; int sign[2]; };
    // quadrant codes of an operand: 0 = 11, 1 = 12, 2 = 21, 3 = 22
    static const Prod prods[7] = {
        {1, -1, 1, -1, 2, {0, 3}, {1, 1}},      // M1 = S1^T T1 -> C11, C22
        {2, -1, 0, 0, 2, {2, 3}, {1, -1}},      // M2 = S2^T Y11 -> C21, -C22
        {0, 0, 2, -1, 2, {1, 3}, {1, 1}},       // M3 = X11^T T2 -> C12, C22
        {0, 3, 3, -1, 2, {0, 2}, {1, 1}},       // M4 = X22^T T3 -> C11, C21
        {3, -1, 0, 3, 2, {0, 1}, {-1, 1}},      // M5 = S3^T Y22 -> -C11, C12
        {4, -1, 4, -1, 1, {3, 0}, {1, 0}},      // M6 = S4^T T4 -> C22
        {5, -1, 5, -1, 1, {0, 0}, {1, 0}},      // M7 = S5^T T5 -> C11
    };
    // the first product to reach each quadrant overwrites it
    static const int first_of[4] = {0, 2, 1, 0};   // C11: M1, C12: M3, C21: M2, C22: M1
    // S_i = a + sign b over quadrants of X (T_i over Y)
    static const int ssum[5][3] = {{0, 3, 1}, {1, 3, 1}, {0, 2, 1}, {1, 0, -1}, {2, 3, -1}};
    static const int tsum[5][3] = {{0, 3, 1}, {1, 3, -1}, {2, 0, -1}, {0, 1, 1}, {2, 3, 1}};
    struct Node { View X, Y; Target t; };
    int max_level = 0, max_root_levels = 0;
    for (const auto& r : roots) {
        max_level = std::max(max_level, r.level);
        max_root_levels = std::max(max_root_levels, bld.levels(r.X.rows, r.X.cols, r.Y.cols, 0));
    }
    // stages of the roots for D sequential levels; adds the sequential nodes
    // to *nodes and returns the largest stage arena
    auto make_stages = [&](int D, std::vector<Plan>& out, int64_t* nodes, int32_t* levels) {
        int64_t amax = 0;
        for (int lv = 0; lv <= max_level; ++lv) {
            std::vector<const Builder::Root*> grp;
            int dg = D;
            for (const auto& r : roots)
                if (r.level == lv) {
                    grp.push_back(&r);
                    dg = std::min(dg, bld.levels(r.X.rows, r.X.cols, r.Y.cols, 0));
                }
            if (grp.empty() || dg <= 0) continue;
            int64_t nseq = 1;
            for (int j = 0; j < dg; ++j) nseq *= 7;
            for (const auto* r : grp) {
                int64_t pw = 1;
                for (int j = 0; j < dg; ++j) { *nodes += pw; pw *= 7; }
                (void)r;
            }
            *levels = std::max(*levels, dg);
            for (int64_t seq = 0; seq < nseq; ++seq) {
                int dig[16];
                int64_t q = seq;
                for (int j = dg - 1; j >= 0; --j) { dig[j] = (int)(q % 7); q /= 7; }
                auto all_after = [&](int j, int v) {   // digits after level j (0-based) all equal v
                    for (int u = j + 1; u < dg; ++u)
                        if (dig[u] != v) return false;
                    return true;
                };
                Plan s;
                s.mode = mode;
                s.m = m;
                s.n = n;
                s.lda = lda;
                s.b = p.b;
                s.max_depth = p.max_depth;
                s.tile_cfg = p.tile_cfg;
                s.own_packings = true;
                s.sums.resize(dg);
                s.accum.resize(dg);
                Builder sb(s);
                // level buffers of every root first, at the same offsets in every stage
                std::vector<std::vector<int64_t>> soff(grp.size()), toff(grp.size()), moff(grp.size());
                for (size_t g = 0; g < grp.size(); ++g) {
                    int64_t mm = grp[g]->X.rows, nn = grp[g]->X.cols, kk = grp[g]->Y.cols;
                    for (int j = 0; j < dg; ++j) {
                        mm -= mm / 2; nn -= nn / 2; kk -= kk / 2;
                        soff[g].push_back(s.alloc(mm * nn));
                        toff[g].push_back(s.alloc(mm * kk));
                        moff[g].push_back(s.alloc(nn * kk));
                    }
                }
                for (size_t g = 0; g < grp.size(); ++g) {
                    const Builder::Root& r = *grp[g];
                    Node nd{r.X, r.Y, r.t};
                    for (int j = 0; j < dg; ++j) {
                        const View& X = nd.X;
                        const View& Y = nd.Y;
                        const int64_t mm = X.rows, nx = X.cols, k = Y.cols;
                        const int64_t m1 = mm / 2, m2 = mm - m1, n1 = nx / 2, n2 = nx - n1, k1 = k / 2, k2 = k - k1;
                        const View Xq[4] = {sub(X, 0, m1, m2, 0, n1, n2), sub(X, 0, m1, m2, n1, n2, n2),
                                            sub(X, m1, m2, m2, 0, n1, n2), sub(X, m1, m2, m2, n1, n2, n2)};
                        const View Yq[4] = {sub(Y, 0, m1, m2, 0, k1, k2), sub(Y, 0, m1, m2, k1, k2, k2),
                                            sub(Y, m1, m2, m2, 0, k1, k2), sub(Y, m1, m2, m2, k1, k2, k2)};
                        const int i = dig[j];
                        const Prod& pr = prods[i];
                        const bool start = all_after(j, 0);   // this prefix begins: form its sums
                        auto operand = [&](int sidx, int qd, const View* Vq, const int (*tab)[3], int64_t cols,
                                           int64_t off) {
                            if (sidx == 0) return Vq[qd];
                            if (start) {
                                Sum2Desc d{};
                                d.a = Vq[tab[sidx - 1][0]];
                                d.b = Vq[tab[sidx - 1][1]];
                                d.sign = tab[sidx - 1][2];
                                d.rows = m2;
                                d.cols = cols;
                                d.out_off = off;
                                d.elems = m2 * cols;
                                d.pred_node = r.pn;
                                d.pred_value = r.pv;
                                s.sums[j].push_back(d);
                            }
                            return arena_view(off, m2, cols);
                        };
                        const View Xo = operand(pr.sx, pr.qx, Xq, ssum, n2, soff[g][j]);
                        const View Yo = operand(pr.sy, pr.qy, Yq, tsum, k2, toff[g][j]);
                        if (all_after(j, 6)) {                // the product is finished in this stage
                            AccumDesc a{};
                            a.m_off = moff[g][j];
                            a.n1 = n1; a.n2 = n2; a.k1 = k1; a.k2 = k2;
                            a.out_kind = nd.t.kind;
                            a.out_off = nd.t.off; a.out_ld = nd.t.ld; a.out_row0 = nd.t.row0; a.out_col0 = nd.t.col0;
                            a.elems = n2 * k2;
                            a.pred_node = r.pn;
                            a.pred_value = r.pv;
                            a.nq = pr.nq;
                            for (int u = 0; u < pr.nq; ++u) {
                                a.quad[u] = pr.quad[u];
                                a.sign[u] = pr.sign[u];
                                a.first[u] = first_of[pr.quad[u]] == i ? 1 : 0;
                            }
                            s.accum[dg - 1 - j].push_back(a);    // deepest level first
                        }
                        nd = Node{Xo, Yo, Target{OUT_DENSE, moff[g][j], k2, 0, 0}};
                    }
                    sb.strassen(nd.X, nd.Y, nd.t, dg, r.pn, r.pv);
                }
                if (mode == MODE_BF16X3 && m > 0) assign_packed(s);
                if (mode == MODE_FP8 && m > 0) assign_quant(s);
                if (opt.split_target > 0) split_leaves(s, opt.split_target);
                if (opt.slots > 0) balance_tail(s, opt.slots);
                finalize_plan(s);
                for (auto& lvl : s.sums) {
                    int64_t e = 0;
                    for (auto& d : lvl) { d.elem_begin = e; e = item_align(e + d.elems); }
                }
                for (auto& lvl : s.accum) {
                    int64_t e = 0;
                    for (auto& d : lvl) { d.elem_begin = e; e = item_align(e + d.elems); }
                }
                while (!s.sums.empty() && s.sums.back().empty()) s.sums.pop_back();
                amax = std::max(amax, s.arena_elems);
                out.push_back(std::move(s));
            }
        }
        return amax;
    };
    std::vector<Plan> rest;
    if (!roots.empty()) {
        const double target = 1.5 * (double)n * (double)std::max(m, n);
        int D = opt.seq_levels > 0 ? std::min(opt.seq_levels, max_root_levels) : 1;
        for (;;) {
            rest.clear();
            int64_t nodes = 0;
            int32_t lv = 0;
            const int64_t amax = std::max(p.arena_elems, make_stages(D, rest, &nodes, &lv));
            if (opt.seq_levels > 0 || (double)amax <= target || D >= max_root_levels) {
                p.stats.strassen_nodes += nodes;
                p.stats.max_levels = std::max(p.stats.max_levels, lv);
                break;
            }
            ++D;
        }
    }
    for (auto& s : rest) {
        p.stats.gemm_leaves += s.stats.gemm_leaves;
        p.stats.strassen_nodes += s.stats.strassen_nodes;
        p.stats.mults += s.stats.mults;
        p.stats.max_levels = std::max(p.stats.max_levels, s.stats.max_levels);
        stages.push_back(std::move(s));
    }
    if (!roots.empty()) p.stats.max_levels = std::max<int32_t>(p.stats.max_levels, 1);
    stages.insert(stages.begin(), std::move(p));
    return stages;
}

void fuse_pack_into_norms(Plan& p, std::vector<ColDesc>& col1) {
    if (p.mode != MODE_BF16X3) return;
    for (auto& c : col1) {
        if (c.n <= 0 || c.m <= 0) continue;
        for (size_t i = 0; i < p.pack.size(); ++i) {
            const PackDesc& d = p.pack[i];
            if (d.prob != c.prob || d.pred_node >= 0 || d.src.base != BASE_A || d.src.off != 0 ||
                d.src.ld != c.lda || d.src.prows != c.m || d.src.pcols != c.n || d.cols != c.n ||
                d.groups != cdiv(c.m, 8))
                continue;
            c.pack = 1;
            c.pack_dst = d.dst;
            c.pack_lo = d.lo_delta;
            p.pack.erase(p.pack.begin() + (std::ptrdiff_t)i);
            break;
        }
    }
    int64_t e = 0;
    for (auto& d : p.pack) { d.elem_begin = e; e = item_align(e + d.elems); }
    // the leaves that read A's packing no longer wait for a pack launch
    if (p.overlap) finalize_plan(p);
}

void number_pack8(Plan& p);

void fuse_norms_into_quant(Plan& p, std::vector<ColDesc>& col1, std::vector<ColDesc>& col2,
                           int64_t& partial_total) {
    if (p.mode != MODE_FP8 || p.pack8.empty()) return;
    std::vector<ColDesc> keep;
    std::vector<int32_t> fused_probs;
    for (const auto& c : col1) {
        if (c.n <= 0) continue;                          // the placeholder of an empty list
        if (c.m <= 0) {                                  // pass 1 writes its zero norms
            keep.push_back(c);
            continue;
        }
        // unpredicated quantisations of full-height column slices of A that
        // cover its columns exactly once, widest first at each column
        std::vector<size_t> chain;
        int64_t pos = 0;
        while (pos < c.n) {
            size_t best = p.pack8.size();
            for (size_t i = 0; i < p.pack8.size(); ++i) {
                const Pack8Desc& d = p.pack8[i];
                if (d.norm || d.prob != c.prob || d.pred_node >= 0 || d.src.base != BASE_A || d.src.off != pos ||
                    d.src.ld != c.lda || d.src.prows != c.m || d.src.pcols <= 0 || pos + d.src.pcols > c.n)
                    continue;
                if (best == p.pack8.size() || d.src.pcols > p.pack8[best].src.pcols) best = i;
            }
            if (best == p.pack8.size()) break;
            chain.push_back(best);
            pos += p.pack8[best].src.pcols;
        }
        if (pos != c.n) {
            keep.push_back(c);
            continue;
        }
        for (size_t i : chain) p.pack8[i].norm = 1;
        fused_probs.push_back(c.prob);
    }
    if (fused_probs.empty()) return;
    // partial layout: each problem's pass 2 sums nchunks rows of n doubles,
    // from its pass 1 task or from its quantisations' 128-row block rows
    int64_t off = 0;
    for (auto& c2 : col2) {
        if (c2.n <= 0) continue;
        if (std::find(fused_probs.begin(), fused_probs.end(), c2.prob) != fused_probs.end())
            c2.nchunks = cdiv(c2.m, 128);
        c2.part_off = off;
        for (auto& c1 : keep)
            if (c1.prob == c2.prob) c1.part_off = off;
        for (auto& d : p.pack8)
            if (d.norm && d.prob == c2.prob) {
                d.part_off = off + d.src.off;
                d.part_ld = c2.n;
            }
        off += c2.nchunks * c2.n;
    }
    partial_total = off;
    int64_t e = 0;
    for (auto& c : keep) { c.elem_begin = e; e = item_align(e + c.elems); }
    p.norm_pass1 = !keep.empty();
    if (keep.empty()) keep.push_back(ColDesc{});
    col1 = std::move(keep);
    std::stable_partition(p.pack8.begin(), p.pack8.end(), [](const Pack8Desc& d) { return d.norm != 0; });
    p.pack8_norm = 0;
    for (const auto& d : p.pack8) p.pack8_norm += d.norm;
    if (p.overlap) finalize_plan(p);
    else number_pack8(p);
}

void build_colnorm_tasks(const int64_t* m, const int64_t* n, const int64_t* lda, int64_t count,
                         std::vector<ColDesc>& col1, std::vector<ColDesc>& col2,
                         int64_t* partial_total) {
    col1.clear();
    col2.clear();
    int64_t part_off = 0, nu_off = 0, e1 = 0, e2 = 0;
    for (int64_t i = 0; i < count; ++i) {
        // up to about 4096 workgroups of 256 columns x (4 waves x rows / 4)
        // per problem, each wave summing at least 32 rows (four rounds of
        // eight 16-byte loads in flight), so that even a mid-sized matrix
        // has eight waves per SIMD in flight
        const int64_t xblocks = cdiv(std::max<int64_t>(n[i], 1), 256);
        int64_t chunks = std::max<int64_t>(1, std::min(cdiv(4096, xblocks), cdiv(std::max<int64_t>(m[i], 1), 128)));
        // rows per chunk: a multiple of 32, so each wave's quarter starts on
        // an 8-row group (the split-BF16 packing's unit)
        int64_t rows = cdiv(cdiv(std::max<int64_t>(m[i], 1), chunks), 32) * 32;
        chunks = cdiv(std::max<int64_t>(m[i], 1), rows);
        ColDesc d{};
        d.m = m[i];
        d.n = n[i];
        d.lda = lda[i];
        d.rows = rows;
        d.nchunks = chunks;
        d.part_off = part_off;
        d.nu_off = nu_off;
        d.prob = (int32_t)i;
        part_off += chunks * n[i];
        nu_off += n[i];
        if (n[i] == 0) continue;
        ColDesc d1 = d, d2 = d;
        d1.elems = chunks * xblocks * ITEM_BLOCK;
        d1.elem_begin = e1;
        e1 = item_align(e1 + d1.elems);
        d2.elems = n[i];
        d2.elem_begin = e2;
        e2 = item_align(e2 + d2.elems);
        col1.push_back(d1);
        col2.push_back(d2);
    }
    if (col1.empty()) {
        ColDesc z{};
        col1.push_back(z);
        col2.push_back(z);
    }
    *partial_total = part_off;
}

Plan make_gemm_plan(int32_t mode, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                    int64_t ldc, const PlanOptions& opt) {
    if (mode < MODE_F64 || mode > MODE_FP8) throw std::invalid_argument("mode");
    if (m < 0 || n < 0 || k < 0 || lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, k) ||
        ldc < std::max<int64_t>(1, k))
        throw std::invalid_argument("sizes");
    Plan p;
    p.mode = mode;
    p.gemm = true;
    p.m = m;
    p.n = n;
    p.k = k;
    p.lda = lda;
    p.ldb = ldb;
    p.ldc = ldc;
    p.b = opt.leaf_cutoff > 0 ? opt.leaf_cutoff : default_leaf_cutoff(mode, m, std::max(n, k), opt.tile_cfg);
    p.max_depth = opt.max_depth >= 0 ? opt.max_depth : default_max_depth(mode, m);
    p.fallback = false;
    p.tile_cfg = mode == MODE_BF16X3 ? opt.tile_cfg : (mode == MODE_FP8 || mode == MODE_F32) && opt.tile_cfg == 3 ? 3 : mode == MODE_F32 && opt.tile_cfg == 2 ? 2 : 0;
    p.fuse = opt.fuse_presum;
    p.fuse_combine = opt.fuse_combine;
    p.variant = opt.variant;
    if (n == 0 || k == 0) return p;
    Builder bld(p);
    View X{};
    X.base = BASE_A;
    X.ld = lda;
    X.rows = X.prows = m;
    X.cols = X.pcols = n;
    View Y{};
    Y.base = BASE_B;
    Y.ld = ldb;
    Y.rows = Y.prows = m;
    Y.cols = Y.pcols = k;
    bld.strassen(X, Y, Target{OUT_CDENSE, 0, ldc, 0, 0}, 0, -1, 0);
    if (mode == MODE_BF16X3 && m > 0) assign_packed(p);
    if (mode == MODE_FP8 && m > 0) assign_quant(p);
    if (opt.split_target > 0) split_leaves(p, opt.split_target);
    if (opt.slots > 0) balance_tail(p, opt.slots);
    finalize_plan(p);
    return p;
}

namespace {

// Row granule of a K chunk: the FP64 and FP32 engines take any multiple of
// their 16- or 32-row slabs, the packed split-BF16 and FP8 operands 256.
// The FP64 fallback reads its operands unpacked.
int64_t split_granule(const Plan& p) { return p.mode == MODE_F64 || p.mode == MODE_F32 ? 128 : 256; }

// Cuts leaf L into K chunks of a multiple of the granule: about K / s each in
// the mode's launch and, for a leaf under the spread check, about K / s_fb
// each in the FP64 fallback's launch (partial buffers and one reduce task).
// False if neither side ends up with two chunks.
bool split_leaf(Plan& p, LeafDesc& L, int64_t s, int64_t s_fb = 1) {
    bool cut = false;
    if (s >= 2) {
        const int64_t g = split_granule(p);
        const int64_t kchunk = cdiv(cdiv(L.K, s), g) * g;
        s = cdiv(L.K, kchunk);
        if (s >= 2) {
            L.ksplit = (int32_t)s;
            L.kchunk = kchunk;
            L.tiles_split = L.tiles;
            L.tiles *= s;
            L.part_off = p.alloc(s * L.rows * L.cols);
            cut = true;
        }
    }
    if (L.fb_node >= 0 && s_fb >= 2) {
        const int64_t kchunk = cdiv(cdiv(L.K, s_fb), 128) * 128;
        s_fb = cdiv(L.K, kchunk);
        if (s_fb >= 2) {
            L.fb_ksplit = (int32_t)s_fb;
            L.fb_kchunk = kchunk;
            L.part64_off = p.alloc(2 * s_fb * L.rows * L.cols);
            cut = true;
        }
    }
    if (!cut) return false;
    ReduceDesc R{};
    R.kind = L.kind;
    R.out_kind = L.out_kind;
    R.rows = L.rows;
    R.cols = L.cols;
    R.part_off = L.part_off;
    R.part64_off = L.part64_off;
    R.out_off = L.out_off;
    R.out_ld = L.out_ld;
    R.out_row0 = L.out_row0;
    R.out_col0 = L.out_col0;
    R.ksplit = L.ksplit > 1 ? L.ksplit : 1;
    R.ksplit_fb = L.fb_ksplit > 1 ? L.fb_ksplit : 1;
    R.fb_node = L.fb_node;
    R.pred_node = L.pred_node;
    R.pred_value = L.pred_value;
    R.prob = L.prob;
    R.elems = L.rows * L.cols;
    p.reduce.push_back(R);
    return true;
}

}  // namespace

void split_leaves(Plan& p, int64_t target, int64_t min_chunk) {
    if (target <= 0) return;
    int64_t t_mode = 0, t_fb = 0;
    for (const auto& L : p.leaves) {
        if (L.ksplit > 1 || L.fb_ksplit > 1) return;   // already split
        t_mode += L.tiles;
        if (L.fb_node >= 0)
            t_fb += syrk_tiles(cdiv(L.rows, TILE_M), cdiv(L.cols, TILE_N), TILE_M / TILE_N);
    }
    // a launch with fewer tiles than two per CU may cut K into chunks as short
    // as 256 rows (small problems are otherwise latency-bound on their K loops)
    auto chunk_min = [&](int64_t tiles, int64_t g) { return tiles < 512 ? std::min<int64_t>(min_chunk, g) : min_chunk; };
    // each launch is split for its own tile count: the fallback's launch of a
    // leaf under the spread check may be cut while the mode's is not
    for (auto& L : p.leaves) {
        const int64_t most = L.K / chunk_min(t_mode, split_granule(p));
        const int64_t s = t_mode > 0 && t_mode < target && most >= 2 ? std::min(target / t_mode, most) : 1;
        const int64_t most_fb = L.K / chunk_min(t_fb, 128);
        const int64_t s_fb = L.fb_node >= 0 && t_fb > 0 && t_fb < target && most_fb >= 2
                                 ? std::min(target / t_fb, most_fb) : 1;
        if ((s < 2 && s_fb < 2) || L.nq > 0) continue;   // (an epilogue combine needs the whole K)
        split_leaf(p, L, s, s_fb);
    }
}

namespace {

// Contraction rows per tile of a leaf (what the kernels loop over), and the
// rows a tile of it costs in a launch: the plain alternative of a flagged
// node (pred_value 1) usually finds its node unflagged and exits at once.
int64_t tile_rows(const LeafDesc& L) { return L.ksplit > 1 ? L.kchunk : L.K; }
int64_t tile_cost(const LeafDesc& L) {
    return L.pred_node >= 0 && L.pred_value == 1 ? 0 : tile_rows(L);
}

// Makespan of list scheduling: tiles in longest-first launch order, each
// taken by the first free slot.  `split[i]` > 1 cuts leaf i into that many K
// chunks (as split_leaf would).
int64_t simulate_makespan(const Plan& p, const std::vector<int64_t>& split, int64_t slots) {
    struct Run { int64_t rows, cost, tiles; };
    std::vector<Run> runs;
    runs.reserve(p.leaves.size());
    for (size_t i = 0; i < p.leaves.size(); ++i) {
        const LeafDesc& L = p.leaves[i];
        int64_t rows = tile_rows(L), cost = tile_cost(L), tiles = L.tiles;
        if (split[i] > 1) {
            const int64_t g = split_granule(p);
            const int64_t kchunk = cdiv(cdiv(L.K, split[i]), g) * g;
            rows = cost = kchunk;
            tiles = L.tiles * cdiv(L.K, kchunk);
        }
        runs.push_back(Run{rows, cost, tiles});
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.rows > b.rows; });
    std::priority_queue<int64_t, std::vector<int64_t>, std::greater<int64_t>> free_at;
    for (int64_t i = 0; i < slots; ++i) free_at.push(0);
    int64_t end = 0;
    for (const Run& r : runs) {
        for (int64_t t = 0; t < r.tiles; ++t) {
            const int64_t f = free_at.top() + r.cost;
            free_at.pop();
            free_at.push(f);
            end = std::max(end, f);
        }
    }
    return end;
}

}  // namespace

void balance_tail(Plan& p, int64_t slots, int32_t max_split) {
    if (slots <= 0 || p.leaves.empty()) return;
    int64_t total_tiles = 0;
    for (const auto& L : p.leaves) {
        if (L.ksplit > 1) return;                  // split_leaves has cut this launch
        if (L.nq > 0) return;                      // launch rounds: no single last round
        total_tiles += L.tiles;
    }
    if (total_tiles > 64 * slots) return;         // the tail is a small part of the launch
    const size_t nl = p.leaves.size();
    std::vector<int64_t> none(nl, 1);
    const int64_t base = simulate_makespan(p, none, slots);
    // candidates: smallest work first (fewest partials), later leaves first on ties
    std::vector<size_t> cand;
    for (size_t i = 0; i < nl; ++i) {
        const LeafDesc& L = p.leaves[i];
        if (L.fb_node >= 0 || tile_cost(L) == 0 || L.K < 2 * split_granule(p)) continue;
        cand.push_back(i);
    }
    std::stable_sort(cand.begin(), cand.end(), [&](size_t a, size_t b) {
        const int64_t wa = p.leaves[a].tiles * p.leaves[a].K, wb = p.leaves[b].tiles * p.leaves[b].K;
        return wa != wb ? wa < wb : a > b;
    });
    // Partial sums cost HBM time: each chunk tile writes its partial tile and
    // the reduce reads it back.  In the makespan's unit (contraction rows of
    // one tile on one slot) at the mode's peak MFMA rate per CU and 5 TB/s:
    // rows = bytes * 2 / 5000 B/ns / (ns per tile row).
    const double flop_ns_per_cu = p.mode == MODE_F64 ? 307.0 : p.mode == MODE_F32 ? 614.0
                                : p.mode == MODE_BF16X3 ? 9766.0 / 3.0 : 19531.0;
    const double tile_row_ns = 2.0 * tile_m_for(p.mode, p.tile_cfg) * tile_n_for(p.mode, p.tile_cfg) / flop_ns_per_cu;
    const double row_per_byte = 2.0 / 5000.0 / tile_row_ns;
    const int64_t part_cap = int64_t(1) << 28;    // bytes of partials at most
    auto partial_bytes = [&](const LeafDesc& L, int64_t s) {
        const int64_t g = split_granule(p);
        const int64_t kchunk = cdiv(cdiv(L.K, s), g) * g;
        return cdiv(L.K, kchunk) * L.rows * L.cols * p.elem_bytes();
    };
    double best = (double)base;
    int64_t best_s = 0;
    size_t best_n = 0;
    for (const int32_t s : {2, 3, 4, 6, 8, 12, 16, 24, 32}) {
        if (s > max_split) break;
        std::vector<int64_t> split(nl, 1);
        int64_t sel = 0, last_bucket = -1, bytes = 0;
        for (size_t j = 0; j < cand.size(); ++j) {
            const LeafDesc& L = p.leaves[cand[j]];
            if (L.K / split_granule(p) < s) continue;
            bytes += partial_bytes(L, s);
            if (bytes > part_cap) break;
            split[cand[j]] = s;
            sel += L.tiles;
            if (sel > 2 * slots) break;            // more than a tail
            const int64_t bucket = sel * s * 16 / slots;    // simulate once per 1/16 round of chunk tiles
            if (bucket == last_bucket && j + 1 < cand.size()) continue;
            last_bucket = bucket;
            const double t = (double)simulate_makespan(p, split, slots) + (double)bytes * row_per_byte;
            if (t < best) {
                best = t;
                best_s = s;
                best_n = j + 1;
            }
        }
    }
    if (best_s == 0 || best > 0.96 * (double)base) return;
    int32_t cut = 0;
    int64_t bytes = 0;
    for (size_t j = 0; j < best_n; ++j) {
        LeafDesc& L = p.leaves[cand[j]];
        if (L.K / split_granule(p) < best_s) continue;
        bytes += partial_bytes(L, best_s);
        if (bytes > part_cap) break;
        if (split_leaf(p, L, best_s)) ++cut;
    }
    p.tail_leaves = cut;
    p.tail_chunks = (int32_t)best_s;
}

// Work items of the quantisations, numbered from 0 in each of their launches:
// [0, pack8_norm) with the column norms, [pack8_norm, q) before the pre-sums
// and [q, end) after them, q = max(pack8_split, pack8_norm).
void number_pack8(Plan& p) {
    const int32_t q = std::max(p.pack8_split, p.pack8_norm);
    int64_t e = 0;
    for (size_t i = 0; i < p.pack8.size(); ++i) {
        if ((int32_t)i == p.pack8_norm || (int32_t)i == q) e = 0;
        p.pack8[i].elem_begin = e;
        e += p.pack8[i].elems;
    }
}

void finalize_plan(Plan& p) {
    // LPT: longest per-tile contraction first (a split leaf's tiles cover one
    // K chunk; stable, so ties keep tree order)
    auto tile_k = [](const LeafDesc& L) { return L.ksplit > 1 ? L.kchunk : L.K; };
    // overlap: leaves that read only A (no pre-sum operand) first, each group
    // longest first; the packings and quantisations of views of A run before
    // the pre-sums
    const bool rounds = std::any_of(p.leaves.begin(), p.leaves.end(), [](const LeafDesc& L) { return L.nq > 0; });
    const bool ov = p.overlap && !p.presum.empty() && !rounds;
    auto indep = [&](const LeafDesc& L) {
        return L.X.base == BASE_A && L.Y.base == BASE_A && (L.sx2 == 0 || L.X2.base == BASE_A) &&
               (L.sy2 == 0 || L.Y2.base == BASE_A);
    };
    std::stable_sort(p.leaves.begin(), p.leaves.end(), [&](const LeafDesc& a, const LeafDesc& c) {
        if (ov && indep(a) != indep(c)) return indep(a);
        return tile_k(a) > tile_k(c);
    });
    constexpr int kRounds = 5;
    if (rounds) {
        // the epilogue combines fix their products' rounds; every other leaf
        // (longest first) joins the round with the least work so far
        double load[kRounds] = {0, 0, 0, 0, 0};
        for (const auto& L : p.leaves)
            if (L.nq > 0) load[L.round] += (double)L.tiles * (double)tile_cost(L);
        for (auto& L : p.leaves) {
            if (L.nq > 0) continue;
            const int r = (int)(std::min_element(load, load + kRounds) - load);
            L.round = r;
            load[r] += (double)L.tiles * (double)tile_cost(L);
        }
        std::stable_sort(p.leaves.begin(), p.leaves.end(),
                         [](const LeafDesc& a, const LeafDesc& c) { return a.round < c.round; });
    } else {
        for (auto& L : p.leaves) L.round = 0;
    }
    int64_t t = 0;
    p.indep_tiles = 0;
    for (auto& L : p.leaves) {
        L.tile_begin = t;
        t += L.tiles;
        if (ov && indep(L)) p.indep_tiles = t;
    }
    p.total_tiles = t;
    p.round_tiles.clear();
    if (rounds) {
        p.round_tiles.assign(kRounds + 1, t);
        for (auto it = p.leaves.rbegin(); it != p.leaves.rend(); ++it) p.round_tiles[it->round] = it->tile_begin;
        for (int r = kRounds - 1; r >= 0; --r) p.round_tiles[r] = std::min(p.round_tiles[r], p.round_tiles[r + 1]);
    }
    if (p.indep_tiles >= p.total_tiles) p.indep_tiles = 0;   // nothing to overlap with
    t = 0;
    p.fb_leaves.clear();
    for (const auto& L : p.leaves) {
        if (L.fb_node >= 0) {
            // the FP64 fallback kernel works on TILE_M x TILE_N tiles
            LeafDesc F = L;
            F.tiles_m = (int32_t)cdiv(F.rows, TILE_M);
            F.tiles_n = (int32_t)cdiv(F.cols, TILE_N);
            F.tiles = syrk_tiles(F.tiles_m, F.tiles_n, TILE_M / TILE_N);
            F.ksplit = L.fb_ksplit > 1 ? L.fb_ksplit : 1;
            F.kchunk = L.fb_kchunk;
            if (F.ksplit > 1) {
                F.tiles_split = F.tiles;
                F.tiles *= F.ksplit;
            }
            F.tile_begin = t;
            t += F.tiles;
            p.fb_leaves.push_back(F);
        }
    }
    p.fb_tiles = t;
    for (auto& lvl : p.presum) {
        int64_t e = 0;
        for (auto& d : lvl) { d.elem_begin = e; e = item_align(e + d.elems); }
    }
    for (auto& lvl : p.combine) {
        int64_t e = 0;
        for (auto& d : lvl) { d.elem_begin = e; e = item_align(e + d.elems); }
    }
    p.pack_split = p.pack8_split = 0;
    if (ov) {
        auto pa = std::stable_partition(p.pack.begin(), p.pack.end(),
                                        [](const PackDesc& d) { return d.src.base == BASE_A; });
        p.pack_split = (int32_t)(pa - p.pack.begin());
        auto qa = std::stable_partition(p.pack8.begin(), p.pack8.end(),
                                        [](const Pack8Desc& d) { return d.src.base == BASE_A; });
        p.pack8_split = (int32_t)(qa - p.pack8.begin());
    }
    int64_t e = 0;
    for (size_t i = 0; i < p.pack.size(); ++i) {
        if ((int32_t)i == p.pack_split) e = 0;
        p.pack[i].elem_begin = e;
        e = item_align(e + p.pack[i].elems);
    }
    number_pack8(p);
    e = 0;
    for (auto& d : p.reduce) { d.elem_begin = e; e = item_align(e + d.elems); }
}

namespace {

void shift_view(View& v, int64_t ab) {
    if (v.base == BASE_ARENA || v.base == BASE_PACKED) v.off += ab;
}

}  // namespace

Plan merge_plans(std::vector<Plan>& parts, int64_t split_target, int64_t slots) {
    Plan out;
    if (parts.empty()) return out;
    out.mode = parts[0].mode;
    out.nprob = (int32_t)parts.size();
    out.tile_cfg = parts[0].tile_cfg;
    out.fuse = parts[0].fuse;
    out.variant = parts[0].variant;
    out.max_depth = 0;
    int64_t node_base = 0;
    for (size_t q = 0; q < parts.size(); ++q) {
        Plan& p = parts[q];
        const int32_t prob = (int32_t)q;
        const int64_t ab = out.arena_elems;
        const int32_t nb = (int32_t)node_base;
        auto pn = [&](int32_t x) { return x >= 0 ? x + nb : x; };
        out.fallback = out.fallback || p.fallback;
        out.b = std::max(out.b, p.b);
        out.max_depth = std::max(out.max_depth, p.max_depth);
        for (auto L : p.leaves) {
            shift_view(L.X, ab);
            shift_view(L.Y, ab);
            shift_view(L.X2, ab);
            shift_view(L.Y2, ab);
            if (L.out_kind == OUT_DENSE) L.out_off += ab;
            L.PX.off += ab; L.PX.end += ab; L.PY.off += ab; L.PY.end += ab;
            L.QX.off += ab; L.QX.scales += ab; L.QX.end += ab;
            L.QY.off += ab; L.QY.scales += ab; L.QY.end += ab;
            L.pred_node = pn(L.pred_node);
            L.fb_node = pn(L.fb_node);
            L.prob = prob;
            out.leaves.push_back(L);
        }
        if (out.presum.size() < p.presum.size()) out.presum.resize(p.presum.size());
        for (size_t l = 0; l < p.presum.size(); ++l)
            for (auto d : p.presum[l]) {
                shift_view(d.V, ab);
                d.out_off += ab;
                d.pred_node = pn(d.pred_node);
                d.prob = prob;
                out.presum[l].push_back(d);
            }
        if (out.combine.size() < p.combine.size()) out.combine.resize(p.combine.size());
        for (size_t l = 0; l < p.combine.size(); ++l)
            for (auto d : p.combine[l]) {
                d.m_off += ab;
                if (d.out_kind == OUT_DENSE) d.out_off += ab;
                d.pred_node = pn(d.pred_node);
                d.prob = prob;
                out.combine[l].push_back(d);
            }
        for (auto d : p.pack) {
            shift_view(d.src, ab);
            d.dst += ab;
            d.pred_node = pn(d.pred_node);
            d.prob = prob;
            out.pack.push_back(d);
        }
        for (auto d : p.pack8) {
            shift_view(d.src, ab);
            d.dst += ab;
            d.scales += ab;
            d.pred_node = pn(d.pred_node);
            d.prob = prob;
            out.pack8.push_back(d);
        }
        out.arena_elems += p.arena_elems;
        node_base += (int64_t)p.nodes.size();
        out.stats.ata_nodes += p.stats.ata_nodes;
        out.stats.syrk_leaves += p.stats.syrk_leaves;
        out.stats.gemm_leaves += p.stats.gemm_leaves;
        out.stats.strassen_nodes += p.stats.strassen_nodes;
        out.stats.mults += p.stats.mults;
        out.stats.max_levels = std::max(out.stats.max_levels, p.stats.max_levels);
    }
    // nodes: columns of each problem are offset by the problem's first norm
    // index, so one flags launch covers the batch
    int64_t nu_base = 0;
    for (auto& p : parts) {
        for (auto nd : p.nodes) {
            nd.c0 += nu_base;
            out.nodes.push_back(nd);
        }
        nu_base += p.n;
    }
    split_leaves(out, split_target);
    if (slots > 0) balance_tail(out, slots);
    finalize_plan(out);
    return out;
}


}  // namespace ata
