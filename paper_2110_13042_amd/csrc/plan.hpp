// Plan of one Gram product: the AtA recursion tree flattened into launch
// phases, plus the plain-old-data task descriptors the kernels read.
//
// The recursion is Alg. 1 (Sec. 3.1) in its rows-kept form: an AtA node on
// the column range [c0, c0 + w) is a SYRK leaf when w <= b; otherwise it
// splits w into n1 = floor(w/2), n2 = ceil(w/2) (Eq. "submatA"), recurses on
// both column halves for the diagonal blocks C11 and C22 and hands the
// off-diagonal block C21 = A[:, c0+n1:]^T A[:, c0:c0+n1] (Eq. "Cij") to a
// Strassen node.  A Strassen node computing C = X^T Y splits m, n and k
// floor/ceil, forms five sums of X blocks and five of Y blocks at the ceil
// dimensions (operands one row or column short act as if padded with zeros,
// Sec. 3.1's simulated padding), multiplies seven pairs and combines the
// products into the four quadrants (Strassen's scheme, Sec. 3.2).
//
// The GPU runs every level's pre-sums in one launch (top-down), every leaf
// product of the whole tree in one grouped launch, then every level's
// combines in one launch (bottom-up).  All temporaries sit in one arena
// (Sec. 3.3's preallocated workspace).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ata {

enum Mode : int32_t { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16X3 = 2, MODE_FP8 = 3 };

// Base buffers a view can point into.
// BASE_PACKED: a split-BF16 operand that a pre-sum wrote directly in the
// packed hi/lo layout (see Packed) at arena offset `off`, `rows` x `cols`.
// BASE_B: the second input of a general product C = A^T B.
enum Base : int32_t { BASE_A = 0, BASE_ARENA = 1, BASE_PACKED = 2, BASE_B = 3 };

// Element (r, c) of the rows x cols logical operand is
// base[off + r * ld + c] when r < prows and c < pcols, and 0 otherwise.
struct View {
    int32_t base;
    int32_t pad_;
    int64_t off, ld;
    int64_t rows, cols;       // logical
    int64_t prows, pcols;     // physical extent (<= logical)
};

// A leaf operand repacked for the BF16 MFMAs: hi and lo bf16 arrays of
// `groups` row-groups x `cols` columns of 16-byte chunks; chunk (g, c) holds
// rows 8g..8g+7 of column c (zero beyond the source's physical extent), so a
// chunk is exactly the eight consecutive k values one MFMA lane consumes.
// Offsets and strides are in floats (4 bytes) of the arena.
struct Packed {
    int64_t off;        // chunk (0, 0) of this operand in the hi array
    int64_t lo_delta;   // hi array -> lo array
    int64_t gstride;    // one row-group (= total columns of the array * 4)
    int64_t end;        // end of the hi array (bounds every load)
};

// A leaf operand quantised for the FP8 MFMA: e4m3 bytes in 16-byte chunks of
// 16 consecutive rows of one column, chunk (g, c) at byte (g * cols_p + c) * 16;
// rows and columns padded with zeros to multiples of 128.  Block (bi, bj) of
// 128 x 128 elements has the scale 2^e, e = scales[bi * (cols_p / 128) + bj]
// (int32).  Offsets in floats of the arena.
struct Packed8 {
    int64_t off;        // data array (at the view's first column)
    int64_t scales;     // int32 exponents (at the view's first block column)
    int64_t cols_p;     // padded columns of the view
    int64_t end;        // end of the data array (bounds every load)
    int64_t ld;         // padded columns of the quantised array: the stride of a
                        // 16-row group and, / 128, of a row of block scales
                        // (above cols_p for a column slice of a wider array)
};

enum LeafKind : int32_t { LEAF_SYRK = 0, LEAF_GEMM = 1 };
// OUT_PACKED: packed lower C at (out_row0, out_col0); OUT_DENSE: arena
// buffer at out_off with row stride out_ld; OUT_CDENSE: the caller's dense
// C (row stride out_ld) at (out_row0, out_col0).
enum OutKind : int32_t { OUT_PACKED = 0, OUT_DENSE = 1, OUT_CDENSE = 2 };

// One leaf product out = X^T Y (SYRK: X == Y, lower triangle only).
struct LeafDesc {
    int32_t kind;             // LeafKind
    int32_t out_kind;         // OutKind
    int32_t tiles_m, tiles_n; // output tile grid (SYRK: tiles_m == tiles_n)
    int64_t tile_begin;       // first global tile index of this task
    int64_t tiles;            // tiles of this task
    int64_t K;                // contraction length (rows)
    View X, Y;
    // Fused Strassen pre-sums (FP32 and FP64 leaves of a node whose seven
    // products are all leaves): operand = X + sx2 * X2 (sx2 = +1 or -1, each
    // term zero outside its own physical extent), formed as the operand is
    // loaded; sx2 = 0: X alone.  Likewise Y.
    View X2, Y2;
    int32_t sx2, sy2;
    int64_t rows, cols;       // logical output (rows = X.cols, cols = Y.cols)
    int64_t out_off, out_ld;  // OUT_DENSE: arena element offset and row stride
    int64_t out_row0, out_col0;  // OUT_PACKED: position in C
    int32_t pred_node;        // run only when flags[pred_node] == pred_value (-1: always)
    int32_t pred_value;
    int32_t fb_node;          // SYRK leaves: FP64 path when flags[fb_node] != 0 (-1: never)
    int32_t depth;            // Strassen level of the leaf (0 = directly in C)
    Packed PX, PY;            // split-BF16 mode: packed operands
    Packed8 QX, QY;           // FP8 mode: quantised operands
    int32_t prob;             // problem of a batch (selects its A and C)
    int32_t ksplit;           // K chunks (1: none); tile q covers chunk q / tiles_split
    int64_t kchunk;           // rows per K chunk (a multiple of 256; 128 for FP64 and FP32)
    int64_t tiles_split;      // tiles of one K chunk
    int64_t part_off;         // split: arena offset of [ksplit][rows][cols] partials (mode type)
    int64_t part64_off;       // split SYRK leaves under the spread check: FP64 partials
                              // of the fallback (arena float offset, 8-byte aligned)
    // The FP64 fallback's own K split of a leaf under the spread check (its
    // launch is small, so it may cut where the mode's launch need not):
    // fb_ksplit chunks of fb_kchunk rows (<= 1: none), partials at part64_off.
    int32_t fb_ksplit;
    int32_t round;            // launch round of a plan with combines in the epilogue (0 otherwise)
    int64_t fb_kchunk;
    // Strassen combine in the epilogue (PlanOptions::fuse_combine): product
    // M_i of a node whose seven products are all leaves goes straight into
    // its one or two quadrants of the node's target (out_*).  Quadrant q
    // (0: C11, 1: C12, 2: C21, 3: C22) starts at row (q >= 2 ? qn1 : 0) and
    // column (q odd ? qk1 : 0) of the target and takes the product's
    // elements that fall inside it (C11 and C12 have qn1 rows, C11 and C21
    // qk1 columns); the first contribution to a quadrant overwrites it, the
    // later ones add qsign times the product to what the earlier launch
    // rounds left there.
    int32_t nq;               // 0: plain store; 1 or 2 quadrants
    int32_t quad[2], qsign[2], qfirst[2];
    int32_t qpad_;
    int64_t qn1, qk1;
};

// Sum of the K-chunk partials of a split leaf (one work item per output
// element), in chunk order, in FP64, rounded once into the leaf's target.
// A leaf under the spread check takes the fallback's partials when its node
// is flagged, the mode's otherwise; an unsplit side wrote the target itself.
struct ReduceDesc {
    int32_t kind, out_kind;
    int64_t rows, cols;
    int64_t part_off, part64_off;
    int64_t out_off, out_ld, out_row0, out_col0;
    int32_t ksplit, fb_node;      // the mode's chunks (<= 1: its leaf wrote the target)
    int32_t pred_node, pred_value;
    int32_t prob, ksplit_fb;      // the fallback's chunks (<= 1: it wrote the target)
    int64_t elem_begin, elems;
};

// Quantise one FP32 operand view to block-scaled e4m3 (one work item per
// 128 x 128 block).
struct Pack8Desc {
    View src;
    int64_t dst, scales;
    int64_t rows_p, cols_p;
    int64_t elem_begin, elems;
    int32_t pred_node, pred_value;
    int32_t prob;
    int32_t norm;             // also writes column-norm partials (one per 128-row block row)
    int64_t part_off;         // those partials: partial[part_off + block_row * part_ld + column of the view]
    int64_t part_ld;
};

// Split one FP32 operand view into the packed hi/lo layout (one work item per
// 16-byte chunk).
struct PackDesc {
    View src;
    int64_t dst;              // arena float offset of the hi array
    int64_t lo_delta;
    int64_t groups, cols;
    int64_t elem_begin, elems;
    int32_t pred_node, pred_value;
    int32_t prob, pad_;
};

// Pre-sums of one operand: Strassen's five (X side: S1..S5, Y side: T1..T5)
// or Winograd's four chained ones (variant 1).
struct PresumDesc {
    View V;                   // the parent operand (m x n logical)
    int64_t m1, m2, n1, n2;
    int64_t out_off;          // arena: five m2 x n2 buffers, row stride n2
    int64_t elem_begin;       // first global work item (groups of 4 columns)
    int64_t elems;
    int32_t side;             // 0 = X (S sums), 1 = Y (T sums)
    int32_t pred_node, pred_value;
    int32_t packed_out;       // 1: write the sums split and packed (work item = one
                              // 16-byte chunk; sum i at out_off + i * ceil(m2/8) * n2 * 8)
    int32_t prob;
    int32_t variant;          // 0: Strassen, five sums; 1: Winograd, four sums
    int32_t unit;             // columns per work item: 4 (16-byte vectors) or 1 (any alignment)
    int32_t pad_;
};

// Strassen (or Winograd) combine: seven n2 x k2 products into the four
// quadrants.
struct CombineDesc {
    int64_t m_off;            // arena: seven n2 x k2 buffers, row stride k2
    int64_t n1, n2, k1, k2;
    int32_t out_kind;
    int32_t pred_node;
    int64_t out_off, out_ld;      // OUT_DENSE target (parent's product buffer)
    int64_t out_row0, out_col0;   // OUT_PACKED target (C21 block of C)
    int64_t elem_begin, elems;
    int32_t pred_value;
    int32_t prob;
    int32_t variant;              // 0: Strassen, 1: Winograd
    int32_t unit;                 // columns per work item: 4 or 1 (k2 not a multiple of 4)
};

// Bounded workspace (PlanOptions::bounded): one sum of a Strassen root's
// product operand, formed on its own into a dense buffer (row stride cols):
// out = a + sign * b over rows x cols, each view read as zero outside its
// physical extent (the same IEEE sum the pre-sum pass stores).
struct Sum2Desc {
    View a, b;
    int64_t rows, cols;
    int64_t out_off;               // arena element offset
    int64_t elem_begin, elems;     // one work item per element
    int32_t sign;                  // +1 or -1
    int32_t pred_node, pred_value;
    int32_t prob;
};

// Bounded workspace: product i (n2 x k2, row stride k2) of a Strassen root
// added into its one or two quadrants of the root's target.  The products
// run in order and the first contribution to a quadrant overwrites it, so
// every quadrant receives the combine's own left-to-right sum (C11 =
// ((M1 + M4) - M5) + M7, C12 = M3 + M5, C21 = M2 + M4, C22 = ((M1 - M2) + M3)
// + M6).
struct AccumDesc {
    int64_t m_off;
    int64_t n1, n2, k1, k2;
    int64_t out_off, out_ld, out_row0, out_col0;
    int64_t elem_begin, elems;     // one work item per product element
    int32_t out_kind;
    int32_t pred_node, pred_value;
    int32_t nq;                    // targets: 1 or 2
    int32_t quad[2];               // 0: C11, 1: C12, 2: C21, 3: C22
    int32_t sign[2];               // +1 or -1
    int32_t first[2];              // 1: the quadrant's first contribution (overwrite)
    int32_t prob, pad_;
};

// Column-norm task of one problem.  Pass 1: a workgroup sums the squares of
// 256 columns over one chunk of `rows` rows (elems = chunks x column blocks x
// ITEM_BLOCK items); pass 2: one item per column sums the chunks in order.
struct ColDesc {
    int64_t m, n, lda, rows;      // rows per chunk (a multiple of 32)
    int64_t nchunks;
    int64_t part_off, nu_off;     // doubles in the partial and norm arrays
    int64_t elem_begin, elems;
    int32_t prob;
    int32_t pack;                 // pass 1 also writes A's split-BF16 packing (one read of A)
    int64_t pack_dst, pack_lo;    // that packing: hi array and hi -> lo distance (floats)
};

// AtA node for the spread flags: columns [c0, c0 + w).
struct NodeDesc {
    int64_t c0, w;
};

struct PlanOptions {
    int64_t leaf_cutoff = 0;       // 0: default for the mode
    int32_t max_depth = -1;        // -1: default for the mode
    int32_t tile_cfg = 0;          // leaf tile: 0 = 128 x 128; split-BF16 1 = 256 x 128, 2, 3 = 256 x 256; FP32 2, 3 and FP8 3 = 256 x 256
    double spread_tau = 4096.0;    // <= 0: no fallback
    int64_t split_target = 2048;   // split K when a launch has fewer tiles (0: never)
    bool fuse_presum = false;      // FP32/FP64: last-level pre-sums formed in the leaf loads
    int32_t variant = 0;           // Strassen node: 0 = Strassen's form, 1 = Winograd's
    int64_t slots = 0;             // > 0: balance the leaf launch's last round over this
                                   // many resident workgroups (balance_tail)
    bool overlap = false;          // order the leaves that read only A first (indep_tiles)
    bool fuse_combine = false;     // last-level combines in the leaf epilogues (Strassen form)
    bool bounded = false;          // make_staged_plan: Strassen roots product by product
    int32_t seq_levels = 0;        // make_staged_plan: top levels run product by product
                                   // (0: the fewest that keep the workspace within
                                   // 3/2 n max(m, n) elements)
};

struct PlanStats {
    int64_t ata_nodes = 0, syrk_leaves = 0, gemm_leaves = 0, strassen_nodes = 0;
    int64_t mults = 0;
    int32_t max_levels = 0;
};

struct Plan {
    int32_t mode = MODE_F32;
    int32_t nprob = 1;
    int64_t m = 0, n = 0, lda = 0;
    bool gemm = false;                              // C = A^T B (n x k, dense) instead of AtA
    int64_t k = 0, ldb = 0, ldc = 0;                // the general product's B and C
    int64_t b = 0;
    int32_t max_depth = 0;
    int32_t tile_cfg = 0;
    bool fallback = false;
    bool fuse = false;                              // last-level pre-sums fused into the leaves
    int32_t variant = 0;                            // 0: Strassen nodes, 1: Winograd nodes
    int32_t tail_leaves = 0, tail_chunks = 0;       // leaves balance_tail cut, K chunks each
    std::vector<std::vector<PresumDesc>> presum;    // [level-1] top-down
    std::vector<PackDesc> pack;                     // split-BF16 operand packing
    std::vector<Pack8Desc> pack8;                   // FP8 operand quantisation
    std::vector<LeafDesc> leaves;                   // LPT order (longest first)
    std::vector<LeafDesc> fb_leaves;                // SYRK leaves under the spread check
    std::vector<ReduceDesc> reduce;                 // split leaves: partial sums
    std::vector<std::vector<CombineDesc>> combine;  // [height-1] bottom-up
    std::vector<std::vector<Sum2Desc>> sums;        // bounded stages: single pre-sums, top-down (first)
    std::vector<std::vector<AccumDesc>> accum;      // bounded stages: products into quadrants, bottom-up (last)
    bool own_packings = false;                      // split-BF16: pack each leaf operand on its own
    // Combines in the leaf epilogues: a node whose seven products are all
    // leaves gets no product buffers and no combine; its products run in five
    // dependent launch rounds, {M1}, {M2}, {M3, M4}, {M5, M6}, {M7}, so that
    // every quadrant element has one writer per round and receives the
    // combine's own left-to-right sum.  Round r is the tiles [round_tiles[r],
    // round_tiles[r + 1]) of the leaf order (empty: one leaf launch).
    bool fuse_combine = false;
    std::vector<int64_t> round_tiles;
    // Overlap of the pre-sums with the leaf products: with `overlap` set, the
    // leaves whose operands are ready before any pre-sum (views of A, read
    // directly or, for split-BF16, through the column-norm pass's packing)
    // come first in the leaf order, and indep_tiles counts their tiles; the
    // executor runs them on a second stream while the pre-sums run.
    bool overlap = false;
    int64_t indep_tiles = 0;
    // With overlap, the packings (split-BF16) and quantisations (FP8) of views
    // of A come first in their lists and run before the pre-sums, in their
    // own launch: pack_split / pack8_split descriptors, whose work items are
    // numbered apart from the rest's (0: one launch after the pre-sums).
    int32_t pack_split = 0, pack8_split = 0;
    // FP8 with column norms: the first pack8_norm quantisations (column
    // slices of A that cover each such problem's columns once) also write
    // its column-norm partials and run in their own launch before norm
    // pass 2; norm_pass1 is false when no problem is left for pass 1.
    int32_t pack8_norm = 0;
    bool norm_pass1 = true;
    std::vector<NodeDesc> nodes;                    // AtA nodes (flags)
    std::vector<ColDesc> col1, col2;                // column-norm passes (when fallback)
    int64_t col_partial = 0;                        // doubles of the pass-1 partial sums
    int64_t arena_elems = 0;                        // in the mode's sum/product type
    int64_t total_tiles = 0;
    int64_t fb_tiles = 0;
    PlanStats stats;
    int64_t elem_bytes() const { return mode == MODE_F64 ? 8 : 4; }
    int64_t alloc(int64_t elems);                   // 256-byte aligned arena carve
    int64_t launches() const;
};

int64_t default_leaf_cutoff(int32_t mode, int64_t m, int64_t n, int32_t tile_cfg = 0);
// Leaf tile of a shape with no explicit choice and no autotune entry: the
// 256 x 256 eight-wave engines once the output has enough tiles of them.
int32_t default_leaf_tile(int32_t mode, int64_t m, int64_t n);
// Default Strassen depth cap of a mode for contractions of m rows.
int32_t default_max_depth(int32_t mode, int64_t m);

// Builds the plan (host only).  Throws std::invalid_argument on bad sizes.
Plan make_plan(int32_t mode, int64_t m, int64_t n, int64_t lda, const PlanOptions& opt);

// Bounded-workspace form of make_plan (Sec. 3.3's buffer reuse): stage 0 is
// the AtA plan with every Strassen root's C21 block taken out (SYRK leaves,
// depth-0 blocks, column norms and flags).  The top D levels of every root
// then run product by product: for each AtA level that has Strassen roots
// and each sequence (i_1, .., i_D) of products, one stage forms the operand
// sums that sequence needs on their own (Sum2Desc; a level's sums once per
// prefix), runs the remaining Strassen levels of the sequence's product
// resident into one buffer, and adds each finished product into its parent's
// quadrants (AccumDesc), bottom-up.  Level j's buffers (one product's sums
// and result) sit at the same arena offsets in every stage and persist while
// their prefix is unchanged; everything below them is reused by every stage.
// Stage 0's stats are the whole computation's (multiplications, leaves,
// nodes, levels).  Strassen's form only (variant 0); no fused pre-sums.
std::vector<Plan> make_staged_plan(int32_t mode, int64_t m, int64_t n, int64_t lda, const PlanOptions& opt);

// Plan of the general product C = A^T B (A m x n, B m x k, C n x k dense):
// one Strassen recursion (the paper's FastStrassen step on A^T B) writing
// the caller's C.  No spread check applies.
Plan make_gemm_plan(int32_t mode, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                    int64_t ldc, const PlanOptions& opt);

// Column-norm tasks of `count` problems (problem i: m[i] x n[i], row stride
// lda[i]); partial sums and norms of problem i start at the returned offsets.
// Problems with n = 0 get no task.  col1 / col2 never end up empty (a zero
// task stands in), and *partial_total is the partial array's length.
void build_colnorm_tasks(const int64_t* m, const int64_t* n, const int64_t* lda, int64_t count,
                         std::vector<ColDesc>& col1, std::vector<ColDesc>& col2,
                         int64_t* partial_total);

// Split-K: when a leaf launch (the mode's, or the FP64 fallback's) has fewer
// than `target` tiles, leaves with K >= 2 * min_chunk are cut into K chunks
// of at least min_chunk rows (multiples of 256, or of 128 for FP64, FP32
// and the FP64 fallback; down to that granule when the launch has fewer
// than 512 tiles), each chunk's tiles writing partial sums that a reduce
// pass adds.  The two launches are judged on their own tile counts.  Called before finalize_plan; merged batch plans are
// split once, after merging.
constexpr int64_t SPLIT_MIN_CHUNK = 8192;
void split_leaves(Plan& p, int64_t target, int64_t min_chunk = SPLIT_MIN_CHUNK);
// Tail balancing of the leaf launch.  Its tiles run longest-first on `slots`
// resident workgroups; when the last round is left partly idle (for example
// 528 equal tiles on 256 slots: two full rounds and 16 tiles), the smallest
// leaves covering that tail are cut into K chunks (same machinery as above),
// so their chunk tiles run last and fill the final round.  The cut is chosen
// by simulating list scheduling of the tiles' contraction lengths, and kept
// only when it shortens that makespan by at least 4%.  Plans that
// split_leaves has already split are left alone, and so are leaves under the
// spread check and the idle alternatives of flagged nodes.
void balance_tail(Plan& p, int64_t slots, int32_t max_split = 16);

// Split-BF16 plans with column norms: hand each problem's whole-A packing to
// its column-norm pass 1 task (which reads A anyway) and drop it from the
// pack launch.  Applied by the caller to the plan it executes (a single
// plan, or a batch's merged plan with its own pass 1 tasks), never to the
// parts of a batch.
void fuse_pack_into_norms(Plan& p, std::vector<ColDesc>& col1);

// FP8 plans with column norms, the other way round: for each problem whose
// quantisations include unpredicated full-height column slices of A that
// cover its columns once (the whole of A, or the diagonal leaves' slices),
// those quantisations also sum their column squares (per 128-row block row;
// pass 2 then sums the block rows in order) and the problem drops out of
// norm pass 1.  They move to the front of the list (pack8_norm); the pass 1 /
// pass 2 partial layout is rebuilt and its size returned in `partial_total`.
// Applied like fuse_pack_into_norms.
void fuse_norms_into_quant(Plan& p, std::vector<ColDesc>& col1, std::vector<ColDesc>& col2,
                           int64_t& partial_total);

// Orders the leaves (longest contraction first) and fills the tile and
// work-item prefix sums of every phase.
void finalize_plan(Plan& p);

// One plan for a batch of independent problems: every problem's phases are
// merged (arena offsets, node indices and problem indices shifted) so that
// each phase is one launch for the whole batch.
Plan merge_plans(std::vector<Plan>& parts, int64_t split_target = 0, int64_t slots = 0);

// Work items of the streaming kernels (pre-sums, packing, combines, column
// norms) run 256 to a workgroup; every task's first item is a multiple of
// this, so a workgroup never spans two tasks and finds its task once.
constexpr int64_t ITEM_BLOCK = 256;
inline int64_t item_align(int64_t e) { return (e + ITEM_BLOCK - 1) / ITEM_BLOCK * ITEM_BLOCK; }

// Output tile of the leaf kernels (shared with the device code): 128 x 128
// for FP64/FP32 (and the FP64 fallback), 256 x 128 for split-BF16.  A SYRK
// leaf tiles its lower triangle with tile rows of TM and tile columns of TN:
// tile row ti holds the tiles tj < min(rho (ti + 1), tiles_n), rho = TM / TN.
constexpr int TILE_M = 128;
constexpr int TILE_N = 128;
constexpr int tile_m_for(int32_t mode, int32_t tile_cfg) {
    return (mode == MODE_BF16X3 && tile_cfg >= 1) || (mode == MODE_FP8 && tile_cfg == 3) || (mode == MODE_F32 && tile_cfg >= 2) ? 256 : 128;
}
constexpr int tile_n_for(int32_t mode, int32_t tile_cfg) {
    return (mode == MODE_BF16X3 && tile_cfg >= 2) || (mode == MODE_FP8 && tile_cfg == 3) || (mode == MODE_F32 && tile_cfg >= 2) ? 256 : 128;
}
int64_t syrk_tiles(int64_t tm, int64_t tn, int64_t rho);

}  // namespace ata
