/*
 * ata.h -- C ABI of the MI355X (gfx950) AtA library.
 *
 * The library computes the symmetric Gram product C = A^T A of a rectangular
 * matrix A with the AtA method of Arrigoni, Maggioli, Massini and Rodola,
 * "Efficiently Parallelizable Strassen-Based Multiplication of a Matrix by
 * its Transpose" (arXiv 2110.13042):
 *   - Sec. 3.1, Eq. "submatA"/"Cij" and Alg. 1: split A into 2x2 blocks with
 *     floor/ceil halves; the diagonal blocks C11 and C22 come from recursive
 *     AtA calls, the off-diagonal block C21 from Strassen's seven-product
 *     scheme applied to A^T B, and C12 = C21^T is never formed;
 *   - Sec. 3.2: the cost is about 2/3 of Strassen's;
 *   - Sec. 3.3: Strassen temporaries live in one preallocated workspace.
 * Only the lower triangle of C is produced, in packed form (Sec. 4.3.1 packs
 * the lower triangle of A^T A results; the element order is this library's).
 *
 * Conventions for every entry point:
 *   - A is row-major: element (r, c) is A[r * lda + c], 0 <= r < m,
 *     0 <= c < n, lda >= max(1, n).  A and C_packed are DEVICE pointers on
 *     the handle's device; the caller owns them.
 *   - Output: C_packed[i * (i + 1) / 2 + j] = sum_r A[r][i] * A[r][j] for
 *     0 <= j <= i < n (row-major lower packed, n(n+1)/2 elements).  The
 *     library overwrites C (alpha = 1, beta = 0; Sec. 3.1 drops beta because
 *     C can be scaled beforehand).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     hipStream_t is itself an opaque pointer type, so the two are the same
 *     value at the ABI level; the header takes void* so that it needs no HIP
 *     header.  All device work is enqueued on it; no entry point of the
 *     compute path synchronises the host, except where stated.
 *   - Workspace: a handle keeps one workspace and grows it when a call needs
 *     more.  Calls may be recorded into a caller's graph (stream capture)
 *     once the same call has run eagerly, so that nothing is allocated while
 *     capturing.  After a call has been recorded, a later call that grows the
 *     workspace keeps the superseded buffers alive until ata_destroy, so a
 *     live graph never points at freed memory; the graph itself still uses
 *     the old buffers, which later eager calls no longer write.
 *   - Errors are returned, never thrown.  Argument errors are detected before
 *     anything is enqueued, and C is left untouched.  Device faults are
 *     asynchronous and surface at a later call or at the caller's sync.
 *   - A handle must not be used by two host threads at once.
 */
#ifndef ATA_H
#define ATA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ata_ctx* ata_handle_t;

typedef enum {
    ATA_OK = 0,
    ATA_ERR_INVALID_VALUE = 1,   /* bad argument: nothing enqueued            */
    ATA_ERR_NOT_SUPPORTED = 2,   /* valid request the library cannot serve    */
    ATA_ERR_OUT_OF_MEMORY = 3,   /* workspace above the limit or hipMalloc failed */
    ATA_ERR_HIP = 4,             /* a HIP runtime call failed                 */
    ATA_ERR_INTERNAL = 5
} ata_status_t;

typedef enum {
    ATA_F64 = 0,          /* A: double, C: double; FP64 MFMA leaves            */
    ATA_F32 = 1,          /* A: float,  C: float;  FP32 MFMA leaves            */
    ATA_F32_BF16X3 = 2,   /* A: float,  C: float;  split-BF16 hi/lo operands,
                             three BF16 MFMA products, FP32 accumulation       */
    ATA_F32_FP8E4M3 = 3   /* A: float,  C: float;  e4m3 operands with one
                             power-of-two scale per 128x128 block, FP32 acc.   */
} ata_dtype_t;

typedef enum {
    /* Leaf cutoff b (Sec. 3.1 base case): an AtA call on w columns is a SYRK
       leaf iff w <= b; a Strassen call on an n x k output is a GEMM leaf iff
       max(n, k) <= b.  0 = the planner's choice (default). */
    ATA_OPT_LEAF_CUTOFF = 0,
    /* Maximum Strassen levels under one AtA node; -1 = the mode's default
       (F64: unlimited, F32: 3, BF16X3: 2, FP8: 1; F32 and BF16X3 take 0
       when m >= 65536, since a level's rounding error adds to that of the
       long contraction).  ata_gram and ata_gemm_tn use fewer levels when the
       plan's workspace would not fit in the device's free memory (plus the
       arena the handle holds) with 1 GiB to spare: every level's sums and
       products are resident at once, about 7/4 more per level. */
    ATA_OPT_MAX_STRASSEN_DEPTH = 1,
    /* Spread threshold tau on column norms for the FP32-family FP64 fallback:
       an AtA node whose max/min squared column norm exceeds tau^2 runs its
       diagonal leaves in FP64 and its off-diagonal block without Strassen.
       <= 0 disables the check (default 4096). Ignored by ATA_F64. */
    ATA_OPT_SPREAD_TAU = 2,
    /* 1 = after each ata_gram, compute the FP64 Freivalds residual
       ||C x - A^T (A x)|| / (||A||_F^2 ||x||), x in {-1,+1}^n (default 0). */
    ATA_OPT_RESIDUAL = 3,
    /* Upper bound in bytes on the workspace; 0 = no bound (default). */
    ATA_OPT_WORKSPACE_LIMIT = 4,
    /* Seed of the residual probe signs (SplitMix64 counter stream). */
    ATA_OPT_RESIDUAL_SEED = 5,
    /* 1 = record HIP events on the call's stream around each launch phase of
       every ata_gram call; ata_get_report then synchronises and returns the
       summed phase times since the option was last set (default 0). */
    ATA_OPT_PROFILE = 6,
    /* Output tile of the leaf kernel.  -1 (default) = automatic: the
       autotune table's tile for the shape's bucket, else tile 2 for FP32
       when m, n >= 2048 (with leaf cutoff 2048 unless set) and for
       split-BF16 when m, n >= 4096, else tile 0; an explicit value also
       wins over the table.  Split-BF16: 0 = 128 x 128, 1 = 256 x 128,
       2 = 256 x 256 on eight waves, 3 = 256 x 256 on four waves of
       128 x 128 with operands streamed into LDS by buffer loads, 4 = the same
       stream on eight waves of 128 x 64.  FP8: 0 = 128 x 128, 3 = 256 x 256
       on four waves of 128 x 128 (1 and 2 act as 0).  FP32: 0 = 128 x 128,
       2 = 256 x 256 on eight waves of 128 x 64, 3 = 256 x 256 on four waves
       of 128 x 128 (1 acts as 0).  FP64 ignores it.  Batches use tile 0
       unless set or chosen by the batch autotuner. */
    ATA_OPT_LEAF_TILE = 7,
    /* ata_gram_batched: 1 = capture the batch's launch sequence once per
       shape signature in a hipGraph and replay it (default); 0 = enqueue the
       launches directly on the caller's stream. */
    ATA_OPT_BATCH_GRAPH = 8,
    /* Batched leaf products: 0 = one workgroup per tile in longest-first,
       XCD-grouped order, scheduled by the hardware dispatcher; 1 = a
       persistent grid (resident workgroups only) pulling tiles from per-XCD
       queues; -1 = as ATA_OPT_LEAF_PERSISTENT's automatic choice (default).
       Results are identical. */
    ATA_OPT_BATCH_PERSISTENT = 9,
    /* Leaf tile order (performance only; results are identical): in every
       window of 8 x XCD_CHUNK consecutive tiles each XCD gets XCD_CHUNK
       consecutive ones, so tiles sharing operand panels share an L2; GEMM
       leaves number their tiles in bands of TILE_BAND tile rows, column by
       column.  Both in [1, 4096]. */
    ATA_OPT_XCD_CHUNK = 10,
    ATA_OPT_TILE_BAND = 11,
    /* Split-K: when a leaf launch (the dtype's, or the FP64 fallback's) has
       fewer tiles than this, leaves with a contraction of at least 16384
       rows are cut into K chunks of at least 8192 rows (when the launch has
       fewer than 512 tiles: contractions of 512 rows or more, chunks of at
       least 256 rows) whose partial sums a reduce pass adds in chunk order,
       in FP64, rounding once (default 2048; 0 = never split).  Tall-skinny
       and small problems get enough tiles to fill the GPU. */
    ATA_OPT_SPLIT_TARGET = 12,
    /* ata_gram_batched: 1 = each member takes the per-shape autotune table
       entry of its own shape bucket; 0 (default) = members use the handle's
       options, else the batch autotuner's choice for the batch signature
       (ata_autotune_batched), else the defaults.  Per-shape choices are
       timed one problem at a time and need not suit a merged launch. */
    ATA_OPT_BATCH_USE_TABLE = 13,
    /* ata_gram, FP32-family dtypes: 1 = column equilibration instead of the
       FP64 fallback.  Column j of A is scaled by 2^-e_j (e_j = the binary
       exponent of its norm, so every scaled norm lies in [0.5, 1)) into a
       workspace copy (m n floats), the plan runs on the copy without the
       spread check, and C_ij is scaled back by 2^(e_i + e_j).  All scalings
       are exact; rounding errors become relative to ||a_i|| ||a_j||.  The
       residual option then checks the scaled product.  Default 0. */
    ATA_OPT_EQUILIBRATE = 14,
    /* Leaf products of single-problem calls (ata_gram, ata_gemm_tn and the
       forms built on them): 0 = one workgroup per tile, scheduled by the
       hardware dispatcher; 1 = a persistent grid pulling tiles from per-XCD
       queues; -1 = automatic (default): persistent for the 256 x 256 FP32
       tile, whose one resident workgroup per CU leaves the dispatcher's
       placement of tiles with unequal contractions far from longest-first,
       and one workgroup per tile otherwise (the persistent loop raises the
       register use of the smaller tiles).  Results are identical. */
    ATA_OPT_LEAF_PERSISTENT = 15,
    /* FP64 and FP32: 1 = a Strassen node whose seven products are all leaves
       forms its pre-sums S1..S5, T1..T5 (Sec. 3.2) while its leaves load
       their operands: each operand element is the same single IEEE sum or
       difference of two quadrant elements that the pre-sum pass would have
       stored, so results are bit-identical, without the pass and its
       workspace; 0 = the pre-sums are written to the workspace first
       (default: on MI355X the leaves reading two quadrants per fused
       operand lose more time than the streaming pre-sum pass costs).
       Split-BF16 and FP8 always form their last-level pre-sums in the
       operand packing / quantisation pass. */
    ATA_OPT_FUSE_PRESUM = 16,
    /* Form of every Strassen node (the AtB step of Sec. 3.2, Alg. 1):
       0 (default) = Strassen's seven products with ten pre-sums and eight
       post-additions, as the paper uses; 1 = Winograd's variant with the
       same seven-product count but four chained pre-sums per operand
       (S2 = S1 - X11, S4 = X21 - S2; T2 = Y22 - T1, T4 = T2 - Y21) and seven
       post-additions sharing partial sums, so two fewer workspace sums per
       node.  Both are exact in exact arithmetic; Winograd's rounding-error
       constant is somewhat larger.  With 1, ATA_OPT_FUSE_PRESUM is ignored
       (a chained sum is not one rounding of two quadrant elements). */
    ATA_OPT_STRASSEN_FORM = 17,
    /* 1 (default) = balance the last round of the leaf launch.  The leaf
       tiles run longest-first on the device's resident workgroups (CUs x
       workgroups per CU).  When the final round would leave most of them
       idle (for example 528 equal 256 x 256 tiles on 256 slots: two full
       rounds, then 16 tiles), the smallest leaves covering that tail are
       cut into K chunks whose partial sums the split-K reduce adds in FP64
       (rounded once), so the chunk tiles fill the last round.  The cut is
       chosen on the host by simulating the launch's list scheduling, and
       kept only when it shortens the simulated time by 4% or more; plans
       already split for a small launch, leaves under the spread check and
       the plain alternatives of flagged nodes are left alone.  Results of
       a cut leaf can differ from the uncut ones by rounding only.
       ata_report_t.tail_split_leaves tells whether a plan was cut.
       0 = never. */
    ATA_OPT_BALANCE_TAIL = 18,
    /* 1 = bounded workspace (Sec. 3.3 reuses one set of Strassen buffers per
       level instead of holding every level at once): ata_gram runs each
       Strassen root (the C21 block of an AtA node that gets Strassen levels)
       product by product.  For each AtA level with roots and each product
       i = 1..7, one stage forms product i's operand sums on their own, runs
       the product's remaining Strassen levels (resident) into one buffer and
       adds it into the root's quadrants in the combine's own order; every
       stage reuses the workspace from its start.  The number of top levels
       run this way is the smallest that keeps the workspace within
       3/2 n max(m, n) elements (Sec. 3.3's 3/2 n^2 for square A; about n^2
       for 30000 x 30000 FP64 at the default depth).  With split-K and tail
       cuts off (ATA_OPT_SPLIT_TARGET 0, ATA_OPT_BALANCE_TAIL 0) results are
       bit-identical to the default schedule's with the same leaf cutoff,
       depth and tile (the same sums, leaves and additions, in the same
       order); otherwise a stage's smaller launch may cut a contraction into
       K chunks where the resident launch does not, which changes rounding
       only.  Strassen's form
       only (ATA_OPT_STRASSEN_FORM and ATA_OPT_FUSE_PRESUM are ignored).
       Applies to ata_gram; ata_gram_noalloc, ata_gram_batched and
       ata_gemm_tn ignore it.  0 = every level resident (default). */
    ATA_OPT_BOUNDED_WORKSPACE = 19,
    /* Overlap of the Strassen pre-sums with leaf products.  The leaves whose
       operands are views of A (SYRK leaves and depth-0 blocks, and with them
       the FP64 fallback) need no pre-sum: they run in their own launch on a
       second stream (created by the handle, default priority), forked from
       `stream` after the column norms and joined back before the split-K
       reduce, while `stream` runs the pre-sums and the other leaves.  Plans
       without Strassen levels, FP8 plans and split-BF16 plans that pack A
       outside the column-norm pass (spread check off) run as one launch.
       Results are bit-identical either way (the same tiles, each computed
       once).  Profiling: phase 1 (pre-sums) then includes the first leaf
       launch's time, so the leaf time is phases 1 + 2.  Off by default: the
       256 x 256 leaf engines fill every CU's register file, so the pre-sums
       cannot run beside them and the split leaf launch loses its single
       longest-first order (measured slower on the 16384 x 16384 FP32 and
       split-BF16 plans).  1 = on, 0 = off (default), -1 = the default.
       Ignored by ata_gram_noalloc, batches, ata_gemm_tn and bounded-workspace
       plans. */
    ATA_OPT_OVERLAP = 20,
    /* Strassen combine in the leaf epilogues (Sec. 3.2's post-additions moved
       into the products).  A Strassen node whose seven products are all
       leaves gets no product buffers and no combine pass: each product's
       leaf adds its tiles straight into its one or two quadrants of the
       node's target.  The products run in five dependent leaf launches,
       {M1}, {M2}, {M3, M4}, {M5, M6}, {M7}, so that every quadrant element
       has one writer per launch and receives the combine's own left-to-right
       sum (C11 = ((M1 + M4) - M5) + M7, C12 = M3 + M5, C21 = M2 + M4, C22 =
       ((M1 - M2) + M3) + M6); the other leaves are spread over the five
       launches.  Results are bit-identical to the default schedule's when no
       leaf is cut into K chunks (ATA_OPT_SPLIT_TARGET 0, ATA_OPT_BALANCE_TAIL
       0): the leaves with epilogue combines are never cut, so other cuts can
       differ.  Strassen's form only; not with the 256 x 256 four-wave FP32
       and split-BF16 tiles (ATA_OPT_LEAF_TILE 3 runs without it).  Applies to
       ata_gram, ata_gram_noalloc and ata_gemm_tn; batches and
       bounded-workspace plans ignore it.  Off by default (measured slower:
       the product's read-modify-write of its quadrants moves as many bytes
       as the combine pass, and five launches leave five tails).
       1 = on, 0 = off (default). */
    ATA_OPT_FUSE_COMBINE = 21
} ata_option_t;

/* Plan and run summary of the last ata_gram call on a handle. */
typedef struct {
    int64_t m, n, lda;
    int32_t dtype;
    int32_t strassen_levels;      /* deepest Strassen recursion in the plan    */
    int64_t leaf_cutoff;          /* b used                                    */
    int64_t ata_nodes;            /* AtA calls in the recursion (incl. leaves) */
    int64_t syrk_leaves;
    int64_t gemm_leaves;
    int64_t strassen_nodes;
    int64_t multiplications;      /* scalar multiplications of the plan
                                     (leaf sizes at the ceil dimensions)       */
    int64_t workspace_bytes;      /* device workspace the plan needs           */
    int64_t kernel_launches;      /* launches per ata_gram call                */
    int64_t flagged_nodes;        /* AtA nodes flagged for the FP64 fallback;
                                     -1 if not evaluated (syncs the stream)   */
    double residual;              /* Freivalds residual; -1 if not computed   */
    int64_t profiled_calls;       /* calls timed since ATA_OPT_PROFILE was set */
    double phase_ms[5];           /* summed ms: column norms + flags, pre-sums,
                                     leaf products, combines, residual        */
    int32_t leaf_tile;            /* leaf tile configuration of the plan
                                     (ATA_OPT_LEAF_TILE's values)             */
    int32_t leaf_persistent;      /* 1 = the leaf products ran as a persistent
                                     grid, 0 = one workgroup per tile          */
    int32_t tail_split_leaves;    /* leaves cut by the tail balancer (0: none) */
    int32_t tail_split_chunks;    /* K chunks per cut leaf                     */
    int32_t overlapped;           /* 1 = the leaves reading only A ran beside
                                     the pre-sums (ATA_OPT_OVERLAP)            */
    int32_t leaf_rounds;          /* leaf launches in sequence: 1, or the
                                     launch rounds of the combines in the leaf
                                     epilogues (ATA_OPT_FUSE_COMBINE)          */
} ata_report_t;

/* One leaf of a plan, as returned by ata_plan_query. */
typedef struct {
    int32_t kind;                 /* 0 = SYRK (diagonal), 1 = GEMM             */
    int32_t depth;                /* Strassen level of the leaf (0 = none)     */
    int64_t rows, cols, contraction;  /* output rows x cols, summed length     */
    int64_t out_row0, out_col0;   /* position in C when written there, else -1 */
    int32_t ksplit;               /* K chunks (split-K; 1 = not split)         */
    int32_t pad_;
} ata_leaf_t;

/* Create a handle bound to the current HIP device.  The first handle on a
   device also looks up that device's address of the static workspace of
   ata_gram_noalloc (which loads the library's code object there).  Returns
   ATA_ERR_HIP when no device is usable or the lookup fails.  *out is set to
   NULL on failure. */
ata_status_t ata_create(ata_handle_t* out);

/* Destroy a handle and free its device memory.  No work that uses the handle
   may still be in flight.  NULL is accepted (no-op). */
ata_status_t ata_destroy(ata_handle_t h);

/* C_packed = lower(A^T A) (Alg. 1 AtA with the handle's options).
   m = 0 zero-fills C; n = 0 is a no-op.  A and C must not overlap.
   A and C hold doubles for ATA_F64 and floats for the other dtypes.
   Returns ATA_ERR_INVALID_VALUE for a null handle or pointer with nonzero
   size, negative m or n, lda < max(1, n), an unknown dtype or overlapping A
   and C; ATA_ERR_NOT_SUPPORTED when a split-BF16 or FP8 leaf operand would
   need a packed array of 4 GiB or more (those arrays are read through 32-bit
   buffer offsets; when one packing of all of A would, split-BF16 packs each
   leaf operand on its own instead); ATA_ERR_OUT_OF_MEMORY when the workspace cannot be
   allocated or exceeds ATA_OPT_WORKSPACE_LIMIT; ATA_ERR_HIP when a launch
   fails.  The first call for a (shape, dtype, options) combination builds and
   uploads the plan (host work and a synchronous copy); later calls only
   enqueue kernels. */
ata_status_t ata_gram(ata_handle_t h, const void* A, int64_t m, int64_t n,
                      int64_t lda, ata_dtype_t dtype, void* C_packed,
                      void* stream);

/* Size in bytes of the static device workspace of ata_gram_noalloc: one
   array per GPU in the library's code object, allocated when the code
   object is loaded on that GPU (at the first ata_create there) and held until
   the process ends. */
#define ATA_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under stream capture,
   tight serving loops, harnesses that forbid hipMalloc): ata_gram with every
   workspace buffer (plan descriptors, Strassen sums and products, packed
   operands, split-K partials, column norms, spread flags, queue heads) in the
   GPU's static ATA_NOALLOC_SCRATCH_BYTES array.  The call allocates no device
   or pinned memory and calls no allocating library routine; it copies the
   plan's descriptors into the array on `stream` (hipMemcpyAsync from host
   memory the handle keeps) and then enqueues the same kernels as ata_gram.
   Arguments, layout, output and argument errors are ata_gram's.  The plan is
   ata_gram's for the same handle options, with the Strassen depth lowered
   (then split-K and tail cuts dropped) until its workspace fits the array;
   results equal ata_gram's whenever the plans agree.  Returns
   ATA_ERR_OUT_OF_MEMORY, with nothing enqueued and C untouched, when even
   that plan does not fit (for example split-BF16 needs 4 bytes per element
   of A for its packed operands), or exceeds ATA_OPT_WORKSPACE_LIMIT; and
   ATA_ERR_NOT_SUPPORTED when the handle has ATA_OPT_EQUILIBRATE or
   ATA_OPT_RESIDUAL set.  ATA_OPT_PROFILE is ignored, and the report's
   flagged-node count and residual are not available (-1).
   Every call on one GPU shares that GPU's array and leaves its contents
   there: calls that may overlap on one GPU (different streams, handles or
   threads without ordering between them) race and must be serialised by the
   caller; calls in order on one stream are safe.  The queue heads the leaf
   launch needs at zero are cleared by a kernel on `stream` in every call. */
ata_status_t ata_gram_noalloc(ata_handle_t h, const void* A, int64_t m, int64_t n,
                              int64_t lda, ata_dtype_t dtype, void* C_packed,
                              void* stream);

/* batch independent Gram products, C_packed[i] = lower(A[i]^T A[i]), of
   uneven shapes.  Every problem's plan is merged into one: each phase is a
   single launch for the whole batch, and all leaf products of all problems
   run in one launch, longest contraction first (one workgroup per tile, or
   with ATA_OPT_BATCH_PERSISTENT a persistent grid pulling tiles from per-XCD
   queues).  Each problem takes its own leaf cutoff and depth (options, else
   the autotune table, else the defaults); the leaf tile shape is the
   handle's.  The first call for a shape signature
   (the m, n, lda of every member plus the handle's options) builds the plan
   and captures the launch sequence in a hipGraph; later calls replay it on an
   internal stream ordered after `stream` by events (the caller's stream
   waits for the replay).  The host arrays are read during the call only; when
   the pointers differ from the previous call of the same signature, the call
   first waits for that call's replay to finish.  Any invalid member fails the
   whole call with nothing enqueued; the first bad index is in the report's
   `m` field as -(index + 1).  No residual is computed for batches. */
ata_status_t ata_gram_batched(ata_handle_t h, int64_t batch,
                              const void* const* A, const int64_t* m,
                              const int64_t* n, const int64_t* lda,
                              ata_dtype_t dtype, void* const* C_packed,
                              void* stream);

/* C_packed = alpha * lower(A^T A) + beta * C_packed (the BLAS ?syrk form of
   the problem statement of Sec. 3.1; ata_gram is alpha = 1, beta = 0).
   beta = 0: C is not read.  Otherwise the product goes to a workspace
   buffer of n(n+1)/2 elements first and a final pass combines it with C.
   Non-finite alpha or beta: ATA_ERR_INVALID_VALUE.  Other errors as for
   ata_gram. */
ata_status_t ata_gram_scaled(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                             ata_dtype_t dtype, double alpha, double beta, void* C_packed,
                             void* stream);

/* C_packed = lower(A A^T) for row-major A (m x n, lda >= max(1, n)); C is
   m x m packed lower (m(m+1)/2 elements).  A is transposed once into a
   workspace buffer (m n elements), then the AtA plan runs on the n x m
   transpose.  n = 0 zero-fills C; m = 0 is a no-op.  Errors as for
   ata_gram. */
ata_status_t ata_gram_aat(ata_handle_t h, const void* A, int64_t m, int64_t n, int64_t lda,
                          ata_dtype_t dtype, void* C_packed, void* stream);

/* Full symmetric n x n matrix C_full (row-major, row stride ldf >= max(1, n))
   from packed lower storage: C_full[i][j] = C_packed[max(i,j)(max(i,j)+1)/2 +
   min(i,j)].  The two buffers must not overlap. */
ata_status_t ata_unpack(ata_handle_t h, const void* C_packed, int64_t n, ata_dtype_t dtype,
                        void* C_full, int64_t ldf, void* stream);

/* General product C = A^T B by the Strassen recursion alone (the step AtA
   applies to its off-diagonal blocks, Sec. 3.1, Eq. "Cij"; Strassen's seven
   products on the 2 x 2 blocks of A^T and B).  A is m x n (row stride lda >=
   max(1, n)), B is m x k (ldb >= max(1, k)), C is n x k dense row-major
   (ldc >= max(1, k)); all device pointers of the dtype's element type.  C is
   overwritten; m = 0 zero-fills it; n = 0 or k = 0 is a no-op.  The handle's
   leaf cutoff, depth cap, tile and split options apply (the autotune table is
   consulted with the bucket of max(n, k)); there is no spread check.  Errors
   as for ata_gram; C must not overlap A or B. */
ata_status_t ata_gemm_tn(ata_handle_t h, const void* A, const void* B, int64_t m, int64_t n,
                         int64_t k, int64_t lda, int64_t ldb, ata_dtype_t dtype, void* C,
                         int64_t ldc, void* stream);

/* Freivalds probe of a given product (the check ATA_OPT_RESIDUAL runs after
   ata_gram): *result = ||C x - A^T (A x)||_2 / (||A||_F^2 ||x||_2) with
   x_j = +1 if the top bit of SplitMix64 output j of stream `seed` is 0, else
   -1; computed in FP64 on the device.  A is m x n (lda), C_packed the packed
   lower triangle of an n x n symmetric matrix, both device pointers of the
   dtype's element type (double for ATA_F64, float otherwise).  Blocks until
   the result is on the host (synchronises `stream`). */
ata_status_t ata_residual(ata_handle_t h, const void* A, int64_t m, int64_t n,
                          int64_t lda, ata_dtype_t dtype, const void* C_packed,
                          uint64_t seed, double* result, void* stream);

/* Sampled-column check in FP64 on the GPU (the residual's column form):
   for the `count` column indices in the host array `cols` (each in [0, n),
   repeats allowed), forms the reference columns (A^T A)[:, j] = A^T a_j with
   FP64 products and sums (a product of two FP32 inputs is exact in FP64),
   reads the same columns of the packed C (C[i][j] for i >= j, C[j][i]
   above the diagonal), and stores ||C_S - (A^T A)_S||_F / ||(A^T A)_S||_F
   in *result (0 for n = 0 or count = 0; +inf when the reference is zero and
   C is not).  Reported, not enforced.  A and C_packed are device buffers of
   the dtype's element type.  Allocates and frees a temporary of about
   8 (m count + n count / 512) bytes; blocks until the result is on the host
   (synchronises `stream`).  ATA_ERR_INVALID_VALUE for a bad size, a null
   pointer or a column index out of range, before any device work. */
ata_status_t ata_check_columns(ata_handle_t h, const void* A, int64_t m, int64_t n,
                               int64_t lda, ata_dtype_t dtype, const void* C_packed,
                               const int64_t* cols, int64_t count, double* result,
                               void* stream);

/* One autotuned plan choice. */
typedef struct {
    int64_t leaf_cutoff;
    int32_t max_depth;
    int32_t leaf_tile;
    double ms;                    /* measured time of one ata_gram call */
} ata_tune_entry_t;

/* Autotuner: times ata_gram on (A, C_packed) -- device buffers of the given
   shape; A is only read, C_packed is overwritten -- for every candidate leaf
   cutoff (powers of two from 128 up to the first at or above n), Strassen
   depth cap (0 up to the smaller of 3 and the dtype's default) and leaf
   tile (ATA_F32_BF16X3: 0..4; ATA_F32: 0, 2 or 3; ATA_F32_FP8E4M3: 0 or 3)
   once, times the four fastest again in three interleaved rounds (each
   scoring its best round), keeps the winner in the handle's table under
   (dtype, shape bucket) and returns
   it in *best (may be NULL).  Buckets are half-octaves of m and of n.
   ata_gram and ata_gram_batched use the table whenever the leaf cutoff and
   depth options are left at their defaults (0 and -1).  Synchronises
   `stream`. */
ata_status_t ata_autotune(ata_handle_t h, const void* A, int64_t m, int64_t n,
                          int64_t lda, ata_dtype_t dtype, void* C_packed,
                          void* stream, ata_tune_entry_t* best);

/* Batch autotuner: times ata_gram_batched on the given batch (A read, C
   overwritten) for candidate leaf cutoffs (128 .. 4096), Strassen depth caps
   (0 up to the smaller of 2 and the dtype's default) and, for
   ATA_F32_BF16X3, leaf tiles, and keeps the fastest for the batch's
   signature (dtype, and m, n, lda of every member) in the handle; later
   ata_gram_batched calls with that signature and default leaf cutoff / depth
   options use it.  Every candidate builds and caches its plan and graph.
   Synchronises `stream`.  Batch choices are not saved by ata_tune_save. */
ata_status_t ata_autotune_batched(ata_handle_t h, int64_t batch, const void* const* A,
                                  const int64_t* m, const int64_t* n, const int64_t* lda,
                                  ata_dtype_t dtype, void* const* C_packed, void* stream,
                                  ata_tune_entry_t* best);

/* Save / load the handle's tune table as JSON (one object per entry with the
   device architecture, dtype, buckets and choice).  Loading merges entries of
   the current architecture and skips others. */
ata_status_t ata_tune_save(ata_handle_t h, const char* path);
ata_status_t ata_tune_load(ata_handle_t h, const char* path);

/* Set an option (see ata_option_t); takes effect at the next call. */
ata_status_t ata_set_option(ata_handle_t h, ata_option_t key, double value);

/* Copy the last call's report.  When the last call computed a residual or a
   fallback flag count, this synchronises the stream of that call first. */
ata_status_t ata_get_report(ata_handle_t h, ata_report_t* out);

/* Host-only planning query: no device needed, no handle.  Fills *info (may be
   NULL) and up to `cap` leaves; *n_leaves receives the total leaf count.
   leaf_cutoff <= 0 and max_depth < 0 select the defaults. */
ata_status_t ata_plan_query(int64_t m, int64_t n, ata_dtype_t dtype,
                            int64_t leaf_cutoff, int32_t max_depth,
                            ata_report_t* info, ata_leaf_t* leaves, int64_t cap,
                            int64_t* n_leaves);

/* Column norms and spread flags of the last ata_gram call, when that call ran
   the spread check of the FP64 fallback (an FP32-family dtype with
   ATA_OPT_SPREAD_TAU > 0, m > 0, no equilibration).  nu (host, n doubles,
   n must equal that call's n) receives nu_j = sum_r A[r][j]^2 summed in FP64;
   node_c0, node_w and flags (host arrays of `cap` entries) receive, for each
   AtA node of the plan in the recursion's pre-order (a node, then its left
   column half, then its right half: Alg. 1's call order), its first column,
   its width and its flag (1 when max nu / min nu over the node's nonzero
   columns exceeds tau^2, else 0).  Any of the arrays may be NULL; *count
   (may be NULL) receives the number of nodes.  Synchronises the stream of
   that call when nu or flags is requested.  ATA_ERR_INVALID_VALUE when the
   handle's last call was not such an ata_gram call (a later call of
   another compute entry point clears it) or n differs. */
ata_status_t ata_get_spread(ata_handle_t h, double* nu, int64_t n, int64_t* node_c0,
                            int64_t* node_w, uint8_t* flags, int64_t cap, int64_t* count);

/* Static description of a status code. */
const char* ata_status_string(ata_status_t s);

#ifdef __cplusplus
}
#endif

#endif /* ATA_H */
