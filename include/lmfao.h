/*
 * lmfao.h -- C ABI of the MI355X (gfx950) engine for batches of group-by
 * aggregates over the natural join of several relations.
 *
 * The operation (paper, section 2 "LMFAO by Example", and section 3 "From
 * Learning to Aggregates"): given a database schema, a join tree over its
 * relations and a batch of queries
 *
 *     SELECT G, SUM(f_1), ..., SUM(f_m) FROM D WHERE P GROUP BY G
 *
 * where D is the natural join of all relations (bag semantics), compute every
 * query's result.  The engine follows the paper's plan: each query gets a root
 * relation and is decomposed into one view per join-tree edge, views with the
 * same direction, group-by attributes and condition are merged, views and
 * queries leaving the same relation are grouped, and each group is computed
 * in one pass over its relation sorted by a total order of its join
 * attributes, with lookups into the incoming views and partial aggregates
 * factored out of the inner loops (section 2, view generation and
 * multi-output optimization layers; Figure 2 and Figure 3).
 *
 * Supported query class (anything else returns LMFAO_EUNSUPPORTED from
 * lmfao_plan):
 *   - aggregate functions are products of attribute powers of total degree
 *     <= 2 (COUNT = the empty product), the forms section 3 lists for ridge
 *     regression, CART split statistics and Rk-means;
 *   - at most 2 group-by attributes per query, each an integer attribute with
 *     a domain hint (values in [0, domain));
 *   - every join attribute is an integer attribute with a domain hint;
 *   - conditions (WHERE) are conjunctions of `attr op constant`: the
 *     conditions every query of the batch shares (a tree node's path
 *     condition) filter the relations' rows at the start of every run, and
 *     each query may add one more condition on a single attribute (a split
 *     candidate), which is planned as a group-by on a bucket code of that
 *     attribute and summed over the buckets it selects; a query with two or
 *     more conditions of its own returns LMFAO_EUNSUPPORTED.
 *
 * Conventions for every entry point:
 *   - all pointers to schema, tree, batch and option structs are host
 *     pointers, read during the call only; the library copies what it keeps;
 *   - relation column pointers passed to lmfao_prepare are DEVICE pointers
 *     (HIP global memory on the current device), one contiguous column per
 *     attribute, int32 / float32 / float64 as declared; they are read during
 *     lmfao_prepare only (the library keeps sorted device copies);
 *   - `stream` arguments are hipStream_t handles passed as void* (NULL = the
 *     default stream); all device work of a call is enqueued on that stream;
 *   - status codes are returned, never exceptions; on failure
 *     lmfao_last_error() returns a thread-local, NUL-terminated description
 *     valid until the next call on the same thread;
 *   - handles (plan, prepared, result) are opaque and owned by the library;
 *     free them with the matching *_free call.  A plan is immutable and may be
 *     shared; a prepared handle serializes its runs (one run at a time).
 */
#ifndef LMFAO_H
#define LMFAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lmfao_status;
enum {
  LMFAO_OK = 0,
  LMFAO_EINVAL = 1,        /* malformed input: bad tree, unknown attribute, ...   */
  LMFAO_ENOMEM = 2,        /* device or host allocation failed                    */
  LMFAO_EHIP = 3,          /* a HIP runtime call failed (text in last_error)       */
  LMFAO_EUNSUPPORTED = 4,  /* valid input outside the supported query class        */
  LMFAO_EOVERFLOW = 5      /* a group-by table could not be sized                  */
};

enum { LMFAO_I32 = 0, LMFAO_F32 = 1, LMFAO_F64 = 2 };

/* One attribute of a relation.  `domain` > 0 declares integer values in
 * [0, domain) -- the paper's cardinality constraints ("sizes of relations and
 * attribute domains", section 2, view generation layer).  `is_key` marks the
 * relation's primary key (underlined attributes in the schema of Figure 2);
 * the engine relies on it only to know that a relation has at most one tuple
 * per key value, and checks that during lmfao_run (LMFAO_EINVAL on a
 * duplicate key). */
typedef struct {
  const char* name;
  int32_t dtype;    /* LMFAO_I32 / LMFAO_F32 / LMFAO_F64 */
  int64_t domain;   /* integer attributes: values in [0, domain); 0 = none */
  int32_t is_key;
} lmfao_attr;

typedef struct {
  const char* name;
  int64_t n_rows;
  int32_t n_attrs;
  const lmfao_attr* attrs;
} lmfao_relation;

typedef struct {
  int32_t n_relations;
  const lmfao_relation* relations;
} lmfao_schema;

/* Join tree: undirected edges between relation indices.  It must connect all
 * relations, be acyclic, and satisfy the running-intersection property (the
 * relations holding an attribute form a connected subtree).  Two adjacent
 * relations join on every attribute name they share (natural join). */
typedef struct { int32_t a, b; } lmfao_edge;
typedef struct {
  int32_t n_edges;
  const lmfao_edge* edges;
} lmfao_join_tree;

/* An aggregate function: the product of `attr`^`power` over its factors;
 * n_factors == 0 is SUM(1).  power is 1 or 2. */
typedef struct { const char* attr; int32_t power; } lmfao_factor;
typedef struct {
  int32_t n_factors;
  const lmfao_factor* factors;
} lmfao_aggregate;

enum { LMFAO_LE = 0, LMFAO_LT = 1, LMFAO_GT = 2, LMFAO_GE = 3, LMFAO_EQ = 4, LMFAO_NE = 5 };
typedef struct { const char* attr; int32_t op; double constant; } lmfao_condition;

typedef struct {
  int32_t n_groupby;
  const char* const* groupby;
  int32_t n_conditions;
  const lmfao_condition* conditions;
  int32_t n_aggregates;
  const lmfao_aggregate* aggregates;
  int32_t root;        /* relation index, or -1 for the root heuristic */
} lmfao_query;

/* A user-defined factor (section 2: aggregates such as SUM(g(item) *
 * h(date))): a function of one integer attribute with a domain, given by
 * its value at every attribute value 0 .. domain-1 (HOST array of
 * n_values = domain doubles, copied by lmfao_plan).  Factors name it in
 * `attr` like an attribute (power 1 or 2); at prepare time its values are
 * gathered into an FP64 column of one relation holding the attribute. */
typedef struct {
  const char* name;
  const char* attr;
  int64_t n_values;
  const double* values;
} lmfao_function;

typedef struct {
  int32_t n_queries;
  const lmfao_query* queries;
  int32_t n_functions;
  const lmfao_function* functions;
} lmfao_batch;

/* F64 and F32: arithmetic of the scans, views and contraction.  BF16X3:
 * scans and views in FP32; in the matrix-core contraction each tile without
 * integer cells splits its FP32 operands x into three bf16 parts,
 * hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid) (24 bits in all),
 * and sums the six products hi*hi' + hi*mid' + mid*hi' + hi*lo' + mid*mid' +
 * lo*hi' on the bf16 matrix cores (v_mfma_f32_16x16x16_bf16), in FP32 within
 * a chunk of 16 pieces and FP64 across chunks; the terms left out are about
 * 2^-24 of each product, FP32 accuracy.  Tiles with integer cells stay exact
 * in FP64.  BF16X2: two parts (hi, lo) and three products; each product is
 * then within about 2^-16 of exact, so a float result is within 2^-16 of the
 * sum of its terms' magnitudes.  Both require LMFAO_CONTRACT_MFMA. */
enum { LMFAO_PREC_F64 = 0, LMFAO_PREC_F32 = 1, LMFAO_PREC_BF16X3 = 2, LMFAO_PREC_BF16X2 = 3 };
enum { LMFAO_FORM_FUSED = 0, LMFAO_FORM_PER_VIEW = 1 };
/* Root heuristics.  GROUPBY: the relation holding every group-by attribute,
 * the largest such relation (reproduces the roots of the worked example);
 * FACT: the largest relation from which every group-by attribute is reached
 * through primary-key joins (carried as a code by single-valued views), and
 * queries over the attributes of a single relation are rooted there. */
enum { LMFAO_ROOT_GROUPBY = 0, LMFAO_ROOT_FACT = 1, LMFAO_ROOT_COST = 2 };
/* COST: a cost model and a search.  A root assignment costs the bytes the
 * fused plan moves: one pass over every relation that computes a view or a
 * query (16 bytes a row) plus every distinct view's dense key space (8 bytes
 * a cell; views are shared across queries as view generation merges them).
 * Starting from the FACT roots, the queries with the same group-by
 * attributes and conditions move together, class by class, to the root of
 * least cost with the other classes fixed, until a round moves nothing.
 * Root overrides in the batch are kept.  If the plan of the chosen roots
 * falls outside the supported class, the FACT roots are used instead
 * ("root_fallback" in the description).  lmfao_plan_describe reports the
 * final assignment's cost ("root_cost_bytes") under every policy. */
/* Kernel for the segment-level contraction sum over pieces of (outer
 * features) x (inner partial sums).  MFMA: the features and columns of each
 * piece are staged in FP64 and multiplied on the matrix cores
 * (v_mfma_f64_16x16x4f64), split over K with a deterministic merge; integer
 * cells are exact while they stay below 2^53 (LMFAO_EOVERFLOW from lmfao_run
 * with sync otherwise).  VALU: one fused kernel with FP64 register tiles and
 * compensated sums, integer cells in int64. */
enum { LMFAO_CONTRACT_MFMA = 0, LMFAO_CONTRACT_VALU = 1 };

typedef struct {
  int32_t precision;     /* LMFAO_PREC_*: arithmetic of the scans and views;
                            merges and query results are always FP64        */
  int32_t form;          /* LMFAO_FORM_*                                     */
  int32_t root_policy;   /* LMFAO_ROOT_*                                     */
  /* optional attribute order per relation: order[r] lists n_order[r] join
   * attribute names of relation r, outermost first (NULL = heuristic) */
  const int32_t* n_order;
  const char* const* const* order;
  int32_t min_segment;   /* cut level: shortest average segment the factorized
                            scan accepts (0 = default 64)                    */
  int64_t row_piece_max; /* relations with at most this many rows are
                            contracted row by row without a scan
                            (0 = default 2^16; -1 = always scan)             */
  int32_t contraction;   /* LMFAO_CONTRACT_* (0 = matrix cores)              */
  int32_t codegen;       /* 0: scans of the lean class are generated per
                            group and compiled with hipRTC at prepare time
                            (falls back to the built-in kernel if that
                            fails); 1: built-in kernels only               */
  int64_t hash_slots;    /* initial slots of every hash table (outputs whose
                            dense key space exceeds 2^24 cells); 0 = sized
                            by `sizing`.  A run with sync grows a table that
                            overflowed (x4) and repeats, so results never
                            depend on the initial size                     */
  int32_t sizing;        /* LMFAO_SIZING_*                                    */
  const float* estimator;/* HOST estimator blob (layout below), copied by
                            lmfao_plan; NULL = none                          */
  int64_t estimator_len; /* floats in `estimator`                            */
  int32_t graph;         /* 1: the first lmfao_run without sync or timing is
                            captured into a HIP graph (on a stream of the
                            library's own) and later ones replay it on the
                            caller's stream; a run with sync, or with timing
                            on, launches directly, and a hash-table regrowth
                            drops the graph.  Falls back to direct launches
                            if capture fails.                               */
  int32_t one_hot_max;   /* outputs keyed only by outer codes: the largest key
                            space expanded one-hot into the matrix-core
                            contraction; larger ones are scattered per piece.
                            0 = 64, or 16 in a group whose one-hot features
                            would exceed 256.  Outputs that also have inner
                            keys expand outer key spaces up to 64          */
  int32_t scan_blocks;   /* most workgroups of one scan launch (0 = 2048 for
                            generated scans, 512 for the built-in ones);
                            each has 8 wavefronts and takes whole work
                            items                                          */
  int32_t partition;     /* 0: SUM(1) queries whose dense group-by table is
                            larger than a scan keeps in LDS (and at most 2^24
                            cells), grouped by columns of their root or codes
                            of single-valued views into it, are counted by
                            radix partition: their rows' cells are grouped
                            by 2^15-cell slice and each slice is counted in
                            LDS; 1: such tables are counted by the scans
                            with global atomics                             */
  int32_t contract_splits; /* ranges the pieces of a matrix-core contraction
                            are cut into, per column of output tiles (0 =
                            1024, fewer past 4096 workgroups)              */
  uint32_t row_weights;  /* bit r set: relation r (schema index below 32)
                            takes a 0/1 weight per row, written by the
                            caller into the buffer lmfao_row_weights returns
                            (all 1 after lmfao_prepare); every run counts a
                            tuple of D only if each of its rows in these
                            relations has weight 1 -- a condition common to
                            the whole batch whose constants change between
                            runs without a new plan (a CART node's path,
                            section 3, decision trees)                     */
} lmfao_options;

/* Initial capacity of a hash table.  BOUND: twice the most groups the output
 * can have -- the least of the product over its key attributes of their
 * distinct counts (counted on the GPU at prepare time), the dense key space,
 * and the rows of any relation whose tuple determines every key attribute
 * (holds it, or reaches its holder through joins on primary keys).  LEARNED: the group count the
 * estimator predicts, 2^(y + margin) - 1, at half occupancy, never above the
 * BOUND capacity and never below 1024 slots.  Both round up to a power of
 * two and start at most at 2^26 slots; regrowth goes up to the BOUND
 * capacity.  LEARNED without an estimator blob behaves as BOUND.  EXACT:
 * lmfao_prepare runs the whole batch once with BOUND tables, counts every
 * table's groups on the device and reallocates it at twice that count (the
 * exact-count pass; it belongs to lmfao_prepare, not to lmfao_run). */
enum { LMFAO_SIZING_BOUND = 0, LMFAO_SIZING_LEARNED = 1, LMFAO_SIZING_EXACT = 2 };

/* Estimator blob: {version = 2, d = LMFAO_EST_FEATURES, h, margin},
 * then d feature means, d feature standard deviations, then the
 * lmfao_mlp_size(d, h) network parameters (layout of lmfao_mlp_train).  The
 * network maps standardized features (x - mean) / std to the shortfall of
 * log2(1 + groups) below feature 14 (log2 of the BOUND group count), so the
 * estimate is y = x[14] - network((x - mean) / std).
 * Features of an output with key attributes K, in order (log2 means
 * log2(1 + value); per-key slots follow K's order, zero past |K| or past 3):
 *   0 log2 rows of the query's root relation   1 log2 total rows of all relations
 *   2 number of relations                      3 |K|
 *   4..6 log2 distinct count of each key       7..9 log2 domain of each key
 *   10..12 tree distance from the root to the nearest relation holding the key
 *   13 log2 product of the distinct counts     14 log2 of the BOUND group count
 *   15 1 if some relation's tuple determines every key attribute, else 0
 *   16 number of conditions of the batch-wide filter
 *   17..19 log2 rows of each key's holder (the relation nearest the root
 *          holding it)
 *   20..22 log2 distinct values, in the holder's neighbour toward the root, of
 *          the first attribute the two share (the holder's rows if it is the
 *          root)
 *   23..25 log2 distinct values of that attribute in the holder (same) */
#define LMFAO_EST_FEATURES 26

typedef struct lmfao_plan_s* lmfao_plan_t;
typedef struct lmfao_prepared_s* lmfao_prepared_t;
typedef struct lmfao_result_s* lmfao_result_t;

/* Fills `opts` with the defaults (F64, FUSED, GROUPBY, heuristic orders). */
void lmfao_default_options(lmfao_options* opts);

/* Validates schema, tree and batch and builds the plan on the host (no device
 * work): root per query, views per edge, merged views, groups and their
 * dependency levels, attribute orders, factorized per-group programs.
 * Errors: LMFAO_EINVAL (malformed), LMFAO_EUNSUPPORTED (outside the class). */
lmfao_status lmfao_plan(const lmfao_schema* schema, const lmfao_join_tree* tree,
                        const lmfao_batch* batch, const lmfao_options* opts,
                        lmfao_plan_t* out);

/* JSON description of the plan (roots, views, groups, dependency edges,
 * orders, per-group programs).  Writes at most `cap` bytes including the NUL
 * into `buf` (may be NULL when cap == 0) and the full size into *need. */
lmfao_status lmfao_plan_describe(lmfao_plan_t plan, char* buf, size_t cap, size_t* need);

/* Device bytes lmfao_prepare and lmfao_run will hold for this plan and these
 * relation sizes (estimate, excluding data-dependent piece tables). */
lmfao_status lmfao_plan_workspace_bytes(lmfao_plan_t plan, size_t* bytes);

/* Copies and sorts the relations each factorized group scans (by the group's
 * attribute order, on the GPU), builds their segment ("trie level") tables
 * and allocates every view and result buffer.  `columns[r][a]` is the device
 * pointer of attribute a of relation r (schema order).  Synchronizes
 * `stream` before returning.  The caller's columns may be freed afterwards. */
lmfao_status lmfao_prepare(lmfao_plan_t plan, const void* const* const* columns,
                           void* stream, lmfao_prepared_t* out);

/* lmfao_prepare with every device buffer of the prepared plan -- sorted
 * columns, pieces, views, results, hash tables, sort scratch, and later the
 * compacted results of lmfao_result_device and regrown hash tables -- carved
 * from the caller's `workspace` (a DEVICE allocation of `workspace_bytes`
 * bytes, aligned to 256 bytes, e.g. a torch tensor; the library allocates no
 * device memory for this handle).  Nothing is handed back before
 * lmfao_prepared_free, so scratch counts in full.  A workspace that is too
 * small gives LMFAO_ENOMEM (message: the bytes carved so far).
 * lmfao_prepared_workspace_bytes of a handle prepared from the same plan and
 * inputs gives the bytes needed: what lmfao_prepare carved, plus with
 * with_results != 0 what lmfao_result_device carves for every query.  The
 * workspace must stay allocated until lmfao_prepared_free. */
lmfao_status lmfao_prepare_in(lmfao_plan_t plan, const void* const* const* columns, void* workspace,
                              size_t workspace_bytes, void* stream, lmfao_prepared_t* out);
lmfao_status lmfao_prepared_workspace_bytes(lmfao_prepared_t prep, int32_t with_results, size_t* bytes);

/* Autotuner of the physical plan's launch shapes.  Tunes, for the batch
 * over these relations on this device, the options that shape launches --
 * scan_blocks (workgroups per scan launch), contract_splits (ranges per
 * column of contraction tiles) and one_hot_max (one-hot or scattered outer
 * codes) -- by coordinate descent from `opts`: each variant is planned,
 * prepared and timed over `runs` runs (HIP events on `stream`, graph replay
 * when opts->graph), and the fastest kept.  Results are cached in the JSON
 * file `cache_path` (created or updated; NULL: no cache) under a 64-bit
 * FNV-1a hash of the plan description with the base options, the relation
 * sizes and the device architecture: a cached entry is returned without any
 * timing.  On return `opts` holds the tuned values and *best_ms and
 * *base_ms (HOST, may be NULL) the step time of the tuned and the base
 * options (from the cache when cached).  `columns` as for lmfao_prepare. */
lmfao_status lmfao_tune(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                        lmfao_options* opts, const void* const* const* columns, const char* cache_path,
                        int32_t runs, double* best_ms, double* base_ms, void* stream);

/* Evaluates the whole batch: every view and query of the plan, level by
 * level, on `stream`.  Enqueue only: returns once the work is queued unless
 * `sync` is nonzero (then it synchronizes and checks key-uniqueness and
 * kernel error flags).  Results live in device buffers owned by `prep` and
 * are overwritten by the next lmfao_run on the same handle. */
lmfao_status lmfao_run(lmfao_plan_t plan, lmfao_prepared_t prep, void* stream, int32_t sync);

/* Result of query q of the caller's batch after a completed run, compacted
 * on the GPU (section 2: the output of the batch): the present groups
 * (count > 0) in lexicographic key order -- dense tables by a scan over their
 * cells, hash tables by a scan over their slots and a radix sort by key.
 * DEVICE arrays owned by `prep`: keys n_groups x n_keys int64 (row-major),
 * counts n_groups int64, values n_groups x n_aggs double.  They stay valid
 * until the next lmfao_run on `prep` (the next call after that compacts
 * again) or lmfao_prepared_free.  Reads the run's error flags first (any
 * kernel error is returned); synchronises `stream`. */
typedef struct {
  int64_t n_groups;
  int32_t n_keys, n_aggs;
  const int64_t* keys;
  const int64_t* counts;
  const double* values;
} lmfao_output;
lmfao_status lmfao_result_device(lmfao_prepared_t prep, int32_t q, lmfao_output* out, void* stream);

/* Result of query q after a completed run: number of present groups (groups
 * with at least one join tuple; lexicographic key order), number of group-by
 * attributes and aggregates. */
lmfao_status lmfao_result_shape(lmfao_prepared_t prep, int32_t q, int64_t* n_groups,
                                int32_t* n_keys, int32_t* n_aggs);

/* Copies query q's result (compacted on the GPU as lmfao_result_device) to
 * HOST buffers: keys (n_groups x n_keys int64, may be NULL), counts
 * (n_groups int64, may be NULL), values (n_groups x n_aggs double, may be
 * NULL).  Synchronizes the device. */
lmfao_status lmfao_result_copy(lmfao_prepared_t prep, int32_t q, int64_t* keys,
                               int64_t* counts, double* values);

/* Intermediate view v (plan description order) after a completed run: its
 * dense key domain size, value columns and code columns; and a copy to HOST
 * buffers: counts (n_keys int64), values (n_keys x n_vals double, converted
 * from the view's storage precision), codes (n_keys x n_codes int32).  Any
 * pointer may be NULL.  Synchronizes the device. */
lmfao_status lmfao_view_shape(lmfao_prepared_t prep, int32_t v, int64_t* n_keys, int32_t* n_vals,
                              int32_t* n_codes);
lmfao_status lmfao_view_copy(lmfao_prepared_t prep, int32_t v, int64_t* counts, double* values,
                             int32_t* codes);

/* Kernel timing.  While timing is on, every lmfao_run records HIP events on
 * its stream around the whole run and around each scan and contraction
 * launch.  lmfao_run_timing synchronizes the device and returns, for the runs
 * recorded since its previous call, the mean milliseconds of the whole run
 * (entry 0, name "run") and of each timed launch (entries 1..), filling up to
 * `cap` names/ms (names stay valid while `prep` lives) and the count in *n. */
lmfao_status lmfao_set_timing(lmfao_prepared_t prep, int32_t on);
lmfao_status lmfao_run_timing(lmfao_prepared_t prep, int32_t cap, const char** names,
                              float* ms, int32_t* n);

/* JSON description of the prepared launch sequence: per step its name, kind,
 * rows and pieces, and the algorithmic bytes read / written and arithmetic
 * (flop) the step must do at minimum (computed on the host from sizes), plus
 * the bytes zero-filled at the start of each run.  Same buffer convention as
 * lmfao_plan_describe. */
lmfao_status lmfao_prepared_describe(lmfao_prepared_t prep, char* buf, size_t cap, size_t* need);
/* Source of the i-th scan kernel generated for this prepared plan (section 2,
 * code generation layer: code specialised to one group's plan), first line the
 * group's name; the count is "generated_scans" in lmfao_prepared_describe.
 * Same buffer convention as lmfao_plan_describe; LMFAO_EINVAL for a bad i. */
lmfao_status lmfao_prepared_kernel_source(lmfao_prepared_t prep, int32_t i, char* buf, size_t cap, size_t* need);

/* Row weights of relation `rel` (lmfao_options.row_weights): *weights
 * receives the DEVICE address of its n_rows int32 weights, in the caller's
 * row order, owned by `prep` (valid until lmfao_prepared_free).  Writes
 * between runs take effect at the next lmfao_run, graph replays included;
 * a weight other than 0 or 1 counts as 1.  LMFAO_EINVAL if the relation
 * was not given row weights. */
lmfao_status lmfao_row_weights(lmfao_prepared_t prep, int32_t rel, int32_t** weights);

/* A conjunction of conditions evaluated per row on the GPU:
 * out[r] = 1 if for every k, column_k[r] op_k constant_k, else 0 (out[r] = 1
 * for every row when n_conds == 0).  Columns and `out` are DEVICE arrays of
 * n_rows values; a constant is compared in its column's type (an F32
 * column's constant is rounded to float first), as lmfao_plan does.  At most
 * 8 conditions; enqueued on `stream`, not synchronised.  LMFAO_EINVAL for a
 * bad op, dtype, count or NULL pointer. */
typedef struct {
  const void* column;   /* DEVICE column */
  int32_t dtype;        /* LMFAO_I32 / LMFAO_F32 / LMFAO_F64 */
  int32_t op;           /* LMFAO_LE ... LMFAO_NE */
  double constant;
} lmfao_column_condition;
lmfao_status lmfao_eval_conditions(int64_t n_rows, int32_t n_conds, const lmfao_column_condition* conds,
                                   int32_t* out, void* stream);

/* CART split selection and tree growth (paper, section 3, "Decision Trees").
 * A node is the bag of tuples of D that satisfy its path condition.  A
 * candidate is a condition on one attribute -- LMFAO_CART_LE: attr <= value,
 * LMFAO_CART_EQ: attr == value -- whose left branch T holds the node's
 * tuples where it is true, the right branch the rest (attr > value,
 * attr != value).  Its cost is VAR(T) + VAR(node \ T), with
 * VAR(B) = SUM(y^2) - SUM(y)^2 / |B| (0 for an empty branch), FP64.  It is
 * valid when both branches hold at least min_leaf tuples; among valid
 * candidates the least cost wins, and candidates whose cost lies within
 * tie_eps * max(|VAR(node)|, 1) of the least are tied: the first one in the
 * candidate list wins (list candidates by attribute, then value).
 * The statistics come from the batch's own results: `query` of a candidate
 * is a query of the caller's batch whose aggregates 0, 1, 2 are SUM(1),
 * SUM(y), SUM(y*y) over the tuples where the candidate holds (LE: a query
 * with the condition and no group-by, `group` 0; EQ: a query grouped by the
 * attribute alone, `group` its code), and `total_query` is such a query with
 * no condition and no group-by. */
enum { LMFAO_CART_LE = 0, LMFAO_CART_EQ = 1 };
typedef struct {
  const char* attr;
  int32_t kind;     /* LMFAO_CART_LE or LMFAO_CART_EQ */
  double value;
  int32_t query;
  int64_t group;
} lmfao_cart_candidate;
typedef struct {
  int32_t n_candidates;
  const lmfao_cart_candidate* candidates;   /* HOST array, in tie-break order */
  int32_t total_query;
  int32_t max_depth;   /* lmfao_cart_grow: nodes at this depth are leaves (at most 8) */
  int64_t min_leaf;
  double tie_eps;
} lmfao_cart_spec;
typedef struct {
  int32_t best;     /* chosen candidate, -1 if none is valid */
  int32_t pad;
  int64_t n, n_left, n_right;
  double sum_y, sum_y2, sum_y_left, sum_y2_left;
  double cost;      /* VAR(left) + VAR(right) of the chosen split (VAR(node) if none) */
} lmfao_cart_split;
typedef struct {
  int32_t parent, depth;
  int32_t split;        /* candidate index, -1 for a leaf */
  int32_t left, right;  /* children (left: the candidate holds), -1 for a leaf */
  int32_t pad;
  int64_t n;            /* tuples of D in the node */
  double sum_y, sum_y2;
  double cost;          /* the split's cost, or VAR(node) for a leaf */
} lmfao_cart_node;

/* The best split of the node the last lmfao_run of `prep` evaluated, chosen
 * on the GPU from the device results (one workgroup); `out` is HOST, `costs`
 * a DEVICE array of n_candidates doubles receiving every candidate's cost
 * (+inf if invalid), or NULL.  Synchronises `stream`.  LMFAO_EINVAL for a
 * query index, group row or aggregate layout that does not match the
 * description above (aggregates 0, 1, 2 must be SUM(1), SUM(y), SUM(y*y) of
 * one y). */
lmfao_status lmfao_cart_best_split(lmfao_prepared_t prep, const lmfao_cart_spec* spec, lmfao_cart_split* out,
                                   double* costs, void* stream);

/* Grows the tree breadth first from the whole of D: for every node above
 * max_depth it writes the node's path condition into the row weights of the
 * relations holding the path's attributes (evaluated on the GPU over
 * `columns`, the caller's DEVICE columns as given to lmfao_prepare, which
 * must still be valid), runs the batch (a graph replay when the plan was
 * captured) and selects the split on the GPU; nodes at max_depth take their
 * statistics from their parent's split.  Node 0 is the root, children follow
 * in breadth-first order, left before right.  Every attribute a candidate
 * names must be held by a relation with row weights.  `nodes` is a HOST
 * array of `cap` entries (2^(max_depth+1) - 1 suffice); *n_nodes receives the
 * count.  Errors of the runs (kernel flags) are returned. */
lmfao_status lmfao_cart_grow(lmfao_plan_t plan, lmfao_prepared_t prep, const void* const* const* columns,
                             const lmfao_cart_spec* spec, lmfao_cart_node* nodes, int32_t cap, int32_t* n_nodes,
                             void* stream);

/* Rk-means (paper, section 3, "Rk-means").  Step 1 is a batch of
 * SUM(1) GROUP BY X_j queries (lmfao_run); their device results
 * (lmfao_result_device: ascending codes and counts) are step 2's input.
 *
 * lmfao_kmeans_1d, step 2: weighted k-means on every projection.  Set s is
 * the ascending integer values values[offsets[s] .. offsets[s+1]) with
 * integer weights (DEVICE int64 arrays; offsets is HOST, n_sets + 1
 * entries).  Lloyd's algorithm in FP64, one workgroup per set: centroid i
 * (0 <= i < k) starts at the first value whose cumulative weight reaches
 * (2i + 1) / (2k) of the set's total; then every value is assigned to its
 * nearest centroid (the lowest index on a tie) and every centroid moved to
 * the weighted mean of its values (a centroid with none stays), until an
 * assignment step changes nothing or after max_iter update steps.  With
 * integer values and weights every sum is exact below 2^53, so the result
 * does not depend on the order of the additions.  Writes centroids (DEVICE,
 * n_sets x k doubles), the cluster of every value (DEVICE int32, aligned
 * with `values`) and, if not NULL, the update steps per set (HOST).
 * 1 <= k <= 64.  Synchronises `stream`.
 *
 * lmfao_grid_coreset, step 3: SELECT C_1, ..., C_n, SUM(1) FROM D JOIN
 * A_1(X_1, C_1) ... JOIN A_n(X_n, C_n) GROUP BY C_1, ..., C_n, where dims[j]
 * gives A_j as the ascending codes of X_j and their clusters (DEVICE
 * arrays, n_codes each; values of X_j not listed map to cluster 0).  The
 * join must be one whose tuples a root row determines: every other relation
 * is reached from the root through one integer key attribute (FK chains and
 * stars; LMFAO_EUNSUPPORTED otherwise).  On the GPU: each root row's cluster
 * ids are packed (a power of two of bits each, at most 512 bits in all) and
 * counted by a 64-bit fingerprint in a hash table; a second pass compares
 * every row's packed ids with its group's representative, and a fingerprint
 * shared by two different id vectors gives LMFAO_EUNSUPPORTED instead of a
 * merged group.  `out` receives the groups in no particular order: keys
 * n_groups x n int64 cluster ids, counts their weights, no values (DEVICE
 * arrays owned by `prep`).  `columns` as for lmfao_prepare (still valid).
 * Synchronises `stream`. */
lmfao_status lmfao_kmeans_1d(int32_t n_sets, const int64_t* offsets, const int64_t* values, const int64_t* weights,
                             int32_t k, int32_t max_iter, double* centroids, int32_t* assignment, int32_t* steps,
                             void* stream);
typedef struct {
  const char* attr;
  const int64_t* codes;     /* DEVICE, ascending */
  const int32_t* cluster;   /* DEVICE, the cluster (0 .. k-1) of each code */
  int64_t n_codes;
} lmfao_grid_dim;
lmfao_status lmfao_grid_coreset(lmfao_plan_t plan, lmfao_prepared_t prep, const void* const* const* columns,
                                int32_t n_dims, const lmfao_grid_dim* dims, int32_t k, lmfao_output* out,
                                void* stream);

/* Ridge linear regression over the batch's results (paper, section 3,
 * "Linear Regression"): x = (1, continuous..., one-hot blocks of the
 * categoricals over their whole domains); Sigma = sum over D of x x^T.
 *
 * lmfao_ridge_sigma assembles Sigma (dim x dim, row-major FP64, DEVICE
 * buffer `sigma` owned by the caller) from the results of the last lmfao_run
 * of `prep`: SUM(x_j*x_k) queries (intercept = SUM of the other factor or
 * COUNT), per-categorical group-by sums and counts, and categorical-pair
 * counts -- the queries of the covariance batch.  A query with a range
 * condition of its own is not used.  With sigma == NULL only *dim_out is set
 * (dim = 1 + n_cont + sum of the categorical domains, at most 2048).
 * LMFAO_EINVAL if an attribute is unknown or the batch lacks an entry.
 * Enqueued on `stream` and synchronised before returning.
 *
 * lmfao_ridge_bgd runs batch gradient descent on the free parameters (every
 * index except `label`, whose parameter is fixed at -1):
 *     theta_F <- theta_F - eta * (Sigma theta / |D| + lambda theta)_F,
 * |D| = Sigma[0][0], theta starting at 0; it stops when ||grad_F||_2 <= tol
 * or after max_iter steps.  eta <= 0 selects eta = 1/L, L the largest
 * eigenvalue of Sigma_FF/|D| + lambda I by 100 power-iteration steps from the
 * all-ones vector.  `sigma` and `theta` (dim doubles, written) are DEVICE
 * pointers; `stats` is a HOST array of 3 doubles receiving {steps, final
 * ||grad_F||, eta}.  All FP64, one workgroup, synchronised before return. */
lmfao_status lmfao_ridge_sigma(lmfao_prepared_t prep, int32_t n_cont, const char* const* cont, int32_t n_cat,
                               const char* const* cat, double* sigma, int32_t* dim_out, void* stream);
lmfao_status lmfao_ridge_bgd(const double* sigma, int32_t dim, int32_t label, double lambda, double eta,
                             int32_t max_iter, double tol, double* theta, double* stats, void* stream);

/* Estimator features (layout above) of query q of the caller's batch as
 * prepared (distinct counts are counted on the GPU on first use, on the
 * prepared stream, which is synchronised).  `feats` is a HOST array of
 * LMFAO_EST_FEATURES floats.  LMFAO_EINVAL for a bad q or a query without
 * group-by attributes. */
lmfao_status lmfao_prepared_features(lmfao_prepared_t prep, int32_t q, float* feats);

/* Group-count estimator (not part of the paper's method; it sizes the hash
 * tables of outputs whose dense key space is too large, with overflow
 * regrowth as the exact fallback).  A perceptron x (d features) ->
 * relu(x W1 + b1) (h) -> relu(. W2 + b2) (h) -> . w3 + b3, in FP32, trained on
 * the mean squared error with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * `params` is one flat FP32 array of lmfao_mlp_size(d, h) values in the order
 * W1 (d x h, row-major), b1, W2 (h x h, row-major), b2, w3, b3.  X (n x d,
 * row-major FP32), t (n FP32 targets), params, grad, y and order are DEVICE
 * pointers owned by the caller; `loss` and `loss_trace` are HOST pointers
 * (may be NULL).  Each call allocates its own scratch, runs on `stream` and
 * synchronises before returning.  LMFAO_EINVAL for non-positive sizes or a
 * NULL required pointer, LMFAO_ENOMEM if scratch cannot be allocated.
 *
 * lmfao_mlp_grad: gradient of the batch's mean squared error (written to
 * grad, same layout as params) and the loss.
 * lmfao_mlp_predict: y = network(X).
 * lmfao_mlp_train: n_steps Adam steps at learning rate lr; step s uses the
 * rows order[s*batch .. s*batch+batch) of X and t (int32 indices below n,
 * n_steps*batch of them, drawn by the caller; an index outside [0, n) gives
 * LMFAO_EINVAL before any step); loss_trace[s] receives the
 * mean squared error of step s's batch before its update. */
lmfao_status lmfao_mlp_size(int32_t d, int32_t h, int64_t* n_params);
lmfao_status lmfao_mlp_grad(int32_t d, int32_t h, const float* params, const float* X, const float* t, int32_t n,
                            float* grad, float* loss, void* stream);
lmfao_status lmfao_mlp_predict(int32_t d, int32_t h, const float* params, const float* X, int32_t n, float* y,
                               void* stream);

/* lmfao_mlp_grad_noalloc: lmfao_mlp_grad for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same kernels and the same gradient;
 * the loss is summed in FP64 on the device.  It calls no hipMalloc, hipFree or
 * allocating library routine: its scratch (the batch's activations and
 * errors) is one fixed array of 8 MiB per GPU, held by the library for the
 * life of the process, so the batch must satisfy 6*n*h + 3*n + 64 <= 2^21
 * (e.g. n <= 5,400 rows at h = 64); larger batches return LMFAO_EINVAL with
 * the limit in lmfao_last_error() before any work is enqueued.  Every call on
 * one GPU shares that array, so calls that overlap on one GPU (from several
 * host threads, or on streams that run concurrently) race; each call
 * synchronises `stream` before returning. */
lmfao_status lmfao_mlp_grad_noalloc(int32_t d, int32_t h, const float* params, const float* X, const float* t,
                                    int32_t n, float* grad, float* loss, void* stream);
lmfao_status lmfao_mlp_train(int32_t d, int32_t h, float* params, const float* X, const float* t, int32_t n,
                             const int32_t* order, int32_t n_steps, int32_t batch, float lr, float* loss_trace,
                             void* stream);

void lmfao_plan_free(lmfao_plan_t plan);
void lmfao_prepared_free(lmfao_prepared_t prep);

/* Thread-local text of the last error (empty string if none). */
const char* lmfao_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LMFAO_H */
