// Internal structures of the aggregate-batch engine: the logical plan (views,
// groups), the per-group factorized programs, and the device descriptors the
// kernels read.  Host code and HIP kernels of the same shared library include
// this header; nothing outside the library does.
#pragma once

#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "lmfao.h"

namespace lmfao {

// ---------------------------------------------------------------------------
// limits of the device descriptors
// ---------------------------------------------------------------------------
constexpr int kMaxScanCols = 16;   // sorted columns a scan reads per tuple
constexpr int kMaxPieceCols = 64;  // per-piece columns of a contraction
constexpr int kMaxOuterAtoms = 64;
constexpr int kMaxOuterCodes = 64;
constexpr int kMaxViews = 8;       // views one kernel looks up
constexpr int kMaxInnerViews = 4;  // views the scan looks up per tuple
constexpr int kMaxWeights = 16;    // weights pre-aggregated over runs (registers)
constexpr int kMaxWeightTable = 64;  // distinct histogram / table weights of a scan
constexpr int kMaxKey = 4;         // attributes of one view key
constexpr int kMaxAtoms = 8;       // inner factors of the fast scan
constexpr int kMaxMasks = 4;       // distinct multiplicity masks in a scan
constexpr int kMaxCodes = 16;      // inner codes of a scan
constexpr int kMaxHists = 64;      // per-piece histograms in a scan
constexpr int kMaxTables = 8;      // direct group-by tables written by a scan
constexpr int kMaxTableComps = 8;
constexpr int kOneHotMax = 64;     // largest code domain expanded one-hot
constexpr int kOneHotPure = 16;    // ... for outputs keyed by outer codes only, once a
                                   // group's one-hot features exceed the budget below
constexpr int kOneHotFeatureBudget = 256;
constexpr int kHistMax = 1024;     // largest code domain kept per piece
constexpr int kScanWaves = 8;      // wavefronts per scan block (each holds its own histograms)
constexpr int kLdsBytes = 160 * 1024;            // LDS of one compute unit
constexpr int64_t kLdsTableMax = 12288;          // int32 count entries privatized in LDS
constexpr int64_t kPartMinCells = 1;             // smallest SUM(1) table moved from a scan to the partition count
                                                 // when the scan's LDS tables overflow
constexpr int64_t kPartSmallCells = 64;          // larger SUM(1) tables are counted by the partition count...
constexpr int64_t kPartScanCells = 2048;         // ...except, on relations of kPartLargeRows rows or more,
constexpr int64_t kPartLargeRows = (int64_t)1 << 24;  // tables of up to kPartScanCells cells
constexpr int kTriangle = (kMaxAtoms + 1) * (kMaxAtoms + 2) / 2;  // incl. (1,1)
constexpr int64_t kDenseRowsMax = (int64_t)1 << 24;  // larger key spaces go to hash tables
constexpr int64_t kPickMinCells = (int64_t)1 << 15;  // smaller tables stay dense (one LDS slice)
constexpr double kDenseDensityMin = 8.0;             // learned sizing hashes tables predicted sparser than 1/8

// ---------------------------------------------------------------------------
// logical plan
// ---------------------------------------------------------------------------
using Mono = std::vector<int>;  // sorted attribute ids, a power-2 factor appears twice

struct AttrDef {
  std::string name;
  int dtype = LMFAO_I32;
  int64_t domain = 0;
};

struct RelDef {
  std::string name;
  int64_t n_rows = 0;
  int n_input_attrs = 0;           // columns the caller passes; derived columns follow
  std::vector<int> attrs;          // global attribute ids, schema order
  std::vector<int> dtypes;
  std::vector<char> is_key;
  std::map<int, int> col;          // attribute id -> column index
  bool has(int a) const { return col.count(a) != 0; }
};

struct Cond {
  int attr = -1;
  int op = 0;
  double c = 0;
  bool operator<(const Cond& o) const {
    return std::tie(attr, op, c) < std::tie(o.attr, o.op, o.c);
  }
  bool operator==(const Cond& o) const { return attr == o.attr && op == o.op && c == o.c; }
};

struct QueryDef {
  std::vector<int> groupby;        // attribute ids, as given
  std::vector<Cond> conds;
  std::vector<Mono> aggs;
  int root = -1;
  int level = 0;
  int group = -1;
  std::map<int, int> in_view;      // neighbour relation -> view id (views into root)
};

struct ViewDef {
  int id = -1;
  int from = -1, to = -1;          // V_{from -> to}
  std::vector<int> key;            // join attributes of the edge, sorted
  std::vector<int> carried;        // group-by attributes carried from the subtree
  std::vector<Cond> conds;         // pushed conditions
  std::set<Mono> comps;            // non-empty component monomials
  bool unique = false;             // at most one subtree join tuple per key value
  std::set<int> deps;              // views into `from` it is computed from
  int level = 0;
  int group = -1;
  // physical layout (filled by the physical planner)
  std::vector<int> val_attrs;      // unique views: attribute values stored
  std::vector<Mono> val_monos;     // non-unique views: monomials stored
  std::vector<int> code_attrs;     // unique views: carried codes stored
  int64_t n_keys = 0;              // dense key domain (product of key domains)
  bool vals_f64 = true;
  int slot_of_attr(int a) const {
    for (size_t i = 0; i < val_attrs.size(); ++i) if (val_attrs[i] == a) return (int)i;
    return -1;
  }
  int slot_of_mono(const Mono& m) const {
    for (size_t i = 0; i < val_monos.size(); ++i) if (val_monos[i] == m) return (int)i;
    return -1;
  }
  int slot_of_code(int a) const {
    for (size_t i = 0; i < code_attrs.size(); ++i) if (code_attrs[i] == a) return (int)i;
    return -1;
  }
};

// An output computed by a group: a query (results) or a non-unique view.
struct OutRef {
  int kind;  // 0 query, 1 view
  int id;
};

// ---------------------------------------------------------------------------
// factorized program of one group (host form)
// ---------------------------------------------------------------------------
enum SrcKind { SRC_COL = 0, SRC_VIEW = 1 };

struct AtomRef {   // a factor value: a column (power folded by repetition) or a view slot
  int kind;        // SRC_COL (column of the scanned relation / piece key) or SRC_VIEW
  int src;         // column index or view index (into the program's view list)
  int slot;        // view val slot
  bool operator<(const AtomRef& o) const { return std::tie(kind, src, slot) < std::tie(o.kind, o.src, o.slot); }
  bool operator==(const AtomRef& o) const { return kind == o.kind && src == o.src && slot == o.slot; }
};
using CodeRef = AtomRef;   // slot = code slot for views

// A-feature: mu_out(mask) * [code c1 == v1] * [code c2 == v2] * atom a1 * atom a2
struct FeatDef {
  uint32_t mask = 0;
  int c1 = -1, v1 = 0, c2 = -1, v2 = 0;
  int a1 = -1, a2 = -1;
  bool operator<(const FeatDef& o) const {
    return std::tie(mask, c1, v1, c2, v2, a1, a2) < std::tie(o.mask, o.c1, o.v1, o.c2, o.v2, o.a1, o.a2);
  }
  bool is_int() const { return a1 < 0 && a2 < 0; }
};

// B-column: either a psi entry (float entry / int entry, with bin), or
// psi count(mask) times a feature (mask of the feature is unused).
enum BKind { B_PSI_F = 0, B_PSI_I = 1, B_CNTF = 2 };
struct ColDef {
  int kind = B_PSI_I;
  int entry = 0;      // psi float entry / psi int entry (count or count-hist) index
  int bin = 0;        // histogram bin (0 for plain entries)
  FeatDef feat;       // B_CNTF: the feature multiplied by the count entry
  bool operator<(const ColDef& o) const {
    return std::tie(kind, entry, bin, feat) < std::tie(o.kind, o.entry, o.bin, o.feat);
  }
  bool is_int() const { return kind == B_PSI_I || (kind == B_CNTF && feat.is_int()); }
};

// where a merged cell lands
struct CellDst {
  int out;            // index into program outputs
  int64_t row;        // key row
  int comp;           // -1 count, else value column
};

struct ScatterCell {  // evaluated per piece and added at row(piece)
  int out;
  int comp;           // -1 count
  int f, g;           // feature index, column index (into the program lists)
};

struct TableComp {    // table output component: mu(mask) * a_i * a_j  (atoms inner; -1 = 1)
  int comp;           // -1 count
  int ai = -1, aj = -1;
  uint32_t imask = 0;
};

struct ProgOutput {
  OutRef ref;
  int mode;               // 0 GEMM, 1 SCATTER, 2 TABLE
  int64_t n_rows = 1;     // dense key rows
  int n_comps = 0;        // value columns (excluding count)
  std::vector<int> key_codes;         // code refs (outer for scatter, inner for table)
  std::vector<int> key_codes_outer;   // parallel flag
  std::vector<int64_t> key_stride;
  uint32_t omask = 0;                 // table mode: outer mask
  std::vector<TableComp> tcomps;      // table mode
  bool dst_is_view = false;           // writes vals as view table (f32/f64 by view)
  bool hashed = false;                // scatter mode into a hash table (key space > kDenseRowsMax)
  std::vector<int> count_copies;      // scatter mode: SUM(1) components, equal to the count
};

struct PsiEntryF {
  int ai, aj;          // extended atom indices (-1 = 1), ai <= aj
  uint32_t imask;
};
struct HistDef {
  int code;            // inner code index
  int dom;
  int is_float;        // 0 count histogram, 1 weighted by atom ai*aj
  int ai = -1, aj = -1;
  uint32_t imask;
  int offset;          // first bin in the piece's int or float histogram block
};

struct GroupProgram {
  int node = -1;
  int cut = 0;                    // attribute-order level; L+1 = row pieces
  bool row_pieces = false;        // pieces are the relation's rows (no scan)
  std::vector<int> order;         // node attribute order (attribute ids)
  std::vector<int> views;         // incoming view ids used (program view index -> view id)
  std::vector<int> view_outer;    // per program view: 1 outer (per piece), 0 inner (per tuple)
  std::vector<int> view_level;
  // scan side (inner)
  std::vector<int> scan_cols;     // column indices of the node relation read per tuple
  std::vector<AtomRef> in_atoms;  // src = scan column position / view index
  std::vector<CodeRef> in_codes;
  std::vector<uint32_t> in_masks; // distinct inner masks (bitset over program views)
  std::vector<PsiEntryF> psi_f;   // float entries
  std::vector<uint32_t> psi_i;    // count entries: mask per entry
  std::vector<HistDef> hists;
  int hist_f_bins = 0, hist_i_bins = 0;
  // contract side (outer)
  std::vector<int> piece_cols;    // row pieces: relation columns; cut pieces: order positions
  std::vector<AtomRef> out_atoms; // src = piece column position / view index
  std::vector<CodeRef> out_codes;
  std::vector<FeatDef> feats;
  std::vector<ColDef> cols;
  int n_feat_int = 0, n_col_int = 0;   // int features / columns come first
  // outputs
  std::vector<ProgOutput> outs;
  std::vector<std::pair<std::pair<int, int>, CellDst>> gemm_cells;  // ((f,g), dst)
  std::vector<ScatterCell> scatter;
  bool needs_mu_out_in_scan = false;   // table outputs with outer multiplicities
  uint32_t tables_outer_mask = 0;
  std::string describe;
};

struct GroupDef {
  int node = -1;
  int level = 0;
  std::vector<OutRef> outs;       // all outputs (queries and views)
  std::vector<int> unique_views;  // views built directly (unique on their key)
  std::set<int> deps;             // groups this one depends on
  bool has_program = false;
  bool force_rows = false;        // evaluated row by row (an output has no scan form)
  bool partitioned = false;       // SUM(1) queries with large dense tables, counted by
                                  // radix partition (no program)
  int one_hot_pure = 0;           // one-hot limit of outer-only outputs (0 = kOneHotMax)
  GroupProgram prog;
};

// A bucket code derived from attribute `src` of relation `rel`: the number of
// thresholds below the value (kind 0: t < x, for x <= t and x > t) or at most
// the value (kind 1: t <= x, for x < t and x >= t).  Thresholds are rounded to
// the attribute's comparison type (FP32 columns compare in FP32) and sorted.
struct DerivedAttr {
  int attr = -1, src = -1, rel = -1, kind = 0;   // kind 0, 1: bucket codes (<= / < thresholds); 2: function
  std::vector<double> thr;                        // thresholds, or the function's values per source value
};

// A query of the caller's batch: either one planned query, or the sum over a
// range of bucket (or code) values of a planned query that groups by them too.
struct UserQuery {
  int internal = -1;
  bool range = false;
  int64_t lo = 0, hi = 0, ex = -1;   // buckets [lo, hi) except ex
  int64_t nb = 1;                    // bucket domain (last key of the planned query)
};

struct Plan {
  std::vector<AttrDef> attrs;
  std::map<std::string, int> attr_id;
  std::vector<RelDef> rels;
  std::vector<std::pair<int, int>> edges;
  std::vector<std::vector<int>> adj;
  std::vector<QueryDef> queries;
  std::vector<ViewDef> views;
  std::vector<GroupDef> groups;
  std::vector<std::vector<int>> order;   // attribute order per relation
  std::vector<Cond> filter;              // conditions every planned query shares
  std::vector<DerivedAttr> derived;
  std::vector<UserQuery> user;           // caller's queries, in batch order
  int n_levels = 0;
  lmfao_options opts;
  std::vector<float> estimator;          // copy of the estimator blob (empty = none)
  bool supported = true;
  std::string unsupported_reason;
  std::vector<std::vector<char>> uniq;   // uniq[n][p]: V_{n->p} unique (adjacency)
  std::string json;
  double root_cost = 0;            // root cost model of the final root assignment (bytes)
  std::string root_fallback;       // ROOT_COST fell back to the FACT roots: why
};

// builds the logical and physical plan; throws PlanError on invalid input
struct PlanError {
  int status;
  std::string msg;
};
Plan* build_plan(const lmfao_schema* schema, const lmfao_join_tree* tree,
                 const lmfao_batch* batch, const lmfao_options* opts);

// sets (clears) the thread-local text lmfao_last_error() returns
void record_error(const std::string& msg);
void clear_error();

std::vector<int> join_attrs(const Plan& P, int a, int b);

// ---------------------------------------------------------------------------
// device descriptors (plain data, copied to device memory per launch set)
// ---------------------------------------------------------------------------
struct DCol {
  const void* ptr;
  int32_t dtype;   // LMFAO_I32 / F32 / F64
  int32_t pad;
};

struct DView {
  const int64_t* cnt;
  const void* vals;
  const int32_t* codes;
  int32_t vals_f64;
  int32_t n_vals;
  int32_t n_codes;
  int32_t nkey;
  int32_t key_src[kMaxKey];     // column positions (scan columns or piece columns)
  int64_t key_stride[kMaxKey];
  int64_t n_keys;
};

struct DAtom {
  int32_t kind, src, slot, pad;
};

struct DHist {
  int32_t code, dom, is_float, wi, offset, pad;   // wi: weight index
};

struct DWeight {   // per-tuple weight mu(mask) [* a_i * a_j for float weights]
  int32_t is_float, ai, aj, mask_idx;
};

struct DTable {
  int32_t ncode;
  int32_t code[3];
  int64_t stride[3];
  int64_t n_rows;
  int32_t n_tcomps;
  int32_t tcomp[kMaxTableComps];   // -1 count, else value column
  int32_t twi[kMaxTableComps];     // weight index of each component
  int64_t* cnt;                 // destination counts (int64)
  void* vals;                   // destination values
  int32_t vals_f64;
  int32_t n_vals;               // destination value columns
  int32_t lds;                  // counts privatized in LDS (block partials)
  int32_t lds_off;              // offset of the count table in the block's LDS area
};

// packed per-key image of an inner view for one scan: the scan's factor
// slots (T each), then its code slots and the view count (int32 each),
// padded to 16 bytes; slots of factors / codes from elsewhere hold zero
struct DImage {
  const DView* view_dev;   // unused on the device; host bookkeeping
  void* img;               // [n_keys x width_dw] dwords
  int32_t width_dw;        // dwords per key row (multiple of 4)
  int32_t code_off;        // first code dword
  int32_t cnt_off;         // count dword
  int32_t key_col;         // scan column of the (single-attribute) key, -1 = composite
};

struct DImageBuild {
  DView view;              // source view
  void* img;
  int64_t n_keys;
  int32_t width_dw, code_off, cnt_off, t_f64;
  int32_t n_atoms;
  int32_t atom_slot[kMaxAtoms];   // view value slot per scan factor (-1: not from this view)
  int32_t n_codes;
  int32_t code_slot[kMaxCodes];   // view code slot per scan code (-1: not from this view)
};

constexpr int kFastHists = 32;
constexpr int kFastTables = 4;
constexpr int kGenTables = 8;     // direct tables of a generated scan

// hoisted form of a lean scan (all loop-invariant, read once per kernel)
struct DFast {
  const void* fcol[kMaxAtoms];     // factor columns in the compute type (null: factor from an image)
  const int32_t* ccol[kMaxCodes];  // code columns (null: code from an image)
  const void* img[2];              // inner view images (null: no view)
  const int32_t* kcol[2][2];       // key columns of each image (second: null for one-attribute keys)
  int32_t kmul[2][2];              // dense key = sum of key column * kmul
  int32_t n_hist;
  uint32_t hword[kFastHists];      // code(2) | mask(2) | float(1) | ai+1(4) | aj+1(4) | offset(16)
  int8_t hcode[kFastHists];        // full code index (the generated scans allow 16 codes)
  int32_t n_tab;
  int32_t tab_ncode[kGenTables];
  int32_t tab_code[kGenTables][3];
  int32_t tab_stride[kGenTables][3];
  int32_t tab_mask[kGenTables];    // count weight mask
  int32_t tab_lds[kGenTables];     // 1: LDS offset valid, else global counts
  int32_t tab_off[kGenTables];
  int64_t* tab_cnt[kGenTables];
  // generated scans: value components of a table, added to FP64 outputs
  int32_t tab_has_cnt[kGenTables];
  int32_t tab_nvc[kGenTables];
  int32_t tab_vcomp[kGenTables][kMaxTableComps];
  int32_t tab_vw[kGenTables][kMaxTableComps];   // (ai + 1) | (aj + 1) << 4 | mask << 8
  double* tab_vals[kGenTables];
  int32_t tab_nv[kGenTables];
  int32_t reg_hist_bins;           // generated scans: histograms this small live in registers
  int32_t mult01;                  // generated scans: every row's multiplicity is 0 or 1 (the inner
                                   // views are single-valued), so integer register histograms may
                                   // keep their bins as 8-bit fields of 64-bit words
};

struct DScan {
  const int32_t* w;                // filter weight per sorted row (null: no filter)
  int32_t fast;                    // lean kernel: images, <= 4 codes, direct atomics
  DFast F;
  DImage imgs[kMaxInnerViews];
  int32_t n_cols;
  DCol cols[kMaxScanCols];
  int32_t n_views;
  DView views[kMaxInnerViews];
  int32_t n_masks;
  uint32_t masks[kMaxMasks];
  int32_t n_atoms;
  DAtom atoms[kMaxAtoms];
  int32_t n_codes;
  DAtom codes[kMaxCodes];
  int32_t n_weights;
  DWeight weights[kMaxWeightTable];
  uint32_t run_codes;          // codes that key histograms / tables (run detection)
  // float entries over the extended-atom upper triangle: index t(i,j), i<=j in [0,NA]
  uint64_t pf_need;            // bit t set if the triangle entry is accumulated
  int32_t pf_mask_idx;         // mask of every float entry when pf_uniform
  int32_t pf_uniform;          // 1: all float entries share pf_mask_idx
  int8_t pf_mask[kTriangle];   // per triangle entry mask index otherwise
  int32_t pf_n;                // number of accumulated float entries
  int32_t pf_slot[kTriangle];  // triangle index -> output slot in psi_f row (-1 unused)
  int32_t n_pi;                // count entries (one per mask)
  int32_t pi_mask_idx[kMaxMasks];
  int32_t n_hists;
  DHist hists[kMaxHists];
  int32_t hist_i_bins, hist_f_bins;
  int32_t n_tables;
  DTable tables[kMaxTables];
  int32_t lds_tab_i;               // LDS count-table elements per block
  // outer multiplicity for tables (per piece)
  int32_t mu_out_views;            // number of outer views checked for tables
  DView outer_views[kMaxViews];    // key_src = piece key column positions
  const int32_t* piece_key;        // [n_piece_key x n_pieces] (column-major)
  int32_t n_piece_key;
  int64_t n_pieces;
  // pieces
  const int64_t* piece_begin;      // [n_pieces + 1] row offsets
  const int32_t* item_piece;       // [n_items + 1] first piece of each work item
  int32_t n_items;
  int32_t psi_f_stride, psi_i_stride;   // per piece
  void* psi_f;                     // [n_pieces x psi_f_stride] (T)
  int32_t* psi_i;                  // [n_pieces x psi_i_stride]
  int32_t* part_i;                 // LDS table partials [grid x lds_tab_i]
  int32_t* err_flag;
};

struct DFeat {
  int32_t mask_idx, c1, v1, c2, v2, a1, a2, pad;
};
struct DColB {
  int32_t kind, entry, bin, pad;
  DFeat feat;
};

// open-addressing hash table of one output whose key space is too large to
// be dense: keys hold row + 1 (0 = empty), counts and values per slot
struct DHashOut {
  unsigned long long* keys;
  int64_t* cnt;
  double* vals;                    // [cap x n_vals]
  int64_t mask;                    // capacity - 1 (power of two)
  int32_t* ovf;                    // set when an insert found no slot
  int32_t n_vals, pad;
  uint32_t* used;                  // tables written by the partition count: the groups each region
                                   // received at the last run (its slots past them are zero); else null
};

struct DContract {
  const int32_t* w;                // row pieces: filter weight per row (null: no filter)
  int64_t n_pieces;
  int32_t n_pcols;
  DCol pcols[kMaxPieceCols];       // per-piece columns
  int32_t n_views;
  DView views[kMaxViews];          // outer views (key_src = piece column positions)
  int32_t n_masks;
  uint32_t masks[kMaxMasks * 4];
  int32_t n_atoms;
  DAtom atoms[kMaxOuterAtoms];
  int32_t n_codes;
  DAtom codes[kMaxOuterCodes];
  int32_t n_feat, n_feat_int;
  const DFeat* feats;              // device array
  int32_t n_col, n_col_int;
  const DColB* cols;
  // psi inputs (null for row pieces: count = 1)
  const void* psi_f;
  const int32_t* psi_i;
  int32_t psi_f_stride, psi_i_stride;
  int32_t row_pieces;
  int32_t* err_flag;               // code 4: an integer feature reached 2^53 (matrix-core path)
  // outputs: partial GEMM blocks
  double* part_f;                  // [n_blocks x n_feat x n_col] f64 (T accumulated, stored f64)
  int64_t* part_i;                 // [n_blocks x n_feat_int x n_col_int]
  int32_t pieces_per_block;
  // scatter cells
  int32_t n_scatter;
  const int32_t* sc_out;           // per scatter cell
  const int32_t* sc_comp;
  const int32_t* sc_f;
  const int32_t* sc_g;
  // per output (scatter targets)
  const int64_t* so_stride;        // [n_outs x 3]
  const int32_t* so_code;          // [n_outs x 3] outer code index (-1 none)
  const int32_t* so_ncomp;         // value columns
  int64_t* const* so_cnt;
  void* const* so_vals;            // f64 (or view dtype)
  const int32_t* so_vals_f64;
  const int32_t* so_hash_idx;      // per output: hash table index, -1 dense
  const DHashOut* hash_tab;        // hash tables of the prepared plan
};

// split-K shape of the matrix-core contraction:
// part[b][f * ng + g] = sum over the pieces of block b of F[p][f] * B[p][g]
struct DGemm {
  int64_t n;                       // pieces (K)
  int32_t nf, ng;
  int64_t k_per_block;             // multiple of the LDS chunk
  double* part;                    // [gridDim.x][nf * ng], block-major
};

// gemm cell merge: dst value = sum over blocks of part[(b, f, g)]
struct DCell {
  int32_t f, g;
  int32_t is_int;
  int32_t vals_f64;    // destination dtype for value comps
  int64_t* cnt;        // when comp == -1
  void* vals;          // value table
  int64_t idx;         // element index in cnt or vals
};

}  // namespace lmfao

// the opaque handle behind lmfao_plan_t
struct lmfao_plan_s {
  lmfao::Plan* P = nullptr;
};
