// Launch entry points of the HIP kernels (host side) and the descriptors
// that only the kernels and the runtime share.
#pragma once

#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace lmfao {

struct DViewBuild {
  int64_t n_rows;
  DCol cols[kMaxPieceCols];  // relation columns referenced (original row order)
  int32_t nkey;
  int32_t key_col[kMaxKey];
  int64_t key_stride[kMaxKey];
  int32_t n_views;
  DView views[kMaxViews];    // key_src = positions in cols
  int32_t n_vals;
  int32_t val_kind[64], val_src[64], val_slot[64];
  int32_t n_codes;
  int32_t code_kind[kMaxOuterCodes], code_src[kMaxOuterCodes], code_slot[kMaxOuterCodes];
  int64_t* out_cnt;
  void* out_vals;
  int32_t* out_codes;
  int32_t* err_flag;
  const int32_t* w;          // filter weight per row (null: no filter)
};

// conjunction of conditions on one relation's columns -> 0/1 weight per row
constexpr int kMaxFilterConds = 8;
struct DFilter {
  int64_t n_rows;
  int32_t n_conds;
  DCol cols[kMaxFilterConds];
  int32_t op[kMaxFilterConds];
  double c[kMaxFilterConds];   // constant, already in the column's comparison type
  const int32_t* ext;          // caller's 0/1 row weights in input row order (null: none)
  const uint32_t* perm;        // row r of this order is input row perm[r] (null: input order)
  int32_t* out;
};

// best split of a CART node batch (section 3, decision trees): per candidate
// the left branch's count and sums of y and y^2 are read from the results of
// the last run, the right branch is the node minus the left
struct DCartBest {
  int32_t best;                // candidate index, -1: none valid
  int32_t pad;
  int64_t n, n_left, n_right;  // node and branch tuple counts
  double sy, sy2;              // node sums of y and y^2
  double sy_left, sy2_left;    // the chosen left branch's
  double cost;                 // VAR(left) + VAR(right) of the chosen split
};
void launch_cart_split(const int64_t* const* cand_cnt, const double* const* cand_vals, int n_cand,
                       const int64_t* tot_cnt, const double* tot_vals, int64_t min_leaf, double tie_eps,
                       double* costs, DCartBest* best, hipStream_t s);

// one range query of the caller's batch: sums of a planned query's buckets
struct DFinalize {
  const int64_t* src_cnt;
  const double* src_vals;
  int64_t* dst_cnt;
  double* dst_vals;
  int64_t n_rows;            // rows of the destination (base group-by keys)
  int64_t nb;                // buckets per destination row (last key of the source)
  int32_t n_vals;
  int64_t lo, hi, ex;        // buckets [lo, hi) except ex
};

struct DKeyCols {
  int32_t n;
  const void* cols[kMaxKey * 2];
  int64_t dom[kMaxKey * 2];
  int32_t* err_flag;
};

// SUM(1) components of a table kept in global memory, copied from its counts
struct DCountCopy {
  const int64_t* cnt;
  double* vals;
  int64_t n;
  int32_t nv, n_copy;
  int32_t comp[kMaxTableComps];
};

struct DTableReduce {
  int64_t n;            // elements of this count table
  int32_t n_blocks;
  int64_t stride;       // partial row stride (elements per block)
  int64_t off;          // offset of the table inside a partial row
  const int32_t* part_i;
  int64_t* dst_cnt;
  // SUM(1) components of the table, equal to its count: written from it
  double* copy_vals;         // destination values (FP64 rows of copy_nv columns)
  int32_t copy_nv;
  int32_t n_copy;
  int32_t copy_comp[kMaxTableComps];
};

// Range check of the 32-bit multiplicities a scan sums: the largest count of
// each multi-valued view the scan looks up, times the most rows one workgroup
// of the scan sums into one 32-bit counter, must stay below 2^31 (else error
// bit 16).  `maxv` holds one zero-initialised slot per view; the check resets
// it, so every run starts from zero without a memset.
struct DMultCheck {
  int32_t n;
  int32_t pad;
  const int64_t* cnt[kMaxViews];
  int64_t n_keys[kMaxViews];
  double rows;
  unsigned long long* maxv;
  int32_t* err_flag;
};
void launch_mult_check(const DMultCheck* d, const DMultCheck& h, hipStream_t s);

// Radix-partitioned counting of large group-by tables of SUM(1) queries (key
// spaces above what a scan keeps in LDS): per row a dense cell index from up
// to 3 codes (columns of the relation or codes carried by unique views),
// weighted by the filter and the views' 0/1 counts.  Tables of one 2^15-cell
// slice are counted in LDS straight from the columns; larger ones are ordered
// by slice within tiles of rows (low 15 bits kept) and every slice is then
// counted in LDS from its tile segments; hash tables (key spaces past 2^24
// cells) are ordered by 9 bits of a hash of the cell and every group of cells
// counted in LDS hash tables.
constexpr int kPartOuts = 32;
constexpr int kPartViews = 4;
constexpr int kPartShift = 15;
constexpr int kPartMaxBuckets = 512;
struct DPartCount {
  int64_t n_rows;
  int32_t n_out;
  int32_t pad0;
  const int32_t* w;                        // filter weight per row (null: all 1)
  int32_t n_views;
  int32_t pad;
  const int64_t* vcnt[kPartViews];         // view counts (0/1: unique views)
  const int32_t* vcodes[kPartViews];       // carried codes [n_keys x vncodes]
  int32_t vncodes[kPartViews];
  int32_t vnkey[kPartViews];
  const int32_t* vkey[kPartViews][2];      // key columns of the relation
  int64_t vstride[kPartViews][2];
  int64_t vnkeys[kPartViews];
  uint32_t vmask[kPartOuts];               // views whose counts weight the output
  int32_t nkey[kPartOuts];
  int32_t ksrc[kPartOuts][3];              // -1: column, else view index
  const int32_t* kcol[kPartOuts][3];
  int32_t kslot[kPartOuts][3];
  int64_t kstride[kPartOuts][3];
  int64_t kdom[kPartOuts][3];
  int64_t n_cells[kPartOuts];
  int32_t n_buckets[kPartOuts];            // slices (dense), or hash groups (hashed)
  int64_t* out_cnt[kPartOuts];
  int32_t hashed[kPartOuts];
  int32_t hidx[kPartOuts];                 // index of the output's table in htab
  int32_t slot[kPartOuts];                 // index among the launch set's outputs of its kind (entry arrays)
  int32_t tile_rows[kPartOuts];            // rows per tile of the tile pass
  int32_t n_tiles[kPartOuts];
  int32_t chunks[kPartOuts];               // counting workgroups per slice (1: stores straight to the output)
  int64_t toff_base[kPartOuts];            // the output's [slice + 1][tile] offsets within toff
  int64_t partial_base[kPartOuts];         // the output's [chunk][cell] partial counts within partial
  uint32_t* toff;
  uint32_t* partial;
  uint32_t* btotal;                        // [out][kPartMaxBuckets] entries per group (hashed outputs)
  uint32_t* bstart;                        // [out][kPartMaxBuckets + 1] group starts in part64b
  uint16_t* part;                          // [dense slot][n_rows] low 15 bits of cells, tile-ordered by slice
  uint64_t* part64;                        // [hashed slot][n_rows] cells, tile-ordered by group
  uint64_t* part64b;                       // [hashed slot][n_rows] the cells ordered by group and sub-group
  const DHashOut* htab;
  uint8_t* w8;                             // [n_rows] per row: bit 0 filter weight, bits 1.. the views'
                                           // 0/1 counts (written by the first pass, read by the others)
  int32_t vkeys_needed;                    // some output's key is a code carried by a view
  int32_t keys_cols[kPartOuts];            // every key of the output is a column of the relation
  uint32_t vmult;                          // bit v: view v holds several tuples per key (its count
                                           // is a multiplicity, not 0/1)
  uint32_t* wv[kPartViews];                // [n_rows] per such view: the row's count (first pass)
  int32_t weighted[kPartOuts];             // the output counts each row with the product of the
                                           // counts of its multiplicity views (dense tables only)
  int32_t wslot[kPartOuts];                // weighted outputs of several slices: index in partw
  uint32_t* partw;                         // [weighted slot][n_rows] the entries' weights, tile-ordered
  uint32_t* partwb;                        // [weighted slot][n_rows] hashed outputs: the weights in the
                                           // group and sub-group order of part64b
  int32_t* err_flag;
};
constexpr int kPartHashBits = 8;                   // hashed tables: groups by the top bits of the cell's mix
constexpr int kPartHashBuckets = 1 << kPartHashBits;
// rows per tile of the tile pass (dense and hashed outputs)
int part_tile_rows(bool hashed, bool weighted);
// one pass of the launch set: row bytes, direct counts, slice-ordered tiles,
// slice counts, partial-table sums, hash-ordered tiles, hashed groups
enum {
  kPartPhaseRows = 0,
  kPartPhaseDirect = 1,
  kPartPhaseTile = 2,
  kPartPhaseSlices = 3,
  kPartPhaseReduce = 4,
  kPartPhaseTileHash = 5,
  kPartPhaseHash = 6
};
void launch_part_count(const DPartCount* d, const DPartCount& h, int phase, hipStream_t s);

void launch_fill(void* p, int64_t bytes, hipStream_t s);
// number of nonzero keys (occupied slots) of a hash table, added to *out
void launch_count_keys(const unsigned long long* keys, int64_t n, unsigned long long* out, hipStream_t s);
void launch_filter(const DFilter* d, int64_t n_rows, hipStream_t s);
// the same with the descriptor passed by value (no device copy)
void launch_filter_value(const DFilter& f, hipStream_t s);
void launch_bucketize(const void* src, int dtype, int64_t n, const double* thr, int n_thr, int kind, int32_t* out,
                      hipStream_t s);
void launch_finalize(const DFinalize* d, int n, hipStream_t s);
// out[r] = tab[src[r]] (a tabulated function of an integer column)
void launch_gather_table(const int32_t* src, int64_t n, const double* tab, int64_t nt, double* out, int32_t* err,
                         hipStream_t s);

// covariance-matrix assembly entry: Sigma[a][b] = Sigma[b][a] = *src
struct DSigmaEntry {
  const double* src;
  int32_t a, b;
};
void launch_sigma_assemble(const DSigmaEntry* e, int64_t n, double* sigma, int dim, hipStream_t s);
// ridge batch gradient descent on Sigma (one workgroup); out = {steps, ||grad||, eta}
void launch_ridge_bgd(const double* sigma, int dim, int label, double lam, double eta, int max_iter, double tol,
                      double* theta, double* out, hipStream_t s);
constexpr int kRidgeMaxDim = 2048;
// relations of at least this many rows build their view a thread per row,
// smaller ones a thread per output element
constexpr int64_t kViewBuildRowsMin = 65536;
void launch_view_build(const DViewBuild* d, int64_t n_rows, bool f64, hipStream_t s);
void launch_make_keys(const DKeyCols* d, uint64_t* keys, uint32_t* idx, int64_t n, hipStream_t s);
void launch_sort(uint64_t* keys, uint32_t* idx, uint64_t* keys_tmp, uint32_t* idx_tmp, int64_t n, int bits,
                 uint32_t* hist, hipStream_t s, bool* swapped);
int sort_tile();
// A query's result compacted on the device into its present groups (count
// > 0), keys decomposed per attribute, in lexicographic key order: dense
// tables in row order (the row is the mixed-radix key, first attribute most
// significant), hash tables gathered and then sorted by row.
struct DCompact {
  const int64_t* cnt;                  // [n_src] dense rows or hash slots
  const double* vals;                  // [n_src x n_vals], null: no stored values
  const unsigned long long* hkeys;     // hash tables: row + 1 per slot, 0 = empty; null: dense
  int64_t n_src;
  int32_t n_vals, n_keys;
  uint64_t copy_mask;                  // value components equal to the count, added from it
  int64_t stride[4], dom[4];           // key decomposition of a row
  uint32_t* pos;                       // [n_src + scan tiles + 1]: present flags, then positions
  uint64_t* rows;                      // hash tables: rows of the present groups
  uint32_t* slot;                      // ... and their slots
  int64_t* keys_out;                   // [groups x n_keys]
  int64_t* cnt_out;                    // [groups]
  double* vals_out;                    // [groups x n_vals]
};
// flags, scan and (dense) emission; *groups receives the group count (pos
// must hold scan_tiles(n_src) + 1 more values)
void launch_compact(const DCompact& d, hipStream_t s);
// hash tables after launch_compact: emission of the n sorted groups
void launch_compact_emit(const DCompact& d, int64_t n, hipStream_t s);

// Rk-means step 2: weighted 1-D k-means (Lloyd) per set of ascending
// integer values with integer weights, one workgroup per set
constexpr int kKmMaxClusters = 64;
void launch_kmeans_1d(const int64_t* off, int n_sets, const int64_t* values, const int64_t* weights, int k,
                      int max_iter, double* centroids, int32_t* assignment, int32_t* steps, hipStream_t s);

// Rk-means step 3: the grid coreset over a join whose tuples a root row
// determines (relations in breadth-first order from the root, each reached
// from its parent through one key attribute)
constexpr int kGridMaxWords = 8;     // 512 bits of packed cluster ids
constexpr int kGridMaxRels = 8;
constexpr int kGridMaxDims = 256;
struct DGrid {
  int64_t n_rows;                          // rows of the root relation
  int32_t n_rels, n_dims, bits, n_words;
  int32_t parent[kGridMaxRels];            // breadth-first parent of relation i
  const int32_t* pkey[kGridMaxRels];       // the parent's column of the key reaching relation i
  const int32_t* index[kGridMaxRels];      // key value -> row of relation i (-1: none)
  int64_t index_n[kGridMaxRels];
  const int32_t* col[kGridMaxDims];        // dimension d's column in relation rel[d]
  int32_t rel[kGridMaxDims];
  const int32_t* cluster[kGridMaxDims];    // cluster id of every value of dimension d
  int64_t dom[kGridMaxDims];
  unsigned long long* keys;                // fingerprint per slot (0: empty)
  unsigned long long* cnt;
  int32_t* rep;                            // a root row of the slot's group
  int64_t mask;
  int32_t* flag;                           // 1 fingerprint clash, 2 table full, 4 value outside a domain, 8 key twice
};
void launch_grid_index(const int32_t* key, int64_t n, int32_t* index, int64_t index_n, int32_t* flag,
                       hipStream_t s);
void launch_grid_count(const DGrid* d, int64_t n_rows, hipStream_t s);
// present flags and positions of the slots (pos: slots + scan tiles + 1
// values; the group count lands after the tile sums), then the groups
void launch_grid_positions(const DGrid* d, int64_t slots, uint32_t* pos, hipStream_t s);
void launch_grid_emit(const DGrid* d, int64_t slots, const uint32_t* pos, int64_t* keys_out, int64_t* cnt_out,
                      hipStream_t s);
void launch_code_table(const int64_t* codes, const int32_t* cluster, int64_t n, int32_t* table, int64_t dom,
                       int32_t* flag, hipStream_t s);

// exclusive scan of a[0..m) in place over many workgroups; bsum holds
// scan_tiles(m) + 1 values and receives the tile offsets, then the total
int64_t scan_tiles(int64_t m);
void launch_scan_excl(uint32_t* a, int64_t m, uint32_t* bsum, hipStream_t s);
void launch_gather(const void* src, const uint32_t* perm, void* dst, int64_t n, int elem_bytes, hipStream_t s);
void launch_gather_convert(const void* src, int src_dtype, const uint32_t* perm, void* dst, int64_t n, bool to_f64,
                           hipStream_t s);
void launch_segment_starts(const uint64_t* keys, int64_t n, uint64_t div, unsigned long long* count,
                           int64_t* pos, uint64_t* pkey, int64_t cap, hipStream_t s);
void launch_validate(const int32_t* col, int64_t n, int64_t dom, int32_t* err_flag, hipStream_t s);
// number of distinct values of an integer column with values in [0, dom);
// bits: (dom + 31) / 32 words of scratch, out: one device counter
void launch_distinct(const int32_t* col, int64_t n, int64_t dom, uint32_t* bits, unsigned long long* out,
                     hipStream_t s);

int scan_lds_bytes(const DScan& S, bool f64);
int scan_fast_lds_bytes(const DScan& S, bool f64);
void launch_scan_fast(const DScan* d, int na, bool f64, int grid, int lds, hipStream_t s);
int image_code_slots(int n_codes);
int image_width_dw(int na, bool f64, int n_codes);
int image_code_off(int na, bool f64);
void launch_build_image(const DImageBuild* d, int64_t n_keys, bool f64, hipStream_t s);
void launch_scan(const DScan* d, int na, bool f64, int grid, int lds, hipStream_t s);
int scan_waves_per_block();

int contract_lds_bytes(const DContract& C, bool f64);
int contract_tiles(int nf, int ng);
int contract_threads();
int contract_max_int_cells();
void launch_contract(const DContract* d, bool f64, int grid_x, int grid_y, int lds, hipStream_t s);
int gemm_tile_cols(int ng);
int gemm_macro_tiles(int nf, int ng);
int contract_fused_lds_bytes(const DContract& C, int tn);
int contract_fused_chunk();
// bf16_parts 2 or 3: float-only tiles of the FP32 form on the bf16 matrix
// cores (operands split into 2 or 3 bf16 parts, 3 or 6 products, FP32 within
// a chunk of pieces, FP64 across); 0: FP64 matrix cores
// row pieces whose outputs are all scattered: one thread per row
void launch_scatter_rows(const DContract* c, bool f64, int grid, hipStream_t s);
void launch_contract_fused(const DContract* c, const DGemm* g, bool f64, int bf16_parts, int tn, int gx, int gy,
                           int lds, hipStream_t s);
void launch_merge_bm(const DCell* cells, int64_t n_cells, const double* part, int n_blocks, int ng, int64_t ncell,
                     int32_t* err_flag, hipStream_t s);

void launch_merge_cells(const DCell* cells, int64_t n_cells, const double* part_f, const int64_t* part_i,
                        int n_blocks, int NF, int NG, int NFI, int NGI, hipStream_t s);
void launch_table_reduce(const DTableReduce* d, int64_t n, int n_blocks, hipStream_t s);
void launch_count_copy(const DCountCopy* d, int64_t n, hipStream_t s);

}  // namespace lmfao
