// Runtime and C ABI: plan handles, prepare (validation, sorting by the
// attribute order, trie-level pieces, device descriptors, buffers) and run
// (every group of the plan, dependency level by level, on one HIP stream).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "engine.hpp"
#include "codegen.hpp"
#include "kernels.hpp"
#include "lmfao.h"

namespace lmfao {

struct HipError {
  std::string msg;
};

#define HIP_OK(x)                                                                                       \
  do {                                                                                                  \
    hipError_t e_ = (x);                                                                                \
    if (e_ != hipSuccess) throw HipError{std::string(#x) + ": " + hipGetErrorString(e_)};               \
  } while (0)

static constexpr int64_t kPieceMax = 8192;    // rows of one piece at most
static constexpr int64_t kPieceMaxF64 = 64;   // FP64 plans: short (uncompensated) histogram chains
static constexpr int64_t kItemRows = 4096;    // rows one wavefront takes per work item, at most
static constexpr int64_t kTargetItems = 16384; // work items wanted per scan: ~4 per resident wavefront

struct OutBuf {
  int64_t* cnt = nullptr;
  void* vals = nullptr;
  int32_t* codes = nullptr;
  int64_t n_rows = 0;              // dense rows (the key space)
  int n_vals = 0;
  int n_codes = 0;
  bool f64 = true;
  int hash = -1;                   // index of the hash table holding this output, -1 dense
};

// a hash table of one query output (key space larger than a dense table)
struct HashBuf {
  int query = -1;
  int64_t cap = 0;                 // slots (power of two)
  int64_t bound = 0;               // most groups there can be (distinct keys)
  double est = -1;                 // groups the estimator predicted (-1 = not used)
  unsigned long long* keys = nullptr;
  int64_t* cnt = nullptr;
  double* vals = nullptr;
  int n_vals = 0;
  int fill_step = -1;              // index of its zeroing steps (keys, cnt, vals); -1: none
  bool counts_only = false;        // written by the partition count; every value is the count
  uint32_t* used = nullptr;        // counts-only tables: groups per region at the last run
  std::vector<int> count_copies;   // value columns equal to the count (SUM(1))
};

struct NodeData {
  bool sorted = false;
  std::vector<void*> sorted_col;   // per relation column (nullptr = not gathered)
  std::vector<void*> raw_col;      // library copy of the original columns (row pieces, view builds)
  int64_t n_pieces = 0;
  int64_t* piece_begin = nullptr;
  int32_t* piece_key = nullptr;
  int32_t* item_piece = nullptr;
  int n_items = 0;
  int64_t max_item_rows = 0;       // rows of the longest work item
  int cut = 0;
  uint32_t* perm = nullptr;        // sort permutation, kept until prepare ends
  std::vector<void*> typed_col;    // sorted copies in the compute type (factor columns of lean scans)
  std::vector<const void*> raw_src;  // caller's columns, valid during prepare only
};

struct Step {
  std::string name;
  hipFunction_t gen_fn = nullptr;   // generated kernel (scan steps), else a built-in kernel
  const uint64_t* gen_args = nullptr;
  int gen_block = 0;
  void* dev2 = nullptr;             // second descriptor (fused contraction: the product's)
  int kind;   // 0 fill, 1 view build, 2 scan, 3 table reduce, 4 contract (VALU), 5 merge, 6 image build,
              // 7 (unused), 8 MFMA contraction, 9 block-major merge, 10 filter, 11 finalize,
              // 12 row-by-row scatter, 13 count copy, 14 multiplicity range check,
              // 15 radix-partitioned count
  int fast = 0;
  void* dev = nullptr;
  int64_t n = 0;
  int na = 0;
  int grid = 0, grid_y = 0, lds = 0;
  int64_t bytes = 0;
  // merge
  const double* part_f = nullptr;
  const int64_t* part_i = nullptr;
  int n_blocks = 0, NF = 0, NG = 0, NFI = 0, NGI = 0;
  DMultCheck mult{};                // kind 14: host copy of the descriptor
  DPartCount part{};                // kind 15: host copy of the descriptor
  // the relation pass this launch belongs to: the relation's columns its
  // outputs reference (bucket codes counted as their source column), whether
  // read from HBM or folded by prepare into piece keys
  int relation = -1;
  std::vector<int> pass_cols;
  // accounting (host-computed): bytes the step must move, arithmetic it must do
  double alg_read = 0, alg_write = 0, alg_flop = 0;
  int64_t rows = 0, pieces = 0;
};

// a caller query's result compacted on the device (lmfao_result_device)
struct Compacted {
  int64_t epoch = -1;          // the run it was compacted after (-1: never)
  int64_t n_groups = 0;
  int64_t cap = 0;             // groups the buffers hold
  int64_t* keys = nullptr;     // [cap x n_keys]
  int64_t* cnt = nullptr;      // [cap]
  double* vals = nullptr;      // [cap x n_vals]
};

}  // namespace lmfao


struct lmfao_prepared_s {
  lmfao::Plan* P = nullptr;
  bool f64 = true;
  std::vector<lmfao::OutBuf> qout, vout;
  std::vector<lmfao::OutBuf> uout;                   // range queries of the caller's batch
  std::vector<std::string> gen_sources, gen_failures; // generated scan kernels (and why not)
  std::vector<lmfao::HashBuf> hashes;
  lmfao::DHashOut* hash_dev = nullptr;                // device copy of the hash descriptors
  int hash_regrowths = 0;                             // runs repeated after a hash overflow
  std::map<int, int64_t> distinct;                    // distinct values per integer attribute
  // per (node, row order, views) the partition count's per-row bytes and view
  // counts: the first launch set that reads them writes them each run
  std::map<std::string, std::pair<uint8_t*, std::vector<uint32_t*>>> part_rows;
  std::map<std::pair<int, int>, int64_t> distinct_rel; // ... per (attribute, relation)
  int32_t* hash_ovf = nullptr;                        // per table overflow flag
  std::vector<std::vector<const void*>> ecols;       // caller's columns, then derived bucket codes
  std::vector<const void* const*> ecol_ptrs;
  std::vector<int32_t*> w_raw, w_sorted;             // filter weights per relation (lazily built)
  std::vector<int32_t*> row_w;                       // caller-written row weights (options.row_weights)
  std::vector<uint32_t*> row_perm;                   // sort permutation kept for sorted weights
  void* cart_dev = nullptr;                          // CART split: candidate pointers, best, costs
  size_t cart_bytes = 0;
  char* ws = nullptr;                                // caller's workspace (lmfao_prepare_in), or null
  size_t ws_cap = 0;
  size_t ws_used = 0;                                // bytes carved (workspace or hipMalloc)
  size_t ws_prepared = 0;                            // ... when lmfao_prepare returned
  int64_t run_epoch = 0;                             // runs enqueued
  int picked_hash = 0;                               // dense key spaces the estimator sent to hash tables
  std::vector<lmfao::Compacted> compact;             // device results per caller query
  uint32_t* cpos = nullptr;                          // compaction scratch: flags and positions
  int64_t cpos_n = 0;
  uint64_t *crows = nullptr, *crows2 = nullptr;      // ... hashed groups' rows and slots, sort buffers
  uint32_t *cslot = nullptr, *cslot2 = nullptr, *chist = nullptr;
  int64_t crows_n = 0;
  std::vector<char> w_raw_done, w_sorted_done;
  std::vector<lmfao::NodeData> nodes;
  std::vector<void*> allocs;
  std::vector<lmfao::Step> steps;   // the run, in launch order
  int32_t* err_flag = nullptr;
  bool timing = false;
  std::vector<hipEvent_t> ev;       // event pool: per timed run, a (start, stop) per timed step + run
  int timed_runs = 0;               // runs recorded since the last lmfao_run_timing
  std::vector<float> step_ms;
  hipStream_t stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;                // captured run (graph option)
  hipStream_t capture_stream = nullptr;
  bool graph_failed = false;
  ~lmfao_prepared_s() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
    if (!ws)
      for (auto& H : hashes)
        for (void* p : {(void*)H.keys, (void*)H.cnt, (void*)H.vals})
          if (p) (void)hipFree(p);
  }
};

namespace lmfao {

using Prep = lmfao_prepared_s;

// Device memory of a prepared plan.  With a caller's workspace
// (lmfao_prepare_in) every buffer is carved from it, 256-byte aligned, and
// nothing is returned before the handle is freed; otherwise hipMalloc.  Both
// count the bytes carved, which is what a workspace for the same plan and
// inputs must hold (lmfao_prepared_workspace_bytes).
static void* dmem(Prep& S, size_t bytes) {
  if (bytes == 0) bytes = 8;
  const size_t carved = (bytes + 255) & ~(size_t)255;
  if (S.ws) {
    if (S.ws_used + carved > S.ws_cap)
      throw PlanError{LMFAO_ENOMEM, "workspace of " + std::to_string(S.ws_cap) + " bytes is too small (" +
                                        std::to_string(S.ws_used + carved) + " bytes needed so far)"};
    void* p = S.ws + S.ws_used;
    S.ws_used += carved;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw PlanError{LMFAO_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e)};
  }
  S.ws_used += carved;
  return p;
}
static void dfree(Prep& S, void* p) {
  if (!S.ws && p) (void)hipFree(p);
}
static void* dalloc(Prep& S, size_t bytes) {
  void* p = dmem(S, bytes);
  if (!S.ws) S.allocs.push_back(p);
  return p;
}

template <typename D>
static D* upload(Prep& S, const D& h, hipStream_t st) {
  D* d = (D*)dalloc(S, sizeof(D));
  HIP_OK(hipMemcpyAsync(d, &h, sizeof(D), hipMemcpyHostToDevice, st));
  return d;
}
template <typename D>
static D* upload_vec(Prep& S, const std::vector<D>& h, hipStream_t st) {
  D* d = (D*)dalloc(S, std::max<size_t>(1, h.size()) * sizeof(D));
  if (!h.empty()) HIP_OK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(D), hipMemcpyHostToDevice, st));
  return d;
}

static int dtype_bytes(int dt) { return dt == LMFAO_F64 ? 8 : 4; }

static void add_fill(Prep& S, void* p, int64_t bytes, const std::string& name) {
  Step s;
  s.name = name;
  s.kind = 0;
  s.dev = p;
  s.bytes = bytes;
  S.steps.push_back(s);
}

// strides of a dense key over attribute list (last attribute fastest)
static std::vector<int64_t> strides_of(const Plan& P, const std::vector<int>& attrs) {
  std::vector<int64_t> st(attrs.size(), 1);
  int64_t m = 1;
  for (int i = (int)attrs.size() - 1; i >= 0; --i) {
    st[i] = m;
    m *= P.attrs[attrs[i]].domain;
  }
  return st;
}

static DView dview_of(const Prep& S, int vid) {
  const Plan& P = *S.P;
  const ViewDef& V = P.views[vid];
  const OutBuf& B = S.vout[vid];
  DView d{};
  d.cnt = B.cnt;
  d.vals = B.vals;
  d.codes = B.codes;
  d.vals_f64 = B.f64 ? 1 : 0;
  d.n_vals = B.n_vals;
  d.n_codes = B.n_codes;
  d.nkey = (int)V.key.size();
  if (d.nkey > kMaxKey) throw PlanError{LMFAO_EUNSUPPORTED, "view key with more than 4 attributes"};
  std::vector<int64_t> st = strides_of(P, V.key);
  for (int k = 0; k < d.nkey; ++k) d.key_stride[k] = st[k];
  d.n_keys = V.n_keys;
  return d;
}

// library copy of an original relation column (for row pieces and view builds)
static void* raw_column(Prep& S, int r, int c, const void* const* const* cols, hipStream_t st) {
  NodeData& N = S.nodes[r];
  if (N.raw_col[c]) return N.raw_col[c];
  const RelDef& R = S.P->rels[r];
  size_t bytes = (size_t)R.n_rows * dtype_bytes(R.dtypes[c]);
  void* p = dalloc(S, bytes);
  if (bytes) HIP_OK(hipMemcpyAsync(p, cols[r][c], bytes, hipMemcpyDeviceToDevice, st));
  N.raw_col[c] = p;
  return p;
}

// ---------------------------------------------------------------------------
// prepare: sort a relation by its attribute order and cut it into pieces
// ---------------------------------------------------------------------------
static void prepare_node(Prep& S, int r, int cut, const std::vector<int>& need_cols,
                         const void* const* const* cols, hipStream_t st) {
  const Plan& P = *S.P;
  const RelDef& R = P.rels[r];
  NodeData& N = S.nodes[r];
  const std::vector<int>& order = P.order[r];
  int64_t n = R.n_rows;
  N.cut = cut;
  if (!N.sorted) {
    double bits_d = 0;
    for (int a : order) bits_d += std::log2((double)P.attrs[a].domain);
    int bits = (int)std::ceil(bits_d - 1e-9);
    if (bits > 64) throw PlanError{LMFAO_EUNSUPPORTED, "attribute order of " + R.name + " needs more than 64 key bits"};
    if (bits < 1) bits = 1;
    if (n > (int64_t)UINT32_MAX) throw PlanError{LMFAO_EUNSUPPORTED, "relation larger than 2^32 rows"};
    DKeyCols kc{};
    kc.n = (int)order.size();
    if (kc.n > kMaxKey * 2) throw PlanError{LMFAO_EUNSUPPORTED, "attribute order longer than 8"};
    for (int i = 0; i < kc.n; ++i) {
      kc.cols[i] = cols[r][R.col.at(order[i])];
      kc.dom[i] = P.attrs[order[i]].domain;
    }
    kc.err_flag = S.err_flag;
    DKeyCols* dkc = upload(S, kc, st);
    uint64_t *keys, *keys2;
    uint32_t *idx, *idx2, *hist;
    keys = (uint64_t*)dmem(S, std::max<int64_t>(n, 1) * 8);
    keys2 = (uint64_t*)dmem(S, std::max<int64_t>(n, 1) * 8);
    idx = (uint32_t*)dmem(S, std::max<int64_t>(n, 1) * 4);
    idx2 = (uint32_t*)dmem(S, std::max<int64_t>(n, 1) * 4);
    int nblocks = (int)((n + sort_tile() - 1) / sort_tile());
    // digit counts per block, then the scan's tile sums and total
    const int64_t hist_n = (int64_t)256 * std::max(nblocks, 1);
    hist = (uint32_t*)dmem(S, (size_t)(hist_n + scan_tiles(hist_n) + 1) * 4);
    if (n > 0) {
      launch_make_keys(dkc, keys, idx, n, st);
      bool swapped = false;
      launch_sort(keys, idx, keys2, idx2, n, bits, hist, st, &swapped);
      if (swapped) {
        std::swap(keys, keys2);
        std::swap(idx, idx2);
      }
    }
    N.sorted_col.assign(R.attrs.size(), nullptr);
    // segments at the cut level
    uint64_t div = 1;
    for (int i = cut; i < (int)order.size(); ++i) div *= (uint64_t)P.attrs[order[i]].domain;
    int64_t cap = std::min<int64_t>(std::max<int64_t>(n, 1), 1 << 22);
    std::vector<int64_t> hpos;
    std::vector<uint64_t> hkey;
    for (int attempt = 0; attempt < 2; ++attempt) {
      unsigned long long* dcount;
      int64_t* dpos;
      uint64_t* dkey;
      dcount = (unsigned long long*)dmem(S, 8);
      dpos = (int64_t*)dmem(S, cap * 8);
      dkey = (uint64_t*)dmem(S, cap * 8);
      HIP_OK(hipMemsetAsync(dcount, 0, 8, st));
      if (n > 0) launch_segment_starts(keys, n, div, dcount, dpos, dkey, cap, st);
      unsigned long long cnt = 0;
      HIP_OK(hipMemcpyAsync(&cnt, dcount, 8, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if ((int64_t)cnt <= cap) {
        hpos.resize(cnt);
        hkey.resize(cnt);
        if (cnt) {
          HIP_OK(hipMemcpy(hpos.data(), dpos, cnt * 8, hipMemcpyDeviceToHost));
          HIP_OK(hipMemcpy(hkey.data(), dkey, cnt * 8, hipMemcpyDeviceToHost));
        }
        dfree(S, dcount);
        dfree(S, dpos);
        dfree(S, dkey);
        break;
      }
      cap = (int64_t)cnt;
      dfree(S, dcount);
      dfree(S, dpos);
      dfree(S, dkey);
    }
    HIP_OK(hipStreamSynchronize(st));
    dfree(S, keys);
    dfree(S, keys2);
    dfree(S, idx2);
    dfree(S, hist);
    N.perm = idx;
    // pieces: segments in row order, split so that the scan has about
    // kTargetItems work items of whole 64-row chunks (small relations get
    // short pieces instead of a handful of long ones)
    const int64_t item_rows =
        std::min<int64_t>(kItemRows, std::max<int64_t>(64, ((n + kTargetItems - 1) / kTargetItems + 63) / 64 * 64));
    std::vector<size_t> ord(hpos.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return hpos[a] < hpos[b]; });
    std::vector<int64_t> pb;
    std::vector<std::vector<int32_t>> pk(cut);
    for (size_t i = 0; i < ord.size(); ++i) {
      int64_t b = hpos[ord[i]];
      int64_t e = (i + 1 < ord.size()) ? hpos[ord[i + 1]] : n;
      uint64_t key = hkey[ord[i]];
      std::vector<int32_t> vals(cut);
      for (int l = cut - 1; l >= 0; --l) {
        uint64_t d = (uint64_t)P.attrs[order[l]].domain;
        vals[l] = (int32_t)(key % d);
        key /= d;
      }
      const int64_t pmax = std::min<int64_t>(S.f64 ? kPieceMaxF64 : kPieceMax, item_rows);
      for (int64_t x = b; x < e; x += pmax) {
        pb.push_back(x);
        for (int l = 0; l < cut; ++l) pk[l].push_back(vals[l]);
      }
    }
    N.n_pieces = (int64_t)pb.size();
    pb.push_back(n);
    std::vector<int32_t> items{0};
    int64_t acc = 0;
    for (int64_t p = 0; p < N.n_pieces; ++p) {
      acc += pb[p + 1] - pb[p];
      if (acc >= item_rows) {
        items.push_back((int32_t)(p + 1));
        acc = 0;
      }
    }
    if (items.back() != (int32_t)N.n_pieces) items.push_back((int32_t)N.n_pieces);
    N.n_items = (int)items.size() - 1;
    N.max_item_rows = 0;
    for (int i = 0; i < N.n_items; ++i)
      N.max_item_rows = std::max<int64_t>(N.max_item_rows, pb[items[i + 1]] - pb[items[i]]);
    N.piece_begin = upload_vec(S, pb, st);
    std::vector<int32_t> flat;
    for (int l = 0; l < cut; ++l) flat.insert(flat.end(), pk[l].begin(), pk[l].end());
    N.piece_key = upload_vec(S, flat, st);
    N.item_piece = upload_vec(S, items, st);
    N.sorted = true;
  }
  for (int c : need_cols) {
    if (N.sorted_col[c]) continue;
    int eb = dtype_bytes(R.dtypes[c]);
    void* p = dalloc(S, (size_t)std::max<int64_t>(n, 1) * eb);
    if (n > 0) launch_gather(cols[r][c], N.perm, p, n, eb, st);
    N.sorted_col[c] = p;
  }
}

// sorted copy of a column converted to the compute type (needs the sort permutation)
static void* typed_sorted_column(Prep& S, int r, int c, hipStream_t st) {
  NodeData& N = S.nodes[r];
  if (N.typed_col.empty()) N.typed_col.assign(S.P->rels[r].attrs.size(), nullptr);
  if (N.typed_col[c]) return N.typed_col[c];
  const RelDef& R = S.P->rels[r];
  if (!N.perm) throw PlanError{LMFAO_EINVAL, "internal: typed column without permutation"};
  void* p = dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * (S.f64 ? 8 : 4));
  if (R.n_rows > 0) launch_gather_convert(N.raw_src[c], R.dtypes[c], N.perm, p, R.n_rows, S.f64, st);
  N.typed_col[c] = p;
  return p;
}

// ---------------------------------------------------------------------------
// descriptors of one group program
// ---------------------------------------------------------------------------
// Contraction on the matrix cores: one launch stages the features F and the
// columns B of each chunk of pieces in LDS and multiplies them on the matrix
// cores into block-major partials; a merge adds the partials of every cell of
// the plan into its output.
static void build_contract_mfma(Prep& S, const GroupProgram& g, const std::string& gname, DContract& c,
                                int64_t n_pieces, int psi_f_stride, int psi_i_stride, bool f64, hipStream_t st) {
  const int NF = c.n_feat, NG = c.n_col;
  c.err_flag = S.err_flag;
  c.part_f = nullptr;
  c.part_i = nullptr;
  c.pieces_per_block = 0;
  if (c.row_pieces && g.gemm_cells.empty()) {
    // every output is scattered: the row-by-row kernel, no matrix product
    Step sr;
    sr.name = gname + ":scatter";
    sr.kind = 12;
    sr.dev = upload(S, c, st);
    sr.grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_pieces + 255) / 256, 16384));
    sr.pieces = n_pieces;
    sr.rows = n_pieces;
    for (int i = 0; i < c.n_pcols; ++i) sr.alg_read += (double)n_pieces * (c.pcols[i].dtype == LMFAO_F64 ? 8 : 4);
    for (int v = 0; v < c.n_views; ++v)
      sr.alg_read += (double)std::min<int64_t>(c.views[v].n_keys, n_pieces) *
                     (8 + c.views[v].n_vals * (c.views[v].vals_f64 ? 8 : 4) + c.views[v].n_codes * 4);
    S.steps.push_back(sr);
    return;
  }
  const int tn = gemm_tile_cols(std::max(1, NG));
  const int gy = gemm_macro_tiles(std::max(1, NF), std::max(1, NG));
  const int64_t kc = contract_fused_chunk();
  // Pieces are cut into about 1024 ranges per column of output tiles (fewer
  // when the grid would pass 4096 workgroups): with two to three resident
  // workgroups per CU the three dependent loads of each 16-piece chunk stay
  // hidden, and the FP64 partials to merge stay small.
  const int64_t want = S.P->opts.contract_splits > 0
                           ? (int64_t)S.P->opts.contract_splits
                           : std::max<int64_t>(1, std::min<int64_t>(1024, 4096 / gy));
  int64_t kpb = (n_pieces + want - 1) / want;
  kpb = std::max<int64_t>(kc, (kpb + kc - 1) / kc * kc);
  const int gx = (int)std::max<int64_t>(1, (n_pieces + kpb - 1) / kpb);
  const int64_t ncell = (int64_t)std::max(1, NF) * std::max(1, NG);
  double* part = (double*)dalloc(S, (size_t)gx * ncell * 8);
  const int lds = contract_fused_lds_bytes(c, tn);
  if (lds > 160 * 1024) throw PlanError{LMFAO_EUNSUPPORTED, "contraction needs more LDS than a CU has"};
  DGemm gm{};
  gm.n = n_pieces;
  gm.nf = NF;
  gm.ng = NG;
  gm.k_per_block = kpb;
  gm.part = part;
  Step st2;
  st2.name = gname + ":contract";
  st2.kind = 8;
  st2.dev = upload(S, c, st);
  st2.dev2 = upload(S, gm, st);
  st2.grid = gx;
  st2.grid_y = gy;
  st2.na = tn;
  st2.lds = lds;
  st2.pieces = n_pieces;
  st2.rows = n_pieces;
  for (int i = 0; i < c.n_pcols; ++i) st2.alg_read += (double)n_pieces * (c.pcols[i].dtype == LMFAO_F64 ? 8 : 4);
  st2.alg_read += (double)n_pieces * (psi_f_stride * (f64 ? 8 : 4) + psi_i_stride * 4);
  for (int v = 0; v < c.n_views; ++v)
    st2.alg_read += (double)std::min<int64_t>(c.views[v].n_keys, n_pieces) *
                    (8 + c.views[v].n_vals * (c.views[v].vals_f64 ? 8 : 4) + c.views[v].n_codes * 4);
  st2.alg_write = (double)gx * NF * NG * 8;
  st2.alg_flop = 2.0 * (double)n_pieces * NF * NG;
  S.steps.push_back(st2);
  if (NF == 0 || NG == 0 || g.gemm_cells.empty()) return;

  std::vector<DCell> cells;
  for (auto& gc : g.gemm_cells) {
    const ProgOutput& po = g.outs[gc.second.out];
    const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
    DCell x{};
    x.f = gc.first.first;
    x.g = gc.first.second;
    x.is_int = (x.f < c.n_feat_int && x.g < c.n_col_int) ? 1 : 0;
    x.vals_f64 = O.f64 ? 1 : 0;
    if (gc.second.comp < 0) {
      if (!x.is_int) throw PlanError{LMFAO_EINVAL, "internal: count cell not integral"};
      x.cnt = O.cnt;
      x.vals = nullptr;
      x.idx = gc.second.row;
    } else {
      x.cnt = nullptr;
      x.vals = O.vals;
      x.idx = gc.second.row * O.n_vals + gc.second.comp;
    }
    cells.push_back(x);
  }
  // partial rows are read a 128-byte line of consecutive cells at a time
  std::stable_sort(cells.begin(), cells.end(), [](const DCell& a, const DCell& b) {
    return a.f != b.f ? a.f < b.f : a.g < b.g;
  });
  Step m;
  m.name = gname + ":merge";
  m.kind = 9;
  m.dev = upload_vec(S, cells, st);
  m.n = (int64_t)cells.size();
  m.part_f = part;
  m.n_blocks = gx;
  m.NF = NF;
  m.NG = NG;
  m.alg_read = (double)gx * cells.size() * 8;
  m.alg_write = (double)cells.size() * 8;
  S.steps.push_back(m);
}

// Filter weights of relation r (0/1 per row, raw or sorted row order) for the
// batch-wide conditions on its attributes; null when none applies.  Built once
// per prepared plan as a step of the run, ahead of its first consumer.
static const int32_t* filter_weights(Prep& S, int r, bool sorted, const void* const* const* cols,
                                     hipStream_t st) {
  const Plan& P = *S.P;
  auto& cache = sorted ? S.w_sorted : S.w_raw;
  auto& done = sorted ? S.w_sorted_done : S.w_raw_done;
  if (done[r]) return cache[r];
  done[r] = 1;
  const RelDef& R = P.rels[r];
  DFilter f{};
  f.n_rows = R.n_rows;
  const bool ext = r < (int)S.row_w.size() && S.row_w[r];
  if (ext) {
    f.ext = S.row_w[r];
    if (sorted) {
      // the run reads the caller's weights through the sort permutation
      NodeData& N = S.nodes[r];
      if (!S.row_perm[r]) {
        if (!N.perm) throw PlanError{LMFAO_EINVAL, "internal: row weights without permutation"};
        S.row_perm[r] = (uint32_t*)dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * 4);
        if (R.n_rows > 0)
          HIP_OK(hipMemcpyAsync(S.row_perm[r], N.perm, (size_t)R.n_rows * 4, hipMemcpyDeviceToDevice, st));
      }
      f.perm = S.row_perm[r];
    }
  }
  for (const Cond& c : P.filter) {
    if (!R.has(c.attr)) continue;
    if (f.n_conds >= kMaxFilterConds) throw PlanError{LMFAO_EUNSUPPORTED, "too many conditions on " + R.name};
    const int col = R.col.at(c.attr);
    const void* ptr;
    if (sorted) {
      NodeData& N = S.nodes[r];
      if (!N.sorted_col[col]) {
        if (!N.perm) throw PlanError{LMFAO_EINVAL, "internal: filter column without permutation"};
        const int eb = dtype_bytes(R.dtypes[col]);
        void* q = dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * eb);
        if (R.n_rows > 0) launch_gather(cols[r][col], N.perm, q, R.n_rows, eb, st);
        N.sorted_col[col] = q;
      }
      ptr = N.sorted_col[col];
    } else {
      ptr = raw_column(S, r, col, cols, st);
    }
    f.cols[f.n_conds] = DCol{ptr, R.dtypes[col], 0};
    f.op[f.n_conds] = c.op;
    f.c[f.n_conds] = c.c;
    f.n_conds++;
  }
  if (f.n_conds == 0 && !ext) return nullptr;
  f.out = (int32_t*)dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * 4);
  Step s;
  s.name = "filter:" + R.name + (sorted ? ":sorted" : ":raw");
  s.kind = 10;
  s.dev = upload(S, f, st);
  s.n = R.n_rows;
  s.rows = R.n_rows;
  s.alg_read = 0;
  for (int k = 0; k < f.n_conds; ++k) s.alg_read += (double)R.n_rows * dtype_bytes(f.cols[k].dtype);
  if (ext) s.alg_read += (double)R.n_rows * (sorted ? 8 : 4);
  s.alg_write = (double)R.n_rows * 4;
  S.steps.push_back(s);
  cache[r] = f.out;
  return f.out;
}

// the input column a (possibly derived bucket-code) column of relation r stands for
static int source_column(const Plan& P, int r, int c) {
  const RelDef& R = P.rels[r];
  if (c < R.n_input_attrs) return c;
  for (const DerivedAttr& D : P.derived)
    if (D.rel == r && D.attr == R.attrs[c]) return R.col.at(D.src);
  return c;
}

// A group of SUM(1) queries with large dense tables (planner: partitioned):
// their cells are counted by radix partition, up to kPartOuts queries per
// launch set, over the relation in its sorted order when a scan of the same
// node sorts it (the views' keys then come in order), else in input order.
static void build_partition(Prep& S, int gi, const void* const* const* cols, hipStream_t st) {
  Plan& P = *S.P;
  GroupDef& G = P.groups[gi];
  const int r = G.node;
  const RelDef& R = P.rels[r];
  NodeData& N = S.nodes[r];
  const std::string gname = "g" + std::to_string(gi) + ":" + R.name;
  int cut = -1;
  for (const GroupDef& H : P.groups)
    if (H.node == r && H.has_program && !H.prog.row_pieces) {
      cut = H.prog.cut;
      break;
    }
  const bool sorted = cut >= 0;
  for (size_t base = 0; base < G.outs.size(); base += kPartOuts) {
    const size_t end = std::min(G.outs.size(), base + (size_t)kPartOuts);
    // relation columns and views the launch set reads
    std::vector<int> views, need;
    for (size_t k = base; k < end; ++k) {
      const QueryDef& Q = P.queries[G.outs[k].id];
      for (auto& kv : Q.in_view)
        if (std::find(views.begin(), views.end(), kv.second) == views.end()) views.push_back(kv.second);
      for (int a : Q.groupby)
        if (R.has(a)) need.push_back(R.col.at(a));
    }
    if ((int)views.size() > kPartViews) throw PlanError{LMFAO_EUNSUPPORTED, "partitioned count with more than 4 views"};
    for (int vid : views)
      for (int a : P.views[vid].key) need.push_back(R.col.at(a));
    std::sort(need.begin(), need.end());
    need.erase(std::unique(need.begin(), need.end()), need.end());
    if (sorted) prepare_node(S, r, cut, need, cols, st);
    auto col = [&](int c) -> const int32_t* {
      if (R.dtypes[c] != LMFAO_I32) throw PlanError{LMFAO_EINVAL, "internal: partitioned key column not int32"};
      return sorted ? (const int32_t*)N.sorted_col[c] : (const int32_t*)raw_column(S, r, c, cols, st);
    };
    DPartCount d{};
    d.n_rows = R.n_rows;
    d.w = filter_weights(S, r, sorted, cols, st);
    d.n_views = (int)views.size();
    for (int v = 0; v < d.n_views; ++v) {
      const ViewDef& V = P.views[views[v]];
      const DView dv = dview_of(S, views[v]);
      // a view of several subtree tuples per key: its count weights the row
      if (!V.unique) d.vmult |= 1u << v;
      d.vcnt[v] = dv.cnt;
      d.vcodes[v] = dv.codes;
      d.vncodes[v] = dv.n_codes;
      d.vnkey[v] = (int)V.key.size();
      d.vnkeys[v] = V.n_keys;
      for (int q = 0; q < d.vnkey[v]; ++q) {
        d.vkey[v][q] = col(R.col.at(V.key[q]));
        d.vstride[v][q] = dv.key_stride[q];
      }
    }
    d.n_out = (int)(end - base);
    std::vector<DCountCopy> copies;
    double rows_bytes = 0;
    for (int o = 0; o < d.n_out; ++o) {
      const int qid = G.outs[base + o].id;
      const QueryDef& Q = P.queries[qid];
      const OutBuf& B = S.qout[qid];
      d.out_cnt[o] = B.cnt;
      d.n_cells[o] = B.n_rows;
      if (B.hash >= 0) {
        d.hashed[o] = 1;
        d.hidx[o] = B.hash;
        d.n_buckets[o] = kPartHashBuckets;
        // SUM(1) components equal the count: added when the table is read
        HashBuf& H = S.hashes[B.hash];
        H.count_copies.clear();
        for (int k = 0; k < B.n_vals; ++k) H.count_copies.push_back(k);
      } else {
        d.n_buckets[o] = (int)((B.n_rows + (1 << kPartShift) - 1) >> kPartShift);
        if (d.n_buckets[o] > kPartMaxBuckets) throw PlanError{LMFAO_EINVAL, "internal: partitioned table too large"};
      }
      for (auto& kv : Q.in_view) {
        const int v = (int)(std::find(views.begin(), views.end(), kv.second) - views.begin());
        d.vmask[o] |= 1u << v;
      }
      d.weighted[o] = (d.vmask[o] & d.vmult) ? 1 : 0;
      const std::vector<int64_t> st_ = strides_of(P, Q.groupby);
      d.nkey[o] = (int)Q.groupby.size();
      for (int k = 0; k < d.nkey[o]; ++k) {
        const int a = Q.groupby[k];
        d.kstride[o][k] = st_[k];
        d.kdom[o][k] = P.attrs[a].domain;
        if (R.has(a)) {
          d.ksrc[o][k] = -1;
          d.kcol[o][k] = col(R.col.at(a));
          d.kslot[o][k] = 0;
          rows_bytes += 4;
        } else {
          d.ksrc[o][k] = -1;
          for (int v = 0; v < d.n_views; ++v)
            if (((d.vmask[o] >> v) & 1u) && P.views[views[v]].slot_of_code(a) >= 0) {
              d.ksrc[o][k] = v;
              d.kslot[o][k] = P.views[views[v]].slot_of_code(a);
              break;
            }
          if (d.ksrc[o][k] < 0) throw PlanError{LMFAO_EINVAL, "internal: partitioned key attribute not found"};
        }
      }
      if (B.n_vals > 0 && B.hash < 0) {
        DCountCopy cc{};
        cc.cnt = B.cnt;
        cc.vals = (double*)B.vals;
        cc.n = B.n_rows;
        cc.nv = B.n_vals;
        cc.n_copy = B.n_vals;
        if (cc.n_copy > kMaxTableComps) throw PlanError{LMFAO_EUNSUPPORTED, "too many SUM(1) components"};
        for (int k = 0; k < cc.n_copy; ++k) cc.comp[k] = k;
        copies.push_back(cc);
      }
    }
    const int64_t n = R.n_rows;
    if (n > (int64_t)INT32_MAX - (1 << 16))
      throw PlanError{LMFAO_EUNSUPPORTED, "partitioned count of a relation of 2^31 rows or more"};
    // entry arrays per kind, tile offsets and per-chunk partial tables
    int n_dense_slots = 0, n_hash_slots = 0, n_weight_slots = 0;
    int64_t toff_total = 0, partial_total = 0;
    for (int o = 0; o < d.n_out; ++o) {
      d.slot[o] = -1;
      d.wslot[o] = -1;
      d.chunks[o] = 1;
      if (d.hashed[o] || d.n_buckets[o] > 1) {
        d.slot[o] = d.hashed[o] ? n_hash_slots++ : n_dense_slots++;
        if (d.weighted[o]) d.wslot[o] = n_weight_slots++;
        d.tile_rows[o] = part_tile_rows(d.hashed[o] != 0, d.weighted[o] != 0);
        d.n_tiles[o] = (int)((n + d.tile_rows[o] - 1) / d.tile_rows[o]);
        d.toff_base[o] = toff_total;
        toff_total += (int64_t)d.n_tiles[o] * (d.n_buckets[o] + 1);
        // about 64 counting workgroups per dense output, each at least 16 tiles
        if (!d.hashed[o])
          d.chunks[o] = (int)std::max<int64_t>(
              1, std::min<int64_t>((64 + d.n_buckets[o] - 1) / d.n_buckets[o], d.n_tiles[o] / 16));
      } else {
        // one slice: chunks of at least 64k rows, at most 64
        d.chunks[o] = (int)std::max<int64_t>(1, std::min<int64_t>(64, n / 65536));
      }
      if (d.chunks[o] > 1) {
        d.partial_base[o] = partial_total;
        partial_total += (int64_t)d.chunks[o] * d.n_cells[o];
      }
    }
    d.toff = toff_total ? (uint32_t*)dalloc(S, (size_t)toff_total * 4) : nullptr;
    d.partial = partial_total ? (uint32_t*)dalloc(S, (size_t)partial_total * 4) : nullptr;
    d.bstart = (uint32_t*)dalloc(S, (size_t)d.n_out * (kPartMaxBuckets + 1) * 4);
    d.btotal = (uint32_t*)dalloc(S, (size_t)d.n_out * kPartMaxBuckets * 4);
    d.part = n_dense_slots ? (uint16_t*)dalloc(S, (size_t)n_dense_slots * std::max<int64_t>(n, 1) * 2) : nullptr;
    // the slice totals of hashed outputs start at zero (k_part_bases zeroes
    // them again after each use)
    launch_fill(d.btotal, (int64_t)d.n_out * kPartMaxBuckets * 4, st);
    HIP_OK(hipGetLastError());
    d.partw = n_weight_slots ? (uint32_t*)dalloc(S, (size_t)n_weight_slots * std::max<int64_t>(n, 1) * 4) : nullptr;
    bool weighted_hashed = false;
    for (int o = 0; o < d.n_out; ++o) weighted_hashed |= d.weighted[o] && d.hashed[o];
    d.partwb = weighted_hashed ? (uint32_t*)dalloc(S, (size_t)n_weight_slots * std::max<int64_t>(n, 1) * 4) : nullptr;
    // per-row bytes and view counts: shared with an earlier launch set of the
    // node that reads the same views in the same row order
    std::string rows_key = std::to_string(r) + (sorted ? ":sorted" : ":raw");
    for (int vid : views) rows_key += "," + std::to_string(vid);
    auto rows_hit = S.part_rows.find(rows_key);
    const bool shared_rows = rows_hit != S.part_rows.end();
    if (shared_rows) {
      d.w8 = rows_hit->second.first;
      for (int v = 0; v < d.n_views; ++v) d.wv[v] = rows_hit->second.second[v];
    } else {
      d.w8 = (uint8_t*)dalloc(S, (size_t)std::max<int64_t>(n, 1));
      for (int v = 0; v < d.n_views; ++v)
        if ((d.vmult >> v) & 1u) d.wv[v] = (uint32_t*)dalloc(S, (size_t)std::max<int64_t>(n, 1) * 4);
      S.part_rows[rows_key] = {d.w8, std::vector<uint32_t*>(d.wv, d.wv + kPartViews)};
    }
    for (int o = 0; o < d.n_out; ++o) {
      d.keys_cols[o] = 1;
      for (int k = 0; k < d.nkey[o]; ++k) {
        d.vkeys_needed |= d.ksrc[o][k] >= 0 ? 1 : 0;
        d.keys_cols[o] &= d.ksrc[o][k] < 0 ? 1 : 0;
      }
    }
    d.part64 = n_hash_slots ? (uint64_t*)dalloc(S, (size_t)n_hash_slots * std::max<int64_t>(n, 1) * 8) : nullptr;
    d.part64b = n_hash_slots ? (uint64_t*)dalloc(S, (size_t)n_hash_slots * std::max<int64_t>(n, 1) * 8) : nullptr;
    d.htab = S.hash_dev;
    d.err_flag = S.err_flag;
    // one step per pass of the launch set (each a kernel of its own, timed
    // and profiled alone): bytes are what the pass must read and write once
    const void* ddev = upload(S, d, st);
    std::set<int> rc(need.begin(), need.end());
    std::vector<int> pcols;
    for (int c : rc) pcols.push_back(source_column(P, r, c));
    std::sort(pcols.begin(), pcols.end());
    pcols.erase(std::unique(pcols.begin(), pcols.end()), pcols.end());
    const std::string suffix = base ? std::to_string(base / kPartOuts) : std::string();
    bool any_single = false, any_multi = false, any_hashed = false, any_chunks = false;
    double key_single = 0, key_multi = 0, key_hashed = 0, cells_single = 0, cells_multi = 0, groups_hashed = 0;
    double part_single = 0, part_multi = 0, outs_multi = 0, outs_hashed = 0, offs = 0, tiles_multi = 0;
    for (int o = 0; o < d.n_out; ++o) {
      const double keys = (double)n * 4 * d.nkey[o];
      if (d.hashed[o]) {
        any_hashed = true;
        key_hashed += keys;
        outs_hashed += 1;
        groups_hashed += (double)std::min<int64_t>(S.hashes[d.hidx[o]].bound, n);
        offs += (double)d.n_tiles[o] * (d.n_buckets[o] + 1) * 4;
      } else if (d.n_buckets[o] <= 1) {
        any_single = true;
        key_single += keys;
        cells_single += (double)d.n_cells[o];
        part_single += d.chunks[o] > 1 ? (double)d.chunks[o] * d.n_cells[o] : 0.0;
      } else {
        any_multi = true;
        key_multi += keys;
        cells_multi += (double)d.n_cells[o];
        outs_multi += 1;
        tiles_multi = std::max(tiles_multi, (double)d.n_tiles[o]);
        part_multi += d.chunks[o] > 1 ? (double)d.chunks[o] * d.n_cells[o] : 0.0;
      }
      any_chunks |= d.chunks[o] > 1;
    }
    auto add_phase = [&](int phase, const char* what, double rd, double wr) {
      Step s;
      s.name = gname + ":" + what + suffix;
      s.kind = 15;
      s.na = phase;
      s.dev = (void*)ddev;
      s.part = d;
      s.rows = n;
      s.grid = (int)((n + part_tile_rows(false, false) - 1) / part_tile_rows(false, false));
      s.alg_read = rd;
      s.alg_write = wr;
      s.relation = r;
      s.pass_cols = pcols;
      S.steps.push_back(s);
    };
    double vkeys = 0, nvm = 0, w_single = 0, w_multi = 0;
    for (int v = 0; v < d.n_views; ++v) {
      vkeys += (double)n * 4 * d.vnkey[v];
      nvm += (d.vmult >> v) & 1u;
    }
    for (int o = 0; o < d.n_out; ++o)
      if (d.weighted[o]) (d.n_buckets[o] <= 1 ? w_single : w_multi) += 1;
    // weighted outputs: the rows' view counts (4 bytes per view) and, past
    // one slice, each entry's weight written and read back
    if (!shared_rows)
      add_phase(kPartPhaseRows, "part_rows", vkeys + (d.w ? (double)n * 4 : 0.0), (double)n * (1 + 4 * nvm));
    if (any_single)
      add_phase(kPartPhaseDirect, "part_direct", key_single + (double)n + (double)n * 4 * nvm * w_single,
                part_single > 0 ? part_single * 4 : cells_single * 8);
    if (any_multi) {
      add_phase(kPartPhaseTile, "part_tile", key_multi + (double)n * outs_multi + (double)n * 4 * nvm * w_multi,
                (double)n * 2 * outs_multi + (double)n * 4 * w_multi + tiles_multi * outs_multi * 4);
      add_phase(kPartPhaseSlices, "part_slices", (double)n * 2 * outs_multi + (double)n * 4 * w_multi,
                part_multi > 0 ? part_multi * 4 : cells_multi * 8);
    }
    if (any_chunks) add_phase(kPartPhaseReduce, "part_reduce", (part_single + part_multi) * 4,
                              (cells_single + cells_multi) * 8);
    if (any_hashed) {
      add_phase(kPartPhaseTileHash, "part_tile_hash", key_hashed + (double)n * outs_hashed,
                (double)n * 8 * outs_hashed + offs);
      add_phase(kPartPhaseHash, "part_hash", (double)n * 8 * outs_hashed + offs, groups_hashed * 16);
    }
    (void)rows_bytes;
    for (const DCountCopy& cc : copies) {
      Step t;
      t.name = gname + ":count_copy";
      t.kind = 13;
      t.dev = upload(S, cc, st);
      t.n = cc.n;
      S.steps.push_back(t);
    }
  }
}

static void build_group(Prep& S, int gi, const void* const* const* cols, hipStream_t st) {
  Plan& P = *S.P;
  GroupDef& G = P.groups[gi];
  if (G.partitioned) {
    build_partition(S, gi, cols, st);
    return;
  }
  const int r = G.node;
  const RelDef& R = P.rels[r];
  NodeData& N = S.nodes[r];
  const bool f64 = S.f64;
  const std::string gname = "g" + std::to_string(gi) + ":" + R.name;

  // --- unique views: direct builds
  for (int vid : G.unique_views) {
    const ViewDef& V = P.views[vid];
    DViewBuild b{};
    b.n_rows = R.n_rows;
    b.w = filter_weights(S, r, false, cols, st);
    std::vector<int> colpos;   // relation columns referenced
    auto cpos = [&](int c) {
      for (size_t i = 0; i < colpos.size(); ++i)
        if (colpos[i] == c) return (int)i;
      if ((int)colpos.size() >= kMaxPieceCols) throw PlanError{LMFAO_EUNSUPPORTED, "too many columns in a view build"};
      colpos.push_back(c);
      return (int)colpos.size() - 1;
    };
    b.nkey = (int)V.key.size();
    std::vector<int64_t> kst = strides_of(P, V.key);
    for (int k = 0; k < b.nkey; ++k) {
      b.key_col[k] = cpos(R.col.at(V.key[k]));
      b.key_stride[k] = kst[k];
    }
    std::vector<int> deps(V.deps.begin(), V.deps.end());
    b.n_views = (int)deps.size();
    if (b.n_views > kMaxViews) throw PlanError{LMFAO_EUNSUPPORTED, "too many views in a view build"};
    for (int i = 0; i < b.n_views; ++i) {
      b.views[i] = dview_of(S, deps[i]);
      const ViewDef& C = P.views[deps[i]];
      for (int k = 0; k < (int)C.key.size(); ++k) b.views[i].key_src[k] = cpos(R.col.at(C.key[k]));
    }
    auto from_view = [&](int a, bool code) {
      for (int i = 0; i < b.n_views; ++i) {
        const ViewDef& C = P.views[deps[i]];
        if ((code ? C.slot_of_code(a) : C.slot_of_attr(a)) >= 0) return i;
      }
      return -1;
    };
    b.n_vals = (int)V.val_attrs.size();
    if (b.n_vals > 64) throw PlanError{LMFAO_EUNSUPPORTED, "view with more than 64 values"};
    for (int s = 0; s < b.n_vals; ++s) {
      int a = V.val_attrs[s];
      if (R.has(a)) {
        b.val_kind[s] = SRC_COL;
        b.val_src[s] = cpos(R.col.at(a));
        b.val_slot[s] = 0;
      } else {
        int i = from_view(a, false);
        if (i < 0) throw PlanError{LMFAO_EINVAL, "internal: value source of view"};
        b.val_kind[s] = SRC_VIEW;
        b.val_src[s] = i;
        b.val_slot[s] = P.views[deps[i]].slot_of_attr(a);
      }
    }
    b.n_codes = (int)V.code_attrs.size();
    if (b.n_codes > kMaxOuterCodes) throw PlanError{LMFAO_EUNSUPPORTED, "view with more than 64 codes"};
    for (int s = 0; s < b.n_codes; ++s) {
      int a = V.code_attrs[s];
      if (R.has(a)) {
        b.code_kind[s] = SRC_COL;
        b.code_src[s] = cpos(R.col.at(a));
      } else {
        int i = from_view(a, true);
        if (i < 0) throw PlanError{LMFAO_EINVAL, "internal: code source of view"};
        b.code_kind[s] = SRC_VIEW;
        b.code_src[s] = i;
        b.code_slot[s] = P.views[deps[i]].slot_of_code(a);
      }
    }
    for (size_t i = 0; i < colpos.size(); ++i) {
      b.cols[i].ptr = raw_column(S, r, colpos[i], cols, st);
      b.cols[i].dtype = R.dtypes[colpos[i]];
    }
    const OutBuf& O = S.vout[vid];
    b.out_cnt = O.cnt;
    b.out_vals = O.vals;
    b.out_codes = O.codes;
    b.err_flag = S.err_flag;
    Step s;
    s.name = gname + ":view_build:V" + std::to_string(vid);
    s.kind = 1;
    s.dev = upload(S, b, st);
    s.n = R.n_rows;
    S.steps.push_back(s);
  }
  if (!G.has_program) return;
  GroupProgram& g = G.prog;

  // program view index -> device descriptors
  std::vector<int> scan_view(g.views.size(), -1), con_view(g.views.size(), -1);
  int n_in = 0, n_out = 0;
  for (size_t k = 0; k < g.views.size(); ++k) {
    if (g.view_outer[k]) con_view[k] = n_out++;
    else scan_view[k] = n_in++;
  }
  auto remap_mask = [&](uint32_t m, const std::vector<int>& map) {
    uint32_t o = 0;
    for (size_t k = 0; k < map.size(); ++k)
      if ((m >> k) & 1u) {
        if (map[k] < 0) throw PlanError{LMFAO_EINVAL, "internal: mask view on wrong side"};
        o |= 1u << map[k];
      }
    return o;
  };

  void* psi_f = nullptr;
  int32_t* psi_i = nullptr;
  int psi_f_stride = 0, psi_i_stride = 0;
  std::vector<int> pcols_key;   // contract piece columns (order positions or relation columns)
  pcols_key = g.piece_cols;

  if (!g.row_pieces) {
    // ---- scan descriptor
    std::vector<int> scols = g.scan_cols;
    auto scol = [&](int c) {
      for (size_t i = 0; i < scols.size(); ++i)
        if (scols[i] == c) return (int)i;
      if ((int)scols.size() >= kMaxScanCols) throw PlanError{LMFAO_EUNSUPPORTED, "too many scanned columns"};
      scols.push_back(c);
      return (int)scols.size() - 1;
    };
    DScan d{};
    if (n_in > kMaxInnerViews) throw PlanError{LMFAO_EUNSUPPORTED, "more than 4 views looked up per tuple"};
    d.n_views = n_in;
    for (size_t k = 0; k < g.views.size(); ++k) {
      if (scan_view[k] < 0) continue;
      DView v = dview_of(S, g.views[k]);
      const ViewDef& V = P.views[g.views[k]];
      for (int q = 0; q < (int)V.key.size(); ++q) v.key_src[q] = scol(R.col.at(V.key[q]));
      d.views[scan_view[k]] = v;
    }
    if (g.in_masks.size() > (size_t)kMaxMasks) throw PlanError{LMFAO_EUNSUPPORTED, "too many inner masks"};
    d.n_masks = (int)g.in_masks.size();
    auto mask_idx = [&](uint32_t m) {
      for (size_t i = 0; i < g.in_masks.size(); ++i)
        if (g.in_masks[i] == m) return (int)i;
      throw PlanError{LMFAO_EINVAL, "internal: unknown mask"};
    };
    for (int i = 0; i < d.n_masks; ++i) d.masks[i] = remap_mask(g.in_masks[i], scan_view);
    // atoms, with duplicates where two float entries need one triangle slot under different masks
    std::vector<AtomRef> atoms = g.in_atoms;
    std::vector<std::pair<int, int>> ent(g.psi_f.size());
    std::map<std::pair<int, int>, int> taken;   // (ai,aj) -> mask idx
    for (size_t e = 0; e < g.psi_f.size(); ++e) {
      int ai = g.psi_f[e].ai, aj = g.psi_f[e].aj;
      int mi = mask_idx(g.psi_f[e].imask);
      auto it = taken.find({ai, aj});
      if (it != taken.end() && it->second != mi) {
        int src = aj >= 0 ? aj : ai;
        atoms.push_back(atoms[src]);
        int dup = (int)atoms.size() - 1;
        if (aj >= 0) aj = dup; else ai = dup;
        if (ai > aj) std::swap(ai, aj);
      }
      taken[{ai, aj}] = mi;
      ent[e] = {ai, aj};
    }
    const int NA = (int)atoms.size();
    if (NA > kMaxAtoms) throw PlanError{LMFAO_EUNSUPPORTED, "more than 8 inner factors at " + R.name};
    d.n_atoms = NA;
    // column atoms already hold their position in the scanned-column list
    auto atom_dev = [&](const AtomRef& a) {
      DAtom x{};
      x.kind = a.kind;
      x.src = a.kind == SRC_COL ? a.src : scan_view[a.src];
      x.slot = a.slot;
      return x;
    };
    for (int i = 0; i < NA; ++i) d.atoms[i] = atom_dev(atoms[i]);
    if (g.in_codes.size() > (size_t)kMaxCodes) throw PlanError{LMFAO_EUNSUPPORTED, "too many inner codes"};
    d.n_codes = (int)g.in_codes.size();
    for (int i = 0; i < d.n_codes; ++i) d.codes[i] = atom_dev(g.in_codes[i]);
    // float entries on the extended triangle (index 0 = constant 1)
    auto tri = [&](int i, int j) { return i * (NA + 1) - i * (i - 1) / 2 + (j - i); };
    d.pf_need = 0;
    for (int t = 0; t < kTriangle; ++t) { d.pf_slot[t] = -1; d.pf_mask[t] = 0; }
    bool uniform = true;
    int first_mask = -1;
    for (size_t e = 0; e < g.psi_f.size(); ++e) {
      int t = tri(ent[e].first + 1, ent[e].second + 1);
      if (t == 0 || t >= 64) throw PlanError{LMFAO_EINVAL, "internal: float entry index"};
      d.pf_need |= 1ull << t;
      d.pf_slot[t] = (int)e;
      int mi = mask_idx(g.psi_f[e].imask);
      d.pf_mask[t] = (int8_t)mi;
      if (first_mask < 0) first_mask = mi;
      uniform &= mi == first_mask;
    }
    d.pf_uniform = uniform ? 1 : 0;
    d.pf_mask_idx = first_mask < 0 ? 0 : first_mask;
    d.pf_n = (int)g.psi_f.size();
    if (g.psi_i.size() > (size_t)kMaxMasks) throw PlanError{LMFAO_EUNSUPPORTED, "too many count entries"};
    d.n_pi = (int)g.psi_i.size();
    for (int i = 0; i < d.n_pi; ++i) d.pi_mask_idx[i] = mask_idx(g.psi_i[i]);
    // distinct per-tuple weights of histograms and direct tables
    std::vector<DWeight> weights;
    auto weight_idx = [&](int is_float, int ai, int aj, int mi) {
      if (ai > aj) std::swap(ai, aj);
      for (size_t i = 0; i < weights.size(); ++i)
        if (weights[i].is_float == is_float && weights[i].ai == ai && weights[i].aj == aj &&
            weights[i].mask_idx == mi)
          return (int)i;
      if ((int)weights.size() >= kMaxWeightTable) throw PlanError{LMFAO_EUNSUPPORTED, "too many distinct scan weights"};
      weights.push_back(DWeight{is_float, ai, aj, mi});
      return (int)weights.size() - 1;
    };
    uint32_t run_codes = 0;
    if (g.hists.size() > (size_t)kMaxHists) throw PlanError{LMFAO_EUNSUPPORTED, "too many histograms"};
    d.n_hists = (int)g.hists.size();
    for (int i = 0; i < d.n_hists; ++i) {
      const HistDef& h = g.hists[i];
      int wi = h.is_float ? weight_idx(1, h.ai, h.aj, mask_idx(h.imask)) : weight_idx(0, -1, -1, mask_idx(h.imask));
      d.hists[i] = DHist{h.code, h.dom, h.is_float, wi, h.offset, 0};
      run_codes |= 1u << h.code;
    }
    d.hist_i_bins = g.hist_i_bins;
    d.hist_f_bins = g.hist_f_bins;
    // direct tables
    int ntab = 0;
    int lds_used = 0;
    uint32_t tab_omask = 0;
    bool tab_omask_set = false;
    std::vector<std::pair<int, int>> lds_tables;   // (output index, lds offset)
    std::map<int, std::vector<int>> table_copies;    // output index -> SUM(1) components copied from the count
    std::vector<DCountCopy> count_copies;             // the same for tables kept in global memory
    for (size_t oi = 0; oi < g.outs.size(); ++oi) {
      const ProgOutput& po = g.outs[oi];
      if (po.mode != 2) continue;
      if (ntab >= kMaxTables) throw PlanError{LMFAO_EUNSUPPORTED, "too many direct group-by tables"};
      DTable& T = d.tables[ntab++];
      T.ncode = (int)po.key_codes.size();
      if (T.ncode > 3) throw PlanError{LMFAO_EUNSUPPORTED, "table key with more than 3 attributes"};
      for (int k = 0; k < T.ncode; ++k) {
        T.code[k] = po.key_codes[k];
        T.stride[k] = po.key_stride[k];
      }
      T.n_rows = po.n_rows;
      if (po.tcomps.size() > (size_t)kMaxTableComps) throw PlanError{LMFAO_EUNSUPPORTED, "too many table components"};
      const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
      const bool in_lds = lds_used + po.n_rows <= kLdsTableMax;
      // a SUM(1) component under the count's mask equals the count: an LDS
      // table writes it from the reduced counts instead of accumulating it
      uint32_t count_mask = 0;
      for (const TableComp& tc : po.tcomps)
        if (tc.comp < 0) count_mask = tc.imask;
      std::vector<int> copies;
      T.n_tcomps = 0;
      for (const TableComp& tc : po.tcomps) {
        if (tc.comp >= 0 && tc.ai < 0 && tc.aj < 0 && tc.imask == count_mask && O.f64) {
          copies.push_back(tc.comp);
          continue;
        }
        T.tcomp[T.n_tcomps] = tc.comp;
        T.twi[T.n_tcomps] = tc.comp < 0 ? weight_idx(0, -1, -1, mask_idx(tc.imask))
                                        : weight_idx(1, tc.ai, tc.aj, mask_idx(tc.imask));
        T.n_tcomps++;
      }
      table_copies[(int)oi] = copies;
      for (int k = 0; k < T.ncode; ++k) run_codes |= 1u << T.code[k];
      T.cnt = O.cnt;
      T.vals = O.vals;
      T.vals_f64 = O.f64 ? 1 : 0;
      T.n_vals = O.n_vals;
      if (in_lds) {
        T.lds = 1;
        T.lds_off = lds_used;
        lds_tables.push_back({(int)oi, lds_used});
        lds_used += (int)po.n_rows;
      } else if (!copies.empty()) {
        // a global table's SUM(1) components: copied from its counts after the scan
        DCountCopy cc{};
        cc.cnt = O.cnt;
        cc.vals = (double*)O.vals;
        cc.n = po.n_rows;
        cc.nv = O.n_vals;
        cc.n_copy = (int)copies.size();
        for (size_t k = 0; k < copies.size(); ++k) cc.comp[k] = copies[k];
        count_copies.push_back(cc);
      }
      if (po.omask) {
        if (tab_omask_set && tab_omask != po.omask)
          throw PlanError{LMFAO_EUNSUPPORTED, "direct tables with different outer multiplicities"};
        tab_omask = po.omask;
        tab_omask_set = true;
      }
    }
    d.n_tables = ntab;
    d.lds_tab_i = lds_used;
    d.n_weights = (int)weights.size();
    for (size_t i = 0; i < weights.size(); ++i) d.weights[i] = weights[i];
    d.run_codes = run_codes;
    d.mu_out_views = 0;
    for (size_t k = 0; k < g.views.size(); ++k) {
      if (!((tab_omask >> k) & 1u)) continue;
      DView v = dview_of(S, g.views[k]);
      const ViewDef& V = P.views[g.views[k]];
      std::vector<int> pos(V.key.size());
      for (int q = 0; q < (int)V.key.size(); ++q) {
        auto it = std::find(g.order.begin(), g.order.end(), V.key[q]);
        v.key_src[q] = (int)(it - g.order.begin());
      }
      d.outer_views[d.mu_out_views++] = v;
    }
    // columns and pieces
    std::vector<int> need = scols;
    prepare_node(S, r, g.cut, need, cols, st);
    d.w = filter_weights(S, r, true, cols, st);   // needs the sort permutation
    d.n_cols = (int)scols.size();
    for (int i = 0; i < d.n_cols; ++i) {
      d.cols[i].ptr = N.sorted_col[scols[i]];
      d.cols[i].dtype = R.dtypes[scols[i]];
    }
    d.piece_key = N.piece_key;
    d.n_piece_key = g.cut;
    d.n_pieces = N.n_pieces;
    d.piece_begin = N.piece_begin;
    d.item_piece = N.item_piece;
    d.n_items = N.n_items;
    psi_f_stride = d.pf_n + d.hist_f_bins;
    psi_i_stride = d.n_pi + d.hist_i_bins;
    d.psi_f_stride = psi_f_stride;
    d.psi_i_stride = psi_i_stride;
    psi_f = dalloc(S, (size_t)std::max<int64_t>(1, N.n_pieces) * std::max(1, psi_f_stride) * (f64 ? 8 : 4));
    psi_i = (int32_t*)dalloc(S, (size_t)std::max<int64_t>(1, N.n_pieces) * std::max(1, psi_i_stride) * 4);
    d.psi_f = psi_f;
    d.psi_i = psi_i;
    d.err_flag = S.err_flag;
    // lean scans: inner views through per-key images (keys of at most two
    // attributes), at most 2 inner views, one multiplicity mask for all float
    // entries, count-only direct tables.  The built-in lean kernel takes 4
    // codes and 4 tables; a generated one takes 16 codes and 8 tables.
    bool lean = n_in <= 2 && d.n_codes <= kMaxCodes && d.n_masks <= 4 && d.n_pi <= 4 &&
                R.n_rows < ((int64_t)1 << 31) && d.n_hists <= kFastHists && d.n_tables <= kGenTables &&
                d.pf_uniform;
    d.n_atoms = NA;
    for (int v = 0; v < n_in; ++v)
      lean = lean && d.views[v].n_keys < ((int64_t)1 << 31) && d.views[v].nkey <= 2;
    for (int i = 0; i < d.n_hists; ++i) lean = lean && d.hists[i].offset + d.hists[i].dom < (1 << 19);
    // tables: keys of at most 3 codes, at most one count component; value
    // components (generated scans only) go to FP64 outputs
    bool counts_only = true;
    for (int t = 0; t < d.n_tables; ++t) {
      const DTable& TB = d.tables[t];
      int n_cnt = 0;
      bool vals = false;
      for (int k = 0; k < TB.n_tcomps; ++k) {
        if (TB.tcomp[k] < 0) ++n_cnt;
        else vals = true;
      }
      lean = lean && TB.ncode <= 3 && TB.n_rows < ((int64_t)1 << 31) && n_cnt <= 1 && (!vals || TB.vals_f64);
      counts_only = counts_only && TB.n_tcomps == 1 && TB.tcomp[0] < 0;
    }
    const bool builtin = lean && counts_only && d.n_codes <= 4 && d.n_tables <= kFastTables;
    const bool fast = builtin || (lean && S.P->opts.codegen == 0);
    d.fast = fast ? 1 : 0;
    // generated scans gain from more resident wavefronts; the built-in ones
    // (descriptor-driven, more registers) do best with fewer
    const int waves = scan_waves_per_block();
    const bool expect_gen = lean && S.P->opts.codegen == 0;
    // and every workgroup keeps at least 2048 rows, so that on a small
    // relation the per-workgroup partial tables stay cheap to merge
    const int max_blocks =
        S.P->opts.scan_blocks > 0
            ? S.P->opts.scan_blocks
            : (int)std::min<int64_t>(expect_gen ? 2048 : 512, std::max<int64_t>(256, (R.n_rows + 2047) / 2048));
    int grid = (int)std::min<int64_t>((N.n_items + waves - 1) / waves, max_blocks);
    grid = std::max(grid, 1);
    d.part_i = (int32_t*)dalloc(S, (size_t)grid * std::max(1, lds_used) * 4);
    if (fast) {
      DFast& F = d.F;
      for (int a = 0; a < NA; ++a)
        F.fcol[a] = atoms[a].kind == SRC_COL ? typed_sorted_column(S, r, scols[atoms[a].src], st) : nullptr;
      for (int c = 0; c < kMaxCodes; ++c)
        F.ccol[c] = (c < d.n_codes && g.in_codes[c].kind == SRC_COL)
                        ? (const int32_t*)N.sorted_col[scols[g.in_codes[c].src]] : (const int32_t*)nullptr;
      F.n_hist = d.n_hists;
      // per-lane register histograms pay off when a piece spans at least one
      // 64-row chunk (their wavefront sums are taken once per piece)
      F.reg_hist_bins = R.n_rows >= 64 * std::max<int64_t>(1, N.n_pieces) ? 16 : 0;
      // a lane adds at most ceil(kPieceMax / 64) rows of one piece to a bin:
      // with multiplicities 0 or 1 an 8-bit field holds it (cleared below for
      // inner views of several tuples per key)
      static_assert(kPieceMax / 64 < 256, "8-bit register histogram fields");
      F.mult01 = 1;
      for (int i = 0; i < d.n_hists; ++i) {
        const DHist& H = d.hists[i];
        F.hcode[i] = (int8_t)H.code;
        const DWeight& Wt = weights[H.wi];
        // factor slots: 0 is the constant 1, so an absent factor multiplies by 1
        // the packed code field holds the built-in kernel's 4 codes; the full
        // index (generated kernels take 16 codes) is in hcode
        uint32_t w = ((uint32_t)H.code & 3u) | ((uint32_t)Wt.mask_idx << 2) | ((uint32_t)(H.is_float ? 1 : 0) << 4);
        if (H.is_float) w |= ((uint32_t)(Wt.ai + 1) << 5) | ((uint32_t)(Wt.aj + 1) << 9);
        w |= (uint32_t)H.offset << 13;
        F.hword[i] = w;
      }
      F.n_tab = d.n_tables;
      for (int t = 0; t < d.n_tables; ++t) {
        const DTable& TB = d.tables[t];
        F.tab_ncode[t] = TB.ncode;
        for (int k = 0; k < TB.ncode; ++k) {
          F.tab_code[t][k] = TB.code[k];
          F.tab_stride[t][k] = (int32_t)TB.stride[k];
        }
        F.tab_mask[t] = 0;
        F.tab_has_cnt[t] = 0;
        F.tab_nvc[t] = 0;
        for (int k = 0; k < TB.n_tcomps; ++k) {
          const DWeight& Wk = weights[TB.twi[k]];
          if (TB.tcomp[k] < 0) {
            F.tab_has_cnt[t] = 1;
            F.tab_mask[t] = Wk.mask_idx;
          } else {
            F.tab_vcomp[t][F.tab_nvc[t]] = TB.tcomp[k];
            F.tab_vw[t][F.tab_nvc[t]] = (Wk.ai + 1) | ((Wk.aj + 1) << 4) | (Wk.mask_idx << 8);
            F.tab_nvc[t]++;
          }
        }
        F.tab_vals[t] = (double*)TB.vals;
        F.tab_nv[t] = TB.n_vals;
        F.tab_lds[t] = TB.lds;
        F.tab_off[t] = TB.lds_off;
        F.tab_cnt[t] = TB.cnt;
      }
      const int W = image_width_dw(NA, f64, d.n_codes);
      const int code_off = image_code_off(NA, f64);
      const int code_slots = image_code_slots(d.n_codes);
      for (size_t k = 0; k < g.views.size(); ++k) {
        int v = scan_view[k];
        if (v < 0) continue;
        const DView& V = d.views[v];
        if (!P.views[g.views[k]].unique) F.mult01 = 0;
        DImageBuild ib{};
        ib.view = V;
        ib.n_keys = V.n_keys;
        ib.width_dw = W;
        ib.code_off = code_off;
        ib.cnt_off = code_off + code_slots;
        ib.t_f64 = f64 ? 1 : 0;
        ib.n_atoms = NA;
        for (int a = 0; a < NA; ++a)
          ib.atom_slot[a] = (atoms[a].kind == SRC_VIEW && atoms[a].src == (int)k) ? atoms[a].slot : -1;
        ib.n_codes = d.n_codes;
        for (int c = 0; c < d.n_codes; ++c)
          ib.code_slot[c] = (g.in_codes[c].kind == SRC_VIEW && g.in_codes[c].src == (int)k) ? g.in_codes[c].slot : -1;
        ib.img = dalloc(S, (size_t)V.n_keys * W * 4);
        d.imgs[v].img = ib.img;
        d.imgs[v].width_dw = W;
        d.imgs[v].code_off = code_off;
        d.imgs[v].cnt_off = code_off + code_slots;
        d.imgs[v].key_col = V.nkey == 1 ? V.key_src[0] : -1;
        F.img[v] = ib.img;
        for (int k = 0; k < 2; ++k) {
          F.kcol[v][k] = k < V.nkey ? (const int32_t*)N.sorted_col[scols[V.key_src[k]]] : nullptr;
          F.kmul[v][k] = k < V.nkey ? (int32_t)V.key_stride[k] : 0;
        }
        Step b;
        b.name = gname + ":image";
        b.kind = 6;
        b.dev = upload(S, ib, st);
        b.n = V.n_keys;
        b.alg_read = (double)V.n_keys * (8 + V.n_vals * (V.vals_f64 ? 8 : 4) + V.n_codes * 4);
        b.alg_write = (double)V.n_keys * W * 4;
        S.steps.push_back(b);
      }
    }
    int lds = builtin ? scan_fast_lds_bytes(d, f64) : scan_lds_bytes(d, f64);
    if (lds > 160 * 1024) throw PlanError{LMFAO_EUNSUPPORTED, "scan needs more LDS than a CU has"};
    {
      // multiplicities of multi-valued views reach the scan's 32-bit counters
      // (per-piece counts, LDS tables summed per workgroup, image records):
      // check their range on the device before the scan
      DMultCheck mc{};
      for (int vid : g.views)
        if (!P.views[vid].unique && mc.n < kMaxViews) {
          mc.cnt[mc.n] = S.vout[vid].cnt;
          mc.n_keys[mc.n] = S.vout[vid].n_rows;
          mc.n++;
        }
      if (mc.n) {
        const int64_t per_block = (N.n_items + (int64_t)grid * waves - 1) / ((int64_t)grid * waves);
        mc.rows = (double)std::min<int64_t>(R.n_rows, per_block * waves * std::max<int64_t>(N.max_item_rows, 1));
        mc.maxv = (unsigned long long*)dalloc(S, kMaxViews * 8);
        HIP_OK(hipMemsetAsync(mc.maxv, 0, kMaxViews * 8, st));
        mc.err_flag = S.err_flag;
        Step m;
        m.name = gname + ":mult_check";
        m.kind = 14;
        m.dev = upload(S, mc, st);
        m.mult = mc;
        S.steps.push_back(m);
      }
    }
    Step s;
    s.name = gname + ":scan";
    s.kind = 2;
    s.fast = builtin ? 1 : 0;
    s.dev = upload(S, d, st);
    if (fast && S.P->opts.codegen == 0) {
      GenKernel gk;
      std::string why;
      if (gen_scan_kernel(d, NA, f64, gname, gk, why)) {
        s.gen_fn = gk.fn;
        s.gen_args = upload_vec(S, gk.args, st);
        s.gen_block = gk.block;
        lds = gk.lds;
        S.gen_sources.push_back(gname + "\n" + gk.source);
      } else {
        S.gen_failures.push_back(gname + ": " + why);
      }
    }
    s.na = NA;
    s.grid = grid;
    s.lds = lds;
    // bytes the scan must move: each scanned column once, the piece offsets,
    // each inner view's rows once, the per-piece partial sums (the per-block
    // table partials depend on the launch, not on the work, and are left out)
    s.rows = R.n_rows;
    s.pieces = N.n_pieces;
    for (int i = 0; i < d.n_cols; ++i) s.alg_read += (double)R.n_rows * (d.cols[i].dtype == LMFAO_F64 ? 8 : 4);
    s.alg_read += (double)(N.n_pieces + 1) * 8 + (double)(N.n_items + 1) * 4;
    for (int v = 0; v < d.n_views; ++v)
      s.alg_read += fast ? (double)d.views[v].n_keys * d.imgs[v].width_dw * 4
                         : (double)d.views[v].n_keys * (8 + d.views[v].n_vals * (d.views[v].vals_f64 ? 8 : 4) +
                                                        d.views[v].n_codes * 4);
    s.alg_write += (double)N.n_pieces * (psi_f_stride * (f64 ? 8 : 4) + psi_i_stride * 4);
    s.alg_flop = (double)R.n_rows * 2 * (double)std::max(1, d.pf_n);
    {
      std::set<int> rc;
      for (int c : scols) rc.insert(source_column(P, r, c));
      for (int l = 0; l < g.cut && l < (int)g.order.size(); ++l) rc.insert(source_column(P, r, R.col.at(g.order[l])));
      s.relation = r;
      s.pass_cols.assign(rc.begin(), rc.end());
    }
    S.steps.push_back(s);
    for (auto& lt : lds_tables) {
      const ProgOutput& po = g.outs[lt.first];
      const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
      DTableReduce tr{};
      tr.n = po.n_rows;
      tr.n_blocks = grid;
      tr.stride = lds_used;
      tr.off = lt.second;
      tr.part_i = d.part_i;
      tr.dst_cnt = O.cnt;
      const std::vector<int>& cp = table_copies[lt.first];
      tr.copy_vals = (double*)O.vals;
      tr.copy_nv = O.n_vals;
      tr.n_copy = (int)cp.size();
      for (size_t k = 0; k < cp.size(); ++k) tr.copy_comp[k] = cp[k];
      Step t;
      t.name = gname + ":table_reduce";
      t.kind = 3;
      t.dev = upload(S, tr, st);
      t.n = po.n_rows;
      t.n_blocks = grid;
      S.steps.push_back(t);
    }
    for (const DCountCopy& cc : count_copies) {
      Step t;
      t.name = gname + ":count_copy";
      t.kind = 13;
      t.dev = upload(S, cc, st);
      t.n = cc.n;
      S.steps.push_back(t);
    }
  }

  // ---- contraction
  if (g.feats.empty() && g.scatter.empty()) return;
  DContract c{};
  std::vector<int> pk = pcols_key;
  auto pcol = [&](int key) {
    for (size_t i = 0; i < pk.size(); ++i)
      if (pk[i] == key) return (int)i;
    if ((int)pk.size() >= kMaxPieceCols) throw PlanError{LMFAO_EUNSUPPORTED, "too many piece columns"};
    pk.push_back(key);
    return (int)pk.size() - 1;
  };
  c.n_views = n_out;
  for (size_t k = 0; k < g.views.size(); ++k) {
    if (con_view[k] < 0) continue;
    DView v = dview_of(S, g.views[k]);
    const ViewDef& V = P.views[g.views[k]];
    for (int q = 0; q < (int)V.key.size(); ++q) {
      int a = V.key[q];
      int key;
      if (g.row_pieces) key = R.col.at(a);
      else key = (int)(std::find(g.order.begin(), g.order.end(), a) - g.order.begin());
      v.key_src[q] = pcol(key);
    }
    c.views[con_view[k]] = v;
  }
  // masks of the features
  std::vector<uint32_t> cmasks;
  auto cmask_idx = [&](uint32_t m) {
    for (size_t i = 0; i < cmasks.size(); ++i)
      if (cmasks[i] == m) return (int)i;
    cmasks.push_back(m);
    return (int)cmasks.size() - 1;
  };
  std::vector<DFeat> feats;
  for (auto& f : g.feats)
    feats.push_back(DFeat{cmask_idx(f.mask), f.c1, f.v1, f.c2, f.v2, f.a1, f.a2, 0});
  if (cmasks.empty()) cmask_idx(0);
  if (cmasks.size() > (size_t)kMaxMasks * 4) throw PlanError{LMFAO_EUNSUPPORTED, "too many outer masks"};
  c.n_masks = (int)cmasks.size();
  for (int i = 0; i < c.n_masks; ++i) c.masks[i] = remap_mask(cmasks[i], con_view);
  std::vector<DColB> colsb;
  for (auto& cd : g.cols) {
    DColB b{};
    b.kind = cd.kind;
    b.entry = cd.entry;
    b.bin = 0;
    b.feat = DFeat{0, cd.feat.c1, cd.feat.v1, cd.feat.c2, cd.feat.v2, cd.feat.a1, cd.feat.a2, 0};
    colsb.push_back(b);
  }
  if (g.out_atoms.size() > (size_t)kMaxOuterAtoms) throw PlanError{LMFAO_EUNSUPPORTED, "too many outer factors"};
  if (g.out_codes.size() > (size_t)kMaxOuterCodes) throw PlanError{LMFAO_EUNSUPPORTED, "too many outer codes"};
  // column atoms and codes already hold their position in the piece-column list
  c.n_atoms = (int)g.out_atoms.size();
  for (int i = 0; i < c.n_atoms; ++i) {
    const AtomRef& a = g.out_atoms[i];
    c.atoms[i] = DAtom{a.kind, a.kind == SRC_COL ? a.src : con_view[a.src], a.slot, 0};
  }
  c.n_codes = (int)g.out_codes.size();
  for (int i = 0; i < c.n_codes; ++i) {
    const AtomRef& a = g.out_codes[i];
    c.codes[i] = DAtom{a.kind, a.kind == SRC_COL ? a.src : con_view[a.src], a.slot, 0};
  }
  int64_t n_pieces;
  if (g.row_pieces) {
    n_pieces = R.n_rows;
    c.w = filter_weights(S, r, false, cols, st);
    c.n_pcols = (int)pk.size();
    for (int i = 0; i < c.n_pcols; ++i) {
      c.pcols[i].ptr = raw_column(S, r, pk[i], cols, st);
      c.pcols[i].dtype = R.dtypes[pk[i]];
    }
    c.row_pieces = 1;
  } else {
    n_pieces = N.n_pieces;
    c.n_pcols = (int)pk.size();
    for (int i = 0; i < c.n_pcols; ++i) {
      c.pcols[i].ptr = N.piece_key + (int64_t)pk[i] * N.n_pieces;
      c.pcols[i].dtype = LMFAO_I32;
    }
    c.row_pieces = 0;
    c.psi_f = psi_f;
    c.psi_i = psi_i;
    c.psi_f_stride = psi_f_stride;
    c.psi_i_stride = psi_i_stride;
  }
  c.n_pieces = n_pieces;
  c.n_feat = (int)feats.size();
  c.n_feat_int = g.n_feat_int;
  c.n_col = (int)colsb.size();
  c.n_col_int = g.n_col_int;

  c.feats = upload_vec(S, feats, st);
  c.cols = upload_vec(S, colsb, st);
  // about one block row per CU; the FP64 accumulators make long chains safe
  int64_t ppb = std::max<int64_t>(64, (n_pieces + 255) / 256);
  int grid_x = (int)std::max<int64_t>(1, (n_pieces + ppb - 1) / ppb);
  int tiles = contract_tiles(c.n_feat, c.n_col);
  int64_t icells = (int64_t)c.n_feat_int * c.n_col_int;
  int grid_y = std::max(1, (tiles + contract_threads() - 1) / contract_threads());
  grid_y = std::max<int>(grid_y, (int)((icells + contract_max_int_cells() - 1) / contract_max_int_cells()));
  c.pieces_per_block = (int32_t)ppb;
  // scatter
  std::vector<int32_t> sc_out, sc_comp, sc_f, sc_g;
  for (auto& sc : g.scatter) {
    sc_out.push_back(sc.out);
    sc_comp.push_back(sc.comp);
    sc_f.push_back(sc.f);
    sc_g.push_back(sc.g);
  }
  c.n_scatter = (int)g.scatter.size();
  c.sc_out = upload_vec(S, sc_out, st);
  c.sc_comp = upload_vec(S, sc_comp, st);
  c.sc_f = upload_vec(S, sc_f, st);
  c.sc_g = upload_vec(S, sc_g, st);
  std::vector<int64_t> so_stride;
  std::vector<int32_t> so_code, so_ncomp, so_f64, so_hash;
  std::vector<int64_t*> so_cnt;
  std::vector<void*> so_vals;
  for (auto& po : g.outs) {
    const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
    for (int k = 0; k < 3; ++k) {
      if (po.mode == 1 && k < (int)po.key_codes.size()) {
        so_code.push_back(po.key_codes[k]);
        so_stride.push_back(po.key_stride[k]);
      } else {
        so_code.push_back(-1);
        so_stride.push_back(0);
      }
    }
    if (po.mode == 1 && po.key_codes.size() > 3) throw PlanError{LMFAO_EUNSUPPORTED, "scatter key with > 3 codes"};
    so_ncomp.push_back(O.n_vals);
    so_f64.push_back(O.f64 ? 1 : 0);
    so_cnt.push_back(O.cnt);
    so_vals.push_back(O.vals);
    so_hash.push_back(po.ref.kind == 0 ? O.hash : -1);
    if (O.hash >= 0 && po.mode != 1)
      throw PlanError{LMFAO_EINVAL, "internal: hashed output not in scatter mode"};
  }
  c.so_hash_idx = upload_vec(S, so_hash, st);
  c.hash_tab = S.hash_dev;
  c.so_stride = upload_vec(S, so_stride, st);
  c.so_code = upload_vec(S, so_code, st);
  c.so_ncomp = upload_vec(S, so_ncomp, st);
  c.so_vals_f64 = upload_vec(S, so_f64, st);
  c.so_cnt = upload_vec(S, so_cnt, st);
  c.so_vals = upload_vec(S, so_vals, st);
  if (S.P->opts.contraction == LMFAO_CONTRACT_MFMA) {
    const size_t first = S.steps.size();
    build_contract_mfma(S, g, gname, c, n_pieces, psi_f_stride, psi_i_stride, f64, st);
    if (g.row_pieces) {
      // a row-by-row pass reads the relation's columns itself
      std::set<int> rc;
      for (int c2 : pk) rc.insert(source_column(P, r, c2));
      for (size_t i = first; i < S.steps.size(); ++i)
        if (S.steps[i].kind == 12 || S.steps[i].kind == 8) {
          S.steps[i].relation = r;
          S.steps[i].pass_cols.assign(rc.begin(), rc.end());
        }
    }
    return;
  }
  c.part_f = (double*)dalloc(S, (size_t)grid_x * std::max(1, c.n_feat * c.n_col) * 8);
  c.part_i = (int64_t*)dalloc(S, (size_t)grid_x * std::max(1, c.n_feat_int * c.n_col_int) * 8);
  int lds = contract_lds_bytes(c, f64);
  if (lds > 160 * 1024) throw PlanError{LMFAO_EUNSUPPORTED, "contraction needs more LDS than a CU has"};
  Step s;
  s.name = gname + ":contract";
  s.kind = 4;
  s.dev = upload(S, c, st);
  s.grid = grid_x;
  s.grid_y = grid_y;
  s.lds = lds;
  s.pieces = n_pieces;
  s.rows = g.row_pieces ? R.n_rows : N.n_pieces;
  for (int i = 0; i < c.n_pcols; ++i) s.alg_read += (double)n_pieces * (c.pcols[i].dtype == LMFAO_F64 ? 8 : 4);
  s.alg_read += (double)n_pieces * (psi_f_stride * (f64 ? 8 : 4) + psi_i_stride * 4);
  for (int v = 0; v < c.n_views; ++v)
    s.alg_read += (double)std::min<int64_t>(c.views[v].n_keys, n_pieces) *
                  (8 + c.views[v].n_vals * (c.views[v].vals_f64 ? 8 : 4) + c.views[v].n_codes * 4);
  s.alg_write += (double)grid_x * ((double)c.n_feat * c.n_col * 8 + (double)icells * 8);
  s.alg_flop = 2.0 * (double)n_pieces * c.n_feat * c.n_col;
  S.steps.push_back(s);
  // merge cells
  if (!g.gemm_cells.empty()) {
    std::vector<DCell> cells;
    for (auto& gc : g.gemm_cells) {
      const ProgOutput& po = g.outs[gc.second.out];
      const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
      DCell x{};
      x.f = gc.first.first;
      x.g = gc.first.second;
      x.is_int = (x.f < c.n_feat_int && x.g < c.n_col_int) ? 1 : 0;
      x.vals_f64 = O.f64 ? 1 : 0;
      if (gc.second.comp < 0) {
        if (!x.is_int) throw PlanError{LMFAO_EINVAL, "internal: count cell not integral"};
        x.cnt = O.cnt;
        x.vals = nullptr;
        x.idx = gc.second.row;
      } else {
        x.cnt = nullptr;
        x.vals = O.vals;
        x.idx = gc.second.row * O.n_vals + gc.second.comp;
      }
      cells.push_back(x);
    }
    Step m;
    m.name = gname + ":merge";
    m.kind = 5;
    m.dev = upload_vec(S, cells, st);
    m.n = (int64_t)cells.size();
    m.part_f = c.part_f;
    m.part_i = c.part_i;
    m.n_blocks = grid_x;
    m.NF = c.n_feat;
    m.NG = c.n_col;
    m.NFI = c.n_feat_int;
    m.NGI = c.n_col_int;
    S.steps.push_back(m);
  }
}

// Distinct values of integer attribute a in relation r, counted on the GPU
// (a bitmap over the domain); the domain when a has none declared.
static int64_t distinct_in(Prep& S, int a, int r, hipStream_t st) {
  auto it = S.distinct_rel.find({a, r});
  if (it != S.distinct_rel.end()) return it->second;
  Plan& P = *S.P;
  const AttrDef& A = P.attrs[a];
  auto c = P.rels[r].col.find(a);
  int64_t d = A.domain > 0 ? A.domain : INT64_MAX;
  if (c != P.rels[r].col.end() && P.rels[r].dtypes[c->second] == LMFAO_I32 && A.domain > 0) {
    const int best = r, bc = c->second;
    const int64_t words = (A.domain + 31) / 32;
    void* bits = dmem(S, (size_t)words * 4);
    void* cnt = dmem(S, 8);
    launch_distinct((const int32_t*)S.ecols[best][bc], P.rels[best].n_rows, A.domain, (uint32_t*)bits,
                    (unsigned long long*)cnt, st);
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, cnt, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(S, bits);
    dfree(S, cnt);
    if (e != hipSuccess) throw PlanError{LMFAO_EHIP, std::string("distinct count: ") + hipGetErrorString(e)};
    d = (int64_t)h;
  }
  S.distinct_rel[{a, r}] = d;
  return d;
}

// Distinct values of an integer attribute in the smallest relation that
// holds it (every value of D is among them).
static int64_t distinct_of(Prep& S, int a, hipStream_t st) {
  auto it = S.distinct.find(a);
  if (it != S.distinct.end()) return it->second;
  Plan& P = *S.P;
  int best = -1;
  for (size_t r = 0; r < P.rels.size(); ++r) {
    auto c = P.rels[r].col.find(a);
    if (c == P.rels[r].col.end() || P.rels[r].dtypes[c->second] != LMFAO_I32) continue;
    if (best < 0 || P.rels[r].n_rows < P.rels[best].n_rows) best = (int)r;
  }
  const int64_t d = best >= 0 ? distinct_in(S, a, best, st) : (P.attrs[a].domain > 0 ? P.attrs[a].domain : INT64_MAX);
  S.distinct[a] = d;
  return d;
}

// Fewest rows of a relation whose tuple determines every key attribute: the
// relation holds the attribute, or the attribute lies in a subtree that joins
// it on primary keys (at most one subtree tuple per tuple of the relation).
// Every tuple of D contains one tuple of that relation and its key is a
// function of it, so there are at most that many groups.  -1 if none.
static int64_t determining_rows(const Plan& P, const std::vector<int>& keys) {
  int64_t best = -1;
  const int n = (int)P.rels.size();
  for (int s = 0; s < n; ++s) {
    std::vector<char> det(n, 0);
    det[s] = 1;
    std::vector<std::pair<int, int>> todo;
    for (int c : P.adj[s]) todo.push_back({c, s});
    while (!todo.empty()) {
      const auto [u, par] = todo.back();
      todo.pop_back();
      if (!P.uniq[u][par]) continue;
      det[u] = 1;
      for (int v : P.adj[u])
        if (v != par) todo.push_back({v, u});
    }
    bool all = true;
    for (int a : keys) {
      bool held = false;
      for (int r = 0; r < n && !held; ++r) held = det[r] && P.rels[r].col.count(a);
      all = all && held;
    }
    if (all && (best < 0 || P.rels[s].n_rows < best)) best = P.rels[s].n_rows;
  }
  return best;
}

// most groups a query can have: dense key space, product of distinct counts,
// rows of a relation that determines the key
static double query_bound(Prep& S, const QueryDef& Q, hipStream_t st) {
  const Plan& P = *S.P;
  double dense = 1, pd = 1;
  for (int a : Q.groupby) {
    dense *= (double)P.attrs[a].domain;
    pd *= (double)distinct_of(S, a, st);
  }
  double b = std::min(dense, pd);
  const int64_t dr = determining_rows(P, Q.groupby);
  if (dr >= 0) b = std::min(b, (double)dr);
  return std::max(1.0, b);
}

// estimator features of a query (layout declared with LMFAO_EST_FEATURES)
static void query_features(Prep& S, const QueryDef& Q, float* f, hipStream_t st) {
  const Plan& P = *S.P;
  auto lg = [](double x) { return (float)std::log2(1.0 + std::max(0.0, x)); };
  for (int i = 0; i < LMFAO_EST_FEATURES; ++i) f[i] = 0.f;
  double total = 0;
  for (const RelDef& R : P.rels) total += (double)R.n_rows;
  f[0] = lg((double)P.rels[Q.root].n_rows);
  f[1] = lg(total);
  f[2] = (float)P.rels.size();
  f[3] = (float)Q.groupby.size();
  // tree distances from the root
  std::vector<int> dist(P.rels.size(), -1), queue{Q.root};
  dist[Q.root] = 0;
  for (size_t i = 0; i < queue.size(); ++i)
    for (int v : P.adj[queue[i]])
      if (dist[v] < 0) dist[v] = dist[queue[i]] + 1, queue.push_back(v);
  double pd = 1;
  for (size_t k = 0; k < Q.groupby.size(); ++k) {
    const int a = Q.groupby[k];
    const double dc = (double)distinct_of(S, a, st);
    pd *= dc;
    if (k >= 3) continue;
    int near = 1 << 20, h = -1;
    for (size_t r = 0; r < P.rels.size(); ++r)
      if (P.rels[r].col.count(a) && dist[r] >= 0 && dist[r] < near) near = dist[r], h = (int)r;
    f[4 + k] = lg(dc);
    f[7 + k] = lg((double)P.attrs[a].domain);
    f[10 + k] = (float)(near == (1 << 20) ? 0 : near);
    if (h < 0) continue;
    // the key's holder (nearest the root) and how much of it the join toward
    // the root reaches: distinct values of the first join attribute on the
    // root side and in the holder
    const double hrows = (double)P.rels[h].n_rows;
    f[17 + k] = lg(hrows);
    f[20 + k] = f[17 + k];
    f[23 + k] = f[17 + k];
    if (h == Q.root) continue;
    int par = -1;
    for (int v : P.adj[h])
      if (dist[v] == dist[h] - 1) par = v;
    for (int j : P.rels[h].attrs) {
      if (!P.rels[par].col.count(j)) continue;
      f[20 + k] = lg((double)distinct_in(S, j, par, st));
      f[23 + k] = lg((double)distinct_in(S, j, h, st));
      break;
    }
  }
  f[13] = lg(pd);
  f[14] = lg(query_bound(S, Q, st));
  f[15] = determining_rows(P, Q.groupby) >= 0 ? 1.f : 0.f;
  f[16] = (float)P.filter.size();
}

// log2(1 + groups) the estimator predicts from the features (FP32, host):
// the bound feature less the network's shortfall
static double estimate_log2_groups(const std::vector<float>& blob, const float* x) {
  const int d = LMFAO_EST_FEATURES, h = (int)blob[2];
  const float* mean = blob.data() + 4;
  const float* sd = mean + d;
  const float* W1 = sd + d;
  const float* b1 = W1 + (size_t)d * h;
  const float* W2 = b1 + h;
  const float* b2 = W2 + (size_t)h * h;
  const float* w3 = b2 + h;
  const float* b3 = w3 + h;
  std::vector<float> z(d), h1(h), h2(h);
  for (int i = 0; i < d; ++i) z[i] = (x[i] - mean[i]) / (sd[i] > 0.f ? sd[i] : 1.f);
  for (int j = 0; j < h; ++j) {
    float a = b1[j];
    for (int i = 0; i < d; ++i) a += z[i] * W1[(size_t)i * h + j];
    h1[j] = a > 0.f ? a : 0.f;
  }
  for (int j = 0; j < h; ++j) {
    float a = b2[j];
    for (int i = 0; i < h; ++i) a += h1[i] * W2[(size_t)i * h + j];
    h2[j] = a > 0.f ? a : 0.f;
  }
  float y = b3[0];
  for (int j = 0; j < h; ++j) y += h2[j] * w3[j];
  return (double)x[14] - (double)y;
}

// largest initial hash table (2^26 slots, 1.5 GiB with one value); larger
// ones are reached by regrowth when the groups are really there
constexpr int64_t kHashInitSlots = (int64_t)1 << 26;

// (re)allocates the slots of a hash table for H.cap slots.  The new arrays
// are allocated first; the old ones are released only once all three exist,
// so a failed allocation leaves the table as it was (H.cap restored) and
// throws PlanError{LMFAO_ENOMEM}.  A counts-only table is cleared here, on
// the stream, once: the partition count then keeps every slot past each
// region's groups at zero by clearing only what the previous run left there.
static void alloc_hash(Prep& S, HashBuf& H, hipStream_t st, int64_t old_cap = 0) {
  void* fresh[3] = {nullptr, nullptr, nullptr};
  // a counts-only table's values are never read (they are its counts)
  const size_t bytes[3] = {(size_t)H.cap * 8, (size_t)H.cap * 8,
                           H.counts_only ? (size_t)8 : (size_t)H.cap * 8 * std::max(1, H.n_vals)};
  for (int i = 0; i < 3; ++i) {
    try {
      fresh[i] = dmem(S, std::max<size_t>(bytes[i], 8));
    } catch (const PlanError& e) {
      for (int j = 0; j < i; ++j) dfree(S, fresh[j]);
      const int64_t want = H.cap;
      if (old_cap) H.cap = old_cap;
      throw PlanError{LMFAO_ENOMEM, "hash table of " + std::to_string(want) + " slots: " + e.msg};
    }
  }
  for (void* p : {(void*)H.keys, (void*)H.cnt, (void*)H.vals})
    if (p) dfree(S, p);
  H.keys = (unsigned long long*)fresh[0];
  H.cnt = (int64_t*)fresh[1];
  H.vals = (double*)fresh[2];
  if (H.counts_only) {
    if (!H.used) H.used = (uint32_t*)dalloc(S, kPartHashBuckets * 4);
    launch_fill(H.keys, H.cap * 8, st);
    launch_fill(H.used, kPartHashBuckets * 4, st);
    HIP_OK(hipGetLastError());
  }
}

static void prepare_all(Prep& S, const void* const* const* user_cols, hipStream_t st) {
  Plan& P = *S.P;
  S.nodes.assign(P.rels.size(), NodeData{});
  S.w_raw.assign(P.rels.size(), nullptr);
  S.w_sorted.assign(P.rels.size(), nullptr);
  S.w_raw_done.assign(P.rels.size(), 0);
  S.w_sorted_done.assign(P.rels.size(), 0);
  S.err_flag = (int32_t*)dalloc(S, 8);
  HIP_OK(hipMemsetAsync(S.err_flag, 0, 8, st));
  // caller-written row weights, all 1 until written
  S.row_w.assign(P.rels.size(), nullptr);
  S.row_perm.assign(P.rels.size(), nullptr);
  for (size_t r = 0; r < P.rels.size() && r < 32; ++r) {
    if (!((P.opts.row_weights >> r) & 1u)) continue;
    S.row_w[r] = (int32_t*)dalloc(S, (size_t)std::max<int64_t>(P.rels[r].n_rows, 1) * 4);
    DFilter ones{};
    ones.n_rows = P.rels[r].n_rows;
    ones.out = S.row_w[r];
    launch_filter_value(ones, st);
  }
  // the caller's columns, then the derived bucket codes of condition thresholds
  S.ecols.assign(P.rels.size(), {});
  S.ecol_ptrs.assign(P.rels.size(), nullptr);
  for (size_t r = 0; r < P.rels.size(); ++r) {
    const RelDef& R = P.rels[r];
    S.ecols[r].assign(R.attrs.size(), nullptr);
    for (int c = 0; c < R.n_input_attrs; ++c) S.ecols[r][c] = user_cols[r][c];
  }
  for (const DerivedAttr& D : P.derived) {
    const RelDef& R = P.rels[D.rel];
    const int sc = R.col.at(D.src), dc = R.col.at(D.attr);
    if (R.n_rows > 0 && !S.ecols[D.rel][sc])
      throw PlanError{LMFAO_EINVAL, "null column " + P.attrs[D.src].name + " of " + R.name};
    const double* thr = upload_vec(S, D.thr, st);
    if (D.kind == 2) {
      // a user-defined factor: its table at every row's argument value
      double* out = (double*)dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * 8);
      launch_gather_table((const int32_t*)S.ecols[D.rel][sc], R.n_rows, thr, (int64_t)D.thr.size(), out,
                          S.err_flag, st);
      S.ecols[D.rel][dc] = out;
      continue;
    }
    int32_t* out = (int32_t*)dalloc(S, (size_t)std::max<int64_t>(R.n_rows, 1) * 4);
    launch_bucketize(S.ecols[D.rel][sc], R.dtypes[sc], R.n_rows, thr, (int)D.thr.size(), D.kind, out, st);
    S.ecols[D.rel][dc] = out;
  }
  for (size_t r = 0; r < P.rels.size(); ++r) S.ecol_ptrs[r] = S.ecols[r].data();
  const void* const* const* cols = S.ecol_ptrs.data();
  for (size_t r = 0; r < P.rels.size(); ++r) {
    S.nodes[r].raw_col.assign(P.rels[r].attrs.size(), nullptr);
    S.nodes[r].raw_src.assign(cols[r], cols[r] + P.rels[r].attrs.size());
  }
  // validate integer columns against their domains
  for (size_t r = 0; r < P.rels.size(); ++r) {
    const RelDef& R = P.rels[r];
    for (size_t c = 0; c < R.attrs.size(); ++c) {
      const AttrDef& A = P.attrs[R.attrs[c]];
      if (R.dtypes[c] == LMFAO_I32 && A.domain > 0 && R.n_rows > 0) {
        if (!cols[r][c]) throw PlanError{LMFAO_EINVAL, "null column " + A.name + " of " + R.name};
        launch_validate((const int32_t*)cols[r][c], R.n_rows, A.domain, S.err_flag, st);
      }
      if (R.n_rows > 0 && !cols[r][c]) throw PlanError{LMFAO_EINVAL, "null column " + A.name + " of " + R.name};
    }
  }
  int32_t flag = 0;
  HIP_OK(hipMemcpyAsync(&flag, S.err_flag, 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (flag & 2) throw PlanError{LMFAO_EINVAL, "an integer column holds a value outside its declared domain"};
  // column statistics: distinct counts of every group-by attribute and of
  // the join attributes the estimator features read (while the caller's
  // columns are at hand)
  for (const QueryDef& Q : P.queries) {
    for (int a : Q.groupby) distinct_of(S, a, st);
    if (!Q.groupby.empty()) {
      float f[LMFAO_EST_FEATURES];
      query_features(S, Q, f, st);
    }
  }
  // output buffers: every view and query result lives in one arena that a
  // single fill zeroes at the start of each run
  S.vout.resize(P.views.size());
  S.qout.resize(P.queries.size());
  std::vector<std::pair<void**, size_t>> carve;
  for (auto& V : P.views) {
    OutBuf& B = S.vout[V.id];
    B.n_rows = V.n_keys;
    B.f64 = V.unique ? S.f64 : true;
    B.n_vals = V.unique ? (int)V.val_attrs.size() : (int)V.val_monos.size();
    B.n_codes = V.unique ? (int)V.code_attrs.size() : 0;
    carve.push_back({(void**)&B.cnt, (size_t)B.n_rows * 8});
    carve.push_back({&B.vals, (size_t)B.n_rows * B.n_vals * (B.f64 ? 8 : 4)});
    carve.push_back({(void**)&B.codes, (size_t)B.n_rows * B.n_codes * 4});
  }
  for (size_t q = 0; q < P.queries.size(); ++q) {
    const QueryDef& Q = P.queries[q];
    OutBuf& B = S.qout[q];
    double dense = 1;
    B.n_rows = 1;
    for (int a : Q.groupby) {
      dense *= (double)P.attrs[a].domain;
      B.n_rows = dense > 9e18 ? INT64_MAX : B.n_rows * P.attrs[a].domain;
    }
    B.f64 = true;
    B.n_vals = (int)Q.aggs.size();
    const bool learned = P.opts.sizing == LMFAO_SIZING_LEARNED && !P.estimator.empty();
    double est = -1.0;
    auto estimate = [&]() {
      if (est < 0) {
        float f[LMFAO_EST_FEATURES];
        query_features(S, Q, f, st);
        const double y = estimate_log2_groups(P.estimator, f) + (double)P.estimator[3];
        est = std::max(0.0, std::exp2(std::min(y, 62.0)) - 1.0);
      }
      return est;
    };
    bool hashed = dense > (double)kDenseRowsMax;
    // Learned sizing also picks dense or hash for the tables the partition
    // count keeps (it counts either kind per output): a table past one LDS
    // slice whose predicted group count is below 1/kDenseDensityMin of its
    // key range is hashed (the regrowth fallback keeps results exact
    // whatever the prediction).  Tables with range queries stay dense, and so
    // do tables counted with view multiplicities.
    bool weighted = false;   // counted with view multiplicities: the partition count keeps it dense
    for (auto& kv : Q.in_view) weighted |= !P.views[kv.second].unique;
    if (!hashed && learned && !weighted && dense > (double)kPickMinCells && Q.group >= 0 &&
        P.groups[Q.group].partitioned) {
      bool ranged = false;
      for (const UserQuery& U : P.user) ranged |= U.internal == (int)q && U.range;
      if (!ranged && estimate() * kDenseDensityMin < dense) {
        hashed = true;
        S.picked_hash++;
      }
    }
    if (hashed) {
      // hash table: at most one group per tuple of the root relation
      HashBuf H;
      H.query = (int)q;
      H.bound = (int64_t)std::min(query_bound(S, Q, st), 4e18);
      H.n_vals = B.n_vals;
      int64_t top = 1;
      while (top < std::max<int64_t>(1024, 2 * H.bound)) top <<= 1;
      top = std::min(top, kHashInitSlots);
      int64_t want = top;
      if (P.opts.hash_slots > 0) {
        want = P.opts.hash_slots;
      } else if (P.opts.sizing == LMFAO_SIZING_EXACT) {
        want = top;   // the exact-count run at the end of prepare resizes it
      } else if (learned) {
        H.est = estimate();
        want = (int64_t)std::min<double>((double)top, std::max(1024.0, 2.0 * H.est));
      }
      H.cap = 1;
      while (H.cap < want) H.cap <<= 1;
      B.hash = (int)S.hashes.size();
      S.hashes.push_back(H);
      continue;
    }
    carve.push_back({(void**)&B.cnt, (size_t)B.n_rows * 8});
    carve.push_back({&B.vals, (size_t)B.n_rows * B.n_vals * 8});
  }
  S.uout.resize(P.user.size());
  for (size_t u = 0; u < P.user.size(); ++u) {
    const UserQuery& U = P.user[u];
    if (!U.range) continue;
    const OutBuf& Q = S.qout[U.internal];
    if (Q.hash >= 0) throw PlanError{LMFAO_EUNSUPPORTED, "a range condition on a query kept in a hash table"};
    OutBuf& B = S.uout[u];
    B.n_rows = Q.n_rows / U.nb;
    B.f64 = true;
    B.n_vals = Q.n_vals;
    carve.push_back({(void**)&B.cnt, (size_t)B.n_rows * 8});
    carve.push_back({&B.vals, (size_t)B.n_rows * B.n_vals * 8});
  }
  size_t arena = 0;
  for (auto& c : carve) arena += (c.second + 255) & ~(size_t)255;
  char* base = (char*)dalloc(S, std::max<size_t>(arena, 256));
  size_t off = 0;
  for (auto& c : carve) {
    *c.first = base + off;
    off += (c.second + 255) & ~(size_t)255;
  }
  add_fill(S, base, (int64_t)arena, "zero");
  add_fill(S, S.err_flag, 8, "flags");
  if (!S.hashes.empty()) {
    S.hash_ovf = (int32_t*)dalloc(S, S.hashes.size() * 4);
    add_fill(S, S.hash_ovf, (int64_t)S.hashes.size() * 4, "hash flags");
    std::vector<DHashOut> hd(S.hashes.size());
    for (size_t i = 0; i < S.hashes.size(); ++i) {
      HashBuf& H = S.hashes[i];
      // tables counted by radix partition are written whole by their last
      // pass (every slot, groups or empty), and their values are the counts
      const QueryDef& QH = P.queries[H.query];
      H.counts_only = QH.group >= 0 && P.groups[QH.group].partitioned;
      alloc_hash(S, H, st);
      if (!H.counts_only) {
        H.fill_step = (int)S.steps.size();
        add_fill(S, H.keys, H.cap * 8, "hash keys");
        add_fill(S, H.cnt, H.cap * 8, "hash counts");
        add_fill(S, H.vals, H.cap * 8 * std::max(1, H.n_vals), "hash values");
      }
      hd[i] = DHashOut{H.keys, H.cnt, H.vals, H.cap - 1, S.hash_ovf + i, H.n_vals, 0, H.used};
    }
    S.hash_dev = upload_vec(S, hd, st);
  }
  // groups in dependency-level order
  std::vector<int> gorder(P.groups.size());
  std::iota(gorder.begin(), gorder.end(), 0);
  std::stable_sort(gorder.begin(), gorder.end(),
                   [&](int a, int b) { return P.groups[a].level < P.groups[b].level; });
  for (int gi : gorder) {
    build_group(S, gi, cols, st);
    // SUM(1) components of scattered outputs: copied from the counts once the
    // group's steps are done (hash tables: when the results are read)
    const GroupDef& G = P.groups[gi];
    if (!G.has_program) continue;
    for (const ProgOutput& po : G.prog.outs) {
      if (po.count_copies.empty()) continue;
      const OutBuf& O = po.ref.kind == 0 ? S.qout[po.ref.id] : S.vout[po.ref.id];
      if (O.hash >= 0) {
        S.hashes[O.hash].count_copies = po.count_copies;
        continue;
      }
      if (!O.f64) throw PlanError{LMFAO_EINVAL, "internal: count copy into an FP32 output"};
      DCountCopy cc{};
      cc.cnt = O.cnt;
      cc.vals = (double*)O.vals;
      cc.n = O.n_rows;
      cc.nv = O.n_vals;
      cc.n_copy = (int)po.count_copies.size();
      if (cc.n_copy > kMaxTableComps) throw PlanError{LMFAO_EUNSUPPORTED, "too many SUM(1) components"};
      for (int k = 0; k < cc.n_copy; ++k) cc.comp[k] = po.count_copies[k];
      Step t;
      t.name = "g" + std::to_string(gi) + ":" + P.rels[G.node].name + ":count_copy";
      t.kind = 13;
      t.dev = upload(S, cc, st);
      t.n = cc.n;
      S.steps.push_back(t);
    }
  }
  // range queries: sums over the bucket ranges their conditions select
  std::vector<DFinalize> fin;
  for (size_t u = 0; u < P.user.size(); ++u) {
    const UserQuery& U = P.user[u];
    if (!U.range) continue;
    const OutBuf& Q = S.qout[U.internal];
    const OutBuf& B = S.uout[u];
    DFinalize d{};
    d.src_cnt = Q.cnt;
    d.src_vals = (const double*)Q.vals;
    d.dst_cnt = B.cnt;
    d.dst_vals = (double*)B.vals;
    d.n_rows = B.n_rows;
    d.nb = U.nb;
    d.n_vals = B.n_vals;
    d.lo = U.lo;
    d.hi = U.hi;
    d.ex = U.ex;
    fin.push_back(d);
  }
  if (!fin.empty()) {
    Step s;
    s.name = "finalize";
    s.kind = 11;
    s.dev = upload_vec(S, fin, st);
    s.n = (int64_t)fin.size();
    S.steps.push_back(s);
  }
  HIP_OK(hipStreamSynchronize(st));
  for (auto& N : S.nodes)
    if (N.perm) {
      dfree(S, N.perm);
      N.perm = nullptr;
    }
}

// timed steps: scans and contractions (the kernels that move the data); the
// whole run is timed as well.  Slot 0 of a run = whole run.
static bool timed_step(const Step& s) {
  return s.kind == 2 || s.kind == 4 || s.kind == 8 || s.kind == 12 || s.kind == 15;
}
static int timed_slots(const Prep& S) {
  int n = 1;
  for (auto& s : S.steps) n += timed_step(s);
  return n;
}

static void enqueue_run(Prep& S, hipStream_t st) {
  int base = 0;
  if (S.timing) {
    int slots = timed_slots(S);
    base = S.timed_runs * slots * 2;
    size_t need = (size_t)base + slots * 2;
    while (S.ev.size() < need) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      S.ev.push_back(e);
    }
    HIP_OK(hipEventRecord(S.ev[base], st));
  }
  int slot = 1;
  for (size_t i = 0; i < S.steps.size(); ++i) {
    Step& s = S.steps[i];
    bool t = S.timing && timed_step(s);
    if (t) HIP_OK(hipEventRecord(S.ev[base + 2 * slot], st));
    switch (s.kind) {
      case 0: launch_fill(s.dev, s.bytes, st); break;
      case 1: launch_view_build((const DViewBuild*)s.dev, s.n, S.f64, st); break;
      case 2:
        if (s.gen_fn) {
          void* params[] = {(void*)&s.gen_args};
          HIP_OK(hipModuleLaunchKernel(s.gen_fn, s.grid, 1, 1, s.gen_block, 1, 1, s.lds, st, params, nullptr));
        } else if (s.fast) {
          launch_scan_fast((const DScan*)s.dev, s.na, S.f64, s.grid, s.lds, st);
        } else {
          launch_scan((const DScan*)s.dev, s.na, S.f64, s.grid, s.lds, st);
        }
        break;
      case 6: launch_build_image((const DImageBuild*)s.dev, s.n, S.f64, st); break;
      case 3: launch_table_reduce((const DTableReduce*)s.dev, s.n, s.n_blocks, st); break;
      case 4: launch_contract((const DContract*)s.dev, S.f64, s.grid, s.grid_y, s.lds, st); break;
      case 5:
        launch_merge_cells((const DCell*)s.dev, s.n, s.part_f, s.part_i, s.n_blocks, s.NF, s.NG, s.NFI, s.NGI, st);
        break;
      case 12:
        launch_scatter_rows((const DContract*)s.dev, S.f64, s.grid, st);
        break;
      case 13: launch_count_copy((const DCountCopy*)s.dev, s.n, st); break;
      case 14: launch_mult_check((const DMultCheck*)s.dev, s.mult, st); break;
      case 15: launch_part_count((const DPartCount*)s.dev, s.part, s.na, st); break;
      case 8:
        launch_contract_fused((const DContract*)s.dev, (const DGemm*)s.dev2, S.f64,
                              S.P->opts.precision == LMFAO_PREC_BF16X3   ? 3
                              : S.P->opts.precision == LMFAO_PREC_BF16X2 ? 2
                                                                         : 0,
                              s.na, s.grid, s.grid_y, s.lds, st);
        break;
      case 9:
        launch_merge_bm((const DCell*)s.dev, s.n, s.part_f, s.n_blocks, s.NG, (int64_t)s.NF * s.NG, S.err_flag, st);
        break;
      case 10: launch_filter((const DFilter*)s.dev, s.n, st); break;
      case 11: launch_finalize((const DFinalize*)s.dev, (int)s.n, st); break;
    }
    if (t) {
      HIP_OK(hipEventRecord(S.ev[base + 2 * slot + 1], st));
      ++slot;
    }
  }
  if (S.timing) {
    HIP_OK(hipEventRecord(S.ev[base + 1], st));
    S.timed_runs++;
  }
  HIP_OK(hipGetLastError());
}

}  // namespace lmfao

// ===========================================================================
// C ABI
// ===========================================================================
using namespace lmfao;

static lmfao_status set_err(lmfao_status st, const std::string& m) {
  record_error(m);
  return st;
}

extern "C" {

lmfao_status lmfao_plan_workspace_bytes(lmfao_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return set_err(LMFAO_EINVAL, "null argument");
  const Plan& P = *plan->P;
  size_t b = 0;
  bool f64 = P.opts.precision == LMFAO_PREC_F64;
  for (auto& V : P.views)
    b += (size_t)V.n_keys * (8 + (V.unique ? V.val_attrs.size() * (f64 ? 8 : 4) + V.code_attrs.size() * 4
                                           : V.val_monos.size() * 8));
  for (auto& Q : P.queries) {
    size_t rows = 1;
    for (int a : Q.groupby) rows *= (size_t)P.attrs[a].domain;
    b += rows * (8 + Q.aggs.size() * 8);
  }
  for (auto& G : P.groups)
    if (G.has_program && !G.prog.row_pieces) {
      const RelDef& R = P.rels[G.node];
      for (int c : G.prog.scan_cols) b += (size_t)R.n_rows * (R.dtypes[c] == LMFAO_F64 ? 8 : 4);
    }
  *bytes = b;
  return LMFAO_OK;
}

static void exact_sizes(Prep& S, hipStream_t st);

static const OutBuf& user_out(const lmfao_prepared_s* prep, int q, int* n_keys);

static lmfao_status prepare_impl(lmfao_plan_t plan, const void* const* const* columns, void* workspace,
                                 size_t ws_bytes, void* stream, lmfao_prepared_t* out) {
  clear_error();
  if (!plan || !columns || !out) return set_err(LMFAO_EINVAL, "null argument");
  *out = nullptr;
  std::unique_ptr<lmfao_prepared_s> S(new lmfao_prepared_s);
  S->P = plan->P;
  S->f64 = plan->P->opts.precision == LMFAO_PREC_F64;
  S->stream = (hipStream_t)stream;
  S->ws = (char*)workspace;
  S->ws_cap = workspace ? ws_bytes : 0;
  for (size_t r = 0; r < plan->P->rels.size(); ++r)
    if (!columns[r]) return set_err(LMFAO_EINVAL, "null column list of relation " + plan->P->rels[r].name);
  try {
    prepare_all(*S, columns, (hipStream_t)stream);
    if (plan->P->opts.sizing == LMFAO_SIZING_EXACT && plan->P->opts.hash_slots <= 0)
      exact_sizes(*S, (hipStream_t)stream);
  } catch (const PlanError& e) {
    return set_err(e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  S->ws_prepared = S->ws_used;
  *out = S.release();
  return LMFAO_OK;
}

lmfao_status lmfao_prepare(lmfao_plan_t plan, const void* const* const* columns, void* stream,
                           lmfao_prepared_t* out) {
  return prepare_impl(plan, columns, nullptr, 0, stream, out);
}

lmfao_status lmfao_prepare_in(lmfao_plan_t plan, const void* const* const* columns, void* workspace,
                              size_t workspace_bytes, void* stream, lmfao_prepared_t* out) {
  if (!workspace || (uintptr_t)workspace % 256 != 0)
    return set_err(LMFAO_EINVAL, "the workspace must be a device address aligned to 256 bytes");
  return prepare_impl(plan, columns, workspace, workspace_bytes, stream, out);
}

lmfao_status lmfao_prepared_workspace_bytes(lmfao_prepared_t prep, int32_t with_results, size_t* bytes) {
  clear_error();
  if (!prep || !bytes) return set_err(LMFAO_EINVAL, "null argument");
  size_t b = prep->ws_prepared;
  if (with_results) {
    // what lmfao_result_device carves for every query: its compacted arrays,
    // the shared scan scratch and the shared hash-sort scratch
    auto carve = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const Plan& P = *prep->P;
    int64_t pos_max = 0, rows_max = 0;
    for (size_t q = 0; q < P.user.size(); ++q) {
      int nk = 0;
      const OutBuf& B = user_out(prep, (int)q, &nk);
      const int64_t n = B.hash >= 0 ? prep->hashes[B.hash].cap : B.n_rows;
      b += carve((size_t)std::max<int64_t>(n * nk, 1) * 8) + carve((size_t)n * 8) +
           carve((size_t)std::max<int64_t>(n * B.n_vals, 1) * 8);
      pos_max = std::max(pos_max, n + scan_tiles(n) + 1);
      if (B.hash >= 0) rows_max = std::max(rows_max, n);
    }
    b += carve((size_t)pos_max * 4);
    if (rows_max) {
      const int64_t hist_n = (int64_t)256 * ((rows_max + sort_tile() - 1) / sort_tile() + 1);
      b += 2 * carve((size_t)rows_max * 8) + 2 * carve((size_t)rows_max * 4) +
           carve((size_t)(hist_n + scan_tiles(hist_n) + 1) * 4);
    }
  }
  *bytes = b;
  return LMFAO_OK;
}

// Grows every hash table whose inserts overflowed (x4, up to twice its bound)
// and refreshes the descriptors the kernels read.  Returns false when a
// table is already at its largest size.
// Reallocates hash table i at `cap` slots and points the run's fill steps and
// the table's device descriptor at the new arrays.
static void resize_hash(Prep& S, size_t i, int64_t cap, hipStream_t st) {
  HashBuf& H = S.hashes[i];
  const int64_t old_cap = H.cap;
  H.cap = cap;
  alloc_hash(S, H, st, old_cap);
  if (H.fill_step >= 0) {
    S.steps[H.fill_step].dev = H.keys;
    S.steps[H.fill_step].bytes = H.cap * 8;
    S.steps[H.fill_step + 1].dev = H.cnt;
    S.steps[H.fill_step + 1].bytes = H.cap * 8;
    S.steps[H.fill_step + 2].dev = H.vals;
    S.steps[H.fill_step + 2].bytes = H.cap * 8 * std::max(1, H.n_vals);
  }
  DHashOut d{H.keys, H.cnt, H.vals, H.cap - 1, S.hash_ovf + i, H.n_vals, 0, H.used};
  HIP_OK(hipMemcpyAsync(S.hash_dev + i, &d, sizeof d, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
}

static int64_t bound_capacity(const HashBuf& H) {
  int64_t top = 1;
  while (top < 2 * H.bound) top <<= 1;
  return std::max<int64_t>(top, 1024);
}

static bool grow_hashes(Prep& S, hipStream_t st) {
  std::vector<int32_t> ovf(S.hashes.size(), 0);
  HIP_OK(hipMemcpy(ovf.data(), S.hash_ovf, ovf.size() * 4, hipMemcpyDeviceToHost));
  bool grown = false;
  for (size_t i = 0; i < S.hashes.size(); ++i) {
    if (!ovf[i]) continue;
    HashBuf& H = S.hashes[i];
    if (H.used) {
      // a table of the partition count knows how many groups each of its
      // regions received (also past a full region): the smallest power-of-two
      // region that holds the largest one
      std::vector<uint32_t> u(kPartHashBuckets);
      HIP_OK(hipMemcpy(u.data(), H.used, u.size() * 4, hipMemcpyDeviceToHost));
      const int64_t need = *std::max_element(u.begin(), u.end());
      int64_t region = 1;
      while (region < need) region <<= 1;
      // no larger region needed: the overflow was not a full region
      if (region * kPartHashBuckets <= H.cap) return false;
      resize_hash(S, i, region * kPartHashBuckets, st);
      grown = true;
      continue;
    }
    const int64_t top = bound_capacity(H);
    if (H.cap >= top) return false;
    resize_hash(S, i, std::min(H.cap * 4, top), st);
    grown = true;
  }
  return grown;
}

// EXACT sizing: one whole run (its tables start at the BOUND capacity), then
// every table is counted on the device and reallocated at twice its exact
// group count; the run is part of lmfao_prepare, not of the timed lmfao_run.
static void exact_sizes(Prep& S, hipStream_t st) {
  if (S.hashes.empty()) return;
  enqueue_run(S, st);
  HIP_OK(hipStreamSynchronize(st));
  int32_t flag = 0;
  HIP_OK(hipMemcpy(&flag, S.err_flag, 4, hipMemcpyDeviceToHost));
  while (flag & 8) {
    if (!grow_hashes(S, st)) throw PlanError{LMFAO_EOVERFLOW, "a hash table at its largest size still overflowed"};
    S.hash_regrowths++;
    enqueue_run(S, st);
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(&flag, S.err_flag, 4, hipMemcpyDeviceToHost));
  }
  unsigned long long* cnt = (unsigned long long*)dalloc(S, S.hashes.size() * 8);
  HIP_OK(hipMemsetAsync(cnt, 0, S.hashes.size() * 8, st));
  for (size_t i = 0; i < S.hashes.size(); ++i) launch_count_keys(S.hashes[i].keys, S.hashes[i].cap, cnt + i, st);
  std::vector<unsigned long long> groups(S.hashes.size());
  HIP_OK(hipMemcpyAsync(groups.data(), cnt, groups.size() * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (size_t i = 0; i < S.hashes.size(); ++i) {
    HashBuf& H = S.hashes[i];
    H.est = (double)groups[i];
    int64_t cap = 1024;
    while (cap < 2 * (int64_t)groups[i]) cap <<= 1;
    if (cap != H.cap) resize_hash(S, i, cap, st);
  }
}

// Replays the run as a HIP graph, capturing it first (on the library's own
// stream: the caller's may be the legacy default stream, which cannot be
// captured).  Returns false when capture is not possible; the caller then
// launches directly.
static bool run_graph(Prep& S, hipStream_t st) {
  if (S.graph_failed) return false;
  if (!S.graph_exec) {
    if (!S.capture_stream && hipStreamCreateWithFlags(&S.capture_stream, hipStreamNonBlocking) != hipSuccess) {
      S.graph_failed = true;
      return false;
    }
    if (hipStreamBeginCapture(S.capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      S.graph_failed = true;
      (void)hipGetLastError();
      return false;
    }
    bool ok = true;
    try {
      enqueue_run(S, S.capture_stream);
    } catch (const HipError&) {
      ok = false;
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(S.capture_stream, &g);
    if (ok && e == hipSuccess && g) ok = hipGraphInstantiate(&S.graph_exec, g, nullptr, nullptr, 0) == hipSuccess;
    else ok = false;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
      S.graph_exec = nullptr;
      S.graph_failed = true;
      (void)hipGetLastError();
      return false;
    }
  }
  HIP_OK(hipGraphLaunch(S.graph_exec, st));
  return true;
}

static void drop_graph(Prep& S) {
  if (S.graph_exec) (void)hipGraphExecDestroy(S.graph_exec);
  S.graph_exec = nullptr;
}

static lmfao_status flag_status(int32_t flag) {
  if (flag & 1) return set_err(LMFAO_EINVAL, "a relation has duplicate values of its declared primary key");
  if (flag & 2) return set_err(LMFAO_EINVAL, "an integer column holds a value outside its declared domain");
  if (flag & 4)
    return set_err(LMFAO_EOVERFLOW, "an integer aggregate reached 2^53 in the FP64 matrix-core contraction "
                                    "(use the VALU contraction)");
  if (flag & 16)
    return set_err(LMFAO_EOVERFLOW, "a join multiplicity times the rows a scan block sums exceeds the range of "
                                    "the scan's 32-bit counters");
  return LMFAO_OK;
}

lmfao_status lmfao_run(lmfao_plan_t plan, lmfao_prepared_t prep, void* stream, int32_t sync) {
  clear_error();
  if (!plan || !prep || prep->P != plan->P) return set_err(LMFAO_EINVAL, "plan and prepared handle do not match");
  hipStream_t st = (hipStream_t)stream;
  prep->run_epoch++;
  try {
    if (!(prep->P->opts.graph && !sync && !prep->timing && run_graph(*prep, st))) enqueue_run(*prep, st);
    if (sync) {
      HIP_OK(hipStreamSynchronize(st));
      int32_t flag = 0;
      HIP_OK(hipMemcpy(&flag, prep->err_flag, 4, hipMemcpyDeviceToHost));
      // a hash table that was sized too small: enlarge it and run again
      while (flag & 8) {
        if (!grow_hashes(*prep, st))
          return set_err(LMFAO_EOVERFLOW, "a hash table at its largest size still overflowed");
        drop_graph(*prep);   // the captured launches point at the old tables
        prep->hash_regrowths++;
        enqueue_run(*prep, st);
        HIP_OK(hipStreamSynchronize(st));
        HIP_OK(hipMemcpy(&flag, prep->err_flag, 4, hipMemcpyDeviceToHost));
      }
      lmfao_status fs = flag_status(flag);
      if (fs) return fs;
    }
  } catch (const PlanError& e) {
    // a hash table that could not be regrown: the status names the cause
    return set_err(e.status == LMFAO_ENOMEM ? LMFAO_EOVERFLOW : e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

// The error bits the kernels of a run set, read after the run completed:
// 1 duplicate primary key, 2 a value outside its declared domain, 4 an
// integer cell reached 2^53 in the FP64 matrix-core contraction, 8 a hash
// table overflowed (regrown by a run with sync), 16 a join multiplicity that
// the scan's 32-bit counters cannot hold.
static lmfao_status read_flags(const lmfao_prepared_s* prep) {
  int32_t flag = 0;
  try {
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(&flag, prep->err_flag, 4, hipMemcpyDeviceToHost));
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  if (flag & 8) return set_err(LMFAO_EOVERFLOW, "a hash table overflowed in the last run (run with sync)");
  return flag_status(flag);
}

// the output buffer and group-by attributes of query q of the caller's batch
static const OutBuf& user_out(const lmfao_prepared_s* prep, int q, int* n_keys) {
  const Plan& P = *prep->P;
  const UserQuery& U = P.user[q];
  const int nk = (int)P.queries[U.internal].groupby.size();
  if (U.range) {
    *n_keys = nk - 1;   // the bucket attribute is the planned query's last key
    return prep->uout[q];
  }
  *n_keys = nk;
  return prep->qout[U.internal];
}

}  // extern "C"

namespace lmfao {

// Compacts caller query q's result of the last run on the device (once per
// run): present groups, keys per attribute, lexicographic order.  Hash tables
// are gathered by a scan over their slots and sorted by row (the LSD radix
// sort of prepare); dense tables keep row order.  Synchronises `st` (the
// group count sizes the hash sort).
static lmfao_status compact_result(lmfao_prepared_s* prep, int q, hipStream_t st) {
  const Plan& P = *prep->P;
  if (prep->compact.size() != P.user.size()) prep->compact.assign(P.user.size(), Compacted{});
  Compacted& C = prep->compact[q];
  if (C.epoch == prep->run_epoch && prep->run_epoch > 0) return LMFAO_OK;
  if (lmfao_status fs = read_flags(prep)) return fs;
  const QueryDef& Q = P.queries[P.user[q].internal];
  int nk = 0;
  const OutBuf& B = user_out(prep, q, &nk);
  if (nk > 4) return set_err(LMFAO_EUNSUPPORTED, "more than 4 group-by attributes");
  try {
    Prep& S = *prep;
    DCompact d{};
    d.n_vals = B.n_vals;
    d.n_keys = nk;
    std::vector<int64_t> dom(nk);
    for (int i = 0; i < nk; ++i) dom[i] = P.attrs[Q.groupby[i]].domain;
    int64_t m = 1;
    for (int i = nk - 1; i >= 0; --i) {
      d.stride[i] = m;
      d.dom[i] = dom[i];
      m = m * std::max<int64_t>(dom[i], 1);
    }
    const HashBuf* H = B.hash >= 0 ? &S.hashes[B.hash] : nullptr;
    d.cnt = H ? H->cnt : B.cnt;
    d.vals = H ? (H->counts_only ? nullptr : H->vals) : (B.n_vals ? (const double*)B.vals : nullptr);
    d.hkeys = H ? H->keys : nullptr;
    d.n_src = H ? H->cap : B.n_rows;
    if (H)
      for (int k : H->count_copies) d.copy_mask |= 1ull << k;
    // scratch shared by all queries, sized once for the largest (a regrown
    // hash table may need more later)
    int64_t pos_max = 0, rows_max = 0;
    for (size_t u = 0; u < P.user.size(); ++u) {
      int uk = 0;
      const OutBuf& UB = user_out(prep, (int)u, &uk);
      const int64_t un = UB.hash >= 0 ? S.hashes[UB.hash].cap : UB.n_rows;
      pos_max = std::max(pos_max, un + scan_tiles(un) + 1);
      if (UB.hash >= 0) rows_max = std::max(rows_max, un);
    }
    if (S.cpos_n < pos_max) {
      S.cpos = (uint32_t*)dalloc(S, (size_t)pos_max * 4);
      S.cpos_n = pos_max;
    }
    d.pos = S.cpos;
    const int64_t bound = d.n_src;   // groups at most
    if (H && S.crows_n < rows_max) {
      S.crows = (uint64_t*)dalloc(S, (size_t)rows_max * 8);
      S.crows2 = (uint64_t*)dalloc(S, (size_t)rows_max * 8);
      S.cslot = (uint32_t*)dalloc(S, (size_t)rows_max * 4);
      S.cslot2 = (uint32_t*)dalloc(S, (size_t)rows_max * 4);
      const int64_t hist_n = (int64_t)256 * ((rows_max + sort_tile() - 1) / sort_tile() + 1);
      S.chist = (uint32_t*)dalloc(S, (size_t)(hist_n + scan_tiles(hist_n) + 1) * 4);
      S.crows_n = rows_max;
    }
    d.rows = S.crows;
    d.slot = S.cslot;
    // the compacted arrays hold every group a dense table could have, or
    // every slot of the hash table (its size changes only by regrowth)
    if (C.cap < bound) {
      C.keys = (int64_t*)dalloc(S, (size_t)std::max<int64_t>(bound * nk, 1) * 8);
      C.cnt = (int64_t*)dalloc(S, (size_t)bound * 8);
      C.vals = (double*)dalloc(S, (size_t)std::max<int64_t>(bound * B.n_vals, 1) * 8);
      C.cap = bound;
    }
    d.keys_out = C.keys;
    d.cnt_out = C.cnt;
    d.vals_out = C.vals;
    launch_compact(d, st);
    HIP_OK(hipGetLastError());
    uint32_t n = 0;
    HIP_OK(hipMemcpyAsync(&n, d.pos + d.n_src + scan_tiles(d.n_src), 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (H && n > 0) {
      int bits = 1;
      while (bits < 63 && ((B.n_rows - 1) >> bits) != 0) ++bits;
      bool swapped = false;
      launch_sort(d.rows, d.slot, S.crows2, S.cslot2, n, bits, S.chist, st, &swapped);
      if (swapped) {
        d.rows = S.crows2;
        d.slot = S.cslot2;
      }
      launch_compact_emit(d, n, st);
      HIP_OK(hipGetLastError());
      HIP_OK(hipStreamSynchronize(st));
    }
    C.n_groups = n;
    C.epoch = prep->run_epoch;
  } catch (const PlanError& e) {
    return set_err(e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

}  // namespace lmfao

extern "C" {

lmfao_status lmfao_result_device(lmfao_prepared_t prep, int32_t q, lmfao_output* out, void* stream) {
  clear_error();
  if (!prep || !out || q < 0 || q >= (int)prep->P->user.size()) return set_err(LMFAO_EINVAL, "bad query index");
  if (lmfao_status e = compact_result(prep, q, (hipStream_t)stream)) return e;
  const Compacted& C = prep->compact[q];
  int nk = 0;
  const OutBuf& B = user_out(prep, q, &nk);
  out->n_groups = C.n_groups;
  out->n_keys = nk;
  out->n_aggs = B.n_vals;
  out->keys = C.keys;
  out->counts = C.cnt;
  out->values = C.vals;
  return LMFAO_OK;
}

lmfao_status lmfao_result_shape(lmfao_prepared_t prep, int32_t q, int64_t* n_groups, int32_t* n_keys,
                                int32_t* n_aggs) {
  lmfao_output o{};
  if (lmfao_status e = lmfao_result_device(prep, q, &o, nullptr)) return e;
  if (n_groups) *n_groups = o.n_groups;
  if (n_keys) *n_keys = o.n_keys;
  if (n_aggs) *n_aggs = o.n_aggs;
  return LMFAO_OK;
}

lmfao_status lmfao_result_copy(lmfao_prepared_t prep, int32_t q, int64_t* keys, int64_t* counts, double* values) {
  lmfao_output o{};
  if (lmfao_status e = lmfao_result_device(prep, q, &o, nullptr)) return e;
  try {
    if (keys && o.n_groups * o.n_keys)
      HIP_OK(hipMemcpy(keys, o.keys, (size_t)o.n_groups * o.n_keys * 8, hipMemcpyDeviceToHost));
    if (counts && o.n_groups) HIP_OK(hipMemcpy(counts, o.counts, (size_t)o.n_groups * 8, hipMemcpyDeviceToHost));
    if (values && o.n_groups * o.n_aggs)
      HIP_OK(hipMemcpy(values, o.values, (size_t)o.n_groups * o.n_aggs * 8, hipMemcpyDeviceToHost));
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

// ---------------------------------------------------------------------------
// ridge regression over the batch's results (section 3, linear regression)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// autotuner of launch shapes (JSON cache keyed by plan hash)
// ---------------------------------------------------------------------------
}  // extern "C"

namespace lmfao {

static uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

struct TuneEntry {
  int scan_blocks = 0, contract_splits = 0, one_hot_max = 0;
  double ms = 0, base_ms = 0;
};

// the cache: {"entries": {"<key>": {"scan_blocks": n, ...}, ...}}, one entry
// per line as this writer emits it
static std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  if (!path) return m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char key[64];
    TuneEntry e;
    if (sscanf(line, " \"%63[0-9a-f]\": {\"scan_blocks\": %d, \"contract_splits\": %d, \"one_hot_max\": %d, "
                     "\"ms\": %lf, \"base_ms\": %lf",
               key, &e.scan_blocks, &e.contract_splits, &e.one_hot_max, &e.ms, &e.base_ms) == 6)
      m[key] = e;
  }
  fclose(f);
  return m;
}

static void write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) throw PlanError{LMFAO_EINVAL, std::string("cannot write ") + path};
  fprintf(f, "{\"entries\": {\n");
  size_t i = 0;
  for (auto& kv : m) {
    const TuneEntry& e = kv.second;
    fprintf(f, "  \"%s\": {\"scan_blocks\": %d, \"contract_splits\": %d, \"one_hot_max\": %d, \"ms\": %.6f, "
               "\"base_ms\": %.6f}%s\n",
            kv.first.c_str(), e.scan_blocks, e.contract_splits, e.one_hot_max, e.ms, e.base_ms,
            ++i < m.size() ? "," : "");
  }
  fprintf(f, "}}\n");
  fclose(f);
  if (rename(tmp.c_str(), path) != 0) throw PlanError{LMFAO_EINVAL, std::string("cannot replace ") + path};
}

}  // namespace lmfao

extern "C" {

lmfao_status lmfao_tune(const lmfao_schema* schema, const lmfao_join_tree* tree, const lmfao_batch* batch,
                        lmfao_options* opts, const void* const* const* columns, const char* cache_path,
                        int32_t runs, double* best_ms, double* base_ms, void* stream) {
  clear_error();
  if (!schema || !tree || !batch || !opts || !columns) return set_err(LMFAO_EINVAL, "null argument");
  if (runs <= 0) runs = 5;
  hipStream_t st = (hipStream_t)stream;
  // the key: the plan with the base options, the relation sizes, the device
  lmfao_plan_t base = nullptr;
  if (lmfao_status e = lmfao_plan(schema, tree, batch, opts, &base)) return e;
  std::string ident = base->P->json;
  lmfao_plan_free(base);
  for (int r = 0; r < schema->n_relations; ++r) ident += "|" + std::to_string(schema->relations[r].n_rows);
  hipDeviceProp_t prop{};
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) ident += prop.gcnArchName;
  char key[32];
  snprintf(key, sizeof key, "%016llx", (unsigned long long)fnv1a(ident));
  try {
    std::map<std::string, TuneEntry> cache = read_tune_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
      opts->scan_blocks = hit->second.scan_blocks;
      opts->contract_splits = hit->second.contract_splits;
      opts->one_hot_max = hit->second.one_hot_max;
      if (best_ms) *best_ms = hit->second.ms;
      if (base_ms) *base_ms = hit->second.base_ms;
      return LMFAO_OK;
    }
    // one variant: plan, prepare, a checked run, then `runs` timed runs
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    auto measure = [&](const lmfao_options& o, double* ms) -> lmfao_status {
      lmfao_plan_t pl = nullptr;
      lmfao_prepared_t pr = nullptr;
      lmfao_status e = lmfao_plan(schema, tree, batch, &o, &pl);
      if (!e) e = lmfao_prepare(pl, columns, stream, &pr);
      if (!e) e = lmfao_run(pl, pr, stream, 1);
      if (!e) e = lmfao_run(pl, pr, stream, 0);   // captures the graph when asked
      if (!e) {
        (void)hipEventRecord(e0, st);
        for (int i = 0; i < runs && !e; ++i) e = lmfao_run(pl, pr, stream, 0);
        (void)hipEventRecord(e1, st);
        float t = 0;
        if (!e && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
          *ms = (double)t / runs;
        else if (!e)
          e = set_err(LMFAO_EHIP, "timing events failed");
      }
      if (pr) lmfao_prepared_free(pr);
      if (pl) lmfao_plan_free(pl);
      return e;
    };
    lmfao_options best = *opts;
    double best_t = 0;
    lmfao_status e = measure(best, &best_t);
    const double base_t = best_t;
    // coordinate descent over the three shapes (0 = the library's default)
    static const int kScan[] = {0, 512, 1024, 4096};
    static const int kSplit[] = {0, 256, 512, 2048, 4096};
    static const int kOneHot[] = {0, 16, 64};
    for (int param = 0; param < 3 && !e; ++param) {
      const int* vals = param == 0 ? kScan : param == 1 ? kSplit : kOneHot;
      const int nv = param == 0 ? 4 : param == 1 ? 5 : 3;
      const int cur = param == 0 ? best.scan_blocks : param == 1 ? best.contract_splits : best.one_hot_max;
      for (int i = 0; i < nv && !e; ++i) {
        if (vals[i] == cur) continue;
        lmfao_options o = best;
        (param == 0 ? o.scan_blocks : param == 1 ? o.contract_splits : o.one_hot_max) = vals[i];
        double t = 0;
        e = measure(o, &t);
        if (!e && t < best_t) {
          best = o;
          best_t = t;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e) return e;
    opts->scan_blocks = best.scan_blocks;
    opts->contract_splits = best.contract_splits;
    opts->one_hot_max = best.one_hot_max;
    if (best_ms) *best_ms = best_t;
    if (base_ms) *base_ms = base_t;
    cache[key] = TuneEntry{best.scan_blocks, best.contract_splits, best.one_hot_max, best_t, base_t};
    write_tune_cache(cache_path, cache);
  } catch (const PlanError& e) {
    return set_err(e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

// ---------------------------------------------------------------------------
// Rk-means steps 2 and 3 (section 3, Rk-means)
// ---------------------------------------------------------------------------
lmfao_status lmfao_kmeans_1d(int32_t n_sets, const int64_t* offsets, const int64_t* values, const int64_t* weights,
                             int32_t k, int32_t max_iter, double* centroids, int32_t* assignment, int32_t* steps,
                             void* stream) {
  clear_error();
  if (n_sets < 0 || (n_sets && (!offsets || !centroids))) return set_err(LMFAO_EINVAL, "null argument");
  if (k < 1 || k > kKmMaxClusters || max_iter < 0) return set_err(LMFAO_EINVAL, "k must be in [1, 64]");
  for (int i = 0; i < n_sets; ++i)
    if (offsets[i] < 0 || offsets[i + 1] < offsets[i]) return set_err(LMFAO_EINVAL, "offsets must not decrease");
  if (n_sets && offsets[n_sets] > 0 && (!values || !weights || !assignment))
    return set_err(LMFAO_EINVAL, "null values, weights or assignment");
  if (n_sets == 0) return LMFAO_OK;
  hipStream_t st = (hipStream_t)stream;
  void* doff = nullptr;
  void* dsteps = nullptr;
  try {
    HIP_OK(hipMalloc(&doff, (size_t)(n_sets + 1) * 8));
    HIP_OK(hipMalloc(&dsteps, (size_t)n_sets * 4));
    HIP_OK(hipMemcpyAsync(doff, offsets, (size_t)(n_sets + 1) * 8, hipMemcpyHostToDevice, st));
    launch_kmeans_1d((const int64_t*)doff, n_sets, values, weights, k, max_iter, centroids, assignment,
                     (int32_t*)dsteps, st);
    HIP_OK(hipGetLastError());
    std::vector<int32_t> hs(n_sets);
    HIP_OK(hipMemcpyAsync(hs.data(), dsteps, (size_t)n_sets * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (steps) std::copy(hs.begin(), hs.end(), steps);
  } catch (const HipError& e) {
    (void)hipFree(doff);
    (void)hipFree(dsteps);
    return set_err(LMFAO_EHIP, e.msg);
  }
  (void)hipFree(doff);
  (void)hipFree(dsteps);
  return LMFAO_OK;
}

}  // extern "C"

// breadth-first parents of the join tree from `root` (-1 for the root)
static std::vector<int> bfs_parents(const lmfao::Plan& P, int root) {
  std::vector<int> parent(P.rels.size(), -1), order{root};
  std::vector<char> seen(P.rels.size(), 0);
  seen[root] = 1;
  for (size_t i = 0; i < order.size(); ++i)
    for (int v : P.adj[order[i]])
      if (!seen[v]) {
        seen[v] = 1;
        parent[v] = order[i];
        order.push_back(v);
      }
  return parent;
}

extern "C" {

lmfao_status lmfao_grid_coreset(lmfao_plan_t plan, lmfao_prepared_t prep, const void* const* const* columns,
                                int32_t n_dims, const lmfao_grid_dim* dims, int32_t k, lmfao_output* out,
                                void* stream) {
  clear_error();
  if (!plan || !prep || prep->P != plan->P || !columns || !out || n_dims < 1 || !dims)
    return set_err(LMFAO_EINVAL, "null argument");
  if (k < 1 || k > 256) return set_err(LMFAO_EINVAL, "k must be in [1, 256]");
  const Plan& P = *prep->P;
  const int n = (int)P.rels.size();
  hipStream_t st = (hipStream_t)stream;
  // the root: every other relation reached through one key attribute (the
  // view toward the root is single-valued); the largest such relation
  int root = -1;
  for (int r = 0; r < n; ++r) {
    const std::vector<int> parent = bfs_parents(P, r);
    bool ok = true;
    for (int u = 0; u < n && ok; ++u)
      if (u != r) ok = P.uniq[u][parent[u]] && join_attrs(P, u, parent[u]).size() == 1;
    if (ok && (root < 0 || P.rels[r].n_rows > P.rels[root].n_rows)) root = r;
  }
  if (root < 0) return set_err(LMFAO_EUNSUPPORTED, "the grid coreset needs a join whose tuples a root row determines");
  if (n > kGridMaxRels) return set_err(LMFAO_EUNSUPPORTED, "more than 8 relations");
  int bits = 1;
  while ((1 << bits) < k) bits <<= 1;
  if (k == 1) bits = 1;
  const int words = (n_dims * bits + 63) / 64;
  if (n_dims > kGridMaxDims || words > kGridMaxWords)
    return set_err(LMFAO_EUNSUPPORTED, "more than 512 bits of packed cluster ids");
  try {
    Prep& S = *prep;
    const std::vector<int> parent = bfs_parents(P, root);
    std::vector<int> order{root};
    for (size_t i = 0; i < order.size(); ++i)
      for (int v : P.adj[order[i]])
        if (v != parent[order[i]]) order.push_back(v);
    std::vector<int> pos_of(n, -1);
    for (int i = 0; i < n; ++i) pos_of[order[i]] = i;
    int32_t* flag = (int32_t*)dalloc(S, 8);
    HIP_OK(hipMemsetAsync(flag, 0, 8, st));
    DGrid g{};
    g.n_rows = P.rels[root].n_rows;
    g.n_rels = n;
    g.n_dims = n_dims;
    g.bits = bits;
    g.n_words = words;
    g.flag = flag;
    for (int i = 1; i < n; ++i) {
      const int u = order[i], p = parent[u];
      const int a = join_attrs(P, u, p)[0];
      g.parent[i] = pos_of[p];
      g.pkey[i] = (const int32_t*)columns[p][P.rels[p].col.at(a)];
      g.index_n[i] = P.attrs[a].domain;
      int32_t* idx = (int32_t*)dalloc(S, (size_t)std::max<int64_t>(g.index_n[i], 1) * 4);
      HIP_OK(hipMemsetAsync(idx, 0xff, (size_t)std::max<int64_t>(g.index_n[i], 1) * 4, st));
      launch_grid_index((const int32_t*)columns[u][P.rels[u].col.at(a)], P.rels[u].n_rows, idx, g.index_n[i], flag,
                        st);
      g.index[i] = idx;
    }
    for (int d = 0; d < n_dims; ++d) {
      auto it = dims[d].attr ? P.attr_id.find(dims[d].attr) : P.attr_id.end();
      if (it == P.attr_id.end()) return set_err(LMFAO_EINVAL, "unknown grid attribute");
      const int a = it->second;
      if (P.attrs[a].dtype != LMFAO_I32 || P.attrs[a].domain <= 0 || dims[d].n_codes < 0 ||
          (dims[d].n_codes && (!dims[d].codes || !dims[d].cluster)))
        return set_err(LMFAO_EINVAL, "grid attributes are integer attributes with a domain and a code list");
      int rel = -1;
      for (int i = 0; i < n && rel < 0; ++i)
        if (P.rels[order[i]].has(a) && P.rels[order[i]].col.at(a) < P.rels[order[i]].n_input_attrs) rel = i;
      if (rel < 0) return set_err(LMFAO_EINVAL, "grid attribute held by no relation");
      g.rel[d] = rel;
      g.col[d] = (const int32_t*)columns[order[rel]][P.rels[order[rel]].col.at(a)];
      g.dom[d] = P.attrs[a].domain;
      int32_t* table = (int32_t*)dalloc(S, (size_t)g.dom[d] * 4);
      HIP_OK(hipMemsetAsync(table, 0, (size_t)g.dom[d] * 4, st));
      launch_code_table(dims[d].codes, dims[d].cluster, dims[d].n_codes, table, g.dom[d], flag, st);
      g.cluster[d] = table;
    }
    // at most one group per root row and k^n id vectors; half occupancy
    double bound = (double)std::max<int64_t>(g.n_rows, 1);
    bound = std::min(bound, std::pow((double)k, (double)n_dims));
    int64_t cap = 1024;
    while ((double)cap < 2.0 * bound) cap <<= 1;
    for (int attempt = 0;; ++attempt) {
      g.mask = cap - 1;
      g.keys = (unsigned long long*)dalloc(S, (size_t)cap * 8);
      g.cnt = (unsigned long long*)dalloc(S, (size_t)cap * 8);
      g.rep = (int32_t*)dalloc(S, (size_t)cap * 4);
      HIP_OK(hipMemsetAsync(g.keys, 0, (size_t)cap * 8, st));
      HIP_OK(hipMemsetAsync(g.cnt, 0, (size_t)cap * 8, st));
      DGrid* dg = upload(S, g, st);
      launch_grid_count(dg, g.n_rows, st);
      HIP_OK(hipGetLastError());
      int32_t f = 0;
      HIP_OK(hipMemcpyAsync(&f, flag, 4, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (f & 8) return set_err(LMFAO_EINVAL, "a key value held by two rows of a relation");
      if (f & 4) return set_err(LMFAO_EINVAL, "a value outside its domain, or a cluster id past k");
      if (f & 2) {
        if (attempt >= 2) return set_err(LMFAO_EOVERFLOW, "grid coreset table full");
        cap <<= 2;
        HIP_OK(hipMemsetAsync(flag, 0, 4, st));
        continue;
      }
      if (f & 1) return set_err(LMFAO_EUNSUPPORTED, "two grid points share a 64-bit fingerprint");
      uint32_t* posv = (uint32_t*)dalloc(S, (size_t)(cap + scan_tiles(cap) + 1) * 4);
      launch_grid_positions(dg, cap, posv, st);
      uint32_t ng = 0;
      HIP_OK(hipMemcpyAsync(&ng, posv + cap + scan_tiles(cap), 4, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      int64_t* kout = (int64_t*)dalloc(S, (size_t)std::max<int64_t>((int64_t)ng * n_dims, 1) * 8);
      int64_t* cout_ = (int64_t*)dalloc(S, (size_t)std::max<uint32_t>(ng, 1) * 8);
      launch_grid_emit(dg, cap, posv, kout, cout_, st);
      HIP_OK(hipGetLastError());
      HIP_OK(hipStreamSynchronize(st));
      out->n_groups = ng;
      out->n_keys = n_dims;
      out->n_aggs = 0;
      out->keys = kout;
      out->counts = cout_;
      out->values = nullptr;
      break;
    }
  } catch (const PlanError& e) {
    return set_err(e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

lmfao_status lmfao_row_weights(lmfao_prepared_t prep, int32_t rel, int32_t** weights) {
  clear_error();
  if (!prep || !weights) return set_err(LMFAO_EINVAL, "null argument");
  if (rel < 0 || rel >= (int)prep->row_w.size() || !prep->row_w[rel])
    return set_err(LMFAO_EINVAL, "relation without row weights (lmfao_options.row_weights)");
  *weights = prep->row_w[rel];
  return LMFAO_OK;
}

lmfao_status lmfao_eval_conditions(int64_t n_rows, int32_t n_conds, const lmfao_column_condition* conds,
                                   int32_t* out, void* stream) {
  clear_error();
  if (n_rows < 0 || n_conds < 0 || (n_conds && !conds) || (n_rows && !out)) return set_err(LMFAO_EINVAL, "bad argument");
  if (n_conds > kMaxFilterConds) return set_err(LMFAO_EINVAL, "more than 8 conditions");
  DFilter f{};
  f.n_rows = n_rows;
  f.n_conds = n_conds;
  f.out = out;
  for (int k = 0; k < n_conds; ++k) {
    const lmfao_column_condition& c = conds[k];
    if (!c.column && n_rows) return set_err(LMFAO_EINVAL, "null column");
    if (c.dtype != LMFAO_I32 && c.dtype != LMFAO_F32 && c.dtype != LMFAO_F64) return set_err(LMFAO_EINVAL, "bad dtype");
    if (c.op < LMFAO_LE || c.op > LMFAO_NE) return set_err(LMFAO_EINVAL, "bad op");
    f.cols[k] = DCol{c.column, c.dtype, 0};
    f.op[k] = c.op;
    f.c[k] = c.dtype == LMFAO_F32 ? (double)(float)c.constant : c.constant;
  }
  try {
    launch_filter_value(f, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

}  // extern "C"

namespace lmfao {

// device pointers of every candidate's count and (SUM(1), SUM(y), SUM(y^2))
// values and of the node totals, checked against the batch: each query's
// aggregates 0, 1, 2 must be SUM(1), SUM(y), SUM(y*y) of one y
static lmfao_status cart_inputs(lmfao_prepared_s* prep, const lmfao_cart_spec* spec,
                                std::vector<const void*>& ptrs) {
  const Plan& P = *prep->P;
  if (!spec || spec->n_candidates < 0 || (spec->n_candidates && !spec->candidates))
    return set_err(LMFAO_EINVAL, "bad CART specification");
  int y = -1;
  auto agg_ok = [&](int q) {
    if (q < 0 || q >= (int)P.user.size()) return false;
    const QueryDef& Q = P.queries[P.user[q].internal];
    if (Q.aggs.size() < 3 || !Q.aggs[0].empty() || Q.aggs[1].size() != 1 || Q.aggs[2].size() != 2) return false;
    const int a = Q.aggs[1][0];
    if (Q.aggs[2][0] != a || Q.aggs[2][1] != a) return false;
    if (y < 0) y = a;
    return y == a;
  };
  const int n = spec->n_candidates;
  ptrs.assign((size_t)2 * n + 2, nullptr);
  for (int i = 0; i < n; ++i) {
    const lmfao_cart_candidate& c = spec->candidates[i];
    if (!agg_ok(c.query)) return set_err(LMFAO_EINVAL, "candidate query without SUM(1), SUM(y), SUM(y*y)");
    if (c.kind != LMFAO_CART_LE && c.kind != LMFAO_CART_EQ) return set_err(LMFAO_EINVAL, "bad candidate kind");
    int nk = 0;
    const OutBuf& B = user_out(prep, c.query, &nk);
    if (B.hash >= 0) return set_err(LMFAO_EINVAL, "candidate query kept in a hash table");
    if ((c.kind == LMFAO_CART_LE && (nk != 0 || c.group != 0)) || (c.kind == LMFAO_CART_EQ && nk != 1) ||
        c.group < 0 || c.group >= B.n_rows)
      return set_err(LMFAO_EINVAL, "candidate group row does not match its query");
    ptrs[i] = B.cnt + c.group;
    ptrs[n + i] = (const double*)B.vals + c.group * B.n_vals;
  }
  int nk = 0;
  if (!agg_ok(spec->total_query)) return set_err(LMFAO_EINVAL, "total query without SUM(1), SUM(y), SUM(y*y)");
  const OutBuf& T = user_out(prep, spec->total_query, &nk);
  if (nk != 0 || T.hash >= 0) return set_err(LMFAO_EINVAL, "total query has group-by attributes");
  ptrs[2 * n] = T.cnt;
  ptrs[2 * n + 1] = T.vals;
  return LMFAO_OK;
}

// uploads the pointers and runs the split kernel; *best on the host
static lmfao_status cart_split(lmfao_prepared_s* prep, const lmfao_cart_spec* spec,
                               const std::vector<const void*>& ptrs, double* costs, lmfao_cart_split* out,
                               hipStream_t st) {
  const int n = spec->n_candidates;
  const size_t need = ptrs.size() * 8 + sizeof(DCartBest) + (size_t)std::max(n, 1) * 8 + 256;
  try {
    if (prep->cart_bytes < need) {
      prep->cart_dev = dalloc(*prep, need);
      prep->cart_bytes = need;
    }
    char* base = (char*)prep->cart_dev;
    const void** dptr = (const void**)base;
    DCartBest* dbest = (DCartBest*)(base + ((ptrs.size() * 8 + 255) & ~(size_t)255));
    double* dcost = costs ? costs : (double*)((char*)dbest + 256);
    HIP_OK(hipMemcpyAsync(dptr, ptrs.data(), ptrs.size() * 8, hipMemcpyHostToDevice, st));
    launch_cart_split((const int64_t* const*)dptr, (const double* const*)(dptr + n), n,
                      (const int64_t*)ptrs[2 * n], (const double*)ptrs[2 * n + 1], spec->min_leaf, spec->tie_eps,
                      dcost, dbest, st);
    HIP_OK(hipGetLastError());
    DCartBest b{};
    HIP_OK(hipMemcpyAsync(&b, dbest, sizeof b, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *out = lmfao_cart_split{b.best, 0, b.n, b.n_left, b.n_right, b.sy, b.sy2, b.sy_left, b.sy2_left, b.cost};
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

}  // namespace lmfao

extern "C" {

lmfao_status lmfao_cart_best_split(lmfao_prepared_t prep, const lmfao_cart_spec* spec, lmfao_cart_split* out,
                                   double* costs, void* stream) {
  clear_error();
  if (!prep || !out) return set_err(LMFAO_EINVAL, "null argument");
  std::vector<const void*> ptrs;
  if (lmfao_status e = cart_inputs(prep, spec, ptrs)) return e;
  if (lmfao_status e = read_flags(prep)) return e;
  return cart_split(prep, spec, ptrs, costs, out, (hipStream_t)stream);
}

lmfao_status lmfao_cart_grow(lmfao_plan_t plan, lmfao_prepared_t prep, const void* const* const* columns,
                             const lmfao_cart_spec* spec, lmfao_cart_node* nodes, int32_t cap, int32_t* n_nodes,
                             void* stream) {
  clear_error();
  if (!plan || !prep || prep->P != plan->P || !columns || !nodes || !n_nodes || cap < 1)
    return set_err(LMFAO_EINVAL, "null argument");
  std::vector<const void*> ptrs;
  if (lmfao_status e = cart_inputs(prep, spec, ptrs)) return e;
  if (spec->max_depth < 0 || spec->max_depth > kMaxFilterConds)
    return set_err(LMFAO_EINVAL, "max_depth must be between 0 and 8");
  const Plan& P = *prep->P;
  hipStream_t st = (hipStream_t)stream;
  // the relation (with row weights) and column holding each candidate's attribute
  const int nc = spec->n_candidates;
  std::vector<int> crel(nc), ccol(nc);
  for (int i = 0; i < nc; ++i) {
    const char* nm = spec->candidates[i].attr;
    auto it = nm ? P.attr_id.find(nm) : P.attr_id.end();
    if (it == P.attr_id.end()) return set_err(LMFAO_EINVAL, "unknown candidate attribute");
    crel[i] = -1;
    for (size_t r = 0; r < P.rels.size() && crel[i] < 0; ++r)
      if (prep->row_w[r] && P.rels[r].has(it->second) && P.rels[r].col.at(it->second) < P.rels[r].n_input_attrs) {
        crel[i] = (int)r;
        ccol[i] = P.rels[r].col.at(it->second);
      }
    if (crel[i] < 0) return set_err(LMFAO_EINVAL, "a candidate attribute is held by no relation with row weights");
  }
  struct Pending {
    int parent, depth;
    std::vector<std::pair<int, bool>> path;
    int64_t n;             // statistics from the parent's split (leaves at max_depth)
    double sy, sy2;
  };
  auto var_of = [](int64_t n, double sy, double sy2) { return n > 0 ? sy2 - sy * sy / (double)n : 0.0; };
  std::vector<Pending> queue{{-1, 0, {}, 0, 0.0, 0.0}};
  int count = 0;
  for (size_t qi = 0; qi < queue.size(); ++qi) {
    if (count >= cap) return set_err(LMFAO_EINVAL, "node array too small");
    const Pending nd = queue[qi];
    lmfao_cart_node& out = nodes[count];
    out = lmfao_cart_node{nd.parent, nd.depth, -1, -1, -1, 0, nd.n, nd.sy, nd.sy2, var_of(nd.n, nd.sy, nd.sy2)};
    const int self = count++;
    if (nd.depth >= spec->max_depth) continue;   // a leaf, statistics from its parent's split
    // the path condition, pushed into the row weights of the relations holding its attributes
    try {
      for (size_t r = 0; r < P.rels.size(); ++r) {
        if (!prep->row_w[r]) continue;
        DFilter f{};
        f.n_rows = P.rels[r].n_rows;
        f.out = prep->row_w[r];
        for (const auto& pc : nd.path) {
          const int i = pc.first;
          if (crel[i] != (int)r) continue;
          const lmfao_cart_candidate& c = spec->candidates[i];
          const int dt = P.rels[r].dtypes[ccol[i]];
          f.cols[f.n_conds] = DCol{columns[r][ccol[i]], dt, 0};
          f.op[f.n_conds] = c.kind == LMFAO_CART_LE ? (pc.second ? LMFAO_LE : LMFAO_GT)
                                                    : (pc.second ? LMFAO_EQ : LMFAO_NE);
          f.c[f.n_conds] = dt == LMFAO_F32 ? (double)(float)c.value : c.value;
          f.n_conds++;
        }
        launch_filter_value(f, st);
      }
      HIP_OK(hipGetLastError());
    } catch (const HipError& e) {
      return set_err(LMFAO_EHIP, e.msg);
    }
    if (lmfao_status e = lmfao_run(plan, prep, stream, 0)) return e;
    if (lmfao_status e = read_flags(prep)) return e;
    lmfao_cart_split sp{};
    if (lmfao_status e = cart_split(prep, spec, ptrs, nullptr, &sp, st)) return e;
    out.n = sp.n;
    out.sum_y = sp.sum_y;
    out.sum_y2 = sp.sum_y2;
    out.cost = sp.cost;
    if (sp.best < 0) continue;
    out.split = sp.best;
    // children in breadth-first order: left (the candidate holds), then right
    Pending L{self, nd.depth + 1, nd.path, sp.n_left, sp.sum_y_left, sp.sum_y2_left};
    Pending R{self, nd.depth + 1, nd.path, sp.n_right, sp.sum_y - sp.sum_y_left, sp.sum_y2 - sp.sum_y2_left};
    L.path.push_back({sp.best, true});
    R.path.push_back({sp.best, false});
    out.left = (int32_t)queue.size();
    out.right = (int32_t)queue.size() + 1;
    queue.push_back(L);
    queue.push_back(R);
  }
  *n_nodes = count;
  return LMFAO_OK;
}
lmfao_status lmfao_ridge_sigma(lmfao_prepared_t prep, int32_t n_cont, const char* const* cont, int32_t n_cat,
                               const char* const* cat, double* sigma, int32_t* dim_out, void* stream) {
  clear_error();
  if (!prep || n_cont < 0 || n_cat < 0 || (n_cont && !cont) || (n_cat && !cat))
    return set_err(LMFAO_EINVAL, "null argument");
  const Plan& P = *prep->P;
  auto lookup = [&](const char* nm, int& id) {
    if (!nm) return false;
    auto it = P.attr_id.find(nm);
    if (it == P.attr_id.end()) return false;
    id = it->second;
    return true;
  };
  std::vector<int> ca(n_cont), ka(n_cat);
  for (int i = 0; i < n_cont; ++i)
    if (!lookup(cont[i], ca[i])) return set_err(LMFAO_EINVAL, "unknown continuous attribute");
  std::vector<int64_t> off(n_cat);
  int64_t dim = 1 + n_cont;
  for (int i = 0; i < n_cat; ++i) {
    if (!lookup(cat[i], ka[i]) || P.attrs[ka[i]].dtype != LMFAO_I32 || P.attrs[ka[i]].domain <= 0)
      return set_err(LMFAO_EINVAL, "categorical attribute unknown or without a domain");
    off[i] = dim;
    dim += P.attrs[ka[i]].domain;
  }
  if (dim > kRidgeMaxDim) return set_err(LMFAO_EUNSUPPORTED, "covariance matrix larger than 2048 x 2048");
  if (dim_out) *dim_out = (int32_t)dim;
  if (!sigma) return LMFAO_OK;
  // (group-by attributes, monomial) -> output values of a planned query without a range
  std::map<std::pair<std::vector<int>, Mono>, std::pair<const OutBuf*, int>> have;
  for (size_t u = 0; u < P.user.size(); ++u) {
    if (P.user[u].range || prep->qout[P.user[u].internal].hash >= 0) continue;
    const QueryDef& Q = P.queries[P.user[u].internal];
    for (size_t k = 0; k < Q.aggs.size(); ++k)
      have.emplace(std::make_pair(Q.groupby, Q.aggs[k]), std::make_pair(&prep->qout[P.user[u].internal], (int)k));
  }
  std::vector<DSigmaEntry> ent;
  std::string missing;
  auto find = [&](std::vector<int> gb, Mono m, int64_t row, int a, int b) {
    std::sort(m.begin(), m.end());
    auto it = have.find({gb, m});
    if (it == have.end()) {
      missing = "the batch has no query for a covariance entry";
      return;
    }
    const OutBuf* B = it->second.first;
    ent.push_back(DSigmaEntry{(const double*)B->vals + row * B->n_vals + it->second.second, a, b});
  };
  // continuous block, the intercept first
  for (int i = 0; i <= n_cont; ++i)
    for (int j = i; j <= n_cont; ++j) {
      Mono m;
      if (i) m.push_back(ca[i - 1]);
      if (j) m.push_back(ca[j - 1]);
      find({}, m, 0, i, j);
    }
  for (int c = 0; c < n_cat; ++c) {
    const int64_t dc = P.attrs[ka[c]].domain;
    for (int64_t v = 0; v < dc; ++v) {
      for (int i = 0; i <= n_cont; ++i) {
        Mono m;
        if (i) m.push_back(ca[i - 1]);
        find({ka[c]}, m, v, (int)(off[c] + v), i);
      }
      find({ka[c]}, {}, v, (int)(off[c] + v), (int)(off[c] + v));
    }
    for (int c2 = c + 1; c2 < n_cat; ++c2) {
      const int64_t d2 = P.attrs[ka[c2]].domain;
      const bool fwd = have.count({{ka[c], ka[c2]}, Mono{}}) != 0;
      for (int64_t v = 0; v < dc; ++v)
        for (int64_t w = 0; w < d2; ++w) {
          if (fwd) find({ka[c], ka[c2]}, {}, v * d2 + w, (int)(off[c] + v), (int)(off[c2] + w));
          else find({ka[c2], ka[c]}, {}, w * dc + v, (int)(off[c] + v), (int)(off[c2] + w));
        }
    }
  }
  if (!missing.empty()) return set_err(LMFAO_EINVAL, missing);
  try {
    hipStream_t st = (hipStream_t)stream;
    DSigmaEntry* d = nullptr;
    HIP_OK(hipMalloc(&d, std::max<size_t>(1, ent.size()) * sizeof(DSigmaEntry)));
    HIP_OK(hipMemcpyAsync(d, ent.data(), ent.size() * sizeof(DSigmaEntry), hipMemcpyHostToDevice, st));
    launch_sigma_assemble(d, (int64_t)ent.size(), sigma, (int)dim, st);
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipFree(d));
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

lmfao_status lmfao_ridge_bgd(const double* sigma, int32_t dim, int32_t label, double lambda, double eta,
                             int32_t max_iter, double tol, double* theta, double* stats, void* stream) {
  clear_error();
  if (!sigma || !theta || !stats) return set_err(LMFAO_EINVAL, "null argument");
  if (dim < 2 || dim > kRidgeMaxDim || label < 0 || label >= dim || max_iter < 0 || !(lambda >= 0))
    return set_err(LMFAO_EINVAL, "bad dimension, label, iteration count or lambda");
  try {
    hipStream_t st = (hipStream_t)stream;
    double* out = nullptr;
    HIP_OK(hipMalloc(&out, 3 * sizeof(double)));
    launch_ridge_bgd(sigma, dim, label, lambda, eta, max_iter, tol, theta, out, st);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(stats, out, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipFree(out));
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

lmfao_status lmfao_view_shape(lmfao_prepared_t prep, int32_t v, int64_t* n_keys, int32_t* n_vals,
                              int32_t* n_codes) {
  if (!prep || v < 0 || v >= (int)prep->vout.size()) return set_err(LMFAO_EINVAL, "bad view index");
  const OutBuf& B = prep->vout[v];
  if (n_keys) *n_keys = B.n_rows;
  if (n_vals) *n_vals = B.n_vals;
  if (n_codes) *n_codes = B.n_codes;
  return LMFAO_OK;
}

lmfao_status lmfao_view_copy(lmfao_prepared_t prep, int32_t v, int64_t* counts, double* values, int32_t* codes) {
  if (!prep || v < 0 || v >= (int)prep->vout.size()) return set_err(LMFAO_EINVAL, "bad view index");
  const OutBuf& B = prep->vout[v];
  if (lmfao_status fs = read_flags(prep)) return fs;
  try {
    if (counts) HIP_OK(hipMemcpy(counts, B.cnt, B.n_rows * 8, hipMemcpyDeviceToHost));
    if (values && B.n_vals) {
      size_t n = (size_t)B.n_rows * B.n_vals;
      if (B.f64) {
        HIP_OK(hipMemcpy(values, B.vals, n * 8, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> tmp(n);
        HIP_OK(hipMemcpy(tmp.data(), B.vals, n * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i) values[i] = tmp[i];
      }
    }
    if (codes && B.n_codes) HIP_OK(hipMemcpy(codes, B.codes, (size_t)B.n_rows * B.n_codes * 4, hipMemcpyDeviceToHost));
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

lmfao_status lmfao_set_timing(lmfao_prepared_t prep, int32_t on) {
  if (!prep) return set_err(LMFAO_EINVAL, "null prepared handle");
  prep->timing = on != 0;
  return LMFAO_OK;
}

lmfao_status lmfao_run_timing(lmfao_prepared_t prep, int32_t cap, const char** names, float* ms, int32_t* n) {
  if (!prep) return set_err(LMFAO_EINVAL, "null prepared handle");
  int slots = timed_slots(*prep);
  if (prep->timed_runs > 0) {
    // mean over the runs recorded since the last call; entry 0 = whole run
    prep->step_ms.assign(slots, 0.f);
    try {
      HIP_OK(hipDeviceSynchronize());
      for (int r = 0; r < prep->timed_runs; ++r)
        for (int k = 0; k < slots; ++k) {
          float x = 0;
          int b = r * slots * 2;
          HIP_OK(hipEventElapsedTime(&x, prep->ev[b + 2 * k], prep->ev[b + 2 * k + 1]));
          prep->step_ms[k] += x / prep->timed_runs;
        }
    } catch (const HipError& e) {
      return set_err(LMFAO_EHIP, e.msg);
    }
    prep->timed_runs = 0;
  }
  int32_t k = (int32_t)prep->step_ms.size();
  if (n) *n = k;
  static const char* whole = "run";
  std::vector<const char*> nm{whole};
  for (auto& s : prep->steps)
    if (timed_step(s)) nm.push_back(s.name.c_str());
  for (int32_t i = 0; i < std::min(cap, k); ++i) {
    if (names) names[i] = nm[i];
    if (ms) ms[i] = prep->step_ms[i];
  }
  return LMFAO_OK;
}

lmfao_status lmfao_prepared_features(lmfao_prepared_t prep, int32_t q, float* feats) {
  if (!prep || !feats) return set_err(LMFAO_EINVAL, "null argument");
  const Plan& P = *prep->P;
  if (q < 0 || q >= (int)P.user.size()) return set_err(LMFAO_EINVAL, "query index out of range");
  const QueryDef& Q = P.queries[P.user[q].internal];
  if (Q.groupby.empty()) return set_err(LMFAO_EINVAL, "query has no group-by attributes");
  try {
    query_features(*prep, Q, feats, prep->stream);
  } catch (const PlanError& e) {
    return set_err(e.status, e.msg);
  } catch (const HipError& e) {
    return set_err(LMFAO_EHIP, e.msg);
  }
  return LMFAO_OK;
}

lmfao_status lmfao_prepared_kernel_source(lmfao_prepared_t prep, int32_t i, char* buf, size_t cap, size_t* need) {
  if (!prep) return set_err(LMFAO_EINVAL, "null prepared handle");
  if (i < 0 || i >= (int)prep->gen_sources.size()) return set_err(LMFAO_EINVAL, "no generated kernel with that index");
  const std::string& j = prep->gen_sources[i];
  if (need) *need = j.size() + 1;
  if (buf && cap) {
    size_t n = std::min(cap - 1, j.size());
    std::memcpy(buf, j.data(), n);
    buf[n] = 0;
  }
  return LMFAO_OK;
}

lmfao_status lmfao_prepared_describe(lmfao_prepared_t prep, char* buf, size_t cap, size_t* need) {
  if (!prep) return set_err(LMFAO_EINVAL, "null prepared handle");
  std::string j = "{\"steps\":[";
  bool first = true;
  for (auto& s : prep->steps) {
    if (s.kind == 0) continue;
    if (!first) j += ",";
    first = false;
    static const char* kinds[] = {"fill",  "view_build", "scan",     "table_reduce", "contract", "merge",
                                  "image", "stage",      "contract", "merge",        "filter",   "finalize",
                                  "scatter", "count_copy", "mult_check", "partition"};
    static_assert(sizeof(kinds) / sizeof(kinds[0]) == 16, "one name per step kind");
    char tmp[512];
    snprintf(tmp, sizeof(tmp),
             "{\"name\":\"%s\",\"kind\":\"%s\",\"rows\":%lld,\"pieces\":%lld,\"alg_read_bytes\":%.0f,"
             "\"alg_write_bytes\":%.0f,\"alg_flop\":%.0f,\"grid\":%d,\"grid_y\":%d,\"lds\":%d,\"lean\":%d",
             s.name.c_str(), kinds[s.kind], (long long)s.rows, (long long)s.pieces, s.alg_read, s.alg_write,
             s.alg_flop, s.grid, s.grid_y, s.lds, s.gen_fn ? 2 : s.fast);
    j += tmp;
    if (s.relation >= 0) {
      const RelDef& R = prep->P->rels[s.relation];
      double pass = 0;
      std::string pc, pw;
      for (size_t k = 0; k < s.pass_cols.size(); ++k) {
        const int w = R.dtypes[s.pass_cols[k]] == LMFAO_F64 ? 8 : 4;
        pass += (double)R.n_rows * w;
        pc += (k ? "," : "") + std::to_string(s.pass_cols[k]);
        pw += (k ? "," : "") + std::to_string(w);
      }
      j += ",\"relation\":\"" + R.name + "\",\"relation_rows\":" + std::to_string(R.n_rows) +
           ",\"pass_read_bytes\":" + std::to_string((long long)pass) + ",\"pass_cols\":[" + pc +
           "],\"pass_col_bytes\":[" + pw + "]";
    }
    j += "}";
  }
  int64_t fill_bytes = 0;
  for (auto& s : prep->steps)
    if (s.kind == 0) fill_bytes += s.bytes;
  j += "],\"fill_bytes\":" + std::to_string(fill_bytes) + ",\"picked_hash\":" + std::to_string(prep->picked_hash) +
       ",\"codegen_failures\":[";
  for (size_t i = 0; i < prep->gen_failures.size(); ++i) {
    if (i) j += ",";
    std::string m;
    for (char ch : prep->gen_failures[i]) {
      if (ch == '"' || ch == '\\') m += '\\';
      if (ch == '\n') { m += "\\n"; continue; }
      if ((unsigned char)ch < 0x20) continue;
      m += ch;
    }
    j += "\"" + m + "\"";
  }
  j += "],\"generated_scans\":" + std::to_string(prep->gen_sources.size());
  j += ",\"hash_tables\":[";
  for (size_t i = 0; i < prep->hashes.size(); ++i) {
    if (i) j += ",";
    const HashBuf& H = prep->hashes[i];
    int user = -1;
    for (size_t u = 0; u < prep->P->user.size() && user < 0; ++u)
      if (prep->P->user[u].internal == H.query) user = (int)u;
    char tmp[160];
    snprintf(tmp, sizeof tmp, "{\"query\":%d,\"slots\":%lld,\"bound\":%lld,\"est_groups\":%.17g}", user,
             (long long)H.cap, (long long)H.bound, H.est);
    j += tmp;
  }
  j += "],\"hash_regrowths\":" + std::to_string(prep->hash_regrowths);
  j += ",\"graph\":{\"captured\":" + std::to_string(prep->graph_exec ? 1 : 0) +
       ",\"failed\":" + std::to_string(prep->graph_failed ? 1 : 0) + "}}";
  if (need) *need = j.size() + 1;
  if (buf && cap) {
    size_t n = std::min(cap - 1, j.size());
    std::memcpy(buf, j.data(), n);
    buf[n] = 0;
  }
  return LMFAO_OK;
}

void lmfao_prepared_free(lmfao_prepared_t prep) { delete prep; }


}  // extern "C"
