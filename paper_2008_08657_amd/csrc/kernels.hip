// HIP kernels for gfx950 (MI355X): 64-lane wavefronts, 160 KB LDS per CU.
//
//  k_fill            zero-fill of views and results
//  k_view_build      views whose subtree has one join tuple per key: one
//                    pass over the relation, dense key-indexed tables (a
//                    thread per output element; k_view_build_rows, a thread
//                    per row, on large relations)
//  k_build_image     per key of a view, the record a scan gathers (factors,
//                    codes, multiplicity), written a dword per lane
//  k_radix_*         stable LSD radix sort of packed trie keys (prepare)
//  k_segment_starts  trie-level segment boundaries of a sorted relation
//  k_scan<T,NA>      the node scan: one wavefront per run of pieces of the
//                    sorted relation; per tuple it looks up the inner views,
//                    multiplies inner factors and accumulates the per-piece
//                    partial sums (running sums of the paper's Figure 3),
//                    per-piece code histograms and direct group-by tables
//  k_contract<T>     per piece: outer views looked up once, outer features
//                    (products of factors and one-hot codes) times the
//                    piece's partial sums, accumulated as a dense block
//                    product over pieces (partial aggregates pushed past the
//                    inner loops); per-block partials, no atomics
//  k_merge_cells     FP64 reduction of the block partials into result cells
//                    (fixed order: deterministic)
//  k_table_reduce    reduction of the scan's LDS-privatized table partials
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "kernels.hpp"

namespace lmfao {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t ld_int(const DCol& c, int64_t r) {
  return (int64_t)((const int32_t*)c.ptr)[r];
}
template <typename T>
__device__ __forceinline__ T ld_val(const DCol& c, int64_t r) {
  if (c.dtype == LMFAO_F32) return (T)((const float*)c.ptr)[r];
  if (c.dtype == LMFAO_F64) return (T)((const double*)c.ptr)[r];
  return (T)((const int32_t*)c.ptr)[r];
}
template <typename T>
__device__ __forceinline__ T view_val(const DView& v, int64_t row, int slot) {
  if (v.vals_f64) return (T)((const double*)v.vals)[row * v.n_vals + slot];
  return (T)((const float*)v.vals)[row * v.n_vals + slot];
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
// Neumaier-compensated accumulation s + c += x for double; plain add for float
__device__ __forceinline__ void kadd(float& s, float& c, float x) { s += x; }
__device__ __forceinline__ void kadd(double& s, double& c, double x) {
  double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}
// wave sum of (s, c) pairs; for double every combining add is error-free
// transformed, so the result carries the lanes' compensations
__device__ __forceinline__ float wave_sum_comp(float s, float c) { return wave_sum(s); }
__device__ __forceinline__ double wave_sum_comp(double s, double c) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double s2 = __shfl_xor(s, o, 64), c2 = __shfl_xor(c, o, 64);
    double t = s + s2;
    double bb = t - s;
    double e = (s - (t - bb)) + (s2 - bb);   // TwoSum error
    s = t;
    c = c + c2 + e;
  }
  return s + c;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

// ---------------------------------------------------------------------------
// scatter targets: dense rows, or a hash table for large key spaces
// ---------------------------------------------------------------------------
constexpr int kMaxProbe = 256;   // linear probes before an insert reports overflow

__device__ __forceinline__ int64_t hash_find(const DHashOut& H, int64_t row) {
  const unsigned long long k = (unsigned long long)row + 1ull;
  unsigned long long h = k * 0x9E3779B97F4A7C15ull;
  h ^= h >> 31;
  int64_t slot = (int64_t)(h & (unsigned long long)H.mask);
  for (int probe = 0; probe < kMaxProbe; ++probe) {
    const unsigned long long cur = __hip_atomic_load(&H.keys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == k) return slot;
    if (cur == 0ull) {
      const unsigned long long prev = atomicCAS(&H.keys[slot], 0ull, k);
      if (prev == 0ull || prev == k) return slot;
    }
    slot = (slot + 1) & H.mask;
  }
  return -1;
}

__device__ __forceinline__ void scatter_count(const DContract* C, int o, int64_t row, int64_t v) {
  const int hi = C->so_hash_idx ? C->so_hash_idx[o] : -1;
  if (hi < 0) {
    atomic_add_i64(&C->so_cnt[o][row], v);
    return;
  }
  const DHashOut& H = C->hash_tab[hi];
  const int64_t slot = hash_find(H, row);
  if (slot < 0) {
    atomicOr(H.ovf, 1);
    atomicOr(C->err_flag, 8);
    return;
  }
  atomic_add_i64(&H.cnt[slot], v);
}

__device__ __forceinline__ void scatter_value(const DContract* C, int o, int64_t row, int comp, double v) {
  const int hi = C->so_hash_idx ? C->so_hash_idx[o] : -1;
  if (hi < 0) {
    const int64_t idx = row * C->so_ncomp[o] + comp;
    if (C->so_vals_f64[o]) atomic_add_f64(&((double*)C->so_vals[o])[idx], v);
    else atomicAdd(&((float*)C->so_vals[o])[idx], (float)v);
    return;
  }
  const DHashOut& H = C->hash_tab[hi];
  const int64_t slot = hash_find(H, row);
  if (slot < 0) {
    atomicOr(H.ovf, 1);
    atomicOr(C->err_flag, 8);
    return;
  }
  atomic_add_f64(&H.vals[slot * H.n_vals + comp], v);
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return;
  if (bytes % 8 == 0) {
    int64_t n = bytes / 8;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, (uint64_t*)p, n, 0ull);
  } else {
    int64_t n = bytes / 4;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, (uint32_t*)p, n, 0u);
  }
}

// ---------------------------------------------------------------------------
// conditions: per-row filter weights and bucket codes of thresholds
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ld_cmp(const DCol& c, int64_t r) {
  if (c.dtype == LMFAO_I32) return (double)((const int32_t*)c.ptr)[r];
  if (c.dtype == LMFAO_F32) return (double)((const float*)c.ptr)[r];
  return ((const double*)c.ptr)[r];
}
__device__ __forceinline__ bool cond_holds(double x, int op, double c) {
  switch (op) {
    case LMFAO_LE: return x <= c;
    case LMFAO_LT: return x < c;
    case LMFAO_GT: return x > c;
    case LMFAO_GE: return x >= c;
    case LMFAO_EQ: return x == c;
    default: return x != c;
  }
}

__device__ __forceinline__ void filter_rows(const DFilter& F) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < F.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    int w = 1;
    if (F.ext) w = F.ext[F.perm ? (int64_t)F.perm[r] : r] != 0 ? 1 : 0;
    for (int k = 0; k < F.n_conds; ++k) w &= cond_holds(ld_cmp(F.cols[k], r), F.op[k], F.c[k]) ? 1 : 0;
    F.out[r] = w;
  }
}
__global__ __launch_bounds__(256) void k_filter(const DFilter* __restrict__ F) { filter_rows(*F); }
__global__ __launch_bounds__(256) void k_filter_value(const DFilter F) { filter_rows(F); }
void launch_filter(const DFilter* d, int64_t n_rows, hipStream_t s) {
  if (n_rows <= 0) return;
  const int grid = (int)std::min<int64_t>((n_rows + 255) / 256, 8192);
  hipLaunchKernelGGL(k_filter, dim3(grid), dim3(256), 0, s, d);
}
void launch_filter_value(const DFilter& f, hipStream_t s) {
  if (f.n_rows <= 0) return;
  const int grid = (int)std::min<int64_t>((f.n_rows + 255) / 256, 8192);
  hipLaunchKernelGGL(k_filter_value, dim3(grid), dim3(256), 0, s, f);
}

// ---------------------------------------------------------------------------
// CART split selection (section 3, decision trees)
// ---------------------------------------------------------------------------
// One workgroup.  Cost of candidate i = VAR(left) + VAR(right) with
// VAR(B) = SUM(y^2) - SUM(y)^2 / |B| (0 for an empty branch), in FP64; a
// candidate is valid when both branches hold at least min_leaf tuples.  The
// least valid cost is found first; the chosen candidate is the first one
// (lowest index) within tie_eps * max(|VAR(node)|, 1) of it.
__device__ __forceinline__ double cart_var(int64_t n, double sy, double sy2) {
  return n > 0 ? sy2 - sy * sy / (double)n : 0.0;
}

__global__ void __launch_bounds__(1024) k_cart_split(const int64_t* const* __restrict__ cand_cnt,
                                                     const double* const* __restrict__ cand_vals, int n_cand,
                                                     const int64_t* __restrict__ tot_cnt,
                                                     const double* __restrict__ tot_vals, int64_t min_leaf,
                                                     double tie_eps, double* __restrict__ costs,
                                                     DCartBest* __restrict__ best) {
  __shared__ double red_d[16];
  __shared__ int red_i[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t n = *tot_cnt;
  const double sy = tot_vals[1], sy2 = tot_vals[2];
  double least = INFINITY;
  for (int i = threadIdx.x; i < n_cand; i += blockDim.x) {
    const int64_t nl = *cand_cnt[i];
    const double syl = cand_vals[i][1], sy2l = cand_vals[i][2];
    const int64_t nr = n - nl;
    const bool ok = nl >= min_leaf && nr >= min_leaf;
    const double c = cart_var(nl, syl, sy2l) + cart_var(nr, sy - syl, sy2 - sy2l);
    costs[i] = ok ? c : INFINITY;
    if (ok) least = fmin(least, c);
  }
  for (int o = 32; o > 0; o >>= 1) least = fmin(least, __shfl_xor(least, o, 64));
  if (lane == 0) red_d[wid] = least;
  __syncthreads();
  least = INFINITY;
  for (int w = 0; w < nw; ++w) least = fmin(least, red_d[w]);
  const double tol = tie_eps * fmax(fabs(cart_var(n, sy, sy2)), 1.0);
  int first = INT_MAX;
  if (least < INFINITY)
    for (int i = threadIdx.x; i < n_cand; i += blockDim.x)
      if (costs[i] <= least + tol) {
        first = min(first, i);
        break;   // later indices of this thread are larger
      }
  for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
  if (lane == 0) red_i[wid] = first;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < nw; ++w) first = min(first, red_i[w]);
    DCartBest b{};
    b.best = first == INT_MAX ? -1 : first;
    b.n = n;
    b.sy = sy;
    b.sy2 = sy2;
    if (b.best >= 0) {
      b.n_left = *cand_cnt[first];
      b.n_right = n - b.n_left;
      b.sy_left = cand_vals[first][1];
      b.sy2_left = cand_vals[first][2];
      b.cost = costs[first];
    } else {
      b.cost = cart_var(n, sy, sy2);
    }
    *best = b;
  }
}

void launch_cart_split(const int64_t* const* cand_cnt, const double* const* cand_vals, int n_cand,
                       const int64_t* tot_cnt, const double* tot_vals, int64_t min_leaf, double tie_eps,
                       double* costs, DCartBest* best, hipStream_t s) {
  hipLaunchKernelGGL(k_cart_split, dim3(1), dim3(1024), 0, s, cand_cnt, cand_vals, n_cand, tot_cnt, tot_vals,
                     min_leaf, tie_eps, costs, best);
}

// a function of an integer attribute, tabulated: out[r] = tab[src[r]]; an
// argument outside the table flags error 2 and gives 0
__global__ __launch_bounds__(256) void k_gather_table(const int32_t* __restrict__ src, int64_t n,
                                                     const double* __restrict__ tab, int64_t nt,
                                                     double* __restrict__ out, int32_t* err) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = src[r];
    const bool ok = v >= 0 && (int64_t)v < nt;
    if (!ok) atomicOr(err, 2);
    out[r] = ok ? tab[v] : 0.0;
  }
}
void launch_gather_table(const int32_t* src, int64_t n, const double* tab, int64_t nt, double* out, int32_t* err,
                         hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_gather_table, dim3(grid), dim3(256), 0, s, src, n, tab, nt, out, err);
}

// bucket = number of thresholds below the value (kind 0) or at most the value
// (kind 1); thresholds sorted ascending, in the column's comparison type
__global__ __launch_bounds__(256) void k_bucketize(DCol src, int64_t n, const double* __restrict__ thr, int n_thr,
                                                   int kind, int32_t* __restrict__ out) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const double x = ld_cmp(src, r);
    int lo = 0, hi = n_thr;   // first index whose threshold is not below (kind 0) / above (kind 1) x
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const bool before = kind == 0 ? thr[mid] < x : thr[mid] <= x;
      if (before) lo = mid + 1;
      else hi = mid;
    }
    out[r] = lo;
  }
}
void launch_bucketize(const void* src, int dtype, int64_t n, const double* thr, int n_thr, int kind, int32_t* out,
                      hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  DCol c{src, dtype, 0};
  hipLaunchKernelGGL(k_bucketize, dim3(grid), dim3(256), 0, s, c, n, thr, n_thr, kind, out);
}

// block per range query, thread per destination row; buckets in order
__global__ __launch_bounds__(256) void k_finalize(const DFinalize* __restrict__ D) {
  const DFinalize& F = D[blockIdx.x];
  for (int64_t r = threadIdx.x; r < F.n_rows; r += blockDim.x) {
    int64_t cnt = 0;
    for (int64_t b = F.lo; b < F.hi; ++b)
      if (b != F.ex) cnt += F.src_cnt[r * F.nb + b];
    F.dst_cnt[r] = cnt;
    for (int k = 0; k < F.n_vals; ++k) {
      double v = 0.0, cc = 0.0;
      for (int64_t b = F.lo; b < F.hi; ++b)
        if (b != F.ex) kadd(v, cc, F.src_vals[(r * F.nb + b) * F.n_vals + k]);
      F.dst_vals[r * F.n_vals + k] = v + cc;
    }
  }
}
void launch_finalize(const DFinalize* d, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(256), 0, s, d);
}

static void allow_lds(const void* fn, int lds) {
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// ---------------------------------------------------------------------------
// ridge regression (section 3, linear regression): the covariance matrix
// from the batch's results, then batch gradient descent in FP64
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sigma_assemble(const DSigmaEntry* __restrict__ e, int64_t n,
                                                        double* __restrict__ S, int dim) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = *e[i].src;
    S[(int64_t)e[i].a * dim + e[i].b] = v;
    S[(int64_t)e[i].b * dim + e[i].a] = v;
  }
}
void launch_sigma_assemble(const DSigmaEntry* e, int64_t n, double* sigma, int dim, hipStream_t s) {
  const int64_t cells = (int64_t)dim * dim;
  launch_fill(sigma, cells * 8, s);
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sigma_assemble, dim3(grid), dim3(256), 0, s, e, n, sigma, dim);
}

constexpr int kRidgeThreads = 1024;

// fixed-order block sum (every thread gets the result)
__device__ double block_sum(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = kRidgeThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// y_i = (Sigma_i. x)/n + lam x_i on the free entries (0 at the label)
__device__ void ridge_apply(const double* S, int dim, int label, double inv_n, double lam, const double* x,
                            double* y) {
  for (int i = threadIdx.x; i < dim; i += kRidgeThreads) {
    double acc = 0.0;
    const double* row = S + (int64_t)i * dim;
    for (int j = 0; j < dim; ++j) acc += row[j] * x[j];
    y[i] = i == label ? 0.0 : acc * inv_n + lam * x[i];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kRidgeThreads) void k_ridge_bgd(const double* __restrict__ S, int dim, int label,
                                                              double lam, double eta, int max_iter, double tol,
                                                              double* __restrict__ theta, double* __restrict__ out) {
  extern __shared__ double sm[];
  double* th = sm;               // [dim]
  double* g = th + dim;          // [dim]
  double* red = g + dim;         // [kRidgeThreads]
  const double inv_n = 1.0 / S[0];
  if (eta <= 0.0) {
    // power iteration on A = Sigma_FF/n + lam I from the all-ones vector
    const double v0 = 1.0 / sqrt((double)(dim - 1));
    for (int i = threadIdx.x; i < dim; i += kRidgeThreads) th[i] = i == label ? 0.0 : v0;
    __syncthreads();
    for (int it = 0; it < 100; ++it) {
      ridge_apply(S, dim, label, inv_n, lam, th, g);
      double p = 0.0;
      for (int i = threadIdx.x; i < dim; i += kRidgeThreads) p += g[i] * g[i];
      const double nrm = sqrt(block_sum(p, red));
      for (int i = threadIdx.x; i < dim; i += kRidgeThreads) th[i] = g[i] / nrm;
      __syncthreads();
    }
    ridge_apply(S, dim, label, inv_n, lam, th, g);
    double p = 0.0;
    for (int i = threadIdx.x; i < dim; i += kRidgeThreads) p += th[i] * g[i];
    eta = 1.0 / block_sum(p, red);
  }
  for (int i = threadIdx.x; i < dim; i += kRidgeThreads) th[i] = i == label ? -1.0 : 0.0;
  __syncthreads();
  int steps = 0;
  double gn = 0.0;
  for (;;) {
    ridge_apply(S, dim, label, inv_n, lam, th, g);
    double p = 0.0;
    for (int i = threadIdx.x; i < dim; i += kRidgeThreads) p += g[i] * g[i];
    gn = sqrt(block_sum(p, red));
    if (gn <= tol || steps >= max_iter) break;
    for (int i = threadIdx.x; i < dim; i += kRidgeThreads)
      if (i != label) th[i] -= eta * g[i];
    __syncthreads();
    ++steps;
  }
  for (int i = threadIdx.x; i < dim; i += kRidgeThreads) theta[i] = th[i];
  if (threadIdx.x == 0) {
    out[0] = (double)steps;
    out[1] = gn;
    out[2] = eta;
  }
}
void launch_ridge_bgd(const double* sigma, int dim, int label, double lam, double eta, int max_iter, double tol,
                      double* theta, double* out, hipStream_t s) {
  const int lds = (2 * dim + kRidgeThreads) * 8;
  allow_lds((const void*)&k_ridge_bgd, lds);
  hipLaunchKernelGGL(k_ridge_bgd, dim3(1), dim3(kRidgeThreads), lds, s, sigma, dim, label, lam, eta, max_iter, tol,
                     theta, out);
}

// ---------------------------------------------------------------------------
// view build for single-valued subtrees
// ---------------------------------------------------------------------------
// One thread per output element: a row of the view is a multiplicity, n_vals
// values and n_codes codes, and a workgroup takes about 256 such elements of
// consecutive relation rows, so that rows which land in order (a relation
// stored in key order) give coalesced stores and a view of a few thousand
// rows still spreads over many workgroups.  Where each element comes from is
// resolved once per workgroup into LDS.  The thread of a row's multiplicity
// also checks that the key is unique.
constexpr int kVBCols = 1 + 64 + kMaxOuterCodes;
enum VBSrc : int8_t { VB_I32 = 0, VB_F32 = 1, VB_F64 = 2, VB_VIEW_F32 = 3, VB_VIEW_F64 = 4, VB_VIEW_CODE = 5 };

template <typename T>
__global__ __launch_bounds__(256) void k_view_build(const DViewBuild* __restrict__ B) {
  __shared__ const void* s_ptr[kVBCols];
  __shared__ int32_t s_slot[kVBCols], s_stride[kVBCols];
  __shared__ int8_t s_src[kVBCols], s_view[kVBCols];
  const int64_t n = B->n_rows;
  const int nvals = B->n_vals, ncodes = B->n_codes;
  const int width = 1 + nvals + ncodes;
  for (int c = threadIdx.x; c < width; c += 256) {
    const void* p = nullptr;
    int8_t src = VB_I32, view = -1;
    int32_t slot = 0, stride = 0;
    if (c >= 1 && c <= nvals) {
      const int sl = c - 1;
      if (B->val_kind[sl] == SRC_COL) {
        const DCol& C = B->cols[B->val_src[sl]];
        p = C.ptr;
        src = C.dtype == LMFAO_F64 ? VB_F64 : C.dtype == LMFAO_F32 ? VB_F32 : VB_I32;
      } else {
        view = (int8_t)B->val_src[sl];
        const DView& V = B->views[view];
        p = V.vals;
        src = V.vals_f64 ? VB_VIEW_F64 : VB_VIEW_F32;
        slot = B->val_slot[sl];
        stride = V.n_vals;
      }
    } else if (c > nvals) {
      const int sl = c - 1 - nvals;
      if (B->code_kind[sl] == SRC_COL) {
        p = B->cols[B->code_src[sl]].ptr;
      } else {
        view = (int8_t)B->code_src[sl];
        const DView& V = B->views[view];
        p = V.codes;
        src = VB_VIEW_CODE;
        slot = B->code_slot[sl];
        stride = V.n_codes;
      }
    }
    s_ptr[c] = p;
    s_src[c] = src;
    s_view[c] = view;
    s_slot[c] = slot;
    s_stride[c] = stride;
  }
  __syncthreads();
  const int rpt = width >= 256 ? 1 : 256 / width;   // relation rows per tile
  const int64_t n_tiles = (n + rpt - 1) / rpt;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t r0 = t * rpt;
    const int m = (int)(n - r0 < rpt ? n - r0 : rpt);
    for (int j = threadIdx.x; j < m * width; j += 256) {
      const int i = j / width, col = j - i * width;
      const int64_t r = r0 + i;
      int64_t row = 0;
      for (int k = 0; k < B->nkey; ++k) row += ld_int(B->cols[B->key_col[k]], r) * B->key_stride[k];
      const int my_view = s_view[col];
      int64_t mu = 1, my_vr = 0;
      for (int v = 0; v < B->n_views; ++v) {
        const DView& V = B->views[v];
        int64_t vr = 0;
        for (int k = 0; k < V.nkey; ++k) vr += ld_int(B->cols[V.key_src[k]], r) * V.key_stride[k];
        mu *= V.cnt[vr];
        if (v == my_view) my_vr = vr;
      }
      if (B->w) mu *= B->w[r];
      if (mu == 0) continue;
      const void* p = s_ptr[col];
      const int src = s_src[col];
      const int64_t at = my_view >= 0 ? my_vr * s_stride[col] + s_slot[col] : r;
      if (col == 0) {
        unsigned long long old = atomicAdd((unsigned long long*)&B->out_cnt[row], (unsigned long long)mu);
        if (old != 0 || mu != 1) atomicOr(B->err_flag, 1);   // key not unique
      } else if (col <= nvals) {
        T x;
        if (src == VB_F64 || src == VB_VIEW_F64) x = (T)((const double*)p)[at];
        else if (src == VB_F32 || src == VB_VIEW_F32) x = (T)((const float*)p)[at];
        else x = (T)((const int32_t*)p)[at];
        ((T*)B->out_vals)[row * nvals + (col - 1)] = x;
      } else {
        B->out_codes[row * ncodes + (col - 1 - nvals)] = ((const int32_t*)p)[at];
      }
    }
  }
}

// One thread per relation row, for large relations: every element of a row
// is written by the row's thread, with the value and code loops uniform over
// the workgroup (descriptor reads stay scalar).
template <typename T>
__global__ __launch_bounds__(256) void k_view_build_rows(const DViewBuild* __restrict__ B) {
  const int64_t n = B->n_rows;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = 0;
    for (int k = 0; k < B->nkey; ++k) row += ld_int(B->cols[B->key_col[k]], r) * B->key_stride[k];
    int64_t mu = 1;
    int64_t vrow[kMaxViews];
    for (int v = 0; v < B->n_views; ++v) {
      const DView& V = B->views[v];
      int64_t vr = 0;
      for (int k = 0; k < V.nkey; ++k) vr += ld_int(B->cols[V.key_src[k]], r) * V.key_stride[k];
      vrow[v] = vr;
      mu *= V.cnt[vr];
    }
    if (B->w) mu *= B->w[r];
    if (mu == 0) continue;
    unsigned long long old = atomicAdd((unsigned long long*)&B->out_cnt[row], (unsigned long long)mu);
    if (old != 0 || mu != 1) atomicOr(B->err_flag, 1);   // key not unique
    auto val = [&](int sl) -> T {
      if (B->val_kind[sl] == SRC_COL) return ld_val<T>(B->cols[B->val_src[sl]], r);
      const int v = B->val_src[sl];
      return view_val<T>(B->views[v], vrow[v], B->val_slot[sl]);
    };
    auto code = [&](int sl) -> int32_t {
      if (B->code_kind[sl] == SRC_COL) return (int32_t)ld_int(B->cols[B->code_src[sl]], r);
      const int v = B->code_src[sl];
      return B->views[v].codes[vrow[v] * B->views[v].n_codes + B->code_slot[sl]];
    };
    // 16-byte stores where the row stride allows (view buffers are 256-byte
    // aligned): a quarter of the store instructions of one per element
    T* ov = (T*)B->out_vals;
    const int nv = B->n_vals, nc = B->n_codes;
    if constexpr (sizeof(T) == 4) {
      if ((nv & 3) == 0) {
        for (int sl = 0; sl < nv; sl += 4)
          *(float4*)(ov + row * nv + sl) = make_float4(val(sl), val(sl + 1), val(sl + 2), val(sl + 3));
      } else {
        for (int sl = 0; sl < nv; ++sl) ov[row * nv + sl] = val(sl);
      }
    } else {
      if ((nv & 1) == 0) {
        for (int sl = 0; sl < nv; sl += 2) *(double2*)(ov + row * nv + sl) = make_double2(val(sl), val(sl + 1));
      } else {
        for (int sl = 0; sl < nv; ++sl) ov[row * nv + sl] = val(sl);
      }
    }
    if ((nc & 1) == 0) {
      for (int sl = 0; sl < nc; sl += 2) *(int2*)(B->out_codes + row * nc + sl) = make_int2(code(sl), code(sl + 1));
    } else {
      for (int sl = 0; sl < nc; ++sl) B->out_codes[row * nc + sl] = code(sl);
    }
  }
}

void launch_view_build(const DViewBuild* d, int64_t n_rows, bool f64, hipStream_t s) {
  if (n_rows <= 0) return;
  if (n_rows >= kViewBuildRowsMin) {
    // large relations: a thread per row (measured faster there than a thread
    // per element, whose keys are re-read once per element)
    const int grid = (int)std::min<int64_t>((n_rows + 255) / 256, 8192);
    if (f64) hipLaunchKernelGGL(k_view_build_rows<double>, dim3(grid), dim3(256), 0, s, d);
    else hipLaunchKernelGGL(k_view_build_rows<float>, dim3(grid), dim3(256), 0, s, d);
    return;
  }
  // a tile holds 256 / (1 + n_vals + n_codes) rows, at least one: one
  // workgroup per row covers every tile, the surplus exits at once
  const int grid = (int)std::min<int64_t>(n_rows, 8192);
  if (f64) hipLaunchKernelGGL(k_view_build<double>, dim3(grid), dim3(256), 0, s, d);
  else hipLaunchKernelGGL(k_view_build<float>, dim3(grid), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------------------
// prepare: packed trie keys and LSD radix sort (8-bit digits, stable)
// ---------------------------------------------------------------------------
__global__ void k_make_keys(const DKeyCols* __restrict__ K, uint64_t* keys, uint32_t* idx, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = 0;
    for (int j = 0; j < K->n; ++j) {
      int64_t v = ((const int32_t*)K->cols[j])[i];
      if (v < 0 || v >= K->dom[j]) { atomicOr(K->err_flag, 2); v = 0; }
      k = k * (uint64_t)K->dom[j] + (uint64_t)v;
    }
    keys[i] = k;
    idx[i] = (uint32_t)i;
  }
}

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                             int shift, uint32_t* hist, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    int64_t i = base + j * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// ---------------------------------------------------------------------------
// exclusive scan of a uint32 array over many workgroups: per tile of
// kScanTile values its sum, a scan of the tile sums in one workgroup, then
// every tile rescanned from its offset (in place); the total is written
// after the tile sums (bsum[n_tiles])
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t x = __shfl_up(incl, d, 64);
    if (lane >= d) incl += x;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t x = wsum[w];
    before += w < wid ? x : 0u;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint32_t* __restrict__ a, int64_t m,
                                                           uint32_t* __restrict__ bsum) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) s += base + u < m ? a[base + u] : 0u;
  uint32_t total;
  (void)block_scan_excl(s, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t* __restrict__ bsum, int64_t nb) {
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? bsum[b] : 0u;
    uint32_t total;
    const uint32_t ex = block_scan_excl(v, &total);
    if (b < nb) bsum[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_rescan(uint32_t* __restrict__ a, int64_t m,
                                                             const uint32_t* __restrict__ bsum) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer], s = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    v[u] = base + u < m ? a[base + u] : 0u;
    s += v[u];
  }
  uint32_t total;
  uint32_t run = bsum[blockIdx.x] + block_scan_excl(s, &total);
#pragma unroll
  for (int u = 0; u < kScanPer; ++u)
    if (base + u < m) {
      a[base + u] = run;
      run += v[u];
    }
}

int64_t scan_tiles(int64_t m) { return (m + kScanTile - 1) / kScanTile; }

void launch_scan_excl(uint32_t* a, int64_t m, uint32_t* bsum, hipStream_t s) {
  const int64_t nb = scan_tiles(m);
  if (nb > 0) hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, m, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, bsum, nb);
  if (nb > 0) hipLaunchKernelGGL(k_tile_rescan, dim3((unsigned)nb), dim3(kScanThreads), 0, s, a, m, bsum);
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* kout, uint32_t* vout, int64_t n,
                                                                int shift, const uint32_t* __restrict__ offs,
                                                                int nblocks) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kSortThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    int64_t i = base + j * kSortThreads + tid;
    bool valid = i < n;
    uint64_t k = valid ? kin[i] : 0;
    uint32_t v = valid ? vin[i] : 0;
    uint32_t d = valid ? (uint32_t)((k >> shift) & 255u) : 256u;
    for (int q = 0; q < kSortThreads / 64; ++q) wcnt[q][tid] = 0;   // 256 digits, one per thread
    __syncthreads();
    // peers with the same digit inside the wavefront
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      uint64_t b = __ballot(valid && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? b : ~b;
    }
    uint32_t rank = __popcll(peers & lt);
    uint32_t total = __popcll(peers);
    bool leader = valid && rank == 0;
    if (leader) wcnt[w][d] = total;
    __syncthreads();
    if (valid) {
      uint32_t before = 0;
      for (int q = 0; q < w; ++q) before += wcnt[q][d];
      uint32_t dst = run[d] + before + rank;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    {
      uint32_t s = 0;
      for (int q = 0; q < kSortThreads / 64; ++q) s += wcnt[q][tid];
      run[tid] += s;
    }
    __syncthreads();
  }
}

void launch_sort(uint64_t* keys, uint32_t* idx, uint64_t* keys_tmp, uint32_t* idx_tmp, int64_t n, int bits,
                 uint32_t* hist, hipStream_t s, bool* swapped) {
  int nblocks = (int)((n + kSortTile - 1) / kSortTile);
  int passes = (bits + 7) / 8;
  uint64_t *ka = keys, *kb = keys_tmp;
  uint32_t *va = idx, *vb = idx_tmp;
  for (int p = 0; p < passes; ++p) {
    int shift = p * 8;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortThreads), 0, s, ka, n, shift, hist, nblocks);
    launch_scan_excl(hist, (int64_t)256 * nblocks, hist + (int64_t)256 * nblocks, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift,
                       hist, nblocks);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *swapped = (passes % 2) == 1;
}

int sort_tile() { return kSortTile; }

// ---------------------------------------------------------------------------
// result compaction (present groups, lexicographic order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool compact_present(const DCompact& D, int64_t i) {
  return (!D.hkeys || D.hkeys[i] != 0ull) && D.cnt[i] > 0;
}

__device__ __forceinline__ void compact_emit_one(const DCompact& D, int64_t p, int64_t row, int64_t slot) {
  for (int k = 0; k < D.n_keys; ++k) D.keys_out[p * D.n_keys + k] = (row / D.stride[k]) % D.dom[k];
  const int64_t c = D.cnt[slot];
  D.cnt_out[p] = c;
  for (int j = 0; j < D.n_vals; ++j)
    D.vals_out[p * D.n_vals + j] =
        (D.vals ? D.vals[slot * D.n_vals + j] : 0.0) + (((D.copy_mask >> j) & 1ull) ? (double)c : 0.0);
}

__global__ void k_compact_flags(const DCompact D) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D.n_src; i += (int64_t)gridDim.x * blockDim.x)
    D.pos[i] = compact_present(D, i) ? 1u : 0u;
}

__global__ void k_compact_place(const DCompact D) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D.n_src;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!compact_present(D, i)) continue;
    const int64_t p = D.pos[i];
    if (D.hkeys) {
      D.rows[p] = D.hkeys[i] - 1ull;
      D.slot[p] = (uint32_t)i;
    } else {
      compact_emit_one(D, p, i, i);
    }
  }
}

__global__ void k_compact_emit(const DCompact D, int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
    compact_emit_one(D, p, (int64_t)D.rows[p], (int64_t)D.slot[p]);
}

void launch_compact(const DCompact& d, hipStream_t s) {
  const int grid = (int)std::min<int64_t>(std::max<int64_t>((d.n_src + 255) / 256, 1), 8192);
  hipLaunchKernelGGL(k_compact_flags, dim3(grid), dim3(256), 0, s, d);
  launch_scan_excl(d.pos, d.n_src, d.pos + d.n_src, s);
  hipLaunchKernelGGL(k_compact_place, dim3(grid), dim3(256), 0, s, d);
}

void launch_compact_emit(const DCompact& d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_compact_emit, dim3(grid), dim3(256), 0, s, d, n);
}

__global__ void k_validate(const int32_t* __restrict__ col, int64_t n, int64_t dom, int32_t* err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = col[i];
    if (v < 0 || (int64_t)v >= dom) atomicOr(err, 2);
  }
}
void launch_validate(const int32_t* col, int64_t n, int64_t dom, int32_t* err_flag, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_validate, dim3(grid), dim3(256), 0, s, col, n, dom, err_flag);
}

// distinct values of an integer column with values in [0, dom): one bit per
// value, then a population count of the bitmap.  Values were validated
// against the domain at prepare time.
__global__ void k_mark_values(const int32_t* __restrict__ col, int64_t n, uint32_t* __restrict__ bits) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = (uint32_t)col[i], m = 1u << (v & 31);
    // most values repeat: test the bit before paying for the atomic (a
    // stale read only costs a redundant atomic)
    if (!(bits[v >> 5] & m)) atomicOr(bits + (v >> 5), m);
  }
}
__global__ void k_popcount(const uint32_t* __restrict__ bits, int64_t words, unsigned long long* __restrict__ out) {
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    c += __popc(bits[i]);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}
void launch_distinct(const int32_t* col, int64_t n, int64_t dom, uint32_t* bits, unsigned long long* out,
                     hipStream_t s) {
  const int64_t words = (dom + 31) / 32;
  (void)hipMemsetAsync(bits, 0, (size_t)std::max<int64_t>(words, 1) * 4, s);
  (void)hipMemsetAsync(out, 0, 8, s);
  if (n > 0) {
    int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_mark_values, dim3(grid), dim3(256), 0, s, col, n, bits);
  }
  int grid = (int)std::min<int64_t>((words + 255) / 256, 2048);
  hipLaunchKernelGGL(k_popcount, dim3(std::max(grid, 1)), dim3(256), 0, s, bits, words, out);
}

void launch_make_keys(const DKeyCols* d, uint64_t* keys, uint32_t* idx, int64_t n, hipStream_t s) {
  int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_make_keys, dim3(grid), dim3(256), 0, s, d, keys, idx, n);
}

template <typename E>
__global__ void k_gather(const E* __restrict__ src, const uint32_t* __restrict__ perm, E* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[perm[i]];
}
template <typename D>
__global__ void k_gather_to(const void* __restrict__ src, int src_dtype, const uint32_t* __restrict__ perm, D* dst,
                            int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t j = perm[i];
    D x;
    if (src_dtype == LMFAO_F32) x = (D)((const float*)src)[j];
    else if (src_dtype == LMFAO_F64) x = (D)((const double*)src)[j];
    else x = (D)((const int32_t*)src)[j];
    dst[i] = x;
  }
}
void launch_gather_convert(const void* src, int src_dtype, const uint32_t* perm, void* dst, int64_t n, bool to_f64,
                           hipStream_t s) {
  int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  if (to_f64) hipLaunchKernelGGL(k_gather_to<double>, dim3(grid), dim3(256), 0, s, src, src_dtype, perm, (double*)dst, n);
  else hipLaunchKernelGGL(k_gather_to<float>, dim3(grid), dim3(256), 0, s, src, src_dtype, perm, (float*)dst, n);
}

void launch_gather(const void* src, const uint32_t* perm, void* dst, int64_t n, int elem_bytes, hipStream_t s) {
  int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_gather<uint64_t>, dim3(grid), dim3(256), 0, s, (const uint64_t*)src, perm, (uint64_t*)dst, n);
  else
    hipLaunchKernelGGL(k_gather<uint32_t>, dim3(grid), dim3(256), 0, s, (const uint32_t*)src, perm, (uint32_t*)dst, n);
}

// segment starts at a trie level: positions where key / div changes
__global__ void k_segment_starts(const uint64_t* __restrict__ keys, int64_t n, uint64_t div,
                                 unsigned long long* count, int64_t* pos, uint64_t* pkey, int64_t cap) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t pk = keys[i] / div;
    if (i == 0 || keys[i - 1] / div != pk) {
      unsigned long long slot = atomicAdd(count, 1ull);
      if ((int64_t)slot < cap) { pos[slot] = i; pkey[slot] = pk; }
    }
  }
}
void launch_segment_starts(const uint64_t* keys, int64_t n, uint64_t div, unsigned long long* count,
                           int64_t* pos, uint64_t* pkey, int64_t cap, hipStream_t s) {
  int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_segment_starts, dim3(grid), dim3(256), 0, s, keys, n, div, count, pos, pkey, cap);
}

// ---------------------------------------------------------------------------
// node scan
// ---------------------------------------------------------------------------
// kScanWaves (wavefronts per scan block) is shared with the planner

__device__ __forceinline__ int tri_index(int i, int j, int n) {
  // extended atoms 0..n (0 = constant 1), i <= j; row-major upper triangle
  return i * (n + 1) - i * (i - 1) / 2 + (j - i);
}

// select one of four per-lane values by a wave-uniform index (no private array)
template <typename X>
__device__ __forceinline__ X sel4(int i, X a, X b, X c, X d) {
  return i == 0 ? a : (i == 1 ? b : (i == 2 ? c : d));
}

// One wavefront per work item (a run of pieces).  Lanes take consecutive rows
// of a piece, so equal group-by codes of the sorted relation sit in runs of
// neighbouring lanes; each run is summed with a segmented lane scan and only
// its last lane issues the LDS atomics of the histograms and direct tables.
// Per-lane values that histograms / tables address by a runtime index (codes,
// run totals) go through a per-wave LDS slot area, never a private array.
template <typename T, int NA>
__global__ __launch_bounds__(kScanWaves * 64) void k_scan(const DScan* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  constexpr int NT = (NA + 1) * (NA + 2) / 2;
  int32_t* tab_i = (int32_t*)smem;
  unsigned char* wbase = (unsigned char*)smem + (((size_t)S->lds_tab_i * 4 + 15) & ~(size_t)15);
  const int hist_i_bytes = (S->hist_i_bins * 4 + 7) & ~7;
  const int hist_bytes = hist_i_bytes + S->hist_f_bins * (int)sizeof(T);
  const int slot_bytes = (S->n_codes * 4 + (S->n_weights <= kMaxWeights ? S->n_weights * 8 : 0)) * 64;
  const int wave_stride = (((hist_bytes + 15) & ~15) + slot_bytes + 15) & ~15;
  unsigned char* wmem = wbase + wid * wave_stride;
  int32_t* hist_i = (int32_t*)wmem;
  T* hist_f = (T*)(wmem + hist_i_bytes);
  int32_t* slot_c = (int32_t*)(wmem + ((hist_bytes + 15) & ~15));   // [n_codes][64]
  double* slot_w = (double*)(slot_c + S->n_codes * 64);             // [n_weights][64] (int or T, as double bits)

  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x) tab_i[i] = 0;
  __syncthreads();

  const int n_views = S->n_views;
  const int n_masks = S->n_masks;
  const int n_codes = S->n_codes;
  const int n_w = S->n_weights;
  const bool runs = (S->n_hists + S->n_tables) > 0;
  const bool direct = n_w > kMaxWeights;   // too many weights to pre-aggregate in registers
  const uint64_t need = S->pf_need;
  const int pf_mask = S->pf_mask_idx;
  const uint32_t m0b = n_masks > 0 ? S->masks[0] : 0, m1b = n_masks > 1 ? S->masks[1] : 0;
  const uint32_t m2b = n_masks > 2 ? S->masks[2] : 0, m3b = n_masks > 3 ? S->masks[3] : 0;

  for (int item = blockIdx.x * kScanWaves + wid; item < S->n_items; item += gridDim.x * kScanWaves) {
    const int p0 = S->item_piece[item], p1 = S->item_piece[item + 1];
    for (int p = p0; p < p1; ++p) {
      const int64_t rb = S->piece_begin[p], re = S->piece_begin[p + 1];
      int64_t mu_out = 1;   // outer multiplicity of the direct tables
      for (int v = 0; v < S->mu_out_views; ++v) {
        const DView& V = S->outer_views[v];
        int64_t vr = 0;
        for (int k = 0; k < V.nkey; ++k)
          vr += (int64_t)S->piece_key[(int64_t)V.key_src[k] * S->n_pieces + p] * V.key_stride[k];
        mu_out *= V.cnt[vr];
      }
      for (int i = lane; i < S->hist_i_bins; i += 64) hist_i[i] = 0;
      for (int i = lane; i < S->hist_f_bins; i += 64) hist_f[i] = (T)0;
      __builtin_amdgcn_wave_barrier();
      T acc[NT];
      T cmp[NT];   // Neumaier compensation (FP64 plans only; folded away for float)
#pragma unroll
      for (int t = 0; t < NT; ++t) { acc[t] = (T)0; cmp[t] = (T)0; }
      int64_t cacc[kMaxMasks];
#pragma unroll
      for (int m = 0; m < kMaxMasks; ++m) cacc[m] = 0;

      for (int64_t r0 = rb; r0 < re; r0 += 64) {
        const int64_t r = r0 + lane;
        const bool valid = r < re;
        const int64_t rr = valid ? r : rb;   // in-bounds row for invalid lanes
        // multiplicity per mask; a row failing the filter has multiplicity 0
        const int64_t w0 = valid ? (S->w ? (int64_t)S->w[rr] : 1) : 0;
        int64_t mu0 = w0, mu1 = w0, mu2 = w0, mu3 = w0;
        T av[NA + 1];
        av[0] = (T)1;
        int32_t cv[kMaxCodes];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          av[a + 1] = (T)0;
          if (S->atoms[a].kind == SRC_COL) av[a + 1] = ld_val<T>(S->cols[S->atoms[a].src], rr);
        }
#pragma unroll
        for (int c = 0; c < kMaxCodes; ++c) {
          cv[c] = 0;
          if (c < n_codes && S->codes[c].kind == SRC_COL) cv[c] = (int32_t)ld_int(S->cols[S->codes[c].src], rr);
        }
        // inner views: looked up once per tuple, consumed in place
#pragma unroll
        for (int v = 0; v < kMaxInnerViews; ++v) {
          if (v < n_views) {
            const DView& V = S->views[v];
            int64_t vr = 0;
            for (int k = 0; k < V.nkey; ++k) vr += ld_int(S->cols[V.key_src[k]], rr) * V.key_stride[k];
            const int64_t vc = valid ? V.cnt[vr] : 0;
            const uint32_t bit = 1u << v;
            if (m0b & bit) mu0 *= vc;
            if (m1b & bit) mu1 *= vc;
            if (m2b & bit) mu2 *= vc;
            if (m3b & bit) mu3 *= vc;
#pragma unroll
            for (int a = 0; a < NA; ++a)
              if (S->atoms[a].kind == SRC_VIEW && S->atoms[a].src == v)
                av[a + 1] = view_val<T>(V, vr, S->atoms[a].slot);
#pragma unroll
            for (int c = 0; c < kMaxCodes; ++c)
              if (c < n_codes && S->codes[c].kind == SRC_VIEW && S->codes[c].src == v)
                cv[c] = V.codes[vr * V.n_codes + S->codes[c].slot];
          }
        }
        // float partial sums over the extended-atom triangle
        if (S->pf_uniform) {
          const T muT = (T)sel4(pf_mask, mu0, mu1, mu2, mu3);
#pragma unroll
          for (int i = 0; i <= NA; ++i) {
            const T xi = muT * av[i];
#pragma unroll
            for (int j = i; j <= NA; ++j) {
              const int t = tri_index(i, j, NA);
              if (t > 0 && ((need >> t) & 1ull)) kadd(acc[t], cmp[t], xi * av[j]);
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i <= NA; ++i) {
#pragma unroll
            for (int j = i; j <= NA; ++j) {
              const int t = tri_index(i, j, NA);
              if (t > 0 && ((need >> t) & 1ull))
                kadd(acc[t], cmp[t], (T)sel4((int)S->pf_mask[t], mu0, mu1, mu2, mu3) * av[i] * av[j]);
            }
          }
        }
#pragma unroll
        for (int m = 0; m < kMaxMasks; ++m)
          if (m < S->n_pi) cacc[m] += sel4(S->pi_mask_idx[m], mu0, mu1, mu2, mu3);
        if (!runs) continue;
        // codes to the lane slots
#pragma unroll
        for (int c = 0; c < kMaxCodes; ++c)
          if (c < n_codes) slot_c[c * 64 + lane] = cv[c];
        if (direct) {
          // each tuple updates the histograms / tables itself
          if (valid) {
            for (int h = 0; h < S->n_hists; ++h) {
              const DHist& H = S->hists[h];
              const DWeight& W = S->weights[H.wi];
              const int32_t code = slot_c[H.code * 64 + lane];
              int64_t m = sel4(W.mask_idx, mu0, mu1, mu2, mu3);
              if (!m) continue;
              if (!H.is_float) {
                atomicAdd(&hist_i[H.offset + code], (int32_t)m);
              } else {
                T x = (T)m;
#pragma unroll
                for (int a = 1; a <= NA; ++a) {
                  if (a == W.ai + 1) x *= av[a];
                  if (a == W.aj + 1) x *= av[a];
                }
                atomicAdd(&hist_f[H.offset + code], x);
              }
            }
            for (int tb = 0; tb < S->n_tables; ++tb) {
              const DTable& TB = S->tables[tb];
              int64_t row = 0;
              for (int k = 0; k < TB.ncode; ++k) row += (int64_t)slot_c[TB.code[k] * 64 + lane] * TB.stride[k];
              for (int q = 0; q < TB.n_tcomps; ++q) {
                const DWeight& W = S->weights[TB.twi[q]];
                int64_t m = mu_out * sel4(W.mask_idx, mu0, mu1, mu2, mu3);
                if (!m) continue;
                if (TB.tcomp[q] < 0) {
                  if (TB.lds) atomicAdd(&tab_i[TB.lds_off + row], (int32_t)m);
                  else atomic_add_i64(&TB.cnt[row], m);
                } else {
                  T x = (T)m;
#pragma unroll
                  for (int a = 1; a <= NA; ++a) {
                    if (a == W.ai + 1) x *= av[a];
                    if (a == W.aj + 1) x *= av[a];
                  }
                  int64_t di = row * TB.n_vals + TB.tcomp[q];
                  if (TB.vals_f64) atomic_add_f64(&((double*)TB.vals)[di], (double)x);
                  else atomicAdd(&((float*)TB.vals)[di], (float)x);
                }
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
          continue;
        }
        // runs of equal keyed codes across neighbouring lanes
        bool head = (lane == 0) || !valid;
#pragma unroll
        for (int c = 0; c < kMaxCodes; ++c)
          if (c < n_codes && ((S->run_codes >> c) & 1u)) {
            int32_t up = __shfl_up(cv[c], 1, 64);
            head |= (lane > 0) && up != cv[c];
          }
        int start = head ? lane : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          int s2 = __shfl_up(start, d, 64);
          if (lane >= d) start = max(start, s2);
        }
        const bool next_head = __shfl_down((int)head, 1, 64) != 0;
        const bool tail = valid && (lane == 63 || next_head);
        // per-run totals of every weight (segmented inclusive scan) to the lane slots
#pragma unroll
        for (int w = 0; w < kMaxWeights; ++w) {
          if (w < n_w) {
            const DWeight& W = S->weights[w];
            const int64_t m = sel4(W.mask_idx, mu0, mu1, mu2, mu3);
            if (!W.is_float) {
              int32_t x = (int32_t)m;
#pragma unroll
              for (int d = 1; d < 64; d <<= 1) {
                int32_t x2 = __shfl_up(x, d, 64);
                if (lane - d >= start) x += x2;
              }
              ((int32_t*)slot_w)[(w * 64 + lane) * 2] = x;
            } else {
              T x = (T)m;
#pragma unroll
              for (int a = 1; a <= NA; ++a) {
                if (a == W.ai + 1) x *= av[a];
                if (a == W.aj + 1) x *= av[a];
              }
#pragma unroll
              for (int d = 1; d < 64; d <<= 1) {
                T x2 = __shfl_up(x, d, 64);
                if (lane - d >= start) x += x2;
              }
              slot_w[w * 64 + lane] = (double)x;
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (tail) {
          for (int h = 0; h < S->n_hists; ++h) {
            const DHist& H = S->hists[h];
            const int32_t code = slot_c[H.code * 64 + lane];
            if (!H.is_float) {
              int32_t x = ((const int32_t*)slot_w)[(H.wi * 64 + lane) * 2];
              if (x) atomicAdd(&hist_i[H.offset + code], x);
            } else {
              T x = (T)slot_w[H.wi * 64 + lane];
              if (x != (T)0) atomicAdd(&hist_f[H.offset + code], x);
            }
          }
          for (int tb = 0; tb < S->n_tables; ++tb) {
            const DTable& TB = S->tables[tb];
            int64_t row = 0;
            for (int k = 0; k < TB.ncode; ++k) row += (int64_t)slot_c[TB.code[k] * 64 + lane] * TB.stride[k];
            for (int q = 0; q < TB.n_tcomps; ++q) {
              const int w = TB.twi[q];
              if (TB.tcomp[q] < 0) {
                int64_t x = mu_out * (int64_t)((const int32_t*)slot_w)[(w * 64 + lane) * 2];
                if (!x) continue;
                if (TB.lds) atomicAdd(&tab_i[TB.lds_off + row], (int32_t)x);
                else atomic_add_i64(&TB.cnt[row], x);
              } else {
                T x = (T)mu_out * (T)slot_w[w * 64 + lane];
                if (x == (T)0) continue;
                int64_t di = row * TB.n_vals + TB.tcomp[q];
                if (TB.vals_f64) atomic_add_f64(&((double*)TB.vals)[di], (double)x);
                else atomicAdd(&((float*)TB.vals)[di], (float)x);
              }
            }
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      // close the piece: reduce the lanes' partial sums and store the psi row
      T* prow = (T*)S->psi_f + (int64_t)p * S->psi_f_stride;
      int32_t* irow = S->psi_i + (int64_t)p * S->psi_i_stride;
#pragma unroll
      for (int t = 1; t < NT; ++t) {
        if ((need >> t) & 1ull) {
          T sm = wave_sum_comp(acc[t], cmp[t]);
          if (lane == 0) prow[S->pf_slot[t]] = sm;
        }
      }
#pragma unroll
      for (int m = 0; m < kMaxMasks; ++m)
        if (m < S->n_pi) {
          int64_t sm = wave_sum_i64(cacc[m]);
          if (lane == 0) irow[m] = (int32_t)sm;
        }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int i = lane; i < S->hist_i_bins; i += 64) irow[S->n_pi + i] = hist_i[i];
      for (int i = lane; i < S->hist_f_bins; i += 64) prow[S->pf_n + i] = hist_f[i];
      __builtin_amdgcn_wave_barrier();
    }
  }
  // flush LDS-privatized count tables as block partials
  __syncthreads();
  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x)
    S->part_i[(int64_t)blockIdx.x * S->lds_tab_i + i] = tab_i[i];
}


// ---------------------------------------------------------------------------
// lean scan: inner views read through per-key images
// ---------------------------------------------------------------------------
template <typename T>
struct ImgLayout {
  static constexpr int s = sizeof(T) / 4;   // dwords per factor slot
};
template <typename T, int NA>
struct ImgShape {
  static constexpr int code_off = NA * ImgLayout<T>::s;
  static constexpr int cnt_off = code_off + 4;
  static constexpr int width = ((cnt_off + 1) + 3) & ~3;
};

// image record: factor slots, code slots (4, or one per code past 4), count
int image_code_slots(int n_codes) { return n_codes > 4 ? n_codes : 4; }
int image_width_dw(int na, bool f64, int n_codes) {
  int code_off = na * (f64 ? 2 : 1);
  return ((code_off + image_code_slots(n_codes) + 1) + 3) & ~3;
}
int image_code_off(int na, bool f64) { return na * (f64 ? 2 : 1); }

// One dword of key k's image record: a factor (or half of an FP64 one), a
// code, or the multiplicity; zero elsewhere and for keys without tuples
template <typename T>
__device__ __forceinline__ uint32_t image_dword(const DImageBuild* __restrict__ B, const DView& V, int64_t k,
                                                int64_t cnt, int col) {
  constexpr int s = sizeof(T) / 4;
  if (col == B->cnt_off) return (uint32_t)cnt;
  if (cnt == 0) return 0u;
  if (col < B->code_off) {
    const int a = col / s;
    const int slot = a < B->n_atoms ? B->atom_slot[a] : -1;
    if (slot < 0) return 0u;
    const T x = view_val<T>(V, k, slot);
    if (s == 1) return __float_as_uint((float)x);
    const uint64_t u = (uint64_t)__double_as_longlong((double)x);
    return (col & 1) ? (uint32_t)(u >> 32) : (uint32_t)u;
  }
  if (col - B->code_off < B->n_codes) {
    const int slot = B->code_slot[col - B->code_off];
    if (slot >= 0) return (uint32_t)V.codes[k * V.n_codes + slot];
  }
  return 0u;
}

// Each workgroup fills the images of 64 consecutive keys, a contiguous run of
// 64 * width dwords, four dwords per lane per store (widths are multiples of
// 4 and the image buffer is allocated on its own, so every store is aligned).
template <typename T>
__global__ __launch_bounds__(256) void k_build_image(const DImageBuild* __restrict__ B) {
  const DView& V = B->view;
  const int W4 = B->width_dw >> 2;
  const int64_t n_tiles = (B->n_keys + 63) / 64;
  uint4* img = (uint4*)B->img;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t k0 = t * 64;
    const int m = (int)(B->n_keys - k0 < 64 ? B->n_keys - k0 : 64);
    for (int j = threadIdx.x; j < m * W4; j += 256) {
      const int i = j / W4, c0 = (j - i * W4) * 4;
      const int64_t k = k0 + i;
      const int64_t cnt = V.cnt[k];
      img[k0 * W4 + j] = make_uint4(image_dword<T>(B, V, k, cnt, c0), image_dword<T>(B, V, k, cnt, c0 + 1),
                                    image_dword<T>(B, V, k, cnt, c0 + 2), image_dword<T>(B, V, k, cnt, c0 + 3));
    }
  }
}
void launch_build_image(const DImageBuild* d, int64_t n_keys, bool f64, hipStream_t s) {
  if (n_keys <= 0) return;
  int grid = (int)std::min<int64_t>((n_keys + 63) / 64, 8192);
  if (f64) hipLaunchKernelGGL(k_build_image<double>, dim3(grid), dim3(256), 0, s, d);
  else hipLaunchKernelGGL(k_build_image<float>, dim3(grid), dim3(256), 0, s, d);
}

// loads through global (address space 1) pointers: the descriptor holds
// generic pointers, which would otherwise become flat loads
template <typename T>
__device__ __forceinline__ T gld(const T* p, int64_t i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 gld4(const uint4* p, int64_t i) {
  return ((const __attribute__((address_space(1))) u32x4*)p)[i];
}

template <typename T>
__device__ __forceinline__ T img_val(const uint32_t* dw, int a) {
  if constexpr (sizeof(T) == 4) return __uint_as_float(dw[a]);
  else return __longlong_as_double((long long)(((uint64_t)dw[2 * a + 1] << 32) | dw[2 * a]));
}

// Per-row inputs of the lean scan that come from the sorted relation itself:
// factor columns (absent: 0, the factor comes from an image), code columns
// (absent: 0) and the dense key of each inner view image.
template <typename T, int NA>
struct RowCols {
  T f[NA > 0 ? NA : 1];
  int c[4];
  int k[2];
  int w;   // filter weight
};
template <typename T, int NA>
__device__ __forceinline__ void load_row_cols(const DScan* __restrict__ S, int rr, RowCols<T, NA>& o) {
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const T* fc = (const T*)S->F.fcol[a];
    o.f[a] = fc ? gld(fc, rr) : (T)0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) o.c[c] = S->F.ccol[c] ? gld(S->F.ccol[c], rr) : 0;
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    int key = 0;
    if (S->F.img[v]) {
      key = gld(S->F.kcol[v][0], rr) * S->F.kmul[v][0];
      if (S->F.kcol[v][1]) key += gld(S->F.kcol[v][1], rr) * S->F.kmul[v][1];
    }
    o.k[v] = key;
  }
  o.w = S->w ? gld(S->w, rr) : 1;
}

// Per tuple: column loads, one vector load per inner view image, factor
// products into per-lane partial sums, direct LDS atomics for histograms and
// direct tables.  Everything the row loop needs is hoisted into registers
// before it; private arrays are indexed at compile time only.
template <typename T, int NA>
__global__ __launch_bounds__(kScanWaves * 64) void k_scan_fast(const DScan* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  using Shape = ImgShape<T, NA>;
  constexpr int W = Shape::width;
  constexpr int NT = (NA + 1) * (NA + 2) / 2;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  int32_t* tab_i = (int32_t*)smem;
  unsigned char* wbase = (unsigned char*)smem + (((size_t)S->lds_tab_i * 4 + 15) & ~(size_t)15);
  const int hist_i_bytes = (S->hist_i_bins * 4 + 7) & ~7;
  const int hist_bytes = hist_i_bytes + S->hist_f_bins * (int)sizeof(T);
  const int wave_stride = ((hist_bytes + 15) & ~15) + (NA + 1 + 4) * 64 * (int)sizeof(T);
  int32_t* hist_i = (int32_t*)(wbase + wid * wave_stride);
  T* hist_f = (T*)((unsigned char*)hist_i + hist_i_bytes);
  // per-lane slots: factors 0..NA (0 = 1) then codes, read back by histogram index
  T* slot_a = (T*)(wbase + wid * wave_stride + ((hist_bytes + 15) & ~15));
  int32_t* slot_c = (int32_t*)(slot_a + (NA + 1) * 64);

  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x) tab_i[i] = 0;
  __syncthreads();

  const int n_hist = S->F.n_hist;
  const int n_tab = S->F.n_tab;
  const uint64_t need = S->pf_need;
  const int pf_mask = S->pf_mask_idx;
  const int n_masks = S->n_masks;
  const uint32_t m0b = n_masks > 0 ? S->masks[0] : 0, m1b = n_masks > 1 ? S->masks[1] : 0;
  const uint32_t m2b = n_masks > 2 ? S->masks[2] : 0, m3b = n_masks > 3 ? S->masks[3] : 0;
  const int n_pi = S->n_pi;
  const int pim0 = S->pi_mask_idx[0], pim1 = S->pi_mask_idx[1], pim2 = S->pi_mask_idx[2], pim3 = S->pi_mask_idx[3];
  const int32_t* pb = (const int32_t*)nullptr;
  (void)pb;

  for (int item = blockIdx.x * kScanWaves + wid; item < S->n_items; item += gridDim.x * kScanWaves) {
    const int p0 = S->item_piece[item], p1 = S->item_piece[item + 1];
    for (int p = p0; p < p1; ++p) {
      const int rb = (int)S->piece_begin[p], re = (int)S->piece_begin[p + 1];
      int mu_out = 1;
      for (int v = 0; v < S->mu_out_views; ++v) {
        const DView& V = S->outer_views[v];
        int64_t vr = 0;
        for (int k = 0; k < V.nkey; ++k)
          vr += (int64_t)S->piece_key[(int64_t)V.key_src[k] * S->n_pieces + p] * V.key_stride[k];
        mu_out *= (int)V.cnt[vr];
      }
      for (int i = lane; i < S->hist_i_bins; i += 64) hist_i[i] = 0;
      for (int i = lane; i < S->hist_f_bins; i += 64) hist_f[i] = (T)0;
      __builtin_amdgcn_wave_barrier();
      // per-lane sums: FP64 pieces hold at most 64 rows (one term per lane),
      // FP32 pieces are reduced in FP64 afterwards, so no compensation here
      T acc[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = (T)0;
      int cacc0 = 0, cacc1 = 0, cacc2 = 0, cacc3 = 0;

      // the next 64-row chunk's columns are loaded while the current one is
      // combined with its view images (one chunk of prefetch per wavefront)
      RowCols<T, NA> nx;
      load_row_cols<T, NA>(S, rb + lane < re ? rb + lane : rb, nx);
      for (int r0 = rb; r0 < re; r0 += 64) {
        const int r = r0 + lane;
        const bool valid = r < re;
        const RowCols<T, NA> cu = nx;
        if (r0 + 64 < re) load_row_cols<T, NA>(S, r + 64 < re ? r + 64 : rb, nx);
        T av[NA + 1];
        av[0] = (T)1;
#pragma unroll
        for (int a = 0; a < NA; ++a) av[a + 1] = cu.f[a];
        int c0 = cu.c[0], c1 = cu.c[1], c2 = cu.c[2], c3 = cu.c[3];
        const int wv = valid ? cu.w : 0;
        int mu0 = wv, mu1 = wv, mu2 = wv, mu3 = wv;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const uint4* img = (const uint4*)S->F.img[v];
          if (img) {
            const uint4* q = img + (int64_t)cu.k[v] * (W / 4);
            uint32_t dw[W];
#pragma unroll
            for (int j = 0; j < W / 4; ++j) {
              const u32x4 x = gld4(q, j);
              dw[4 * j] = x[0];
              dw[4 * j + 1] = x[1];
              dw[4 * j + 2] = x[2];
              dw[4 * j + 3] = x[3];
            }
#pragma unroll
            for (int a = 0; a < NA; ++a) av[a + 1] += img_val<T>(dw, a);
            c0 += (int)dw[Shape::code_off];
            c1 += (int)dw[Shape::code_off + 1];
            c2 += (int)dw[Shape::code_off + 2];
            c3 += (int)dw[Shape::code_off + 3];
            const int vc = valid ? (int)dw[Shape::cnt_off] : 0;
            const uint32_t bit = 1u << v;
            if (m0b & bit) mu0 *= vc;
            if (m1b & bit) mu1 *= vc;
            if (m2b & bit) mu2 *= vc;
            if (m3b & bit) mu3 *= vc;
          }
        }
        {
          // every monomial of degree <= 2 of the row's factors, without a
          // branch per monomial: the needed ones are written when the piece
          // closes (one multiplicity mask for all of them)
          const T muT = (T)sel4(pf_mask, mu0, mu1, mu2, mu3);
#pragma unroll
          for (int i = 0; i <= NA; ++i) {
            const T xi = muT * av[i];
#pragma unroll
            for (int j = i; j <= NA; ++j) {
              const int t = tri_index(i, j, NA);
              if (t > 0) acc[t] += xi * av[j];
            }
          }
        }
        if (n_pi > 0) cacc0 += sel4(pim0, mu0, mu1, mu2, mu3);
        if (n_pi > 1) cacc1 += sel4(pim1, mu0, mu1, mu2, mu3);
        if (n_pi > 2) cacc2 += sel4(pim2, mu0, mu1, mu2, mu3);
        if (n_pi > 3) cacc3 += sel4(pim3, mu0, mu1, mu2, mu3);
        if (n_hist > 0) {
#pragma unroll
          for (int a = 0; a <= NA; ++a) slot_a[a * 64 + lane] = av[a];
          slot_c[lane] = c0;
          slot_c[64 + lane] = c1;
          slot_c[128 + lane] = c2;
          slot_c[192 + lane] = c3;
          __builtin_amdgcn_wave_barrier();
          for (int h = 0; h < n_hist; ++h) {
            const uint32_t w = S->F.hword[h];
            const int code = slot_c[(int)(w & 3u) * 64 + lane];
            const int m = sel4((int)((w >> 2) & 3u), mu0, mu1, mu2, mu3);
            const int off = (int)(w >> 13);
            if (!m) continue;
            if ((w >> 4) & 1u) {
              const int ai = (int)((w >> 5) & 15u), aj = (int)((w >> 9) & 15u);
              const T x = (T)m * slot_a[ai * 64 + lane] * slot_a[aj * 64 + lane];
              atomicAdd(&hist_f[off + code], x);
            } else {
              atomicAdd(&hist_i[off + code], m);
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int tb = 0; tb < kFastTables; ++tb) {
          if (tb < n_tab) {
            int row = 0;
            for (int k = 0; k < S->F.tab_ncode[tb]; ++k)
              row += sel4(S->F.tab_code[tb][k], c0, c1, c2, c3) * S->F.tab_stride[tb][k];
            const int m = mu_out * sel4(S->F.tab_mask[tb], mu0, mu1, mu2, mu3);
            if (m) {
              if (S->F.tab_lds[tb]) atomicAdd(&tab_i[S->F.tab_off[tb] + row], m);
              else atomic_add_i64(&S->F.tab_cnt[tb][row], (int64_t)m);
            }
          }
        }
      }
      // close the piece
      T* prow = (T*)S->psi_f + (int64_t)p * S->psi_f_stride;
      int32_t* irow = S->psi_i + (int64_t)p * S->psi_i_stride;
#pragma unroll
      for (int t = 1; t < NT; ++t) {
        if ((need >> t) & 1ull) {
          T sm = wave_sum_comp(acc[t], (T)0);
          if (lane == 0) prow[S->pf_slot[t]] = sm;
        }
      }
      if (n_pi > 0) { int sm = wave_sum((int)cacc0); if (lane == 0) irow[0] = sm; }
      if (n_pi > 1) { int sm = wave_sum((int)cacc1); if (lane == 0) irow[1] = sm; }
      if (n_pi > 2) { int sm = wave_sum((int)cacc2); if (lane == 0) irow[2] = sm; }
      if (n_pi > 3) { int sm = wave_sum((int)cacc3); if (lane == 0) irow[3] = sm; }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int i = lane; i < S->hist_i_bins; i += 64) irow[n_pi + i] = hist_i[i];
      for (int i = lane; i < S->hist_f_bins; i += 64) prow[S->pf_n + i] = hist_f[i];
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x)
    S->part_i[(int64_t)blockIdx.x * S->lds_tab_i + i] = tab_i[i];
}

int scan_fast_lds_bytes(const DScan& S, bool f64) {
  int hist_bytes = ((S.hist_i_bins * 4 + 7) & ~7) + S.hist_f_bins * (f64 ? 8 : 4);
  int wave_stride = ((hist_bytes + 15) & ~15) + (S.n_atoms + 1 + 4) * 64 * (f64 ? 8 : 4);
  return (int)(((S.lds_tab_i * 4 + 15) & ~15) + kScanWaves * wave_stride);
}

int scan_lds_bytes(const DScan& S, bool f64) {
  int hist_bytes = ((S.hist_i_bins * 4 + 7) & ~7) + S.hist_f_bins * (f64 ? 8 : 4);
  int slot_bytes = (S.n_codes * 4 + (S.n_weights <= kMaxWeights ? S.n_weights * 8 : 0)) * 64;
  int wave_stride = (((hist_bytes + 15) & ~15) + slot_bytes + 15) & ~15;
  return (int)(((S.lds_tab_i * 4 + 15) & ~15) + kScanWaves * wave_stride);
}


template <typename T>
static void launch_scan_fast_t(const DScan* d, int na, int grid, int lds, hipStream_t s) {
  dim3 b(kScanWaves * 64);
  switch (na) {
#define CASE(N)                                                         \
  case N:                                                               \
    allow_lds((const void*)&k_scan_fast<T, N>, lds);                    \
    hipLaunchKernelGGL((k_scan_fast<T, N>), dim3(grid), b, lds, s, d);  \
    break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}
void launch_scan_fast(const DScan* d, int na, bool f64, int grid, int lds, hipStream_t s) {
  if (f64) launch_scan_fast_t<double>(d, na, grid, lds, s);
  else launch_scan_fast_t<float>(d, na, grid, lds, s);
}

template <typename T>
static void launch_scan_t(const DScan* d, int na, int grid, int lds, hipStream_t s) {
  dim3 b(kScanWaves * 64);
  switch (na) {
#define CASE(N)                                                         \
  case N:                                                               \
    allow_lds((const void*)&k_scan<T, N>, lds);                         \
    hipLaunchKernelGGL((k_scan<T, N>), dim3(grid), b, lds, s, d);       \
    break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}
void launch_scan(const DScan* d, int na, bool f64, int grid, int lds, hipStream_t s) {
  if (f64) launch_scan_t<double>(d, na, grid, lds, s);
  else launch_scan_t<float>(d, na, grid, lds, s);
}
int scan_waves_per_block() { return kScanWaves; }

// ---------------------------------------------------------------------------
// contraction over pieces
// ---------------------------------------------------------------------------
constexpr int kCThreads = 256;
constexpr int kCPieces = 16;   // pieces staged in LDS at a time
constexpr int kTile = 4;       // register tile (features x columns) per thread

template <typename T>
__device__ __forceinline__ T feat_value(const DContract* C, const DFeat& F, const int64_t* mu,
                                        const int32_t* codes, const T* atoms) {
  int64_t m = mu[F.mask_idx];
  if (F.c1 >= 0 && codes[F.c1] != F.v1) m = 0;
  if (F.c2 >= 0 && codes[F.c2] != F.v2) m = 0;
  T x = (T)m;
  if (F.a1 >= 0) x *= atoms[F.a1];
  if (F.a2 >= 0) x *= atoms[F.a2];
  return x;
}
__device__ __forceinline__ int64_t feat_int(const DFeat& F, const int64_t* mu, const int32_t* codes) {
  int64_t m = mu[F.mask_idx];
  if (F.c1 >= 0 && codes[F.c1] != F.v1) m = 0;
  if (F.c2 >= 0 && codes[F.c2] != F.v2) m = 0;
  return m;
}

template <typename T>
__global__ __launch_bounds__(kCThreads) void k_contract(const DContract* __restrict__ C) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int NF = C->n_feat, NG = C->n_col, NFI = C->n_feat_int, NGI = C->n_col_int;
  const int NA = C->n_atoms, NC = C->n_codes, NM = C->n_masks;
  // LDS layout per staged piece chunk
  T* A = (T*)smem;                                      // [kCPieces][NF]
  T* Bm = A + kCPieces * NF;                            // [kCPieces][NG]
  int64_t* Ai = (int64_t*)(Bm + kCPieces * NG);         // [kCPieces][NFI]
  int64_t* Bi = Ai + kCPieces * NFI;                    // [kCPieces][NGI]
  T* atom_s = (T*)(Bi + kCPieces * NGI);                // [kCPieces][NA]
  int32_t* code_s = (int32_t*)(atom_s + kCPieces * NA); // [kCPieces][NC]
  int64_t* mu_s = (int64_t*)(((uintptr_t)(code_s + kCPieces * NC) + 7) & ~(uintptr_t)7);  // [kCPieces][NM]
  int64_t* vrow_s = mu_s + kCPieces * NM;               // [kCPieces][kMaxViews]
  int64_t* vcnt_s = vrow_s + kCPieces * kMaxViews;

  // this block's register tile (float block) and int cells
  const int tiles_g = (NG + kTile - 1) / kTile;
  const int tiles_f = (NF + kTile - 1) / kTile;
  const int tile = blockIdx.y * kCThreads + threadIdx.x;
  const bool has_tile = tile < tiles_f * tiles_g;
  const int f0 = has_tile ? (tile / tiles_g) * kTile : 0;
  const int g0 = has_tile ? (tile % tiles_g) * kTile : 0;
  // products of two FP32 values are exact in FP64, so FP32 inputs lose
  // nothing to the FP64 accumulation; FP64 inputs are also compensated
  double acc[kTile][kTile], cmp[kTile][kTile];
#pragma unroll
  for (int i = 0; i < kTile; ++i)
#pragma unroll
    for (int j = 0; j < kTile; ++j) { acc[i][j] = 0.0; cmp[i][j] = 0.0; }
  // int cells owned by this thread: block row y takes cells [y*8*T, (y+1)*8*T)
  const int icell0 = blockIdx.y * 8 * kCThreads;
  const int n_icells = std::max(0, std::min(8 * kCThreads, NFI * NGI - icell0));
  int64_t iacc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) iacc[q] = 0;

  const int64_t pbeg = (int64_t)blockIdx.x * C->pieces_per_block;
  const int64_t pend = std::min<int64_t>(C->n_pieces, pbeg + C->pieces_per_block);
  for (int64_t cb = pbeg; cb < pend; cb += kCPieces) {
    const int np = (int)std::min<int64_t>(kCPieces, pend - cb);
    // 1. views of each piece
    for (int t = threadIdx.x; t < np * C->n_views; t += kCThreads) {
      int pi = t / C->n_views, v = t % C->n_views;
      int64_t p = cb + pi;
      const DView& V = C->views[v];
      int64_t vr = 0;
      for (int k = 0; k < V.nkey; ++k) vr += ld_int(C->pcols[V.key_src[k]], p) * V.key_stride[k];
      vrow_s[pi * kMaxViews + v] = vr;
      vcnt_s[pi * kMaxViews + v] = V.cnt[vr];
    }
    __syncthreads();
    // 2. masks, atoms, codes
    for (int t = threadIdx.x; t < np * NM; t += kCThreads) {
      int pi = t / NM, m = t % NM;
      uint32_t bits = C->masks[m];
      int64_t x = 1;
      for (int v = 0; v < C->n_views; ++v)
        if (bits & (1u << v)) x *= vcnt_s[pi * kMaxViews + v];
      mu_s[pi * NM + m] = x;
    }
    for (int t = threadIdx.x; t < np * NA; t += kCThreads) {
      int pi = t / NA, a = t % NA;
      int64_t p = cb + pi;
      const DAtom& At = C->atoms[a];
      T x;
      if (At.kind == SRC_COL) x = ld_val<T>(C->pcols[At.src], p);
      else {
        int v = At.src;
        x = vcnt_s[pi * kMaxViews + v] ? view_val<T>(C->views[v], vrow_s[pi * kMaxViews + v], At.slot) : (T)0;
      }
      atom_s[pi * NA + a] = x;
    }
    for (int t = threadIdx.x; t < np * NC; t += kCThreads) {
      int pi = t / NC, c = t % NC;
      int64_t p = cb + pi;
      const DAtom& Cd = C->codes[c];
      int32_t x;
      if (Cd.kind == SRC_COL) x = (int32_t)ld_int(C->pcols[Cd.src], p);
      else {
        int v = Cd.src;
        const DView& V = C->views[v];
        x = vcnt_s[pi * kMaxViews + v] ? V.codes[vrow_s[pi * kMaxViews + v] * V.n_codes + Cd.slot] : -1;
      }
      code_s[pi * NC + c] = x;
    }
    __syncthreads();
    // 3. features and columns
    for (int t = threadIdx.x; t < np * NF; t += kCThreads) {
      int pi = t / NF, f = t % NF;
      A[pi * NF + f] = feat_value<T>(C, C->feats[f], mu_s + pi * NM, code_s + pi * NC, atom_s + pi * NA);
      if (f < NFI) Ai[pi * NFI + f] = feat_int(C->feats[f], mu_s + pi * NM, code_s + pi * NC);
    }
    for (int t = threadIdx.x; t < np * NG; t += kCThreads) {
      int pi = t / NG, g = t % NG;
      int64_t p = cb + pi;
      const DColB& B = C->cols[g];
      T x;
      int64_t xi = 0;
      if (B.kind == B_PSI_F) {
        x = ((const T*)C->psi_f)[p * C->psi_f_stride + B.entry];
      } else if (B.kind == B_PSI_I) {
        xi = C->row_pieces ? (C->w ? C->w[p] : 1) : C->psi_i[p * C->psi_i_stride + B.entry];
        x = (T)xi;
      } else {
        int64_t cnt = C->row_pieces ? (C->w ? C->w[p] : 1) : C->psi_i[p * C->psi_i_stride + B.entry];
        // feature without multiplicity (the A side carries it)
        DFeat F = B.feat;
        int64_t m = cnt;
        if (F.c1 >= 0 && code_s[pi * NC + F.c1] != F.v1) m = 0;
        if (F.c2 >= 0 && code_s[pi * NC + F.c2] != F.v2) m = 0;
        xi = m;
        x = (T)m;
        if (F.a1 >= 0) x *= atom_s[pi * NA + F.a1];
        if (F.a2 >= 0) x *= atom_s[pi * NA + F.a2];
      }
      Bm[pi * NG + g] = x;
      if (g < NGI) Bi[pi * NGI + g] = xi;
    }
    __syncthreads();
    // 4. block product over the staged pieces
    if (has_tile) {
      for (int pi = 0; pi < np; ++pi) {
        T a[kTile], b[kTile];
#pragma unroll
        for (int i = 0; i < kTile; ++i) a[i] = (f0 + i < NF) ? A[pi * NF + f0 + i] : (T)0;
#pragma unroll
        for (int j = 0; j < kTile; ++j) b[j] = (g0 + j < NG) ? Bm[pi * NG + g0 + j] : (T)0;
#pragma unroll
        for (int i = 0; i < kTile; ++i)
#pragma unroll
          for (int j = 0; j < kTile; ++j) {
            double pr = (double)a[i] * (double)b[j];
            if constexpr (sizeof(T) == 8) kadd(acc[i][j], cmp[i][j], pr);
            else acc[i][j] += pr;
          }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int cell = threadIdx.x + q * kCThreads;
      if (cell < n_icells) {
        int f = (icell0 + cell) / NGI, g = (icell0 + cell) % NGI;
        int64_t s = 0;
        for (int pi = 0; pi < np; ++pi) s += Ai[pi * NFI + f] * Bi[pi * NGI + g];
        iacc[q] += s;
      }
    }
    // 5. scatter cells of this chunk (first block row only)
    const int n_sc = blockIdx.y == 0 ? C->n_scatter : 0;
    for (int t = threadIdx.x; t < np * n_sc; t += kCThreads) {
      int pi = t / n_sc, sc = t % n_sc;
      int o = C->sc_out[sc];
      int64_t row = 0;
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        int cidx = C->so_code[o * 3 + k];
        if (cidx < 0) continue;
        int32_t cval = code_s[pi * NC + cidx];
        if (cval < 0) ok = false;
        row += (int64_t)cval * C->so_stride[o * 3 + k];
      }
      if (!ok) continue;
      int f = C->sc_f[sc], g = C->sc_g[sc];
      int comp = C->sc_comp[sc];
      if (comp < 0) {
        int64_t v = feat_int(C->feats[f], mu_s + pi * NM, code_s + pi * NC);
        // column value as integer
        const DColB& B = C->cols[g];
        int64_t cnt = C->row_pieces ? (C->w ? C->w[cb + pi] : 1) : C->psi_i[(cb + pi) * C->psi_i_stride + B.entry];
        if (B.kind == B_CNTF) {
          const DFeat& F = B.feat;
          if (F.c1 >= 0 && code_s[pi * NC + F.c1] != F.v1) cnt = 0;
          if (F.c2 >= 0 && code_s[pi * NC + F.c2] != F.v2) cnt = 0;
        }
        v *= cnt;
        if (v) scatter_count(C, o, row, v);
      } else {
        T v = A[pi * NF + f] * Bm[pi * NG + g];
        if (v != (T)0) scatter_value(C, o, row, comp, (double)v);
      }
    }
    __syncthreads();
  }
  // partials
  // partials are cell-major: the merge reads each cell's block partials contiguously
  const int64_t nb = gridDim.x;
  if (has_tile) {
#pragma unroll
    for (int i = 0; i < kTile; ++i)
#pragma unroll
      for (int j = 0; j < kTile; ++j)
        if (f0 + i < NF && g0 + j < NG)
          C->part_f[((int64_t)(f0 + i) * NG + g0 + j) * nb + blockIdx.x] = acc[i][j] + cmp[i][j];
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int cell = threadIdx.x + q * kCThreads;
    if (cell < n_icells) C->part_i[(int64_t)(icell0 + cell) * nb + blockIdx.x] = iacc[q];
  }
}

int contract_lds_bytes(const DContract& C, bool f64) {
  int t = f64 ? 8 : 4;
  int64_t b = (int64_t)kCPieces * (C.n_feat + C.n_col) * t + (int64_t)kCPieces * (C.n_feat_int + C.n_col_int) * 8 +
              (int64_t)kCPieces * C.n_atoms * t + (int64_t)kCPieces * C.n_codes * 4 + 8 +
              (int64_t)kCPieces * C.n_masks * 8 + (int64_t)kCPieces * kMaxViews * 16;
  return (int)((b + 15) & ~15);
}
int contract_tiles(int nf, int ng) {
  return ((nf + kTile - 1) / kTile) * ((ng + kTile - 1) / kTile);
}
int contract_threads() { return kCThreads; }
int contract_max_int_cells() { return 8 * kCThreads; }

void launch_contract(const DContract* d, bool f64, int grid_x, int grid_y, int lds, hipStream_t s) {
  if (f64) {
    allow_lds((const void*)&k_contract<double>, lds);
    hipLaunchKernelGGL(k_contract<double>, dim3(grid_x, grid_y), dim3(kCThreads), lds, s, d);
  } else {
    allow_lds((const void*)&k_contract<float>, lds);
    hipLaunchKernelGGL(k_contract<float>, dim3(grid_x, grid_y), dim3(kCThreads), lds, s, d);
  }
}

// ---------------------------------------------------------------------------
// contraction on the matrix cores.  Stage 1 writes, per piece, the outer
// feature row F[p] and the column row B[p] (both FP64; integer entries are
// exact below 2^53).  Stage 2 is the segment-level product sum_p F[p]^T B[p]
// as a split-K FP64 MFMA GEMM (v_mfma_f64_16x16x4f64) with block-major
// partials, merged deterministically afterwards.
// ---------------------------------------------------------------------------
constexpr int kSPieces = 64;                       // pieces per staging round
constexpr double kExactInt = 9007199254740992.0;   // 2^53

__device__ __forceinline__ double feat_d(const DFeat& F, const int64_t* mu, const int32_t* codes,
                                         const double* atoms, bool is_int) {
  const int64_t m = feat_int(F, mu, codes);
  double x = (double)m;
  if (!is_int) {
    if (F.a1 >= 0) x *= atoms[F.a1];
    if (F.a2 >= 0) x *= atoms[F.a2];
  }
  return x;
}

template <typename T>
__device__ __forceinline__ double col_d(const DContract* C, const DColB& B, int64_t p, const int32_t* codes,
                                        const double* atoms) {
  if (B.kind == B_PSI_F) return (double)((const T*)C->psi_f)[p * C->psi_f_stride + B.entry];
  const int64_t cnt = C->row_pieces ? (C->w ? C->w[p] : 1) : C->psi_i[p * C->psi_i_stride + B.entry];
  if (B.kind == B_PSI_I) return (double)cnt;
  const DFeat& F = B.feat;
  int64_t m = cnt;
  if (F.c1 >= 0 && codes[F.c1] != F.v1) m = 0;
  if (F.c2 >= 0 && codes[F.c2] != F.v2) m = 0;
  double x = (double)m;
  if (F.a1 >= 0) x *= atoms[F.a1];
  if (F.a2 >= 0) x *= atoms[F.a2];
  return x;
}

// col_d in two steps: the global load of the piece's partial sum or count,
// which depends on nothing staged in LDS, and the code tests and factors
// applied to it afterwards
template <typename T>
__device__ __forceinline__ double col_raw(const DContract* C, const DColB& B, int64_t p) {
  if (B.kind == B_PSI_F) return (double)((const T*)C->psi_f)[p * C->psi_f_stride + B.entry];
  return (double)(C->row_pieces ? (C->w ? C->w[p] : 1) : C->psi_i[p * C->psi_i_stride + B.entry]);
}
__device__ __forceinline__ double col_finish(const DColB& B, double raw, const int32_t* codes, const double* atoms) {
  if (B.kind == B_PSI_F || B.kind == B_PSI_I) return raw;
  const DFeat& F = B.feat;
  double x = raw;
  if (F.c1 >= 0 && codes[F.c1] != F.v1) x = 0.0;
  if (F.c2 >= 0 && codes[F.c2] != F.v2) x = 0.0;
  if (F.a1 >= 0) x *= atoms[F.a1];
  if (F.a2 >= 0) x *= atoms[F.a2];
  return x;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kGemmMT = 64;   // features per block: 4 wavefronts x 16 rows

int gemm_tile_cols(int ng) { return std::min(8, std::max(1, (ng + 15) / 16)); }
int gemm_macro_tiles(int nf, int ng) {
  const int nt = 16 * gemm_tile_cols(ng);
  return ((nf + kGemmMT - 1) / kGemmMT) * ((ng + nt - 1) / nt);
}

// Fused contraction: per chunk of kFKC pieces the block stages the pieces
// outer view rows, multiplicities, factors and codes in LDS, builds its slice
// of F (features x pieces) and B (columns x pieces) there, and multiplies them
// on the matrix cores; F and B never travel through HBM.  Block (x, y): K
// range x, macro-tile y (64 features x 16*TN columns).  Scatter cells are
// evaluated by the y == 0 blocks.  The loads of a chunk that need nothing
// from LDS (the piece keys of the outer views and the pieces' partial sums)
// are issued into registers while the chunk before it is built and
// multiplied, so a chunk waits on two rounds of dependent loads instead of
// four.  This holds for the FP64 tile kernels; in the BF16 split kernels
// the registers it takes would cost a wave per SIMD of occupancy.  The
// descriptors that lanes index by their own view, atom or column (views,
// piece columns, outer atoms and codes) are copied to LDS once per block, so
// that no global load of a descriptor precedes the load of a value.
constexpr int kFKC = 16;
constexpr int kFThreads = 256;   // one B entry per thread and column tile of 16
static_assert(kFKC * 16 == kFThreads, "each thread builds TN entries of the B slice");
static_assert(kFKC * kMaxViews <= kFThreads, "each thread looks up at most one view row");

int contract_fused_lds_bytes(const DContract& C, int tn) {
  const int nt = 16 * tn;
  const int sb = (nt % 32 == 0) ? nt + 16 : nt;
  int64_t b = (int64_t)kFKC * (kGemmMT + 16) * 8 + (int64_t)kFKC * sb * 8;
  b += (int64_t)kFKC * (2 * kMaxViews * 8 + C.n_masks * 8 + C.n_atoms * 8) + (int64_t)kFKC * C.n_codes * 4;
  b = (b + 15) & ~(int64_t)15;
  b += (int64_t)kGemmMT * sizeof(DFeat) + (int64_t)nt * sizeof(DColB);
  b += (int64_t)C.n_pcols * sizeof(DCol) + (int64_t)C.n_views * sizeof(DView) +
       (int64_t)(C.n_atoms + C.n_codes) * sizeof(DAtom);
  return (int)((b + 15) & ~(int64_t)15);
}
int contract_fused_chunk() { return kFKC; }

// BF16 split of a value into NS parts, each the bf16 (nearest even) of what
// the parts before it leave of the FP32 value.  NS = 2: hi*hi' + hi*lo' +
// lo*hi' leaves out lo*lo' and the residues below lo, about 2^-16 of the
// product at most.
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
// NS = 3 adds mid: x = hi + mid + lo to 24 bits, and the six products
// hi*hi' + hi*mid' + mid*hi' + hi*lo' + mid*mid' + lo*hi' reach FP32 accuracy
template <int NS>
__device__ __forceinline__ void bf16_split(double x, uint16_t* part) {
  float r = (float)x;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    part[k] = bf16_rne(r);
    r -= __uint_as_float((uint32_t)part[k] << 16);
  }
}
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kBKS = kFKC + 4;   // bf16 row stride of the split tiles (8-byte aligned rows of 40 bytes)

template <typename T, int TN, int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NS > 0 ? 1 : TN < 8 ? 4 : 3))) void k_contract_fused(const DContract* __restrict__ C, const DGemm* __restrict__ G) {
  constexpr int NT = 16 * TN;
  constexpr int SA = kGemmMT + 16;
  constexpr int SB = (NT % 32 == 0) ? NT + 16 : NT;
  extern __shared__ __align__(16) unsigned char smem[];
  double* As = (double*)smem;                              // [kFKC][SA]
  double* Bs = As + kFKC * SA;                             // [kFKC][SB]
  int64_t* vrow_s = (int64_t*)(Bs + kFKC * SB);            // [kFKC][kMaxViews]
  int64_t* vcnt_s = vrow_s + kFKC * kMaxViews;
  const int NF = C->n_feat, NG = C->n_col, NFI = C->n_feat_int;
  const int NA = C->n_atoms, NC = C->n_codes, NM = C->n_masks, NV = C->n_views;
  int64_t* mu_s = vcnt_s + kFKC * kMaxViews;               // [kFKC][NM]
  double* atom_s = (double*)(mu_s + kFKC * NM);            // [kFKC][NA]
  int32_t* code_s = (int32_t*)(atom_s + kFKC * NA);        // [kFKC][NC]
  unsigned char* dp = (unsigned char*)(code_s + kFKC * NC);
  dp = (unsigned char*)(((uintptr_t)dp + 15) & ~(uintptr_t)15);
  DFeat* feat_s = (DFeat*)dp;                              // this block's features
  DColB* col_s = (DColB*)(feat_s + kGemmMT);               // this block's columns
  DCol* pcol_d = (DCol*)(col_s + NT);                      // descriptors: [n_pcols]
  DView* view_d = (DView*)(pcol_d + C->n_pcols);           // [NV]
  DAtom* atom_d = (DAtom*)(view_d + NV);                   // [NA]
  DAtom* code_d = atom_d + NA;                             // [NC]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n_ntiles = (NG + NT - 1) / NT;
  const int f0 = (blockIdx.y / n_ntiles) * kGemmMT;
  const int g0 = (blockIdx.y % n_ntiles) * NT;
  for (int i = threadIdx.x; i < kGemmMT; i += blockDim.x)
    if (f0 + i < NF) feat_s[i] = C->feats[f0 + i];
  for (int i = threadIdx.x; i < NT; i += blockDim.x)
    if (g0 + i < NG) col_s[i] = C->cols[g0 + i];
  for (int i = threadIdx.x; i < C->n_pcols; i += blockDim.x) pcol_d[i] = C->pcols[i];
  for (int i = threadIdx.x; i < NV; i += blockDim.x) view_d[i] = C->views[i];
  for (int i = threadIdx.x; i < NA; i += blockDim.x) atom_d[i] = C->atoms[i];
  for (int i = threadIdx.x; i < NC; i += blockDim.x) code_d[i] = C->codes[i];
  const int64_t kb = (int64_t)blockIdx.x * G->k_per_block;
  const int64_t ke = std::min<int64_t>(G->n, kb + G->k_per_block);
  const bool do_scatter = blockIdx.y == 0;
  // split (BF16) tiles hold no integer cell (integer features and columns come
  // first); the others stay on the exact FP64 path
  const bool split = NS > 0 && (f0 >= C->n_feat_int || g0 >= C->n_col_int);
  uint16_t* Asp = (uint16_t*)As;                           // NS planes of [kGemmMT][kBKS]
  uint16_t* Bsp = (uint16_t*)Bs;                           // NS planes of [NT][kBKS]
  bool over = false;
  f64x4 acc[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // entry i of this thread's (FP64, piece-major) B slice: piece and column
  // of t = tid + 256 i
  const int tid = threadIdx.x;
  int tq = tid;   // made opaque once per chunk: the column records stay in LDS, not in registers
  auto b_pi = [&](int i) { return (tq + kFThreads * i) / NT; };
  auto b_gl = [&](int i) { return (tq + kFThreads * i) % NT; };
  constexpr bool kPreB = NS == 0;
  int64_t nx_vr = 0;
  double nx_b[TN];
  auto prefetch = [&](int64_t c0) {
    const int npn = (int)std::min<int64_t>(kFKC, ke - c0);
    if (kPreB && tid < npn * NV) {
      const int pi = tid / NV, v = tid % NV;
      const DView& V = view_d[v];
      int64_t vr = 0;
      for (int k = 0; k < V.nkey; ++k) vr += ld_int(pcol_d[V.key_src[k]], c0 + pi) * V.key_stride[k];
      nx_vr = vr;
    }
    if constexpr (kPreB) {
#pragma unroll
      for (int i = 0; i < TN; ++i) {
        const int pi = b_pi(i), gl = b_gl(i);
        nx_b[i] = (pi < npn && g0 + gl < NG) ? col_raw<T>(C, col_s[gl], c0 + pi) : 0.0;
      }
    }
  };
  __syncthreads();
  if (kPreB && kb < ke) prefetch(kb);
  for (int64_t cb = kb; cb < ke; cb += kFKC) {
    const int np = (int)std::min<int64_t>(kFKC, ke - cb);
    if constexpr (kPreB) {
      asm volatile("" : "+v"(tq));
      if (tid < np * NV) {
        const int pi = tid / NV, v = tid % NV;
        vrow_s[pi * kMaxViews + v] = nx_vr;
        vcnt_s[pi * kMaxViews + v] = view_d[v].cnt[nx_vr];
      }
    } else {
      for (int t = threadIdx.x; t < np * NV; t += blockDim.x) {
        const int pi = t / NV, v = t % NV;
        const DView& V = view_d[v];
        int64_t vr = 0;
        for (int k = 0; k < V.nkey; ++k) vr += ld_int(pcol_d[V.key_src[k]], cb + pi) * V.key_stride[k];
        vrow_s[pi * kMaxViews + v] = vr;
        vcnt_s[pi * kMaxViews + v] = V.cnt[vr];
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < np * NM; t += blockDim.x) {
      const int pi = t / NM, m = t % NM;
      const uint32_t bits = C->masks[m];
      int64_t x = 1;
      for (int v = 0; v < NV; ++v)
        if (bits & (1u << v)) x *= vcnt_s[pi * kMaxViews + v];
      mu_s[pi * NM + m] = x;
    }
    for (int t = threadIdx.x; t < np * NA; t += blockDim.x) {
      const int pi = t / NA, a = t % NA;
      const DAtom& At = atom_d[a];
      T x;
      if (At.kind == SRC_COL) x = ld_val<T>(pcol_d[At.src], cb + pi);
      else {
        const int v = At.src;
        x = vcnt_s[pi * kMaxViews + v] ? view_val<T>(view_d[v], vrow_s[pi * kMaxViews + v], At.slot) : (T)0;
      }
      atom_s[pi * NA + a] = (double)x;
    }
    for (int t = threadIdx.x; t < np * NC; t += blockDim.x) {
      const int pi = t / NC, c = t % NC;
      const DAtom& Cd = code_d[c];
      int32_t x;
      if (Cd.kind == SRC_COL) x = (int32_t)ld_int(pcol_d[Cd.src], cb + pi);
      else {
        const int v = Cd.src;
        const DView& V = view_d[v];
        x = vcnt_s[pi * kMaxViews + v] ? V.codes[vrow_s[pi * kMaxViews + v] * V.n_codes + Cd.slot] : -1;
      }
      code_s[pi * NC + c] = x;
    }
    __syncthreads();
    // the F and B slices of the chunk; rows past the chunk and columns past
    // the matrix are zero
    if (split) {
      for (int t = threadIdx.x; t < kFKC * kGemmMT; t += blockDim.x) {
        const int pi = t % kFKC, fl = t / kFKC, f = f0 + fl;
        double x = 0.0;
        if (pi < np && f < NF) x = feat_d(feat_s[fl], mu_s + pi * NM, code_s + pi * NC, atom_s + pi * NA, f < NFI);
        uint16_t part[NS > 0 ? NS : 1];
        bf16_split<NS>(x, part);
#pragma unroll
        for (int k = 0; k < NS; ++k) Asp[k * kGemmMT * kBKS + fl * kBKS + pi] = part[k];
      }
      for (int t = threadIdx.x; t < kFKC * NT; t += blockDim.x) {
        const int pi = t % kFKC, gl = t / kFKC, g = g0 + gl;
        const double x =
            (pi < np && g < NG) ? col_d<T>(C, col_s[gl], cb + pi, code_s + pi * NC, atom_s + pi * NA) : 0.0;
        uint16_t part[NS > 0 ? NS : 1];
        bf16_split<NS>(x, part);
#pragma unroll
        for (int k = 0; k < NS; ++k) Bsp[k * NT * kBKS + gl * kBKS + pi] = part[k];
      }
    } else {
    for (int t = threadIdx.x; t < kFKC * kGemmMT; t += blockDim.x) {
      const int pi = t / kGemmMT, fl = t % kGemmMT, f = f0 + fl;
      double x = 0.0;
      if (pi < np && f < NF) {
        x = feat_d(feat_s[fl], mu_s + pi * NM, code_s + pi * NC, atom_s + pi * NA, f < NFI);
        if (f < NFI && !(x < kExactInt)) over = true;
      }
      As[pi * SA + fl] = x;
    }
    if constexpr (kPreB) {
#pragma unroll
      for (int i = 0; i < TN; ++i) {
        const int pi = b_pi(i), gl = b_gl(i), g = g0 + gl;
        Bs[pi * SB + gl] =
            (pi < np && g < NG) ? col_finish(col_s[gl], nx_b[i], code_s + pi * NC, atom_s + pi * NA) : 0.0;
      }
    } else {
      for (int t = threadIdx.x; t < kFKC * NT; t += blockDim.x) {
        const int pi = t / NT, gl = t % NT, g = g0 + gl;
        Bs[pi * SB + gl] =
            (pi < np && g < NG) ? col_d<T>(C, col_s[gl], cb + pi, code_s + pi * NC, atom_s + pi * NA) : 0.0;
      }
    }
    }
    if (kPreB && cb + kFKC < ke) prefetch(cb + kFKC);
    if (do_scatter) {
      const int n_sc = C->n_scatter;
      for (int t = threadIdx.x; t < np * n_sc; t += blockDim.x) {
        const int pi = t / n_sc, sc = t % n_sc;
        const int o = C->sc_out[sc];
        int64_t row = 0;
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
          const int cidx = C->so_code[o * 3 + k];
          if (cidx < 0) continue;
          const int32_t cval = code_s[pi * NC + cidx];
          if (cval < 0) ok = false;
          row += (int64_t)cval * C->so_stride[o * 3 + k];
        }
        if (!ok) continue;
        const int f = C->sc_f[sc], g = C->sc_g[sc];
        const int comp = C->sc_comp[sc];
        const DColB& B = C->cols[g];
        if (comp < 0) {
          int64_t v = feat_int(C->feats[f], mu_s + pi * NM, code_s + pi * NC);
          int64_t cnt = C->row_pieces ? (C->w ? C->w[cb + pi] : 1) : C->psi_i[(cb + pi) * C->psi_i_stride + B.entry];
          if (B.kind == B_CNTF) {
            const DFeat& F = B.feat;
            if (F.c1 >= 0 && code_s[pi * NC + F.c1] != F.v1) cnt = 0;
            if (F.c2 >= 0 && code_s[pi * NC + F.c2] != F.v2) cnt = 0;
          }
          v *= cnt;
          if (v) scatter_count(C, o, row, v);
        } else {
          const double a = feat_d(C->feats[f], mu_s + pi * NM, code_s + pi * NC, atom_s + pi * NA, f < NFI);
          const double b = col_d<T>(C, B, cb + pi, code_s + pi * NC, atom_s + pi * NA);
          const double v = a * b;
          if (v != 0.0) scatter_value(C, o, row, comp, v);
        }
      }
    }
    __syncthreads();
    if (split) {
      // one K=16 step per chunk: lane l holds rows l%16, k = 4*(l/16)..+3
      const int ko = 4 * (lane >> 4);
      bf16x4 a[NS > 0 ? NS : 1];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        a[k] = *(const bf16x4*)(Asp + k * kGemmMT * kBKS + (16 * w + (lane & 15)) * kBKS + ko);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        bf16x4 b[NS > 0 ? NS : 1];
#pragma unroll
        for (int k = 0; k < NS; ++k)
          b[k] = *(const bf16x4*)(Bsp + k * NT * kBKS + (16 * j + (lane & 15)) * kBKS + ko);
        // smallest products first; every pair whose parts sum to at most NS - 1
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int sum = NS - 1; sum >= 0; --sum)
#pragma unroll
          for (int i = 0; i <= sum; ++i)
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[sum - i], c, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] += (double)c[i];
      }
    } else {
#pragma unroll
    for (int kk = 0; kk < kFKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a = As[kr * SA + 16 * w + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const double b = Bs[kr * SB + 16 * j + (lane & 15)];
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
      }
    }
    }
    __syncthreads();
  }
  if (over) atomicOr(C->err_flag, 4);
  const int64_t ncell = (int64_t)NF * NG;
  double* out = G->part + (int64_t)blockIdx.x * ncell;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int g = g0 + 16 * j + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // output rows of lane l: (l/16) + 4i for the FP64 16x16x4 product,
      // 4(l/16) + i for the bf16 16x16x16 one
      const int f = f0 + 16 * w + (split ? 4 * (lane >> 4) + i : (lane >> 4) + 4 * i);
      if (f < NF && g < NG) out[(int64_t)f * NG + g] = acc[j][i];
    }
  }
}

template <typename T, int NS>
static void launch_contract_fused_t(const DContract* c, const DGemm* g, int tn, int gx, int gy, int lds,
                                    hipStream_t s) {
  dim3 grid(gx, gy), b(kFThreads);
  switch (tn) {
#define CASE(N)                                                               \
  case N:                                                                     \
    allow_lds((const void*)&k_contract_fused<T, N, NS>, lds);                 \
    hipLaunchKernelGGL((k_contract_fused<T, N, NS>), grid, b, lds, s, c, g);  \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}
void launch_contract_fused(const DContract* c, const DGemm* g, bool f64, int bf16_parts, int tn, int gx, int gy,
                           int lds, hipStream_t s) {
  if (f64) launch_contract_fused_t<double, 0>(c, g, tn, gx, gy, lds, s);
  else if (bf16_parts == 2) launch_contract_fused_t<float, 2>(c, g, tn, gx, gy, lds, s);
  else if (bf16_parts == 3) launch_contract_fused_t<float, 3>(c, g, tn, gx, gy, lds, s);
  else launch_contract_fused_t<float, 0>(c, g, tn, gx, gy, lds, s);
}

// Row-by-row evaluation of a group whose outputs are all scattered (hash
// tables, or keys with no scan form): one thread per row looks up the outer
// views, forms the multiplicities, factors and codes, and adds every scatter
// cell of the row into its output.  No staging, no barriers: the cost is the
// row's loads and the table updates.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_rows(const DContract* __restrict__ C) {
  const int NA = C->n_atoms, NC = C->n_codes, NM = C->n_masks, NV = C->n_views, n_sc = C->n_scatter;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < C->n_pieces;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t vrow[kMaxViews], vcnt[kMaxViews];
    for (int v = 0; v < NV; ++v) {
      const DView& V = C->views[v];
      int64_t vr = 0;
      for (int k = 0; k < V.nkey; ++k) vr += ld_int(C->pcols[V.key_src[k]], p) * V.key_stride[k];
      vrow[v] = vr;
      vcnt[v] = V.cnt[vr];
    }
    int64_t mu[kMaxMasks * 4];
    for (int m = 0; m < NM; ++m) {
      const uint32_t bits = C->masks[m];
      int64_t x = 1;
      for (int v = 0; v < NV; ++v)
        if (bits & (1u << v)) x *= vcnt[v];
      mu[m] = x;
    }
    double atom[kMaxOuterAtoms];
    for (int a = 0; a < NA; ++a) {
      const DAtom& At = C->atoms[a];
      T x;
      if (At.kind == SRC_COL) x = ld_val<T>(C->pcols[At.src], p);
      else x = vcnt[At.src] ? view_val<T>(C->views[At.src], vrow[At.src], At.slot) : (T)0;
      atom[a] = (double)x;
    }
    int32_t code[kMaxOuterCodes];
    for (int c = 0; c < NC; ++c) {
      const DAtom& Cd = C->codes[c];
      int32_t x;
      if (Cd.kind == SRC_COL) x = (int32_t)ld_int(C->pcols[Cd.src], p);
      else {
        const DView& V = C->views[Cd.src];
        x = vcnt[Cd.src] ? V.codes[vrow[Cd.src] * V.n_codes + Cd.slot] : -1;
      }
      code[c] = x;
    }
    for (int sc = 0; sc < n_sc; ++sc) {
      const int o = C->sc_out[sc];
      int64_t row = 0;
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        const int cidx = C->so_code[o * 3 + k];
        if (cidx < 0) continue;
        const int32_t cval = code[cidx];
        if (cval < 0) ok = false;
        row += (int64_t)cval * C->so_stride[o * 3 + k];
      }
      if (!ok) continue;
      const int f = C->sc_f[sc], g = C->sc_g[sc];
      const int comp = C->sc_comp[sc];
      const DColB& B = C->cols[g];
      if (comp < 0) {
        int64_t v = feat_int(C->feats[f], mu, code);
        int64_t cnt = C->w ? C->w[p] : 1;
        if (B.kind == B_CNTF) {
          const DFeat& F = B.feat;
          if (F.c1 >= 0 && code[F.c1] != F.v1) cnt = 0;
          if (F.c2 >= 0 && code[F.c2] != F.v2) cnt = 0;
        }
        v *= cnt;
        if (v) scatter_count(C, o, row, v);
      } else {
        const double a = feat_d(C->feats[f], mu, code, atom, f < C->n_feat_int);
        const double b = col_d<T>(C, B, p, code, atom);
        const double v = a * b;
        if (v != 0.0) scatter_value(C, o, row, comp, v);
      }
    }
  }
}
void launch_scatter_rows(const DContract* c, bool f64, int grid, hipStream_t s) {
  if (f64) hipLaunchKernelGGL(k_scatter_rows<double>, dim3(grid), dim3(256), 0, s, c);
  else hipLaunchKernelGGL(k_scatter_rows<float>, dim3(grid), dim3(256), 0, s, c);
}

// Block-major partial merge: block x takes 16 consecutive cells (one 128-byte
// line per partial row) and 16 lanes' worth of partial blocks per cell; each
// thread sums its blocks in order (compensated), then the 16 partial sums of a
// cell are combined in a fixed order.  Integer cells are sums of exact
// integers below 2^53 and are converted exactly (err_flag code 4 otherwise).
__global__ __launch_bounds__(256) void k_merge_bm(const DCell* __restrict__ cells, int64_t n_cells,
                                                  const double* __restrict__ part, int n_blocks, int ng,
                                                  int64_t ncell, int32_t* err_flag) {
  __shared__ double ps[16][17], pc[16][17];
  const int cl = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t c = (int64_t)blockIdx.x * 16 + cl;
  double s = 0.0, cc = 0.0;
  int64_t off = 0;
  if (c < n_cells) {
    off = (int64_t)cells[c].f * ng + cells[c].g;
    for (int b = grp; b < n_blocks; b += 16) kadd(s, cc, part[(int64_t)b * ncell + off]);
  }
  ps[grp][cl] = s;
  pc[grp][cl] = cc;
  __syncthreads();
  if (grp == 0 && c < n_cells) {
    double t = 0.0, tc = 0.0;
    for (int j = 0; j < 16; ++j) {
      kadd(t, tc, ps[j][cl]);
      kadd(t, tc, pc[j][cl]);
    }
    t += tc;
    const DCell& X = cells[c];
    if (X.is_int) {
      if (!(fabs(t) < kExactInt)) atomicOr(err_flag, 4);
      const int64_t v = (int64_t)llrint(t);
      if (X.vals) {
        if (X.vals_f64) ((double*)X.vals)[X.idx] += (double)v;
        else ((float*)X.vals)[X.idx] += (float)v;
      } else {
        X.cnt[X.idx] += v;
      }
    } else {
      if (X.vals_f64) ((double*)X.vals)[X.idx] += t;
      else ((float*)X.vals)[X.idx] += (float)t;
    }
  }
}
void launch_merge_bm(const DCell* cells, int64_t n_cells, const double* part, int n_blocks, int ng, int64_t ncell,
                     int32_t* err_flag, hipStream_t s) {
  if (n_cells <= 0) return;
  const int grid = (int)((n_cells + 15) / 16);
  hipLaunchKernelGGL(k_merge_bm, dim3(grid), dim3(256), 0, s, cells, n_cells, part, n_blocks, ng, ncell, err_flag);
}

// ---------------------------------------------------------------------------
// deterministic merges
// ---------------------------------------------------------------------------
// one wavefront per cell: lanes read the cell's block partials (contiguous),
// fixed-order lane sums and a fixed butterfly -> deterministic
__global__ __launch_bounds__(256) void k_merge_cells(const DCell* __restrict__ cells, int64_t n_cells,
                                                     const double* __restrict__ part_f,
                                                     const int64_t* __restrict__ part_i, int n_blocks, int NF,
                                                     int NG, int NFI, int NGI) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t c = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); c < n_cells; c += waves) {
    const DCell& X = cells[c];
    if (X.is_int) {
      const int64_t* src = part_i + ((int64_t)X.f * NGI + X.g) * n_blocks;
      int64_t s = 0;
      for (int b = lane; b < n_blocks; b += 64) s += src[b];
      s = wave_sum_i64(s);
      if (lane == 0) {
        if (X.vals) {
          if (X.vals_f64) ((double*)X.vals)[X.idx] += (double)s;
          else ((float*)X.vals)[X.idx] += (float)s;
        } else {
          X.cnt[X.idx] += s;
        }
      }
    } else {
      const double* src = part_f + ((int64_t)X.f * NG + X.g) * n_blocks;
      double s = 0, cc = 0;
      for (int b = lane; b < n_blocks; b += 64) kadd(s, cc, src[b]);
      s = wave_sum_comp(s, cc);
      if (lane == 0) {
        if (X.vals_f64) ((double*)X.vals)[X.idx] += s;
        else ((float*)X.vals)[X.idx] += (float)s;
      }
    }
  }
}
void launch_merge_cells(const DCell* cells, int64_t n_cells, const double* part_f, const int64_t* part_i,
                        int n_blocks, int NF, int NG, int NFI, int NGI, hipStream_t s) {
  if (n_cells <= 0) return;
  int grid = (int)std::min<int64_t>((n_cells + 3) / 4, 4096);
  hipLaunchKernelGGL(k_merge_cells, dim3(grid), dim3(256), 0, s, cells, n_cells, part_f, part_i, n_blocks, NF, NG,
                     NFI, NGI);
}

// table partials: dst[i] += sum_b part[b * stride + off + i]
// block y sums a slice of the partial rows; slices meet in integer atomics
// (exact, so the order does not matter)
constexpr int kReduceSlice = 16;   // partial rows per thread
__global__ void k_table_reduce(const DTableReduce* __restrict__ R) {
  const int b0 = blockIdx.y * kReduceSlice;
  const int b1 = min(R->n_blocks, b0 + kReduceSlice);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R->n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t s = 0;
    for (int b = b0; b < b1; ++b) s += R->part_i[(int64_t)b * R->stride + R->off + i];
    if (s == 0) continue;
    atomic_add_i64(&R->dst_cnt[i], s);
    for (int k = 0; k < R->n_copy; ++k) atomic_add_f64(&R->copy_vals[i * R->copy_nv + R->copy_comp[k]], (double)s);
  }
}
__global__ void k_count_copy(const DCountCopy* __restrict__ C) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < C->n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = C->cnt[i];
    if (c == 0) continue;
    for (int k = 0; k < C->n_copy; ++k) C->vals[i * C->nv + C->comp[k]] += (double)c;
  }
}
void launch_count_copy(const DCountCopy* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_count_copy, dim3((int)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s, d);
}

__global__ void k_count_keys(const unsigned long long* __restrict__ keys, int64_t n, unsigned long long* out) {
  unsigned long long c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += keys[i] != 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}
void launch_count_keys(const unsigned long long* keys, int64_t n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_count_keys, dim3((int)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, keys, n,
                     out);
}

// ---------------------------------------------------------------------------
// radix-partitioned counting of large group-by tables of SUM(1)
// ---------------------------------------------------------------------------
// Every launch set runs, in order:
//   k_part_w8          per row one byte: filter weight and the views' 0/1 counts
//   k_part_direct      tables of one slice (at most 2^15 cells): a chunk of rows
//                      per workgroup counted in LDS straight from the key columns
//   k_part_tile        tables of several slices and hashed tables: a tile of
//                      rows per workgroup, its entries (low 15 bits of the cell,
//                      or the whole cell) ordered by slice in LDS and written
//                      back contiguously, with the tile's slice offsets
//   k_part_bases       entries per slice summed over tiles, slice starts
//   k_part_slice_count one workgroup per (slice, chunk of tiles): the slice's
//                      segments of every tile counted in LDS
//   k_part_reduce      per-chunk partial tables summed into the output
//   k_part_hash        hashed tables: one workgroup per group of cells
// No pass scatters single entries to global memory and no pass adds to a
// global counter per row, so the counting runs at the rate of the key-column
// reads and the contiguous entry round trip.
constexpr int kPartSlice = 1 << kPartShift;        // cells one LDS table holds
constexpr int kPartTileThreads = 1024;
constexpr int kPartCountThreads = 1024;
constexpr int kPartDirectUnroll = 8;               // rows per thread in flight in the direct count (int32 cells)
constexpr int kPartSegUnroll = 8;                  // entries per lane in flight in the segment count

struct PartRow {
  int64_t v0, v1, v2, v3;   // the row's key in each view (named fields: kept in registers)
  uint32_t vok;             // bit v: the row has a partner tuple in view v (count 1)
  int32_t w;
};

__device__ __forceinline__ int64_t part_view_key(const DPartCount& D, int v, int64_t row) {
  int64_t k = (int64_t)D.vkey[v][0][row] * D.vstride[v][0];
  if (D.vnkey[v] > 1) k += (int64_t)D.vkey[v][1][row] * D.vstride[v][1];
  return k;
}

__device__ __forceinline__ void part_row(const DPartCount& D, int64_t row, PartRow& R) {
  R.w = D.w ? D.w[row] : 1;
  R.vok = 0;
  R.v0 = R.v1 = R.v2 = R.v3 = 0;
  const int nv = D.n_views;
  if (nv > 0) R.v0 = part_view_key(D, 0, row);
  if (nv > 1) R.v1 = part_view_key(D, 1, row);
  if (nv > 2) R.v2 = part_view_key(D, 2, row);
  if (nv > 3) R.v3 = part_view_key(D, 3, row);
  if (nv > 0 && R.v0 >= 0 && R.v0 < D.vnkeys[0] && D.vcnt[0][R.v0] > 0) R.vok |= 1u;
  if (nv > 1 && R.v1 >= 0 && R.v1 < D.vnkeys[1] && D.vcnt[1][R.v1] > 0) R.vok |= 2u;
  if (nv > 2 && R.v2 >= 0 && R.v2 < D.vnkeys[2] && D.vcnt[2][R.v2] > 0) R.vok |= 4u;
  if (nv > 3 && R.v3 >= 0 && R.v3 < D.vnkeys[3] && D.vcnt[3][R.v3] > 0) R.vok |= 8u;
}

// the same from the byte k_part_w8 stored (view keys recomputed only when
// some output reads a view's code)
__device__ __forceinline__ void part_row_w8(const DPartCount& D, int64_t row, PartRow& R) {
  const uint32_t x = D.w8[row];
  R.w = (int32_t)(x & 1u);
  R.vok = x >> 1;
  R.v0 = R.v1 = R.v2 = R.v3 = 0;
  if (D.vkeys_needed) {
    const int nv = D.n_views;
    if (nv > 0) R.v0 = part_view_key(D, 0, row);
    if (nv > 1) R.v1 = part_view_key(D, 1, row);
    if (nv > 2) R.v2 = part_view_key(D, 2, row);
    if (nv > 3) R.v3 = part_view_key(D, 3, row);
  }
}

__device__ __forceinline__ int64_t part_vrow(const PartRow& R, int v) {
  return v == 0 ? R.v0 : v == 1 ? R.v1 : v == 2 ? R.v2 : R.v3;
}

// dense cell of output o for the row; -1: the row does not count (weight 0);
// -2: a key outside its declared domain
__device__ __forceinline__ int64_t part_cell(const DPartCount& D, int o, int64_t row, const PartRow& R) {
  if (!R.w || (D.vmask[o] & ~R.vok)) return -1;
  int64_t cell = 0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < D.nkey[o]) {
      const int src = D.ksrc[o][k];
      const int32_t c =
          src < 0 ? D.kcol[o][k][row] : D.vcodes[src][part_vrow(R, src) * D.vncodes[src] + D.kslot[o][k]];
      bad |= c < 0 || c >= D.kdom[o][k];
      cell += (int64_t)c * D.kstride[o][k];
    }
  }
  return bad ? -2 : cell;
}

// the cell of output o for a row in range, -1 otherwise; a key outside its
// domain gives -1 and sets *bad (no side effect here, so that the callers'
// loads of several rows stay in flight together)
__device__ __forceinline__ int64_t part_row_cell(const DPartCount& D, int o, int64_t row, bool in, bool* bad) {
  if (!in) return -1;
  PartRow R;
  part_row_w8(D, row, R);
  const int64_t cell = part_cell(D, o, row, R);
  *bad |= cell == -2;
  return cell < 0 ? -1 : cell;
}

// The cells of output o for U rows first + u * stride (rows at or past r_end
// give -1), with every load of the batch issued before any is used: row
// indices are clamped into range so that no load sits behind a branch.
// Outputs whose keys are all columns of the relation take this straight
// path; keys carried by views go through part_row_w8 and part_cell, a row
// at a time.  C is int32_t for dense tables (at most 2^24 cells) and
// int64_t for hashed ones.
template <int U, typename C>
__device__ __forceinline__ void part_load_cells(const DPartCount& D, int o, int32_t first, int32_t stride,
                                                int32_t r_end, C (&cell)[U], bool& bad) {
  const int32_t last = r_end - 1;
  if (!D.keys_cols[o]) {
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      const C v = (C)part_row_cell(D, o, r < r_end ? r : last, r < r_end, &bad);
#pragma unroll
      for (int j = 0; j < U; ++j)   // keeps cell[] in registers (no dynamic index)
        if (j == u) cell[j] = v;
    }
    return;
  }
  uint32_t wb[U];
  int32_t k0[U], k1[U], k2[U];
  {
    const uint8_t* w8 = D.w8;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      wb[u] = w8[r < r_end ? r : last];
    }
  }
  const int nk = D.nkey[o];
  {
    const int32_t* c = D.kcol[o][0];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      k0[u] = c[r < r_end ? r : last];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) k1[u] = k2[u] = 0;
  if (nk > 1) {
    const int32_t* c = D.kcol[o][1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      k1[u] = c[r < r_end ? r : last];
    }
  }
  if (nk > 2) {
    const int32_t* c = D.kcol[o][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      k2[u] = c[r < r_end ? r : last];
    }
  }
  const uint32_t vm = D.vmask[o];
  const int64_t d0 = D.kdom[o][0], d1 = nk > 1 ? D.kdom[o][1] : 1, d2 = nk > 2 ? D.kdom[o][2] : 1;
  const int64_t s0 = D.kstride[o][0], s1 = nk > 1 ? D.kstride[o][1] : 0, s2 = nk > 2 ? D.kstride[o][2] : 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool in = first + u * stride < r_end;
    const bool counts = in && (wb[u] & 1u) && !(vm & ~(wb[u] >> 1));
    const bool out = k0[u] < 0 || k0[u] >= d0 || k1[u] < 0 || k1[u] >= d1 || k2[u] < 0 || k2[u] >= d2;
    bad |= counts && out;
    if (sizeof(C) == 4)
      cell[u] = counts && !out ? (C)((uint32_t)k0[u] * (uint32_t)s0 + (uint32_t)k1[u] * (uint32_t)s1 +
                                     (uint32_t)k2[u] * (uint32_t)s2)
                               : (C)-1;
    else
      cell[u] = counts && !out ? (C)((int64_t)k0[u] * s0 + (int64_t)k1[u] * s1 + (int64_t)k2[u] * s2) : (C)-1;
  }
}

// The weights of the same rows for a weighted output: the product of the
// counts of the output's multiplicity views per row (0 where the cell is
// -1), loads issued together; a product of 2^32 or more sets `big` (the
// partition count's LDS tables hold 32-bit counts).
template <int U, typename C>
__device__ __forceinline__ void part_load_weights(const DPartCount& D, int o, int32_t first, int32_t stride,
                                                  int32_t r_end, const C (&cell)[U], uint32_t (&wt)[U], bool& big) {
  const int32_t last = r_end - 1;
  uint64_t p[U];
#pragma unroll
  for (int u = 0; u < U; ++u) p[u] = 1;
  const uint32_t m = D.vmask[o] & D.vmult;
#pragma unroll
  for (int v = 0; v < kPartViews; ++v) {
    if (!((m >> v) & 1u)) continue;
    const uint32_t* wv = D.wv[v];
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t r = first + u * stride;
      x[u] = wv[r < r_end ? r : last];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t q = p[u] * x[u];   // both factors below 2^32: no 64-bit overflow
      big |= cell[u] >= 0 && q > 0xffffffffull;
      p[u] = q > 0xffffffffull ? 0xffffffffull : q;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) wt[u] = cell[u] >= 0 ? (uint32_t)p[u] : 0u;
}

// bits of a cell for the hashed outputs' grouping (a 64-bit finalising mix)
__device__ __forceinline__ uint64_t part_mix(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

// pass 0: the per-row byte (bit 0 filter weight, bits 1.. the views' 0/1
// counts) for every later pass and the counts of multiplicity views (shared
// by the launch sets of the node that read the same views)
__global__ void __launch_bounds__(256) k_part_w8(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < D.n_rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    PartRow R;
    part_row(D, row, R);
    D.w8[row] = (uint8_t)((R.w ? 1u : 0u) | (R.vok << 1));
    // the counts of the views with several tuples per key (weights of the
    // weighted outputs; a key outside the view counts 0)
    for (int v = 0; v < D.n_views; ++v) {
      if (!((D.vmult >> v) & 1u)) continue;
      const int64_t k = part_vrow(R, v);
      const int64_t c = k >= 0 && k < D.vnkeys[v] ? D.vcnt[v][k] : 0;
      if (c > (int64_t)0xffffffff) atomicOr(D.err_flag, 16);
      D.wv[v][row] = c <= 0 ? 0u : c > (int64_t)0xffffffff ? 0xffffffffu : (uint32_t)c;
    }
  }
}

// flush of an LDS table of one slice: the output's cells [base, base + n)
// (one chunk: plain stores, the cells are the workgroup's own), else the
// chunk's partial table
__device__ __forceinline__ void part_flush(const DPartCount& D, int o, int c, int64_t base, const uint32_t* bins) {
  const int64_t n = min((int64_t)kPartSlice, D.n_cells[o] - base);
  if (D.chunks[o] <= 1) {
    int64_t* out = D.out_cnt[o] + base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = (int64_t)bins[i];
  } else {
    uint32_t* out = D.partial + D.partial_base[o] + (int64_t)c * D.n_cells[o] + base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = bins[i];
  }
}

// pass 1a, tables of one slice: workgroup (chunk, output) counts the chunk's
// rows in LDS; every thread keeps kPartDirectUnroll rows' loads in flight
// (W: the weighted outputs, each row adding its weight)
template <bool W>
__global__ void __launch_bounds__(kPartCountThreads) k_part_direct(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  const int o = blockIdx.y, c = blockIdx.x;
  if (o >= D.n_out || D.hashed[o] || D.n_buckets[o] != 1 || c >= D.chunks[o] || (D.weighted[o] != 0) != W) return;
  extern __shared__ uint32_t bins[];
  for (int i = threadIdx.x; i < kPartSlice; i += blockDim.x) bins[i] = 0;
  __syncthreads();
  const int64_t per = (D.n_rows + D.chunks[o] - 1) / D.chunks[o];
  const int64_t r0 = (int64_t)c * per, r1 = min(D.n_rows, r0 + per);
  const int64_t step = (int64_t)kPartDirectUnroll * blockDim.x;
  bool bad = false, big = false;
  for (int64_t base = r0; base < r1; base += step) {
    int32_t cell[kPartDirectUnroll];
    const int32_t first = (int32_t)base + (int32_t)threadIdx.x;
    part_load_cells<kPartDirectUnroll>(D, o, first, (int32_t)blockDim.x, (int32_t)r1, cell, bad);
    uint32_t wt[kPartDirectUnroll];
    if (W) part_load_weights<kPartDirectUnroll>(D, o, first, (int32_t)blockDim.x, (int32_t)r1, cell, wt, big);
#pragma unroll
    for (int u = 0; u < kPartDirectUnroll; ++u)
      if (cell[u] >= 0) {
        if (W) {
          // a weighted add that wraps the 32-bit LDS count is reported, not returned wrong
          const uint32_t old = atomicAdd(&bins[cell[u]], wt[u]);
          big |= (uint32_t)(old + wt[u]) < old;
        } else {
          atomicAdd(&bins[cell[u]], 1u);
        }
      }
  }
  if (bad) atomicOr(D.err_flag, 2);
  if (W && big) atomicOr(D.err_flag, 16);
  __syncthreads();
  part_flush(D, o, c, 0, bins);
}

// pass 1b: workgroup (tile, output) orders its tile's entries by slice (a
// counting sort in LDS: rank within the slice by an LDS atomic, slice starts
// by a scan) and writes them to the tile's region of the output's entry
// array, contiguously, with the tile's S + 1 slice offsets.  Dense tables
// store the low 15 bits of the cell (the slice is implied by the position),
// hashed tables the whole cell, grouped by the top kPartHashBits bits of
// its mix.
template <typename E, int TILE, bool W>
__global__ void __launch_bounds__(kPartTileThreads) k_part_tile(const DPartCount* __restrict__ Dp) {
  constexpr bool kHashed = sizeof(E) == 8;
  constexpr int PER = TILE / kPartTileThreads;
  const DPartCount& D = *Dp;
  const int o = blockIdx.y, tile = blockIdx.x;
  if (o >= D.n_out || (D.hashed[o] != 0) != kHashed || (!kHashed && D.n_buckets[o] <= 1) ||
      tile >= D.n_tiles[o] || (D.weighted[o] != 0) != W)
    return;
  __shared__ uint32_t off[kPartMaxBuckets + 1];
  __shared__ E stage[TILE];
  __shared__ uint32_t wstage[W ? TILE : 1];   // weighted outputs: the entries' weights
  const int S = D.n_buckets[o];
  for (int i = threadIdx.x; i <= S; i += blockDim.x) off[i] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)tile * TILE;
  typedef typename std::conditional<kHashed, int64_t, int32_t>::type C;
  C cell[PER];
  bool bad = false;
  part_load_cells<PER>(D, o, (int32_t)r0 + (int32_t)threadIdx.x, kPartTileThreads, (int32_t)D.n_rows, cell, bad);
  if (bad) atomicOr(D.err_flag, 2);
  uint32_t wt[PER];
  if (W) {
    bool big = false;
    part_load_weights<PER>(D, o, (int32_t)r0 + (int32_t)threadIdx.x, kPartTileThreads, (int32_t)D.n_rows, cell, wt,
                           big);
    if (big) atomicOr(D.err_flag, 16);
  }
  uint32_t sr[PER];   // slice << 16 | rank within the slice; ~0: no entry
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    sr[u] = ~0u;
    if (cell[u] >= 0) {
      const uint32_t s = kHashed ? (uint32_t)(part_mix((uint64_t)cell[u]) >> (64 - kPartHashBits)) : (uint32_t)(cell[u] >> kPartShift);
      sr[u] = (s << 16) | atomicAdd(&off[s + 1], 1u);
    }
  }
  __syncthreads();
  // inclusive scan of off[1..S] by the first wavefront: off[s] = start of slice s
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    constexpr int kPer = (kPartMaxBuckets + 63) / 64;
    uint32_t v[kPer], run = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int s = 1 + lane * kPer + i;
      v[i] = s <= S ? off[s] : 0u;
      run += v[i];
    }
    uint32_t incl = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    uint32_t acc = incl - run;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int s = 1 + lane * kPer + i;
      acc += v[i];
      if (s <= S) off[s] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (sr[u] != ~0u) {
      const uint32_t pos = off[sr[u] >> 16] + (sr[u] & 0xffffu);
      stage[pos] = kHashed ? (E)(uint64_t)cell[u] : (E)((uint64_t)cell[u] & (kPartSlice - 1));
      if (W) wstage[pos] = wt[u];
    }
  __syncthreads();
  const int n = (int)off[S];
  E* dst = (kHashed ? (E*)(D.part64 + (int64_t)D.slot[o] * D.n_rows) : (E*)(D.part + (int64_t)D.slot[o] * D.n_rows)) + r0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = stage[i];
  if (W) {
    uint32_t* wd = D.partw + (int64_t)D.wslot[o] * D.n_rows + r0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) wd[i] = wstage[i];
  }
  // slice-major: the offsets of one slice over consecutive tiles are adjacent
  uint32_t* to = D.toff + D.toff_base[o] + tile;
  const int64_t nt = D.n_tiles[o];
  for (int i = threadIdx.x; i <= S; i += blockDim.x) to[(int64_t)i * nt] = off[i];
  for (int i = threadIdx.x; i < S; i += blockDim.x)
    if (off[i + 1] > off[i]) atomicAdd(&D.btotal[o * kPartMaxBuckets + i], off[i + 1] - off[i]);
}

// slice starts per output (exclusive scan of the slice totals)
__global__ void __launch_bounds__(kPartMaxBuckets) k_part_bases(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  const int o = blockIdx.x;
  if (o >= D.n_out || !D.hashed[o]) return;
  __shared__ uint32_t tmp[kPartMaxBuckets];
  const int nb = D.n_buckets[o];
  const uint32_t v = (int)threadIdx.x < nb ? D.btotal[(int64_t)o * kPartMaxBuckets + threadIdx.x] : 0u;
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < kPartMaxBuckets; d <<= 1) {
    const uint32_t x = (int)threadIdx.x >= d ? tmp[threadIdx.x - d] : 0u;
    __syncthreads();
    tmp[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t* bs = D.bstart + (int64_t)o * (kPartMaxBuckets + 1);
  if ((int)threadIdx.x < nb) {
    bs[threadIdx.x] = tmp[threadIdx.x] - v;
    D.btotal[(int64_t)o * kPartMaxBuckets + threadIdx.x] = 0;   // zero again for the next run's tile pass
  }
  if (threadIdx.x == 0) bs[nb] = tmp[kPartMaxBuckets - 1];
}

// Visits every entry of slice s in tiles [t0, t1) of output o.  The
// workgroup takes one tile per thread at a time, flattens the tiles'
// segments of slice s (a block scan of their lengths) and gives each thread
// kPartSegUnroll consecutive entries per round (the loads in flight
// together), so every wavefront has work however the entries spread over
// the tiles.  visit(entry, weight) is called per entry: the entry's weight
// from `wsrc` (same positions as `src`) when W, else 1.  sh_start and
// sh_excl hold blockDim entries, sh_w 16 + 1.
template <typename E, bool W, typename F>
__device__ __forceinline__ void part_segments(const DPartCount& D, int o, int s, int t0, int t1, const E* src,
                                              const uint32_t* wsrc, int64_t* sh_start, uint32_t* sh_excl,
                                              uint32_t* sh_w, F&& visit) {
  const int lane = (int)__lane_id();
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int B = blockDim.x;
  const int tile_rows = D.tile_rows[o];
  const int64_t nt = D.n_tiles[o];
  const uint32_t* to = D.toff + D.toff_base[o];
  for (int tb = t0; tb < t1; tb += B) {
    const int t = tb + threadIdx.x;
    uint32_t lo = 0, hi = 0;
    if (t < t1) {
      lo = to[(int64_t)s * nt + t];
      hi = to[(int64_t)(s + 1) * nt + t];
    }
    const uint32_t len = hi - lo;
    uint32_t incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    if (lane == 63) sh_w[wid] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
      const uint32_t x = sh_w[w];
      before += w < wid ? x : 0u;
      total += x;
    }
    sh_excl[threadIdx.x] = before + incl - len;
    sh_start[threadIdx.x] = (int64_t)t * tile_rows + lo;
    __syncthreads();
    for (uint32_t k0 = (uint32_t)threadIdx.x * kPartSegUnroll; k0 < total; k0 += (uint32_t)B * kPartSegUnroll) {
      // the last tile whose segment starts at or before k0
      int lo_i = 0, hi_i = B - 1;
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (sh_excl[mid] <= k0) lo_i = mid;
        else hi_i = mid - 1;
      }
      int cur = lo_i;
      int64_t idx[kPartSegUnroll];
#pragma unroll
      for (int u = 0; u < kPartSegUnroll; ++u) {
        const uint32_t k = k0 + (uint32_t)u;
        idx[u] = -1;
        if (k < total) {
          while (cur + 1 < B && sh_excl[cur + 1] <= k) ++cur;
          idx[u] = sh_start[cur] + (k - sh_excl[cur]);
        }
      }
      // the loads, unconditional (an index past the range reads entry 0)
      E e[kPartSegUnroll];
      uint32_t w[kPartSegUnroll];
#pragma unroll
      for (int u = 0; u < kPartSegUnroll; ++u) {
        e[u] = src[idx[u] >= 0 ? idx[u] : 0];
        w[u] = W ? wsrc[idx[u] >= 0 ? idx[u] : 0] : 1u;
      }
#pragma unroll
      for (int u = 0; u < kPartSegUnroll; ++u)
        if (idx[u] >= 0) visit(e[u], w[u]);
    }
    __syncthreads();
  }
}

// pass 2, dense tables of several slices: workgroup (slice x chunk, output)
// counts the slice's segments of the chunk's tiles in LDS
template <bool W>
__global__ void __launch_bounds__(kPartCountThreads) k_part_slice_count(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  const int o = blockIdx.y;
  if (o >= D.n_out || D.hashed[o] || D.n_buckets[o] <= 1 || (D.weighted[o] != 0) != W) return;
  const int C = D.chunks[o];
  const int x = blockIdx.x;
  if (x >= D.n_buckets[o] * C) return;
  const int s = x / C, c = x % C;
  extern __shared__ uint32_t bins[];
  __shared__ int64_t sh_start[kPartCountThreads];
  __shared__ uint32_t sh_excl[kPartCountThreads];
  __shared__ uint32_t sh_w[kPartCountThreads / 64];
  for (int i = threadIdx.x; i < kPartSlice; i += blockDim.x) bins[i] = 0;
  __syncthreads();
  const int nt = D.n_tiles[o];
  const int t0 = (int)((int64_t)c * nt / C), t1 = (int)((int64_t)(c + 1) * nt / C);
  bool big = false;
  part_segments<uint16_t, W>(D, o, s, t0, t1, D.part + (int64_t)D.slot[o] * D.n_rows,
                             W ? D.partw + (int64_t)D.wslot[o] * D.n_rows : nullptr, sh_start, sh_excl, sh_w,
                             [&](uint16_t v, uint32_t w) {
                               if (W) {
                                 // a weighted add that wraps the 32-bit LDS count is reported
                                 const uint32_t old = atomicAdd(&bins[v], w);
                                 big |= (uint32_t)(old + w) < old;
                               } else {
                                 atomicAdd(&bins[v], 1u);
                               }
                             });
  if (W && big) atomicOr(D.err_flag, 16);
  __syncthreads();
  part_flush(D, o, c, (int64_t)s << kPartShift, bins);
}

// per-chunk partial tables summed into the outputs (grid-stride per output)
__global__ void k_part_reduce(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  const int o = blockIdx.y;
  if (o >= D.n_out || D.hashed[o] || D.chunks[o] <= 1) return;
  const int C = D.chunks[o];
  const int64_t n = D.n_cells[o];
  const uint32_t* p = D.partial + D.partial_base[o];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t s = 0;
    for (int c = 0; c < C; ++c) s += p[(int64_t)c * n + i];
    D.out_cnt[o][i] = (int64_t)s;
  }
}

// pass 2 of hashed outputs, one workgroup per group of cells: the group's
// segments are gathered from every tile and ordered by sub-group (a counting
// sort on the next hash bits, into the group's region of part64b;
// sub-groups of at most kPartSubCells entries), then every wavefront counts whole
// sub-groups in an LDS hash table of its own (kPartWaveSlots slots; no workgroup
// barrier between sub-groups) and writes their (cell, count) pairs to the
// group's own region of the output's table (cap / kPartHashBuckets slots, positions from
// an LDS counter: no global atomics).  The region's slots past its groups
// stay zero: the table is cleared once when allocated, and each run clears
// only the slots the previous run filled past this run's groups (the group
// count per region is kept beside the table; it also sizes a regrowth).  A
// full LDS table or a full region sets the table's overflow flag (the run is
// repeated with a larger table).
constexpr int kPartWaveSlots = 512;
constexpr int kPartHashWaves = 16;
constexpr int kPartSubCells = 384;
constexpr int kPartMaxSub = 4096;
constexpr int kPartHashLds = kPartWaveSlots * kPartHashWaves * 12 + (2 * kPartMaxSub + 2) * 4;
template <bool W>
__global__ void __launch_bounds__(kPartHashWaves * 64) k_part_hash(const DPartCount* __restrict__ Dp) {
  const DPartCount& D = *Dp;
  const int o = blockIdx.y;
  if (o >= D.n_out || !D.hashed[o] || (D.weighted[o] != 0) != W) return;
  extern __shared__ unsigned long long lkeys[];
  __shared__ int64_t sh_start[kPartHashWaves * 64];
  __shared__ uint32_t sh_excl[kPartHashWaves * 64];
  __shared__ uint32_t sh_w[kPartHashWaves];
  uint32_t* lcnt = (uint32_t*)(lkeys + kPartWaveSlots * kPartHashWaves);
  uint32_t* suboff = lcnt + kPartWaveSlots * kPartHashWaves;   // [S + 1]
  uint32_t* cursor = suboff + kPartMaxSub + 1;                 // [S]; cursor[kPartMaxSub] = entries written
  const DHashOut& H = D.htab[D.hidx[o]];
  const int64_t cap = H.mask + 1;
  const int b = blockIdx.x;
  const int64_t region = cap / kPartHashBuckets;
  const int64_t region0 = (int64_t)b * region;
  const uint32_t* bs = D.bstart + (int64_t)o * (kPartMaxBuckets + 1);
  const int64_t s0 = bs[b], s1 = bs[b + 1];
  const int lane = (int)__lane_id(), wid = threadIdx.x >> 6;
  __shared__ uint32_t sh_prev;   // groups the last run left in this region (only thread 0 touches the record)
  if (threadIdx.x == 0) {
    cursor[kPartMaxSub] = 0;
    sh_prev = H.used ? H.used[b] : 0xffffffffu;
  }
  int S = 1, sbits = 0;
  while (S < kPartMaxSub && (int64_t)S * kPartSubCells < s1 - s0) {
    S <<= 1;
    ++sbits;
  }
  const uint64_t* part = D.part64 + (int64_t)D.slot[o] * D.n_rows;
  uint64_t* sorted = D.part64b + (int64_t)D.slot[o] * D.n_rows;
  // weighted outputs: each entry's weight travels with it through the sort
  const uint32_t* part_w = W ? D.partw + (int64_t)D.wslot[o] * D.n_rows : nullptr;
  uint32_t* sorted_w = W ? D.partwb + (int64_t)D.wslot[o] * D.n_rows : nullptr;
  constexpr unsigned long long kEmpty = ~0ull;
  auto sub_of = [&](uint64_t cell) {
    return sbits ? (int)((part_mix(cell) >> (64 - kPartHashBits - sbits)) & (uint64_t)(S - 1)) : 0;
  };
  if (s0 < s1) {
    // counting sort of the group by sub-group, gathered from the tiles
    for (int i = threadIdx.x; i <= S; i += blockDim.x) suboff[i] = 0;
    __syncthreads();
    const int nt = D.n_tiles[o];
    part_segments<uint64_t, false>(D, o, b, 0, nt, part, nullptr, sh_start, sh_excl, sh_w,
                                   [&](uint64_t cell, uint32_t) { atomicAdd(&suboff[sub_of(cell) + 1], 1u); });
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 1; i <= S; ++i) suboff[i] += suboff[i - 1];
    __syncthreads();
    for (int i = threadIdx.x; i < S; i += blockDim.x) cursor[i] = suboff[i];
    __syncthreads();
    part_segments<uint64_t, W>(D, o, b, 0, nt, part, part_w, sh_start, sh_excl, sh_w, [&](uint64_t cell, uint32_t w) {
      const uint32_t pos = atomicAdd(&cursor[sub_of(cell)], 1u);
      sorted[s0 + pos] = cell;
      if (W) sorted_w[s0 + pos] = w;
    });
    __threadfence_block();
    __syncthreads();
    unsigned long long* wkeys = lkeys + wid * kPartWaveSlots;
    uint32_t* wcnt = lcnt + wid * kPartWaveSlots;
    bool full = false, big = false;
    for (int sub = wid; sub < S; sub += kPartHashWaves) {
      const int64_t r0 = s0 + suboff[sub], r1 = s0 + suboff[sub + 1];
      if (r0 >= r1) continue;
      for (int i = lane; i < kPartWaveSlots; i += 64) {
        wkeys[i] = kEmpty;
        wcnt[i] = 0;
      }
      __builtin_amdgcn_wave_barrier();
      for (int64_t i0 = r0 + lane; i0 < r1; i0 += 4 * 64) {
        uint64_t cv[4];
        uint32_t wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t i = i0 + (int64_t)u * 64;
          cv[u] = sorted[i < r1 ? i : r0];
          wv[u] = W ? sorted_w[i < r1 ? i : r0] : 1u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (i0 + (int64_t)u * 64 >= r1) continue;
          const uint64_t cell = cv[u];
          uint32_t slot = (uint32_t)part_mix(cell) & (kPartWaveSlots - 1);
          bool done = false;
          for (int probe = 0; probe < kPartWaveSlots && !done; ++probe) {
            const unsigned long long prev = atomicCAS(&wkeys[slot], kEmpty, (unsigned long long)cell);
            if (prev == kEmpty || prev == cell) {
              if (W) {
                // a weighted add that wraps the 32-bit LDS count is reported
                const uint32_t old = atomicAdd(&wcnt[slot], wv[u]);
                big |= (uint32_t)(old + wv[u]) < old;
              } else {
                atomicAdd(&wcnt[slot], 1u);
              }
              done = true;
            }
            slot = (slot + 1) & (kPartWaveSlots - 1);
          }
          full |= !done;
        }
      }
      __builtin_amdgcn_wave_barrier();
      for (int base = 0; base < kPartWaveSlots; base += 64) {
        const int slot = base + lane;
        const unsigned long long key = wkeys[slot];
        const bool occ = key != kEmpty;
        const unsigned long long m = __ballot(occ);
        uint32_t p0 = 0;
        if (lane == 0 && m) p0 = atomicAdd(&cursor[kPartMaxSub], (uint32_t)__popcll(m));
        p0 = __shfl(p0, 0, 64);
        if (occ) {
          const int64_t pos = (int64_t)p0 + __popcll(m & ((1ull << lane) - 1ull));
          if (pos < region) {
            H.keys[region0 + pos] = key + 1ull;
            H.cnt[region0 + pos] = (int64_t)wcnt[slot];
          } else {
            full = true;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (full) {
      atomicOr(H.ovf, 1);
      atomicOr(D.err_flag, 8);
    }
    if (W && big) atomicOr(D.err_flag, 16);
  }
  __syncthreads();
  // the region's slots past this run's groups hold none: the table was
  // cleared when it was allocated, so only the slots the last run filled
  // beyond them are cleared (every slot, for a table without the record)
  const int64_t total = (int64_t)cursor[kPartMaxSub];
  const int64_t used = min(total, region);
  const int64_t prev = min((int64_t)sh_prev, region);
  for (int64_t i = used + threadIdx.x; i < prev; i += blockDim.x) H.keys[region0 + i] = 0ull;
  if (H.used && threadIdx.x == 0) H.used[b] = (uint32_t)total;
}

constexpr int kPartTileDense = 16384;
constexpr int kPartTileHash = 16384;
constexpr int kPartTileHashW = 8192;   // weighted hashed tiles stage a 4-byte weight per entry too
int part_tile_rows(bool hashed, bool weighted) {
  return hashed ? (weighted ? kPartTileHashW : kPartTileHash) : kPartTileDense;
}

void launch_part_count(const DPartCount* d, const DPartCount& h, int phase, hipStream_t s) {
  if (h.n_rows <= 0 || h.n_out <= 0) return;
  // grids per kind; [1]: the weighted outputs' kernels
  int tiles_dense[2] = {0, 0}, slice_chunks[2] = {0, 0}, direct_chunks[2] = {0, 0}, tiles_hash[2] = {0, 0};
  for (int o = 0; o < h.n_out; ++o) {
    const int w = h.weighted[o] ? 1 : 0;
    if (h.hashed[o]) {
      tiles_hash[w] = std::max(tiles_hash[w], h.n_tiles[o]);
    } else if (h.n_buckets[o] <= 1) {
      direct_chunks[w] = std::max(direct_chunks[w], h.chunks[o]);
    } else {
      tiles_dense[w] = std::max(tiles_dense[w], h.n_tiles[o]);
      slice_chunks[w] = std::max(slice_chunks[w], h.n_buckets[o] * h.chunks[o]);
    }
  }
  switch (phase) {
    case kPartPhaseRows: {
      const int g8 = (int)std::min<int64_t>((h.n_rows + 255) / 256, 8192);
      hipLaunchKernelGGL(k_part_w8, dim3(g8), dim3(256), 0, s, d);
      break;
    }
    case kPartPhaseDirect:
      if (direct_chunks[0])
        hipLaunchKernelGGL(k_part_direct<false>, dim3(direct_chunks[0], h.n_out), dim3(kPartCountThreads),
                           kPartSlice * 4, s, d);
      if (direct_chunks[1])
        hipLaunchKernelGGL(k_part_direct<true>, dim3(direct_chunks[1], h.n_out), dim3(kPartCountThreads),
                           kPartSlice * 4, s, d);
      break;
    case kPartPhaseTile:
      if (tiles_dense[0])
        hipLaunchKernelGGL((k_part_tile<uint16_t, kPartTileDense, false>), dim3(tiles_dense[0], h.n_out),
                           dim3(kPartTileThreads), 0, s, d);
      if (tiles_dense[1])
        hipLaunchKernelGGL((k_part_tile<uint16_t, kPartTileDense, true>), dim3(tiles_dense[1], h.n_out),
                           dim3(kPartTileThreads), 0, s, d);
      break;
    case kPartPhaseSlices:
      if (slice_chunks[0])
        hipLaunchKernelGGL(k_part_slice_count<false>, dim3(slice_chunks[0], h.n_out), dim3(kPartCountThreads),
                           kPartSlice * 4, s, d);
      if (slice_chunks[1])
        hipLaunchKernelGGL(k_part_slice_count<true>, dim3(slice_chunks[1], h.n_out), dim3(kPartCountThreads),
                           kPartSlice * 4, s, d);
      break;
    case kPartPhaseReduce:
      hipLaunchKernelGGL(k_part_reduce, dim3(256, h.n_out), dim3(256), 0, s, d);
      break;
    case kPartPhaseTileHash:
      if (tiles_hash[0])
        hipLaunchKernelGGL((k_part_tile<uint64_t, kPartTileHash, false>), dim3(tiles_hash[0], h.n_out),
                           dim3(kPartTileThreads), 0, s, d);
      if (tiles_hash[1])
        hipLaunchKernelGGL((k_part_tile<uint64_t, kPartTileHashW, true>), dim3(tiles_hash[1], h.n_out),
                           dim3(kPartTileThreads), 0, s, d);
      if (tiles_hash[0] || tiles_hash[1])
        hipLaunchKernelGGL(k_part_bases, dim3(h.n_out), dim3(kPartMaxBuckets), 0, s, d);
      break;
    case kPartPhaseHash:
      if (tiles_hash[0])
        hipLaunchKernelGGL(k_part_hash<false>, dim3(kPartHashBuckets, h.n_out), dim3(kPartHashWaves * 64),
                           kPartHashLds, s, d);
      if (tiles_hash[1])
        hipLaunchKernelGGL(k_part_hash<true>, dim3(kPartHashBuckets, h.n_out), dim3(kPartHashWaves * 64),
                           kPartHashLds, s, d);
      break;
    default:
      break;
  }
}

// largest count of each listed view (grid-stride, one atomicMax per block)
__global__ void k_mult_max(const DMultCheck* __restrict__ D) {
  __shared__ unsigned long long red[4];
  for (int v = 0; v < D->n; ++v) {
    unsigned long long m = 0;
    const int64_t* c = D->cnt[v];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < D->n_keys[v];
         i += (int64_t)gridDim.x * blockDim.x)
      m = max(m, (unsigned long long)max<int64_t>(c[i], 0));
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
      if (m) atomicMax(&D->maxv[v], m);
    }
    __syncthreads();
  }
}

// rows x product of the largest multiplicities against 2^31 - 1; resets maxv
__global__ void k_mult_verdict(const DMultCheck* __restrict__ D) {
  if (threadIdx.x != 0) return;
  double prod = D->rows;
  for (int v = 0; v < D->n; ++v) {
    const unsigned long long m = D->maxv[v];
    prod *= (double)(m ? m : 1ull);
    D->maxv[v] = 0;
  }
  if (prod > 2147483647.0) atomicOr(D->err_flag, 16);
}

void launch_mult_check(const DMultCheck* d, const DMultCheck& h, hipStream_t s) {
  int64_t most = 1;
  for (int v = 0; v < h.n; ++v) most = std::max(most, h.n_keys[v]);
  hipLaunchKernelGGL(k_mult_max, dim3((int)std::min<int64_t>((most + 255) / 256, 1024)), dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_mult_verdict, dim3(1), dim3(64), 0, s, d);
}

void launch_table_reduce(const DTableReduce* d, int64_t n, int n_blocks, hipStream_t s) {
  if (n <= 0) return;
  const int gy = std::max(1, (n_blocks + kReduceSlice - 1) / kReduceSlice);
  const int gx = (int)std::min<int64_t>((n + 255) / 256, std::max<int64_t>(1, 8192 / gy));
  hipLaunchKernelGGL(k_table_reduce, dim3(gx, gy), dim3(256), 0, s, d);
}

}  // namespace lmfao
