// HIP kernels for gfx950 (MI355X): 64-lane wavefronts, 160 KB LDS per CU.
//
//  k_fill            zero-fill of views and results
//  k_view_build      views whose subtree has one join tuple per key: one
//                    pass over the relation, dense key-indexed tables
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
// view build for single-valued subtrees
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_view_build(const DViewBuild* __restrict__ B) {
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
    if (mu == 0) continue;
    unsigned long long old = atomicAdd((unsigned long long*)&B->out_cnt[row], (unsigned long long)mu);
    if (old != 0 || mu != 1) atomicOr(B->err_flag, 1);   // key not unique
    T* ov = (T*)B->out_vals;
    for (int s = 0; s < B->n_vals; ++s) {
      T x;
      if (B->val_kind[s] == SRC_COL) x = ld_val<T>(B->cols[B->val_src[s]], r);
      else {
        int v = B->val_src[s];
        x = view_val<T>(B->views[v], vrow[v], B->val_slot[s]);
      }
      ov[row * B->n_vals + s] = x;
    }
    for (int s = 0; s < B->n_codes; ++s) {
      int32_t c;
      if (B->code_kind[s] == SRC_COL) c = (int32_t)ld_int(B->cols[B->code_src[s]], r);
      else {
        int v = B->code_src[s];
        c = B->views[v].codes[vrow[v] * B->views[v].n_codes + B->code_slot[s]];
      }
      B->out_codes[row * B->n_codes + s] = c;
    }
  }
}

void launch_view_build(const DViewBuild* d, int64_t n_rows, bool f64, hipStream_t s) {
  if (n_rows <= 0) return;
  int grid = (int)std::min<int64_t>((n_rows + 255) / 256, 8192);
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

// exclusive scan of hist[0..m) in one block of 1024 threads (chunked)
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* a, int64_t m) {
  __shared__ uint32_t part[1024];
  int64_t chunk = (m + 1023) / 1024;
  int64_t b = threadIdx.x * chunk, e = std::min<int64_t>(m, b + chunk);
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += a[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int64_t i = b; i < e; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
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
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, hist, (int64_t)256 * nblocks);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift,
                       hist, nblocks);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *swapped = (passes % 2) == 1;
}

int sort_tile() { return kSortTile; }

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

void launch_make_keys(const DKeyCols* d, uint64_t* keys, uint32_t* idx, int64_t n, hipStream_t s) {
  int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_make_keys, dim3(grid), dim3(256), 0, s, d, keys, idx, n);
}

template <typename E>
__global__ void k_gather(const E* __restrict__ src, const uint32_t* __restrict__ perm, E* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[perm[i]];
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
constexpr int kScanWaves = 4;   // wavefronts per block

__device__ __forceinline__ int tri_index(int i, int j, int n) {
  // extended atoms 0..n (0 = constant 1), i <= j; row-major upper triangle
  return i * (n + 1) - i * (i - 1) / 2 + (j - i);
}

template <typename T, int NA>
__global__ __launch_bounds__(kScanWaves * 64) void k_scan(const DScan* __restrict__ S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  constexpr int NT = (NA + 1) * (NA + 2) / 2;
  // LDS: block count tables (int32), then per-wave histogram bins
  int32_t* tab_i = (int32_t*)smem;
  unsigned char* wbase = (unsigned char*)smem + (((size_t)S->lds_tab_i * 4 + 15) & ~(size_t)15);
  const int hist_i_bytes = (S->hist_i_bins * 4 + 7) & ~7;
  const int hist_bytes = hist_i_bytes + S->hist_f_bins * (int)sizeof(T);
  const int hist_stride = (hist_bytes + 15) & ~15;
  int32_t* hist_i = (int32_t*)(wbase + wid * hist_stride);
  T* hist_f = (T*)((unsigned char*)hist_i + hist_i_bytes);

  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x) tab_i[i] = 0;
  __syncthreads();

  const int n_views = S->n_views;
  const int n_masks = S->n_masks;
  const uint64_t need = S->pf_need;
  const int pf_mask = S->pf_mask_idx;

  for (int item = blockIdx.x * kScanWaves + wid; item < S->n_items; item += gridDim.x * kScanWaves) {
    const int p0 = S->item_piece[item], p1 = S->item_piece[item + 1];
    for (int p = p0; p < p1; ++p) {
      const int64_t rb = S->piece_begin[p], re = S->piece_begin[p + 1];
      // outer multiplicity of direct tables
      int64_t mu_out = 1;
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

      for (int64_t r = rb + lane; r < re; r += 64) {
        // inner views
        int64_t vrow[kMaxViews];
        int64_t vcnt[kMaxViews];
#pragma unroll
        for (int v = 0; v < kMaxViews; ++v) {
          if (v < n_views) {
            const DView& V = S->views[v];
            int64_t vr = 0;
            for (int k = 0; k < V.nkey; ++k) vr += ld_int(S->cols[V.key_src[k]], r) * V.key_stride[k];
            vrow[v] = vr;
            vcnt[v] = V.cnt[vr];
          } else {
            vrow[v] = 0;
            vcnt[v] = 1;
          }
        }
        int64_t mu[kMaxMasks];
#pragma unroll
        for (int m = 0; m < kMaxMasks; ++m) {
          int64_t x = 1;
          if (m < n_masks) {
            uint32_t bits = S->masks[m];
#pragma unroll
            for (int v = 0; v < kMaxViews; ++v)
              if (bits & (1u << v)) x *= vcnt[v];
          }
          mu[m] = x;
        }
        // inner factors
        T av[NA + 1];
        av[0] = (T)1;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const DAtom& A = S->atoms[a];
          T x;
          if (A.kind == SRC_COL) {
            x = ld_val<T>(S->cols[A.src], r);
          } else {
            int64_t vr = 0;
#pragma unroll
            for (int v = 0; v < kMaxViews; ++v)
              if (A.src == v) vr = vrow[v];
            x = view_val<T>(S->views[A.src], vr, A.slot);
          }
          av[a + 1] = x;
        }
        if (S->pf_uniform) {
          int64_t muf = 1;
#pragma unroll
          for (int m = 0; m < kMaxMasks; ++m)
            if (m == pf_mask) muf = mu[m];
          const T muT = (T)muf;
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
              if (t > 0 && ((need >> t) & 1ull)) {
                int mi = S->pf_mask[t];
                int64_t x = 1;
#pragma unroll
                for (int q = 0; q < kMaxMasks; ++q)
                  if (q == mi) x = mu[q];
                kadd(acc[t], cmp[t], (T)x * av[i] * av[j]);
              }
            }
          }
        }
#pragma unroll
        for (int m = 0; m < kMaxMasks; ++m)
          if (m < S->n_pi) {
            int mi = S->pi_mask_idx[m];
            int64_t x = 1;
#pragma unroll
            for (int q = 0; q < kMaxMasks; ++q)
              if (q == mi) x = mu[q];
            cacc[m] += x;
          }
        // codes
        int32_t cv[kMaxCodes];
#pragma unroll
        for (int c = 0; c < kMaxCodes; ++c) {
          cv[c] = 0;
          if (c < S->n_codes) {
            const DAtom& C = S->codes[c];
            if (C.kind == SRC_COL) {
              cv[c] = (int32_t)ld_int(S->cols[C.src], r);
            } else {
              int64_t vr = 0;
#pragma unroll
              for (int v = 0; v < kMaxViews; ++v)
                if (C.src == v) vr = vrow[v];
              const DView& V = S->views[C.src];
              cv[c] = V.codes[vr * V.n_codes + C.slot];
            }
          }
        }
        // per-piece histograms
        for (int h = 0; h < S->n_hists; ++h) {
          const DHist& H = S->hists[h];
          int32_t code = 0;
#pragma unroll
          for (int c = 0; c < kMaxCodes; ++c)
            if (c == H.code) code = cv[c];
          int64_t m = 1;
#pragma unroll
          for (int q = 0; q < kMaxMasks; ++q)
            if (q == H.mask_idx) m = mu[q];
          if (m == 0) continue;
          if (!H.is_float) {
            atomicAdd(&hist_i[H.offset + code], (int32_t)m);
          } else {
            T w = (T)m;
#pragma unroll
            for (int a = 0; a <= NA; ++a) {
              if (a == H.ai + 1) w *= av[a];
              if (a == H.aj + 1) w *= av[a];
            }
            atomicAdd(&hist_f[H.offset + code], w);
          }
        }
        // direct group-by tables
        for (int tb = 0; tb < S->n_tables; ++tb) {
          const DTable& TB = S->tables[tb];
          int64_t row = 0;
          for (int k = 0; k < TB.ncode; ++k) {
            int32_t code = 0;
#pragma unroll
            for (int c = 0; c < kMaxCodes; ++c)
              if (c == TB.code[k]) code = cv[c];
            row += (int64_t)code * TB.stride[k];
          }
          for (int q = 0; q < TB.n_tcomps; ++q) {
            int64_t m = mu_out;
#pragma unroll
            for (int z = 0; z < kMaxMasks; ++z)
              if (z == TB.tmask[q]) m *= mu[z];
            if (m == 0) continue;
            if (TB.tcomp[q] < 0) {
              if (TB.lds) atomicAdd(&tab_i[TB.lds_off + row], (int32_t)m);
              else atomic_add_i64(&TB.cnt[row], m);
            } else {
              T w = (T)m;
#pragma unroll
              for (int a = 0; a <= NA; ++a) {
                if (a == TB.tai[q] + 1) w *= av[a];
                if (a == TB.taj[q] + 1) w *= av[a];
              }
              int64_t di = row * TB.n_vals + TB.tcomp[q];
              if (TB.vals_f64) atomic_add_f64(&((double*)TB.vals)[di], (double)w);
              else atomicAdd(&((float*)TB.vals)[di], (float)w);
            }
          }
        }
      }
      // close the piece: reduce the lanes' partial sums and store the psi row
      T* prow = (T*)S->psi_f + (int64_t)p * S->psi_f_stride;
      int32_t* irow = S->psi_i + (int64_t)p * S->psi_i_stride;
#pragma unroll
      for (int t = 1; t < NT; ++t) {
        if ((need >> t) & 1ull) {
          T s = wave_sum_comp(acc[t], cmp[t]);
          if (lane == 0) prow[S->pf_slot[t]] = s;
        }
      }
#pragma unroll
      for (int m = 0; m < kMaxMasks; ++m)
        if (m < S->n_pi) {
          int64_t s = wave_sum_i64(cacc[m]);
          if (lane == 0) irow[m] = (int32_t)s;
        }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int i = lane; i < S->hist_i_bins; i += 64) irow[S->n_pi + i] = hist_i[i];
      for (int i = lane; i < S->hist_f_bins; i += 64) prow[S->pf_n + i] = hist_f[i];
      __builtin_amdgcn_wave_barrier();
    }
  }
  // flush LDS-privatized tables as block partials
  __syncthreads();
  for (int i = threadIdx.x; i < S->lds_tab_i; i += blockDim.x)
    S->part_i[(int64_t)blockIdx.x * S->lds_tab_i + i] = tab_i[i];
}

int scan_lds_bytes(const DScan& S, bool f64) {
  int hist_bytes = ((S.hist_i_bins * 4 + 7) & ~7) + S.hist_f_bins * (f64 ? 8 : 4);
  int hist_stride = (hist_bytes + 15) & ~15;
  return (int)(((S.lds_tab_i * 4 + 15) & ~15) + kScanWaves * hist_stride);
}

static void allow_lds(const void* fn, int lds) {
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
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
        xi = C->row_pieces ? 1 : C->psi_i[p * C->psi_i_stride + B.entry];
        x = (T)xi;
      } else {
        int64_t cnt = C->row_pieces ? 1 : C->psi_i[p * C->psi_i_stride + B.entry];
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
        int64_t cnt = C->row_pieces ? 1 : C->psi_i[(cb + pi) * C->psi_i_stride + B.entry];
        if (B.kind == B_CNTF) {
          const DFeat& F = B.feat;
          if (F.c1 >= 0 && code_s[pi * NC + F.c1] != F.v1) cnt = 0;
          if (F.c2 >= 0 && code_s[pi * NC + F.c2] != F.v2) cnt = 0;
        }
        v *= cnt;
        if (v) atomic_add_i64(&C->so_cnt[o][row], v);
      } else {
        T v = A[pi * NF + f] * Bm[pi * NG + g];
        if (v != (T)0) {
          int64_t idx = row * C->so_ncomp[o] + comp;
          if (C->so_vals_f64[o]) atomic_add_f64(&((double*)C->so_vals[o])[idx], (double)v);
          else atomicAdd(&((float*)C->so_vals[o])[idx], (float)v);
        }
      }
    }
    __syncthreads();
  }
  // partials
  if (has_tile) {
    double* part = C->part_f + (int64_t)blockIdx.x * NF * NG;
#pragma unroll
    for (int i = 0; i < kTile; ++i)
#pragma unroll
      for (int j = 0; j < kTile; ++j)
        if (f0 + i < NF && g0 + j < NG) part[(int64_t)(f0 + i) * NG + g0 + j] = acc[i][j] + cmp[i][j];
  }
  {
    int64_t* part = C->part_i + (int64_t)blockIdx.x * NFI * NGI + icell0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int cell = threadIdx.x + q * kCThreads;
      if (cell < n_icells) part[cell] = iacc[q];
    }
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
// deterministic merges
// ---------------------------------------------------------------------------
__global__ void k_merge_cells(const DCell* __restrict__ cells, int64_t n_cells, const double* __restrict__ part_f,
                              const int64_t* __restrict__ part_i, int n_blocks, int NF, int NG, int NFI, int NGI) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cells; c += (int64_t)gridDim.x * blockDim.x) {
    const DCell& X = cells[c];
    if (X.is_int) {
      int64_t s = 0;
      for (int b = 0; b < n_blocks; ++b) s += part_i[(int64_t)b * NFI * NGI + (int64_t)X.f * NGI + X.g];
      if (X.vals) {
        if (X.vals_f64) ((double*)X.vals)[X.idx] += (double)s;
        else ((float*)X.vals)[X.idx] += (float)s;
      } else {
        X.cnt[X.idx] += s;
      }
    } else {
      double s = 0, c = 0;
      for (int b = 0; b < n_blocks; ++b) kadd(s, c, part_f[(int64_t)b * NF * NG + (int64_t)X.f * NG + X.g]);
      s += c;
      if (X.vals_f64) ((double*)X.vals)[X.idx] += s;
      else ((float*)X.vals)[X.idx] += (float)s;
    }
  }
}
void launch_merge_cells(const DCell* cells, int64_t n_cells, const double* part_f, const int64_t* part_i,
                        int n_blocks, int NF, int NG, int NFI, int NGI, hipStream_t s) {
  if (n_cells <= 0) return;
  int grid = (int)std::min<int64_t>((n_cells + 255) / 256, 4096);
  hipLaunchKernelGGL(k_merge_cells, dim3(grid), dim3(256), 0, s, cells, n_cells, part_f, part_i, n_blocks, NF, NG,
                     NFI, NGI);
}

// table partials: dst[i] += sum_b part[b * stride + off + i]
__global__ void k_table_reduce(const DTableReduce* __restrict__ R) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R->n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t s = 0;
    for (int b = 0; b < R->n_blocks; ++b) s += R->part_i[(int64_t)b * R->stride + R->off + i];
    R->dst_cnt[i] += s;
  }
}
void launch_table_reduce(const DTableReduce* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_table_reduce, dim3(grid), dim3(256), 0, s, d);
}

}  // namespace lmfao
