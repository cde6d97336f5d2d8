// Rk-means steps 2 and 3 (paper, section 3, "Rk-means"): weighted 1-D
// k-means on every projection of D (the step-1 group counts), and the
// grid-coreset query SELECT C_1..C_n, SUM(1) FROM D JOIN A_1 .. A_n GROUP BY
// C_1..C_n over joins whose tuples a root row determines (every other
// relation reached through a key).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace lmfao {

// ---------------------------------------------------------------------------
// step 2: Lloyd's algorithm per set, one workgroup each (FP64)
// ---------------------------------------------------------------------------
constexpr int kKmThreads = 256;

__device__ __forceinline__ double km_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

__global__ void __launch_bounds__(kKmThreads) k_kmeans_1d(const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ values,
                                                         const int64_t* __restrict__ weights, int k, int max_iter,
                                                         double* __restrict__ centroids,
                                                         int32_t* __restrict__ assignment,
                                                         int32_t* __restrict__ steps_out) {
  __shared__ double c[kKmMaxClusters];
  __shared__ double sw[kKmMaxClusters], swv[kKmMaxClusters];
  __shared__ double red[kKmThreads / 64];
  __shared__ double carry_s;
  __shared__ int changed;
  const int set = blockIdx.x;
  const int64_t b = off[set], e = off[set + 1], m = e - b;
  if (m <= 0) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) centroids[(int64_t)set * k + i] = 0.0;
    if (threadIdx.x == 0) steps_out[set] = 0;
    return;
  }
  // total weight (integer weights: exact in FP64)
  double part = 0.0;
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) part += (double)weights[j];
  const double total = km_block_sum(part, red);
  // start: centroid i = first value whose cumulative weight reaches
  // (2i + 1) / (2k) of the total (chunks of blockDim values, block scan)
  if (threadIdx.x == 0) carry_s = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) c[i] = (double)values[e - 1];
  __syncthreads();
  for (int64_t j0 = b; j0 < e; j0 += blockDim.x) {
    const int64_t j = j0 + threadIdx.x;
    const double w = j < e ? (double)weights[j] : 0.0;
    double incl = w;
    for (int d = 1; d < 64; d <<= 1) {
      const double x = __shfl_up(incl, d, 64);
      if ((threadIdx.x & 63) >= d) incl += x;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = incl;
    __syncthreads();
    double before = carry_s;
    for (int w8 = 0; w8 < (int)(threadIdx.x >> 6); ++w8) before += red[w8];
    const double cum = before + incl, prev = cum - w;
    if (j < e)
      for (int i = 0; i < k; ++i) {
        const double t = (double)(2 * i + 1) / (double)(2 * k) * total;
        if (prev < t && cum >= t) c[i] = (double)values[j];
      }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) carry_s = cum;
    __syncthreads();
  }
  // Lloyd: assign to the nearest centroid (lowest index on ties), move each
  // centroid to the weighted mean of its values; stop when nothing moves
  int steps = 0;
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
    const double v = (double)values[j];
    int best = 0;
    double bd = fabs(v - c[0]);
    for (int i = 1; i < k; ++i) {
      const double d = fabs(v - c[i]);
      if (d < bd) {
        bd = d;
        best = i;
      }
    }
    assignment[j] = best;
  }
  __syncthreads();
  while (steps < max_iter) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) sw[i] = swv[i] = 0.0;
    __syncthreads();
    for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
      const double w = (double)weights[j];
      const int a = assignment[j];
      atomicAdd(&sw[a], w);                       // integer weights and values: every partial
      atomicAdd(&swv[a], w * (double)values[j]);  // sum is an exact integer below 2^53
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x)
      if (sw[i] > 0.0) c[i] = swv[i] / sw[i];
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    ++steps;
    int moved = 0;
    for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
      const double v = (double)values[j];
      int best = 0;
      double bd = fabs(v - c[0]);
      for (int i = 1; i < k; ++i) {
        const double d = fabs(v - c[i]);
        if (d < bd) {
          bd = d;
          best = i;
        }
      }
      moved |= best != assignment[j];
      assignment[j] = best;
    }
    if (moved) atomicOr(&changed, 1);
    __syncthreads();
    if (!changed) break;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) centroids[(int64_t)set * k + i] = c[i];
  if (threadIdx.x == 0) steps_out[set] = steps;
}

void launch_kmeans_1d(const int64_t* off, int n_sets, const int64_t* values, const int64_t* weights, int k,
                      int max_iter, double* centroids, int32_t* assignment, int32_t* steps, hipStream_t s) {
  if (n_sets <= 0) return;
  hipLaunchKernelGGL(k_kmeans_1d, dim3(n_sets), dim3(kKmThreads), 0, s, off, values, weights, k, max_iter,
                     centroids, assignment, steps);
}

// ---------------------------------------------------------------------------
// step 3: the grid coreset
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t grid_mix(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

// the packed cluster ids of the tuple of D a root row determines (false: the
// row has no partner in some relation, it is not in D)
__device__ __forceinline__ bool grid_key(const DGrid& D, int64_t r0, uint64_t (&w)[kGridMaxWords], bool& bad) {
  int32_t row[kGridMaxRels];
  row[0] = (int32_t)r0;
#pragma unroll
  for (int i = 1; i < kGridMaxRels; ++i) {
    if (i >= D.n_rels) break;
    int32_t pr = 0;
#pragma unroll
    for (int q = 0; q < kGridMaxRels; ++q)
      if (q == D.parent[i]) pr = row[q];
    const int32_t key = D.pkey[i][pr];
    if (key < 0 || (int64_t)key >= D.index_n[i]) return false;
    const int32_t rr = D.index[i][key];
    if (rr < 0) return false;
    row[i] = rr;
  }
#pragma unroll
  for (int j = 0; j < kGridMaxWords; ++j) w[j] = 0ull;
  for (int d = 0; d < D.n_dims; ++d) {
    int32_t rr = 0;
#pragma unroll
    for (int q = 0; q < kGridMaxRels; ++q)
      if (q == D.rel[d]) rr = row[q];
    const int32_t v = D.col[d][rr];
    int32_t c = 0;
    if (v >= 0 && (int64_t)v < D.dom[d]) c = D.cluster[d][v];
    else bad = true;
    if (c < 0 || c >= (1 << D.bits)) {
      bad = true;
      c = 0;
    }
    const int bit = d * D.bits;
#pragma unroll
    for (int j = 0; j < kGridMaxWords; ++j)
      if (j == (bit >> 6)) w[j] |= (uint64_t)(uint32_t)c << (bit & 63);
  }
  return true;
}

__device__ __forceinline__ uint64_t grid_hash(const uint64_t (&w)[kGridMaxWords], int n_words) {
  uint64_t h = 0x9e3779b97f4a7c15ull;
#pragma unroll
  for (int j = 0; j < kGridMaxWords; ++j)
    if (j < n_words) h = grid_mix(h ^ w[j]) + (uint64_t)j;
  return h ? h : 1ull;
}

__global__ void k_grid_index(const int32_t* __restrict__ key, int64_t n, int32_t* __restrict__ index,
                             int64_t index_n, int32_t* flag) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = key[r];
    if (k < 0 || (int64_t)k >= index_n) {
      atomicOr(flag, 4);
      continue;
    }
    if (atomicExch(&index[k], (int32_t)r) != -1) atomicOr(flag, 8);   // a key held twice
  }
}

__global__ void k_grid_count(const DGrid* __restrict__ Dp) {
  const DGrid& D = *Dp;
  bool bad = false, full = false;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < D.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[kGridMaxWords];
    if (!grid_key(D, r, w, bad)) continue;
    const uint64_t h = grid_hash(w, D.n_words);
    uint64_t slot = h & (uint64_t)D.mask;
    bool done = false;
    for (int probe = 0; probe < 4096 && !done; ++probe) {
      const unsigned long long prev = atomicCAS(&D.keys[slot], 0ull, (unsigned long long)h);
      if (prev == 0ull) {
        D.rep[slot] = (int32_t)r;
        atomicAdd(&D.cnt[slot], 1ull);
        done = true;
      } else if (prev == h) {
        atomicAdd(&D.cnt[slot], 1ull);
        done = true;
      }
      slot = (slot + 1) & (uint64_t)D.mask;
    }
    full |= !done;
  }
  if (bad) atomicOr(D.flag, 4);
  if (full) atomicOr(D.flag, 2);
}

// every row's packed key against its group's representative: equal
// fingerprints of different keys are reported (flag 1), never merged silently
__global__ void k_grid_verify(const DGrid* __restrict__ Dp) {
  const DGrid& D = *Dp;
  bool bad = false, clash = false;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < D.n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[kGridMaxWords], x[kGridMaxWords];
    if (!grid_key(D, r, w, bad)) continue;
    const uint64_t h = grid_hash(w, D.n_words);
    uint64_t slot = h & (uint64_t)D.mask;
    int32_t rep = -1;
    for (int probe = 0; probe < 4096; ++probe) {
      const unsigned long long k = D.keys[slot];
      if (k == h) {
        rep = D.rep[slot];
        break;
      }
      if (k == 0ull) break;
      slot = (slot + 1) & (uint64_t)D.mask;
    }
    if (rep < 0 || !grid_key(D, rep, x, bad)) {
      clash = true;
      continue;
    }
#pragma unroll
    for (int j = 0; j < kGridMaxWords; ++j) clash |= j < D.n_words && w[j] != x[j];
  }
  if (clash) atomicOr(D.flag, 1);
}

// compaction of the occupied slots (positions from a scan of present flags)
__global__ void k_grid_flags(const DGrid* __restrict__ Dp, uint32_t* pos) {
  const DGrid& D = *Dp;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= D.mask; i += (int64_t)gridDim.x * blockDim.x)
    pos[i] = D.keys[i] != 0ull ? 1u : 0u;
}

__global__ void k_grid_emit(const DGrid* __restrict__ Dp, const uint32_t* __restrict__ pos, int64_t* keys_out,
                            int64_t* cnt_out) {
  const DGrid& D = *Dp;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= D.mask; i += (int64_t)gridDim.x * blockDim.x) {
    if (D.keys[i] == 0ull) continue;
    const int64_t p = pos[i];
    uint64_t w[kGridMaxWords];
    grid_key(D, D.rep[i], w, bad);
    const uint64_t m = (D.bits == 64) ? ~0ull : ((1ull << D.bits) - 1ull);
    for (int d = 0; d < D.n_dims; ++d) {
      const int bit = d * D.bits;
      uint64_t word = 0;
#pragma unroll
      for (int j = 0; j < kGridMaxWords; ++j)
        if (j == (bit >> 6)) word = w[j];
      keys_out[p * D.n_dims + d] = (int64_t)((word >> (bit & 63)) & m);
    }
    cnt_out[p] = (int64_t)D.cnt[i];
  }
}

void launch_grid_index(const int32_t* key, int64_t n, int32_t* index, int64_t index_n, int32_t* flag,
                       hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_grid_index, dim3(grid), dim3(256), 0, s, key, n, index, index_n, flag);
}

void launch_grid_count(const DGrid* d, int64_t n_rows, hipStream_t s) {
  if (n_rows <= 0) return;
  const int grid = (int)std::min<int64_t>((n_rows + 255) / 256, 16384);
  hipLaunchKernelGGL(k_grid_count, dim3(grid), dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_grid_verify, dim3(grid), dim3(256), 0, s, d);
}

void launch_grid_positions(const DGrid* d, int64_t slots, uint32_t* pos, hipStream_t s) {
  const int grid = (int)std::min<int64_t>((slots + 255) / 256, 8192);
  hipLaunchKernelGGL(k_grid_flags, dim3(grid), dim3(256), 0, s, d, pos);
  launch_scan_excl(pos, slots, pos + slots, s);
}

void launch_grid_emit(const DGrid* d, int64_t slots, const uint32_t* pos, int64_t* keys_out, int64_t* cnt_out,
                      hipStream_t s) {
  const int grid = (int)std::min<int64_t>((slots + 255) / 256, 8192);
  hipLaunchKernelGGL(k_grid_emit, dim3(grid), dim3(256), 0, s, d, pos, keys_out, cnt_out);
}

// dense table of a dimension's cluster ids from (code, cluster) pairs
__global__ void k_code_table(const int64_t* __restrict__ codes, const int32_t* __restrict__ cluster, int64_t n,
                             int32_t* __restrict__ table, int64_t dom, int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = codes[i];
    if (v < 0 || v >= dom) {
      atomicOr(flag, 4);
      continue;
    }
    table[v] = cluster[i];
  }
}
void launch_code_table(const int64_t* codes, const int32_t* cluster, int64_t n, int32_t* table, int64_t dom,
                       int32_t* flag, hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_code_table, dim3(grid), dim3(256), 0, s, codes, cluster, n, table, dom, flag);
}

}  // namespace lmfao
