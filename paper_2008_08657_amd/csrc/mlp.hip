// Group-count estimator: a two-hidden-layer perceptron trained on the GPU.
//
// Not part of the paper's method: hash tables of outputs whose key space is
// too large for a dense table are sized from a predicted group count, with the
// run's overflow regrowth as the exact fallback, so results never depend on
// the prediction.  Network (FP32): x (d) -> relu(x W1 + b1) (h) ->
// relu(. W2 + b2) (h) -> . w3 + b3; loss: mean squared error against
// log2(1 + groups); optimiser: Adam.  Parameters are one flat array in the
// order W1 (d x h, row-major), b1, W2 (h x h), b2, w3, b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"
#include "lmfao.h"

namespace lmfao {
namespace {

struct Net {
  int d, h;
  int64_t oW1, ob1, oW2, ob2, ow3, ob3, n;
  Net(int d_, int h_) : d(d_), h(h_) {
    oW1 = 0;
    ob1 = oW1 + (int64_t)d * h;
    oW2 = ob1 + h;
    ob2 = oW2 + (int64_t)h * h;
    ow3 = ob2 + h;
    ob3 = ow3 + h;
    n = ob3 + 1;
  }
};

// z[s][j] = b[j] + sum_i in[s][i] W[i][j]; a = relu(z)
__global__ void k_layer(const float* __restrict__ in, const int32_t* __restrict__ rows, int n, int din,
                        const float* __restrict__ W, const float* __restrict__ b, int dout, float* __restrict__ z,
                        float* __restrict__ a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * dout) return;
  const int s = (int)(i / dout), j = (int)(i % dout);
  const int64_t src = rows ? rows[s] : s;
  float acc = b[j];
  for (int k = 0; k < din; ++k) acc += in[src * din + k] * W[(int64_t)k * dout + j];
  z[i] = acc;
  a[i] = acc > 0.f ? acc : 0.f;
}

// y[s] = b3 + sum_j h2[s][j] w3[j]; dy[s] = 2 (y - t) / n
__global__ void k_out(const float* __restrict__ h2, int n, int h, const float* __restrict__ w3,
                      const float* __restrict__ b3, const float* __restrict__ t, const int32_t* __restrict__ rows,
                      float* __restrict__ y, float* __restrict__ dy) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float acc = b3[0];
  for (int j = 0; j < h; ++j) acc += h2[(int64_t)s * h + j] * w3[j];
  y[s] = acc;
  if (dy) dy[s] = 2.f * (acc - t[rows ? rows[s] : s]) / (float)n;
}

// gW[i][j] = sum_s in[s][i] d[s][j], gb[j] = sum_s d[s][j]  (s in order)
__global__ void k_wgrad(const float* __restrict__ in, const int32_t* __restrict__ rows, int n, int din,
                        const float* __restrict__ d, int dout, float* __restrict__ gW, float* __restrict__ gb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < (int64_t)din * dout) {
    const int r = (int)(i / dout), c = (int)(i % dout);
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += in[(rows ? (int64_t)rows[s] : s) * din + r] * d[(int64_t)s * dout + c];
    gW[i] = acc;
  }
  if (i < dout) {
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += d[(int64_t)s * dout + i];
    gb[i] = acc;
  }
}

// the last layer's gradients and the error at h2: dh2[s][j] = dy[s] w3[j] [z2 > 0]
__global__ void k_outgrad(const float* __restrict__ h2, const float* __restrict__ z2, const float* __restrict__ dy,
                          int n, int h, const float* __restrict__ w3, float* __restrict__ gw3,
                          float* __restrict__ gb3, float* __restrict__ dh2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < h) {
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += h2[(int64_t)s * h + i] * dy[s];
    gw3[i] = acc;
  }
  if (i == 0) {
    float acc = 0.f;
    for (int s = 0; s < n; ++s) acc += dy[s];
    gb3[0] = acc;
  }
  if (i < (int64_t)n * h) {
    const int s = (int)(i / h), j = (int)(i % h);
    dh2[i] = z2[i] > 0.f ? dy[s] * w3[j] : 0.f;
  }
}

// dprev[s][k] = (sum_j d[s][j] W[k][j]) [zprev > 0]
__global__ void k_backprop(const float* __restrict__ d, int n, int dout, const float* __restrict__ W, int din,
                           const float* __restrict__ zprev, float* __restrict__ dprev) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * din) return;
  const int s = (int)(i / din), k = (int)(i % din);
  float acc = 0.f;
  for (int j = 0; j < dout; ++j) acc += d[(int64_t)s * dout + j] * W[(int64_t)k * dout + j];
  dprev[i] = zprev[i] > 0.f ? acc : 0.f;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// squared residuals for the loss: r[s] = (y - t)^2
__global__ void k_sqerr(const float* __restrict__ y, const float* __restrict__ t, const int32_t* __restrict__ rows,
                        int n, float* __restrict__ r) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float e = y[s] - t[rows ? rows[s] : s];
  r[s] = e * e;
}

inline int blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

// sum of r[0..n) in FP64 by one workgroup, written to *out
__global__ void k_sum(const float* __restrict__ r, int n, double* __restrict__ out) {
  __shared__ double part[256];
  double a = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += (double)r[i];
  part[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

struct Work {
  float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr, *dh2 = nullptr,
        *dh1 = nullptr, *sq = nullptr;
  std::vector<void*> all;
  bool make(int n, int h) {
    auto get = [&](float*& p, int64_t cnt) {
      if (hipMalloc(&p, std::max<int64_t>(cnt, 1) * sizeof(float)) != hipSuccess) return false;
      all.push_back(p);
      return true;
    };
    return get(z1, (int64_t)n * h) && get(h1, (int64_t)n * h) && get(z2, (int64_t)n * h) &&
           get(h2, (int64_t)n * h) && get(y, n) && get(dy, n) && get(dh2, (int64_t)n * h) &&
           get(dh1, (int64_t)n * h) && get(sq, n);
  }
  ~Work() {
    for (void* p : all) (void)hipFree(p);
  }
};

// forward (and, with g != null, the gradient) of a batch given by rows
void pass(const Net& N, const float* P, const float* X, const float* t, const int32_t* rows, int n, Work& w,
          float* g, hipStream_t s) {
  const int d = N.d, h = N.h;
  hipLaunchKernelGGL(k_layer, dim3(blocks((int64_t)n * h)), dim3(256), 0, s, X, rows, n, d, P + N.oW1, P + N.ob1, h,
                     w.z1, w.h1);
  hipLaunchKernelGGL(k_layer, dim3(blocks((int64_t)n * h)), dim3(256), 0, s, w.h1, (const int32_t*)nullptr, n, h,
                     P + N.oW2, P + N.ob2, h, w.z2, w.h2);
  hipLaunchKernelGGL(k_out, dim3(blocks(n)), dim3(256), 0, s, w.h2, n, h, P + N.ow3, P + N.ob3, t, rows, w.y,
                     g ? w.dy : (float*)nullptr);
  if (!g) return;
  hipLaunchKernelGGL(k_outgrad, dim3(blocks((int64_t)n * h)), dim3(256), 0, s, w.h2, w.z2, w.dy, n, h, P + N.ow3,
                     g + N.ow3, g + N.ob3, w.dh2);
  hipLaunchKernelGGL(k_wgrad, dim3(blocks((int64_t)h * h)), dim3(256), 0, s, w.h1, (const int32_t*)nullptr, n, h,
                     w.dh2, h, g + N.oW2, g + N.ob2);
  hipLaunchKernelGGL(k_backprop, dim3(blocks((int64_t)n * h)), dim3(256), 0, s, w.dh2, n, h, P + N.oW2, h, w.z1,
                     w.dh1);
  hipLaunchKernelGGL(k_wgrad, dim3(blocks((int64_t)d * h)), dim3(256), 0, s, X, rows, n, d, w.dh1, h, g + N.oW1,
                     g + N.ob1);
}

float mean_sq(const float* y, const float* t, const int32_t* rows, int n, Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_sqerr, dim3(blocks(n)), dim3(256), 0, s, y, t, rows, n, w.sq);
  std::vector<float> h(n);
  if (hipMemcpyAsync(h.data(), w.sq, n * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess) return NAN;
  if (hipStreamSynchronize(s) != hipSuccess) return NAN;
  double acc = 0;
  for (float x : h) acc += x;
  return (float)(acc / n);
}

// Device scratch of lmfao_mlp_grad_noalloc: the batch's activations and
// back-propagated errors (6 n h floats), the outputs, their errors and squared
// errors (3 n floats) and the FP64 loss, in one file-scope array of fixed
// size that each GPU holds for the life of the process.
constexpr int64_t kMlpScratchFloats = (int64_t)2 << 20;   // 8 MiB
constexpr int64_t kMlpScratchTail = 64;                   // loss accumulator (floats)
__device__ __align__(256) float scratch[kMlpScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// the scratch array's device address on the current GPU, looked up once per
// device (the array's host-side name is not a device address)
hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace lmfao

using namespace lmfao;

extern "C" {

lmfao_status lmfao_mlp_size(int32_t d, int32_t h, int64_t* n_params) {
  if (d <= 0 || h <= 0 || !n_params) return LMFAO_EINVAL;
  *n_params = Net(d, h).n;
  return LMFAO_OK;
}

lmfao_status lmfao_mlp_grad(int32_t d, int32_t h, const float* params, const float* X, const float* t, int32_t n,
                            float* grad, float* loss, void* stream) {
  if (d <= 0 || h <= 0 || n <= 0 || !params || !X || !t || !grad) return LMFAO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Net N(d, h);
  Work w;
  if (!w.make(n, h)) return LMFAO_ENOMEM;
  pass(N, params, X, t, nullptr, n, w, grad, s);
  const float l = mean_sq(w.y, t, nullptr, n, w, s);
  if (loss) *loss = l;
  return std::isnan(l) ? LMFAO_EHIP : LMFAO_OK;
}

lmfao_status lmfao_mlp_grad_noalloc(int32_t d, int32_t h, const float* params, const float* X, const float* t,
                                    int32_t n, float* grad, float* loss, void* stream) {
  if (d <= 0 || h <= 0 || n <= 0 || !params || !X || !t || !grad) {
    record_error("lmfao_mlp_grad_noalloc: non-positive size or null pointer");
    return LMFAO_EINVAL;
  }
  const int64_t need = 6 * (int64_t)n * h + 3 * (int64_t)n + kMlpScratchTail;
  if (need > kMlpScratchFloats) {
    record_error("lmfao_mlp_grad_noalloc: a batch of " + std::to_string(n) + " rows with " + std::to_string(h) +
                 " hidden units needs " + std::to_string(need * 4) + " bytes of scratch; the fixed scratch holds " +
                 std::to_string(kMlpScratchFloats * 4) + " (6*n*h + 3*n + 64 floats at most)");
    return LMFAO_EINVAL;
  }
  float* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) {
    record_error(std::string("lmfao_mlp_grad_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    return LMFAO_EHIP;
  }
  hipStream_t s = (hipStream_t)stream;
  Net N(d, h);
  Work w;   // points into the scratch array; owns nothing
  const int64_t nh = (int64_t)n * h;
  float* q = base;
  for (float** p : {&w.z1, &w.h1, &w.z2, &w.h2, &w.dh2, &w.dh1}) {
    *p = q;
    q += nh;
  }
  for (float** p : {&w.y, &w.dy, &w.sq}) {
    *p = q;
    q += n;
  }
  double* acc = (double*)(base + kMlpScratchFloats - kMlpScratchTail);
  pass(N, params, X, t, nullptr, n, w, grad, s);
  hipLaunchKernelGGL(k_sqerr, dim3(blocks(n)), dim3(256), 0, s, w.y, t, (const int32_t*)nullptr, n, w.sq);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, w.sq, n, acc);
  double sum = 0;
  e = hipMemcpyAsync(&sum, acc, sizeof sum, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    record_error(std::string("lmfao_mlp_grad_noalloc: ") + hipGetErrorString(e));
    return LMFAO_EHIP;
  }
  if (loss) *loss = (float)(sum / n);
  return LMFAO_OK;
}

lmfao_status lmfao_mlp_predict(int32_t d, int32_t h, const float* params, const float* X, int32_t n, float* y,
                               void* stream) {
  if (d <= 0 || h <= 0 || n <= 0 || !params || !X || !y) return LMFAO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Net N(d, h);
  Work w;
  if (!w.make(n, h)) return LMFAO_ENOMEM;
  pass(N, params, X, nullptr, nullptr, n, w, nullptr, s);
  if (hipMemcpyAsync(y, w.y, n * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess) return LMFAO_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? LMFAO_OK : LMFAO_EHIP;
}

lmfao_status lmfao_mlp_train(int32_t d, int32_t h, float* params, const float* X, const float* t, int32_t n,
                             const int32_t* order, int32_t n_steps, int32_t batch, float lr, float* loss_trace,
                             void* stream) {
  if (d <= 0 || h <= 0 || n <= 0 || !params || !X || !t || !order || n_steps < 0 || batch <= 0)
    return LMFAO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // every row index is checked on the host before a kernel reads through it
  const int64_t n_idx = (int64_t)n_steps * batch;
  if (n_idx > 0) {
    std::vector<int32_t> idx(n_idx);
    if (hipMemcpyAsync(idx.data(), order, n_idx * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LMFAO_EHIP;
    for (int32_t r : idx)
      if (r < 0 || r >= n) return LMFAO_EINVAL;
  }
  Net N(d, h);
  Work w;
  if (!w.make(std::max(batch, n), h)) return LMFAO_ENOMEM;
  float *g = nullptr, *m = nullptr, *v = nullptr;
  if (hipMalloc(&g, N.n * sizeof(float)) != hipSuccess) return LMFAO_ENOMEM;
  w.all.push_back(g);
  if (hipMalloc(&m, N.n * sizeof(float)) != hipSuccess) return LMFAO_ENOMEM;
  w.all.push_back(m);
  if (hipMalloc(&v, N.n * sizeof(float)) != hipSuccess) return LMFAO_ENOMEM;
  w.all.push_back(v);
  if (hipMemsetAsync(m, 0, N.n * sizeof(float), s) != hipSuccess) return LMFAO_EHIP;
  if (hipMemsetAsync(v, 0, N.n * sizeof(float), s) != hipSuccess) return LMFAO_EHIP;
  const float b1 = 0.9f, b2 = 0.999f;
  float p1 = 1.f, p2 = 1.f;
  for (int it = 0; it < n_steps; ++it) {
    const int32_t* rows = order + (int64_t)it * batch;
    pass(N, params, X, t, rows, batch, w, g, s);
    p1 *= b1;
    p2 *= b2;
    hipLaunchKernelGGL(k_adam, dim3(blocks(N.n)), dim3(256), 0, s, params, g, m, v, N.n, lr, b1, b2, 1e-8f,
                       1.f - p1, 1.f - p2);
    if (loss_trace) loss_trace[it] = mean_sq(w.y, t, rows, batch, w, s);
  }
  return hipStreamSynchronize(s) == hipSuccess && hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_EHIP;
}

}  // extern "C"
