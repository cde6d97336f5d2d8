// Code generation of scan kernels specialised to one group's program.
//
// The paper's engine compiles the multi-output plan of every group into code
// specialised to the schema and the join tree (section 2, code generation
// layer).  This is the GPU form of that step: from a lean scan descriptor
// (one pass over the sorted relation: per-row factor columns, up to two
// inner view images, the monomials of the inner factors, code histograms,
// direct count tables) it emits HIP source whose loops over factors, masks,
// histograms and tables are unrolled into straight-line code with every
// offset, stride and mask a literal, compiles it with hipRTC for gfx950 and
// caches the function by source text for the life of the process.  The
// kernel computes exactly what the generic lean scan computes.
#include <hip/hip_runtime.h>

#include <cctype>
#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <algorithm>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "codegen.hpp"

namespace lmfao {

namespace {

constexpr int kGenWaves = 8;   // wavefronts per workgroup
constexpr int kMaxRep = 4;     // most copies of each per-piece histogram
constexpr int kRegHist = 16;   // histograms up to this many bins are kept in registers
constexpr int kTreeMin = 8;    // piece totals of this many values or more share one butterfly

struct Emit {
  std::ostringstream o;
  template <typename X>
  Emit& operator<<(const X& x) {
    o << x;
    return *this;
  }
};

std::string hex64(uint64_t v) {
  char b[32];
  snprintf(b, sizeof b, "0x%llxull", (unsigned long long)v);
  return b;
}

// value of multiplicity mask m (0..3) in the generated code
std::string mu(int m) { return "mu" + std::to_string(m); }

}  // namespace

bool gen_scan_kernel(const DScan& d, int NA, bool f64, const std::string& tag, GenKernel& out, std::string& why) {
  // kernel name: lmfao_scan_ plus the tag's letters and digits (profiles
  // tell the groups apart by it)
  std::string kname = "lmfao_scan_";
  for (char ch : tag) kname += std::isalnum((unsigned char)ch) ? ch : '_';
  const DFast& F = d.F;
  if (!d.fast) {
    why = "not a lean scan";
    return false;
  }
  const char* T = f64 ? "double" : "float";
  const int s = f64 ? 2 : 1;                       // dwords per factor slot in an image
  const int NCS = d.n_codes > 4 ? d.n_codes : 4;   // code slots of an image record and code registers
  const int code_off = NA * s, cnt_off = code_off + NCS;
  const int W = ((cnt_off + 1) + 3) & ~3;
  const int tsz = f64 ? 8 : 4;
  std::vector<uint64_t> args;
  auto arg = [&](uint64_t v) {
    args.push_back(v);
    return (int)args.size() - 1;
  };
  Emit e;
  e << "// generated scan kernel\n";
  e << "typedef " << T << " T;\n";
  // wave sums on the DPP path (no LDS traffic): prefix sums inside rows of
  // 16 lanes, then the row totals broadcast into the next rows; lane 63 holds
  // the total, which readlane hands to every lane
  e << "__device__ __forceinline__ int dppi(int v, int ctrl, int rows) {\n"
       "  switch (ctrl) {\n"
       "    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);\n"
       "    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);\n"
       "    case 4: return __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);\n"
       "    case 8: return __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);\n"
       "    case 15: return __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);\n"
       "    default: return __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);\n"
       "  }\n}\n";
  e << "__device__ __forceinline__ int wsumi(int x) {\n"
       "  x += dppi(x, 1, 0); x += dppi(x, 2, 0); x += dppi(x, 4, 0); x += dppi(x, 8, 0);\n"
       "  x += dppi(x, 15, 0); x += dppi(x, 31, 0);\n"
       "  return __builtin_amdgcn_readlane(x, 63);\n}\n";
  // inclusive prefix sum over the wave (the same DPP steps as the sum)
  e << "__device__ __forceinline__ int wscani(int x) {\n"
       "  x += dppi(x, 1, 0); x += dppi(x, 2, 0); x += dppi(x, 4, 0); x += dppi(x, 8, 0);\n"
       "  x += dppi(x, 15, 0); x += dppi(x, 31, 0);\n  return x;\n}\n";
  // Adjacent lanes adding to the same bin (sorted keys make runs) combine:
  // the last lane of each run adds the run's total, taken as a difference of
  // the exact integer prefix sums.  Returns the amount this lane must add.
  e << "__device__ __forceinline__ int run_total(int bin, int m, int lane) {\n"
       "  const int P = wscani(m);\n"
       "  const int prev = __builtin_amdgcn_update_dpp(-1, bin, 0x138, 0xf, 0xf, false);\n"
       "  const unsigned long long H = __ballot(lane == 0 || prev != bin);\n"
       "  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);\n"
       "  const int start = 63 - __clzll(H & upto);\n"
       "  const int before = __shfl(P, start > 0 ? start - 1 : 0, 64);\n"
       "  const bool tail = lane == 63 || ((H >> (lane + 1)) & 1ull);\n"
       "  return tail ? P - (start > 0 ? before : 0) : 0;\n}\n";
  // the same for FP64 values: a scan segmented at the run starts, so the last
  // lane of a run holds the run's sum (no difference of prefix sums)
  e << "__device__ __forceinline__ double run_total_d(int bin, double x, int lane) {\n"
       "  const int prev = __builtin_amdgcn_update_dpp(-1, bin, 0x138, 0xf, 0xf, false);\n"
       "  const unsigned long long H = __ballot(lane == 0 || prev != bin);\n"
       "  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);\n"
       "  const int start = 63 - __clzll(H & upto);\n"
       "  double P = x;\n"
       "  for (int o = 1; o < 64; o <<= 1) {\n"
       "    const double y = __shfl_up(P, o, 64);\n"
       "    if (lane - o >= start) P += y;\n  }\n"
       "  const bool tail = lane == 63 || ((H >> (lane + 1)) & 1ull);\n"
       "  return tail ? P : 0.0;\n}\n";
  if (f64) {
    e << "__device__ __forceinline__ T wsum(T x) {\n"
         "  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);\n  return x;\n}\n";
  } else {
    e << "__device__ __forceinline__ float wsum(float x) {\n"
         "  x += __int_as_float(dppi(__float_as_int(x), 1, 0)); x += __int_as_float(dppi(__float_as_int(x), 2, 0));\n"
         "  x += __int_as_float(dppi(__float_as_int(x), 4, 0)); x += __int_as_float(dppi(__float_as_int(x), 8, 0));\n"
         "  x += __int_as_float(dppi(__float_as_int(x), 15, 0)); x += __int_as_float(dppi(__float_as_int(x), 31, 0));\n"
         "  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));\n}\n";
  }
  if (f64) {
    // TwoSum butterfly: every combining add is error-free transformed
    e << "__device__ __forceinline__ double wsumc(double s) {\n"
         "  double c = 0.0;\n"
         "  for (int o = 32; o > 0; o >>= 1) {\n"
         "    double s2 = __shfl_xor(s, o, 64), c2 = __shfl_xor(c, o, 64);\n"
         "    double t = s + s2, bb = t - s, er = (s - (t - bb)) + (s2 - bb);\n"
         "    s = t; c = c + c2 + er;\n  }\n  return s + c;\n}\n";
  } else {
    e << "__device__ __forceinline__ float wsumc(float s) { return wsum(s); }\n";
  }
  e << "extern \"C\" __global__ __launch_bounds__(" << kGenWaves * 64
    << ") void " << kname << "(const unsigned long long* __restrict__ A) {\n";
  e << "  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];\n";
  e << "  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;\n";
  // arguments
  e << "  const long long* __restrict__ piece_begin = (const long long*)A[" << arg((uint64_t)d.piece_begin) << "];\n";
  e << "  const int* __restrict__ item_piece = (const int*)A[" << arg((uint64_t)d.item_piece) << "];\n";
  e << "  const int n_items = (int)A[" << arg((uint64_t)d.n_items) << "];\n";
  e << "  T* __restrict__ psi_f = (T*)A[" << arg((uint64_t)d.psi_f) << "];\n";
  e << "  int* __restrict__ psi_i = (int*)A[" << arg((uint64_t)d.psi_i) << "];\n";
  std::vector<int> fcol_arg(NA, -1);
  for (int a = 0; a < NA; ++a)
    if (F.fcol[a]) {
      fcol_arg[a] = arg((uint64_t)F.fcol[a]);
      e << "  const T* __restrict__ fc" << a << " = (const T*)A[" << fcol_arg[a] << "];\n";
    }
  for (int c = 0; c < NCS; ++c)
    if (F.ccol[c]) e << "  const int* __restrict__ cc" << c << " = (const int*)A[" << arg((uint64_t)F.ccol[c]) << "];\n";
  for (int v = 0; v < 2; ++v) {
    if (!F.img[v]) continue;
    e << "  const uint4* __restrict__ img" << v << " = (const uint4*)A[" << arg((uint64_t)F.img[v]) << "];\n";
    for (int k = 0; k < 2; ++k)
      if (F.kcol[v][k])
        e << "  const int* __restrict__ kc" << v << k << " = (const int*)A[" << arg((uint64_t)F.kcol[v][k]) << "];\n";
  }
  if (d.w) e << "  const int* __restrict__ wf = (const int*)A[" << arg((uint64_t)d.w) << "];\n";
  const bool has_mu_out = d.mu_out_views > 0;
  if (has_mu_out) {
    e << "  const int* __restrict__ pkey = (const int*)A[" << arg((uint64_t)d.piece_key) << "];\n";
    for (int v = 0; v < d.mu_out_views; ++v)
      e << "  const long long* __restrict__ ov" << v << " = (const long long*)A["
        << arg((uint64_t)d.outer_views[v].cnt) << "];\n";
  }
  bool any_global_tab = false;
  for (int t = 0; t < F.n_tab; ++t)
    if (F.tab_nvc[t] > 0)
      e << "  double* __restrict__ tv" << t << " = (double*)A[" << arg((uint64_t)F.tab_vals[t]) << "];\n";
  for (int t = 0; t < F.n_tab; ++t)
    if (!F.tab_lds[t]) {
      any_global_tab = true;
      e << "  unsigned long long* __restrict__ tab" << t << " = (unsigned long long*)A[" << arg((uint64_t)F.tab_cnt[t])
        << "];\n";
    }
  (void)any_global_tab;
  if (d.lds_tab_i > 0) e << "  int* __restrict__ part_i = (int*)A[" << arg((uint64_t)d.part_i) << "];\n";

  // LDS: count tables (block), then a histogram area per wavefront.  Each
  // histogram is kept in kRep copies, lane & (kRep-1) choosing the copy, so
  // that lanes adding to the same bin mostly meet in different copies; the
  // copies are summed when the piece closes.  Up to kMaxRep copies while the
  // block fits in 64 KB, fewer for large histograms; large direct tables in
  // LDS take the block up to the whole LDS of a CU.
  const int hib = d.hist_i_bins, hfb = d.hist_f_bins;
  const int tab_bytes = (d.lds_tab_i * 4 + 15) & ~15;
  auto lds_for = [&](int rep) {
    const int hb = ((rep * hib * 4 + 7) & ~7) + rep * hfb * tsz;
    return tab_bytes + kGenWaves * ((hb + 15) & ~15);
  };
  int kRep = kMaxRep;
  while (kRep > 1 && lds_for(kRep) > 65536) kRep /= 2;
  const int hist_i_bytes = (kRep * hib * 4 + 7) & ~7;
  const int hist_bytes = hist_i_bytes + kRep * hfb * tsz;
  const int wave_stride = (hist_bytes + 15) & ~15;
  const int lds = tab_bytes + kGenWaves * wave_stride;
  if (lds > 160 * 1024) {
    why = "generated scan would need more LDS than a CU has";
    return false;
  }
  e << "  int* tab_i = (int*)smem;\n";
  e << "  int* hist_i = (int*)(smem + " << tab_bytes << " + wid * " << wave_stride << ");\n";
  e << "  T* hist_f = (T*)((unsigned char*)hist_i + " << hist_i_bytes << ");\n";
  if (d.lds_tab_i > 0) {
    e << "  for (int i = threadIdx.x; i < " << d.lds_tab_i << "; i += " << kGenWaves * 64 << ") tab_i[i] = 0;\n";
  }
  e << "  __syncthreads();\n";

  // row loader: factor columns, code columns, image keys, filter weight
  auto emit_load = [&](const char* pre, const char* row) {
    for (int a = 0; a < NA; ++a)
      if (F.fcol[a]) e << "      " << pre << "f" << a << " = fc" << a << "[" << row << "];\n";
    for (int c = 0; c < NCS; ++c)
      if (F.ccol[c]) e << "      " << pre << "c" << c << " = cc" << c << "[" << row << "];\n";
    for (int v = 0; v < 2; ++v) {
      if (!F.img[v]) continue;
      e << "      " << pre << "k" << v << " = kc" << v << "0[" << row << "] * " << F.kmul[v][0];
      if (F.kcol[v][1]) e << " + kc" << v << "1[" << row << "] * " << F.kmul[v][1];
      e << ";\n";
    }
    if (d.w) e << "      " << pre << "w = wf[" << row << "];\n";
  };
  auto emit_decl = [&](const char* pre) {
    for (int a = 0; a < NA; ++a)
      if (F.fcol[a]) e << "      T " << pre << "f" << a << ";\n";
    for (int c = 0; c < NCS; ++c)
      if (F.ccol[c]) e << "      int " << pre << "c" << c << ";\n";
    for (int v = 0; v < 2; ++v)
      if (F.img[v]) e << "      int " << pre << "k" << v << ";\n";
    if (d.w) e << "      int " << pre << "w;\n";
  };

  // needed monomials: triangle index t(i, j) over the extended factors (0 = 1)
  auto tri = [&](int i, int j) { return i * (NA + 1) - i * (i - 1) / 2 + (j - i); };
  std::vector<std::pair<int, int>> terms;   // (i, j) of each needed entry, in triangle order
  for (int i = 0; i <= NA; ++i)
    for (int j = i; j <= NA; ++j) {
      const int t = tri(i, j);
      if (t > 0 && ((d.pf_need >> t) & 1ull)) terms.push_back({i, j});
    }
  const int n_masks = d.n_masks;

  e << "  for (int item = blockIdx.x * " << kGenWaves << " + wid; item < n_items; item += gridDim.x * " << kGenWaves
    << ") {\n";
  e << "    const int p0 = item_piece[item], p1 = item_piece[item + 1];\n";
  e << "    for (int p = p0; p < p1; ++p) {\n";
  e << "      const int rb = (int)piece_begin[p], re = (int)piece_begin[p + 1];\n";
  if (has_mu_out) {
    e << "      int mu_out = 1;\n";
    for (int v = 0; v < d.mu_out_views; ++v) {
      const DView& V = d.outer_views[v];
      e << "      { long long vr = 0;\n";
      for (int k = 0; k < V.nkey; ++k)
        e << "        vr += (long long)pkey[" << (int64_t)V.key_src[k] * d.n_pieces << "ll + p] * " << V.key_stride[k]
          << "ll;\n";
      e << "        mu_out *= (int)ov" << v << "[vr]; }\n";
    }
  }
  if (hib > 0) e << "      for (int i = lane; i < " << kRep * hib << "; i += 64) hist_i[i] = 0;\n";
  if (hfb > 0) e << "      for (int i = lane; i < " << kRep * hfb << "; i += 64) hist_f[i] = (T)0;\n";
  if (hib > 0 || hfb > 0) {
    e << "      const int rep_i = (lane & " << kRep - 1 << ") * " << hib << ";\n";
    e << "      const int rep_f = (lane & " << kRep - 1 << ") * " << hfb << ";\n";
  }
  e << "      __builtin_amdgcn_wave_barrier();\n";
  for (size_t k = 0; k < terms.size(); ++k) e << "      T acc" << k << " = (T)0;\n";
  // small histograms: a private counter per lane and bin, summed over the
  // wavefront when the piece closes (no LDS atomics on skewed codes)
  auto reg_hist = [&](int h) { return d.hists[h].dom <= std::min(kRegHist, (int)F.reg_hist_bins); };
  // integer register histograms with multiplicities 0 or 1: the bins are
  // 8-bit fields of one or two 64-bit words (a row adds its multiplicity
  // shifted to its code's field; a lane adds at most 128 rows of a piece),
  // unpacked into the per-bin counts when the piece closes
  auto packed = [&](int h) { return F.mult01 && reg_hist(h) && !((F.hword[h] >> 4) & 1u); };
  for (int h = 0; h < F.n_hist; ++h) {
    if (!reg_hist(h)) continue;
    const bool fl = (F.hword[h] >> 4) & 1u;
    if (packed(h)) {
      for (int wi = 0; wi * 8 < d.hists[h].dom; ++wi) e << "      unsigned long long pk" << h << "_" << wi << " = 0ull;\n";
      continue;
    }
    for (int b = 0; b < d.hists[h].dom; ++b)
      e << "      " << (fl ? "T" : "int") << " rh" << h << "_" << b << " = " << (fl ? "(T)0" : "0") << ";\n";
  }
  for (int k = 0; k < d.n_pi; ++k) e << "      int cnt" << k << " = 0;\n";
  emit_decl("n");
  e << "      {\n        const int r = rb + lane < re ? rb + lane : rb;\n";
  emit_load("n", "r");
  e << "      }\n";
  e << "      for (int r0 = rb; r0 < re; r0 += 64) {\n";
  e << "        const int r = r0 + lane;\n        const bool valid = r < re;\n";
  // current row values = prefetched ones
  for (int a = 0; a < NA; ++a)
    if (F.fcol[a]) e << "        const T cf" << a << " = nf" << a << ";\n";
  for (int c = 0; c < NCS; ++c)
    if (F.ccol[c]) e << "        const int cc_" << c << " = nc" << c << ";\n";
  for (int v = 0; v < 2; ++v)
    if (F.img[v]) e << "        const int ck" << v << " = nk" << v << ";\n";
  if (d.w) e << "        const int cw = nw;\n";
  e << "        if (r0 + 64 < re) {\n          const int rn = r + 64 < re ? r + 64 : rb;\n";
  emit_load("  n", "rn");
  e << "        }\n";
  // factor values: a0 = 1, column part + image parts
  e << "        const T a0 = (T)1;\n";
  for (int a = 0; a < NA; ++a) e << "        T a" << a + 1 << " = " << (F.fcol[a] ? "cf" + std::to_string(a) : "(T)0") << ";\n";
  for (int c = 0; c < NCS; ++c)
    e << "        int c" << c << " = " << (F.ccol[c] ? "cc_" + std::to_string(c) : "0") << ";\n";
  e << "        const int wv = valid ? " << (d.w ? "cw" : "1") << " : 0;\n";
  for (int m = 0; m < 4; ++m) e << "        int " << mu(m) << " = wv;\n";
  for (int v = 0; v < 2; ++v) {
    if (!F.img[v]) continue;
    e << "        {\n          const uint4* q = img" << v << " + (long long)ck" << v << " * " << W / 4 << ";\n";
    for (int j = 0; j < W / 4; ++j) e << "          const uint4 x" << j << " = q[" << j << "];\n";
    auto dw = [&](int i) {
      static const char* comp[] = {"x", "y", "z", "w"};
      return "x" + std::to_string(i / 4) + "." + comp[i % 4];
    };
    for (int a = 0; a < NA; ++a) {
      if (f64)
        e << "          a" << a + 1 << " += __longlong_as_double((long long)(((unsigned long long)" << dw(2 * a + 1)
          << " << 32) | " << dw(2 * a) << "));\n";
      else
        e << "          a" << a + 1 << " += __uint_as_float(" << dw(a) << ");\n";
    }
    for (int c = 0; c < NCS; ++c) e << "          c" << c << " += (int)" << dw(code_off + c) << ";\n";
    e << "          const int vc = valid ? (int)" << dw(cnt_off) << " : 0;\n";
    for (int m = 0; m < n_masks; ++m)
      if (d.masks[m] & (1u << v)) e << "          " << mu(m) << " *= vc;\n";
    e << "        }\n";
  }
  // monomials (one multiplicity mask for all of them)
  if (!terms.empty()) {
    e << "        const T mt = (T)" << mu(d.pf_mask_idx) << ";\n";
    std::vector<char> xi(NA + 1, 0);
    for (auto& ij : terms) xi[ij.first] = 1;
    for (int i = 0; i <= NA; ++i)
      if (xi[i]) e << "        const T x" << i << " = mt * a" << i << ";\n";
    for (size_t k = 0; k < terms.size(); ++k)
      e << "        acc" << k << " += x" << terms[k].first << " * a" << terms[k].second << ";\n";
  }
  for (int k = 0; k < d.n_pi; ++k) e << "        cnt" << k << " += " << mu(d.pi_mask_idx[k]) << ";\n";
  // histograms
  for (int h = 0; h < F.n_hist; ++h) {
    const uint32_t w = F.hword[h];
    const int code = F.hcode[h], m = (int)((w >> 2) & 3u), off = (int)(w >> 13);
    if (reg_hist(h)) {
      if ((w >> 4) & 1u) {
        const int ai = (int)((w >> 5) & 15u), aj = (int)((w >> 9) & 15u);
        e << "        { const T hv = (T)" << mu(m) << " * a" << ai << " * a" << aj << ";";
        for (int b = 0; b < d.hists[h].dom; ++b)
          e << " rh" << h << "_" << b << " += c" << code << " == " << b << " ? hv : (T)0;";
        e << " }\n";
      } else if (packed(h)) {
        const int dom = d.hists[h].dom;
        // the multiplicity is selected (0 for a code outside the word) before
        // the shift, whose count is kept below 64
        e << "        { const unsigned hv = (unsigned)" << mu(m) << "; const unsigned cu = (unsigned)c" << code << ";";
        for (int wi = 0; wi * 8 < dom; ++wi) {
          const int lo = wi * 8, n = std::min(8, dom - lo);
          e << " { const unsigned cw = cu - " << lo << "u; pk" << h << "_" << wi
            << " += (unsigned long long)(cw < " << n << "u ? hv : 0u) << ((cw & 7u) * 8u); }";
        }
        e << " }\n";
      } else {
        e << "        { const int hv = " << mu(m) << ";";
        for (int b = 0; b < d.hists[h].dom; ++b)
          e << " rh" << h << "_" << b << " += c" << code << " == " << b << " ? hv : 0;";
        e << " }\n";
      }
      continue;
    }
    if ((w >> 4) & 1u) {
      const int ai = (int)((w >> 5) & 15u), aj = (int)((w >> 9) & 15u);
      e << "        if (" << mu(m) << ") atomicAdd(&hist_f[rep_f + " << off << " + c" << code << "], (T)" << mu(m)
        << " * a" << ai << " * a" << aj << ");\n";
    } else {
      e << "        { const int rt = run_total(c" << code << ", " << mu(m) << ", lane);\n"
        << "          if (rt) atomicAdd(&hist_i[rep_i + " << off << " + c" << code << "], rt); }\n";
    }
  }
  // direct count tables
  for (int t = 0; t < F.n_tab; ++t) {
    e << "        {\n          const int row = 0";
    for (int k = 0; k < F.tab_ncode[t]; ++k) e << " + c" << F.tab_code[t][k] << " * " << F.tab_stride[t][k];
    e << ";\n";
    if (F.tab_has_cnt[t]) {
      e << "          const int m = run_total(row, " << (has_mu_out ? "mu_out * " : "") << mu(F.tab_mask[t])
        << ", lane);\n";
      if (F.tab_lds[t])
        e << "          if (m) atomicAdd(&tab_i[" << F.tab_off[t] << " + row], m);\n";
      else
        e << "          if (m) atomicAdd(&tab" << t << "[row], (unsigned long long)(long long)m);\n";
    }
    // value components: multiplicity times their factors, summed over each
    // run of equal rows in FP64, one atomic per run
    for (int k = 0; k < F.tab_nvc[t]; ++k) {
      const int w = F.tab_vw[t][k];
      e << "          { const double vs = run_total_d(row, (double)((T)(" << (has_mu_out ? "mu_out * " : "")
        << mu((w >> 8) & 3) << ") * a" << (w & 15) << " * a" << ((w >> 4) & 15) << "), lane);\n"
        << "            if (vs != 0.0) atomicAdd(&tv" << t << "[(long long)row * " << F.tab_nv[t] << " + "
        << F.tab_vcomp[t][k] << "], vs); }\n";
    }
    e << "        }\n";
  }
  e << "      }\n";
  // close the piece (packed histograms unpacked into their bins first)
  for (int h = 0; h < F.n_hist; ++h) {
    if (!packed(h)) continue;
    for (int b = 0; b < d.hists[h].dom; ++b)
      e << "      const int rh" << h << "_" << b << " = (int)((pk" << h << "_" << b / 8 << " >> " << 8 * (b % 8)
        << ") & 0xffull);\n";
  }
  e << "      T* prow = psi_f + (long long)p * " << d.psi_f_stride << ";\n";
  e << "      int* irow = psi_i + (long long)p * " << d.psi_i_stride << ";\n";
  // The piece's wavefront totals, each value placed at its destination index
  // v: floats at prow[v] (v < pf_n) or, for register histograms, the first
  // LDS copy at hist_f[v - pf_n]; integers at irow[v] (v < n_pi) or
  // hist_i[v - n_pi] (the LDS bins of register histograms are zero).
  std::vector<std::string> fv((size_t)d.pf_n + hfb), iv((size_t)d.n_pi + hib);
  for (size_t k = 0; k < terms.size(); ++k) fv[d.pf_slot[tri(terms[k].first, terms[k].second)]] = "acc" + std::to_string(k);
  for (int k = 0; k < d.n_pi; ++k) iv[k] = "cnt" + std::to_string(k);
  for (int h = 0; h < F.n_hist; ++h) {
    if (!reg_hist(h)) continue;
    const uint32_t w = F.hword[h];
    const bool fl = (w >> 4) & 1u;
    const int off = (int)(w >> 13);
    for (int b = 0; b < d.hists[h].dom; ++b)
      (fl ? fv[(size_t)d.pf_n + off + b] : iv[(size_t)d.n_pi + off + b]) =
          "rh" + std::to_string(h) + "_" + std::to_string(b);
  }
  // Many values: a transposed butterfly over each block of 64.  At the step
  // with lane mask m every lane pairs values (2i, 2i+1), keeps the one its
  // lane bit selects, sends the other to lane ^ m and adds what it receives;
  // after six steps lane L holds the wavefront total of value
  // bitreverse6(L).  About 4 operations per value in all, against 13 for a
  // separate reduction per value.  FP64 plans keep the compensated
  // reduction per value.
  // A block whose present values are too sparse for the butterfly to pay
  // (about 4 operations per pair it combines, against 13 per separate
  // reduction) reduces them one by one.
  auto close_values = [&](const std::vector<std::string>& vals, const char* ty, const std::string& nm,
                          const std::string& dst_lo, int n_lo, const std::string& dst_hi, bool tree_ok,
                          const char* sumfn) {
    auto one_by_one = [&](size_t lo, size_t hi) {
      for (size_t v = lo; v < hi; ++v) {
        if (vals[v].empty()) continue;
        e << "      { const " << ty << " sm = " << sumfn << "(" << vals[v] << "); if (lane == 0) ";
        if ((int)v < n_lo) e << dst_lo << "[" << v << "] = sm; }\n";
        else e << dst_hi << "[" << v - n_lo << "] = sm; }\n";
      }
    };
    std::vector<size_t> tree_blocks;
    for (size_t base = 0; base < vals.size(); base += 64) {
      size_t nb = 0;
      int present = 0;
      for (size_t v = 0; v < 64 && base + v < vals.size(); ++v)
        if (!vals[base + v].empty()) {
          nb = v + 1;
          ++present;
        }
      int pairs = 0;   // pairs combined over the six steps
      for (size_t n = nb, st = 0; st < 6; ++st) {
        n = (n + 1) / 2;
        pairs += (int)n;
      }
      if (tree_ok && present >= kTreeMin && 13 * present >= 4 * pairs) tree_blocks.push_back(base);
    }
    if (!tree_blocks.empty()) {
      e << "      {\n        const int bv = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);\n";
      for (int st = 0; st < 6; ++st)
        e << "        const bool " << nm << "b" << st << " = (lane & " << (32 >> st) << ") != 0;\n";
      for (size_t base : tree_blocks) {
        const size_t nb = std::min<size_t>(64, vals.size() - base);
        uint64_t mask = 0;
        std::vector<std::string> cur;
        size_t last = 0;
        for (size_t v = 0; v < nb; ++v)
          if (!vals[base + v].empty()) last = v + 1;
        for (size_t v = 0; v < last; ++v) {
          if (!vals[base + v].empty()) mask |= 1ull << v;
          cur.push_back(vals[base + v].empty() ? std::string("(") + ty + ")0" : vals[base + v]);
        }
        const std::string pre = nm + std::to_string(base / 64) + "_";
        for (int st = 0; st < 6; ++st) {
          const int m = 32 >> st;
          const std::string bit = nm + "b" + std::to_string(st);
          std::vector<std::string> nxt;
          for (size_t i = 0; 2 * i < cur.size(); ++i) {
            const std::string x = cur[2 * i],
                              y = 2 * i + 1 < cur.size() ? cur[2 * i + 1] : std::string("(") + ty + ")0";
            const std::string out = pre + std::to_string(st) + "_" + std::to_string(i);
            e << "        const " << ty << " " << out << " = (" << bit << " ? " << y << " : " << x
              << ") + __shfl_xor(" << bit << " ? " << x << " : " << y << ", " << m << ", 64);\n";
            nxt.push_back(out);
          }
          cur = nxt;
        }
        e << "        if ((" << mask << "ull >> bv) & 1ull) {\n"
          << "          const int v = " << base << " + bv;\n"
          << "          if (v < " << n_lo << ") " << dst_lo << "[v] = " << cur[0] << ";\n"
          << "          else " << dst_hi << "[v - " << n_lo << "] = " << cur[0] << ";\n"
          << "        }\n";
      }
      e << "      }\n";
    }
    for (size_t base = 0; base < vals.size(); base += 64) {
      if (std::find(tree_blocks.begin(), tree_blocks.end(), base) != tree_blocks.end()) continue;
      one_by_one(base, std::min<size_t>(vals.size(), base + 64));
    }
  };
  // The butterfly's exchanges go through the LDS crossbar: a scan that also
  // keeps histograms in LDS (atomics per row) measured slower with it, so
  // there every value keeps its own reduction.
  bool lds_hists = false;
  for (int h = 0; h < F.n_hist; ++h) lds_hists = lds_hists || !reg_hist(h);
  close_values(fv, "T", "bf", "prow", d.pf_n, "hist_f", !f64 && !lds_hists, "wsumc");
  close_values(iv, "int", "bi", "irow", d.n_pi, "hist_i", !lds_hists, "wsumi");
  e << "      __builtin_amdgcn_wave_barrier();\n      __builtin_amdgcn_fence(__ATOMIC_RELEASE, \"wavefront\");\n";
  if (hib > 0) {
    e << "      for (int i = lane; i < " << hib << "; i += 64) irow[" << d.n_pi << " + i] = hist_i[i]";
    for (int r = 1; r < kRep; ++r) e << " + hist_i[" << r * hib << " + i]";
    e << ";\n";
  }
  if (hfb > 0) {
    e << "      for (int i = lane; i < " << hfb << "; i += 64) prow[" << d.pf_n << " + i] = hist_f[i]";
    for (int r = 1; r < kRep; ++r) e << " + hist_f[" << r * hfb << " + i]";
    e << ";\n";
  }
  e << "      __builtin_amdgcn_wave_barrier();\n";
  e << "    }\n  }\n";
  if (d.lds_tab_i > 0) {
    e << "  __syncthreads();\n";
    e << "  for (int i = threadIdx.x; i < " << d.lds_tab_i << "; i += " << kGenWaves * 64 << ") part_i[(long long)blockIdx.x * "
      << d.lds_tab_i << " + i] = tab_i[i];\n";
  }
  e << "}\n";

  std::string src = e.o.str();
  // the source holds no pointer values (they travel as arguments), so equal
  // programs share one compiled function
  static std::mutex mtx;
  static std::map<std::string, hipFunction_t> cache;
  std::lock_guard<std::mutex> lock(mtx);
  auto it = cache.find(src);
  if (it == cache.end()) {
    hipFunction_t fn = nullptr;
    if (!compile_kernel(src, kname.c_str(), fn, why)) return false;
    it = cache.emplace(src, fn).first;
  }
  out.fn = it->second;
  out.args = args;
  out.lds = lds;
  out.block = kGenWaves * 64;
  out.source = src;
  return true;
}

bool compile_kernel(const std::string& src, const char* name, hipFunction_t& fn, std::string& why) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "lmfao_gen.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    why = "hiprtcCreateProgram failed";
    return false;
  }
  // packed FP32 instructions stay off, as in the library's own kernels
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-munsafe-fp-atomics", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    why = std::string("hipRTC compile failed: ") + hiprtcGetErrorString(r) + "\n" + log;
    hiprtcDestroyProgram(&prog);
    return false;
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  std::vector<char> code(n);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  hipModule_t mod;
  if (hipModuleLoadData(&mod, code.data()) != hipSuccess) {
    why = "hipModuleLoadData failed";
    return false;
  }
  if (hipModuleGetFunction(&fn, mod, name) != hipSuccess) {
    why = "hipModuleGetFunction failed";
    return false;
  }
  return true;
}

}  // namespace lmfao
