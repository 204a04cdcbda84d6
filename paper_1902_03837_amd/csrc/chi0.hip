// chi0_GG'(q, i w) as a weighted Hermitian rank-K update on MFMA (Eq. X_IP with
// the App. A split: frequency-free outer products rho_t rho_t^H, one real
// frequency factor per transition).
//
//   chi0[w][G][G'] = -pref sum_t W_t(w) rho_t(G) conj(rho_t(G')),
//   W_t(w) = 2 D_t / (w^2 + D_t^2).
//
// Real form. With K' = 2K real columns (t, a), a in {re, im}:
//   Re chi0 ~ sum_{t,a} [W rho_a(G)]                     rho_a(G')
//   Im chi0 ~ sum_{t,a} [W (a = re ? rho_im : -rho_re)(G)] rho_a(G')
// so both share the unweighted right operand B[(t,a)][G'] = rho_a(G', t), and the
// left operand carries the weight of each frequency. One workgroup owns one
// 16 x 16 block (G-block i <= G'-block j) for a group of frequencies; its four
// waves each reduce a disjoint slice of the transitions, and a second kernel
// adds the slices in a fixed order (deterministic), applies -pref and writes the
// block and its Hermitian mirror.
//
// Operand/result layout of the 16x16 MFMA tiles (v_mfma_*_16x16x4, one block):
//   A[i][k]: lane = i + 16 k,  B[k][j]: lane = j + 16 k.
//   Result register r of a lane: f32 and bf16 forms D[4 (lane/16) + r][lane%16];
//   the f64 form D[lane/16 + 4 r][lane%16] (checked on the device).
// bf16 variant (v_mfma_f32_16x16x32_bf16): lane = i + 16 q holds k = 8 q .. 8 q + 7.

#include <algorithm>
#include <type_traits>
#include <vector>

#include "bf16x3.h"
#include "xo_common.h"

namespace xo {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;
constexpr int kWaves = 4;

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef d4 type;
  // row of result register r in lane group kk (lane / 16)
  static __device__ __forceinline__ int row(int kk, int r) { return kk + 4 * r; }
};
template <>
struct Acc<float> {
  typedef f4 type;
  static __device__ __forceinline__ int row(int kk, int r) { return 4 * kk + r; }
};

// Per-transition frequency factors W[t][j] = 2 D_t / (w_j^2 + D_t^2); counts bad D.
template <typename T>
__global__ void pole_factors(const double* __restrict__ dE, int nt, const double* __restrict__ w, int nw,
                             int nwpad, T* __restrict__ W, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double d = dE[t];
  if (!(d > 0.0) && bad) atomicAdd(bad, 1);
  for (int j = 0; j < nwpad; ++j) {
    double v = 0.0;
    if (j < nw) v = 2.0 * d / (w[j] * w[j] + d * d);
    W[(size_t)t * nwpad + j] = (T)v;
  }
}

struct TileArgs {
  const void* rho;     // [nt][ng] complex T
  const void* W;       // [nt][nwpad] T
  int nwpad, w0;       // frequency stride and first frequency of this group
  int ng, nt;
  const int2* tiles;   // (block i, block j), i <= j
  int ntiles;
  int kper;            // transitions per wave slice
  void* part;          // [slice][tile][NWG][2][256] T
};

// FP64 / FP32: one 16x16x4 MFMA per (frequency, re/im row) and pair of transitions.
template <typename T, int NWG>
__global__ void __launch_bounds__(256) chi0_tiles(TileArgs A) {
  typedef typename Acc<T>::type V4;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x;
  const int slice = blockIdx.y * kWaves + wave;
  const int2 bij = A.tiles[tile];
  const int i = lane & 15;
  const int kk = lane >> 4;
  const int a = kk & 1;
  const int tsub = kk >> 1;
  const int Gi = bij.x * kTile + i;
  const int Gj = bij.y * kTile + i;
  const cplx<T>* rho = static_cast<const cplx<T>*>(A.rho);
  const T* W = static_cast<const T*>(A.W) + A.w0;
  V4 acc[NWG][2];
#pragma unroll
  for (int w = 0; w < NWG; ++w) {
    acc[w][0] = V4{0, 0, 0, 0};
    acc[w][1] = V4{0, 0, 0, 0};
  }
  const int t_begin = slice * A.kper;
  const int t_end = min(A.nt, t_begin + A.kper);
  const bool gi_ok = Gi < A.ng, gj_ok = Gj < A.ng;
  for (int s = t_begin; s < t_end; s += 2) {
    const int t = s + tsub;
    const bool tv = t < t_end;
    cplx<T> ra = {T(0), T(0)}, rb = {T(0), T(0)};
    if (tv && gi_ok) ra = rho[(size_t)t * A.ng + Gi];
    if (tv && gj_ok) rb = rho[(size_t)t * A.ng + Gj];
    const T bval = a ? rb.y : rb.x;
    const T are = a ? ra.y : ra.x;
    const T aim = a ? -ra.x : ra.y;
#pragma unroll
    for (int w = 0; w < NWG; ++w) {
      const T wt = tv ? W[(size_t)t * A.nwpad + w] : T(0);
      acc[w][0] = mfma4(wt * are, bval, acc[w][0]);
      acc[w][1] = mfma4(wt * aim, bval, acc[w][1]);
    }
  }
  T* out = static_cast<T*>(A.part) + ((size_t)slice * A.ntiles + tile) * NWG * 2 * 256;
#pragma unroll
  for (int w = 0; w < NWG; ++w)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(w * 2 + r) * 256 + Acc<T>::row(kk, e) * 16 + i] = acc[w][r][e];
}

// BF16 x 3 (split-bf16 products, FP32 accumulation): 16 transitions (32 real
// columns) per MFMA step. The weighted left operand of the Re row is split once
// per frequency; the Im row's operand (w rho_im, -w rho_re) is the same bits
// with the halves swapped and one sign flipped.
template <int NWG>
__global__ void __launch_bounds__(256) chi0_tiles_bf16x3(TileArgs A) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x;
  const int slice = blockIdx.y * kWaves + wave;
  const int2 bij = A.tiles[tile];
  const int i = lane & 15;
  const int q = lane >> 4;  // this lane holds k = 8q .. 8q+7 -> transitions 4q .. 4q+3, (re, im)
  const int Gi = bij.x * kTile + i;
  const int Gj = bij.y * kTile + i;
  const cplx<float>* rho = static_cast<const cplx<float>*>(A.rho);
  const float* W = static_cast<const float*>(A.W) + A.w0;
  f4 acc[NWG][2];
#pragma unroll
  for (int w = 0; w < NWG; ++w) {
    acc[w][0] = f4{0, 0, 0, 0};
    acc[w][1] = f4{0, 0, 0, 0};
  }
  const int t_begin = slice * A.kper;
  const int t_end = min(A.nt, t_begin + A.kper);
  const bool gi_ok = Gi < A.ng, gj_ok = Gj < A.ng;
  for (int s = t_begin; s < t_end; s += 16) {
    cplx<float> ra[4];
    float wt[4][NWG];
    uint32_t bhh[4], bll[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = s + 4 * q + u;
      const bool tv = t < t_end;
      ra[u] = (tv && gi_ok) ? rho[(size_t)t * A.ng + Gi] : cplx<float>{0.f, 0.f};
      const cplx<float> rb = (tv && gj_ok) ? rho[(size_t)t * A.ng + Gj] : cplx<float>{0.f, 0.f};
      split2(rb.x, rb.y, bhh[u], bll[u]);
#pragma unroll
      for (int w = 0; w < NWG; ++w) wt[u][w] = tv ? W[(size_t)t * A.nwpad + w] : 0.f;
    }
    const u4 bh = u4{bhh[0], bhh[1], bhh[2], bhh[3]}, bl = u4{bll[0], bll[1], bll[2], bll[3]};
#pragma unroll
    for (int w = 0; w < NWG; ++w) {
      uint32_t h[4], l[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) split2(wt[u][w] * ra[u].x, wt[u][w] * ra[u].y, h[u], l[u]);
      const u4 reh = u4{h[0], h[1], h[2], h[3]}, rel = u4{l[0], l[1], l[2], l[3]};
      const u4 imh = u4{rot_pos(h[0]), rot_pos(h[1]), rot_pos(h[2]), rot_pos(h[3])};
      const u4 iml = u4{rot_pos(l[0]), rot_pos(l[1]), rot_pos(l[2]), rot_pos(l[3])};
      acc[w][0] = mma3(reh, rel, bh, bl, acc[w][0]);
      acc[w][1] = mma3(imh, iml, bh, bl, acc[w][1]);
    }
  }
  float* out = static_cast<float*>(A.part) + ((size_t)slice * A.ntiles + tile) * NWG * 2 * 256;
#pragma unroll
  for (int w = 0; w < NWG; ++w)
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(w * 2 + r) * 256 + (4 * q + e) * 16 + i] = acc[w][r][e];
}

// Fixed-order FP64 sum of the slices, scale by -pref, write the block and its mirror.
template <typename T, int NWG>
__global__ void chi0_reduce(const T* __restrict__ part, int nslice, int ntiles, const int2* __restrict__ tiles,
                            int ng, int w0, int nw, double pref, int accumulate, double* __restrict__ chi0) {
  const int tile = blockIdx.x;
  const int w = blockIdx.y;
  const int e = threadIdx.x;  // 0..255
  if (w0 + w >= nw) return;
  const int2 bij = tiles[tile];
  const int ii = e >> 4, jj = e & 15;
  const int G = bij.x * kTile + ii, Gp = bij.y * kTile + jj;
  if (G >= ng || Gp >= ng) return;
  if (bij.x == bij.y && ii > jj) return;  // diagonal blocks: upper triangle is authoritative
  double re = 0.0, im = 0.0;
  for (int sl = 0; sl < nslice; ++sl) {
    const T* p = part + (((size_t)sl * ntiles + tile) * NWG + w) * 2 * 256;
    re += (double)p[e];
    im += (double)p[256 + e];
  }
  re *= -pref;
  im *= -pref;
  if (G == Gp) im = 0.0;
  double* m = chi0 + (size_t)(w0 + w) * ng * ng * 2;
  const size_t up = ((size_t)G * ng + Gp) * 2, lo = ((size_t)Gp * ng + G) * 2;
  if (accumulate) {
    m[up] += re;
    m[up + 1] += im;
    if (G != Gp) {
      m[lo] += re;
      m[lo + 1] -= im;
    }
  } else {
    m[up] = re;
    m[up + 1] = im;
    if (G != Gp) {
      m[lo] = re;
      m[lo + 1] = -im;
    }
  }
}

template <typename T, int NWG>
static int run_group(const TileArgs& base, int nslice_wg, hipStream_t s, int prec, int w0, int nw,
                     double pref, int accumulate, double* chi0) {
  TileArgs A = base;
  A.w0 = w0;
  dim3 grid(A.ntiles, nslice_wg);
  if (prec == XO_BF16X3) {
    if constexpr (std::is_same<T, float>::value) {
      {
        KernelTimer kt_("chi0_tiles_bf16x3", s);
        hipLaunchKernelGGL((chi0_tiles_bf16x3<NWG>), grid, dim3(256), 0, s, A);
      }
    }
  } else {
    {
      KernelTimer kt_("chi0_tiles", s);
      hipLaunchKernelGGL((chi0_tiles<T, NWG>), grid, dim3(256), 0, s, A);
    }
  }
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_("chi0_reduce", s);
    hipLaunchKernelGGL((chi0_reduce<T, NWG>), dim3(A.ntiles, NWG), dim3(256), 0, s,
                       static_cast<const T*>(A.part), nslice_wg * kWaves, A.ntiles, A.tiles, A.ng, w0, nw, pref,
                       accumulate, chi0);
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <typename T>
static int chi0_run(const xo_chi0_args* a, hipStream_t s) {
  const int nb = (a->ng + kTile - 1) / kTile;
  std::vector<int2> tl;
  for (int i = 0; i < nb; ++i)
    for (int j = i; j < nb; ++j) tl.push_back(make_int2(i, j));
  const int ntiles = (int)tl.size();
  const void* dtiles = nullptr;
  XO_RET(device_table(tl.data(), tl.size() * sizeof(int2), s, &dtiles));
  const void* dw = nullptr;
  XO_RET(device_table(a->w, sizeof(double) * a->nw, s, &dw));

  const int nwg = a->nw >= 8 ? 8 : (a->nw >= 4 ? 4 : (a->nw >= 2 ? 2 : 1));
  const int ngroups = (a->nw + nwg - 1) / nwg;
  const int nwpad = ngroups * nwg;
  // transitions per wave slice: aim for ~4096 waves in flight, slices a multiple of 16
  const int step = 16;
  int slices = std::max(kWaves, (4096 + ntiles - 1) / ntiles);
  slices = (slices + kWaves - 1) / kWaves * kWaves;
  int kper = (a->nt + slices - 1) / slices;
  kper = std::max(step, (kper + step - 1) / step * step);
  slices = (a->nt + kper - 1) / kper;
  slices = (slices + kWaves - 1) / kWaves * kWaves;
  const int nslice_wg = slices / kWaves;

  const size_t wbytes = align_up((size_t)a->nt * nwpad * sizeof(T), 256);
  const size_t pbytes = (size_t)slices * ntiles * nwg * 2 * 256 * sizeof(T);
  void* ws = nullptr;
  XO_RET(workspace(s, 1, wbytes + pbytes + 256, &ws));
  T* W = static_cast<T*>(ws);
  void* part = static_cast<char*>(ws) + wbytes;
  int* bad = reinterpret_cast<int*>(static_cast<char*>(ws) + wbytes + pbytes);
  if (a->check_dE) XO_TRY_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  {
    KernelTimer kt_("pole_factors", s);
    hipLaunchKernelGGL((pole_factors<T>), dim3((a->nt + 255) / 256), dim3(256), 0, s, a->dE, a->nt,
                       static_cast<const double*>(dw), a->nw, nwpad, W, a->check_dE ? bad : nullptr);
  }
  XO_CHECK_LAUNCH();
  if (a->check_dE) {
    int* hb = nullptr;
    XO_RET(host_flags(s, sizeof(int), reinterpret_cast<void**>(&hb)));
    XO_TRY_HIP(hipMemcpyAsync(hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    XO_TRY_HIP(hipStreamSynchronize(s));
    XO_ARG(*hb == 0, "xo_chi0: %d pole energies dE are <= 0 or NaN", *hb);
  }
  TileArgs A;
  A.rho = a->rho;
  A.W = W;
  A.nwpad = nwpad;
  A.w0 = 0;
  A.ng = a->ng;
  A.nt = a->nt;
  A.tiles = static_cast<const int2*>(dtiles);
  A.ntiles = ntiles;
  A.kper = kper;
  A.part = part;
  for (int g = 0; g < ngroups; ++g) {
    const int w0 = g * nwg;
    int r;
    switch (nwg) {
      case 8: r = run_group<T, 8>(A, nslice_wg, s, a->prec, w0, a->nw, a->pref, a->accumulate, a->chi0); break;
      case 4: r = run_group<T, 4>(A, nslice_wg, s, a->prec, w0, a->nw, a->pref, a->accumulate, a->chi0); break;
      case 2: r = run_group<T, 2>(A, nslice_wg, s, a->prec, w0, a->nw, a->pref, a->accumulate, a->chi0); break;
      default: r = run_group<T, 1>(A, nslice_wg, s, a->prec, w0, a->nw, a->pref, a->accumulate, a->chi0);
    }
    XO_RET(r);
  }
  return XO_OK;
}

}  // namespace
}  // namespace xo

extern "C" int xo_chi0(const xo_chi0_args* a, void* stream) {
  using namespace xo;
  clear_error();
  XO_ARG(a, "xo_chi0: null argument block");
  XO_ARG(a->nt > 0 && a->ng > 0 && a->nw > 0, "xo_chi0: sizes must be positive (nt=%d ng=%d nw=%d)", a->nt,
         a->ng, a->nw);
  XO_ARG(a->nw <= 64, "xo_chi0: at most 64 frequencies per call (got %d)", a->nw);
  XO_ARG(a->rho && a->dE && a->w && a->chi0, "xo_chi0: null pointer");
  XO_ARG(a->prec == XO_FP64 || a->prec == XO_FP32 || a->prec == XO_BF16X3, "xo_chi0: bad precision %d",
         a->prec);
  for (int j = 0; j < a->nw; ++j) XO_ARG(a->w[j] >= 0.0, "xo_chi0: frequency %d is negative", j);
  XO_ARG(a->pref > 0.0, "xo_chi0: pref must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->prec == XO_FP64) return chi0_run<double>(a, s);
  return chi0_run<float>(a, s);
}
