// Oscillator strengths as a gathered matrix product on MFMA (split or plain bf16,
// FP32 accumulation; FP64 / FP32 further down), many k-pairs per launch.
//
// With both orbitals expanded in plane waves, the cell-averaged transform of
// the product conj(psi_c) psi_v (Eq. rhotw, the umklapp vector G0 from
// k - q = k' + G0) is a finite sum over the conduction sphere:
//
//   rho_cv(G) = sum_a conj(c_c(a)) c_v(a - e),    e = m_G - G0,
//
// terms with a - e outside the valence sphere being zero. This is exactly what
// the FFT of the real-space product gives on any alias-free grid; at the sizes
// of these workloads it costs fewer multiply-adds per transition than the
// transform, and it is a dense contraction. For one k-pair it is a complex
// matrix product:
//
//   rows     (v, G), flattened r = v ng + G            left operand: c_v(a - e), gathered
//   columns  conduction band c                         right operand: c_c(a)
//   K        conduction plane wave a (interleaved re, im)
//
// The gather goes through one table per pair: the box of every difference
// a - e is laid out linearly, so that the offset of a - e splits as
// Oa[a] + Oe[G], and T[offset] is the valence plane-wave index (or the index of
// a zero entry). T and the valence bands of a workgroup's rows sit in LDS; the
// conduction tile is double buffered through LDS.
//
// Complex operands: the right operand holds (re, im) of c_c; the left operand
// of Re rho holds (re, im) of c_v and that of Im rho (im, -re), so that
// sum (vr cr + vi ci) = Re(conj(c) v) and sum (vi cr - vr ci) = Im(conj(c) v).
// Split form (NP = 3): every FP32 value x enters as hi = bf16(x), lo = bf16(x - hi);
// a product is hi*hi + hi*lo + lo*hi, accumulated in FP32. Plain form (NP = 1):
// hi only, one product; coefficients then take one 32-bit word instead of two.

#include <algorithm>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "bf16x3.h"
#include "rho_geom.h"

namespace xo {

int rho_batch_finish(const xo_rho_args* p, int n, hipStream_t s);

namespace {

constexpr int kThreads = 256;
constexpr int kCT = 8;               // column tiles (16 conduction bands each) per workgroup, at most (split form)
constexpr int kRT = 2;               // row tiles (16 (v, G) rows each) per wave
constexpr int kRows = 4 * 16 * kRT;  // rows per workgroup
constexpr size_t kBsBytes = (size_t)2 * 2 * kCT * 4 * 16 * sizeof(u4);  // [buffer][hi, lo][tile][q][column]
// Column tiles per workgroup (CT) and planes of the staged right operand (PL) of a
// form. The plain form keeps one plane; with seven tiles its registers (<= 168) and
// LDS allow three workgroups per CU (three waves per SIMD) instead of two, which it
// takes when seven-tile groups cover the columns in as many groups as eight-tile ones.
template <int NP, int CT>
struct GemmShape {
  static constexpr int PL = NP == 3 ? 2 : 1;
  static constexpr size_t bs_bytes = (size_t)2 * PL * CT * 64 * sizeof(u4);  // [buffer][plane][tile][q][column]
};
constexpr size_t kLdsMax = 160 * 1024;

typedef int i4 __attribute__((ext_vector_type(4)));

// Converted coefficients of one band set: [nb][npwp] entries, zero for j >= npw;
// an entry is the (hi, lo) word pair (NP = 3) or the hi word (NP = 1).
struct SplitDesc {
  const float2* src;  // [nb][npw]
  uint32_t* dst;
  int nb, npw, npwp;
};

template <int NP>
__global__ void __launch_bounds__(kThreads) orb_split(const SplitDesc* __restrict__ d) {
  const SplitDesc D = d[blockIdx.y];
  const int n = D.nb * D.npwp;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    const int b = i / D.npwp, j = i - b * D.npwp;
    const float2 v = j < D.npw ? D.src[(size_t)b * D.npw + j] : make_float2(0.f, 0.f);
    uint32_t h, l;
    split2(v.x, v.y, h, l);
    if constexpr (NP == 3)
      reinterpret_cast<uint2*>(D.dst)[i] = make_uint2(h, l);
    else
      D.dst[i] = h;
  }
}

struct GemmPair {
  const uint32_t* Sc;  // conduction converted coefficients [nc][npwc] entries
  const uint32_t* Sv;  // valence [nv][npwv] entries; entry npw_v of each row is zero
  float2* rho;      // [nv][nc][ng]
  const int* Oa;    // [nK * 16] box offset of each conduction plane wave (a valid offset for padding)
  const int* Oe;    // [ng] box offset of -e = G0 - m_G
  const u4* T;      // [ncell / 8] uint16 valence index of each box cell, npw_v outside the sphere
  int npwc, npwv;   // row strides of Sc and Sv (multiples of 16)
  int nK;           // K steps of 16 conduction plane waves
  int ncell;        // box cells, a multiple of 8
  int nc, nv;
  int nct, ncg;     // column tiles and column groups
  int nrb;          // row blocks of kRows rows
  int wg0;          // first logical workgroup of the pair
};

template <int NP, int CT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(CT <= 7 ? 3 : 2)))
rho_gemm(const GemmPair* __restrict__ pairs, int npairs, int nwg, int ng) {
  constexpr int kW = NP == 3 ? 2 : 1;  // 32-bit words per coefficient
  constexpr int PL = GemmShape<NP, CT>::PL;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // XCD-aware order: workgroup b runs on XCD b % 8, which takes a contiguous
  // logical range, so a pair's tables and coefficients stay in that XCD's L2.
  const int per = (nwg + 7) >> 3;
  const int L = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (L >= nwg) return;
  int plo = 0, phi = npairs - 1;
  while (plo < phi) {
    const int mid = (plo + phi + 1) >> 1;
    if (pairs[mid].wg0 <= L) plo = mid; else phi = mid - 1;
  }
  const GemmPair& P = pairs[plo];
  const int local = L - P.wg0;
  const int cg = local / P.nrb, rb = local - cg * P.nrb;
  const int ct0 = cg * P.nct / P.ncg, nt = (cg + 1) * P.nct / P.ncg - ct0;
  const int nrows = P.nv * ng;
  const int r0 = rb * kRows;
  const int vlo = r0 / ng, vhi = min(P.nv - 1, (r0 + kRows - 1) / ng);
  const int npwv = P.npwv, npwc = P.npwc, nK = P.nK;

  u4* Bs = reinterpret_cast<u4*>(smem);                                // [2][PL][CT][4][16]
  uint32_t* Vs = reinterpret_cast<uint32_t*>(smem + GemmShape<NP, CT>::bs_bytes);  // [vhi - vlo + 1][npwv] entries
  const int nvs = (vhi - vlo + 1) * npwv * kW;                         // words, a multiple of 16
  uint16_t* Ts = reinterpret_cast<uint16_t*>(Vs + nvs);                 // [ncell]

  const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

  // ---- box table and the valence bands of this workgroup's rows into LDS
  for (int k = tid; k < P.ncell / 8; k += kThreads) reinterpret_cast<u4*>(Ts)[k] = gld<u4>(P.T + k);
  {
    const u4* src = reinterpret_cast<const u4*>(P.Sv + (size_t)vlo * npwv * kW);
    for (int k = tid; k < nvs / 4; k += kThreads) reinterpret_cast<u4*>(Vs)[k] = gld<u4>(src + k);
  }

  // ---- rows of this lane: row tile rt holds rows r0 + 32 w + 16 rt + (0..15); lane i gathers row i
  int vb[kRT], oe[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int r = r0 + 32 * w + 16 * rt + i;
    const int v = r < nrows ? r / ng : vlo;
    const int g = r < nrows ? r - v * ng : 0;
    vb[rt] = (v - vlo) * npwv;
    oe[rt] = gld<int>(P.Oe + g);
  }

  // ---- right operand staging: slot s = tid + 256 f is (tile s / 64, quad (s / 16) % 4, column s % 16).
  // Columns past the group or the band count read a valid row (clamped); their
  // products land in outputs that are never stored.
  // (split: two 16-byte loads of (hi, lo) pairs per slot; plain: one of hi words)
  u4 raw[2][2];
  const uint32_t* sp[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int s = tid + kThreads * f;
    const int sq = (s >> 4) & 3, c = min((ct0 + (s >> 6)) * 16 + (s & 15), P.nc - 1);
    sp[f] = P.Sc + ((size_t)c * npwc + 4 * sq) * kW;
  }
#define RHO_GEMM_LOAD(k_)                                                         \
  _Pragma("unroll") for (int f = 0; f < 2; ++f) {                                 \
    raw[f][0] = gld<u4>(sp[f] + 16 * kW * (k_));                                  \
    if constexpr (NP == 3) raw[f][1] = gld<u4>(sp[f] + 16 * kW * (k_) + 4);       \
  }
#define RHO_GEMM_STORE(b_)                                                        \
  _Pragma("unroll") for (int f = 0; f < 2; ++f) {                                 \
    const int s_ = tid + kThreads * f;                                            \
    if (s_ < CT * 64) {                                                           \
      if constexpr (NP == 3) {                                                    \
        Bs[((b_) * PL + 0) * (CT * 64) + s_] = u4{raw[f][0].x, raw[f][0].z, raw[f][1].x, raw[f][1].z}; \
        Bs[((b_) * PL + 1) * (CT * 64) + s_] = u4{raw[f][0].y, raw[f][0].w, raw[f][1].y, raw[f][1].w}; \
      } else {                                                                    \
        Bs[(b_) * (CT * 64) + s_] = raw[f][0];                                    \
      }                                                                           \
    }                                                                             \
  }

  RHO_GEMM_LOAD(0);
  RHO_GEMM_STORE(0);
  // Box offsets of this lane's conduction plane waves, two steps ahead.
  i4 oa1 = gld<i4>(P.Oa + 4 * q);
  i4 oa2 = gld<i4>(P.Oa + 16 * min(1, nK - 1) + 4 * q);
  __syncthreads();

  // Gathered left operand of this lane's rows, c_v(a - e) for a = 16 k + 4 q + (0..3)
  // (hi and lo read as words, straight into the operand registers). The box
  // table and valence bands do not change during the loop, so the next step's
  // gather is issued while this step's products run.
  const uint32_t* Vw = Vs;
  auto gather = [&](i4 oa, u4* gh, u4* gl) {
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      const int o[4] = {oa.x, oa.y, oa.z, oa.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = kW * (vb[rt] + Ts[o[u] + oe[rt]]);
        gh[rt][u] = Vw[j];
        if constexpr (NP == 3) gl[rt][u] = Vw[j + 1];
      }
    }
  };
  u4 ah[kRT], al[kRT] = {};
  gather(oa1, ah, al);
  oa1 = oa2;

  f4 re[kRT][CT], im[kRT][CT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) re[rt][ct] = im[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};

  for (int k = 0; k < nK; ++k) {
    const int buf = k & 1;
    if (k + 1 < nK) {
      RHO_GEMM_LOAD(k + 1);
      oa2 = gld<i4>(P.Oa + 16 * min(k + 2, nK - 1) + 4 * q);
    }
    // next step's gather (the last step re-gathers valid offsets, unused)
    u4 nah[kRT], nal[kRT] = {};
    gather(oa1, nah, nal);
    // Im operand: (im, -re) of the gathered values
    u4 bh[kRT], bl[kRT];
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bh[rt][u] = rot_pos(ah[rt][u]);
        bl[rt][u] = rot_pos(al[rt][u]);
      }
    const u4* Bh = Bs + (buf * PL + 0) * (CT * 64) + lane;
    const u4* Bl = Bs + (buf * PL + PL - 1) * (CT * 64) + lane;  // the lo plane (split form)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (ct < nt) {
        const u4 ch = Bh[ct * 64];
        u4 cl = ch;
        if constexpr (NP == 3) cl = Bl[ct * 64];
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt) {
          re[rt][ct] = mma_np<NP>(ah[rt], al[rt], ch, cl, re[rt][ct]);
          im[rt][ct] = mma_np<NP>(bh[rt], bl[rt], ch, cl, im[rt][ct]);
        }
      }
    }
    if (k + 1 < nK) RHO_GEMM_STORE(buf ^ 1);
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt) {
      ah[rt] = nah[rt];
      al[rt] = nal[rt];
    }
    oa1 = oa2;
    __syncthreads();
  }
#undef RHO_GEMM_LOAD
#undef RHO_GEMM_STORE

  // ---- results: lane holds rows 4 q + (0..3) of each row tile, column i of each column tile
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int rb4 = r0 + 32 * w + 16 * rt + 4 * q;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int c = (ct0 + ct) * 16 + i;
      if (ct >= nt || c >= P.nc) continue;
      const int v4 = rb4 < nrows ? rb4 / ng : 0, g4 = rb4 - v4 * ng;
      float2* o4 = P.rho + ((size_t)v4 * P.nc + c) * ng + g4;
      if (rb4 + 3 < nrows && g4 + 3 < ng && ((uintptr_t)o4 & 15) == 0) {
        // four consecutive G of one band: two 16-byte stores
        f4* out = reinterpret_cast<f4*>(o4);
        gst<f4>(out, f4{re[rt][ct][0], im[rt][ct][0], re[rt][ct][1], im[rt][ct][1]});
        gst<f4>(out + 1, f4{re[rt][ct][2], im[rt][ct][2], re[rt][ct][3], im[rt][ct][3]});
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = rb4 + e;
          if (r >= nrows) break;
          const int v = r / ng, g = r - v * ng;
          gst<f2v>(P.rho + ((size_t)v * P.nc + c) * ng + g, f2v{re[rt][ct][e], im[rt][ct][e]});
        }
      }
    }
  }
}

// ------------------------------------------------- FP64 / FP32 products --
// The same gathered product in the working precision on v_mfma_f64_16x16x4f64 /
// v_mfma_f32_16x16x4f32: K = 4 real columns per instruction, i.e. two plane
// waves (re, im). Lane l = i + 16 kk holds row i (left) or column i (right) at
// K index kk: plane wave 16 k + 2 s + kk / 2, component kk % 2. The left
// operand of Re rho is that component of c_v(a - e), the one of Im rho the
// component of (im, -re); the right operand is the component of c_c(a).
// Coefficients are read straight from the caller's arrays (no split).
typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int kBsTile = 16 * 17;  // staged right-operand tile: 16 plane waves x (16 columns + 1 pad)

template <typename T>
struct FpMma;
template <>
struct FpMma<double> {
  typedef d4v V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kk, int r) { return kk + 4 * r; }  // result register r
};
template <>
struct FpMma<float> {
  typedef f4 V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kk, int r) { return 4 * kk + r; }
};

struct GemmPairFp {
  const void* Cc;  // conduction coefficients [nc][npw_c] complex (caller's)
  const void* Cv;  // valence [nv][npw_v] complex (caller's)
  void* rho;       // [nv][nc][ng] complex
  const int* OaP;  // [nK][2][8] box offsets by step and parity
  const int* Oe;   // [ng]
  const u4* T;     // [ncell / 8] uint16 valence index of each box cell, npw_v outside the sphere
  int npw_c, npw_v, vstride;  // vstride: LDS row of a valence band (npw_v + 1, even)
  int nK, ncell, nc, nv, nct, ncg, nrb, wg0;
};

// complex load through the global address space
template <typename T>
__device__ __forceinline__ cplx<T> gld_c(const cplx<T>* p) {
  typedef T T2 __attribute__((ext_vector_type(2)));
  const T2 x = gld<T2>(p);
  return cplx<T>{x.x, x.y};
}

template <typename T, int CT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
rho_gemm_fp(const GemmPairFp* __restrict__ pairs, int npairs, int nwg, int ng) {
  typedef cplx<T> C;
  typedef typename FpMma<T>::V V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int per = (nwg + 7) >> 3;
  const int L = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (L >= nwg) return;
  int plo = 0, phi = npairs - 1;
  while (plo < phi) {
    const int mid = (plo + phi + 1) >> 1;
    if (pairs[mid].wg0 <= L) plo = mid; else phi = mid - 1;
  }
  const GemmPairFp& P = pairs[plo];
  const int local = L - P.wg0;
  const int cg = local / P.nrb, rb = local - cg * P.nrb;
  const int ct0 = cg * P.nct / P.ncg, nt = (cg + 1) * P.nct / P.ncg - ct0;
  const int nrows = P.nv * ng;
  const int r0 = rb * kRows;
  const int vlo = r0 / ng, vhi = min(P.nv - 1, (r0 + kRows - 1) / ng);
  const int nK = P.nK, npw_c = P.npw_c, vstride = P.vstride;

  C* Bs = reinterpret_cast<C*>(smem);                                    // [2][CT][16 a][17]: 16 columns + pad
  uint16_t* Ts = reinterpret_cast<uint16_t*>(smem + 2 * CT * kBsTile * sizeof(C));  // [ncell]
  C* Vs = reinterpret_cast<C*>(Ts + P.ncell);                            // [vhi - vlo + 1][vstride]
  const int nvs = (vhi - vlo + 1) * vstride;

  const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, kk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

  // ---- box table and the valence bands of this workgroup's rows (zero past each band)
  for (int k = tid; k < P.ncell / 8; k += kThreads) reinterpret_cast<u4*>(Ts)[k] = gld<u4>(P.T + k);
  {
    const C* src = static_cast<const C*>(P.Cv) + (size_t)vlo * P.npw_v;
    for (int k = tid; k < nvs; k += kThreads) {
      const int sl = k / vstride, j = k - sl * vstride;
      const C x = gld_c(src + (size_t)sl * P.npw_v + min(j, P.npw_v - 1));
      Vs[k] = j < P.npw_v ? x : C{T(0), T(0)};
    }
  }
  int vb[kRT], oe[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    const int r = r0 + 32 * w + 16 * rt + i;
    const int v = r < nrows ? r / ng : vlo;
    const int g = r < nrows ? r - v * ng : 0;
    vb[rt] = (v - vlo) * vstride;
    oe[rt] = gld<int>(P.Oe + g);
  }
  // ---- right operand staging: element e = tid + 256 f is (tile e / 256, column (e / 16) % 16,
  // plane wave e % 16); invalid columns and plane waves past the sphere stage zeros
  const C* Cc = static_cast<const C*>(P.Cc);
  int cidx[CT];
  bool cok[CT];
#pragma unroll
  for (int f = 0; f < CT; ++f) {
    const int e = tid + kThreads * f;
    const int c = (ct0 + (e >> 8)) * 16 + ((e >> 4) & 15);
    cok[f] = (e >> 8) < nt && c < P.nc;
    cidx[f] = min(c, P.nc - 1) * npw_c;
  }
  const int al = tid & 15;
  C raw[CT];
  auto load = [&](int k) {
    const int a = 16 * k + al;
#pragma unroll
    for (int f = 0; f < CT; ++f) {
      const C x = gld_c(Cc + cidx[f] + min(a, npw_c - 1));
      raw[f] = (cok[f] && a < npw_c) ? x : C{T(0), T(0)};
    }
  };
  // element e = tid + 256 f goes to [tile e / 256][plane wave e % 16][column (e / 16) % 16]
  auto store = [&](int b) {
#pragma unroll
    for (int f = 0; f < CT; ++f) {
      const int e = tid + kThreads * f;
      Bs[((size_t)b * CT + (e >> 8)) * kBsTile + (e & 15) * 17 + ((e >> 4) & 15)] = raw[f];
    }
  };
  load(0);
  store(0);
  i4 oa0 = gld<i4>(P.OaP + 8 * (kk >> 1)), oa1 = gld<i4>(P.OaP + 8 * (kk >> 1) + 4);
  __syncthreads();

  V re[kRT][CT], im[kRT][CT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) re[rt][ct] = im[rt][ct] = V{T(0), T(0), T(0), T(0)};
  const T* Bw = reinterpret_cast<const T*>(Bs);
  for (int k = 0; k < nK; ++k) {
    const int buf = k & 1;
    i4 na0 = oa0, na1 = oa1;
    if (k + 1 < nK) {
      load(k + 1);
      na0 = gld<i4>(P.OaP + 16 * (k + 1) + 8 * (kk >> 1));
      na1 = gld<i4>(P.OaP + 16 * (k + 1) + 8 * (kk >> 1) + 4);
    }
    const int o[8] = {oa0.x, oa0.y, oa0.z, oa0.w, oa1.x, oa1.y, oa1.z, oa1.w};
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      T xr[kRT], xi[kRT];
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
        const C v = Vs[vb[rt] + Ts[o[st] + oe[rt]]];
        xr[rt] = (kk & 1) ? v.y : v.x;
        xi[rt] = (kk & 1) ? -v.x : v.y;
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (ct < nt) {
          const T bv = Bw[(((size_t)buf * CT + ct) * kBsTile + (2 * st + (kk >> 1)) * 17 + i) * 2 + (kk & 1)];
#pragma unroll
          for (int rt = 0; rt < kRT; ++rt) {
            re[rt][ct] = FpMma<T>::mma(xr[rt], bv, re[rt][ct]);
            im[rt][ct] = FpMma<T>::mma(xi[rt], bv, im[rt][ct]);
          }
        }
      }
    }
    if (k + 1 < nK) store(buf ^ 1);
    oa0 = na0;
    oa1 = na1;
    __syncthreads();
  }
  // ---- results: lane holds rows FpMma::row(kk, r) of each row tile, column i of each column tile
  C* rho = static_cast<C*>(P.rho);
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int c = (ct0 + ct) * 16 + i;
      if (ct >= nt || c >= P.nc) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 32 * w + 16 * rt + FpMma<T>::row(kk, r);
        if (row >= nrows) continue;
        const int v = row / ng, g = row - v * ng;
        rho[((size_t)v * P.nc + c) * ng + g] = C{re[rt][ct][r], im[rt][ct][r]};
      }
    }
}

// ------------------------------------------------------------------ host --
struct GemmGeo {
  std::vector<int> Oa, Oe;
  std::vector<int> OaP;  // Oa by step and parity, [nK][2][8]: OaP[16 k + 8 p + s] = Oa[16 k + 2 s + p]
  std::vector<uint16_t> T;
  int nK = 0;
  const void* dOaP = nullptr;
  const void* dOa = nullptr;
  const void* dOe = nullptr;
  const void* dT = nullptr;
  unsigned gen = 0;
  bool ok = false;
};

// Gather tables of one pair. The box spans every a - e (a over the conduction
// sphere, e = m_G - G0 over the G-set): lo = min a - max e, hi = max a - min e.
static void gemm_geo(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, GemmGeo* g) {
  int lo[3], w[3];
  size_t ncell = 1;
  for (int d = 0; d < 3; ++d) {
    lo[d] = xc.lo[d] - xe.hi[d];
    w[d] = (xc.hi[d] - xe.lo[d]) - lo[d] + 1;
    ncell *= (size_t)w[d];
  }
  g->ok = a->npw_v < 65535 && ncell * 2 <= kLdsMax;
  if (!g->ok) return;
  const long SX = w[0], SY = (long)w[0] * w[1];
  g->nK = (a->npw_c + 15) / 16;
  g->Oa.resize((size_t)g->nK * 16);
  for (int p = 0; p < a->npw_c; ++p)
    g->Oa[p] = (int)((a->mill_c[3 * p] - lo[0]) + SX * (a->mill_c[3 * p + 1] - lo[1]) +
                     SY * (a->mill_c[3 * p + 2] - lo[2]));
  for (size_t p = a->npw_c; p < g->Oa.size(); ++p) g->Oa[p] = g->Oa[0];
  g->OaP.resize(g->Oa.size());
  for (int k = 0; k < g->nK; ++k)
    for (int pp = 0; pp < 2; ++pp)
      for (int st = 0; st < 8; ++st) g->OaP[16 * k + 8 * pp + st] = g->Oa[16 * k + 2 * st + pp];
  g->Oe.resize(a->ng);
  for (int j = 0; j < a->ng; ++j) {
    const long ex = a->mill_g[3 * j] - a->g0[0], ey = a->mill_g[3 * j + 1] - a->g0[1],
               ez = a->mill_g[3 * j + 2] - a->g0[2];
    g->Oe[j] = (int)(-ex - SX * ey - SY * ez);
  }
  g->T.assign((ncell + 7) / 8 * 8, (uint16_t)a->npw_v);
  for (int p = 0; p < a->npw_v; ++p) {
    const int x = a->mill_v[3 * p] - lo[0], y = a->mill_v[3 * p + 1] - lo[1], z = a->mill_v[3 * p + 2] - lo[2];
    // valence plane waves outside the box are never reached by any a - e
    if (x < 0 || y < 0 || z < 0 || x >= w[0] || y >= w[1] || z >= w[2]) continue;
    g->T[x + SX * y + SY * z] = (uint16_t)p;
  }
  (void)xv;
}

// Tables cached by the caller's Miller-list pointers and scalars, confirmed by
// a full comparison of the lists' contents (a reused buffer with new contents
// is a miss), for the life of the device tables.
static int gemm_entry(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, hipStream_t s,
                      const GemmGeo** out) {
  struct Key {
    std::vector<int32_t> mc, mv, mg;
  };
  static std::mutex mu;
  static std::map<std::vector<intptr_t>, std::vector<std::pair<Key, std::unique_ptr<GemmGeo>>>> cache;
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  const std::vector<intptr_t> pk = {dev, a->g0[0], a->g0[1], a->g0[2], a->npw_c, a->npw_v, a->ng,
                                    (intptr_t)a->mill_c, (intptr_t)a->mill_v, (intptr_t)a->mill_g};
  auto same = [&](const Key& k) {
    return std::memcmp(k.mc.data(), a->mill_c, 12 * (size_t)a->npw_c) == 0 &&
           std::memcmp(k.mv.data(), a->mill_v, 12 * (size_t)a->npw_v) == 0 &&
           std::memcmp(k.mg.data(), a->mill_g, 12 * (size_t)a->ng) == 0;
  };
  const unsigned gen = table_generation();
  std::lock_guard<std::mutex> lk(mu);
  auto& bucket = cache[pk];
  std::unique_ptr<GemmGeo>* slotp = nullptr;
  for (auto& kv : bucket)
    if (same(kv.first)) slotp = &kv.second;
  if (slotp && (*slotp)->gen == gen) {
    *out = (*slotp)->ok ? slotp->get() : nullptr;
    return XO_OK;
  }
  GemmGeo e;
  e.gen = gen;
  gemm_geo(a, xc, xv, xe, &e);
  if (e.ok) {
    XO_RET(device_table(e.Oa.data(), e.Oa.size() * sizeof(int), s, &e.dOa));
    XO_RET(device_table(e.OaP.data(), e.OaP.size() * sizeof(int), s, &e.dOaP));
    XO_RET(device_table(e.Oe.data(), e.Oe.size() * sizeof(int), s, &e.dOe));
    XO_RET(device_table(e.T.data(), e.T.size() * sizeof(uint16_t), s, &e.dT));
  }
  if (!slotp) {
    Key k;
    k.mc.assign(a->mill_c, a->mill_c + 3 * a->npw_c);
    k.mv.assign(a->mill_v, a->mill_v + 3 * a->npw_v);
    k.mg.assign(a->mill_g, a->mill_g + 3 * a->ng);
    bucket.emplace_back(std::move(k), nullptr);
    slotp = &bucket.back().second;
  }
  // a stale entry (tables released) is replaced, not freed: callers on other
  // threads may still hold it
  slotp->release();
  *slotp = std::make_unique<GemmGeo>(std::move(e));
  *out = (*slotp)->ok ? slotp->get() : nullptr;
  return XO_OK;
}

inline int padded_row(int npw) { return (npw + 1 + 15) / 16 * 16; }

}  // namespace

// The batch on the gathered-product kernel (NP = 3 split, 1 plain bf16), or
// XO_ERR_UNSUPPORTED (nothing enqueued) when a pair's tables do not fit in LDS.
// All pairs share ng and the G-set.
template <int NP, int CT>
static int rho_batch_gemm_t(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                            hipStream_t s) {
  constexpr int kW = NP == 3 ? 2 : 1;
  const int ng = p[0].ng;
  std::vector<const GemmGeo*> ge(n);
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    XO_RET(gemm_entry(&p[i], xc[i], xv[i], xe[i], s, &ge[i]));
    if (!ge[i]) return XO_ERR_UNSUPPORTED;
    // band slots: the rows [r0, r0 + kRows) of a workgroup span at most this many bands
    int nbs = 1;
    const int nrows = p[i].nv * ng;
    for (int r0 = 0; r0 < nrows; r0 += kRows)
      nbs = std::max(nbs, std::min(p[i].nv - 1, (r0 + kRows - 1) / ng) - r0 / ng + 1);
    const size_t need = GemmShape<NP, CT>::bs_bytes + (size_t)nbs * padded_row(p[i].npw_v) * kW * 4 + ge[i]->T.size() * 2;
    lds = std::max(lds, need);
  }
  if (lds > kLdsMax) return XO_ERR_UNSUPPORTED;

  // split coefficients, once per distinct band set of the batch
  std::map<std::tuple<const void*, int, int>, size_t> sets;
  std::vector<SplitDesc> sd;
  size_t tot = 0;
  auto add = [&](const void* c, int nb, int npw) {
    auto key = std::make_tuple(c, nb, npw);
    if (sets.count(key)) return;
    sets[key] = tot;
    // zeroed first: the padding bytes take part in the table cache's content hash
    SplitDesc d;
    std::memset(&d, 0, sizeof d);
    d.src = static_cast<const float2*>(c);
    d.dst = nullptr;
    d.nb = nb;
    d.npw = npw;
    d.npwp = padded_row(npw);
    sd.push_back(d);
    tot += (size_t)nb * d.npwp;
  };
  for (int i = 0; i < n; ++i) {
    add(p[i].coef_c, p[i].nc, p[i].npw_c);
    add(p[i].coef_v, p[i].nv, p[i].npw_v);
  }
  void* ws = nullptr;
  XO_RET(workspace(s, 3, tot * kW * 4, &ws));
  uint32_t* S0 = static_cast<uint32_t*>(ws);
  int maxn = 0;
  for (auto& d : sd) {
    d.dst = S0 + sets[std::make_tuple(static_cast<const void*>(d.src), d.nb, d.npw)] * kW;
    maxn = std::max(maxn, d.nb * d.npwp);
  }
  const void* dsd = nullptr;
  XO_RET(device_table(sd.data(), sd.size() * sizeof(SplitDesc), s, &dsd));
  {
    KernelTimer kt_("orb_split", s);
    hipLaunchKernelGGL(orb_split<NP>, dim3(std::min(256, (maxn + kThreads - 1) / kThreads), (unsigned)sd.size()),
                       dim3(kThreads), 0, s, static_cast<const SplitDesc*>(dsd));
  }
  XO_CHECK_LAUNCH();

  std::vector<GemmPair> gp(n);
  int nwg = 0;
  for (int i = 0; i < n; ++i) {
    const GemmGeo& g = *ge[i];
    GemmPair& d = gp[i];
    d.Sc = S0 + sets[std::make_tuple(p[i].coef_c, p[i].nc, p[i].npw_c)] * kW;
    d.Sv = S0 + sets[std::make_tuple(p[i].coef_v, p[i].nv, p[i].npw_v)] * kW;
    d.rho = static_cast<float2*>(p[i].rho);
    d.Oa = static_cast<const int*>(g.dOa);
    d.Oe = static_cast<const int*>(g.dOe);
    d.T = static_cast<const u4*>(g.dT);
    d.npwc = padded_row(p[i].npw_c);
    d.npwv = padded_row(p[i].npw_v);
    d.nK = g.nK;
    d.ncell = (int)g.T.size();
    d.nc = p[i].nc;
    d.nv = p[i].nv;
    d.nct = (p[i].nc + 15) / 16;
    d.ncg = (d.nct + CT - 1) / CT;
    d.nrb = (p[i].nv * ng + kRows - 1) / kRows;
    d.wg0 = nwg;
    nwg += d.ncg * d.nrb;
  }
  const void* dgp = nullptr;
  XO_RET(device_table(gp.data(), gp.size() * sizeof(GemmPair), s, &dgp));
  if (lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rho_gemm<NP, CT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    KernelTimer kt_(NP == 3 ? "rho_gemm" : "rho_gemm_bf16", s);
    hipLaunchKernelGGL((rho_gemm<NP, CT>), dim3(8 * ((nwg + 7) / 8)), dim3(kThreads), lds, s,
                       static_cast<const GemmPair*>(dgp), n, nwg, ng);
  }
  XO_CHECK_LAUNCH();
  return rho_batch_finish(p, n, s);
}

// LDS bytes of one gathered-product workgroup for pair a (host geometry only), or 0
// when its gather box does not fit.
static size_t gemm_lds(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, size_t bs_bytes,
                       size_t vrow_bytes) {
  GemmGeo g;
  gemm_geo(a, xc, xv, xe, &g);
  if (!g.ok) return 0;
  int nbs = 1;
  const int nrows = a->nv * a->ng;
  for (int r0 = 0; r0 < nrows; r0 += kRows)
    nbs = std::max(nbs, std::min(a->nv - 1, (r0 + kRows - 1) / a->ng) - r0 / a->ng + 1);
  return bs_bytes + (size_t)nbs * vrow_bytes + g.T.size() * 2;
}

// Workspace bytes the gathered-product path requests for the batch (0 for FP64 / FP32,
// which read the coefficients in place), or XO_ERR_UNSUPPORTED when it cannot take it.
// Host computation only (no device tables are built).
int rho_gemm_ws_bytes(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                      size_t* bytes) {
  const bool bf = p[0].prec == XO_BF16X3 || p[0].prec == XO_BF16;
  const int kW = p[0].prec == XO_BF16X3 ? 2 : 1;
  size_t bs = 0;
  if (p[0].prec == XO_BF16X3) {
    bs = GemmShape<3, kCT>::bs_bytes;
  } else if (p[0].prec == XO_BF16) {
    int nct = 1;
    for (int i = 0; i < n; ++i) nct = std::max(nct, (p[i].nc + 15) / 16);
    bs = (nct + 6) / 7 == (nct + 7) / 8 ? GemmShape<1, 7>::bs_bytes : GemmShape<1, 8>::bs_bytes;
  } else {
    const int CT = p[0].prec == XO_FP64 ? 4 : 8;
    bs = (size_t)2 * CT * kBsTile * (p[0].prec == XO_FP64 ? 16 : 8);
  }
  for (int i = 0; i < n; ++i) {
    const size_t vrow = bf ? (size_t)padded_row(p[i].npw_v) * kW * 4
                           : ((size_t)(p[i].npw_v + 2) & ~(size_t)1) * (p[0].prec == XO_FP64 ? 16 : 8);
    const size_t lds = gemm_lds(&p[i], xc[i], xv[i], xe[i], bs, vrow);
    if (lds == 0 || lds > kLdsMax) return XO_ERR_UNSUPPORTED;
  }
  *bytes = 0;
  if (!bf) return XO_OK;
  std::set<std::tuple<const void*, int, int>> sets;
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    for (int side = 0; side < 2; ++side) {
      const void* c = side ? p[i].coef_v : p[i].coef_c;
      const int nb = side ? p[i].nv : p[i].nc, npw = side ? p[i].npw_v : p[i].npw_c;
      if (sets.insert(std::make_tuple(c, nb, npw)).second) tot += (size_t)nb * padded_row(npw);
    }
  }
  *bytes = tot * kW * 4;
  return XO_OK;
}

int rho_batch_gemm(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                   hipStream_t s) {
  if (p[0].prec == XO_BF16) {
    int nct = 1;
    for (int i = 0; i < n; ++i) nct = std::max(nct, (p[i].nc + 15) / 16);
    if ((nct + 6) / 7 == (nct + 7) / 8) return rho_batch_gemm_t<1, 7>(p, n, xc, xv, xe, s);
    return rho_batch_gemm_t<1, 8>(p, n, xc, xv, xe, s);
  }
  return rho_batch_gemm_t<3, kCT>(p, n, xc, xv, xe, s);
}


// FP64 / FP32 batch on the gathered product, or XO_ERR_UNSUPPORTED (nothing
// enqueued) when a pair's tables do not fit in LDS.
template <typename T, int CT>
static int rho_batch_gemm_fp_t(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                               hipStream_t s) {
  typedef cplx<T> C;
  const int ng = p[0].ng;
  std::vector<const GemmGeo*> ge(n);
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    XO_RET(gemm_entry(&p[i], xc[i], xv[i], xe[i], s, &ge[i]));
    if (!ge[i]) return XO_ERR_UNSUPPORTED;
    int nbs = 1;
    const int nrows = p[i].nv * ng;
    for (int r0 = 0; r0 < nrows; r0 += kRows)
      nbs = std::max(nbs, std::min(p[i].nv - 1, (r0 + kRows - 1) / ng) - r0 / ng + 1);
    const size_t vstride = (size_t)(p[i].npw_v + 2) & ~(size_t)1;
    const size_t need = (size_t)2 * CT * kBsTile * sizeof(C) + ge[i]->T.size() * 2 + nbs * vstride * sizeof(C);
    lds = std::max(lds, need);
  }
  if (lds > kLdsMax) return XO_ERR_UNSUPPORTED;
  std::vector<GemmPairFp> gp(n);
  int nwg = 0;
  for (int i = 0; i < n; ++i) {
    const GemmGeo& g = *ge[i];
    GemmPairFp& d = gp[i];
    d.Cc = p[i].coef_c;
    d.Cv = p[i].coef_v;
    d.rho = p[i].rho;
    d.OaP = static_cast<const int*>(g.dOaP);
    d.Oe = static_cast<const int*>(g.dOe);
    d.T = static_cast<const u4*>(g.dT);
    d.npw_c = p[i].npw_c;
    d.npw_v = p[i].npw_v;
    d.vstride = (p[i].npw_v + 2) & ~1;
    d.nK = g.nK;
    d.ncell = (int)g.T.size();
    d.nc = p[i].nc;
    d.nv = p[i].nv;
    d.nct = (p[i].nc + 15) / 16;
    d.ncg = (d.nct + CT - 1) / CT;
    d.nrb = (p[i].nv * ng + kRows - 1) / kRows;
    d.wg0 = nwg;
    nwg += d.ncg * d.nrb;
  }
  const void* dgp = nullptr;
  XO_RET(device_table(gp.data(), gp.size() * sizeof(GemmPairFp), s, &dgp));
  if (lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rho_gemm_fp<T, CT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    KernelTimer kt_(sizeof(T) == 8 ? "rho_gemm_f64" : "rho_gemm_f32", s);
    hipLaunchKernelGGL((rho_gemm_fp<T, CT>), dim3(8 * ((nwg + 7) / 8)), dim3(kThreads), lds, s,
                       static_cast<const GemmPairFp*>(dgp), n, nwg, ng);
  }
  XO_CHECK_LAUNCH();
  return rho_batch_finish(p, n, s);
}

int rho_batch_gemm_fp(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                      hipStream_t s) {
  if (p[0].prec == XO_FP64) return rho_batch_gemm_fp_t<double, 4>(p, n, xc, xv, xe, s);
  return rho_batch_gemm_fp_t<float, 8>(p, n, xc, xv, xe, s);
}

}  // namespace xo
