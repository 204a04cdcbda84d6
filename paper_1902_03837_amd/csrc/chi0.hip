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
// left operand carries the weight of each frequency.
//
// Work decomposition. A chi0 problem (an "item", one q-point) is cut into units
// (item, block pair i <= j, group of <= 8 frequencies, transition slice). One
// persistent launch serves every unit of every item from an atomic queue ordered
// longest-first; each workgroup's four waves split the unit's transitions, and
// each wave writes its partial 16 x (16 NT) block. A second kernel adds the
// partials of each output block in unit order (bitwise deterministic whatever the
// queue order), applies -pref and writes the block and its Hermitian mirror.
//
// Operand/result layout of the 16x16 MFMA tiles (v_mfma_*_16x16x4, one block):
//   A[i][k]: lane = i + 16 k,  B[k][j]: lane = j + 16 k.
//   Result register r of a lane: f32 and bf16 forms D[4 (lane/16) + r][lane%16];
//   the f64 form D[lane/16 + 4 r][lane%16] (checked on the device).
// bf16 variant (v_mfma_f32_16x16x32_bf16): lane = i + 16 q holds k = 8 q .. 8 q + 7.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <map>
#include <vector>

#include "bf16x3.h"
#include "xo_common.h"

namespace xo {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;
constexpr int kFp32Slice = 65536;  // longest transition slice accumulated in FP32 by default
constexpr int kWaves = 4;
constexpr int MODE_F64 = 0, MODE_F32 = 1, MODE_BF16X3 = 2, MODE_BF16 = 3;
// bf16 forms: products per operand pair (3 split, 1 plain)
constexpr bool is_bf(int mode) { return mode == MODE_BF16X3 || mode == MODE_BF16; }
constexpr int nprod(int mode) { return mode == MODE_BF16X3 ? 3 : 1; }

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

// Real-axis factors of Eq. (X_IP), time-ordered: F = 1/(w - D + i eta) - 1/(w + D - i eta).
// Frequency w_j takes two slots of the Hermitian update: W[t][2j] = -Re F, W[t][2j+1] = -Im F,
// so that -pref sum_t W rho rho^H gives A_j = pref sum Re F rho rho^H and B_j likewise,
// chi0(w_j) = A_j + i B_j.
template <typename T>
__global__ void pole_factors_real(const double* __restrict__ dE, int nt, const double* __restrict__ w, int nwc,
                                  double eta, int nwpad, T* __restrict__ W, int* __restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const double d = dE[t];
  if (!(d > 0.0) && bad) atomicAdd(bad, 1);
  const double e2 = eta * eta;
  for (int j = 0; j < nwpad / 2; ++j) {
    double re = 0.0, im = 0.0;
    if (j < nwc) {
      const double a1 = w[j] - d, a2 = w[j] + d;
      const double i1 = 1.0 / (a1 * a1 + e2), i2 = 1.0 / (a2 * a2 + e2);
      re = a1 * i1 - a2 * i2;
      im = -eta * (i1 + i2);
    }
    W[(size_t)t * nwpad + 2 * j] = (T)(-re);
    W[(size_t)t * nwpad + 2 * j + 1] = (T)(-im);
  }
}

// out[j] (+)= A_j + i B_j from the Hermitian pair (A_j, B_j) in slots 2j, 2j + 1.
__global__ void chi0_combine_real(const double* __restrict__ AB, int ng, int nwc, int accumulate,
                                  double* __restrict__ out) {
  const size_t nn = (size_t)ng * ng;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= nn || j >= nwc) return;
  const double* A = AB + ((size_t)(2 * j) * nn + e) * 2;
  const double* B = AB + ((size_t)(2 * j + 1) * nn + e) * 2;
  double* o = out + ((size_t)j * nn + e) * 2;
  const double re = A[0] - B[1], im = A[1] + B[0];
  if (accumulate) {
    o[0] += re;
    o[1] += im;
  } else {
    o[0] = re;
    o[1] = im;
  }
}

__global__ void zero_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

struct Item {
  const void* rho;  // [nt][ng] complex T
  const void* W;    // [nt][nwpad] T
  double* chi0;     // [nw][ng][ng] complex128
  double pref;
  int nt, ng, nwpad, nw;
  int tile0;        // first entry of this item in the block-pair table
  int accumulate;
};

struct Unit {
  int item, tile, w0, k0, k1;
};

// One wave's share of a unit: its own transition slice of one 16 x (16 NT) block.
template <int MODE, int NWG, int NT>
__device__ __forceinline__ void unit_wave(const Item& I, int2 bij, int w0, int kb, int ke, int lane,
                                          float* __restrict__ outf, double* __restrict__ outd) {
  const int i = lane & 15;
  const int Gi = bij.x * kTile + i;
  const bool gi_ok = Gi < I.ng;
  if constexpr (is_bf(MODE)) {
    constexpr int NP = nprod(MODE);
    const int q = lane >> 4;  // lane holds k = 8q .. 8q+7 -> transitions 4q .. 4q+3, (re, im)
    const cplx<float>* rho = static_cast<const cplx<float>*>(I.rho);
    const float* W = static_cast<const float*>(I.W) + w0;
    f4 acc[NWG][2][NT];
#pragma unroll
    for (int w = 0; w < NWG; ++w)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[w][r][n] = f4{0, 0, 0, 0};
    for (int s = kb; s < ke; s += 16) {
      cplx<float> ra[4];
      float wt[4][NWG];
      uint32_t bhh[NT][4], bll[NT][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = s + 4 * q + u;
        const bool tv = t < ke;
        ra[u] = (tv && gi_ok) ? rho[(size_t)t * I.ng + Gi] : cplx<float>{0.f, 0.f};
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const int Gj = bij.y * kTile * NT + 16 * n + i;
          const cplx<float> rb = (tv && Gj < I.ng) ? rho[(size_t)t * I.ng + Gj] : cplx<float>{0.f, 0.f};
          split2(rb.x, rb.y, bhh[n][u], bll[n][u]);
        }
#pragma unroll
        for (int w = 0; w < NWG; ++w) wt[u][w] = tv ? W[(size_t)t * I.nwpad + w] : 0.f;
      }
      u4 bh[NT], bl[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        bh[n] = u4{bhh[n][0], bhh[n][1], bhh[n][2], bhh[n][3]};
        bl[n] = u4{bll[n][0], bll[n][1], bll[n][2], bll[n][3]};
      }
#pragma unroll
      for (int w = 0; w < NWG; ++w) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) split2(wt[u][w] * ra[u].x, wt[u][w] * ra[u].y, h[u], l[u]);
        const u4 reh = u4{h[0], h[1], h[2], h[3]}, rel = u4{l[0], l[1], l[2], l[3]};
        const u4 imh = u4{rot_pos(h[0]), rot_pos(h[1]), rot_pos(h[2]), rot_pos(h[3])};
        const u4 iml = u4{rot_pos(l[0]), rot_pos(l[1]), rot_pos(l[2]), rot_pos(l[3])};
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          acc[w][0][n] = mma_np<NP>(reh, rel, bh[n], bl[n], acc[w][0][n]);
          acc[w][1][n] = mma_np<NP>(imh, iml, bh[n], bl[n], acc[w][1][n]);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < NWG; ++w)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            outf[((w * 2 + r) * NT + n) * 256 + (4 * q + e) * 16 + i] = acc[w][r][n][e];
  } else {
    typedef typename std::conditional<MODE == MODE_F64, double, float>::type T;
    typedef typename Acc<T>::type V4;
    const int kk = lane >> 4;
    const int a = kk & 1;
    const int tsub = kk >> 1;
    const int Gj = bij.y * kTile + i;
    const bool gj_ok = Gj < I.ng;
    const cplx<T>* rho = static_cast<const cplx<T>*>(I.rho);
    const T* W = static_cast<const T*>(I.W) + w0;
    V4 acc[NWG][2];
#pragma unroll
    for (int w = 0; w < NWG; ++w) {
      acc[w][0] = V4{0, 0, 0, 0};
      acc[w][1] = V4{0, 0, 0, 0};
    }
    // The next step's operands and weights are requested before this step's
    // products (software pipelining: the loads are in flight during the MFMAs).
    // Rows past the slice read the slice's last row with the left operand zeroed;
    // columns past the G-set read column 0 and land in outputs that are dropped.
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int Gic = gi_ok ? Gi : 0, Gjc = gj_ok ? Gj : 0;
    T2 ra, rb;
    T2 wt[NWG / 2 > 0 ? NWG / 2 : 1];
    T wt1 = T(0);
    bool tv = false;
    auto load = [&](int s) {
      const int t = s + tsub;
      tv = t < ke;
      const size_t row = (size_t)min(t, ke - 1);
      ra = gld<T2>(rho + row * I.ng + Gic);
      rb = gld<T2>(rho + row * I.ng + Gjc);
      if constexpr (NWG >= 2) {
#pragma unroll
        for (int w = 0; w < NWG / 2; ++w) wt[w] = gld<T2>(W + row * I.nwpad + 2 * w);
      } else {
        wt1 = gld<T>(W + row * I.nwpad);
      }
    };
    if (kb < ke) load(kb);
#pragma unroll 1
    for (int s = kb; s < ke; s += 2) {
      const T2 ca = tv ? ra : T2{T(0), T(0)}, cb = rb;
      T cw[NWG];
      if constexpr (NWG >= 2) {
#pragma unroll
        for (int w = 0; w < NWG / 2; ++w) {
          cw[2 * w] = wt[w].x;
          cw[2 * w + 1] = wt[w].y;
        }
      } else {
        cw[0] = wt1;
      }
      load(s + 2);  // clamped: the last step re-reads valid rows
      const T bval = a ? cb.y : cb.x;
      const T are = a ? ca.y : ca.x;
      const T aim = a ? -ca.x : ca.y;
#pragma unroll
      for (int w = 0; w < NWG; ++w) {
        acc[w][0] = mfma4(cw[w] * are, bval, acc[w][0]);
        acc[w][1] = mfma4(cw[w] * aim, bval, acc[w][1]);
      }
    }
    T* out = MODE == MODE_F64 ? reinterpret_cast<T*>(outd) : reinterpret_cast<T*>(outf);
#pragma unroll
    for (int w = 0; w < NWG; ++w)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[(w * 2 + r) * 256 + Acc<T>::row(kk, e) * 16 + i] = acc[w][r][e];
  }
}

// Persistent workgroups: take units from the queue until it is exhausted.
template <int MODE, int NWG, int NT>
__global__ void __launch_bounds__(256) chi0_units(const Item* __restrict__ items, const int2* __restrict__ tiles,
                                                  const Unit* __restrict__ units, const int* __restrict__ queue,
                                                  int nunits, int* __restrict__ counter, void* __restrict__ part) {
  __shared__ int su;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int PER = NWG * 2 * NT * 256;  // values per wave partial
  for (;;) {
    if (threadIdx.x == 0) su = atomicAdd(counter, 1);
    __syncthreads();
    const int qpos = __builtin_amdgcn_readfirstlane(su);
    __syncthreads();
    if (qpos >= nunits) break;
    const int uid = queue[qpos];
    const Unit U = units[uid];
    const Item I = items[U.item];
    const int2 bij = tiles[I.tile0 + U.tile];
    const int len = U.k1 - U.k0;
    int sub = (len + kWaves - 1) / kWaves;
    sub = (sub + 15) / 16 * 16;
    const int kb = min(U.k1, U.k0 + wave * sub), ke = min(U.k1, kb + sub);
    const size_t off = ((size_t)uid * kWaves + wave) * PER;
    unit_wave<MODE, NWG, NT>(I, bij, U.w0, kb, ke, lane, static_cast<float*>(part) + off,
                             static_cast<double*>(part) + off);
  }
}

struct Red {
  int item, tile, w0, u0, nu;
};

// Fixed-order sum of the partials of one output block, scale by -pref, write the
// block (upper triangle authoritative) and its Hermitian mirror.
template <typename T, int NWG, int NT>
__global__ void chi0_reduce(const Item* __restrict__ items, const int2* __restrict__ tiles,
                            const Red* __restrict__ reds, const T* __restrict__ part) {
  constexpr int PER = NWG * 2 * NT * 256;
  const Red R = reds[blockIdx.x];
  const int w = blockIdx.y;
  const Item I = items[R.item];
  if (R.w0 + w >= I.nw) return;
  const int2 bij = tiles[I.tile0 + R.tile];
  double* m = I.chi0 + (size_t)(R.w0 + w) * I.ng * I.ng * 2;
  for (int e2 = threadIdx.x; e2 < 256 * NT; e2 += blockDim.x) {
    const int n = e2 >> 8, e = e2 & 255;
    const int ii = e >> 4, jj = e & 15;
    const int G = bij.x * kTile + ii, Gp = bij.y * kTile * NT + 16 * n + jj;
    if (G >= I.ng || Gp >= I.ng || G > Gp) continue;
    double re = 0.0, im = 0.0;
    for (int u = 0; u < R.nu; ++u)
      for (int wv = 0; wv < kWaves; ++wv) {
        const T* p = part + ((size_t)(R.u0 + u) * kWaves + wv) * PER + (size_t)(w * 2) * NT * 256;
        re += (double)p[n * 256 + e];
        im += (double)p[(NT + n) * 256 + e];
      }
    re *= -I.pref;
    im *= -I.pref;
    if (G == Gp) im = 0.0;
    const size_t up = ((size_t)G * I.ng + Gp) * 2, lo = ((size_t)Gp * I.ng + G) * 2;
    if (I.accumulate) {
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
}

constexpr int kBlk = 64;
constexpr int kBW = 4;  // frequencies per unit in the block form
constexpr int kBlkPer = kBW * 2 * kBlk * kBlk;  // partial values per unit

// Block form of the bf16 update (NP = 3 split, 1 plain). A unit is a 64 x 64 output block of the
// Hermitian half, four frequencies and a transition slice; one workgroup of eight waves runs two
// units of the same block and slice that hold consecutive frequency groups (waves 0-3 the first,
// 4-7 the second), so the raw left rows and the split right operand are loaded from the fabric
// and staged in LDS once for both. Wave r of a half owns rows 16 r .. 16 r + 15 and the four
// 16-column tiles (those inside the G-set and, in a diagonal block, on or above the diagonal).
// Each step of 64 transitions (four products deep) stages the raw left rows, the frequency
// factors of both groups and the right operand (split once, in fragment order), double buffered
// (137 KB of LDS) with one barrier per step: the next step is loaded into registers and stored
// in two halves of 32 transitions, each around two of the current step's four products. Each half writes its unit's partials (per thread, contiguous:
// [frequency][re, im][column tile] x 4 rows). A queue entry is a pair (u, v) of units, v = -1
// for a lone unit (its second half computes on the first unit's frequencies and writes nothing).
template <int NP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
chi0_blocks(const Item* __restrict__ items, const int2* __restrict__ tiles, const Unit* __restrict__ units,
           const int2* __restrict__ queue, const int* __restrict__ qoff, int* __restrict__ counters,
           float* __restrict__ part) {
  __shared__ u4 Bs[2][4][2][4][4][16];     // [buffer][quarter step][hi, lo][column tile][q][column]
  __shared__ float4 As[2][kBlk][33];       // [buffer][row][transition pair, + 1 pad]: raw rho of the block rows
  __shared__ float4 Ws[2][2 * kBW][16];    // [buffer][frequency of the pair][transition quad]
  __shared__ int su;
  const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
  const int w8 = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = w8 >> 2, wave = w8 & 3;                       // frequency group of the pair, row tile
  const int fn = (tid >> 6) & 3, fq = (tid >> 4) & 3, fj = tid & 15, fh = tid >> 8;  // right-operand slot
  const int ar = tid & 63, aq = tid >> 6;                        // left-operand row and transition quad
  int home = blockIdx.x & 7, misses = 0;
  for (;;) {
    if (tid == 0) {
      int p = -1;
      while (misses < 8) {
        const int c = qoff[home] + atomicAdd(&counters[home], 1);
        if (c < qoff[home + 1]) {
          p = c;
          misses = 0;
          break;
        }
        home = (home + 1) & 7;
        ++misses;
      }
      su = p;
    }
    __syncthreads();
    const int qpos = __builtin_amdgcn_readfirstlane(su);
    __syncthreads();
    if (qpos < 0) break;
    const int2 pr = queue[qpos];
    const Unit U = units[pr.x];
    const int w0b = pr.y >= 0 ? units[pr.y].w0 : U.w0;
    const Item I = items[U.item];
    const int2 bij = tiles[I.tile0 + U.tile];
    const int ng = I.ng, len = U.k1 - U.k0;
    const int nsteps = (len + 63) / 64;  // steps of 64 transitions, four products deep, staged in two halves
    int nmask = 0;
#pragma unroll
    for (int n = 0; n < 4; ++n)
      if (bij.x * kBlk + 16 * wave < ng && bij.y * kBlk + 16 * n < ng && (bij.x != bij.y || n >= wave))
        nmask |= 1 << n;
    const char* rbase = static_cast<const char*>(I.rho) + (size_t)U.k0 * ng * sizeof(f2v);
    const unsigned rstep = 32u * ng * sizeof(f2v), wstep = 32u * I.nwpad * sizeof(float);  // per half step
    const unsigned Ga = min(bij.x * kBlk + ar, ng - 1), Gb = min(bij.y * kBlk + 16 * fn + fj, ng - 1);
    const unsigned amax = ((unsigned)(len - 1) * ng + Ga) * sizeof(f2v);
    const unsigned bmax = ((unsigned)(len - 1) * ng + Gb) * sizeof(f2v);
    unsigned oa[4], ob[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      oa[u] = ((unsigned)(4 * aq + u) * ng + Ga) * sizeof(f2v);
      ob[u] = ((unsigned)(16 * fh + 4 * fq + u) * ng + Gb) * sizeof(f2v);
    }
    // frequency factors: transition wt, frequency wf of the pair (threads 0..255 load and store)
    const int wt = tid & 31, wf = (tid >> 5) & 7;
    const int wcol = (wf >> 2 ? w0b : U.w0) + (wf & 3);
    const char* wbase = static_cast<const char*>(I.W) + ((size_t)U.k0 * I.nwpad + wcol) * sizeof(float);
    const unsigned ow = (unsigned)wt * I.nwpad * sizeof(float);
    const unsigned wmax = (unsigned)(len - 1) * I.nwpad * sizeof(float);
    f2v raA[4], rbA[4];
    float wvA = 0.f;
#define CHI0_PAIR_LOAD(s_, ra_, rb_, wv_)                                                    \
    {                                                                                        \
      const unsigned d_ = (unsigned)(s_) * rstep;  /* s_: half step */                      \
      _Pragma("unroll") for (int u = 0; u < 4; ++u) {                                        \
        ra_[u] = gld<f2v>(rbase + min(oa[u] + d_, amax));                                    \
        rb_[u] = gld<f2v>(rbase + min(ob[u] + d_, bmax));                                    \
      }                                                                                      \
      wv_ = gld<float>(wbase + min(ow + (unsigned)(s_) * wstep, wmax));                      \
    }
#define CHI0_PAIR_STORE(b_, s_, ra_, rb_, wv_)                                               \
    {                                                                                        \
      const int hh_ = (s_) & 1;  /* half of the buffer */                                    \
      uint32_t h_[4], l_[4];                                                                 \
      _Pragma("unroll") for (int u = 0; u < 4; ++u) split2(rb_[u].x, rb_[u].y, h_[u], l_[u]); \
      Bs[b_][2 * hh_ + fh][0][fn][fq][fj] = u4{h_[0], h_[1], h_[2], h_[3]};                  \
      if constexpr (NP == 3)                                                                 \
        Bs[b_][2 * hh_ + fh][1][fn][fq][fj] = u4{l_[0], l_[1], l_[2], l_[3]};                \
      else                                                                                   \
        Bs[b_][2 * hh_ + fh][1][fn][fq][fj] = u4{rot_neg(h_[0]), rot_neg(h_[1]), rot_neg(h_[2]), rot_neg(h_[3])}; \
      As[b_][ar][16 * hh_ + 2 * aq] = make_float4(ra_[0].x, ra_[0].y, ra_[1].x, ra_[1].y);   \
      As[b_][ar][16 * hh_ + 2 * aq + 1] = make_float4(ra_[2].x, ra_[2].y, ra_[3].x, ra_[3].y); \
      if (tid < 256) reinterpret_cast<float*>(&Ws[b_][wf][0])[32 * hh_ + wt] = 32 * (s_) + wt < len ? wv_ : 0.f; \
    }
    f4 acc[kBW][2][4];
#pragma unroll
    for (int w = 0; w < kBW; ++w)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[w][r][n] = f4{0.f, 0.f, 0.f, 0.f};
    auto products = [&](int buf, int hs) {
      if (!nmask) return;
      const float4 a01 = As[buf][16 * wave + i][8 * hs + 2 * q], a23 = As[buf][16 * wave + i][8 * hs + 2 * q + 1];
      u4 ah[kBW], al[kBW];
#pragma unroll
      for (int w = 0; w < kBW; ++w) {
        const float4 wq = Ws[buf][4 * half + w][4 * hs + q];
        uint32_t h[4], l[4];
        split2(wq.x * a01.x, wq.x * a01.y, h[0], l[0]);
        split2(wq.y * a01.z, wq.y * a01.w, h[1], l[1]);
        split2(wq.z * a23.x, wq.z * a23.y, h[2], l[2]);
        split2(wq.w * a23.z, wq.w * a23.w, h[3], l[3]);
        ah[w] = u4{h[0], h[1], h[2], h[3]};
        al[w] = u4{l[0], l[1], l[2], l[3]};
      }
      u4 b0 = Bs[buf][hs][0][0][q][i], b1 = Bs[buf][hs][1][0][q][i];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        u4 nb0 = b0, nb1 = b1;
        if (n < 3) {
          nb0 = Bs[buf][hs][0][n + 1][q][i];
          nb1 = Bs[buf][hs][1][n + 1][q][i];
        }
        if (nmask & (1 << n)) {
          if constexpr (NP == 3) {
            u4 rh, rl;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              rh[m] = rot_neg(b0[m]);
              rl[m] = rot_neg(b1[m]);
            }
#pragma unroll
            for (int w = 0; w < kBW; ++w) {
              acc[w][0][n] = mma3(ah[w], al[w], b0, b1, acc[w][0][n]);
              acc[w][1][n] = mma3(ah[w], al[w], rh, rl, acc[w][1][n]);
            }
          } else {
#pragma unroll
            for (int w = 0; w < kBW; ++w) {
              acc[w][0][n] = mma(ah[w], b0, acc[w][0][n]);
              acc[w][1][n] = mma(ah[w], b1, acc[w][1][n]);
            }
          }
        }
        b0 = nb0;
        b1 = nb1;
      }
    };
    // half steps 2 k and 2 k + 1 fill buffer k % 2; the next step's halves are loaded and
    // stored one after the other around the current step's two pairs of products
    CHI0_PAIR_LOAD(0, raA, rbA, wvA);
    CHI0_PAIR_STORE(0, 0, raA, rbA, wvA);
    CHI0_PAIR_LOAD(1, raA, rbA, wvA);
    CHI0_PAIR_STORE(0, 1, raA, rbA, wvA);
    __syncthreads();
    for (int k = 0; k < nsteps; ++k) {
      const int buf = k & 1;
      const bool more = k + 1 < nsteps;
#pragma unroll 1
      for (int hh = 0; hh < 2; ++hh) {
        if (more) CHI0_PAIR_LOAD(2 * k + 2 + hh, raA, rbA, wvA);
        products(buf, 2 * hh);
        products(buf, 2 * hh + 1);
        if (more) CHI0_PAIR_STORE(buf ^ 1, 2 * k + 2 + hh, raA, rbA, wvA);
      }
      __syncthreads();
    }
#undef CHI0_PAIR_LOAD
#undef CHI0_PAIR_STORE
    const int uid = half ? pr.y : pr.x;
    if (uid >= 0) {
      f4* out = reinterpret_cast<f4*>(part + ((size_t)uid * 256 + (tid & 255)) * (kBW * 2 * 4 * 4));
#pragma unroll
      for (int w = 0; w < kBW; ++w)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int n = 0; n < 4; ++n) out[(w * 2 + r) * 4 + n] = acc[w][r][n];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Strip form of the bf16 update (NP = 3 split, 1 plain). A unit is a 64-row x 128-column
// block, two frequencies and a transition slice; four waves, wave r owns rows 16 r .. + 15
// and all eight 16-column tiles (2 frequencies x (re, im) x 8 tiles: 32 accumulators). Each
// weighted, split left-operand value feeds eight column tiles instead of four, so the split
// costs half as many instructions per product as in the 64 x 64 form; Im takes the
// rotation (im, -re) of the left operand, converted in the same split from the same
// products, so the right operand enters the products as staged. The staging, the
// transition steps and the loads follow chi0_blocks.
constexpr int kSRows = 64, kSCols = 128, kSF = 2;
constexpr int kSPer = kSF * 2 * kSRows * kSCols;  // partial values per unit (128 per thread)

template <int NP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
chi0_strips(const Item* __restrict__ items, const int2* __restrict__ tiles, const Unit* __restrict__ units,
            const int* __restrict__ queue, const int* __restrict__ qoff, int* __restrict__ counters,
            float* __restrict__ part) {
  constexpr int PB = NP == 3 ? 2 : 1;
  __shared__ u4 Bs[2][PB][8][4][16];   // [buffer][hi, lo][column tile][q][column]
  __shared__ float4 As[2][kSRows][9];  // [buffer][row][transition pair, + 1 pad]: raw rho of the block rows
  __shared__ float4 Ws[2][kSF][4];     // [buffer][frequency][transition quad]
  __shared__ int su;
  const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bc = tid & 127, bh = tid >> 7;  // right-operand slot: column bc, transitions 8 bh .. + 7
  const int ar = tid & 63, aq = tid >> 6;   // left-operand slot: row ar, transitions 4 aq .. + 3
  // queue segments per XCD, as for chi0_blocks
  int home = blockIdx.x & 7, misses = 0;
  for (;;) {
    if (tid == 0) {
      int p = -1;
      while (misses < 8) {
        const int c = qoff[home] + atomicAdd(&counters[home], 1);
        if (c < qoff[home + 1]) {
          p = c;
          misses = 0;
          break;
        }
        home = (home + 1) & 7;
        ++misses;
      }
      su = p;
    }
    __syncthreads();
    const int qpos = __builtin_amdgcn_readfirstlane(su);
    __syncthreads();
    if (qpos < 0) break;
    const int uid = queue[qpos];
    const Unit U = units[uid];
    const Item I = items[U.item];
    const int2 bij = tiles[I.tile0 + U.tile];
    const int ng = I.ng, len = U.k1 - U.k0;
    const int nsteps = (len + 15) / 16;
    // 16 x 16 tiles of this wave: inside the G-set and not wholly below the diagonal
    const int r0 = bij.x * kSRows + 16 * wave;
    int nmask = 0;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const int c0 = bij.y * kSCols + 16 * n;
      if (r0 < ng && c0 < ng && c0 >= r0) nmask |= 1 << n;
    }
    // Loads address the unit's transition slice by 32-bit byte offsets (the host keeps
    // len * ng * 8 below 2^31); rows past the slice and G past the G-set are clamped to
    // valid entries: the former carry a zero weight, the latter land in outputs the
    // reduction drops.
    const char* rbase = static_cast<const char*>(I.rho) + (size_t)U.k0 * ng * sizeof(f2v);
    const char* wbase = static_cast<const char*>(I.W) + ((size_t)U.k0 * I.nwpad + U.w0) * sizeof(float);
    const unsigned trow = (unsigned)ng * sizeof(f2v), rstep = 16u * trow, wstep = 16u * I.nwpad * sizeof(float);
    const unsigned Ga = min(bij.x * kSRows + ar, ng - 1), Gb = min(bij.y * kSCols + bc, ng - 1);
    const unsigned amax = ((unsigned)(len - 1) * ng + Ga) * sizeof(f2v);
    const unsigned bmax = ((unsigned)(len - 1) * ng + Gb) * sizeof(f2v);
    const unsigned oa = ((unsigned)(4 * aq) * ng + Ga) * sizeof(f2v);
    const unsigned ob = ((unsigned)(8 * bh) * ng + Gb) * sizeof(f2v);
    // frequency factors: transition wt, frequency wf of the unit's two (every wave issues
    // the same loads; the first 32 threads store them); rows past the slice read its last
    // row and are zeroed when stored
    const int wt = tid & 15, wf = (tid >> 4) & 1;
    const unsigned ow = ((unsigned)wt * I.nwpad + wf) * sizeof(float);
    const unsigned wmax = ((unsigned)(len - 1) * I.nwpad + wf) * sizeof(float);

    f2v raA[4], rbA[8], raB[4], rbB[8];
    float wvA = 0.f, wvB = 0.f;
    // ---- load step s into register set (ra, rb, wv)
#define CHI0_STR_LOAD(s_, ra_, rb_, wv_)                                                    \
    {                                                                                       \
      const unsigned d_ = (unsigned)(s_) * rstep;                                           \
      _Pragma("unroll") for (int u = 0; u < 4; ++u) ra_[u] = gld<f2v>(rbase + min(oa + (d_ + u * trow), amax)); \
      _Pragma("unroll") for (int u = 0; u < 8; ++u) rb_[u] = gld<f2v>(rbase + min(ob + (d_ + u * trow), bmax)); \
      wv_ = gld<float>(wbase + min(ow + (unsigned)(s_) * wstep, wmax));                     \
    }
    // ---- store step s from register set (ra, rb, wv) into buffer b
#define CHI0_STR_STORE(b_, s_, ra_, rb_, wv_)                                               \
    {                                                                                       \
      _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                       \
        uint32_t h_[4], l_[4];                                                              \
        _Pragma("unroll") for (int u = 0; u < 4; ++u) split2(rb_[4 * h + u].x, rb_[4 * h + u].y, h_[u], l_[u]); \
        Bs[b_][0][bc >> 4][2 * bh + h][bc & 15] = u4{h_[0], h_[1], h_[2], h_[3]};           \
        if constexpr (NP == 3) Bs[b_][1][bc >> 4][2 * bh + h][bc & 15] = u4{l_[0], l_[1], l_[2], l_[3]}; \
      }                                                                                     \
      As[b_][ar][2 * aq] = make_float4(ra_[0].x, ra_[0].y, ra_[1].x, ra_[1].y);              \
      As[b_][ar][2 * aq + 1] = make_float4(ra_[2].x, ra_[2].y, ra_[3].x, ra_[3].y);          \
      if (tid < 32) reinterpret_cast<float*>(&Ws[b_][wf][0])[wt] = 16 * (s_) + wt < len ? wv_ : 0.f; \
    }
    f4 acc[kSF][2][8];
#pragma unroll
    for (int f = 0; f < kSF; ++f)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int n = 0; n < 8; ++n) acc[f][r][n] = f4{0.f, 0.f, 0.f, 0.f};
    // products of the step held in buffer buf
    auto products = [&](int buf) {
      if (!nmask) return;
      // weighted left operand of both frequencies and its rotation, converted once and
      // shared by the eight column tiles
      const float4 a01 = As[buf][16 * wave + i][2 * q], a23 = As[buf][16 * wave + i][2 * q + 1];
      u4 ah[kSF], al[kSF], rh[kSF], rl[kSF];
#pragma unroll
      for (int f = 0; f < kSF; ++f) {
        const float4 wq = Ws[buf][f][q];
        uint32_t h[4], l[4], x[4], y[4];
        split2_rot(wq.x * a01.x, wq.x * a01.y, h[0], l[0], x[0], y[0]);
        split2_rot(wq.y * a01.z, wq.y * a01.w, h[1], l[1], x[1], y[1]);
        split2_rot(wq.z * a23.x, wq.z * a23.y, h[2], l[2], x[2], y[2]);
        split2_rot(wq.w * a23.z, wq.w * a23.w, h[3], l[3], x[3], y[3]);
        ah[f] = u4{h[0], h[1], h[2], h[3]};
        al[f] = u4{l[0], l[1], l[2], l[3]};
        rh[f] = u4{x[0], x[1], x[2], x[3]};
        rl[f] = u4{y[0], y[1], y[2], y[3]};
      }
      // column tiles: Re through the left operand, Im through its rotation; the next
      // tile's right operand is read ahead of the products
      u4 b0 = Bs[buf][0][0][q][i], b1 = b0;
      if constexpr (NP == 3) b1 = Bs[buf][1][0][q][i];
#pragma unroll
      for (int n = 0; n < 8; ++n) {
        u4 nb0 = b0, nb1 = b1;
        if (n < 7) {
          nb0 = Bs[buf][0][n + 1][q][i];
          if constexpr (NP == 3) nb1 = Bs[buf][1][n + 1][q][i];
        }
        if (nmask & (1 << n)) {
#pragma unroll
          for (int f = 0; f < kSF; ++f) {
            acc[f][0][n] = mma_np<NP>(ah[f], al[f], b0, b1, acc[f][0][n]);
            acc[f][1][n] = mma_np<NP>(rh[f], rl[f], b0, b1, acc[f][1][n]);
          }
        }
        b0 = nb0;
        b1 = nb1;
      }
    };
    CHI0_STR_LOAD(0, raA, rbA, wvA);
    CHI0_STR_STORE(0, 0, raA, rbA, wvA);
    if constexpr (NP == 1) {
      // step k sits in buffer k % 2; entering an even k, step k + 1 is in set B and
      // step k + 2 in set A
      CHI0_STR_LOAD(1, raB, rbB, wvB);
      CHI0_STR_LOAD(2, raA, rbA, wvA);
      __syncthreads();
      for (int k = 0; k < nsteps; k += 2) {
        products(0);
        if (k + 1 < nsteps) CHI0_STR_STORE(1, k + 1, raB, rbB, wvB);
        __syncthreads();
        if (k + 1 >= nsteps) break;
        CHI0_STR_LOAD(k + 3, raB, rbB, wvB);
        products(1);
        if (k + 2 < nsteps) CHI0_STR_STORE(0, k + 2, raA, rbA, wvA);
        __syncthreads();
        CHI0_STR_LOAD(k + 4, raA, rbA, wvA);
      }
    } else {
      // the split form has no registers for a second set: one step ahead
      __syncthreads();
      for (int k = 0; k < nsteps; ++k) {
        const int buf = k & 1;
        if (k + 1 < nsteps) CHI0_STR_LOAD(k + 1, raA, rbA, wvA);
        products(buf);
        if (k + 1 < nsteps) CHI0_STR_STORE(buf ^ 1, k + 1, raA, rbA, wvA);
        __syncthreads();
      }
    }
#undef CHI0_STR_LOAD
#undef CHI0_STR_STORE
    // partials of this thread, contiguous: [frequency][re, im][column tile] x 4 rows
    f4* out = reinterpret_cast<f4*>(part + ((size_t)uid * 256 + tid) * (kSF * 2 * 8 * 4));
#pragma unroll
    for (int f = 0; f < kSF; ++f)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int n = 0; n < 8; ++n) out[(f * 2 + r) * 8 + n] = acc[f][r][n];
  }
}

// Write one reduced element of the upper half and its Hermitian mirror: chi0 = -pref * sum.
__device__ __forceinline__ void put_pair(const Item& I, double* m, int G, int Gp, double sre, double sim) {
  const double vr = -I.pref * sre;
  const double vi = G == Gp ? 0.0 : -I.pref * sim;
  const size_t up = ((size_t)G * I.ng + Gp) * 2, lo = ((size_t)Gp * I.ng + G) * 2;
  if (I.accumulate) {
    m[up] += vr;
    m[up + 1] += vi;
    if (G != Gp) {
      m[lo] += vr;
      m[lo + 1] -= vi;
    }
  } else {
    m[up] = vr;
    m[up + 1] = vi;
    if (G != Gp) {
      m[lo] = vr;
      m[lo + 1] = -vi;
    }
  }
}

// Fixed-order sum of the strip partials of one output block and frequency. Thread t reads
// what thread t of chi0_strips wrote: rows 16 (t / 64) + 4 q + e, columns 16 n + i, with
// i = t % 16, q = (t % 64) / 16.
__global__ void __launch_bounds__(256) chi0_reduce_strips(const Item* __restrict__ items,
                                                          const int2* __restrict__ tiles,
                                                          const Red* __restrict__ reds,
                                                          const float* __restrict__ part) {
  const Red R = reds[blockIdx.x];
  const int w = blockIdx.y;
  const Item I = items[R.item];
  if (R.w0 + w >= I.nw) return;
  const int2 bij = tiles[I.tile0 + R.tile];
  const int t = threadIdx.x, i = t & 15, q = (t >> 4) & 3, wave = t >> 6;
  double re[8][4], im[8][4];
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int e = 0; e < 4; ++e) re[n][e] = im[n][e] = 0.0;
  for (int u = 0; u < R.nu; ++u) {
    const f4* p = reinterpret_cast<const f4*>(part + ((size_t)(R.u0 + u) * 256 + t) * (kSF * 2 * 8 * 4)) + w * 16;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const f4 a = p[n], b = p[8 + n];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        re[n][e] += (double)a[e];
        im[n][e] += (double)b[e];
      }
    }
  }
  double* m = I.chi0 + (size_t)(R.w0 + w) * I.ng * I.ng * 2;
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int G = bij.x * kSRows + 16 * wave + 4 * q + e, Gp = bij.y * kSCols + 16 * n + i;
      if (G >= I.ng || Gp >= I.ng || G > Gp) continue;
      put_pair(I, m, G, Gp, re[n][e], im[n][e]);
    }
}

// Fixed-order sum of the block partials of one output block and frequency. Thread
// t reads what thread t of the block kernel wrote: rows 16 (t / 64) + 4 q + e,
// columns 16 n + i, with i = t % 16, q = (t % 64) / 16.
__global__ void __launch_bounds__(256) chi0_reduce_blocks(const Item* __restrict__ items,
                                                          const int2* __restrict__ tiles, const Red* __restrict__ reds,
                                                          const float* __restrict__ part) {
  const Red R = reds[blockIdx.x];
  const int w = blockIdx.y;
  const Item I = items[R.item];
  if (R.w0 + w >= I.nw) return;
  const int2 bij = tiles[I.tile0 + R.tile];
  const int t = threadIdx.x, i = t & 15, q = (t >> 4) & 3, wave = t >> 6;
  double re[4][4], im[4][4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int e = 0; e < 4; ++e) re[n][e] = im[n][e] = 0.0;
  for (int u = 0; u < R.nu; ++u) {
    const f4* p = reinterpret_cast<const f4*>(part + ((size_t)(R.u0 + u) * 256 + t) * (kBW * 2 * 4 * 4)) + w * 8;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const f4 a = p[n], b = p[4 + n];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        re[n][e] += (double)a[e];
        im[n][e] += (double)b[e];
      }
    }
  }
  double* m = I.chi0 + (size_t)(R.w0 + w) * I.ng * I.ng * 2;
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int G = bij.x * kBlk + 16 * wave + 4 * q + e, Gp = bij.y * kBlk + 16 * n + i;
      if (G >= I.ng || Gp >= I.ng || G > Gp) continue;
      put_pair(I, m, G, Gp, re[n][e], im[n][e]);
    }
}

// --------------------------------------------------------------- host side --

// Default form of the bf16 updates: the 64 x 64 blocks (4) unless XO_CHI0_FORM=strips
// (the 64 x 128 strips, 8).
int default_block_form() {
  const char* e = std::getenv("XO_CHI0_FORM");
  if (e && !std::strcmp(e, "strips")) return 8;
  return 4;
}

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

static int validate(const xo_chi0_args* a, bool signed_pref) {
  XO_ARG(a, "xo_chi0: null argument block");
  XO_ARG(a->nt > 0 && a->ng > 0 && a->nw > 0, "xo_chi0: sizes must be positive (nt=%d ng=%d nw=%d)", a->nt,
         a->ng, a->nw);
  XO_ARG(a->nw <= 64, "xo_chi0: at most 64 frequencies per call (got %d)", a->nw);
  XO_ARG(a->rho && a->dE && a->w && a->chi0, "xo_chi0: null pointer");
  XO_ARG(a->prec == XO_FP64 || a->prec == XO_FP32 || a->prec == XO_BF16X3 || a->prec == XO_BF16,
         "xo_chi0: bad precision %d", a->prec);
  for (int j = 0; j < a->nw; ++j) XO_ARG(a->w[j] >= 0.0, "xo_chi0: frequency %d is negative", j);
  XO_ARG(signed_pref ? (a->pref != 0.0 && std::isfinite(a->pref)) : a->pref > 0.0, "xo_chi0: pref must be positive");
  return XO_OK;
}

template <int MODE, int NWG, int NT>
static int launch_units(const void* ditems, const void* dtiles, const void* dunits, const void* dqueue, int nunits,
                        int* counter, void* part, const void* dreds, int nreds, int grid, hipStream_t s) {
  typedef typename std::conditional<MODE == MODE_F64, double, float>::type T;
  hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, counter, 1);
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_(MODE == MODE_BF16X3 ? "chi0_tiles_bf16x3" : (MODE == MODE_BF16 ? "chi0_tiles_bf16" : "chi0_tiles"),
                    s);
    hipLaunchKernelGGL((chi0_units<MODE, NWG, NT>), dim3(grid), dim3(256), 0, s,
                       static_cast<const Item*>(ditems), static_cast<const int2*>(dtiles),
                       static_cast<const Unit*>(dunits), static_cast<const int*>(dqueue), nunits, counter, part);
  }
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_("chi0_reduce", s);
    hipLaunchKernelGGL((chi0_reduce<T, NWG, NT>), dim3(nreds, NWG), dim3(256), 0, s,
                       static_cast<const Item*>(ditems), static_cast<const int2*>(dtiles),
                       static_cast<const Red*>(dreds), static_cast<const T*>(part));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <int MODE, int NWG>
static int launch_nt(int nt_tiles, const void* ditems, const void* dtiles, const void* dunits, const void* dqueue,
                     int nunits, int* counter, void* part, const void* dreds, int nreds, int grid, hipStream_t s) {
  if constexpr (is_bf(MODE)) {
    if (nt_tiles == 2)
      return launch_units<MODE, NWG, 2>(ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid,
                                        s);
  }
  return launch_units<MODE, NWG, 1>(ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid, s);
}

template <int MODE>
static int launch_nwg(int nwg, int nt_tiles, const void* ditems, const void* dtiles, const void* dunits,
                      const void* dqueue, int nunits, int* counter, void* part, const void* dreds, int nreds,
                      int grid, hipStream_t s) {
  switch (nwg) {
    case 8:
      return launch_nt<MODE, 8>(nt_tiles, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid, s);
    case 4:
      return launch_nt<MODE, 4>(nt_tiles, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid, s);
    case 2:
      return launch_nt<MODE, 2>(nt_tiles, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid, s);
    default:
      return launch_nt<MODE, 1>(nt_tiles, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid, s);
  }
}

// Every item of a batch shares the precision and the frequencies.
// With wreal set (host, nw / 2 real frequencies) the nw slots carry the real-axis factor
// pairs of pole_factors_real instead of the imaginary-axis factors.
// With size_only set, the call stops after planning (host work only) and stores there the
// workspace bytes it would request.
static int chi0_batch_run(const xo_chi0_args* a, int n, const xo_tune* tune, hipStream_t s,
                          bool signed_pref = false, const double* wreal = nullptr, double eta = 0.0,
                          size_t* size_only = nullptr) {
  for (int i = 0; i < n; ++i) XO_RET(validate(&a[i], signed_pref));
  const int prec = a[0].prec;
  for (int i = 1; i < n; ++i) {
    XO_ARG(a[i].prec == prec && a[i].nw == a[0].nw, "xo_chi0_batch: items must share precision and frequencies");
    for (int j = 0; j < a[0].nw; ++j)
      XO_ARG(a[i].w[j] == a[0].w[j], "xo_chi0_batch: items must share the frequency list");
  }
  const int mode = prec == XO_FP64 ? MODE_F64 : (prec == XO_FP32 ? MODE_F32 : (prec == XO_BF16 ? MODE_BF16 : MODE_BF16X3));
  const size_t tsz = mode == MODE_F64 ? sizeof(double) : sizeof(float);
  const int nw = a[0].nw;
  // bf16 forms: the 64 x 64 block form (nt_tiles 4, four frequencies per unit) or the
  // 64 x 128 strip form (nt_tiles 8, two frequencies per unit) once there are four
  // frequencies; XO_CHI0_FORM=blocks|strips picks the default between the two
  const int pick = (tune && tune->nt_tiles) ? tune->nt_tiles : (nw >= kBW ? default_block_form() : 1);
  const bool blk = is_bf(mode) && (pick == 4 || pick == 8);
  const bool str = blk && pick == 8;
  const int nwg = str ? kSF : (blk ? kBW : (nw >= 8 ? 8 : (nw >= 4 ? 4 : (nw >= 2 ? 2 : 1))));
  const int ngroups = (nw + nwg - 1) / nwg;
  const int nwpad = ngroups * nwg;
  const int NT = (tune && is_bf(mode) && tune->nt_tiles == 2) ? 2 : 1;
  const int grid_per_cu = (tune && tune->wg_per_cu > 0) ? tune->wg_per_cu : (blk ? 2 : 4);
  const int brow = str ? kSRows : (blk ? kBlk : kTile), bcol = str ? kSCols : (blk ? kBlk : kTile * NT);

  // block pairs: brow-row block i, bcol-column block j, keeping those with a column >= a row
  std::vector<int2> tiles;
  std::vector<Item> items(n);
  std::vector<int> ntl(n);
  std::vector<size_t> woff(n);
  size_t wbytes = 0;
  for (int it = 0; it < n; ++it) {
    const int ng = a[it].ng;
    const int nbr = (ng + brow - 1) / brow, nbc = (ng + bcol - 1) / bcol;
    items[it].tile0 = (int)tiles.size();
    for (int i = 0; i < nbr; ++i)
      for (int j = 0; j < nbc; ++j)
        if (j * bcol + bcol - 1 >= i * brow) tiles.push_back(make_int2(i, j));
    ntl[it] = (int)tiles.size() - items[it].tile0;
    woff[it] = wbytes;
    wbytes += align_up((size_t)a[it].nt * nwpad * tsz, 256);
  }
  long total_blocks = 0;
  for (int it = 0; it < n; ++it) total_blocks += (long)ntl[it] * ngroups;
  // units: cut transitions so the batch holds about four units per persistent wave
  const long want_units = (long)num_cus() * grid_per_cu * 4;
  std::vector<Unit> units;
  std::vector<Red> reds;
  for (int it = 0; it < n; ++it) {
    int kper;
    if (tune && tune->kper > 0) {
      kper = tune->kper;
    } else {
      long slices = std::max(1L, (want_units + total_blocks - 1) / std::max(1L, total_blocks));
      if (blk) slices = (slices + 7) / 8 * 8;  // whole slices per XCD
      kper = (int)((a[it].nt + slices - 1) / slices);
    }
    kper = std::max(64, (kper + 63) / 64 * 64);
    // FP32 accumulators (FP32 and bf16 forms): at most kFp32Slice transitions per
    // unit, so the rounding of the running sums stays bounded and the FP64 reduction
    // adds many short partial sums
    if (mode != MODE_F64 && !(tune && tune->kper > 0)) kper = std::min(kper, kFp32Slice);
    // the block form addresses a slice by 32-bit byte offsets
    if (blk) kper = std::min(kper, std::max(64, (int)(((1u << 31) / (8u * a[it].ng) - 16) / 64 * 64)));
    for (int t = 0; t < ntl[it]; ++t)
      for (int g = 0; g < ngroups; ++g) {
        Red r;
        r.item = it;
        r.tile = t;
        r.w0 = g * nwg;
        r.u0 = (int)units.size();
        for (int k0 = 0; k0 < a[it].nt; k0 += kper)
          units.push_back({it, t, g * nwg, k0, std::min(a[it].nt, k0 + kper)});
        r.nu = (int)units.size() - r.u0;
        reds.push_back(r);
      }
  }
  // queue: costliest units first (transitions times the 16 x 16 tiles the block form
  // computes); among equal costs, transition slice first, so the units in flight
  // together read the same slice of every item's rho (cache reuse)
  auto tile_work = [&](const Unit& u) {
    if (!blk) return 16;
    const int2 b = tiles[items[u.item].tile0 + u.tile];
    const int ng = a[u.item].ng;
    int c = 0;
    if (str) {
      for (int r = 0; r < 4; ++r)
        for (int m = 0; m < 8; ++m) {
          const int r0 = b.x * kSRows + 16 * r, c0 = b.y * kSCols + 16 * m;
          c += r0 < ng && c0 < ng && c0 >= r0;
        }
      return c;
    }
    for (int r = 0; r < 4; ++r)
      for (int m = 0; m < 4; ++m)
        c += b.x * kBlk + 16 * r < ng && b.y * kBlk + 16 * m < ng && (b.x != b.y || m >= r);
    return c;
  };
  std::vector<long> cost(units.size());
  for (size_t u = 0; u < units.size(); ++u) cost[u] = (long)(units[u].k1 - units[u].k0) * tile_work(units[u]);
  std::vector<int> queue(units.size());
  for (size_t u = 0; u < units.size(); ++u) queue[u] = (int)u;
  std::stable_sort(queue.begin(), queue.end(), [&](int x, int y) {
    if (cost[x] != cost[y]) return cost[x] > cost[y];
    return units[x].k0 < units[y].k0;
  });
  // block form: the units of one (item, transition slice) go to one XCD, whose L2 then
  // serves that slice of rho to all of them; slices are dealt to the XCDs costliest first,
  // each to the XCD with the least work so far, and keep the order above inside a segment
  int qoff[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (blk) {
    std::map<std::pair<int, int>, long> gcost;
    for (size_t u = 0; u < units.size(); ++u) gcost[{units[u].item, units[u].k0}] += cost[u];
    std::vector<std::pair<long, std::pair<int, int>>> groups;
    for (const auto& g : gcost) groups.push_back({g.second, g.first});
    std::stable_sort(groups.begin(), groups.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    std::map<std::pair<int, int>, int> xcd_of;
    long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const auto& g : groups) {
      const int x = (int)(std::min_element(load, load + 8) - load);
      xcd_of[g.second] = x;
      load[x] += g.first;
    }
    std::vector<int> seg[8];
    for (int u : queue) seg[xcd_of[{units[u].item, units[u].k0}]].push_back(u);
    queue.clear();
    for (int x = 0; x < 8; ++x) {
      qoff[x] = (int)queue.size();
      queue.insert(queue.end(), seg[x].begin(), seg[x].end());
    }
    qoff[8] = (int)queue.size();
  }
  const int nunits = (int)units.size();
  const size_t per = str ? (size_t)kSPer * sizeof(float)
                         : (blk ? (size_t)kBlkPer * sizeof(float) : (size_t)kWaves * nwg * 2 * NT * 256 * tsz);
  const size_t pbytes = per * nunits;
  bool any_check = false;
  for (int it = 0; it < n; ++it) any_check |= a[it].check_dE != 0;
  if (size_only) {
    *size_only = wbytes + pbytes + 256 + (any_check ? 256 : 0);
    return XO_OK;
  }
  void* ws = nullptr;
  XO_RET(workspace(s, 1, wbytes + pbytes + 256, &ws));
  char* wbase = static_cast<char*>(ws);
  void* part = wbase + wbytes;
  int* counter = reinterpret_cast<int*>(wbase + wbytes + pbytes);

  int* bad = nullptr;
  if (any_check) {
    void* wsb = nullptr;
    XO_RET(workspace(s, 4, 256, &wsb));
    bad = static_cast<int*>(wsb);
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, bad, 1);
    XO_CHECK_LAUNCH();
  }
  const void* dw = nullptr;
  if (wreal)
    XO_RET(device_table(wreal, sizeof(double) * (nw / 2), s, &dw));
  else
    XO_RET(device_table(a[0].w, sizeof(double) * nw, s, &dw));
  for (int it = 0; it < n; ++it) {
    void* W = wbase + woff[it];
    const dim3 pg((a[it].nt + 255) / 256);
    if (wreal) {
      KernelTimer kt_("pole_factors_real", s);
      if (mode == MODE_F64)
        hipLaunchKernelGGL((pole_factors_real<double>), pg, dim3(256), 0, s, a[it].dE, a[it].nt,
                           static_cast<const double*>(dw), nw / 2, eta, nwpad, static_cast<double*>(W),
                           a[it].check_dE ? bad : nullptr);
      else
        hipLaunchKernelGGL((pole_factors_real<float>), pg, dim3(256), 0, s, a[it].dE, a[it].nt,
                           static_cast<const double*>(dw), nw / 2, eta, nwpad, static_cast<float*>(W),
                           a[it].check_dE ? bad : nullptr);
    } else {
      KernelTimer kt_("pole_factors", s);
      if (mode == MODE_F64)
        hipLaunchKernelGGL((pole_factors<double>), pg, dim3(256), 0, s, a[it].dE, a[it].nt,
                           static_cast<const double*>(dw), nw, nwpad, static_cast<double*>(W),
                           a[it].check_dE ? bad : nullptr);
      else
        hipLaunchKernelGGL((pole_factors<float>), pg, dim3(256), 0, s, a[it].dE, a[it].nt,
                           static_cast<const double*>(dw), nw, nwpad, static_cast<float*>(W),
                           a[it].check_dE ? bad : nullptr);
    }
    XO_CHECK_LAUNCH();
    items[it].rho = a[it].rho;
    items[it].W = W;
    items[it].chi0 = a[it].chi0;
    items[it].pref = a[it].pref;
    items[it].nt = a[it].nt;
    items[it].ng = a[it].ng;
    items[it].nwpad = nwpad;
    items[it].nw = nw;
    items[it].accumulate = a[it].accumulate;
  }
  if (any_check) {
    int* hb = nullptr;
    XO_RET(host_flags(s, sizeof(int), reinterpret_cast<void**>(&hb)));
    XO_TRY_HIP(hipMemcpyAsync(hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    XO_TRY_HIP(hipStreamSynchronize(s));
    XO_ARG(*hb == 0, "xo_chi0: %d pole energies dE are <= 0 or NaN", *hb);
  }
  const void *ditems = nullptr, *dtiles = nullptr, *dunits = nullptr, *dqueue = nullptr, *dreds = nullptr;
  XO_RET(device_table(items.data(), items.size() * sizeof(Item), s, &ditems));
  XO_RET(device_table(tiles.data(), tiles.size() * sizeof(int2), s, &dtiles));
  XO_RET(device_table(units.data(), units.size() * sizeof(Unit), s, &dunits));
  XO_RET(device_table(queue.data(), queue.size() * sizeof(int), s, &dqueue));
  XO_RET(device_table(reds.data(), reds.size() * sizeof(Red), s, &dreds));
  const int grid = std::min(nunits, num_cus() * grid_per_cu);
  const int nreds = (int)reds.size();
  if (blk) {
    const void* dqoff = nullptr;
    XO_RET(device_table(qoff, sizeof(qoff), s, &dqoff));
    hipLaunchKernelGGL(zero_ints, dim3(1), dim3(64), 0, s, counter, 8);
    XO_CHECK_LAUNCH();
    if (str) {
      {
        KernelTimer kt_(mode == MODE_BF16 ? "chi0_strips_bf16" : "chi0_strips_bf16x3", s);
        hipLaunchKernelGGL(mode == MODE_BF16 ? chi0_strips<1> : chi0_strips<3>, dim3(grid), dim3(256), 0, s,
                           static_cast<const Item*>(ditems), static_cast<const int2*>(dtiles),
                           static_cast<const Unit*>(dunits), static_cast<const int*>(dqueue),
                           static_cast<const int*>(dqoff), counter, static_cast<float*>(part));
      }
      XO_CHECK_LAUNCH();
      {
        KernelTimer kt_("chi0_reduce", s);
        hipLaunchKernelGGL(chi0_reduce_strips, dim3(nreds, kSF), dim3(256), 0, s, static_cast<const Item*>(ditems),
                           static_cast<const int2*>(dtiles), static_cast<const Red*>(dreds),
                           static_cast<const float*>(part));
      }
      XO_CHECK_LAUNCH();
      return XO_OK;
    }
    // pair the units of one block and slice that hold consecutive frequency groups (adjacent in
    // each XCD segment of the queue)
    std::vector<int2> pq;
    int qoff2[9];
    for (int x = 0; x < 8; ++x) {
      qoff2[x] = (int)pq.size();
      for (int i = qoff[x]; i < qoff[x + 1];) {
        const int u = queue[i];
        if (i + 1 < qoff[x + 1]) {
          const int v = queue[i + 1];
          if (units[v].item == units[u].item && units[v].tile == units[u].tile && units[v].k0 == units[u].k0 &&
              units[v].w0 == units[u].w0 + kBW) {
            pq.push_back(make_int2(u, v));
            i += 2;
            continue;
          }
        }
        pq.push_back(make_int2(u, -1));
        ++i;
      }
    }
    qoff2[8] = (int)pq.size();
    const void *dpq = nullptr, *dqoff2 = nullptr;
    XO_RET(device_table(pq.data(), pq.size() * sizeof(int2), s, &dpq));
    XO_RET(device_table(qoff2, sizeof(qoff2), s, &dqoff2));
    // eight-wave workgroups: half as many per CU as the four-wave forms
    const int grid2 = std::min((int)pq.size(), num_cus() * std::max(1, grid_per_cu / 2));
    {
      KernelTimer kt_(mode == MODE_BF16 ? "chi0_blocks_bf16" : "chi0_blocks_bf16x3", s);
      hipLaunchKernelGGL(mode == MODE_BF16 ? chi0_blocks<1> : chi0_blocks<3>, dim3(grid2), dim3(512), 0, s,
                         static_cast<const Item*>(ditems), static_cast<const int2*>(dtiles),
                         static_cast<const Unit*>(dunits), static_cast<const int2*>(dpq),
                         static_cast<const int*>(dqoff2), counter, static_cast<float*>(part));
    }
    XO_CHECK_LAUNCH();
    {
      KernelTimer kt_("chi0_reduce", s);
      hipLaunchKernelGGL(chi0_reduce_blocks, dim3(nreds, kBW), dim3(256), 0, s, static_cast<const Item*>(ditems),
                         static_cast<const int2*>(dtiles), static_cast<const Red*>(dreds),
                         static_cast<const float*>(part));
    }
    XO_CHECK_LAUNCH();
    return XO_OK;
  }
  if (mode == MODE_F64)
    return launch_nwg<MODE_F64>(nwg, NT, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid,
                                s);
  if (mode == MODE_F32)
    return launch_nwg<MODE_F32>(nwg, NT, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid,
                                s);
  if (mode == MODE_BF16)
    return launch_nwg<MODE_BF16>(nwg, NT, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid,
                                 s);
  return launch_nwg<MODE_BF16X3>(nwg, NT, ditems, dtiles, dunits, dqueue, nunits, counter, part, dreds, nreds, grid,
                                 s);
}

}  // namespace

// The same update with a prefactor of either sign (the terminator subtracts an
// explicit-band sum through it).
int chi0_run_signed(const xo_chi0_args* a, hipStream_t s) { return chi0_batch_run(a, 1, nullptr, s, true); }

// Real-axis chi0 in chunks of kRealChunk frequencies: each chunk is one Hermitian update
// over 2 kRealChunk factor slots into a scratch pair buffer, then the combination.
constexpr int kRealChunk = 32;

int chi0_real_run(const xo_chi0_real_args* a, hipStream_t s) {
  XO_ARG(a, "xo_chi0_real: null argument block");
  XO_ARG(a->nt > 0 && a->ng > 0 && a->nw > 0, "xo_chi0_real: sizes must be positive (nt=%d ng=%d nw=%d)", a->nt,
         a->ng, a->nw);
  XO_ARG(a->rho && a->dE && a->w && a->chi0, "xo_chi0_real: null pointer");
  XO_ARG(a->eta > 0.0 && std::isfinite(a->eta), "xo_chi0_real: eta must be positive and finite");
  for (int j = 0; j < a->nw; ++j)
    XO_ARG(a->w[j] >= 0.0 && std::isfinite(a->w[j]), "xo_chi0_real: frequency %d must be finite and >= 0", j);
  const size_t nn = (size_t)a->ng * a->ng;
  const int nwc_max = std::min(kRealChunk, a->nw);
  void* ws = nullptr;
  XO_RET(workspace(s, 7, 2 * (size_t)nwc_max * nn * 2 * sizeof(double), &ws));
  double* AB = static_cast<double*>(ws);
  for (int j0 = 0; j0 < a->nw; j0 += kRealChunk) {
    const int nwc = std::min(kRealChunk, a->nw - j0);
    std::vector<double> slots(2 * nwc);
    for (int j = 0; j < nwc; ++j) slots[2 * j] = slots[2 * j + 1] = a->w[j0 + j];
    xo_chi0_args c{};
    c.nt = a->nt;
    c.ng = a->ng;
    c.nw = 2 * nwc;
    c.prec = a->prec;
    c.rho = a->rho;
    c.dE = a->dE;
    c.w = slots.data();
    c.pref = a->pref;
    c.accumulate = 0;
    c.check_dE = j0 == 0 ? a->check_dE : 0;
    c.chi0 = AB;
    XO_RET(chi0_batch_run(&c, 1, nullptr, s, false, a->w + j0, a->eta));
    KernelTimer kt_("chi0_combine_real", s);
    hipLaunchKernelGGL(chi0_combine_real, dim3((unsigned)((nn + 255) / 256), nwc), dim3(256), 0, s, AB, a->ng, nwc,
                       a->accumulate, a->chi0 + (size_t)j0 * nn * 2);
    XO_CHECK_LAUNCH();
  }
  return XO_OK;
}

}  // namespace xo

extern "C" int xo_chi0(const xo_chi0_args* a, void* stream) {
  xo::clear_error();
  XO_ARG(a, "xo_chi0: null argument block");
  return xo::chi0_batch_run(a, 1, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" int xo_chi0_real(const xo_chi0_real_args* a, void* stream) {
  xo::clear_error();
  return xo::chi0_real_run(a, static_cast<hipStream_t>(stream));
}

static int check_tune(const xo_chi0_args* items, const xo_tune* tune) {
  if (tune) {
    XO_ARG(tune->nt_tiles == 0 || tune->nt_tiles == 1 || tune->nt_tiles == 2 || tune->nt_tiles == 4 ||
               tune->nt_tiles == 8,
           "xo_chi0_batch: nt_tiles must be 0, 1, 2, 4 or 8");
    XO_ARG(tune->nt_tiles < 4 || items[0].prec == XO_BF16X3 || items[0].prec == XO_BF16,
           "xo_chi0_batch: nt_tiles 4 and 8 are the bf16 block forms (XO_BF16X3, XO_BF16)");
    XO_ARG(tune->kper >= 0 && tune->wg_per_cu >= 0 && tune->wg_per_cu <= 16, "xo_chi0_batch: bad tune values");
  }
  return XO_OK;
}

extern "C" int xo_chi0_batch(const xo_chi0_args* items, int n, const xo_tune* tune, void* stream) {
  xo::clear_error();
  XO_ARG(items && n > 0, "xo_chi0_batch: need a non-empty array of items");
  XO_RET(check_tune(items, tune));
  return xo::chi0_batch_run(items, n, tune, static_cast<hipStream_t>(stream));
}

extern "C" int xo_chi0_workspace_size(const xo_chi0_args* items, int n, const xo_tune* tune, size_t* bytes) {
  xo::clear_error();
  XO_ARG(items && n > 0 && bytes, "xo_chi0_workspace_size: need a non-empty array of items and an output");
  XO_RET(check_tune(items, tune));
  return xo::chi0_batch_run(items, n, tune, nullptr, false, nullptr, 0.0, bytes);
}

extern "C" int xo_chi0_autotune(const xo_chi0_args* items, int n, xo_tune* best, double* best_ms, void* stream) {
  xo::clear_error();
  XO_ARG(items && n > 0 && best, "xo_chi0_autotune: bad arguments");
  // every candidate run overwrites the outputs, so an accumulating item would collect
  // the update once per run
  for (int i = 0; i < n; ++i)
    XO_ARG(items[i].accumulate == 0, "xo_chi0_autotune: item %d has accumulate set (tuning overwrites outputs)", i);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<xo_tune> cands;
  std::vector<int> nts = {1};
  if (items[0].prec == XO_BF16X3 || items[0].prec == XO_BF16) nts = {1, 2, 4, 8};
  int ntmax = 0;
  for (int i = 0; i < n; ++i) ntmax = std::max(ntmax, items[i].nt);
  for (int nt : nts)
    for (int kper : {0, 2048, 8192, 32768})
      for (int wpc : {1, 2, 4, 8}) {
        if (kper > 0 && kper / 2 > ntmax) continue;
        if ((wpc == 1) != (nt >= 4) && wpc < 2) continue;  // one workgroup per CU only for the block forms
        if (nt == 8 && wpc > 2) continue;                   // the strip form fits two per CU
        cands.push_back({nt, kper, wpc});
      }
  hipEvent_t e0, e1;
  XO_TRY_HIP(hipEventCreate(&e0));
  XO_TRY_HIP(hipEventCreate(&e1));
  double tbest = 1e300;
  xo_tune tb = cands[0];
  int rc = XO_OK;
  for (const xo_tune& c : cands) {
    float ms = 0.f;
    rc = xo::chi0_batch_run(items, n, &c, s);  // warm-up: allocations and tables
    if (rc != XO_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { rc = XO_ERR_HIP; break; }
    rc = xo::chi0_batch_run(items, n, &c, s);
    if (rc != XO_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = XO_ERR_HIP;
      break;
    }
    if (ms < tbest) {
      tbest = ms;
      tb = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != XO_OK) return rc;
  *best = tb;
  if (best_ms) *best_ms = tbest;
  return XO_OK;
}
