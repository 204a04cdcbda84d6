// Learned empty-band tail of chi0: a small MLP (forward, backward, MSE, Adam)
// and the feature / apply / guard kernels around it, all in FP32 except where
// chi0 itself (complex128) is read or written.
//
// The paper corrects the slowly converging sum over empty states with the
// extrapolar X-terminator (Eq. X_term_def, Appendix B); here a network trained
// on chi0 produced by the method itself predicts the correction instead, with
// the full band sum as fallback.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "bf16x3.h"
#include "xo_common.h"

namespace xo {
namespace {

__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

// ------------------------------------------------------------------ GEMM ----
// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (+ beta C), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn]; act = 1 also writes H = silu(C). FP32 products on
// v_mfma_f32_32x32x2_f32 (exact products, FP32 sums): a workgroup owns a 64 x 64 tile, its four
// waves a 32 x 32 quarter each; A and B pass through LDS in 32-deep slabs, the next slab is
// fetched into registers while the current one is multiplied. Tiles load along whichever
// stride is 1 so the reads coalesce. With ks > 1 the depth is split over gridDim.z and the
// slices land in P [ks][M][N], summed (with the epilogue) by gemm_reduce.
typedef float f16v __attribute__((ext_vector_type(16)));
constexpr int kGM = 64, kGN = 64, kGK = 32, kGPad = 4;

struct GemmArgs {
  int M, N, K;
  const float* A;
  long sam, sak;
  const float* B;
  long sbk, sbn;
  float* C;
  long ldc;
  const float* bias;
  float beta;
  int act;
  float* H;
  long ldh;
  int kchunk;  // depth per gridDim.z slice
  float* P;    // slices when gridDim.z > 1
};

__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  if (g.bias) v += g.bias[n];
  if (g.beta != 0.f) v += g.beta * g.C[m * g.ldc + n];
  g.C[m * g.ldc + n] = v;
  if (g.act) g.H[m * g.ldh + n] = v * sigm(v);
}

__global__ void __launch_bounds__(256) gemm_mfma(GemmArgs g) {
  __shared__ float As[kGK][kGM + kGPad];
  __shared__ float Bs[kGK][kGN + kGPad];
  const int m0 = blockIdx.y * kGM, n0 = blockIdx.x * kGN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int k_begin = blockIdx.z * g.kchunk, k_end = min(g.K, k_begin + g.kchunk);
  const bool a_k = g.sak == 1, b_n = g.sbn == 1;
  float ra[8], rb[8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * 256 + tid;
      const int am = a_k ? e / kGK : e % kGM, ak = a_k ? e % kGK : e / kGM;
      const int gm = m0 + am, gk = k0 + ak;
      ra[i] = (gm < g.M && gk < k_end) ? g.A[gm * g.sam + gk * g.sak] : 0.f;
      const int bn = b_n ? e % kGN : e / kGK, bk = b_n ? e / kGN : e % kGK;
      const int gn = n0 + bn, gk2 = k0 + bk;
      rb[i] = (gn < g.N && gk2 < k_end) ? g.B[gk2 * g.sbk + gn * g.sbn] : 0.f;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * 256 + tid;
      const int am = a_k ? e / kGK : e % kGM, ak = a_k ? e % kGK : e / kGM;
      As[ak][am] = ra[i];
      const int bn = b_n ? e % kGN : e / kGK, bk = b_n ? e / kGN : e % kGK;
      Bs[bk][bn] = rb[i];
    }
  };
  f16v acc = {};
  if (k_begin < k_end) fetch(k_begin);
  for (int k0 = k_begin; k0 < k_end; k0 += kGK) {
    stash();
    __syncthreads();
    if (k0 + kGK < k_end) fetch(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 2) {
      const float a = As[kk + (lane >> 5)][wm + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wn + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // result register r: row 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m >= g.M || n >= g.N) continue;
    if (gridDim.z > 1)
      g.P[((long)blockIdx.z * g.M + m) * g.N + n] = acc[r];
    else
      gemm_epilogue(g, m, n, acc[r]);
  }
}

// C = sum of the ks depth slices in P, in slice order, then the epilogue.
__global__ void gemm_reduce(GemmArgs g, int ks) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)g.M * g.N) return;
  float v = 0.f;
  for (int z = 0; z < ks; ++z) v += g.P[(long)z * g.M * g.N + e];
  gemm_epilogue(g, (int)(e / g.N), (int)(e % g.N), v);
}

// db[n] = sum_m dZ[m][n] in two fixed-order stages: part[y][n] = sum of the rows m = y (mod S),
// then db[n] = sum_y part[y][n].
__global__ void colsum_part(const float* __restrict__ dZ, int M, int N, float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = blockIdx.y; m < M; m += gridDim.y) s += dZ[(long)m * N + n];
  part[(long)blockIdx.y * N + n] = s;
}
__global__ void colsum_fin(const float* __restrict__ part, int S, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int y = 0; y < S; ++y) s += part[(long)y * N + n];
  db[n] = s;
}

// dZ = dH * silu'(Z)
__global__ void silu_back(const float* __restrict__ Z, const float* __restrict__ dH, long n,
                          float* __restrict__ dZ) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float z = Z[i], s = sigm(z);
    dZ[i] = dH[i] * s * (1.f + z * (1.f - s));
  }
}

// dY = 2 (Y - T) / n;  partial[blockIdx] = sum (Y - T)^2
__global__ void mse_grad(const float* __restrict__ Y, const float* __restrict__ T, long n,
                         float* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[256];
  float s = 0.f;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    if (dY) dY[i] = 2.f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials(const float* __restrict__ partial, int np, long n, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < np; ++i) s += partial[i];
  *loss = (float)(s / (double)n);
}

__global__ void adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                     float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void gather_rows(const float* __restrict__ src, const int* __restrict__ idx, int n, int F,
                            float* __restrict__ dst) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * F) return;
  const int r = (int)(e / F), f = (int)(e - (e / F) * F);
  dst[e] = src[(long)idx[r] * F + f];
}

// Per-column statistics of X [n][F]: out[f] = (mean, standard deviation, min, max),
// one workgroup per column, fixed-order reduction in FP64.
// Per-column statistics of X [n][F]: out[f] = (mean, standard deviation, min, max), FP64 sums in a
// fixed order: workgroup (f, y) reduces the rows i = y (mod S) of column f into part, then one
// workgroup per column reduces the S partial results.
__global__ void __launch_bounds__(256) col_stats_part(const float* __restrict__ X, long n, int F,
                                                      double* __restrict__ part) {
  __shared__ double s1[256], s2[256], mn[256], mx[256];
  const int f = blockIdx.x, y = blockIdx.y, S = gridDim.y;
  double a = 0.0, b = 0.0, lo = 1e300, hi = -1e300;
  for (long i = (long)y * 256 + threadIdx.x; i < n; i += (long)S * 256) {
    const double x = X[i * F + f];
    a += x;
    b += x * x;
    lo = fmin(lo, x);
    hi = fmax(hi, x);
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  mn[threadIdx.x] = lo;
  mx[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* p = part + 4 * ((long)f * S + y);
    p[0] = s1[0];
    p[1] = s2[0];
    p[2] = mn[0];
    p[3] = mx[0];
  }
}

__global__ void col_stats_fin(const double* __restrict__ part, int S, long n, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const int f = blockIdx.x;
  double a = 0.0, b = 0.0, lo = 1e300, hi = -1e300;
  for (int y = 0; y < S; ++y) {
    const double* p = part + 4 * ((long)f * S + y);
    a += p[0];
    b += p[1];
    lo = fmin(lo, p[2]);
    hi = fmax(hi, p[3]);
  }
  const double m = a / (double)n;
  out[4 * f] = m;
  out[4 * f + 1] = sqrt(fmax(b / (double)n - m * m, 0.0));
  out[4 * f + 2] = lo;
  out[4 * f + 3] = hi;
}

// ---------------------------------------------------------------- tail ----
// Features per (w, G, G'), normalised as (f - mu) * isd:
//  0,1  Re, Im of s_G chi_t s_G'          (truncated sum, s = sqrt(4 pi)/|q+G|)
//  2,3  Re, Im of s_G (chi_t - chi_h) s_G' (contribution of the last band block)
//  4,5  |q+G|, |q+G'|   6 |G-G'|   7 w   8 delta_GG'
// Target (when chi_f is given): Re, Im of s_G (chi_f - chi_t) s_G', scaled by tsc.
struct TailGeo {
  const double* qpg;  // [ng] |q+G|
  const double* gc;   // [ng][3] Cartesian G
  const double* w;    // [nw]
  const float* mu;    // [9]
  const float* isd;   // [9]
  int ng, nw;
};

// Normalised features of element e = (iw, i, j) of [nw][ng][ng]; also s_G s_G' and the
// scaled truncated value (tr, ti). The training features and the fused predictor both
// come from here, so they agree bit for bit.
__device__ __forceinline__ void tail_feat(const double* __restrict__ chi_t, const double* __restrict__ chi_h,
                                          const TailGeo& g, long e, float f[9], double& ss, double& tr,
                                          double& ti) {
  const int j = (int)(e % g.ng);
  const int i = (int)((e / g.ng) % g.ng);
  const int iw = (int)(e / ((long)g.ng * g.ng));
  ss = 4.0 * M_PI / (g.qpg[i] * g.qpg[j]);  // s_G s_G'
  tr = chi_t[2 * e] * ss;
  ti = chi_t[2 * e + 1] * ss;
  const double hr = chi_h[2 * e] * ss, hi = chi_h[2 * e + 1] * ss;
  const double dx = g.gc[3 * i] - g.gc[3 * j], dy = g.gc[3 * i + 1] - g.gc[3 * j + 1],
               dz = g.gc[3 * i + 2] - g.gc[3 * j + 2];
  f[0] = (float)tr;
  f[1] = (float)ti;
  f[2] = (float)(tr - hr);
  f[3] = (float)(ti - hi);
  f[4] = (float)g.qpg[i];
  f[5] = (float)g.qpg[j];
  f[6] = (float)sqrt(dx * dx + dy * dy + dz * dz);
  f[7] = (float)g.w[iw];
  f[8] = i == j ? 1.f : 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = (f[k] - g.mu[k]) * g.isd[k];
}

struct FeatArgs {
  const double* chi_t;
  const double* chi_h;
  const double* chi_f;
  TailGeo geo;
  float tsc;
  float* X;
  float* T;
};

__global__ void tail_features(FeatArgs a) {
  const long n = (long)a.geo.nw * a.geo.ng * a.geo.ng;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    float f[9];
    double ss, tr, ti;
    tail_feat(a.chi_t, a.chi_h, a.geo, e, f, ss, tr, ti);
#pragma unroll
    for (int k = 0; k < 9; ++k) a.X[e * 9 + k] = f[k];
    if (a.chi_f && a.T) {
      a.T[e * 2] = (float)((a.chi_f[2 * e] * ss - tr) * a.tsc);
      a.T[e * 2 + 1] = (float)((a.chi_f[2 * e + 1] * ss - ti) * a.tsc);
    }
  }
}

// chi = chi_t + Hermitian part of D / (s_G s_G'), with D = Y / tsc on the scaled grid
// (Y the mean of the ensemble members Y1 and, if given, Y2)
__global__ void tail_apply(const double* __restrict__ chi_t, const float* __restrict__ Y1, const float* __restrict__ Y2,
                           const double* __restrict__ qpg, int ng, int nw, float tsc, double* __restrict__ out) {
  const long n = (long)nw * ng * ng;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e % ng);
    const int i = (int)((e / ng) % ng);
    const long base = e - (long)i * ng - j;
    const long et = base + (long)j * ng + i;
    const double inv = qpg[i] * qpg[j] / (4.0 * M_PI) / (double)tsc;  // 1 / (s_G s_G' tsc)
    double yr = Y1[2 * e], yi = Y1[2 * e + 1], zr = Y1[2 * et], zi = Y1[2 * et + 1];
    if (Y2) {
      yr = 0.5 * (yr + (double)Y2[2 * e]);
      yi = 0.5 * (yi + (double)Y2[2 * e + 1]);
      zr = 0.5 * (zr + (double)Y2[2 * et]);
      zi = 0.5 * (zi + (double)Y2[2 * et + 1]);
    }
    const double dr = 0.5 * (yr + zr) * inv;
    const double di = 0.5 * (yi - zi) * inv;
    out[2 * e] = chi_t[2 * e] + dr;
    out[2 * e + 1] = i == j ? chi_t[2 * e + 1] : chi_t[2 * e + 1] + di;
  }
}

constexpr float kGuardFloor = 1e-6f;

// stats[0] += features outside [lo - m, hi + m], m = max(10% span, kGuardFloor); stats[1] += |Y1 - Y2|^2;
// stats[2] += |Y1 + Y2|^2 / 4. The floor (features are normalised to order one) keeps a feature
// that is zero up to rounding in every training crystal (Im chi0 of a crystal with inversion
// and time reversal) from rejecting data whose rounding differs.
__global__ void tail_guard(const float* __restrict__ X, long n, int F, const float* __restrict__ lo,
                           const float* __restrict__ hi, const float* __restrict__ Y1, const float* __restrict__ Y2,
                           int ny, double* __restrict__ stats) {
  double out = 0.0, dd = 0.0, mm = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    for (int k = 0; k < F; ++k) {
      const float x = X[e * F + k], m = fmaxf(0.1f * (hi[k] - lo[k]), kGuardFloor);
      if (x < lo[k] - m || x > hi[k] + m) out += 1.0;
    }
    for (int k = 0; k < ny; ++k) {
      const double a = Y1[e * ny + k], b = Y2[e * ny + k];
      dd += (a - b) * (a - b);
      mm += 0.25 * (a + b) * (a + b);
    }
  }
  atomicAdd(&stats[0], out);
  atomicAdd(&stats[1], dd);
  atomicAdd(&stats[2], mm);
}

// ------------------------------------------------------ fused predictor ----
// Inference of the tail ensemble on v_mfma_f32_32x32x16_bf16, fused with the features
// and the guard statistics. The product is taken transposed, Z^T = W H^T: rows are a
// layer's output units, columns are elements, so one wave carries 32-element column
// blocks through every layer without the activations leaving its registers.
//   A (weights), lane L: row L % 32, k = 8 (L / 32) .. + 7; B (activations), lane L:
//   column L % 32, same k; result register r of lane L: row 8 (r / 4) + 4 (L / 32) + r % 4.
// A 32-row result block thus already holds, per lane, the 16 values two 16-deep k-blocks of
// the next layer want from it, in the order hidden_unit() gives; the next layer's weight
// columns are packed in that order instead of moving the activations.
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int kPH = 256;                     // hidden width
constexpr int kPMB = kPH / 32;               // 32-row output blocks of a hidden layer
constexpr int kPKB = kPH / 16;               // 16-deep k-blocks of a hidden layer's input
constexpr int kPTile = 256;                  // elements per workgroup
constexpr int kPMaxL = 8;                    // layers
constexpr int kPFrag = 64;                   // u4 words per fragment (64 lanes x 8 bf16)

__device__ __forceinline__ f16v mma32(u4 a, u4 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}

// Input position p (0 .. 255) of a hidden-input layer -> the previous layer's unit that
// the register layout above delivers there.
__host__ __device__ inline int hidden_unit(int p) {
  const int kb = p >> 4, g = (p >> 3) & 1, j = p & 7;
  const int mb = kb >> 1, r = 8 * (kb & 1) + j;
  return 32 * mb + 8 * (r >> 2) + 4 * g + (r & 3);
}

__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2v));
}

// One layer of one member into fragments: fragment (mb, kb) = 64 lanes x 8 bf16, lane L
// holding W[32 mb + L % 32][unit of position 16 kb + 8 (L / 32) + j], j = 0 .. 7 (zero
// outside dout x din); bias padded to 32 MB rows (FP32).
__global__ void tail_pack_layer(const float* __restrict__ W, const float* __restrict__ b, int din, int dout,
                                int perm, int MB, int KB, uint16_t* __restrict__ frag, float* __restrict__ bias) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < MB * KB * 512) {
    const int j = t & 7, lane = (t >> 3) & 63, f = t >> 9;
    const int mb = f / KB, kb = f - (f / KB) * KB;
    const int o = 32 * mb + (lane & 31);
    const int p = 16 * kb + 8 * (lane >> 5) + j;
    const int u = perm ? hidden_unit(p) : p;
    const float v = (o < dout && u < din) ? W[(long)o * din + u] : 0.f;
    frag[t] = __builtin_bit_cast(uint16_t, (__bf16)v);
  }
  if (t < 32 * MB) bias[t] = t < dout ? b[t] : 0.f;
}

struct PredictArgs {
  const double* chi_t;
  const double* chi_h;
  TailGeo geo;
  const float* lo;     // [9]
  const float* hi;     // [9]
  long n;
  int nl, nmem;
  const u4* frag;      // fragments of every member
  const float* bias;   // padded biases of every member
  int fo[kPMaxL + 1];  // fragment offset (u4) of layer l in a member; fo[nl] = member stride
  int bo[kPMaxL + 1];  // bias offset (floats); bo[nl] = member stride
  float* Y;            // [n][2]
  double* part;        // [gridDim.x][3]
};

__device__ __forceinline__ float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// acc = bias of the rows this lane holds in output block mb
__device__ __forceinline__ f16v bias_init(const float* __restrict__ b, int mb, int g) {
  f16v c;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = *reinterpret_cast<const float4*>(b + 32 * mb + 8 * q + 4 * g);
    c[4 * q] = v.x;
    c[4 * q + 1] = v.y;
    c[4 * q + 2] = v.z;
    c[4 * q + 3] = v.w;
  }
  return c;
}

// SiLU of a finished 32-row block, as the two k-block operands of the next layer
__device__ __forceinline__ void silu_pack(const f16v& c, u4& lo, u4& hi) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    lo[q] = bf16_pair(silu_f(c[2 * q]), silu_f(c[2 * q + 1]));
    hi[q] = bf16_pair(silu_f(c[8 + 2 * q]), silu_f(c[8 + 2 * q + 1]));
  }
}

// One hidden layer 256 -> 256 (weights in LDS): hin -> SiLU(W hin + b) as next operands
template <int NC>
__device__ __forceinline__ void hidden_layer(const u4* __restrict__ Wl, const float* __restrict__ b, int g, int lane,
                                             const u4 (&hin)[NC][kPKB], u4 (&hout)[NC][kPKB]) {
#pragma unroll
  for (int mb = 0; mb < kPMB; ++mb) {
    const f16v b0 = bias_init(b, mb, g);
    f16v acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = b0;
#pragma unroll
    for (int kb = 0; kb < kPKB; ++kb) {
      const u4 w = Wl[(mb * kPKB + kb) * kPFrag + lane];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = mma32(w, hin[c][kb], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) silu_pack(acc[c], hout[c][2 * mb], hout[c][2 * mb + 1]);
    // keep the scheduler from hoisting later blocks' operand reads (registers run out)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Stage one hidden layer's fragments (128 KiB) in LDS; every wave must be done with the last.
template <int NT>
__device__ __forceinline__ void stage_layer(u4* __restrict__ Wl, const u4* __restrict__ src) {
  constexpr int kIt = kPMB * kPKB * kPFrag / NT, kGrp = 8;
  static_assert(kIt % kGrp == 0, "whole groups");
  __builtin_amdgcn_sched_barrier(0);
  __syncthreads();
  // straight-line copy in groups of kGrp loads (a loop here lets earlier work sink past it)
#pragma unroll
  for (int k0 = 0; k0 < kIt; k0 += kGrp) {
    u4 v[kGrp];
#pragma unroll
    for (int k = 0; k < kGrp; ++k) v[k] = src[(k0 + k) * NT + threadIdx.x];
#pragma unroll
    for (int k = 0; k < kGrp; ++k) Wl[(k0 + k) * NT + threadIdx.x] = v[k];
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  __builtin_amdgcn_sched_barrier(0);
}

// One ensemble member on this wave's NC column blocks: y[c][0..1] (lane group 0).
template <int NH, int NC, int NT>
__device__ __forceinline__ void run_member(const PredictArgs& a, int m, const u4 (&x)[NC], u4* __restrict__ Wl, int g,
                                           int lane, float (&y)[NC][2]) {
  const u4* F = a.frag + (long)m * a.fo[NH + 2];
  const float* B = a.bias + (long)m * a.bo[NH + 2];
  u4 hA[NC][kPKB], hB[NC][kPKB];
  // layer 0: features -> 256 (one k-block, fragments read from the caches)
#pragma unroll
  for (int mb = 0; mb < kPMB; ++mb) {
    const u4 w = F[a.fo[0] + mb * kPFrag + lane];
    const f16v b0 = bias_init(B + a.bo[0], mb, g);
#pragma unroll
    for (int c = 0; c < NC; ++c) silu_pack(mma32(w, x[c], b0), hA[c][2 * mb], hA[c][2 * mb + 1]);
  }
  // hidden layers through LDS, alternating register sets
  static_assert(NH >= 0 && NH <= 3, "at most three hidden 256 -> 256 layers");
  if constexpr (NH >= 1) {
    stage_layer<NT>(Wl, F + a.fo[1]);
    hidden_layer<NC>(Wl, B + a.bo[1], g, lane, hA, hB);
  }
  if constexpr (NH >= 2) {
    stage_layer<NT>(Wl, F + a.fo[2]);
    hidden_layer<NC>(Wl, B + a.bo[2], g, lane, hB, hA);
  }
  if constexpr (NH >= 3) {
    stage_layer<NT>(Wl, F + a.fo[3]);
    hidden_layer<NC>(Wl, B + a.bo[3], g, lane, hA, hB);
  }
  const u4(&h)[NC][kPKB] = (NH & 1) ? hB : hA;
  // last layer: 256 -> 2 (rows 0 and 1 of one block: registers 0, 1 of lane group 0)
  const f16v b0 = bias_init(B + a.bo[NH + 1], 0, g);
  f16v acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = b0;
#pragma unroll
  for (int kb = 0; kb < kPKB; ++kb) {
    const u4 w = F[a.fo[NH + 1] + kb * kPFrag + lane];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = mma32(w, h[c][kb], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    y[c][0] = acc[c][0];
    y[c][1] = acc[c][1];
  }
}

// NH hidden 256 -> 256 layers (the network has NH + 2 layers); NC 32-element column blocks
// per wave, 8 / NC waves, kPTile elements per workgroup.
template <int NH, int NC>
__global__ void __launch_bounds__(64 * (8 / NC)) tail_predict(PredictArgs a) {
  constexpr int NW = 8 / NC, NT = 64 * NW;
  __shared__ u4 Wl[kPMB * kPKB * kPFrag];  // the hidden layer being applied (128 KiB)
  __shared__ double red[NW][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 5, col = lane & 31;
  const long e0 = (long)blockIdx.x * kPTile + wave * (NC * 32) + col;

  // features -> first layer's operand (positions 8 g .. 8 g + 7 of the 16-deep k-block)
  u4 x[NC];
  double nout = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const long e = e0 + 32 * c;
    float f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = 0.f;
    if (e < a.n) {
      double ss, tr, ti;
      tail_feat(a.chi_t, a.chi_h, a.geo, e, f, ss, tr, ti);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if ((k < 8) != (g == 0)) continue;  // each feature checked by one lane group
        const float m = fmaxf(0.1f * (a.hi[k] - a.lo[k]), kGuardFloor);
        if (f[k] < a.lo[k] - m || f[k] > a.hi[k] + m) nout += 1.0;
      }
    }
    if (g == 0)
      x[c] = u4{bf16_pair(f[0], f[1]), bf16_pair(f[2], f[3]), bf16_pair(f[4], f[5]), bf16_pair(f[6], f[7])};
    else
      x[c] = u4{bf16_pair(f[8], 0.f), 0u, 0u, 0u};
  }

  float y[2][NC][2];
  run_member<NH, NC, NT>(a, 0, x, Wl, g, lane, y[0]);
  __builtin_amdgcn_sched_barrier(0);
  if (a.nmem == 2) run_member<NH, NC, NT>(a, 1, x, Wl, g, lane, y[1]);

  // ensemble mean, guard sums, output
  double dd = 0.0, mm = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const long e = e0 + 32 * c;
    if (g != 0 || e >= a.n) continue;
    float o0 = y[0][c][0], o1 = y[0][c][1];
    if (a.nmem == 2) {
      const double d0 = (double)y[0][c][0] - y[1][c][0], d1 = (double)y[0][c][1] - y[1][c][1];
      dd += d0 * d0 + d1 * d1;
      o0 = 0.5f * (y[0][c][0] + y[1][c][0]);
      o1 = 0.5f * (y[0][c][1] + y[1][c][1]);
      const double s0 = 0.5 * ((double)y[0][c][0] + y[1][c][0]), s1 = 0.5 * ((double)y[0][c][1] + y[1][c][1]);
      mm += s0 * s0 + s1 * s1;
    } else {
      mm += (double)o0 * o0 + (double)o1 * o1;
    }
    *reinterpret_cast<float2*>(a.Y + 2 * e) = make_float2(o0, o1);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    nout += __shfl_xor(nout, o);
    dd += __shfl_xor(dd, o);
    mm += __shfl_xor(mm, o);
  }
  if (lane == 0) {
    red[wave][0] = nout;
    red[wave][1] = dd;
    red[wave][2] = mm;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w][threadIdx.x];
    a.part[3 * (long)blockIdx.x + threadIdx.x] = t;
  }
}

// stats[k] = sum over workgroups of part[.][k], fixed order
__global__ void __launch_bounds__(256) tail_stats_sum(const double* __restrict__ part, long nb,
                                                      double* __restrict__ stats) {
  __shared__ double r[3][256];
  double t[3] = {0.0, 0.0, 0.0};
  for (long b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] += part[3 * b + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k][threadIdx.x] = t[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 3; ++k) r[k][threadIdx.x] += r[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) stats[threadIdx.x] = r[threadIdx.x][0];
}

static int launch_gemm(int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk, long sbn,
                       float* C, long ldc, const float* bias, float beta, int act, float* H, long ldh,
                       hipStream_t s) {
  GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, beta, act, H, ldh, K, nullptr};
  const int tiles = ((N + kGN - 1) / kGN) * ((M + kGM - 1) / kGM);
  // split a deep product over more workgroups when the tiles alone leave the chip idle
  int ks = 1;
  if (tiles < 256 && K >= 2048) ks = std::min((K + 1023) / 1024, std::max(1, 512 / tiles));
  if (ks > 1) {
    g.kchunk = ((K + ks - 1) / ks + kGK - 1) / kGK * kGK;
    ks = (K + g.kchunk - 1) / g.kchunk;
    void* ws = nullptr;
    XO_RET(workspace(s, 10, (size_t)ks * M * N * sizeof(float), &ws));
    g.P = static_cast<float*>(ws);
  }
  dim3 grid((N + kGN - 1) / kGN, (M + kGM - 1) / kGM, ks);
  {
    KernelTimer kt_("mlp_gemm", s);
    hipLaunchKernelGGL(gemm_mfma, grid, dim3(256), 0, s, g);
    if (ks > 1) {
      const long mn = (long)M * N;
      hipLaunchKernelGGL(gemm_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g, ks);
    }
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

// Device copies of the feature geometry: |q+G|, Cartesian G = sum_k m_k b_k (FP64), w, mu, isd.
static int tail_geo(const double* qpg, const int32_t* mill_g, const double* bvec, const double* w, const float* mu,
                    const float* isd, int ng, int nw, hipStream_t s, TailGeo* g) {
  std::vector<double> gc(3 * (size_t)ng);
  for (int i = 0; i < ng; ++i)
    for (int c = 0; c < 3; ++c)
      gc[3 * (size_t)i + c] = mill_g[3 * i] * bvec[c] + mill_g[3 * i + 1] * bvec[3 + c] + mill_g[3 * i + 2] * bvec[6 + c];
  const void *dq = nullptr, *dg = nullptr, *dw = nullptr, *dmu = nullptr, *disd = nullptr;
  XO_RET(device_table(qpg, sizeof(double) * ng, s, &dq));
  XO_RET(device_table(gc.data(), sizeof(double) * gc.size(), s, &dg));
  XO_RET(device_table(w, sizeof(double) * nw, s, &dw));
  XO_RET(device_table(mu, sizeof(float) * 9, s, &dmu));
  XO_RET(device_table(isd, sizeof(float) * 9, s, &disd));
  g->qpg = static_cast<const double*>(dq);
  g->gc = static_cast<const double*>(dg);
  g->w = static_cast<const double*>(dw);
  g->mu = static_cast<const float*>(dmu);
  g->isd = static_cast<const float*>(disd);
  g->ng = ng;
  g->nw = nw;
  return XO_OK;
}

static int check_dims(int nl, const int* dims, int n) {
  XO_ARG(nl >= 1 && nl <= 16 && dims && n > 0, "mlp: bad layer count %d or batch %d", nl, n);
  for (int l = 0; l <= nl; ++l) XO_ARG(dims[l] > 0 && dims[l] <= 4096, "mlp: bad width %d at %d", dims[l], l);
  return XO_OK;
}

}  // namespace
}  // namespace xo

using namespace xo;

extern "C" int xo_mlp_forward(int nl, const int* dims, const float* params, const float* X, int n, float* acts,
                              float* Y, void* stream) {
  clear_error();
  XO_RET(check_dims(nl, dims, n));
  XO_ARG(params && X && acts && Y, "xo_mlp_forward: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float* p = params;
  const float* h = X;
  float* a = acts;
  for (int l = 0; l < nl; ++l) {
    const int din = dims[l], dout = dims[l + 1];
    const float* W = p;
    const float* b = p + (long)din * dout;
    p = b + dout;
    const bool last = l == nl - 1;
    float* Z = last ? Y : a;
    float* H = last ? nullptr : a + (long)n * dout;
    XO_RET(launch_gemm(n, dout, din, h, din, 1, W, 1, din, Z, dout, b, 0.f, last ? 0 : 1, H, dout, s));
    if (!last) {
      h = H;
      a += 2L * n * dout;
    }
  }
  return XO_OK;
}

extern "C" int xo_mlp_backward(int nl, const int* dims, const float* params, const float* X, int n,
                               const float* acts, const float* dY, float* grads, float* work, float* dX,
                               void* stream) {
  clear_error();
  XO_RET(check_dims(nl, dims, n));
  XO_ARG(params && X && acts && dY && grads && work, "xo_mlp_backward: null pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // offsets of each layer's parameters and activations
  std::vector<long> po(nl + 1, 0), ao(nl, 0);
  for (int l = 0; l < nl; ++l) po[l + 1] = po[l] + (long)dims[l] * dims[l + 1] + dims[l + 1];
  for (int l = 1; l < nl; ++l) ao[l] = ao[l - 1] + 2L * n * dims[l];
  int wmax = 0;
  for (int l = 0; l <= nl; ++l) wmax = std::max(wmax, dims[l]);
  float* buf[2] = {work, work + (long)n * wmax};  // dH / dZ of consecutive layers alternate
  int cur = 1;                                     // buffer holding dZ (dZ = dY at the top)
  const float* dZ = dY;
  for (int l = nl - 1; l >= 0; --l) {
    const int din = dims[l], dout = dims[l + 1];
    const float* W = params + po[l];
    float* gW = grads + po[l];
    float* gb = gW + (long)din * dout;
    const float* Hin = l == 0 ? X : acts + ao[l - 1] + (long)n * dims[l];
    // gW[o][i] = sum_m dZ[m][o] Hin[m][i]
    XO_RET(launch_gemm(dout, din, n, dZ, 1, dout, Hin, din, 1, gW, din, nullptr, 0.f, 0, nullptr, 0, s));
    {
      KernelTimer kt_("mlp_colsum", s);
      const int S = std::min(256, (n + 63) / 64);
      void* ws = nullptr;
      XO_RET(workspace(s, 11, (size_t)S * dout * sizeof(float), &ws));
      float* part = static_cast<float*>(ws);
      hipLaunchKernelGGL(colsum_part, dim3((dout + 255) / 256, S), dim3(256), 0, s, dZ, n, dout, part);
      hipLaunchKernelGGL(colsum_fin, dim3((dout + 255) / 256), dim3(256), 0, s, part, S, dout, gb);
    }
    XO_CHECK_LAUNCH();
    if (l == 0 && !dX) break;
    // dH[m][i] = sum_o dZ[m][o] W[o][i], into the buffer that does not hold dZ
    const int nxt = cur ^ 1;
    float* dH = l == 0 ? dX : buf[nxt];
    XO_RET(launch_gemm(n, din, dout, dZ, dout, 1, W, din, 1, dH, din, nullptr, 0.f, 0, nullptr, 0, s));
    if (l == 0) break;
    const float* Zb = acts + ao[l - 1];   // pre-activation of layer l-1
    {
      KernelTimer kt_("mlp_silu_back", s);
      hipLaunchKernelGGL(silu_back, dim3(1024), dim3(256), 0, s, Zb, dH, (long)n * din, dH);
    }
    XO_CHECK_LAUNCH();
    dZ = dH;
    cur = nxt;
  }
  return XO_OK;
}

extern "C" int xo_mse(const float* Y, const float* T, long n, float* dY, float* loss, float* partial,
                      void* stream) {
  clear_error();
  XO_ARG(Y && T && loss && partial && n > 0, "xo_mse: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    KernelTimer kt_("mlp_mse", s);
    hipLaunchKernelGGL(mse_grad, dim3(256), dim3(256), 0, s, Y, T, n, dY, partial);
  }
  XO_CHECK_LAUNCH();
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(64), 0, s, partial, 256, n, loss);
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_adam_step(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                            float eps, int step, void* stream) {
  clear_error();
  XO_ARG(p && g && m && v && n > 0 && step >= 1, "xo_adam_step: bad arguments");
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipStream_t s = static_cast<hipStream_t>(stream);
  {
    KernelTimer kt_("mlp_adam", s);
    hipLaunchKernelGGL(adam, dim3(1024), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_gather_rows(const float* src, const int* idx, int n, int F, float* dst, void* stream) {
  clear_error();
  XO_ARG(src && idx && dst && n > 0 && F > 0, "xo_gather_rows: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long tot = (long)n * F;
  hipLaunchKernelGGL(gather_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, idx, n, F, dst);
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_col_stats(const float* X, long n, int F, double* out, void* stream) {
  clear_error();
  XO_ARG(X && out && n > 0 && F > 0, "xo_col_stats: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int S = (int)std::min<long>(256, (n + 4095) / 4096);
  void* ws = nullptr;
  XO_RET(workspace(s, 12, (size_t)F * S * 4 * sizeof(double), &ws));
  double* part = static_cast<double*>(ws);
  hipLaunchKernelGGL(col_stats_part, dim3(F, S), dim3(256), 0, s, X, n, F, part);
  XO_CHECK_LAUNCH();
  hipLaunchKernelGGL(col_stats_fin, dim3(F), dim3(64), 0, s, part, S, n, out);
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_tail_features(const xo_tail_args* a, void* stream) {
  clear_error();
  XO_ARG(a && a->chi_t && a->chi_h && a->qpg && a->mill_g && a->bvec && a->w && a->mu && a->isd && a->X,
         "xo_tail_features: null pointer");
  XO_ARG(a->ng > 0 && a->nw > 0, "xo_tail_features: bad sizes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  FeatArgs f;
  XO_RET(tail_geo(a->qpg, a->mill_g, a->bvec, a->w, a->mu, a->isd, a->ng, a->nw, s, &f.geo));
  f.chi_t = a->chi_t;
  f.chi_h = a->chi_h;
  f.chi_f = a->chi_f;
  f.tsc = (float)a->tsc;
  f.X = a->X;
  f.T = a->T;
  {
    KernelTimer kt_("tail_features", s);
    hipLaunchKernelGGL(tail_features, dim3(512), dim3(256), 0, s, f);
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_tail_apply(const double* chi_t, const float* Y1, const float* Y2, const double* qpg, int ng,
                             int nw, double tsc, double* out, void* stream) {
  clear_error();
  XO_ARG(chi_t && Y1 && qpg && out && ng > 0 && nw > 0 && tsc > 0, "xo_tail_apply: bad arguments");
  XO_ARG(chi_t != out, "xo_tail_apply: chi_t and out must not alias");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* dq = nullptr;
  XO_RET(device_table(qpg, sizeof(double) * ng, s, &dq));
  {
    KernelTimer kt_("tail_apply", s);
    hipLaunchKernelGGL(tail_apply, dim3(512), dim3(256), 0, s, chi_t, Y1, Y2, static_cast<const double*>(dq), ng,
                       nw, (float)tsc, out);
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_tail_guard(const float* X, long n, int F, const float* lo, const float* hi, const float* Y1,
                             const float* Y2, int ny, double* stats, void* stream) {
  clear_error();
  XO_ARG(X && lo && hi && Y1 && Y2 && stats && n > 0 && F > 0 && F <= 64 && ny > 0,
         "xo_tail_guard: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void *dlo = nullptr, *dhi = nullptr;
  XO_RET(device_table(lo, sizeof(float) * F, s, &dlo));
  XO_RET(device_table(hi, sizeof(float) * F, s, &dhi));
  XO_TRY_HIP(hipMemsetAsync(stats, 0, 3 * sizeof(double), s));
  {
    KernelTimer kt_("tail_guard", s);
    hipLaunchKernelGGL(tail_guard, dim3(256), dim3(256), 0, s, X, n, F, static_cast<const float*>(dlo),
                       static_cast<const float*>(dhi), Y1, Y2, ny, stats);
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

// Column blocks per wave of the fused predictor: 1 (eight waves, two per SIMD: one wave's
// SiLU work runs beside the other's matrix products; 93 ms for 144 M elements on one MI355X),
// or 2 (four waves, one per SIMD, half the LDS reads per product; 131 ms) with XO_TAIL_NC=2.
static int predict_nc() {
  const char* e = std::getenv("XO_TAIL_NC");
  return (e && std::atoi(e) == 2) ? 2 : 1;
}

extern "C" int xo_tail_predict(const xo_tail_predict_args* a, void* stream) {
  clear_error();
  XO_ARG(a && a->chi_t && a->chi_h && a->qpg && a->mill_g && a->bvec && a->w && a->mu && a->isd && a->lo && a->hi &&
             a->dims && a->params && a->Y && a->stats,
         "xo_tail_predict: null pointer");
  XO_ARG(a->ng > 0 && a->nw > 0 && a->nl >= 2 && a->nl <= 5 && (a->nmem == 1 || a->nmem == 2),
         "xo_tail_predict: bad sizes (ng %d, nw %d, nl %d (2 .. 5), nmem %d)", a->ng, a->nw, a->nl, a->nmem);
  for (int l = 0; l <= a->nl; ++l) XO_ARG(a->dims[l] > 0, "xo_tail_predict: bad width %d at %d", a->dims[l], l);
  if (a->dims[0] != 9 || a->dims[a->nl] != 2) {
    set_error("xo_tail_predict: the network must map the 9 tail features to 2 outputs (got %d -> %d)", a->dims[0],
              a->dims[a->nl]);
    return XO_ERR_UNSUPPORTED;
  }
  for (int l = 1; l < a->nl; ++l)
    if (a->dims[l] != kPH) {
      set_error("xo_tail_predict: hidden widths must be %d (layer %d has %d)", kPH, l, a->dims[l]);
      return XO_ERR_UNSUPPORTED;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  PredictArgs p{};
  XO_RET(tail_geo(a->qpg, a->mill_g, a->bvec, a->w, a->mu, a->isd, a->ng, a->nw, s, &p.geo));
  const void *dlo = nullptr, *dhi = nullptr;
  XO_RET(device_table(a->lo, sizeof(float) * 9, s, &dlo));
  XO_RET(device_table(a->hi, sizeof(float) * 9, s, &dhi));
  // fragment and bias layout of one member
  std::vector<int> MB(a->nl), KB(a->nl);
  long P = 0;
  p.fo[0] = p.bo[0] = 0;
  for (int l = 0; l < a->nl; ++l) {
    const int din = a->dims[l], dout = a->dims[l + 1];
    MB[l] = (dout + 31) / 32;
    KB[l] = (din + 15) / 16;
    p.fo[l + 1] = p.fo[l] + MB[l] * KB[l] * kPFrag;
    p.bo[l + 1] = p.bo[l] + 32 * MB[l];
    P += (long)din * dout + dout;
  }
  const long n = (long)a->nw * a->ng * a->ng;
  const long nb = (n + kPTile - 1) / kPTile;
  XO_ARG(nb < (1L << 31), "xo_tail_predict: %ld elements is too many for one launch", n);
  const size_t fbytes = align_up((size_t)a->nmem * p.fo[a->nl] * sizeof(u4), 256);
  const size_t bbytes = align_up((size_t)a->nmem * p.bo[a->nl] * sizeof(float), 256);
  const size_t pbytes = align_up((size_t)nb * 3 * sizeof(double), 256);
  void* ws = nullptr;
  XO_RET(workspace(s, 9, fbytes + bbytes + pbytes, &ws));
  u4* frag = static_cast<u4*>(ws);
  float* bias = reinterpret_cast<float*>(static_cast<char*>(ws) + fbytes);
  double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + fbytes + bbytes);
  {
    KernelTimer kt_("tail_pack", s);
    for (int m = 0; m < a->nmem; ++m) {
      const float* W = a->params + (long)m * P;
      for (int l = 0; l < a->nl; ++l) {
        const int din = a->dims[l], dout = a->dims[l + 1];
        const int tot = MB[l] * KB[l] * 512;
        hipLaunchKernelGGL(tail_pack_layer, dim3((tot + 255) / 256), dim3(256), 0, s, W, W + (long)din * dout, din,
                           dout, l > 0 ? 1 : 0, MB[l], KB[l],
                           reinterpret_cast<uint16_t*>(frag + (long)m * p.fo[a->nl] + p.fo[l]),
                           bias + (long)m * p.bo[a->nl] + p.bo[l]);
        W += (long)din * dout + dout;
      }
    }
  }
  XO_CHECK_LAUNCH();
  p.chi_t = a->chi_t;
  p.chi_h = a->chi_h;
  p.lo = static_cast<const float*>(dlo);
  p.hi = static_cast<const float*>(dhi);
  p.n = n;
  p.nl = a->nl;
  p.nmem = a->nmem;
  p.frag = frag;
  p.bias = bias;
  p.Y = a->Y;
  p.part = part;
  {
    KernelTimer kt_("tail_predict", s);
    const int nh = a->nl - 2;
    const int nc = predict_nc();
    const dim3 grid((unsigned)nb), blk(64 * (8 / nc));
    if (nh == 2 && nc == 2)
      hipLaunchKernelGGL((tail_predict<2, 2>), grid, blk, 0, s, p);
    else if (nh == 2)
      hipLaunchKernelGGL((tail_predict<2, 1>), grid, blk, 0, s, p);
    else if (nh == 1)
      hipLaunchKernelGGL((tail_predict<1, 1>), grid, blk, 0, s, p);
    else if (nh == 3)
      hipLaunchKernelGGL((tail_predict<3, 1>), grid, blk, 0, s, p);
    else
      hipLaunchKernelGGL((tail_predict<0, 1>), grid, blk, 0, s, p);
  }
  XO_CHECK_LAUNCH();
  hipLaunchKernelGGL(tail_stats_sum, dim3(1), dim3(256), 0, s, part, nb, a->stats);
  XO_CHECK_LAUNCH();
  return XO_OK;
}
