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
#include <vector>

#include "xo_common.h"

namespace xo {
namespace {

constexpr int kT = 64;   // output tile (rows and columns)
constexpr int kK = 16;   // depth of one LDS stage

__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

// C[m][n] = alpha * sum_k A(m,k) B(k,n) (+ beta C), with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn]; optional bias[n]; act = 1 also writes H = silu(C).
__global__ void __launch_bounds__(256) gemm_f32(int M, int N, int K, const float* __restrict__ A, long sam,
                                                long sak, const float* __restrict__ B, long sbk, long sbn,
                                                float* __restrict__ C, long ldc, const float* __restrict__ bias,
                                                float beta, int act, float* __restrict__ H, long ldh) {
  __shared__ float As[kK][kT + 4];
  __shared__ float Bs[kK][kT + 4];
  const int m0 = blockIdx.y * kT, n0 = blockIdx.x * kT;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += kK) {
    for (int e = threadIdx.x; e < kK * kT; e += 256) {
      const int kk = e / kT, r = e % kT;
      const int m = m0 + r, k = k0 + kk, n = n0 + r;
      As[kk][r] = (m < M && k < K) ? A[m * sam + k * sak] : 0.f;
      Bs[kk][r] = (n < N && k < K) ? B[k * sbk + n * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= N) continue;
      float v = acc[i][j];
      if (bias) v += bias[n];
      if (beta != 0.f) v += beta * C[m * ldc + n];
      C[m * ldc + n] = v;
      if (act) H[m * ldh + n] = v * sigm(v);
    }
  }
}

// db[n] = sum_m dZ[m][n] (one thread per column, fixed order)
__global__ void colsum(const float* __restrict__ dZ, int M, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(long)m * N + n];
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
__global__ void __launch_bounds__(256) col_stats(const float* __restrict__ X, long n, int F, double* __restrict__ out) {
  __shared__ double s1[256], s2[256], mn[256], mx[256];
  const int f = blockIdx.x;
  double a = 0.0, b = 0.0, lo = 1e300, hi = -1e300;
  for (long i = threadIdx.x; i < n; i += blockDim.x) {
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
    const double m = s1[0] / (double)n;
    out[4 * f] = m;
    out[4 * f + 1] = sqrt(fmax(s2[0] / (double)n - m * m, 0.0));
    out[4 * f + 2] = mn[0];
    out[4 * f + 3] = mx[0];
  }
}

// ---------------------------------------------------------------- tail ----
// Features per (w, G, G'), normalised as (f - mu) * isd:
//  0,1  Re, Im of s_G chi_t s_G'          (truncated sum, s = sqrt(4 pi)/|q+G|)
//  2,3  Re, Im of s_G (chi_t - chi_h) s_G' (contribution of the last band block)
//  4,5  |q+G|, |q+G'|   6 |G-G'|   7 w   8 delta_GG'
// Target (when chi_f is given): Re, Im of s_G (chi_f - chi_t) s_G', scaled by tsc.
struct FeatArgs {
  const double* chi_t;
  const double* chi_h;
  const double* chi_f;
  const double* qpg;
  const double* gdiff;
  const double* w;
  int ng, nw;
  const float* mu;
  const float* isd;
  float tsc;
  float* X;
  float* T;
};

__global__ void tail_features(FeatArgs a) {
  const long n = (long)a.nw * a.ng * a.ng;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e % a.ng);
    const int i = (int)((e / a.ng) % a.ng);
    const int iw = (int)(e / ((long)a.ng * a.ng));
    const double ss = 4.0 * M_PI / (a.qpg[i] * a.qpg[j]);  // s_G s_G'

    const double tr = a.chi_t[2 * e] * ss, ti = a.chi_t[2 * e + 1] * ss;
    const double hr = a.chi_h[2 * e] * ss, hi = a.chi_h[2 * e + 1] * ss;
    float f[9];
    f[0] = (float)tr;
    f[1] = (float)ti;
    f[2] = (float)(tr - hr);
    f[3] = (float)(ti - hi);
    f[4] = (float)a.qpg[i];
    f[5] = (float)a.qpg[j];
    f[6] = (float)a.gdiff[(long)i * a.ng + j];
    f[7] = (float)a.w[iw];
    f[8] = i == j ? 1.f : 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) a.X[e * 9 + k] = (f[k] - a.mu[k]) * a.isd[k];
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

// stats[0] += features outside [lo - m, hi + m], m = max(10% span, kGuardFloor); stats[1] += |Y1 - Y2|^2;
// stats[2] += |Y1 + Y2|^2 / 4. The floor (features are normalised to order one) keeps a feature
// that is zero up to rounding in every training crystal (Im chi0 of a crystal with inversion
// and time reversal) from rejecting data whose rounding differs.
constexpr float kGuardFloor = 1e-6f;
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

static int launch_gemm(int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk, long sbn,
                       float* C, long ldc, const float* bias, float beta, int act, float* H, long ldh,
                       hipStream_t s) {
  dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT);
  {
    KernelTimer kt_("mlp_gemm", s);
    hipLaunchKernelGGL(gemm_f32, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, beta, act,
                       H, ldh);
  }
  XO_CHECK_LAUNCH();
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
      hipLaunchKernelGGL(colsum, dim3((dout + 255) / 256), dim3(256), 0, s, dZ, n, dout, gb);
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
  hipLaunchKernelGGL(col_stats, dim3(F), dim3(256), 0, s, X, n, F, out);
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_tail_features(const xo_tail_args* a, void* stream) {
  clear_error();
  XO_ARG(a && a->chi_t && a->chi_h && a->qpg && a->gdiff && a->w && a->mu && a->isd && a->X,
         "xo_tail_features: null pointer");
  XO_ARG(a->ng > 0 && a->nw > 0, "xo_tail_features: bad sizes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void *dq = nullptr, *dg = nullptr, *dw = nullptr, *dmu = nullptr, *disd = nullptr;
  XO_RET(device_table(a->qpg, sizeof(double) * a->ng, s, &dq));
  XO_RET(device_table(a->gdiff, sizeof(double) * a->ng * a->ng, s, &dg));
  XO_RET(device_table(a->w, sizeof(double) * a->nw, s, &dw));
  XO_RET(device_table(a->mu, sizeof(float) * 9, s, &dmu));
  XO_RET(device_table(a->isd, sizeof(float) * 9, s, &disd));
  FeatArgs f;
  f.chi_t = a->chi_t;
  f.chi_h = a->chi_h;
  f.chi_f = a->chi_f;
  f.qpg = static_cast<const double*>(dq);
  f.gdiff = static_cast<const double*>(dg);
  f.w = static_cast<const double*>(dw);
  f.ng = a->ng;
  f.nw = a->nw;
  f.mu = static_cast<const float*>(dmu);
  f.isd = static_cast<const float*>(disd);
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
