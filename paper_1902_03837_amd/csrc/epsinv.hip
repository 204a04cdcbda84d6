// Inverse dielectric matrix in FP64 (Eq. X_rpa_inv; symmetrised as in Eq. W_def).
//
//   eps~ = I - diag(s) chi0 diag(s),   s_G = sqrt(4 pi) / |q+G|
//
// eps~ is Hermitian positive definite at imaginary frequencies. It is inverted
// in place by blocked Gauss-Jordan elimination without pivoting, all frequencies
// in the same launches. Per block column K (width b):
//   P    = A_KK^-1                  (one workgroup per frequency, LDS)
//   A_K* = P A_K*                   (row block, columns outside K)
//   A_ij -= A_iK A_Kj               (i, j outside K; rank-b update)
//   A_iK = -A_iK P,   A_KK = P
// The pivots met inside the diagonal blocks are the diagonal of eps~ = L D L^H,
// so a pivot with non-positive real part proves eps~ is not positive definite.

#include <algorithm>
#include <cmath>
#include <vector>

#include "xo_common.h"

namespace xo {
namespace {

constexpr int kB = 32;  // block width

typedef cplx<double> z;

__global__ void build_eps(const double* __restrict__ chi0, const double* __restrict__ s, int n,
                          double* __restrict__ A) {
  const size_t w = blockIdx.y;
  const size_t nn = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / n), j = (int)(e - (e / n) * n);
  const double f = s[i] * s[j];
  const double* c = chi0 + (w * nn + e) * 2;
  double* o = A + (w * nn + e) * 2;
  o[0] = (i == j ? 1.0 : 0.0) - f * c[0];
  o[1] = -f * c[1];
}

// In-place Gauss-Jordan inverse of the kb x kb diagonal block K of every matrix.
__global__ void __launch_bounds__(256) diag_inverse(double* __restrict__ Aall, int n, int K, int kb,
                                                   int check_sign, int* __restrict__ flag) {
  __shared__ z D[kB][kB + 1];
  __shared__ z rowk[kB];
  __shared__ z colk[kB];
  const int w = blockIdx.x;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const int o = K * kB;
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    const int i = e / kb, j = e % kb;
    D[i][j] = A[(size_t)(o + i) * n + o + j];
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    const z piv = D[k][k];
    // pivot test (uniform across the block: every thread reads the same value)
    const bool badp = check_sign ? !(piv.x > 0.0) : (piv.x == 0.0 && piv.y == 0.0);
    if (badp && threadIdx.x == 0 && flag[w] == 0) flag[w] = o + k + 1;
    const double den = piv.x * piv.x + piv.y * piv.y;
    const z ip = den > 0.0 ? z{piv.x / den, -piv.y / den} : z{0.0, 0.0};
    if (threadIdx.x < kb) {
      const int j = threadIdx.x;
      rowk[j] = (j == k) ? ip : cmul(D[k][j], ip);
      colk[j] = D[j][k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
      const int i = e / kb, j = e % kb;
      if (i == k) {
        D[i][j] = rowk[j];
      } else if (j == k) {
        const z f = colk[i];
        D[i][j] = z{-(f.x * ip.x - f.y * ip.y), -(f.x * ip.y + f.y * ip.x)};
      } else {
        const z f = colk[i], r = rowk[j];
        D[i][j] = z{D[i][j].x - (f.x * r.x - f.y * r.y), D[i][j].y - (f.x * r.y + f.y * r.x)};
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    const int i = e / kb, j = e % kb;
    A[(size_t)(o + i) * n + o + j] = D[i][j];
  }
}

// Row block: A_Kj <- P A_Kj for 64 columns j outside K per workgroup.
__global__ void __launch_bounds__(256) row_block(double* __restrict__ Aall, int n, int K, int kb) {
  __shared__ z P[kB][kB + 1];
  __shared__ z T[kB][65];
  const int w = blockIdx.y;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const int o = K * kB;
  const int j0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) P[e / kb][e % kb] = A[(size_t)(o + e / kb) * n + o + e % kb];
  for (int e = threadIdx.x; e < kb * 64; e += blockDim.x) {
    const int r = e / 64, c = e % 64, j = j0 + c;
    T[r][c] = (j < n && !(j >= o && j < o + kb)) ? A[(size_t)(o + r) * n + j] : z{0.0, 0.0};
  }
  __syncthreads();
  const int c = threadIdx.x & 63, j = j0 + c;
  if (j >= n || (j >= o && j < o + kb)) return;
  for (int r = threadIdx.x >> 6; r < kb; r += 4) {
    z acc = {0.0, 0.0};
    for (int m = 0; m < kb; ++m) cfma(acc, P[r][m], T[m][c]);
    A[(size_t)(o + r) * n + j] = acc;
  }
}

// Rank-kb update of every element outside row block K and column block K:
//   A_ij -= A_iK A_Kj   (A_iK old column, A_Kj new row).
__global__ void __launch_bounds__(256) rank_update(double* __restrict__ Aall, int n, int K, int kb) {
  __shared__ z L[32][kB + 1];
  __shared__ z R[kB][33];
  const int w = blockIdx.z;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const int o = K * kB;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  if (i0 == o || j0 == o) return;  // tiles are aligned with the 32-wide blocks
  for (int e = threadIdx.x; e < 32 * kb; e += blockDim.x) {
    const int r = e / kb, m = e % kb;
    L[r][m] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + o + m] : z{0.0, 0.0};
    const int m2 = e / 32, c = e % 32;
    R[m2][c] = (j0 + c < n) ? A[(size_t)(o + m2) * n + j0 + c] : z{0.0, 0.0};
  }
  __syncthreads();
  const int c = threadIdx.x & 31;
  const int j = j0 + c;
  if (j >= n) return;
  for (int r = threadIdx.x >> 5; r < 32; r += 8) {
    const int i = i0 + r;
    if (i >= n) break;
    z acc = A[(size_t)i * n + j];
    for (int m = 0; m < kb; ++m) {
      const z a = L[r][m], b = R[m][c];
      acc.x -= a.x * b.x - a.y * b.y;
      acc.y -= a.x * b.y + a.y * b.x;
    }
    A[(size_t)i * n + j] = acc;
  }
}

// Column block: A_iK <- -A_iK P for 64 rows i outside K per workgroup.
__global__ void __launch_bounds__(256) col_block(double* __restrict__ Aall, int n, int K, int kb) {
  __shared__ z P[kB][kB + 1];
  __shared__ z T[64][kB + 1];
  const int w = blockIdx.y;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const int o = K * kB;
  const int i0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) P[e / kb][e % kb] = A[(size_t)(o + e / kb) * n + o + e % kb];
  for (int e = threadIdx.x; e < 64 * kb; e += blockDim.x) {
    const int r = e / kb, m = e % kb, i = i0 + r;
    T[r][m] = (i < n) ? A[(size_t)i * n + o + m] : z{0.0, 0.0};
  }
  __syncthreads();
  const int m = threadIdx.x & 31;
  if (m >= kb) return;
  for (int r = threadIdx.x >> 5; r < 64; r += 8) {
    const int i = i0 + r;
    if (i >= n || (i >= o && i < o + kb)) continue;
    z acc = {0.0, 0.0};
    for (int p = 0; p < kb; ++p) cfma(acc, T[r][p], P[p][m]);
    A[(size_t)i * n + o + m] = z{-acc.x, -acc.y};
  }
}

__global__ void unsymmetrise(double* __restrict__ A, const double* __restrict__ s, int n) {
  const size_t w = blockIdx.y;
  const size_t nn = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / n), j = (int)(e - (e / n) * n);
  const double f = s[i] / s[j];
  double* o = A + (w * nn + e) * 2;
  o[0] *= f;
  o[1] *= f;
}

}  // namespace
}  // namespace xo

extern "C" int xo_epsinv(const xo_eps_args* a, void* stream) {
  using namespace xo;
  clear_error();
  XO_ARG(a, "xo_epsinv: null argument block");
  XO_ARG(a->ng > 0 && a->nw > 0, "xo_epsinv: sizes must be positive (ng=%d nw=%d)", a->ng, a->nw);
  XO_ARG(a->qpg && a->chi0 && a->out, "xo_epsinv: null pointer");
  XO_ARG((a->flags & ~(XO_EPS_NONSYM | XO_EPS_LU_FALLBACK)) == 0, "xo_epsinv: unknown flags 0x%x", a->flags);
  XO_ARG(a->chi0 != a->out, "xo_epsinv: chi0 and out must not alias");
  if (a->ng > 16384 || (size_t)a->ng * a->ng * a->nw > ((size_t)1 << 31)) {
    set_error("xo_epsinv: ng=%d x nw=%d is beyond the supported size", a->ng, a->nw);
    return XO_ERR_UNSUPPORTED;
  }
  const int n = a->ng;
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) {
    XO_ARG(a->qpg[i] > 0.0 && std::isfinite(a->qpg[i]), "xo_epsinv: |q+G| at %d must be positive", i);
    s[i] = std::sqrt(4.0 * M_PI) / a->qpg[i];
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void* ds = nullptr;
  XO_RET(device_table(s.data(), sizeof(double) * n, st, &ds));
  void* ws = nullptr;
  XO_RET(workspace(st, 2, sizeof(int) * a->nw, &ws));
  int* flag = static_cast<int*>(ws);
  XO_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(int) * a->nw, st));
  const size_t nn = (size_t)n * n;
  {
    KernelTimer kt_("eps_build", st);
    hipLaunchKernelGGL(build_eps, dim3((unsigned)((nn + 255) / 256), a->nw), dim3(256), 0, st, a->chi0,
                       static_cast<const double*>(ds), n, a->out);
  }
  XO_CHECK_LAUNCH();
  const int nblk = (n + kB - 1) / kB;
  const int check_sign = (a->flags & XO_EPS_LU_FALLBACK) ? 0 : 1;
  for (int K = 0; K < nblk; ++K) {
    const int kb = std::min(kB, n - K * kB);
    {
      KernelTimer kt_("eps_diag_inverse", st);
      hipLaunchKernelGGL(diag_inverse, dim3(a->nw), dim3(256), 0, st, a->out, n, K, kb, check_sign, flag);
    }
    XO_CHECK_LAUNCH();
    if (nblk > 1) {
      {
        KernelTimer kt_("eps_row_block", st);
        hipLaunchKernelGGL(row_block, dim3((n + 63) / 64, a->nw), dim3(256), 0, st, a->out, n, K, kb);
      }
      XO_CHECK_LAUNCH();
      {
        KernelTimer kt_("eps_rank_update", st);
        hipLaunchKernelGGL(rank_update, dim3((n + 31) / 32, (n + 31) / 32, a->nw), dim3(256), 0, st, a->out, n,
                           K, kb);
      }
      XO_CHECK_LAUNCH();
      {
        KernelTimer kt_("eps_col_block", st);
        hipLaunchKernelGGL(col_block, dim3((n + 63) / 64, a->nw), dim3(256), 0, st, a->out, n, K, kb);
      }
      XO_CHECK_LAUNCH();
    }
  }
  if (a->flags & XO_EPS_NONSYM) {
    {
      KernelTimer kt_("eps_unsymmetrise", st);
      hipLaunchKernelGGL(unsymmetrise, dim3((unsigned)((nn + 255) / 256), a->nw), dim3(256), 0, st, a->out,
                         static_cast<const double*>(ds), n);
    }
    XO_CHECK_LAUNCH();
  }
  int* hf = nullptr;
  XO_RET(host_flags(st, sizeof(int) * a->nw, reinterpret_cast<void**>(&hf)));
  XO_TRY_HIP(hipMemcpyAsync(hf, flag, sizeof(int) * a->nw, hipMemcpyDeviceToHost, st));
  XO_TRY_HIP(hipStreamSynchronize(st));
  for (int w = 0; w < a->nw; ++w) {
    if (hf[w]) {
      set_error("xo_epsinv: eps~ is not positive definite at frequency %d (pivot %d)", w, hf[w] - 1);
      return XO_ERR_NOTPD;
    }
  }
  return XO_OK;
}
