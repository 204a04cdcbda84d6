// Plasmon-pole screening and the diagonal GW self-energy (Quasi-particle
// corrections section: Eq. sigma_c, Eq. I_c, Eq. W_def and the Godby-Needs
// plasmon-pole paragraph), FP64.
//
//   ppa_fit        per element of X = eps~^-1 - 1: the pole pair
//                  X(w) = R [1/(w - Om) - 1/(w + Om)] through X(0) and X(i wp),
//                  Om = wp sqrt(Xp / (X0 - Xp)), R = -X0 Om / 2 where
//                  Re(Xp conj(X0 - Xp)) > 0, else Om = wp, R = -X0 wp / 2;
//                  writes Wr = R v^1/2_G v^1/2_G' (head override at G = G' = 0)
//   Coulomb factors v^1/2_G = sqrt(4 pi)/|q+G| (Coulomb interaction subsection) are formed
//   here from |q+G|; at q = 0 the G = 0 entry is 0 (the wings, odd in q, average to zero
//   over the small cell around q = 0) and the (0, 0) element takes the mean of 4 pi/q^2
//   over the sphere of volume (2 pi)^3/(N_k Omega), 12 pi/q_c^2 with
//   q_c = (6 pi^2/(N_k Omega))^(1/3); pref = 1/(N_k Omega).
//   sigma_c_tiles  Sigma_c,nn(z) = pref sum_m sum_GG' rho_nm(G) conj(rho_nm(G')) Wr_GG'
//                  [f_m / (z - e_m + Om - i eta) + (1 - f_m) / (z - e_m - Om + i eta)];
//                  a workgroup owns a 32 x 32 block of (G, G') held in registers (four
//                  elements per thread), one state n and a chunk of bands m, and writes
//                  one partial per frequency
//   sigma_reduce   fixed-order sum of the partials into Sigma_c
//   sigma_x_part   Sigma_x,nn = -pref sum_m f_m sum_G |rho_nm(G)|^2 v_G: partial sums over
//   + sigma_x_sum  chunks of eight bands, then their fixed-order sum

#include <algorithm>
#include <cmath>
#include <vector>

#include "xo_common.h"

namespace xo {
namespace {

typedef cplx<double> z;

constexpr int kSR = 2, kSC = 2;                 // rows and columns of G per thread
constexpr int kTR = 16 * kSR, kTC = 16 * kSC;   // 32 x 32 block per workgroup
constexpr int kMaxZ = 4;                        // frequencies per state and call

// 1/s: hardware estimate and one Newton step.
__device__ __forceinline__ double recip(double s) {
  const double r = __builtin_amdgcn_rcp(s);
  return fma(r, fma(-s, r, 1.0), r);
}

__device__ __forceinline__ z csqrt_principal(z a) {
  const double r = hypot(a.x, a.y);
  if (r == 0.0) return {0.0, 0.0};
  const double t = sqrt(0.5 * (r + fabs(a.x)));
  if (a.x >= 0.0) return {t, a.y / (2.0 * t)};
  return {fabs(a.y) / (2.0 * t), copysign(t, a.y)};
}

// Validity test of the fit, Re(Xp conj(d)) > 0, with separately rounded products (no
// contraction) so that it is decided exactly as written.
__device__ __forceinline__ bool fit_valid(z xp, z d) {
#pragma clang fp contract(off)
  const double a = xp.x * d.x;
  const double b = xp.y * d.y;
  return a + b > 0.0;
}

__global__ void ppa_fit(const z* __restrict__ e0, const z* __restrict__ ep, int ng, double wp,
                        const double* __restrict__ vs, double head, z* __restrict__ wr, z* __restrict__ om) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ng * ng) return;
  const int g = (int)(e / ng), gp = (int)(e % ng);
  z x0 = e0[e], xp = ep[e];
  if (g == gp) {
    x0.x -= 1.0;
    xp.x -= 1.0;
  }
  const z d = {x0.x - xp.x, x0.y - xp.y};
  z o = {wp, 0.0};
  if (fit_valid(xp, d)) {
    const double inv = 1.0 / (d.x * d.x + d.y * d.y);
    const z r = {(xp.x * d.x + xp.y * d.y) * inv, (xp.y * d.x - xp.x * d.y) * inv};  // xp / d
    const z sq = csqrt_principal(r);
    o = {wp * sq.x, wp * sq.y};
  }
  // R = -x0 om / 2, times the Coulomb factor
  const double c = (head >= 0.0 && g == 0 && gp == 0) ? head : vs[g] * vs[gp];
  const z R = {-0.5 * (x0.x * o.x - x0.y * o.y), -0.5 * (x0.x * o.y + x0.y * o.x)};
  wr[e] = {R.x * c, R.y * c};
  om[e] = o;
}

// acc += w * P / d (w = 1 when WEIGHTED is false)
template <bool WEIGHTED>
__device__ __forceinline__ void add_pole(z& acc, z P, double dx, double dy, double w) {
  double inv = recip(fma(dx, dx, dy * dy));
  if constexpr (WEIGHTED) inv *= w;
  acc.x = fma(fma(P.x, dx, P.y * dy), inv, acc.x);
  acc.y = fma(fma(P.y, dx, -P.x * dy), inv, acc.y);
}

template <bool SWAPPED>
__global__ void __launch_bounds__(256) sigma_c_tiles(const z* __restrict__ rho, const z* __restrict__ wr,
                                                     const z* __restrict__ om, const double* __restrict__ em,
                                                     const double* __restrict__ fm, const z* __restrict__ zz,
                                                     int nm, int nn, int ng, int nz, double eta, int ntc,
                                                     int mchunk, int ntile, int nmc, int per_xcd,
                                                     z* __restrict__ part) {
  __shared__ double red[2 * kMaxZ][8];
  // Workgroups go to the eight XCDs in turn (linear id mod 8); work item u = (state, band
  // chunk, block) in state-major order is given to XCD u / per_xcd, so that each XCD reads
  // the oscillator strengths of its own states, which then stay in its L2.
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= ntile * nmc * nn) return;
  const int tile = u % ntile, mc = (u / ntile) % nmc, n = u / (ntile * nmc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int r0 = (tile / ntc) * kTR, c0 = (tile % ntc) * kTC;
  int G[kSR], Gp[kSC];
  z W[kSR][kSC], O[kSR][kSC];
#pragma unroll
  for (int r = 0; r < kSR; ++r) G[r] = min(r0 + ty + 16 * r, ng - 1);
#pragma unroll
  for (int c = 0; c < kSC; ++c) Gp[c] = min(c0 + tx + 16 * c, ng - 1);
#pragma unroll
  for (int r = 0; r < kSR; ++r)
#pragma unroll
    for (int c = 0; c < kSC; ++c) {
      const size_t e = (size_t)G[r] * ng + Gp[c];
      const bool in = r0 + ty + 16 * r < ng && c0 + tx + 16 * c < ng;
      W[r][c] = in ? wr[e] : z{0.0, 0.0};  // elements past the G-set contribute zero
      O[r][c] = om[e];
    }
  z acc[kMaxZ];
#pragma unroll
  for (int j = 0; j < kMaxZ; ++j) acc[j] = {0.0, 0.0};
  const int m0 = mc * mchunk, m1 = min(nm, m0 + mchunk);
  // oscillator strengths of band m for the block's rows and columns, loaded one band ahead
  z a[kSR], b[kSC];
  auto load = [&](int m, z* a_, z* b_) {
    // rho_nm(G) from [m][n][G], or as conj of the mirrored strengths in [n][m][G]
    const z* rm = rho + (SWAPPED ? ((size_t)n * nm + m) : ((size_t)m * nn + n)) * ng;
#pragma unroll
    for (int r = 0; r < kSR; ++r) {
      a_[r] = rm[G[r]];
      if constexpr (SWAPPED) a_[r].y = -a_[r].y;
    }
#pragma unroll
    for (int c = 0; c < kSC; ++c) {
      b_[c] = rm[Gp[c]];
      if constexpr (SWAPPED) b_[c].y = -b_[c].y;
    }
  };
  if (m0 < m1) load(m0, a, b);
  for (int m = m0; m < m1; ++m) {
    z an[kSR], bn[kSC];
    load(min(m + 1, m1 - 1), an, bn);
    const double e = em[m], f = fm[m];
    z P[kSR][kSC];
#pragma unroll
    for (int r = 0; r < kSR; ++r)
#pragma unroll
      for (int c = 0; c < kSC; ++c) P[r][c] = cmul(cmulc(a[r], b[c]), W[r][c]);
#pragma unroll
    for (int j = 0; j < kMaxZ; ++j) {
      if (j >= nz) break;
      const z zj = zz[(size_t)n * nz + j];
      const double dx = zj.x - e;
      const double dyo = zj.y - eta, dye = zj.y + eta;
      // occupied part: pole at e - Om, below the real axis; empty part: e + Om, above.
      // Occupations 1 and 0 (insulators) take one pole, unweighted; fractional ones both.
      if (f == 1.0) {
#pragma unroll
        for (int r = 0; r < kSR; ++r)
#pragma unroll
          for (int c = 0; c < kSC; ++c) add_pole<false>(acc[j], P[r][c], dx + O[r][c].x, dyo + O[r][c].y, 1.0);
      } else if (f == 0.0) {
#pragma unroll
        for (int r = 0; r < kSR; ++r)
#pragma unroll
          for (int c = 0; c < kSC; ++c) add_pole<false>(acc[j], P[r][c], dx - O[r][c].x, dye - O[r][c].y, 1.0);
      } else {
#pragma unroll
        for (int r = 0; r < kSR; ++r)
#pragma unroll
          for (int c = 0; c < kSC; ++c) {
            add_pole<true>(acc[j], P[r][c], dx + O[r][c].x, dyo + O[r][c].y, f);
            add_pole<true>(acc[j], P[r][c], dx - O[r][c].x, dye - O[r][c].y, 1.0 - f);
          }
      }
    }
#pragma unroll
    for (int r = 0; r < kSR; ++r) a[r] = an[r];
#pragma unroll
    for (int c = 0; c < kSC; ++c) b[c] = bn[c];
  }
  // workgroup sum in a fixed order: wave shuffles, then the four waves through LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kMaxZ; ++j) {
    double x = acc[j].x, y = acc[j].y;
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_xor(x, o);
      y += __shfl_xor(y, o);
    }
    if (lane == 0) {
      red[2 * j][wave] = x;
      red[2 * j + 1][wave] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x < nz) {
    const int j = threadIdx.x;
    const double x = (red[2 * j][0] + red[2 * j][1]) + (red[2 * j][2] + red[2 * j][3]);
    const double y = (red[2 * j + 1][0] + red[2 * j + 1][1]) + (red[2 * j + 1][2] + red[2 * j + 1][3]);
    part[(((size_t)n * nmc + mc) * ntile + tile) * nz + j] = {x, y};
  }
}

// One wave per (n, j): out (+)= pref * sum over chunks and tiles (lane-strided partial
// sums, then a fixed butterfly).
__global__ void __launch_bounds__(64) sigma_reduce(const z* __restrict__ part, int nn, int nz, int nparts,
                                                   double pref, int accumulate, z* __restrict__ out) {
  const int t = blockIdx.x;
  const int n = t / nz, j = t % nz;
  double x = 0.0, y = 0.0;
  for (int p = threadIdx.x; p < nparts; p += 64) {
    const z v = part[((size_t)n * nparts + p) * nz + j];
    x += v.x;
    y += v.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_xor(x, o);
    y += __shfl_xor(y, o);
  }
  if (threadIdx.x == 0) {
    if (accumulate) {
      out[t].x += pref * x;
      out[t].y += pref * y;
    } else {
      out[t] = {pref * x, pref * y};
    }
  }
}

// Sigma_x partial sums: workgroup (n, chunk) over kXB bands and all G (flat index,
// stepped without divisions): part[n][chunk] = sum_m f_m sum_G |rho_nm(G)|^2 v_G.
constexpr int kXB = 8;

__global__ void __launch_bounds__(256) sigma_x_part(const z* __restrict__ rho, const double* __restrict__ fm,
                                                    const double* __restrict__ vs, double head, int nm, int nn,
                                                    int ng, int swapped, double* __restrict__ part) {
  __shared__ double red[256];
  const int n = blockIdx.x, ch = blockIdx.y;
  const int mb = ch * kXB, me = min(nm, mb + kXB);
  double s = 0.0;
  const int dm = 256 / ng, dg = 256 % ng;
  for (int m = mb + threadIdx.x / ng, g = threadIdx.x % ng; m < me;) {
    const double v = (g == 0 && head >= 0.0) ? head : vs[g] * vs[g];
    const z a = rho[(swapped ? ((size_t)n * nm + m) : ((size_t)m * nn + n)) * ng + g];  // |rho|^2 either way
    s = fma(fm[m] * v, fma(a.x, a.x, a.y * a.y), s);
    g += dg;
    m += dm;
    if (g >= ng) {
      g -= ng;
      ++m;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)n * gridDim.y + ch] = red[0];
}

// One wave per state: out[n] (+)= -pref * sum over chunks (fixed order).
__global__ void __launch_bounds__(64) sigma_x_sum(const double* __restrict__ part, int nch, double pref,
                                                  int accumulate, double* __restrict__ out) {
  const int n = blockIdx.x;
  double x = 0.0;
  for (int c = threadIdx.x; c < nch; c += 64) x += part[(size_t)n * nch + c];
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (threadIdx.x == 0) out[n] = (accumulate ? out[n] : 0.0) - pref * x;
}

// v^1/2 table and q = 0 head from |q+G| (host, during the call); returns the head or -1.
static int coulomb_tables(const char* who, const double* qpg, int ng, int q0, double nk_omega,
                          std::vector<double>& vs, double* head) {
  XO_ARG(qpg, "%s: null qpg", who);
  vs.assign(ng, 0.0);
  for (int g = q0 ? 1 : 0; g < ng; ++g) {
    XO_ARG(std::isfinite(qpg[g]) && qpg[g] > 0.0, "%s: |q+G| at %d must be positive and finite", who, g);
    vs[g] = std::sqrt(4.0 * M_PI) / qpg[g];
  }
  *head = -1.0;
  if (q0) {
    XO_ARG(nk_omega > 0.0 && std::isfinite(nk_omega), "%s: nk_omega must be positive at q = 0", who);
    const double qc = std::cbrt(6.0 * M_PI * M_PI / nk_omega);
    *head = 12.0 * M_PI / (qc * qc);
  }
  return XO_OK;
}

}  // namespace
}  // namespace xo

extern "C" int xo_ppa_fit(const xo_ppa_args* a, void* stream) {
  using namespace xo;
  clear_error();
  XO_ARG(a, "xo_ppa_fit: null argument block");
  XO_ARG(a->ng > 0, "xo_ppa_fit: ng must be positive (got %d)", a->ng);
  XO_ARG(a->einv0 && a->einvp && a->wr && a->om, "xo_ppa_fit: null device pointer");
  XO_ARG(a->omega_p > 0.0 && std::isfinite(a->omega_p), "xo_ppa_fit: omega_p must be positive");
  std::vector<double> vs;
  double head = -1.0;
  XO_RET(coulomb_tables("xo_ppa_fit", a->qpg, a->ng, a->q0, a->nk_omega, vs, &head));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* dvs = nullptr;
  XO_RET(device_table(vs.data(), sizeof(double) * a->ng, s, &dvs));
  const size_t ne = (size_t)a->ng * a->ng;
  {
    KernelTimer kt_("ppa_fit", s);
    hipLaunchKernelGGL(ppa_fit, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s,
                       static_cast<const z*>(a->einv0), static_cast<const z*>(a->einvp), a->ng, a->omega_p,
                       static_cast<const double*>(dvs), head, static_cast<z*>(a->wr), static_cast<z*>(a->om));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

extern "C" int xo_sigma(const xo_sigma_args* a, void* stream) {
  using namespace xo;
  clear_error();
  XO_ARG(a, "xo_sigma: null argument block");
  XO_ARG(a->nm > 0 && a->nn > 0 && a->ng > 0 && a->nz >= 0, "xo_sigma: sizes must be positive (nm=%d nn=%d ng=%d nz=%d)",
         a->nm, a->nn, a->ng, a->nz);
  XO_ARG(a->nz <= kMaxZ, "xo_sigma: at most %d frequencies per state (got %d)", kMaxZ, a->nz);
  XO_ARG(a->rho && a->e_m && a->f_m, "xo_sigma: null device pointer");
  XO_ARG(a->nz == 0 || (a->wr && a->om && a->z && a->sigc), "xo_sigma: null device pointer for Sigma_c");
  XO_ARG(a->qpg || !a->sigx, "xo_sigma: Sigma_x needs qpg");
  XO_ARG(a->nk_omega > 0.0 && std::isfinite(a->nk_omega), "xo_sigma: nk_omega must be positive");
  const double pref = 1.0 / a->nk_omega;
  XO_ARG(a->eta >= 0.0 && std::isfinite(a->eta), "xo_sigma: eta must be finite and >= 0");
  XO_ARG((size_t)a->nm * a->nn * a->ng < ((size_t)1 << 40), "xo_sigma: rho too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a->sigx) {
    std::vector<double> vs;
    double head = -1.0;
    XO_RET(coulomb_tables("xo_sigma", a->qpg, a->ng, a->q0, a->nk_omega, vs, &head));
    const void* dvs = nullptr;
    XO_RET(device_table(vs.data(), sizeof(double) * a->ng, s, &dvs));
    const int nch = (a->nm + kXB - 1) / kXB;
    XO_ARG(nch <= 65535, "xo_sigma: too many bands per call (nm=%d)", a->nm);
    void* wx = nullptr;
    XO_RET(workspace(s, 8, (size_t)a->nn * nch * sizeof(double), &wx));
    {
      KernelTimer kt_("sigma_x_part", s);
      hipLaunchKernelGGL(sigma_x_part, dim3(a->nn, nch), dim3(256), 0, s, static_cast<const z*>(a->rho), a->f_m,
                         static_cast<const double*>(dvs), head, a->nm, a->nn, a->ng, a->rho_swapped ? 1 : 0,
                         static_cast<double*>(wx));
    }
    XO_CHECK_LAUNCH();
    {
      KernelTimer kt_("sigma_x_sum", s);
      hipLaunchKernelGGL(sigma_x_sum, dim3(a->nn), dim3(64), 0, s, static_cast<const double*>(wx), nch, pref,
                         a->accumulate, a->sigx);
    }
    XO_CHECK_LAUNCH();
  }
  if (a->nz == 0) return XO_OK;
  const int ntr = (a->ng + kTR - 1) / kTR, ntc = (a->ng + kTC - 1) / kTC, ntile = ntr * ntc;
  // enough workgroups to give every compute unit several: split the bands into chunks
  int nmc = std::max(1, std::min(a->nm, (2048 + ntile * a->nn - 1) / (ntile * a->nn)));
  const int mchunk = (a->nm + nmc - 1) / nmc;
  nmc = (a->nm + mchunk - 1) / mchunk;
  const int nparts = nmc * ntile;
  void* ws = nullptr;
  XO_RET(workspace(s, 6, (size_t)a->nn * nparts * a->nz * sizeof(z), &ws));
  {
    KernelTimer kt_("sigma_c_tiles", s);
    const long total = (long)ntile * nmc * a->nn;
    const long per_xcd = (total + 7) / 8;
    XO_ARG(8 * per_xcd < (1L << 31), "xo_sigma: too many blocks (%ld)", total);
    hipLaunchKernelGGL(a->rho_swapped ? sigma_c_tiles<true> : sigma_c_tiles<false>, dim3((unsigned)(8 * per_xcd)),
                       dim3(256), 0, s, static_cast<const z*>(a->rho), static_cast<const z*>(a->wr),
                       static_cast<const z*>(a->om), a->e_m, a->f_m, static_cast<const z*>(a->z), a->nm, a->nn, a->ng,
                       a->nz, a->eta, ntc, mchunk, ntile, nmc, (int)per_xcd, static_cast<z*>(ws));
  }
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_("sigma_reduce", s);
    hipLaunchKernelGGL(sigma_reduce, dim3(a->nn * a->nz), dim3(64), 0, s, static_cast<const z*>(ws), a->nn,
                       a->nz, nparts, pref, a->accumulate, static_cast<z*>(a->sigc));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}
