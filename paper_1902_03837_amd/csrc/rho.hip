// Oscillator strengths rho_{cv k}(q,G) (Eq. rhotw) on gfx950.
//
// The paper evaluates rho as the 3D Fourier transform of the real-space product
// conj(psi_c) psi_v. Here the transform is factorised so that no full 3D grid is
// ever formed and only the needed outputs are produced:
//
//   1. orbitals -> mixed representation U(x, y, m_z): real space along x and y,
//      plane-wave (Miller) index along z. One pass per band (orb_mixed).
//   2. per transition and x-plane, the z transform of the product is a short
//      correlation of the two orbitals' z spectra,
//          S1(x,y,e_z) = sum_m conj(U_c(x,y,m)) U_v(x,y,m - e_z),
//      exact whenever the grid is alias free (checked on the host), and only
//      for the e_z range the G-set needs (rho_zy, stage 1, registers);
//   3. a pruned DFT along y for the (e_y, e_z) pairs present in the G-set
//      (rho_zy, stage 2, LDS);
//   4. a pruned DFT along x for each G (rho_x).
// Here e = m_G - G0 is the target Miller index of G shifted by the umklapp.
// Twiddles carry exp(+i G.r), and the 1/N_r of the cell average is applied once.

#include <algorithm>
#include <cmath>
#include <vector>

#include "rho_geom.h"

namespace xo {
namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / n, &s, &c);
    tw[k] = {T(c), T(s)};
  }
}



// U[b][x][y][s] = sum_{PW with m_z = zlo + s} c_b(PW) exp(2 pi i (m_x x/Nx + m_y y/Ny)).
// One workgroup per (band, z-slot): scatter the slot's plane waves into a dense
// (m_y, m_x) box in LDS, transform along x, then along y; slots past the sphere's
// z-extent are written as zeros.
template <typename T, int NO>
__global__ void __launch_bounds__(kBlock) orb_mixed(const cplx<T>* __restrict__ coef, int npw,
                                                     const SphereEntry* __restrict__ ent,
                                                     const int* __restrict__ zoff, int nslot, int Nx, int Ny,
                                                     int xlo, int nbx, int ylo, int nby,
                                                     cplx<T>* __restrict__ U) {
  extern __shared__ unsigned char smem[];
  cplx<T>* twx = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* twy = twx + Nx;
  cplx<T>* box = twy + Ny;        // [nby][nbx]
  cplx<T>* V = box + nby * nbx;   // [nby][Nx]
  const int b = blockIdx.x;
  const int s = blockIdx.y;
  cplx<T>* ub = U + (size_t)b * Nx * Ny * NO + s;
  if (s >= nslot) {
    for (int xy = threadIdx.x; xy < Nx * Ny; xy += blockDim.x) ub[(size_t)xy * NO] = {T(0), T(0)};
    return;
  }
  load_twiddles(twx, Nx);
  load_twiddles(twy, Ny);
  for (int e = threadIdx.x; e < nby * nbx; e += blockDim.x) box[e] = {T(0), T(0)};
  __syncthreads();
  const int p0 = zoff[s], p1 = zoff[s + 1];
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const SphereEntry e = ent[p];
    box[e.by * nbx + e.bx] = coef[(size_t)b * npw + e.src];
  }
  __syncthreads();
  // x transform: V[by][x] = sum_bx box[by][bx] exp(2 pi i (xlo + bx) x / Nx)
  for (int it = threadIdx.x; it < nby * Nx; it += blockDim.x) {
    const int by = it / Nx, x = it - (it / Nx) * Nx;
    int k = pmod(xlo * x, Nx);
    cplx<T> acc = {T(0), T(0)};
    for (int bx = 0; bx < nbx; ++bx) {
      cfma(acc, box[by * nbx + bx], twx[k]);
      k += x;
      if (k >= Nx) k -= Nx;
    }
    V[it] = acc;
  }
  __syncthreads();
  // y transform: U[x][y][s] = sum_by V[by][x] exp(2 pi i (ylo + by) y / Ny)
  for (int xy = threadIdx.x; xy < Nx * Ny; xy += blockDim.x) {
    const int x = xy / Ny, y = xy - (xy / Ny) * Ny;
    int k = pmod(ylo * y, Ny);
    cplx<T> acc = {T(0), T(0)};
    for (int by = 0; by < nby; ++by) {
      cfma(acc, V[by * Nx + x], twy[k]);
      k += y;
      if (k >= Ny) k -= Ny;
    }
    ub[(size_t)xy * NO] = acc;
  }
}

struct ZYParams {
  const void* Uc;
  const void* Uv;
  int Nx, Ny;
  int nz4;          // number of e_z outputs rounded up to a multiple of 4
  int d0;           // czmin - vzmin - ezmin
  int nyz;          // number of (e_y, e_z) pairs needed
  const int2* yz;   // (e_y mod Ny, e_z - ezmin) per pair
  int nv, TV;       // valence count and tile height
  int c0;           // first conduction band of this chunk
  int ncc;          // conduction bands in this chunk
  void* S2;         // [nv][ncc][Nx][nyz]
};

// Stages 1 and 2 for one conduction band and a tile of TV valence bands,
// looping over x-planes.
template <typename T, int NO>
__global__ void __launch_bounds__(kBlock) rho_zy(ZYParams P) {
  extern __shared__ unsigned char smem[];
  cplx<T>* twy = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* S1 = twy + P.Ny;  // [TV][Ny][nz4]
  const int vt0 = blockIdx.x * P.TV;
  const int cl = blockIdx.y;
  const int c = P.c0 + cl;
  const int tv = min(P.TV, P.nv - vt0);
  const cplx<T>* Uc = static_cast<const cplx<T>*>(P.Uc);
  const cplx<T>* Uv = static_cast<const cplx<T>*>(P.Uv);
  cplx<T>* S2 = static_cast<cplx<T>*>(P.S2);
  load_twiddles(twy, P.Ny);
  const int nch = P.nz4 >> 2;
  const int n1 = tv * P.Ny * nch;
  const int n2 = tv * P.nyz;
  const size_t plane = (size_t)P.Ny * NO;
  for (int x = 0; x < P.Nx; ++x) {
    // ---- stage 1: z correlation, 4 outputs per item
    for (int it = threadIdx.x; it < n1; it += blockDim.x) {
      const int ch = it % nch;
      const int rest = it / nch;
      const int y = rest % P.Ny;
      const int vl = rest / P.Ny;
      const int v = vt0 + vl;
      const cplx<T>* a = Uc + ((size_t)c * P.Nx + x) * plane + (size_t)y * NO;
      const cplx<T>* bl = Uv + ((size_t)v * P.Nx + x) * plane + (size_t)y * NO;
      cplx<T> A[NO];
#pragma unroll
      for (int j = 0; j < NO; ++j) A[j] = a[j];
      const int iz0 = ch * 4;
      const int base = P.d0 - iz0 - 3;
      cplx<T> W[NO + 3];
#pragma unroll
      for (int w = 0; w < NO + 3; ++w) {
        const int k = base + w;
        W[w] = ((unsigned)k < (unsigned)NO) ? bl[k] : cplx<T>{T(0), T(0)};
      }
      cplx<T> o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = {T(0), T(0)};
#pragma unroll
      for (int j = 0; j < NO; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) cfma_conj(o[i], A[j], W[j - i + 3]);
      }
      cplx<T>* dst = S1 + ((size_t)vl * P.Ny + y) * P.nz4 + iz0;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[i] = o[i];
    }
    __syncthreads();
    // ---- stage 2: pruned DFT along y for the needed (e_y, e_z) pairs
    for (int it = threadIdx.x; it < n2; it += blockDim.x) {
      const int slot = it % P.nyz;
      const int vl = it / P.nyz;
      const int2 q = P.yz[slot];
      const cplx<T>* src = S1 + (size_t)vl * P.Ny * P.nz4 + q.y;
      cplx<T> acc = {T(0), T(0)};
      int k = 0;
      for (int y = 0; y < P.Ny; ++y) {
        cfma(acc, src[(size_t)y * P.nz4], twy[k]);
        k += q.x;
        if (k >= P.Ny) k -= P.Ny;
      }
      const int v = vt0 + vl;
      S2[(((size_t)v * P.ncc + cl) * P.Nx + x) * P.nyz + slot] = acc;
    }
    __syncthreads();
  }
}

// Stage 3: pruned DFT along x and the 1/N_r normalisation.
template <typename T>
__global__ void __launch_bounds__(kBlock) rho_x(const cplx<T>* __restrict__ S2, int Nx, int nyz, int ng,
                                                 const int2* __restrict__ gsel, int ncc, int c0, int nc,
                                                 T scale, cplx<T>* __restrict__ rho) {
  __shared__ cplx<T> twx[kMaxAxis];
  load_twiddles(twx, Nx);
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int cl = blockIdx.y;
  const int v = blockIdx.z;
  if (g >= ng) return;
  const int2 q = gsel[g];  // (slot, e_x mod Nx)
  const cplx<T>* src = S2 + ((size_t)v * ncc + cl) * Nx * nyz + q.x;
  cplx<T> acc = {T(0), T(0)};
  int k = 0;
  for (int x = 0; x < Nx; ++x) {
    cfma(acc, src[(size_t)x * nyz], twx[k]);
    k += q.y;
    if (k >= Nx) k -= Nx;
  }
  rho[((size_t)v * nc + c0 + cl) * ng + g] = {acc.x * scale, acc.y * scale};
}

__global__ void pole_energies(const double* __restrict__ ec, const double* __restrict__ ev, int nc,
                              int nv, double* __restrict__ dE) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * nv) return;
  const int v = i / nc, c = i - (i / nc) * nc;
  dE[i] = ec[c] - ev[v];
}

// q -> 0 head along qhat from velocity matrix elements (Eq. dip, local H):
//   rho^_cv = sum_G conj(c_c(G)) [qhat.(k+G)] c_v(G) / (e_c - e_v), in FP64.
template <typename T>
__global__ void rho_head_q0(const cplx<T>* __restrict__ cc, const cplx<T>* __restrict__ cv, int npw,
                            const double* __restrict__ proj, const double* __restrict__ ec,
                            const double* __restrict__ ev, int nc, int nv, int ng, int g0idx,
                            cplx<T>* __restrict__ rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * nv) return;
  const int v = i / nc, c = i - (i / nc) * nc;
  const cplx<T>* a = cc + (size_t)c * npw;
  const cplx<T>* b = cv + (size_t)v * npw;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < npw; ++p) {
    const double ar = a[p].x, ai = a[p].y, br = b[p].x, bi = b[p].y, w = proj[p];
    re += w * (ar * br + ai * bi);
    im += w * (ar * bi - ai * br);
  }
  const double den = ec[c] - ev[v];
  rho[(size_t)i * ng + g0idx] = {T(re / den), T(im / den)};
}

// ------------------------------------------------------------------ host side

template <typename T>
static int launch_head_q0(const xo_rho_args* a, hipStream_t s) {
  int g0idx = -1;
  for (int g = 0; g < a->ng; ++g)
    if (a->mill_g[3 * g] == 0 && a->mill_g[3 * g + 1] == 0 && a->mill_g[3 * g + 2] == 0) g0idx = g;
  double qn = std::sqrt(a->qhat[0] * a->qhat[0] + a->qhat[1] * a->qhat[1] + a->qhat[2] * a->qhat[2]);
  std::vector<double> proj(a->npw_c);
  for (int p = 0; p < a->npw_c; ++p) {
    double kg[3];
    for (int i = 0; i < 3; ++i)
      kg[i] = a->kcart[i] + a->mill_c[3 * p] * a->bvec[0 + i] + a->mill_c[3 * p + 1] * a->bvec[3 + i] +
              a->mill_c[3 * p + 2] * a->bvec[6 + i];
    proj[p] = (kg[0] * a->qhat[0] + kg[1] * a->qhat[1] + kg[2] * a->qhat[2]) / qn;
  }
  const void* dproj = nullptr;
  XO_RET(device_table(proj.data(), proj.size() * sizeof(double), s, &dproj));
  const int n = a->nc * a->nv;
  {
    KernelTimer kt_("rho_head_q0", s);
    hipLaunchKernelGGL((rho_head_q0<T>), dim3((n + 255) / 256), dim3(256), 0, s,
                       static_cast<const cplx<T>*>(a->coef_c), static_cast<const cplx<T>*>(a->coef_v),
                       a->npw_c, static_cast<const double*>(dproj), a->e_c, a->e_v, a->nc, a->nv, a->ng,
                       g0idx, static_cast<cplx<T>*>(a->rho));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <typename T, int NO>
static int launch_orb(const void* coef, int npw, int nb, const SphereTable& st, const Extent& ex,
                      hipStream_t s, int Nx, int Ny, void* U) {
  const void* dent = nullptr;
  const void* dzoff = nullptr;
  XO_RET(device_table(st.ent.data(), st.ent.size() * sizeof(SphereEntry), s, &dent));
  XO_RET(device_table(st.zoff.data(), st.zoff.size() * sizeof(int), s, &dzoff));
  const int nbx = ex.hi[0] - ex.lo[0] + 1, nby = ex.hi[1] - ex.lo[1] + 1;
  size_t lds = (size_t)(Nx + Ny + nby * nbx + nby * Nx) * sizeof(cplx<T>);
  if (lds > 160 * 1024) {
    set_error("plane-wave sphere of %d coefficients does not fit in LDS", npw);
    return XO_ERR_UNSUPPORTED;
  }
  if (lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&orb_mixed<T, NO>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    KernelTimer kt_("orb_mixed", s);
    hipLaunchKernelGGL((orb_mixed<T, NO>), dim3(nb, NO), dim3(kBlock), lds, s,
                       static_cast<const cplx<T>*>(coef), npw, static_cast<const SphereEntry*>(dent),
                       static_cast<const int*>(dzoff), st.nslot, Nx, Ny, ex.lo[0], nbx, ex.lo[1], nby,
                       static_cast<cplx<T>*>(U));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <typename T, int NO>
static int rho_run(const xo_rho_args* a, hipStream_t s, const Extent& xc, const Extent& xv,
                   const Extent& xe) {
  const int Nx = a->n[0], Ny = a->n[1];
  SphereTable tc = sphere_table(a->mill_c, a->npw_c, xc);
  SphereTable tv = sphere_table(a->mill_v, a->npw_v, xv);

  // needed (e_y, e_z) pairs and per-G selectors
  const int ezmin = xe.lo[2];
  const int nz = xe.hi[2] - xe.lo[2] + 1;
  const int nz4 = (nz + 3) / 4 * 4;
  std::vector<int> slot_of(Ny * nz, -1);
  std::vector<int2> yz;
  std::vector<int2> gsel(a->ng);
  for (int g = 0; g < a->ng; ++g) {
    const int ex = a->mill_g[3 * g] - a->g0[0];
    const int ey = a->mill_g[3 * g + 1] - a->g0[1];
    const int ez = a->mill_g[3 * g + 2] - a->g0[2];
    const int key = pmod(ey, Ny) * nz + (ez - ezmin);
    if (slot_of[key] < 0) {
      slot_of[key] = (int)yz.size();
      yz.push_back(make_int2(pmod(ey, Ny), ez - ezmin));
    }
    gsel[g] = make_int2(slot_of[key], pmod(ex, Nx));
  }
  const int nyz = (int)yz.size();
  const void* dyz = nullptr;
  const void* dgsel = nullptr;
  XO_RET(device_table(yz.data(), yz.size() * sizeof(int2), s, &dyz));
  XO_RET(device_table(gsel.data(), gsel.size() * sizeof(int2), s, &dgsel));

  // workspace: U_c, U_v, S2 chunk
  const size_t ub = (size_t)Nx * Ny * NO * sizeof(cplx<T>);
  const size_t uc_bytes = align_up(ub * a->nc, 256);
  const size_t uv_bytes = align_up(ub * a->nv, 256);
  const size_t per_c = (size_t)a->nv * Nx * nyz * sizeof(cplx<T>);
  const size_t s2_budget = (size_t)1 << 30;
  int ncc = (int)std::max<size_t>(1, std::min<size_t>(a->nc, s2_budget / per_c));
  void* ws = nullptr;
  XO_RET(workspace(s, 0, uc_bytes + uv_bytes + per_c * ncc, &ws));
  char* base = static_cast<char*>(ws);
  void* Uc = base;
  void* Uv = base + uc_bytes;
  void* S2 = base + uc_bytes + uv_bytes;

  XO_RET((launch_orb<T, NO>(a->coef_c, a->npw_c, a->nc, tc, xc, s, Nx, Ny, Uc)));
  XO_RET((launch_orb<T, NO>(a->coef_v, a->npw_v, a->nv, tv, xv, s, Nx, Ny, Uv)));

  int TV = std::min(a->nv, 8);
  auto lds_of = [&](int tvv) { return (size_t)(Ny + (size_t)tvv * Ny * nz4) * sizeof(cplx<T>); };
  while (TV > 1 && lds_of(TV) > 64 * 1024) TV /= 2;
  if (lds_of(TV) > 160 * 1024) {
    set_error("rho: LDS for a %d x %d slab exceeds the CU's 160 KiB", Ny, nz4);
    return XO_ERR_UNSUPPORTED;
  }
  if (lds_of(TV) > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rho_zy<T, NO>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_of(TV)));
  const double scale = 1.0 / ((double)Nx * (double)Ny);
  for (int c0 = 0; c0 < a->nc; c0 += ncc) {
    const int n = std::min(ncc, a->nc - c0);
    ZYParams P;
    P.Uc = Uc;
    P.Uv = Uv;
    P.Nx = Nx;
    P.Ny = Ny;
    P.nz4 = nz4;
    P.d0 = xc.lo[2] - xv.lo[2] - ezmin;
    P.nyz = nyz;
    P.yz = static_cast<const int2*>(dyz);
    P.nv = a->nv;
    P.TV = TV;
    P.c0 = c0;
    P.ncc = n;
    P.S2 = S2;
    {
      KernelTimer kt_("rho_zy", s);
      hipLaunchKernelGGL((rho_zy<T, NO>), dim3((a->nv + TV - 1) / TV, n), dim3(kBlock), lds_of(TV), s, P);
    }
    XO_CHECK_LAUNCH();
    {
      KernelTimer kt_("rho_x", s);
      hipLaunchKernelGGL((rho_x<T>), dim3((a->ng + kBlock - 1) / kBlock, n, a->nv), dim3(kBlock), 0, s,
                         static_cast<const cplx<T>*>(S2), Nx, nyz, a->ng,
                         static_cast<const int2*>(dgsel), n, c0, a->nc, (T)scale,
                         static_cast<cplx<T>*>(a->rho));
    }
    XO_CHECK_LAUNCH();
  }

  if (a->q0) XO_RET(launch_head_q0<T>(a, s));
  if (a->dE) {
    const int n = a->nc * a->nv;
    {
      KernelTimer kt_("pole_energies", s);
      hipLaunchKernelGGL(pole_energies, dim3((n + 255) / 256), dim3(256), 0, s, a->e_c, a->e_v, a->nc,
                         a->nv, a->dE);
    }
    XO_CHECK_LAUNCH();
  }
  return XO_OK;
}

template <typename T>
static int rho_dispatch(const xo_rho_args* a, hipStream_t s, const Extent& xc, const Extent& xv,
                        const Extent& xe) {
  const int no = std::max(xc.hi[2] - xc.lo[2] + 1, xv.hi[2] - xv.lo[2] + 1);
  if (no <= 16) return rho_run<T, 16>(a, s, xc, xv, xe);
  if (no <= 24) return rho_run<T, 24>(a, s, xc, xv, xe);
  if (no <= 32) return rho_run<T, 32>(a, s, xc, xv, xe);
  set_error("rho: plane-wave sphere spans %d Miller steps along z (max 32)", no);
  return XO_ERR_UNSUPPORTED;
}

}  // namespace
}  // namespace xo

namespace xo {

int validate_rho(const xo_rho_args* a, Extent* pxc, Extent* pxv, Extent* pxe) {
  XO_ARG(a, "xo_rho: null argument block");
  for (int i = 0; i < 3; ++i) {
    XO_ARG(a->n[i] > 0, "xo_rho: grid axis %d is %d", i, a->n[i]);
    if (a->n[i] > kMaxAxis) {
      set_error("xo_rho: grid axis %d = %d exceeds %d", i, a->n[i], kMaxAxis);
      return XO_ERR_UNSUPPORTED;
    }
  }
  XO_ARG(a->npw_c > 0 && a->npw_v > 0 && a->nc > 0 && a->nv > 0 && a->ng > 0,
         "xo_rho: sizes must be positive (npw_c=%d npw_v=%d nc=%d nv=%d ng=%d)", a->npw_c, a->npw_v, a->nc,
         a->nv, a->ng);
  XO_ARG(a->mill_c && a->mill_v && a->mill_g, "xo_rho: Miller lists must be host arrays");
  XO_ARG(a->coef_c && a->coef_v && a->rho, "xo_rho: null device pointer");
  XO_ARG(a->prec == XO_FP64 || a->prec == XO_FP32 || a->prec == XO_BF16X3 || a->prec == XO_BF16,
         "xo_rho: bad precision %d", a->prec);
  XO_ARG(!a->dE || (a->e_c && a->e_v), "xo_rho: dE requested without band energies");
  Extent xc = extent_of(a->mill_c, a->npw_c, nullptr);
  Extent xv = extent_of(a->mill_v, a->npw_v, nullptr);
  Extent xe = extent_of(a->mill_g, a->ng, a->g0);
  for (int i = 0; i < 3; ++i) {
    XO_ARG(xc.hi[i] - xc.lo[i] < a->n[i] && xv.hi[i] - xv.lo[i] < a->n[i],
           "xo_rho: a plane-wave sphere wraps onto itself along axis %d of the %d-point grid", i, a->n[i]);
    const int reach = std::max(xc.hi[i] - xv.lo[i] - xe.lo[i], xe.hi[i] - (xc.lo[i] - xv.hi[i]));
    XO_ARG(reach < a->n[i],
           "xo_rho: grid axis %d (%d points) aliases the orbital product: reach %d must be < %d", i,
           a->n[i], reach, a->n[i]);
  }
  if (a->q0) {
    XO_ARG(a->e_c && a->e_v, "xo_rho: q0 needs band energies");
    XO_ARG(a->npw_c == a->npw_v && a->g0[0] == 0 && a->g0[1] == 0 && a->g0[2] == 0,
           "xo_rho: q0 requires k' = k (same sphere, G0 = 0)");
    for (int i = 0; i < 3 * a->npw_c; ++i)
      XO_ARG(a->mill_c[i] == a->mill_v[i], "xo_rho: q0 requires identical Miller lists at k and k'");
    bool has0 = false;
    for (int g = 0; g < a->ng; ++g)
      has0 |= (a->mill_g[3 * g] == 0 && a->mill_g[3 * g + 1] == 0 && a->mill_g[3 * g + 2] == 0);
    XO_ARG(has0, "xo_rho: q0 requires G = 0 in the G-set");
    double qn = a->qhat[0] * a->qhat[0] + a->qhat[1] * a->qhat[1] + a->qhat[2] * a->qhat[2];
    XO_ARG(qn > 0, "xo_rho: q0 requires a nonzero qhat");
  }
  *pxc = xc;
  *pxv = xv;
  *pxe = xe;
  return XO_OK;
}

// q -> 0 head of a pair whose other columns came from the batched MFMA path
// (complex64 output).
int rho_head_f32(const xo_rho_args* a, hipStream_t s) { return launch_head_q0<float>(a, s); }
int rho_head_f64(const xo_rho_args* a, hipStream_t s) { return launch_head_q0<double>(a, s); }

// Workspace bytes the VALU path requests for one pair (U_c, U_v and one chunk of the
// y-z partial sums), as rho_run sizes them. Host only.
int rho_valu_ws_bytes(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, size_t* bytes) {
  const int no = std::max(xc.hi[2] - xc.lo[2] + 1, xv.hi[2] - xv.lo[2] + 1);
  if (no > 32) {
    set_error("rho: plane-wave sphere spans %d Miller steps along z (max 32)", no);
    return XO_ERR_UNSUPPORTED;
  }
  const int NO = no <= 16 ? 16 : (no <= 24 ? 24 : 32);
  const size_t cs = a->prec == XO_FP64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  const int Nx = a->n[0], Ny = a->n[1];
  const int nz = xe.hi[2] - xe.lo[2] + 1;
  std::vector<char> seen((size_t)Ny * nz, 0);
  size_t nyz = 0;
  for (int g = 0; g < a->ng; ++g) {
    const int ey = a->mill_g[3 * g + 1] - a->g0[1], ez = a->mill_g[3 * g + 2] - a->g0[2];
    char& f = seen[(size_t)pmod(ey, Ny) * nz + (ez - xe.lo[2])];
    nyz += f == 0;
    f = 1;
  }
  const size_t ub = (size_t)Nx * Ny * NO * cs;
  const size_t per_c = (size_t)a->nv * Nx * nyz * cs;
  const size_t ncc = std::max<size_t>(1, std::min<size_t>(a->nc, ((size_t)1 << 30) / per_c));
  *bytes = align_up(ub * a->nc, 256) + align_up(ub * a->nv, 256) + per_c * ncc;
  return XO_OK;
}

// VALU path for one pair (FP64 and FP32).
int rho_valu(const xo_rho_args* a, hipStream_t s) {
  Extent xc, xv, xe;
  XO_RET(validate_rho(a, &xc, &xv, &xe));
  if (a->prec == XO_FP64) return rho_dispatch<double>(a, s, xc, xv, xe);
  return rho_dispatch<float>(a, s, xc, xv, xe);
}

}  // namespace xo
