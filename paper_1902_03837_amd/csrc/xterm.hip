// Bruneval-Gonze extrapolar correction of chi0 (X-terminator subsection,
// Eq. X_term_def; Appendix B, Eqs. rhotw-term, F-term, X-term), FP64.
//
// Empty states above the explicit bands share the extrapolar energy ebar, so
// their part of the sum closes over all states at k:
//   sum_{c > N_b'} rho_cv(G) conj(rho_cv(G')) = <v|e^{i(G-G').r}|v> - sum_{n <= N_b'} rho_nv(G) conj(rho_nv(G'))
// (n over every explicit band, occupied included). Three steps per k-pair:
//   xterm_density  D_v(K) = <v|e^{iK.r}|v> = sum_G conj(c_v(G + K)) c_v(G) for the distinct
//                  K = G - G' of the G-set (direct plane-wave sum, exact)
//   explicit bands the weighted update of the chi0 kernels with pole energies ebar - e_v
//                  and the prefactor's sign flipped (so it is subtracted)
//   xterm_closure  out[w][G][G'] += -pref sum_v W(w, ebar - e_v) D_v(G - G')

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "xo_common.h"

namespace xo {

int chi0_run_signed(const xo_chi0_args* a, hipStream_t s);

namespace {

typedef cplx<double> z;

// One thread per (K, v): D[v][K] = sum_p conj(c_v(box(m_p + K))) c_v(p).
__global__ void xterm_density(const z* __restrict__ coef, int npw, int nv, const int* __restrict__ mill,
                              const int* __restrict__ box, int x0, int y0, int z0, int nbx, int nby, int nbz,
                              const int* __restrict__ kmill, int nK, z* __restrict__ D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (k >= nK) return;
  const int kx = kmill[3 * k], ky = kmill[3 * k + 1], kz = kmill[3 * k + 2];
  const z* c = coef + (size_t)v * npw;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < npw; ++p) {
    const int bx = mill[3 * p] + kx - x0, by = mill[3 * p + 1] + ky - y0, bz = mill[3 * p + 2] + kz - z0;
    if (bx < 0 || by < 0 || bz < 0 || bx >= nbx || by >= nby || bz >= nbz) continue;
    const int q = box[(bz * nby + by) * nbx + bx];
    if (q < 0) continue;
    const z a = c[q], b = c[p];  // conj(a) * b
    re += a.x * b.x + a.y * b.y;
    im += a.x * b.y - a.y * b.x;
  }
  D[(size_t)v * nK + k] = {re, im};
}

// Pole energies of the explicit-band update: dE[v nn + n] = ebar - e_v.
__global__ void xterm_poles(const double* __restrict__ ev, double ebar, int nv, int nn, double* __restrict__ dE) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nv * nn) dE[t] = ebar - ev[t / nn];
}

// out[w][G][G'] += -pref sum_v W(w, ebar - e_v) D_v(G - G'); one thread per (G, G').
__global__ void xterm_closure(const z* __restrict__ D, const int* __restrict__ kidx, int nK, int ng, int nv,
                              const double* __restrict__ ev, double ebar, const double* __restrict__ w, int nw,
                              double pref, z* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ng * ng) return;
  const int k = kidx[e];
  for (int j = 0; j < nw; ++j) {
    double re = 0.0, im = 0.0;
    for (int v = 0; v < nv; ++v) {
      const double d = ebar - ev[v];
      const double wt = 2.0 * d / (w[j] * w[j] + d * d);
      const z dv = D[(size_t)v * nK + k];
      re += wt * dv.x;
      im += wt * dv.y;
    }
    z& o = out[(size_t)j * ng * ng + e];
    o.x -= pref * re;
    o.y -= pref * im;
  }
}

}  // namespace
}  // namespace xo

extern "C" int xo_xterm(const xo_xterm_args* a, void* stream) {
  using namespace xo;
  clear_error();
  XO_ARG(a, "xo_xterm: null argument block");
  XO_ARG(a->npw_v > 0 && a->nv > 0 && a->ng > 0 && a->nw > 0 && a->nn > 0,
         "xo_xterm: sizes must be positive (npw_v=%d nv=%d ng=%d nw=%d nn=%d)", a->npw_v, a->nv, a->ng, a->nw,
         a->nn);
  XO_ARG(a->mill_v && a->mill_g && a->w, "xo_xterm: null host array");
  XO_ARG(a->coef_v && a->e_v && a->rho && a->out, "xo_xterm: null device pointer");
  XO_ARG(a->pref > 0.0 && std::isfinite(a->ebar), "xo_xterm: pref must be positive and ebar finite");
  XO_ARG(a->nw <= 64, "xo_xterm: at most 64 frequencies per call (got %d)", a->nw);
  for (int j = 0; j < a->nw; ++j) XO_ARG(a->w[j] >= 0.0, "xo_xterm: frequency %d is negative", j);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ng = a->ng;

  // distinct K = G - G' and the index of each (G, G')
  std::map<std::tuple<int, int, int>, int> kmap;
  std::vector<int> kidx((size_t)ng * ng), kmill;
  for (int i = 0; i < ng; ++i)
    for (int j = 0; j < ng; ++j) {
      const auto key = std::make_tuple(a->mill_g[3 * i] - a->mill_g[3 * j], a->mill_g[3 * i + 1] - a->mill_g[3 * j + 1],
                                       a->mill_g[3 * i + 2] - a->mill_g[3 * j + 2]);
      auto it = kmap.find(key);
      if (it == kmap.end()) {
        it = kmap.emplace(key, (int)kmap.size()).first;
        kmill.insert(kmill.end(), {std::get<0>(key), std::get<1>(key), std::get<2>(key)});
      }
      kidx[(size_t)i * ng + j] = it->second;
    }
  const int nK = (int)kmap.size();
  // dense Miller box of the valence sphere -> plane-wave index (or -1)
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (int p = 0; p < a->npw_v; ++p)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], a->mill_v[3 * p + c]);
      hi[c] = std::max(hi[c], a->mill_v[3 * p + c]);
    }
  const int nbx = hi[0] - lo[0] + 1, nby = hi[1] - lo[1] + 1, nbz = hi[2] - lo[2] + 1;
  std::vector<int> box((size_t)nbx * nby * nbz, -1);
  for (int p = 0; p < a->npw_v; ++p) {
    const size_t b = ((size_t)(a->mill_v[3 * p + 2] - lo[2]) * nby + (a->mill_v[3 * p + 1] - lo[1])) * nbx +
                     (a->mill_v[3 * p] - lo[0]);
    XO_ARG(box[b] < 0, "xo_xterm: Miller vector %d repeats in mill_v", p);
    box[b] = p;
  }
  const void *dkidx = nullptr, *dkm = nullptr, *dbox = nullptr, *dmv = nullptr, *dw = nullptr;
  XO_RET(device_table(kidx.data(), kidx.size() * sizeof(int), s, &dkidx));
  XO_RET(device_table(kmill.data(), kmill.size() * sizeof(int), s, &dkm));
  XO_RET(device_table(box.data(), box.size() * sizeof(int), s, &dbox));
  XO_RET(device_table(a->mill_v, sizeof(int32_t) * 3 * a->npw_v, s, &dmv));
  XO_RET(device_table(a->w, sizeof(double) * a->nw, s, &dw));
  const size_t dbytes = align_up((size_t)a->nv * nK * sizeof(z), 256);
  const size_t ebytes = align_up((size_t)a->nv * a->nn * sizeof(double), 256);
  void* ws = nullptr;
  XO_RET(workspace(s, 5, dbytes + ebytes, &ws));
  z* D = static_cast<z*>(ws);
  double* dE = reinterpret_cast<double*>(static_cast<char*>(ws) + dbytes);
  {
    KernelTimer kt_("xterm_density", s);
    hipLaunchKernelGGL(xterm_density, dim3((nK + 255) / 256, a->nv), dim3(256), 0, s, static_cast<const z*>(a->coef_v),
                       a->npw_v, a->nv, static_cast<const int*>(dmv), static_cast<const int*>(dbox), lo[0], lo[1],
                       lo[2], nbx, nby, nbz, static_cast<const int*>(dkm), nK, D);
  }
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_("xterm_poles", s);
    const int n = a->nv * a->nn;
    hipLaunchKernelGGL(xterm_poles, dim3((n + 255) / 256), dim3(256), 0, s, a->e_v, a->ebar, a->nv, a->nn, dE);
  }
  XO_CHECK_LAUNCH();
  // explicit bands: out += pref sum W(ebar - e_v) rho rho^H (the update with the sign flipped)
  xo_chi0_args c{};
  c.nt = a->nv * a->nn;
  c.ng = ng;
  c.prec = XO_FP64;
  c.rho = a->rho;
  c.nw = a->nw;
  c.dE = dE;
  c.w = a->w;
  c.pref = -a->pref;
  c.accumulate = 1;
  c.check_dE = 1;  // ebar must lie above every occupied energy
  c.chi0 = a->out;
  {
    const int r = chi0_run_signed(&c, s);
    if (r != XO_OK) {
      if (r == XO_ERR_ARG) set_error("xo_xterm: ebar must lie above every occupied band energy");
      return r;
    }
  }
  {
    KernelTimer kt_("xterm_closure", s);
    const size_t ne = (size_t)ng * ng;
    hipLaunchKernelGGL(xterm_closure, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, D,
                       static_cast<const int*>(dkidx), nK, ng, a->nv, a->e_v, a->ebar, static_cast<const double*>(dw),
                       a->nw, a->pref, reinterpret_cast<z*>(a->out));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}
