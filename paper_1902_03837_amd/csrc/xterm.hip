// Bruneval-Gonze extrapolar correction of chi0 (X-terminator subsection,
// Eq. X_term_def; Appendix B, Eqs. rhotw-term, F-term, X-term).
//
// Empty states above the explicit bands share the extrapolar energy ebar, so
// their part of the sum closes over all states at k:
//   sum_{c > N_b'} rho_cv(G) conj(rho_cv(G')) = <v|e^{i(G-G').r}|v> - sum_{n <= N_b'} rho_nv(G) conj(rho_nv(G'))
// (n over every explicit band, occupied included). Per k-pair:
//   xterm_density  D_v(K) = <v|e^{iK.r}|v> = sum_G conj(c_v(G + K)) c_v(G) for every K = G - G'
//                  of the G-set (direct plane-wave sum in FP64, exact)
//   xterm_weigh    C_w(K) = sum_v W(w, ebar - e_v) D_v(K): the closure depends on (G, G') only
//                  through K, so the sum over v is taken once per distinct K
//   explicit bands the weighted update of the chi0 kernels with pole energies ebar - e_v
//                  and the prefactor's sign flipped (so it is subtracted), in the call's precision
//   xterm_closure  out[w][G][G'] -= pref C_w(G - G') (a gather)

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "xo_common.h"

namespace xo {

int chi0_run_signed(const xo_chi0_args* a, hipStream_t s);

namespace {

typedef cplx<double> z;

// One thread per (K, v): D[v][K] = sum_p conj(c_v(box(m_p + K))) c_v(p), accumulated in FP64.
template <typename C>
__global__ void xterm_density(const C* __restrict__ coef, int npw, int nv, const int* __restrict__ mill,
                              const int* __restrict__ box, int x0, int y0, int z0, int nbx, int nby, int nbz,
                              const int* __restrict__ kmill, int nK, z* __restrict__ D) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (k >= nK) return;
  const int kx = kmill[3 * k], ky = kmill[3 * k + 1], kz = kmill[3 * k + 2];
  const C* c = coef + (size_t)v * npw;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < npw; ++p) {
    const int bx = mill[3 * p] + kx - x0, by = mill[3 * p + 1] + ky - y0, bz = mill[3 * p + 2] + kz - z0;
    if (bx < 0 || by < 0 || bz < 0 || bx >= nbx || by >= nby || bz >= nbz) continue;
    const int q = box[(bz * nby + by) * nbx + bx];
    if (q < 0) continue;
    const double ax = c[q].x, ay = c[q].y, bx_ = c[p].x, by_ = c[p].y;  // conj(a) * b
    re += ax * bx_ + ay * by_;
    im += ax * by_ - ay * bx_;
  }
  D[(size_t)v * nK + k] = {re, im};
}

// C[w][K] = sum_v W(w, ebar - e_v) D[v][K], W(w, d) = 2 d / (w^2 + d^2); one thread per (K, w).
__global__ void xterm_weigh(const z* __restrict__ D, int nK, int nv, const double* __restrict__ ev, double ebar,
                            const double* __restrict__ w, int nw, z* __restrict__ Cw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (k >= nK) return;
  double re = 0.0, im = 0.0;
  for (int v = 0; v < nv; ++v) {
    const double d = ebar - ev[v];
    const double wt = 2.0 * d / (w[j] * w[j] + d * d);
    const z dv = D[(size_t)v * nK + k];
    re += wt * dv.x;
    im += wt * dv.y;
  }
  Cw[(size_t)j * nK + k] = {re, im};
}

// Pole energies of the explicit-band update: dE[v nn + n] = ebar - e_v.
__global__ void xterm_poles(const double* __restrict__ ev, double ebar, int nv, int nn, double* __restrict__ dE) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nv * nn) dE[t] = ebar - ev[t / nn];
}

// out[w][G][G'] -= pref C[w][K(G - G')]; one thread per (G, G'), K from the dense box of
// Miller differences.
__global__ void xterm_closure(const z* __restrict__ Cw, const int* __restrict__ kbox, const int* __restrict__ mg,
                              int ng, int kx0, int ky0, int kz0, int nkx, int nky, int nK, int nw, double pref,
                              z* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ng * ng) return;
  const int i = (int)(e / ng), jj = (int)(e - (size_t)i * ng);
  const int dx = mg[3 * i] - mg[3 * jj] - kx0, dy = mg[3 * i + 1] - mg[3 * jj + 1] - ky0,
            dz = mg[3 * i + 2] - mg[3 * jj + 2] - kz0;
  const int k = kbox[((size_t)dz * nky + dy) * nkx + dx];
  for (int j = 0; j < nw; ++j) {
    const z c = Cw[(size_t)j * nK + k];
    z& o = out[(size_t)j * ng * ng + e];
    o.x -= pref * c.x;
    o.y -= pref * c.y;
  }
}

// Distinct Miller differences of a G-set and their dense index box.
struct KSet {
  std::vector<int32_t> mill;  // the G-set it was built for
  std::vector<int> kbox, kmill;
  int k0[3], nk[3];
};

int kset_for(const int32_t* mg, int ng, std::shared_ptr<const KSet>* out) {
  static std::mutex mu;
  static std::vector<std::shared_ptr<KSet>> cache;
  std::lock_guard<std::mutex> lk(mu);
  for (auto& c : cache)
    if ((int)c->mill.size() == 3 * ng && std::equal(c->mill.begin(), c->mill.end(), mg)) {
      *out = c;
      return XO_OK;
    }
  auto k = std::make_shared<KSet>();
  k->mill.assign(mg, mg + 3 * (size_t)ng);
  int glo[3] = {1 << 30, 1 << 30, 1 << 30}, ghi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  for (int i = 0; i < ng; ++i)
    for (int c = 0; c < 3; ++c) {
      glo[c] = std::min(glo[c], mg[3 * i + c]);
      ghi[c] = std::max(ghi[c], mg[3 * i + c]);
    }
  for (int c = 0; c < 3; ++c) {
    k->k0[c] = glo[c] - ghi[c];
    k->nk[c] = 2 * (ghi[c] - glo[c]) + 1;
  }
  XO_ARG((size_t)k->nk[0] * k->nk[1] * k->nk[2] <= (size_t)1 << 28, "xo_xterm: G-set spans too many Miller indices");
  k->kbox.assign((size_t)k->nk[0] * k->nk[1] * k->nk[2], -1);
  for (int i = 0; i < ng; ++i)
    for (int j = 0; j < ng; ++j) {
      const int d0 = mg[3 * i] - mg[3 * j] - k->k0[0], d1 = mg[3 * i + 1] - mg[3 * j + 1] - k->k0[1],
                d2 = mg[3 * i + 2] - mg[3 * j + 2] - k->k0[2];
      int& slot = k->kbox[((size_t)d2 * k->nk[1] + d1) * k->nk[0] + d0];
      if (slot < 0) {
        slot = (int)(k->kmill.size() / 3);
        k->kmill.insert(k->kmill.end(), {d0 + k->k0[0], d1 + k->k0[1], d2 + k->k0[2]});
      }
    }
  if (cache.size() >= 8) cache.erase(cache.begin());
  cache.push_back(k);
  *out = k;
  return XO_OK;
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
  XO_ARG(a->prec >= XO_FP64 && a->prec <= XO_BF16, "xo_xterm: unknown precision %d", a->prec);
  for (int j = 0; j < a->nw; ++j) XO_ARG(a->w[j] >= 0.0, "xo_xterm: frequency %d is negative", j);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ng = a->ng;

  // dense box of the Miller differences K = G - G' -> index of the distinct K (or -1),
  // kept per G-set (every k-pair of a crystal shares it)
  std::shared_ptr<const KSet> ks;
  XO_RET(kset_for(a->mill_g, ng, &ks));
  const int nK = (int)(ks->kmill.size() / 3);
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
  const void *dkbox = nullptr, *dkm = nullptr, *dbox = nullptr, *dmv = nullptr, *dmg = nullptr, *dw = nullptr;
  XO_RET(device_table(ks->kbox.data(), ks->kbox.size() * sizeof(int), s, &dkbox));
  XO_RET(device_table(ks->kmill.data(), ks->kmill.size() * sizeof(int), s, &dkm));
  XO_RET(device_table(box.data(), box.size() * sizeof(int), s, &dbox));
  XO_RET(device_table(a->mill_v, sizeof(int32_t) * 3 * a->npw_v, s, &dmv));
  XO_RET(device_table(a->mill_g, sizeof(int32_t) * 3 * ng, s, &dmg));
  XO_RET(device_table(a->w, sizeof(double) * a->nw, s, &dw));
  const size_t dbytes = align_up((size_t)a->nv * nK * sizeof(z), 256);
  const size_t cbytes = align_up((size_t)a->nw * nK * sizeof(z), 256);
  const size_t ebytes = align_up((size_t)a->nv * a->nn * sizeof(double), 256);
  void* ws = nullptr;
  XO_RET(workspace(s, 5, dbytes + cbytes + ebytes, &ws));
  z* D = static_cast<z*>(ws);
  z* Cw = reinterpret_cast<z*>(static_cast<char*>(ws) + dbytes);
  double* dE = reinterpret_cast<double*>(static_cast<char*>(ws) + dbytes + cbytes);
  {
    KernelTimer kt_("xterm_density", s);
    const dim3 grid((nK + 255) / 256, a->nv);
    if (a->prec == XO_FP64)
      hipLaunchKernelGGL(xterm_density<z>, grid, dim3(256), 0, s, static_cast<const z*>(a->coef_v), a->npw_v, a->nv,
                         static_cast<const int*>(dmv), static_cast<const int*>(dbox), lo[0], lo[1], lo[2], nbx, nby,
                         nbz, static_cast<const int*>(dkm), nK, D);
    else
      hipLaunchKernelGGL(xterm_density<cplx<float>>, grid, dim3(256), 0, s,
                         static_cast<const cplx<float>*>(a->coef_v), a->npw_v, a->nv, static_cast<const int*>(dmv),
                         static_cast<const int*>(dbox), lo[0], lo[1], lo[2], nbx, nby, nbz,
                         static_cast<const int*>(dkm), nK, D);
  }
  XO_CHECK_LAUNCH();
  {
    KernelTimer kt_("xterm_weigh", s);
    hipLaunchKernelGGL(xterm_weigh, dim3((nK + 255) / 256, a->nw), dim3(256), 0, s, D, nK, a->nv, a->e_v, a->ebar,
                       static_cast<const double*>(dw), a->nw, Cw);
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
  c.prec = a->prec;
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
    hipLaunchKernelGGL(xterm_closure, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, Cw,
                       static_cast<const int*>(dkbox), static_cast<const int*>(dmg), ng, ks->k0[0], ks->k0[1], ks->k0[2],
                       ks->nk[0], ks->nk[1], nK, a->nw, a->pref, reinterpret_cast<z*>(a->out));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}
