// Oscillator strengths on MFMA (split bf16, FP32 accumulation), many k-pairs per
// launch.
//
// The transform of the real-space product conj(psi_c) psi_v (Eq. rhotw) is
// factorised by axis. Orbitals are carried real-space along x and as plane-wave
// (Miller) coefficients along y and z:
//
//   U(x, m_y, m_z) = sum_{m_x} c(m) exp(2 pi i m_x x / Nx)                (orb_x)
//
// For one x-plane the y and z part of the transform of the product is then the
// correlation of the two orbitals' (m_y, m_z) spectra, exact with no grid along
// those axes; the x part is a DFT of the plane values over the real-space grid:
//
//   P_x(e_y, e_z) = sum_b conj(U_c(x, b + e)) U_v(x, b)      b over the valence (m_y, m_z)
//   rho(e)        = 1/Nx sum_x exp(2 pi i e_x x / Nx) P_x(e_y, e_z)
//
// with e = m_G - G0 and rho_cv(e) = sum_a conj(c_c(a)) c_v(a - e), the same
// quantity as the 3D FFT of the product on any alias-free grid. Per x-plane the
// correlation is a complex matrix product: rows are the (e_y, e_z) columns of the
// G-set, the contraction runs over the valence (m_y, m_z) support, and the 16
// valence bands of a workgroup form the columns. The left operand is a 2D Toeplitz
// gather from the conduction orbital's plane, held in LDS.
//
// Complex operands use interleaved real K (k = 2b + a): the left operand is the
// raw (re, im) pair of U_c, the right operand of Re P is (re, im) of U_v and that
// of Im P is (im, -re). Every FP32 value x enters as hi = bf16(x) and lo =
// bf16(x - hi); each product is hi*hi + hi*lo + lo*hi, accumulated in FP32.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "bf16x3.h"
#include "rho_geom.h"

namespace xo {

int rho_valu(const xo_rho_args* a, hipStream_t s);
int rho_head_f32(const xo_rho_args* a, hipStream_t s);
int rho_head_f64(const xo_rho_args* a, hipStream_t s);
int rho_batch_gemm(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                   hipStream_t s);
int rho_batch_finish(const xo_rho_args* p, int n, hipStream_t s);
int rho_gemm_ws_bytes(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                      size_t* bytes);
int rho_valu_ws_bytes(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, size_t* bytes);
int rho_batch_gemm_fp(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                      hipStream_t s);

namespace {

constexpr int kBlock = 256;

// --------------------------------------------------------------- orbitals --
struct OrbX {
  const float2* coef;   // [nb][npw]
  const int* boxidx;    // [npw] (col * nbx + bx) of each plane wave, col = by * nbz + bz
  const int* outcol;    // [nout] box column written at each output position, or -1
  uint32_t* Uhi;        // [nb][Nx][nout] split bf16 (re, im) pairs
  uint32_t* Ulo;
  int npw, nb, nout, nbx, ncol, xlo;
};

// One workgroup per (band, side): scatter the plane waves into a dense
// (column, m_x) box in LDS, transform every needed column along x and write
// the split values in the layout the rho kernel reads.
__global__ void __launch_bounds__(kBlock) orb_x(const OrbX* __restrict__ sides, int Nx,
                                                const float2* __restrict__ twt) {
  extern __shared__ unsigned char smem[];
  const OrbX S = sides[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= S.nb) return;
  float2* tw = reinterpret_cast<float2*>(smem);  // [Nx]
  float2* box = tw + Nx;                         // [ncol][nbx]
  for (int k = threadIdx.x; k < Nx; k += kBlock) tw[k] = twt[k];
  for (int e = threadIdx.x; e < S.ncol * S.nbx; e += kBlock) box[e] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int p = threadIdx.x; p < S.npw; p += kBlock) box[S.boxidx[p]] = S.coef[(size_t)b * S.npw + p];
  __syncthreads();
  uint32_t* uh = S.Uhi + (size_t)b * Nx * S.nout;
  uint32_t* ul = S.Ulo + (size_t)b * Nx * S.nout;
  for (int it = threadIdx.x; it < Nx * S.nout; it += kBlock) {
    const int x = it / S.nout, j = it - (it / S.nout) * S.nout;
    const int col = S.outcol[j];
    float2 acc = make_float2(0.f, 0.f);
    if (col >= 0) {
      const float2* row = box + col * S.nbx;
      int k = pmod(S.xlo * x, Nx);
      for (int bx = 0; bx < S.nbx; ++bx) {
        const float2 c = row[bx], w = tw[k];
        acc.x = fmaf(c.x, w.x, fmaf(-c.y, w.y, acc.x));
        acc.y = fmaf(c.x, w.y, fmaf(c.y, w.x, acc.y));
        k += x;
        if (k >= Nx) k -= Nx;
      }
    }
    uint32_t h, l;
    split2(acc.x, acc.y, h, l);
    uh[it] = h;
    ul[it] = l;
  }
}

// ------------------------------------------------------------------- rho --
// Per-pair geometry tables, one int array (offsets below are into it):
//   cpos[ncb]          extended-box position of each conduction box entry, or -1
//   kg[Kp/4]           box offset of each valence K-group (4 consecutive m_z)
//   oe[nE][MT*16]      box offset of each (e_y, e_z) row of each e-group
//   gl[nE][GPT*64]     owned G entries: G | row << 16 | (e_x mod Nx) << 24, or -1
struct PairDesc {
  const uint32_t* Uc_hi;  // [nc][Nx][ncb]
  const uint32_t* Uc_lo;
  const uint32_t* Uv_hi;  // [nv][Nx][Kp]
  const uint32_t* Uv_lo;
  float2* rho;            // [nv][nc][ng]
  const int* tab;
  int cpos, kg, oe, gl;   // offsets into tab
  int nc, nv, nvt, nE, ncb, Kp, CS, wg0;
  int mts;                // M-tile stride of the oe table (the pair's own largest group)
  int mte[8];             // M-tiles used by each e-group (at most 8 groups)
};

constexpr int kMaxGroups = 8;
constexpr int kPS = 18;  // row stride (float2) of the partial sums: 16 bands + 2 padding, spreads LDS banks
constexpr int kMaxPF = 2;  // conduction box entries per thread per plane

template <int MT, int GPT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) rho_yz(const PairDesc* __restrict__ pairs, int npairs, int nwg, int Nx,
                                                  int ng, const float2* __restrict__ twt, float scale) {
  extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
  // XCD-aware order: workgroup b runs on XCD b % 8; XCD x gets the contiguous
  // logical range [x * per, (x + 1) * per), so a pair's valence orbitals stay in
  // that XCD's L2 while its conduction bands stream through.
  const int per = (nwg + 7) >> 3;
  const int L = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (L >= nwg) return;
  int lo = 0, hi = npairs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pairs[mid].wg0 <= L) lo = mid; else hi = mid - 1;
  }
  const PairDesc& P = pairs[lo];
  const int nE = P.nE, nvt = P.nvt, Kp = P.Kp, CS = P.CS, ncb = P.ncb;
  const int local = L - P.wg0;
  const int c = local / (nvt * nE);
  const int rem = local - c * (nvt * nE);
  const int vt = rem / nE, eg = rem - (rem / nE) * nE;
  const int mte = P.mte[eg];
  const int tid = threadIdx.x, l = tid & 63, l16 = l & 15, q = l >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int* tab = P.tab;

  const int NxP = (Nx + 1) & ~1;
  float2* tw = reinterpret_cast<float2*>(lds);                 // [Nx] exp(2 pi i k / Nx)
  float2* twp = tw + NxP;                                       // [2][Nx] this plane's exp(2 pi i e_x x / Nx)
  int* kg = reinterpret_cast<int*>(twp + 2 * NxP);              // [Kp/4], padded to a multiple of 4
  uint32_t* cb = reinterpret_cast<uint32_t*>(kg + ((Kp / 4 + 3) & ~3));  // [2][4][CS]: hi copies, lo copies
  float2* Pp = reinterpret_cast<float2*>(cb + 8 * CS);          // [4][MT*16][kPS]

  for (int k = tid; k < Nx; k += kBlock) tw[k] = twt[k];
  for (int k = tid; k < Kp / 4; k += kBlock) kg[k] = gld<int>(tab + P.kg + k);
  for (int k = tid; k < 8 * CS; k += kBlock) cb[k] = 0u;

  // A-operand row offsets of this lane (row l16 of every M-tile)
  int oe[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) oe[mt] = mt < mte ? gld<int>(tab + P.oe + (eg * P.mts + mt) * 16 + l16) : 0;
  // owned outputs: G entries l + 64 i, valence bands 4w .. 4w+3 of the tile
  int gi[GPT];
  float2 acc[GPT][4];
#pragma unroll
  for (int i = 0; i < GPT; ++i) {
    gi[i] = gld<int>(tab + P.gl + eg * GPT * 64 + l + 64 * i);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = make_float2(0.f, 0.f);
  }
  // conduction entries this thread moves into LDS each plane
  int cp[kMaxPF];
  uint32_t ph[kMaxPF], pl[kMaxPF];
  const size_t cbase = (size_t)c * Nx * ncb;
#pragma unroll
  for (int f = 0; f < kMaxPF; ++f) {
    const int j = tid + kBlock * f;
    cp[f] = j < ncb ? gld<int>(tab + P.cpos + j) : -1;
    ph[f] = cp[f] >= 0 ? gld<uint32_t>(P.Uc_hi + cbase + j) : 0u;
    pl[f] = cp[f] >= 0 ? gld<uint32_t>(P.Uc_lo + cbase + j) : 0u;
  }
  __syncthreads();  // boxes zeroed and twiddles loaded before the first plane
  // work items (K-chunk, M-tile), K-chunk major; wave w takes a contiguous share
  const int nK = Kp / 16;
  const int nit = nK * mte;
  const int it0 = (w * nit) >> 2, it1 = ((w + 1) * nit) >> 2;
  const int v = vt * 16 + l16;
  const bool vok = v < P.nv;
  const size_t vrow = (size_t)(vok ? v : 0) * Nx;

  for (int x = 0; x < Nx; ++x) {
    // ---- conduction plane into the four shifted copies: copy s holds box[j + s] at j
#pragma unroll
    for (int f = 0; f < kMaxPF; ++f) {
      const int p = cp[f];
      if (p >= 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (p >= s) {
            cb[s * CS + p - s] = ph[f];
            cb[(4 + s) * CS + p - s] = pl[f];
          }
        }
      }
    }
    // twiddle row of this plane (double buffered: the previous row may still be read)
    for (int e = tid; e < Nx; e += kBlock) twp[(x & 1) * NxP + e] = tw[(e * x) % Nx];
    if (x + 1 < Nx) {
      const size_t o = cbase + (size_t)(x + 1) * ncb;
#pragma unroll
      for (int f = 0; f < kMaxPF; ++f) {
        if (cp[f] >= 0) {
          ph[f] = gld<uint32_t>(P.Uc_hi + o + tid + kBlock * f);
          pl[f] = gld<uint32_t>(P.Uc_lo + o + tid + kBlock * f);
        }
      }
    }
    __syncthreads();
    // ---- correlation on MFMA
    f4 re[MT], im[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      re[mt] = f4{0.f, 0.f, 0.f, 0.f};
      im[mt] = f4{0.f, 0.f, 0.f, 0.f};
    }
    if (it0 < it1) {
      const int kc0 = it0 / mte, kc1 = (it1 - 1) / mte;
      const uint32_t* vh = P.Uv_hi + (vrow + x) * Kp + 4 * q;
      const uint32_t* vl = P.Uv_lo + (vrow + x) * Kp + 4 * q;
      u4 nbh = vok ? gld<u4>(vh + kc0 * 16) : u4{0u, 0u, 0u, 0u};
      u4 nbl = vok ? gld<u4>(vl + kc0 * 16) : u4{0u, 0u, 0u, 0u};
      for (int kc = kc0; kc <= kc1; ++kc) {
        const u4 bh = nbh, bl = nbl;
        if (kc < kc1 && vok) {
          nbh = gld<u4>(vh + (kc + 1) * 16);
          nbl = gld<u4>(vl + (kc + 1) * 16);
        }
        u4 rh, rl;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          rh[m] = rot_pos(bh[m]);
          rl[m] = rot_pos(bl[m]);
        }
        const int ob = kg[kc * 4 + q];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int item = kc * mte + mt;
          if (mt < mte && item >= it0 && item < it1) {
            const int o = ob + oe[mt];
            const int a = o + (int)__umul24((unsigned)(o & 3), (unsigned)(CS - 1));  // copy (o & 3), aligned
            const u4 ah = *reinterpret_cast<const u4*>(cb + a);
            const u4 al = *reinterpret_cast<const u4*>(cb + 4 * CS + a);
            re[mt] = mma3(ah, al, bh, bl, re[mt]);
            im[mt] = mma3(ah, al, rh, rl, im[mt]);
          }
        }
      }
    }
    // ---- partial sums of this wave: rows mt*16 + 4q + r, column l16
    float2* Pw = Pp + w * (MT * 16 * kPS);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      if (mt < mte) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Pw[(mt * 16 + 4 * q + r) * kPS + l16] = make_float2(re[mt][r], im[mt][r]);
      }
    }
    __syncthreads();
    // ---- fixed-order reduction over the four waves into slice 0
    for (int e = tid; e < mte * 256; e += kBlock) {
      const int o = (e >> 4) * kPS + (e & 15);
      const float2 a0 = Pp[o], a1 = Pp[MT * 16 * kPS + o], a2 = Pp[2 * MT * 16 * kPS + o],
                   a3 = Pp[3 * MT * 16 * kPS + o];
      Pp[o] = make_float2(((a0.x + a1.x) + a2.x) + a3.x, ((a0.y + a1.y) + a2.y) + a3.y);
    }
    __syncthreads();
    // ---- x transform into the owned rho entries
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      if (gi[i] >= 0) {
        const int row = (gi[i] >> 16) & 0xff;
        const float4* sp = reinterpret_cast<const float4*>(Pp + row * kPS + 4 * w);
        const float4 s01 = sp[0], s23 = sp[1];
        const float2 t = twp[(x & 1) * NxP + ((unsigned)gi[i] >> 24)];
        acc[i][0].x = fmaf(s01.x, t.x, fmaf(-s01.y, t.y, acc[i][0].x));
        acc[i][0].y = fmaf(s01.x, t.y, fmaf(s01.y, t.x, acc[i][0].y));
        acc[i][1].x = fmaf(s01.z, t.x, fmaf(-s01.w, t.y, acc[i][1].x));
        acc[i][1].y = fmaf(s01.z, t.y, fmaf(s01.w, t.x, acc[i][1].y));
        acc[i][2].x = fmaf(s23.x, t.x, fmaf(-s23.y, t.y, acc[i][2].x));
        acc[i][2].y = fmaf(s23.x, t.y, fmaf(s23.y, t.x, acc[i][2].y));
        acc[i][3].x = fmaf(s23.z, t.x, fmaf(-s23.w, t.y, acc[i][3].x));
        acc[i][3].y = fmaf(s23.z, t.y, fmaf(s23.w, t.x, acc[i][3].y));
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int vv = vt * 16 + 4 * w + u;
    if (vv < P.nv) {
      float2* out = P.rho + ((size_t)vv * P.nc + c) * ng;
#pragma unroll
      for (int i = 0; i < GPT; ++i)
        if (gi[i] >= 0) gst<f2v>(out + (gi[i] & 0xffff), f2v{acc[i][u].x * scale, acc[i][u].y * scale});
    }
  }
}

struct PoleDesc {
  const double* ec;
  const double* ev;
  double* dE;
  int nc, nv;
};

// dE[v][c] = e_c - e_v for every pair of the batch (blockIdx.y = pair).
__global__ void pole_energies_b(const PoleDesc* __restrict__ pd) {
  const PoleDesc P = pd[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.nc * P.nv; i += gridDim.x * blockDim.x) {
    const int v = i / P.nc, c = i - (i / P.nc) * P.nc;
    P.dE[i] = P.ec[c] - P.ev[v];
  }
}

// ------------------------------------------------------------------ host --
// Box of a plane-wave sphere: dense (m_y, m_z) columns, m_x along the column.
struct SphereBox {
  int xlo, ylo, zlo, nbx, nby, nbz;
  std::vector<int> boxidx;  // per plane wave: (by * nbz + bz) * nbx + bx
};

static SphereBox sphere_box(const int32_t* m, int npw, const Extent& ex) {
  SphereBox b;
  b.xlo = ex.lo[0];
  b.ylo = ex.lo[1];
  b.zlo = ex.lo[2];
  b.nbx = ex.hi[0] - ex.lo[0] + 1;
  b.nby = ex.hi[1] - ex.lo[1] + 1;
  b.nbz = ex.hi[2] - ex.lo[2] + 1;
  b.boxidx.resize(npw);
  for (int i = 0; i < npw; ++i)
    b.boxidx[i] = ((m[3 * i + 1] - b.ylo) * b.nbz + (m[3 * i + 2] - b.zlo)) * b.nbx + (m[3 * i] - b.xlo);
  return b;
}

struct PairGeo {
  std::vector<int> tab;
  std::vector<int> outc, outv;  // output columns of the two orbital transforms
  int cpos = 0, kg = 0, oe = 0, gl = 0;
  int ncb = 0, Kp = 0, CS = 0, nE = 0, MT = 0;
  int mte[kMaxGroups] = {0};
};

// Geometry of one pair: valence K-groups, extended conduction box, e-groups.
// Returns false when the pair does not fit the kernel's limits.
static bool pair_geo(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe,
                     const SphereBox& bc, const SphereBox& bv, int GPT, PairGeo* g) {
  const int Nx = a->n[0];
  // valence K-groups: per m_y row of the sphere, m_z in runs of four
  std::vector<int> zl(bv.nby, 1 << 30), zh(bv.nby, -(1 << 30));
  for (int i = 0; i < a->npw_v; ++i) {
    const int by = a->mill_v[3 * i + 1] - bv.ylo, z = a->mill_v[3 * i + 2];
    zl[by] = std::min(zl[by], z);
    zh[by] = std::max(zh[by], z);
  }
  std::vector<std::pair<int, int>> grp;  // (m_y, first m_z)
  int zmaxg = xv.lo[2];
  for (int by = 0; by < bv.nby; ++by)
    for (int z0 = zl[by]; z0 <= zh[by]; z0 += 4) {
      grp.push_back({bv.ylo + by, z0});
      zmaxg = std::max(zmaxg, z0 + 3);
    }
  while (grp.size() % 4) grp.push_back({INT32_MIN, 0});
  g->Kp = (int)grp.size() * 4;
  g->outv.assign(g->Kp, -1);
  for (size_t k = 0; k < grp.size(); ++k) {
    if (grp[k].first == INT32_MIN) continue;
    for (int j = 0; j < 4; ++j) {
      const int by = grp[k].first - bv.ylo, bz = grp[k].second + j - bv.zlo;
      if (bz < bv.nbz) g->outv[4 * k + j] = by * bv.nbz + bz;
    }
  }
  // extended conduction box: every U_c(b + e) the gather can touch
  const int Y0 = xv.lo[1] + xe.lo[1], Y1 = xv.hi[1] + xe.hi[1];
  const int Z0 = xv.lo[2] + xe.lo[2], Z1 = zmaxg + xe.hi[2];
  const int EY = Y1 - Y0 + 1, EZ = Z1 - Z0 + 1;
  g->CS = (EY * EZ + 4 + 3) & ~3;
  g->ncb = bc.nby * bc.nbz;
  g->outc.resize(g->ncb);
  for (int j = 0; j < g->ncb; ++j) g->outc[j] = j;
  std::vector<int> cpos(g->ncb, -1);
  for (int by = 0; by < bc.nby; ++by)
    for (int bz = 0; bz < bc.nbz; ++bz) {
      const int y = bc.ylo + by, z = bc.zlo + bz;
      if (y >= Y0 && y <= Y1 && z >= Z0 && z <= Z1) cpos[by * bc.nbz + bz] = (y - Y0) * EZ + (z - Z0);
    }
  std::vector<int> kgv(grp.size(), 0);
  for (size_t k = 0; k < grp.size(); ++k)
    if (grp[k].first != INT32_MIN) kgv[k] = (grp[k].first - xv.lo[1]) * EZ + (grp[k].second - xv.lo[2]);
  // e-columns (distinct (e_y, e_z)), sorted; G lists per column
  std::map<std::pair<int, int>, std::vector<int>> cols;
  for (int i = 0; i < a->ng; ++i)
    cols[{a->mill_g[3 * i + 1] - a->g0[1], a->mill_g[3 * i + 2] - a->g0[2]}].push_back(i);
  // e-groups: consecutive columns, at most 128 columns and GPT*64 G each
  std::vector<std::vector<std::pair<int, int>>> groups(1);
  std::vector<int> gcount(1, 0);
  for (auto& kv : cols) {
    const int n = (int)kv.second.size();
    if (n > GPT * 64) return false;
    if (groups.back().size() == 128 || gcount.back() + n > GPT * 64) {
      groups.emplace_back();
      gcount.push_back(0);
    }
    groups.back().push_back(kv.first);
    gcount.back() += n;
  }
  g->nE = (int)groups.size();
  if (g->nE > kMaxGroups) return false;
  g->MT = 0;
  for (int e = 0; e < g->nE; ++e) {
    g->mte[e] = ((int)groups[e].size() + 15) / 16;
    g->MT = std::max(g->MT, g->mte[e]);
  }
  const int MT = g->MT;
  std::vector<int> oe((size_t)g->nE * MT * 16, 0), gl((size_t)g->nE * GPT * 64, -1);
  for (int e = 0; e < g->nE; ++e) {
    std::vector<int> gs;
    for (size_t r = 0; r < groups[e].size(); ++r) {
      const auto& key = groups[e][r];
      oe[(size_t)e * MT * 16 + r] = (key.first - xe.lo[1]) * EZ + (key.second - xe.lo[2]);
      for (int gidx : cols[key]) gs.push_back(gidx | (int)(r << 16));
    }
    // by row, then G: neighbouring lanes read the same or adjacent rows of the partial sums
    std::sort(gs.begin(), gs.end());
    for (size_t j = 0; j < gs.size(); ++j) {
      const int gidx = gs[j] & 0xffff;
      const int ex = pmod(a->mill_g[3 * gidx] - a->g0[0], Nx);
      gl[(size_t)e * GPT * 64 + j] = gs[j] | (ex << 24);
    }
  }
  g->tab.clear();
  g->cpos = 0;
  g->tab.insert(g->tab.end(), cpos.begin(), cpos.end());
  g->kg = (int)g->tab.size();
  g->tab.insert(g->tab.end(), kgv.begin(), kgv.end());
  g->oe = (int)g->tab.size();
  g->tab.insert(g->tab.end(), oe.begin(), oe.end());
  g->gl = (int)g->tab.size();
  g->tab.insert(g->tab.end(), gl.begin(), gl.end());
  (void)xc;
  return true;
}

template <int MT, int GPT>
static int launch_rho(const void* dpairs, int npairs, int nwg, int Nx, int ng, const void* dtw, hipStream_t s,
                      size_t lds) {
  if (lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rho_yz<MT, GPT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    KernelTimer kt_("rho_yz", s);
    hipLaunchKernelGGL((rho_yz<MT, GPT>), dim3(8 * ((nwg + 7) / 8)), dim3(kBlock), lds, s,
                       static_cast<const PairDesc*>(dpairs), npairs, nwg, Nx, ng, static_cast<const float2*>(dtw),
                       (float)(1.0 / (double)Nx));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <int GPT>
static int launch_rho_mt(int MT, const void* dpairs, int npairs, int nwg, int Nx, int ng, const void* dtw,
                         hipStream_t s, size_t lds) {
  switch (MT) {
    case 1: return launch_rho<1, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 2: return launch_rho<2, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 3: return launch_rho<3, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 4: return launch_rho<4, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 5: return launch_rho<5, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 6: return launch_rho<6, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    case 7: return launch_rho<7, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
    default: return launch_rho<8, GPT>(dpairs, npairs, nwg, Nx, ng, dtw, s, lds);
  }
}

// Whether a batch can take one batched MFMA launch (same precision, grid x axis
// and G-set); else each pair runs on its own.
static bool mfma_eligible(const xo_rho_args* p, int n) {
  const xo_rho_args& a0 = p[0];
  if (a0.ng > 65535) return false;
  for (int i = 0; i < n; ++i) {
    if (p[i].prec != a0.prec) return false;
    if (p[i].n[0] != a0.n[0] || p[i].ng != a0.ng) return false;
    if (std::memcmp(p[i].mill_g, a0.mill_g, sizeof(int32_t) * 3 * a0.ng) != 0) return false;
  }
  return true;
}

// Geometry of one pair and its device tables, cached by content (Miller lists,
// G0, grid, G entries per workgroup) for the life of the device tables.
struct GeoEntry {
  SphereBox bc, bv;
  PairGeo g;
  const void* dbox[2];
  const void* dout[2];
  const void* dtab;
  unsigned gen;
};

static int pair_entry(const xo_rho_args* a, const Extent& xc, const Extent& xv, const Extent& xe, int GPT,
                      hipStream_t s, const GeoEntry** out) {
  // Lookup by the caller's Miller-list pointers and scalars, then a full
  // comparison of the lists' contents against the copy kept with the entry
  // (a reused buffer with new contents is a miss).
  struct Key {
    std::vector<int32_t> scal, mc, mv, mg;
  };
  static std::mutex mu;
  static std::map<std::vector<intptr_t>, std::vector<std::pair<Key, std::unique_ptr<GeoEntry>>>> cache;
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  const std::vector<intptr_t> pk = {dev, a->n[0], GPT, a->g0[0], a->g0[1], a->g0[2], a->npw_c, a->npw_v, a->ng,
                                    (intptr_t)a->mill_c, (intptr_t)a->mill_v, (intptr_t)a->mill_g};
  auto same = [&](const Key& k) {
    return std::memcmp(k.mc.data(), a->mill_c, 12 * (size_t)a->npw_c) == 0 &&
           std::memcmp(k.mv.data(), a->mill_v, 12 * (size_t)a->npw_v) == 0 &&
           std::memcmp(k.mg.data(), a->mill_g, 12 * (size_t)a->ng) == 0;
  };
  const unsigned gen = table_generation();
  std::lock_guard<std::mutex> lk(mu);
  auto& bucket = cache[pk];
  std::unique_ptr<GeoEntry>* slotp = nullptr;
  for (auto& kv : bucket)
    if (same(kv.first)) slotp = &kv.second;
  if (slotp && (*slotp)->gen == gen) {
    *out = (*slotp)->g.nE ? slotp->get() : nullptr;
    return XO_OK;
  }
  GeoEntry e;
  e.gen = gen;
  e.bc = sphere_box(a->mill_c, a->npw_c, xc);
  e.bv = sphere_box(a->mill_v, a->npw_v, xv);
  if (!pair_geo(a, xc, xv, xe, e.bc, e.bv, GPT, &e.g) || e.g.ncb > kBlock * kMaxPF || e.g.MT > 8) {
    e.g.nE = 0;  // remembered as unsupported
  } else {
    XO_RET(device_table(e.bc.boxidx.data(), e.bc.boxidx.size() * sizeof(int), s, &e.dbox[0]));
    XO_RET(device_table(e.bv.boxidx.data(), e.bv.boxidx.size() * sizeof(int), s, &e.dbox[1]));
    XO_RET(device_table(e.g.outc.data(), e.g.outc.size() * sizeof(int), s, &e.dout[0]));
    XO_RET(device_table(e.g.outv.data(), e.g.outv.size() * sizeof(int), s, &e.dout[1]));
    XO_RET(device_table(e.g.tab.data(), e.g.tab.size() * sizeof(int), s, &e.dtab));
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
  *slotp = std::make_unique<GeoEntry>(std::move(e));
  *out = (*slotp)->g.nE ? slotp->get() : nullptr;
  return XO_OK;
}

// LDS bytes of the axis-factorised kernel for a batch whose largest row-tile count is MT.
static size_t mfma_lds(int Nx, const PairGeo& g, int MT) {
  return (size_t)3 * ((Nx + 1) & ~1) * sizeof(float2) + (size_t)((g.Kp / 4 + 3) & ~3) * 4 + (size_t)8 * g.CS * 4 +
         (size_t)4 * MT * 16 * kPS * sizeof(float2);
}

// Workspace bytes the axis-factorised path requests for the batch, or XO_ERR_UNSUPPORTED
// when it cannot take it. Host geometry only.
static int mfma_ws_bytes(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                         size_t* bytes) {
  const int Nx = p[0].n[0], GPT = p[0].ng <= 128 ? 2 : 8;
  std::vector<PairGeo> g(n);
  int MT = 1;
  for (int i = 0; i < n; ++i) {
    const SphereBox bc = sphere_box(p[i].mill_c, p[i].npw_c, xc[i]);
    const SphereBox bv = sphere_box(p[i].mill_v, p[i].npw_v, xv[i]);
    if (!pair_geo(&p[i], xc[i], xv[i], xe[i], bc, bv, GPT, &g[i]) || g[i].ncb > kBlock * kMaxPF || g[i].MT > 8)
      return XO_ERR_UNSUPPORTED;
    MT = std::max(MT, g[i].MT);
  }
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    if (mfma_lds(Nx, g[i], MT) > 160 * 1024) return XO_ERR_UNSUPPORTED;
    tot += align_up((size_t)p[i].nc * Nx * g[i].ncb, 64) + align_up((size_t)p[i].nv * Nx * g[i].Kp, 64);
  }
  *bytes = 2 * tot * sizeof(uint32_t);
  return XO_OK;
}

static int rho_batch_mfma(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                          hipStream_t s) {
  const int Nx = p[0].n[0], ng = p[0].ng;
  const int GPT = ng <= 128 ? 2 : 8;
  std::vector<const GeoEntry*> ge(n);
  int MT = 1;
  for (int i = 0; i < n; ++i) {
    XO_RET(pair_entry(&p[i], xc[i], xv[i], xe[i], GPT, s, &ge[i]));
    if (!ge[i]) return XO_ERR_UNSUPPORTED;
    MT = std::max(MT, ge[i]->g.MT);
  }
  // LDS fit checked before anything is enqueued
  for (int i = 0; i < n; ++i)
    if (mfma_lds(Nx, ge[i]->g, MT) > 160 * 1024) return XO_ERR_UNSUPPORTED;
  std::vector<float2> tw(Nx);
  for (int k = 0; k < Nx; ++k) {
    const double th = 2.0 * M_PI * k / Nx;
    tw[k] = make_float2((float)std::cos(th), (float)std::sin(th));
  }
  const void* dtw = nullptr;
  XO_RET(device_table(tw.data(), tw.size() * sizeof(float2), s, &dtw));

  // workspace: transformed orbitals of every pair (conduction box, valence K rows)
  std::vector<size_t> offc(n), offv(n);
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    offc[i] = tot;
    tot += align_up((size_t)p[i].nc * Nx * ge[i]->g.ncb, 64);
    offv[i] = tot;
    tot += align_up((size_t)p[i].nv * Nx * ge[i]->g.Kp, 64);
  }
  void* ws = nullptr;
  XO_RET(workspace(s, 3, 2 * tot * sizeof(uint32_t), &ws));
  uint32_t* Uhi0 = static_cast<uint32_t*>(ws);
  uint32_t* Ulo0 = Uhi0 + tot;

  std::vector<OrbX> sides(2 * n);
  int maxnb = 0;
  size_t orb_lds = 0;
  for (int i = 0; i < n; ++i) {
    for (int side = 0; side < 2; ++side) {
      const GeoEntry& e = *ge[i];
      const SphereBox& b = side ? e.bv : e.bc;
      OrbX& o = sides[2 * i + side];
      o.coef = static_cast<const float2*>(side ? p[i].coef_v : p[i].coef_c);
      o.boxidx = static_cast<const int*>(e.dbox[side]);
      o.outcol = static_cast<const int*>(e.dout[side]);
      o.Uhi = Uhi0 + (side ? offv[i] : offc[i]);
      o.Ulo = Ulo0 + (side ? offv[i] : offc[i]);
      o.npw = side ? p[i].npw_v : p[i].npw_c;
      o.nb = side ? p[i].nv : p[i].nc;
      o.nout = side ? e.g.Kp : e.g.ncb;
      o.nbx = b.nbx;
      o.ncol = b.nby * b.nbz;
      o.xlo = b.xlo;
      maxnb = std::max(maxnb, o.nb);
      orb_lds = std::max(orb_lds, (size_t)(Nx + o.ncol * o.nbx) * sizeof(float2));
    }
  }
  if (orb_lds > 160 * 1024) return XO_ERR_UNSUPPORTED;
  const void* dsides = nullptr;
  XO_RET(device_table(sides.data(), sides.size() * sizeof(OrbX), s, &dsides));
  if (orb_lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&orb_x), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)orb_lds));
  {
    KernelTimer kt_("orb_x", s);
    hipLaunchKernelGGL(orb_x, dim3(maxnb, 2 * n), dim3(kBlock), orb_lds, s, static_cast<const OrbX*>(dsides), Nx,
                       static_cast<const float2*>(dtw));
  }
  XO_CHECK_LAUNCH();

  std::vector<PairDesc> pd(n);
  int nwg = 0;
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    const PairGeo& g = ge[i]->g;
    PairDesc& d = pd[i];
    d.Uc_hi = Uhi0 + offc[i];
    d.Uc_lo = Ulo0 + offc[i];
    d.Uv_hi = Uhi0 + offv[i];
    d.Uv_lo = Ulo0 + offv[i];
    d.rho = static_cast<float2*>(p[i].rho);
    d.tab = static_cast<const int*>(ge[i]->dtab);
    d.cpos = g.cpos;
    d.kg = g.kg;
    d.oe = g.oe;
    d.gl = g.gl;
    d.nc = p[i].nc;
    d.nv = p[i].nv;
    d.nvt = (p[i].nv + 15) / 16;
    d.nE = g.nE;
    d.ncb = g.ncb;
    d.Kp = g.Kp;
    d.CS = g.CS;
    d.mts = g.MT;
    for (int e = 0; e < kMaxGroups; ++e) d.mte[e] = e < g.nE ? g.mte[e] : 0;
    d.wg0 = nwg;
    nwg += d.nc * d.nvt * d.nE;
    lds = std::max(lds, mfma_lds(Nx, g, MT));
  }
  const void* dpairs = nullptr;
  XO_RET(device_table(pd.data(), pd.size() * sizeof(PairDesc), s, &dpairs));
  if (GPT == 2)
    XO_RET(launch_rho_mt<2>(MT, dpairs, n, nwg, Nx, ng, dtw, s, lds));
  else
    XO_RET(launch_rho_mt<8>(MT, dpairs, n, nwg, Nx, ng, dtw, s, lds));
  return rho_batch_finish(p, n, s);
}

}  // namespace

// After the batched MFMA kernels: q -> 0 heads and pole energies of the batch.
int rho_batch_finish(const xo_rho_args* p, int n, hipStream_t s) {
  // q -> 0: the G = 0 column of such pairs is the velocity head, written over the transform's value
  for (int i = 0; i < n; ++i)
    if (p[i].q0) XO_RET(p[i].prec == XO_FP64 ? rho_head_f64(&p[i], s) : rho_head_f32(&p[i], s));

  std::vector<PoleDesc> poles;
  int maxm = 0;
  for (int i = 0; i < n; ++i) {
    if (!p[i].dE) continue;
    poles.push_back({p[i].e_c, p[i].e_v, p[i].dE, p[i].nc, p[i].nv});
    maxm = std::max(maxm, p[i].nc * p[i].nv);
  }
  if (!poles.empty()) {
    const void* dpoles = nullptr;
    XO_RET(device_table(poles.data(), poles.size() * sizeof(PoleDesc), s, &dpoles));
    {
      KernelTimer kt_("pole_energies", s);
      hipLaunchKernelGGL(pole_energies_b, dim3(std::min(64, (maxm + 255) / 256), (unsigned)poles.size()),
                         dim3(256), 0, s, static_cast<const PoleDesc*>(dpoles));
    }
    XO_CHECK_LAUNCH();
  }
  return XO_OK;
}

// Which kernel a batch may take: the gathered product when its tables fit in
// LDS, else the transform (axis-factorised on MFMA in split bf16 for both bf16
// forms, on VALU pair by pair for FP32 / FP64). XO_RHO_KERNEL=gemm or =transform restricts the choice
// to one of them (the other paths still apply when it cannot run).
static int rho_kernel_choice() {
  const char* e = std::getenv("XO_RHO_KERNEL");
  if (!e) return 0;
  if (!std::strcmp(e, "gemm")) return 1;
  if (!std::strcmp(e, "transform")) return 2;
  return 0;
}

// Workspace bytes xo_rho_batch requests for this batch (the path it would take; the
// per-pair VALU path reuses one buffer, so its largest pair counts). Host only.
int rho_batch_ws_bytes(const xo_rho_args* p, int n, size_t* bytes) {
  std::vector<Extent> xc(n), xv(n), xe(n);
  for (int i = 0; i < n; ++i) XO_RET(validate_rho(&p[i], &xc[i], &xv[i], &xe[i]));
  if (mfma_eligible(p, n)) {
    const int choice = rho_kernel_choice();
    if (p[0].prec == XO_BF16X3 || p[0].prec == XO_BF16) {
      if (choice != 2 && rho_gemm_ws_bytes(p, n, xc.data(), xv.data(), xe.data(), bytes) == XO_OK) return XO_OK;
      if (choice != 1 && mfma_ws_bytes(p, n, xc.data(), xv.data(), xe.data(), bytes) == XO_OK) return XO_OK;
    } else if (choice != 2 && rho_gemm_ws_bytes(p, n, xc.data(), xv.data(), xe.data(), bytes) == XO_OK) {
      return XO_OK;
    }
  }
  size_t mx = 0;
  for (int i = 0; i < n; ++i) {
    size_t b = 0;
    XO_RET(rho_valu_ws_bytes(&p[i], xc[i], xv[i], xe[i], &b));
    mx = std::max(mx, b);
  }
  *bytes = mx;
  return XO_OK;
}

int rho_batch(const xo_rho_args* p, int n, hipStream_t s) {
  std::vector<Extent> xc(n), xv(n), xe(n);
  for (int i = 0; i < n; ++i) XO_RET(validate_rho(&p[i], &xc[i], &xv[i], &xe[i]));
  if (mfma_eligible(p, n)) {
    const int choice = rho_kernel_choice();
    if (p[0].prec == XO_BF16X3 || p[0].prec == XO_BF16) {
      if (choice != 2) {
        int r = rho_batch_gemm(p, n, xc.data(), xv.data(), xe.data(), s);
        if (r != XO_ERR_UNSUPPORTED) return r;
      }
      if (choice != 1) {
        int r = rho_batch_mfma(p, n, xc.data(), xv.data(), xe.data(), s);
        if (r != XO_ERR_UNSUPPORTED) return r;
      }
    } else if (choice != 2) {
      int r = rho_batch_gemm_fp(p, n, xc.data(), xv.data(), xe.data(), s);
      if (r != XO_ERR_UNSUPPORTED) return r;
    }
  }
  for (int i = 0; i < n; ++i) XO_RET(rho_valu(&p[i], s));
  return XO_OK;
}

}  // namespace xo

extern "C" int xo_rho(const xo_rho_args* a, void* stream) {
  xo::clear_error();
  if (!a) {
    xo::set_error("xo_rho: null argument block");
    return XO_ERR_ARG;
  }
  return xo::rho_batch(a, 1, static_cast<hipStream_t>(stream));
}

extern "C" int xo_rho_workspace_size(const xo_rho_args* pairs, int npairs, size_t* bytes) {
  xo::clear_error();
  if (!pairs || npairs <= 0 || !bytes) {
    xo::set_error("xo_rho_workspace_size: need a non-empty array of pairs and an output");
    return XO_ERR_ARG;
  }
  return xo::rho_batch_ws_bytes(pairs, npairs, bytes);
}

extern "C" int xo_rho_batch(const xo_rho_args* pairs, int npairs, void* stream) {
  xo::clear_error();
  if (!pairs || npairs <= 0) {
    xo::set_error("xo_rho_batch: need a non-empty array of pairs");
    return XO_ERR_ARG;
  }
  return xo::rho_batch(pairs, npairs, static_cast<hipStream_t>(stream));
}
