// Oscillator strengths on MFMA (split bf16, FP32 accumulation), many k-pairs per
// launch. Same factorisation as the VALU path (rho.hip):
//
//   U(x, y, m_z)  orbitals, real space in x and y, Miller index in z
//   S1(x,y,e_z)   = sum_m conj(U_c(x,y,m)) U_v(x,y,m - e_z)      stage 1
//   S2(x,e_y,e_z) = sum_y exp(2 pi i e_y y/Ny) S1(x,y,e_z)       stage 2
//   rho(G)        = 1/(Nx Ny) sum_x exp(2 pi i e_x x/Nx) S2(x,e_y,e_z)
//
// but stages 1 and 2 run as 16x16 complex matrix products on
// v_mfma_f32_16x16x32_bf16 and stage 3 is fused into the same workgroup:
//
//   stage 1, per (c, x, y): Toeplitz(conj U_c)[e_z][m] x U_v[m][v]   (16 v per tile)
//   stage 2, per (c, x, e_z): F[e_y][y] x S1[y][v]                     (y in chunks of 16)
//   stage 3: every workgroup owns rho[v][c][G] for its 16 valence bands and
//            accumulates exp(2 pi i e_x x/Nx) S2 over its x-planes.
//
// Complex operands use interleaved real K (k = 2n + a): for C = conj(A)^T B,
// the left operand of Re C is the raw (re, im) pair of A and that of Im C is
// (-im, re). Every FP32 value x enters as hi = bf16(x) and lo = bf16(x - hi);
// each product is hi*hi + hi*lo + lo*hi, accumulated in FP32.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "bf16x3.h"
#include "rho_geom.h"

namespace xo {

int rho_valu(const xo_rho_args* a, hipStream_t s);

namespace {

constexpr int kBlock = 256;
constexpr int kLP = 32;  // zero padding on each side of an orbital line in LDS

// --------------------------------------------------------------- orbitals --
struct OrbSide {
  const float2* coef;
  const SphereEntry* ent;
  const int* zoff;
  uint32_t* Uhi;
  uint32_t* Ulo;
  int npw, nb, nslot;
  int xlo, nbx, ylo, nby;
};

// U[b][x][y][s] as split bf16 pairs. One workgroup per (band, side): for z-slots
// in chunks of 8, scatter the plane waves into dense (m_y, m_x) boxes in LDS,
// transform along x, then along y, and write each (x, y)'s chunk contiguously.
constexpr int kSC = 8;

template <int NO>
__global__ void __launch_bounds__(kBlock) orb_split(const OrbSide* __restrict__ sides, int Nx, int Ny,
                                                    const float2* __restrict__ twt) {
  extern __shared__ unsigned char smem[];
  const OrbSide S = sides[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= S.nb) return;
  float2* twx = reinterpret_cast<float2*>(smem);  // [Nx] then [Ny]
  float2* twy = twx + Nx;
  float2* box = twy + Ny;                        // [kSC][nby][nbx]
  float2* V = box + kSC * S.nby * S.nbx;         // [kSC][nby][Nx]
  const int nbb = S.nby * S.nbx;
  for (int k = threadIdx.x; k < Nx + Ny; k += blockDim.x) twx[k] = twt[k];
  uint32_t* uh = S.Uhi + (size_t)b * Nx * Ny * NO;
  uint32_t* ul = S.Ulo + (size_t)b * Nx * Ny * NO;
  for (int s0 = 0; s0 < NO; s0 += kSC) {
    if (s0 >= S.nslot) {
      for (int i = threadIdx.x; i < Nx * Ny * kSC; i += blockDim.x) {
        const int xy = i / kSC, j = i - (i / kSC) * kSC;
        uh[(size_t)xy * NO + s0 + j] = 0u;
        ul[(size_t)xy * NO + s0 + j] = 0u;
      }
      continue;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kSC * nbb; e += blockDim.x) box[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const int s1 = min(s0 + kSC, S.nslot);
    for (int p = S.zoff[s0] + threadIdx.x; p < S.zoff[s1]; p += blockDim.x) {
      const SphereEntry e = S.ent[p];
      // slot of plane wave p: the z-slot whose [zoff[s], zoff[s+1]) range holds p
      int j = 0;
      while (S.zoff[s0 + j + 1] <= p) ++j;
      box[j * nbb + e.by * S.nbx + e.bx] = S.coef[(size_t)b * S.npw + e.src];
    }
    __syncthreads();
    for (int it = threadIdx.x; it < kSC * S.nby * Nx; it += blockDim.x) {
      const int x = it % Nx, jb = it / Nx;           // jb = j * nby + by
      int k = pmod(S.xlo * x, Nx);
      const float2* row = box + jb * S.nbx;
      float2 acc = make_float2(0.f, 0.f);
      for (int bx = 0; bx < S.nbx; ++bx) {
        const float2 c = row[bx], w = twx[k];
        acc.x = fmaf(c.x, w.x, fmaf(-c.y, w.y, acc.x));
        acc.y = fmaf(c.x, w.y, fmaf(c.y, w.x, acc.y));
        k += x;
        if (k >= Nx) k -= Nx;
      }
      V[jb * Nx + x] = acc;
    }
    __syncthreads();
    for (int xy = threadIdx.x; xy < Nx * Ny; xy += blockDim.x) {
      const int x = xy / Ny, y = xy - (xy / Ny) * Ny;
      const int k0 = pmod(S.ylo * y, Ny);
      uint32_t hv[kSC], lv[kSC];
#pragma unroll
      for (int j = 0; j < kSC; ++j) {
        int k = k0;
        float2 acc = make_float2(0.f, 0.f);
        if (s0 + j < S.nslot) {
          for (int by = 0; by < S.nby; ++by) {
            const float2 c = V[(j * S.nby + by) * Nx + x], w = twy[k];
            acc.x = fmaf(c.x, w.x, fmaf(-c.y, w.y, acc.x));
            acc.y = fmaf(c.x, w.y, fmaf(c.y, w.x, acc.y));
            k += y;
            if (k >= Ny) k -= Ny;
          }
        }
        split2(acc.x, acc.y, hv[j], lv[j]);
      }
      u4* dh = reinterpret_cast<u4*>(uh + (size_t)xy * NO + s0);
      u4* dl = reinterpret_cast<u4*>(ul + (size_t)xy * NO + s0);
      dh[0] = u4{hv[0], hv[1], hv[2], hv[3]};
      dh[1] = u4{hv[4], hv[5], hv[6], hv[7]};
      dl[0] = u4{lv[0], lv[1], lv[2], lv[3]};
      dl[1] = u4{lv[4], lv[5], lv[6], lv[7]};
    }
  }
}

// ------------------------------------------------------------------- rho --
struct PairDesc {
  const uint32_t* Uc_hi;
  const uint32_t* Uc_lo;
  const uint32_t* Uv_hi;
  const uint32_t* Uv_lo;
  float2* rho;          // [nv][nc][ng]
  const uint32_t* F;    // [4][16 iz][16 slot][Nyp]: (re hi, re lo, im hi, im lo)
  const int* gtab;      // [ng]: iz | srow << 5 | (e_x mod Nx) << 10
  int nc, nv, nvt, d0, nz, wg0;
};

template <int NK, int GPT>
__global__ void __launch_bounds__(kBlock) rho_mfma(const PairDesc* __restrict__ pairs, int npairs, int nwg,
                                                   int Nx, int Ny, int Nyp, int ng,
                                                   const float2* __restrict__ twtab, float scale) {
  constexpr int NO = 16 * NK;
  constexpr int LW = NO + 2 * kLP;
  extern __shared__ uint32_t lds[];
  uint32_t* Ahi = lds;                 // [Ny][LW]
  uint32_t* Alo = Ahi + Ny * LW;       // [Ny][LW]
  uint32_t* S1hi = Alo + Ny * LW;      // [16 iz][4 yq][16 v][4 y]
  uint32_t* S1lo = S1hi + 4096;
  float2* S2p = reinterpret_cast<float2*>(S1hi);  // [16 iz][16 slot][16 v], aliases S1
  float2* twx = reinterpret_cast<float2*>(S1lo + 4096);  // [Nx e][Nx x]
  int* gt = reinterpret_cast<int*>(twx + Nx * Nx);       // [ng]

  // XCD-aware order: hardware dispatches workgroup b to XCD b % 8, so XCD x gets
  // the contiguous logical range [x * per, (x + 1) * per) and works through whole
  // k-pairs, keeping each pair's valence orbitals resident in that XCD's L2.
  const int per = (nwg + 7) >> 3;
  const int L = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (L >= nwg) return;
  int lo = 0, hi = npairs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pairs[mid].wg0 <= L) lo = mid; else hi = mid - 1;
  }
  const PairDesc P = pairs[lo];
  const int local = L - P.wg0;
  const int c = local / P.nvt, vt = local - (local / P.nvt) * P.nvt;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, l16 = l & 15, q = l >> 4;
  const int vq = tid & 3, gq4 = tid >> 2;  // stage 3 ownership

  for (int i = tid; i < 2 * Ny * LW; i += kBlock) Ahi[i] = 0u;
  for (int i = tid; i < Nx * Nx; i += kBlock) twx[i] = twtab[i];
  for (int i = tid; i < ng; i += kBlock) gt[i] = P.gtab[i];

  float2 acc[GPT][4];
#pragma unroll
  for (int i = 0; i < GPT; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = make_float2(0.f, 0.f);
  const int vb = vt * 16 + l16;
  const bool vok = vb < P.nv;
  const size_t VS = (size_t)16 * 16 * Nyp;  // stride between the four F variants

  for (int x = 0; x < Nx; ++x) {
    __syncthreads();  // previous plane finished with A and S2p
    {
      const size_t cb = ((size_t)c * Nx + x) * Ny * NO;
      for (int i = tid; i < Ny * NO; i += kBlock) {
        const int y = i / NO, n = i - (i / NO) * NO;
        Ahi[y * LW + kLP + n] = P.Uc_hi[cb + i];
        Alo[y * LW + kLP + n] = P.Uc_lo[cb + i];
      }
    }
    __syncthreads();
    f4 s2r[4], s2i[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s2r[j] = f4{0.f, 0.f, 0.f, 0.f};
      s2i[j] = f4{0.f, 0.f, 0.f, 0.f};
    }
    for (int ch = 0; ch < Nyp / 16; ++ch) {
      // ---- stage 1: this wave's four y values of the chunk (y = ch*16 + 4*wave + j)
      f4 cr[4], ci[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int y = ch * 16 + wave * 4 + j;
        cr[j] = f4{0.f, 0.f, 0.f, 0.f};
        ci[j] = f4{0.f, 0.f, 0.f, 0.f};
        if (y < Ny) {
#pragma unroll
          for (int kk = 0; kk < NK; ++kk) {
            const int ab = y * LW + kLP + kk * 16 + 4 * q + l16 - P.d0;
            u4 arh, arl, aih, ail;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              arh[m] = Ahi[ab + m];
              arl[m] = Alo[ab + m];
              aih[m] = rot_neg(arh[m]);
              ail[m] = rot_neg(arl[m]);
            }
            u4 bh = u4{0u, 0u, 0u, 0u}, bl = u4{0u, 0u, 0u, 0u};
            if (vok) {
              const size_t o = (((size_t)vb * Nx + x) * Ny + y) * NO + kk * 16 + 4 * q;
              bh = *reinterpret_cast<const u4*>(P.Uv_hi + o);
              bl = *reinterpret_cast<const u4*>(P.Uv_lo + o);
            }
            cr[j] = mma3(arh, arl, bh, bl, cr[j]);
            ci[j] = mma3(aih, ail, bh, bl, ci[j]);
          }
        }
      }
      // S1 layout [iz][yq][v][4 y]: lane (q, v) holds rows iz = 4q + r for its 4 y values
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        uint32_t hh[4], ll[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) split2(cr[j][r], ci[j][r], hh[j], ll[j]);
        const u4 h = u4{hh[0], hh[1], hh[2], hh[3]}, lw = u4{ll[0], ll[1], ll[2], ll[3]};
        const int idx = (((4 * q + r) * 4 + wave) * 16 + l16) * 4;
        *reinterpret_cast<u4*>(S1hi + idx) = h;
        *reinterpret_cast<u4*>(S1lo + idx) = lw;
      }
      __syncthreads();
      // ---- stage 2: this wave's e_z rows
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int iz = wave + 4 * j;
        if (iz < P.nz) {
          const size_t fb = ((size_t)iz * 16 + l16) * Nyp + ch * 16 + 4 * q;
          const u4 frh = *reinterpret_cast<const u4*>(P.F + fb);
          const u4 frl = *reinterpret_cast<const u4*>(P.F + VS + fb);
          const u4 fih = *reinterpret_cast<const u4*>(P.F + 2 * VS + fb);
          const u4 fil = *reinterpret_cast<const u4*>(P.F + 3 * VS + fb);
          const int so = ((iz * 4 + q) * 16 + l16) * 4;
          const u4 sh = *reinterpret_cast<const u4*>(S1hi + so);
          const u4 sl = *reinterpret_cast<const u4*>(S1lo + so);
          s2r[j] = mma3(frh, frl, sh, sl, s2r[j]);
          s2i[j] = mma3(fih, fil, sh, sl, s2i[j]);
        }
      }
      __syncthreads();
    }
    // ---- S2 plane to LDS (reuses the S1 space)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int iz = wave + 4 * j;
      if (iz < P.nz) {
#pragma unroll
        for (int r = 0; r < 4; ++r) S2p[(iz * 16 + 4 * q + r) * 16 + l16] = make_float2(s2r[j][r], s2i[j][r]);
      }
    }
    __syncthreads();
    // ---- stage 3: x transform into the owned rho entries (G = gq4 + 64 i, v = 4 vq .. 4 vq + 3)
#pragma unroll
    for (int i = 0; i < GPT; ++i) {
      const int G = gq4 + 64 * i;
      if (G < ng) {
        const int t = gt[G];
        const float4* sp = reinterpret_cast<const float4*>(S2p + ((t & 31) * 16 + ((t >> 5) & 31)) * 16 + 4 * vq);
        const float4 s01 = sp[0], s23 = sp[1];
        const float2 w = twx[(t >> 10) * Nx + x];
        acc[i][0].x = fmaf(s01.x, w.x, fmaf(-s01.y, w.y, acc[i][0].x));
        acc[i][0].y = fmaf(s01.x, w.y, fmaf(s01.y, w.x, acc[i][0].y));
        acc[i][1].x = fmaf(s01.z, w.x, fmaf(-s01.w, w.y, acc[i][1].x));
        acc[i][1].y = fmaf(s01.z, w.y, fmaf(s01.w, w.x, acc[i][1].y));
        acc[i][2].x = fmaf(s23.x, w.x, fmaf(-s23.y, w.y, acc[i][2].x));
        acc[i][2].y = fmaf(s23.x, w.y, fmaf(s23.y, w.x, acc[i][2].y));
        acc[i][3].x = fmaf(s23.z, w.x, fmaf(-s23.w, w.y, acc[i][3].x));
        acc[i][3].y = fmaf(s23.z, w.y, fmaf(s23.w, w.x, acc[i][3].y));
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int v = vt * 16 + 4 * vq + u;
    if (v < P.nv) {
      float2* out = P.rho + ((size_t)v * P.nc + c) * ng;
#pragma unroll
      for (int i = 0; i < GPT; ++i) {
        const int G = gq4 + 64 * i;
        if (G < ng) out[G] = make_float2(acc[i][u].x * scale, acc[i][u].y * scale);
      }
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
static uint16_t host_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t r = 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)((u + r) >> 16);
}
static float host_from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
static void host_split(float x, uint16_t& hi, uint16_t& lo) {
  hi = host_bf16(x);
  lo = host_bf16(x - host_from_bf16(hi));
}

struct Geo {
  int nz = 0, ezmin = 0;
  std::vector<uint32_t> F;
  std::vector<int> gtab;
  bool ok = true;
};

// Slot structure of the shifted G-set e = m_G - G0 and the stage-2 DFT operands.
static Geo make_geo(const xo_rho_args* a, int Nx, int Ny, int Nyp) {
  Geo g;
  int ezmin = 1 << 30, ezmax = -(1 << 30);
  for (int i = 0; i < a->ng; ++i) {
    const int ez = a->mill_g[3 * i + 2] - a->g0[2];
    ezmin = std::min(ezmin, ez);
    ezmax = std::max(ezmax, ez);
  }
  g.ezmin = ezmin;
  g.nz = ezmax - ezmin + 1;
  if (g.nz > 16) {
    g.ok = false;
    return g;
  }
  std::vector<std::vector<int>> slots(g.nz);  // e_y mod Ny per slot
  g.gtab.resize(a->ng);
  for (int i = 0; i < a->ng; ++i) {
    const int ex = pmod(a->mill_g[3 * i] - a->g0[0], Nx);
    const int ey = pmod(a->mill_g[3 * i + 1] - a->g0[1], Ny);
    const int iz = a->mill_g[3 * i + 2] - a->g0[2] - ezmin;
    auto& sl = slots[iz];
    int r = (int)(std::find(sl.begin(), sl.end(), ey) - sl.begin());
    if (r == (int)sl.size()) sl.push_back(ey);
    if (r >= 16) {
      g.ok = false;
      return g;
    }
    g.gtab[i] = iz | (r << 5) | (ex << 10);
  }
  const size_t VS = (size_t)16 * 16 * Nyp;
  g.F.assign(4 * VS, 0u);
  for (int iz = 0; iz < g.nz; ++iz)
    for (int r = 0; r < (int)slots[iz].size(); ++r)
      for (int y = 0; y < Ny; ++y) {
        const double th = 2.0 * M_PI * (double)((slots[iz][r] * y) % Ny) / Ny;
        const float fr = (float)std::cos(th), fi = (float)std::sin(th);
        uint16_t h0, l0, h1, l1;
        const size_t o = ((size_t)iz * 16 + r) * Nyp + y;
        host_split(fr, h0, l0);
        host_split(-fi, h1, l1);
        g.F[o] = h0 | ((uint32_t)h1 << 16);
        g.F[VS + o] = l0 | ((uint32_t)l1 << 16);
        host_split(fi, h0, l0);
        host_split(fr, h1, l1);
        g.F[2 * VS + o] = h0 | ((uint32_t)h1 << 16);
        g.F[3 * VS + o] = l0 | ((uint32_t)l1 << 16);
      }
  return g;
}

// Device geometry per (grid, G-set, G0), built once per process and device.
struct DevGeo {
  const void* F = nullptr;
  const void* gtab = nullptr;
  int nz = 0;
};

static int dev_geo(const xo_rho_args* a, int Nx, int Ny, int Nyp, hipStream_t s, const DevGeo** out) {
  static std::mutex mu;
  static std::map<std::vector<int>, DevGeo> cache;
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  std::vector<int> key = {dev, Nx, Ny, a->g0[0], a->g0[1], a->g0[2]};
  key.insert(key.end(), a->mill_g, a->mill_g + 3 * a->ng);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second.nz ? &it->second : nullptr;
    return XO_OK;
  }
  Geo g = make_geo(a, Nx, Ny, Nyp);
  DevGeo d;
  if (g.ok) {
    XO_RET(device_table(g.F.data(), g.F.size() * sizeof(uint32_t), s, &d.F));
    XO_RET(device_table(g.gtab.data(), g.gtab.size() * sizeof(int), s, &d.gtab));
    d.nz = g.nz;
  }
  auto& slot = cache[key];
  slot = d;
  *out = d.nz ? &slot : nullptr;
  return XO_OK;
}

template <int NK, int GPT>
static int launch_rho(const void* dpairs, int npairs, int nwg, int Nx, int Ny, int Nyp, int ng, const void* dtw,
                      hipStream_t s, size_t lds) {
  if (lds > 64 * 1024)
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rho_mfma<NK, GPT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  {
    KernelTimer kt_("rho_mfma", s);
    hipLaunchKernelGGL((rho_mfma<NK, GPT>), dim3(8 * ((nwg + 7) / 8)), dim3(kBlock), lds, s,
                       static_cast<const PairDesc*>(dpairs), npairs, nwg, Nx, Ny, Nyp, ng,
                       static_cast<const float2*>(dtw), (float)(1.0 / ((double)Nx * Ny)));
  }
  XO_CHECK_LAUNCH();
  return XO_OK;
}

template <int NK>
static int launch_rho_g(const void* dpairs, int npairs, int nwg, int Nx, int Ny, int Nyp, int ng, const void* dtw,
                        hipStream_t s, size_t lds) {
  if (ng <= 64 * 2) return launch_rho<NK, 2>(dpairs, npairs, nwg, Nx, Ny, Nyp, ng, dtw, s, lds);
  if (ng <= 64 * 4) return launch_rho<NK, 4>(dpairs, npairs, nwg, Nx, Ny, Nyp, ng, dtw, s, lds);
  if (ng <= 64 * 8) return launch_rho<NK, 8>(dpairs, npairs, nwg, Nx, Ny, Nyp, ng, dtw, s, lds);
  return launch_rho<NK, 16>(dpairs, npairs, nwg, Nx, Ny, Nyp, ng, dtw, s, lds);
}

// Whether a batch can take the MFMA path (else each pair runs the VALU path in FP32).
static bool mfma_eligible(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe) {
  const xo_rho_args& a0 = p[0];
  if (a0.ng > 1024 || a0.n[0] > 72 || a0.n[1] > 128) return false;
  for (int i = 0; i < n; ++i) {
    if (p[i].q0 || p[i].prec != XO_BF16X3) return false;
    if (p[i].n[0] != a0.n[0] || p[i].n[1] != a0.n[1] || p[i].ng != a0.ng) return false;
    if (std::memcmp(p[i].mill_g, a0.mill_g, sizeof(int32_t) * 3 * a0.ng) != 0) return false;
    const int no = std::max(xc[i].hi[2] - xc[i].lo[2] + 1, xv[i].hi[2] - xv[i].lo[2] + 1);
    if (no > 32) return false;
    const int d0 = xc[i].lo[2] - xv[i].lo[2] - xe[i].lo[2];
    if (d0 <= -18 || d0 > kLP) return false;
  }
  return true;
}

static int rho_batch_mfma(const xo_rho_args* p, int n, const Extent* xc, const Extent* xv, const Extent* xe,
                          hipStream_t s) {
  const int Nx = p[0].n[0], Ny = p[0].n[1], ng = p[0].ng;
  const int Nyp = (Ny + 15) / 16 * 16;
  int NO = 16;
  for (int i = 0; i < n; ++i)
    NO = std::max(NO, std::max(xc[i].hi[2] - xc[i].lo[2] + 1, xv[i].hi[2] - xv[i].lo[2] + 1) > 16 ? 32 : 16);

  // per-G0 geometry (stage-2 operands and G selectors), cached by content
  std::map<std::tuple<int, int, int>, std::pair<const void*, const void*>> geos;
  std::map<std::tuple<int, int, int>, int> nzs;
  for (int i = 0; i < n; ++i) {
    auto key = std::make_tuple(p[i].g0[0], p[i].g0[1], p[i].g0[2]);
    if (geos.count(key)) continue;
    const DevGeo* dg = nullptr;
    XO_RET(dev_geo(&p[i], Nx, Ny, Nyp, s, &dg));
    if (!dg) return XO_ERR_UNSUPPORTED;
    geos[key] = {dg->F, dg->gtab};
    nzs[key] = dg->nz;
  }
  std::vector<float2> tw((size_t)Nx * Nx);
  for (int e = 0; e < Nx; ++e)
    for (int x = 0; x < Nx; ++x) {
      const double th = 2.0 * M_PI * (double)((e * x) % Nx) / Nx;
      tw[(size_t)e * Nx + x] = make_float2((float)std::cos(th), (float)std::sin(th));
    }
  const void* dtw = nullptr;
  XO_RET(device_table(tw.data(), tw.size() * sizeof(float2), s, &dtw));
  std::vector<float2> twxy(Nx + Ny);
  for (int k = 0; k < Nx + Ny; ++k) {
    const int nn = k < Nx ? Nx : Ny, kk = k < Nx ? k : k - Nx;
    const double th = 2.0 * M_PI * kk / nn;
    twxy[k] = make_float2((float)std::cos(th), (float)std::sin(th));
  }
  const void* dtwxy = nullptr;
  XO_RET(device_table(twxy.data(), twxy.size() * sizeof(float2), s, &dtwxy));

  // workspace: split orbitals of every pair
  const size_t plane = (size_t)Nx * Ny * NO;
  std::vector<size_t> off(n + 1, 0);
  for (int i = 0; i < n; ++i) off[i + 1] = off[i] + align_up(plane * (p[i].nc + p[i].nv) * 4, 256);
  void* ws = nullptr;
  XO_RET(workspace(s, 3, 2 * off[n], &ws));
  uint32_t* Uhi0 = static_cast<uint32_t*>(ws);
  uint32_t* Ulo0 = Uhi0 + off[n] / 4;

  std::vector<SphereTable> tabs(2 * n);
  std::vector<OrbSide> sides(2 * n);
  int maxnb = 0;
  size_t orb_lds = 0;
  for (int i = 0; i < n; ++i) {
    for (int side = 0; side < 2; ++side) {
      const Extent& ex = side ? xv[i] : xc[i];
      SphereTable& t = tabs[2 * i + side];
      t = sphere_table(side ? p[i].mill_v : p[i].mill_c, side ? p[i].npw_v : p[i].npw_c, ex);
      const void* dent = nullptr;
      const void* dzoff = nullptr;
      XO_RET(device_table(t.ent.data(), t.ent.size() * sizeof(SphereEntry), s, &dent));
      XO_RET(device_table(t.zoff.data(), t.zoff.size() * sizeof(int), s, &dzoff));
      OrbSide& o = sides[2 * i + side];
      o.coef = static_cast<const float2*>(side ? p[i].coef_v : p[i].coef_c);
      o.ent = static_cast<const SphereEntry*>(dent);
      o.zoff = static_cast<const int*>(dzoff);
      const size_t ubase = off[i] / 4 + (side ? plane * p[i].nc : 0);
      o.Uhi = Uhi0 + ubase;
      o.Ulo = Ulo0 + ubase;
      o.npw = side ? p[i].npw_v : p[i].npw_c;
      o.nb = side ? p[i].nv : p[i].nc;
      o.nslot = t.nslot;
      o.xlo = ex.lo[0];
      o.nbx = ex.hi[0] - ex.lo[0] + 1;
      o.ylo = ex.lo[1];
      o.nby = ex.hi[1] - ex.lo[1] + 1;
      maxnb = std::max(maxnb, o.nb);
      orb_lds = std::max(orb_lds, (size_t)(Nx + Ny + kSC * (o.nby * o.nbx + o.nby * Nx)) * sizeof(float2));
    }
  }
  const void* dsides = nullptr;
  XO_RET(device_table(sides.data(), sides.size() * sizeof(OrbSide), s, &dsides));
  if (orb_lds > 160 * 1024) return XO_ERR_UNSUPPORTED;
  {
    auto kfn = NO == 16 ? reinterpret_cast<const void*>(&orb_split<16>) : reinterpret_cast<const void*>(&orb_split<32>);
    if (orb_lds > 64 * 1024)
      XO_TRY_HIP(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)orb_lds));
    KernelTimer kt_("orb_split", s);
    if (NO == 16)
      hipLaunchKernelGGL(orb_split<16>, dim3(maxnb, 2 * n), dim3(kBlock), orb_lds, s,
                         static_cast<const OrbSide*>(dsides), Nx, Ny, static_cast<const float2*>(dtwxy));
    else
      hipLaunchKernelGGL(orb_split<32>, dim3(maxnb, 2 * n), dim3(kBlock), orb_lds, s,
                         static_cast<const OrbSide*>(dsides), Nx, Ny, static_cast<const float2*>(dtwxy));
  }
  XO_CHECK_LAUNCH();

  std::vector<PairDesc> pd(n);
  int nwg = 0;
  for (int i = 0; i < n; ++i) {
    auto key = std::make_tuple(p[i].g0[0], p[i].g0[1], p[i].g0[2]);
    PairDesc& d = pd[i];
    d.Uc_hi = sides[2 * i].Uhi;
    d.Uc_lo = sides[2 * i].Ulo;
    d.Uv_hi = sides[2 * i + 1].Uhi;
    d.Uv_lo = sides[2 * i + 1].Ulo;
    d.rho = static_cast<float2*>(p[i].rho);
    d.F = static_cast<const uint32_t*>(geos[key].first);
    d.gtab = static_cast<const int*>(geos[key].second);
    d.nc = p[i].nc;
    d.nv = p[i].nv;
    d.nvt = (p[i].nv + 15) / 16;
    d.d0 = xc[i].lo[2] - xv[i].lo[2] - xe[i].lo[2];
    d.nz = nzs[key];
    d.wg0 = nwg;
    nwg += d.nc * d.nvt;
  }
  const void* dpairs = nullptr;
  XO_RET(device_table(pd.data(), pd.size() * sizeof(PairDesc), s, &dpairs));
  const int LW = NO + 2 * kLP;
  const size_t lds = (size_t)(2 * Ny * LW + 8192) * 4 + (size_t)Nx * Nx * sizeof(float2) + (size_t)ng * 4;
  if (lds > 160 * 1024) return XO_ERR_UNSUPPORTED;
  if (NO == 16)
    XO_RET(launch_rho_g<1>(dpairs, n, nwg, Nx, Ny, Nyp, ng, dtw, s, lds));
  else
    XO_RET(launch_rho_g<2>(dpairs, n, nwg, Nx, Ny, Nyp, ng, dtw, s, lds));

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

}  // namespace

int rho_batch(const xo_rho_args* p, int n, hipStream_t s) {
  std::vector<Extent> xc(n), xv(n), xe(n);
  for (int i = 0; i < n; ++i) XO_RET(validate_rho(&p[i], &xc[i], &xv[i], &xe[i]));
  if (mfma_eligible(p, n, xc.data(), xv.data(), xe.data())) {
    int r = rho_batch_mfma(p, n, xc.data(), xv.data(), xe.data(), s);
    if (r != XO_ERR_UNSUPPORTED) return r;
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

extern "C" int xo_rho_batch(const xo_rho_args* pairs, int npairs, void* stream) {
  xo::clear_error();
  if (!pairs || npairs <= 0) {
    xo::set_error("xo_rho_batch: need a non-empty array of pairs");
    return XO_ERR_ARG;
  }
  return xo::rho_batch(pairs, npairs, static_cast<hipStream_t>(stream));
}
