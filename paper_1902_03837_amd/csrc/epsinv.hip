// Inverse dielectric matrix in FP64 (Eq. X_rpa_inv; symmetrised as in Eq. W_def).
//
//   eps~ = I - diag(s) chi0 diag(s),   s_G = sqrt(4 pi) / |q+G|
//
// eps~ is Hermitian positive definite at imaginary frequencies. It is inverted
// in place by blocked Gauss-Jordan elimination, all frequencies in the same
// launches; the diagonal blocks are inverted without pivoting (positive definite
// input) or, with XO_EPS_LU_FALLBACK (general eps~), with partial pivoting inside
// the block. Per block column K (width b = 64):
//   P = A_KK^-1                      diag_mfma: one workgroup per frequency, the block
//                                    in registers, one barrier per pivot pair, the pair's
//                                    update on FP64 matrix cores (diag_inverse: the same
//                                    on VALU, and the pivoted form with one barrier per pivot)
//   A_Kj = P A_Kj  (j outside K)     panel_mfma: row strips of the panel, and
//   S_iK = A_iK,  A_iK = -A_iK P     column strips (old column saved in S), on FP64
//                                    matrix cores (row_col: the same on VALU)
//   A_ij -= S_iK A_Kj  (i, j outside K)  rank_update_mfma, 32 x 32 tiles on FP64 matrix cores
//                                        (rank_update: the same on VALU, XO_EPS_RANK=valu)
// The pivots met inside the diagonal blocks are the diagonal of eps~ = L D L^H,
// so a pivot with non-positive real part proves eps~ is not positive definite.
// In the pivoted form a numerically singular diagonal block is reported instead.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "xo_common.h"

namespace xo {
namespace {

constexpr int kB = 64;  // block width

typedef cplx<double> z;

// s_G = sqrt(4 pi) / |q+G| (Coulomb interaction subsection)
__device__ __forceinline__ double coulomb_s(const double* qpg, int i) { return 3.5449077018110318 / qpg[i]; }

__global__ void build_eps(const double* __restrict__ chi0, const double* __restrict__ qpg, int n,
                          double* __restrict__ A) {
  const size_t w = blockIdx.y;
  const size_t nn = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / n), j = (int)(e - (e / n) * n);
  const double f = coulomb_s(qpg, i) * coulomb_s(qpg, j);
  const double* c = chi0 + (w * nn + e) * 2;
  double* o = A + (w * nn + e) * 2;
  o[0] = (i == j ? 1.0 : 0.0) - f * c[0];
  o[1] = -f * c[1];
}

// Largest squared modulus of each frequency's eps~ (before the elimination), as the bits
// of a non-negative double (ordered like the values) in gmax2[w]; gmax2 starts at 0.
__global__ void zero_flags(int* __restrict__ flag, unsigned long long* __restrict__ gmax2, int nw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    flag[i] = 0;
    gmax2[i] = 0ull;
  }
}

__global__ void eps_absmax(const double* __restrict__ A, int n, unsigned long long* __restrict__ gmax2) {
  __shared__ double red[256];
  const size_t w = blockIdx.y;
  const size_t nn = (size_t)n * n;
  const z* a = reinterpret_cast<const z*>(A) + w * nn;
  double m = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x)
    m = fmax(m, a[e].x * a[e].x + a[e].y * a[e].y);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(gmax2 + w, __double_as_longlong(red[0]));
}

// In-place Gauss-Jordan inverse of the kb x kb diagonal block K of every matrix
// (kb <= 64). 4096 / E threads per frequency: thread t holds row t / (64 / E),
// columns E (t % (64 / E)) .. + E - 1 in registers (identity outside kb). Per
// pivot k (per pivot pair in diag_block_pairs) the owners publish column k and the
// pivot row (values before the step) in LDS, double buffered, and every thread updates its own E entries. The pivot row
// is stored transposed ([j][column group]) so that a wave reads it without bank
// conflicts.
//
// This form (general eps~, real frequencies) pivots partially inside the block.
// The pivot of column k is the row of largest modulus among the rows not yet used;
// rows stay in place (the sweep is applied to row p_k and column k), so the result
// R holds R[p_k][j] = B^-1[k][p_j] (B the block) and is written back with that
// permutation undone. A pivot below 1e-13 of the largest entry of the block or of the
// whole eps~ (gmax2: squared, per frequency) marks the block as numerically singular
// (flagged): the blocked elimination has no pivoting across blocks, so the caller gets
// an error instead of an inaccurate inverse.
// The body runs on the kB * kB / E threads of a workgroup for the matrix A of frequency w.
template <int E>
__device__ __forceinline__ void diag_block_lu(z* __restrict__ A, int n, int K, int kb, int w,
                                              int* __restrict__ flag, const unsigned long long* __restrict__ gmax2) {
  constexpr int CG = kB / E;  // column groups
  __shared__ z pcol[2][kB];
  __shared__ z prow[2][E][CG];
  __shared__ int perm[kB], inv[kB];   // pivot row of column k, and its inverse
  __shared__ double wmax[kB * kB / E / 64];
  const int o = K * kB;
  const int t = threadIdx.x, r = t / CG, cq = t % CG, c0 = E * cq, lane = t & 63;
  z a[E];
  double amax = 0.0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int c = c0 + j;
    a[j] = (r < kb && c < kb) ? A[(size_t)(o + r) * n + o + c] : z{r == c ? 1.0 : 0.0, 0.0};
    if (r < kb && c < kb) amax = fmax(amax, a[j].x * a[j].x + a[j].y * a[j].y);
  }
  // squared singularity threshold
  for (int m = 32; m >= 1; m >>= 1) amax = fmax(amax, __shfl_xor(amax, m, 64));
  if (lane == 0) wmax[t >> 6] = amax;
  __syncthreads();
  amax = 0.0;
#pragma unroll
  for (int i = 0; i < kB * kB / E / 64; ++i) amax = fmax(amax, wmax[i]);
  const double thr2 = 1e-26 * fmax(amax, __longlong_as_double(gmax2[w]));
  uint64_t used = 0;  // rows already pivoted (the same in every wave)
  for (int kq = 0; kq < CG; ++kq) {
#pragma unroll
    for (int kk = 0; kk < E; ++kk) {
      const int k = E * kq + kk;
      if (k >= kb) break;
      const int b = k & 1;
      if (cq == kq) pcol[b][r] = a[kk];
      __syncthreads();
      // every wave finds the pivot row: lane l looks at row l (rows past kb and used
      // rows excluded), then a butterfly maximum; ties go to the lower row
      const z v = pcol[b][lane];
      double m2 = (lane < kb && !((used >> lane) & 1)) ? v.x * v.x + v.y * v.y : -1.0;
      int idx = lane;
      for (int m = 32; m >= 1; m >>= 1) {
        const double om = __shfl_xor(m2, m, 64);
        const int oi = __shfl_xor(idx, m, 64);
        if (om > m2 || (om == m2 && oi < idx)) {
          m2 = om;
          idx = oi;
        }
      }
      const int p = __builtin_amdgcn_readfirstlane(idx);
      used |= (uint64_t)1 << p;
      if (t == 0) {
        perm[k] = p;
        inv[p] = k;
        if (!(m2 > thr2)) atomicCAS(flag + w, 0, o + k + 1);  // first singular pivot of this frequency
      }
      if (r == p) {
#pragma unroll
        for (int j = 0; j < E; ++j) prow[b][j][cq] = a[j];
      }
      __syncthreads();
      const z piv = pcol[b][p];
      const double den = piv.x * piv.x + piv.y * piv.y;
      const double rd = den > 0.0 ? 1.0 / den : 0.0;
      const z ip = z{piv.x * rd, -piv.y * rd};
      // one instruction stream for every row: the pivot row is 0 - (-1/p) A_pj,
      // the others A_rj - (A_rk / p) A_pj; column k is set afterwards
      const bool prow_p = r == p;
      const z gr = cmul(pcol[b][r], ip);
      const z g = prow_p ? z{-ip.x, -ip.y} : gr;
      const double keep = prow_p ? 0.0 : 1.0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const z pr = prow[b][j][cq];
        a[j].x = fma(-g.x, pr.x, fma(g.y, pr.y, keep * a[j].x));
        a[j].y = fma(-g.x, pr.y, fma(-g.y, pr.x, keep * a[j].y));
      }
      if (cq == kq) a[kk] = prow_p ? ip : z{-gr.x, -gr.y};
    }
  }
  __syncthreads();  // perm and inv complete
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int c = c0 + j;
    if (r < kb && c < kb) A[(size_t)(o + inv[r]) * n + o + perm[c]] = a[j];
  }
}

// Hermitian positive definite form (imaginary frequencies): the pivots are the diagonal,
// two per barrier. Per pair
// (k, k + 1) the owners publish both pivot columns and both pivot rows (values before the
// pair) and every thread applies the 2 x 2 block step, with P the pivot block and Q = P^-1:
//   pivot rows   A[P][j] <- Q A[P][j],                    A[P][P] <- Q
//   other rows   A[r][j] <- A[r][j] - (A[r][P] Q) A[P][j], A[r][P] <- -A[r][P] Q
// In exact arithmetic this is the two scalar Gauss-Jordan steps of the pair. Their pivots are
// p00 and the Schur complement det(P) / p00, the next two diagonal entries of eps~ = L D L^H,
// so a non-positive real part of either proves eps~ is not positive definite (flagged: the
// first bad pivot of the frequency, 1-based). An odd kb (< 64) pairs its last column with the identity padding, which the
// step leaves as it is. Half as many barriers and LDS round trips as the scalar sweep.
template <int E>
__device__ __forceinline__ void diag_block_pairs(z* __restrict__ A, int n, int K, int kb, int w,
                                                 int* __restrict__ flag) {
  constexpr int CG = kB / E;  // column groups
  static_assert(E % 2 == 0, "a pivot pair stays in one column group");
  __shared__ z pcol[2][2][kB];     // [buffer][pivot column k, k + 1][row]
  __shared__ z prow[2][2][E][CG];  // [buffer][pivot row k, k + 1][j][column group]
  const int o = K * kB;
  const int t = threadIdx.x, r = t / CG, cq = t % CG, c0 = E * cq;
  z a[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int c = c0 + j;
    a[j] = (r < kb && c < kb) ? A[(size_t)(o + r) * n + o + c] : z{r == c ? 1.0 : 0.0, 0.0};
  }
  for (int kq = 0; kq < CG; ++kq) {
#pragma unroll
    for (int kk = 0; kk < E; kk += 2) {
      const int k = E * kq + kk;
      if (k >= kb) break;
      const int b = (k >> 1) & 1;
      if (cq == kq) {
        pcol[b][0][r] = a[kk];
        pcol[b][1][r] = a[kk + 1];
      }
      if (r == k || r == k + 1) {
#pragma unroll
        for (int j = 0; j < E; ++j) prow[b][r - k][j][cq] = a[j];
      }
      __syncthreads();
      const z p00 = pcol[b][0][k], p01 = pcol[b][1][k], p10 = pcol[b][0][k + 1], p11 = pcol[b][1][k + 1];
      const z pp = cmul(p00, p11), qq = cmul(p01, p10);
      const z det = z{pp.x - qq.x, pp.y - qq.y};
      if (t == 0) {
        // Re(det / p00) has the sign of Re(det conj(p00)) once p00 has a positive real part
        if (!(p00.x > 0.0))
          atomicCAS(flag + w, 0, o + k + 1);  // first bad pivot of this frequency
        else if (!(det.x * p00.x + det.y * p00.y > 0.0))
          atomicCAS(flag + w, 0, o + k + 2);
      }
      const double den = det.x * det.x + det.y * det.y;
      const double rd = den > 0.0 ? 1.0 / den : 0.0;
      const z id = z{det.x * rd, -det.y * rd};
      const z q00 = cmul(p11, id), q11 = cmul(p00, id);
      const z m01 = cmul(p01, id), m10 = cmul(p10, id);
      const z q01 = z{-m01.x, -m01.y}, q10 = z{-m10.x, -m10.y};
      // one instruction stream for every row: a pivot row is 0 - (-Q[row]) A[P][j], any
      // other row A[r][j] - (A[r][P] Q) A[P][j]; the pivot columns are set afterwards
      const bool pv0 = r == k, pv1 = r == k + 1;
      const z c0v = pcol[b][0][r], c1v = pcol[b][1][r];
      z g0 = cmul(c0v, q00), g1 = cmul(c0v, q01);
      cfma(g0, c1v, q10);
      cfma(g1, c1v, q11);
      if (pv0) {
        g0 = z{-q00.x, -q00.y};
        g1 = z{-q01.x, -q01.y};
      }
      if (pv1) {
        g0 = z{-q10.x, -q10.y};
        g1 = z{-q11.x, -q11.y};
      }
      const double keep = (pv0 || pv1) ? 0.0 : 1.0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const z r0 = prow[b][0][j][cq], r1 = prow[b][1][j][cq];
        z v = z{keep * a[j].x, keep * a[j].y};
        v.x = fma(-g0.x, r0.x, fma(g0.y, r0.y, v.x));
        v.y = fma(-g0.x, r0.y, fma(-g0.y, r0.x, v.y));
        v.x = fma(-g1.x, r1.x, fma(g1.y, r1.y, v.x));
        v.y = fma(-g1.x, r1.y, fma(-g1.y, r1.x, v.y));
        a[j] = v;
      }
      if (cq == kq) {
        a[kk] = pv0 ? q00 : (pv1 ? q10 : z{-g0.x, -g0.y});
        a[kk + 1] = pv0 ? q01 : (pv1 ? q11 : z{-g1.x, -g1.y});
      }
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int c = c0 + j;
    if (r < kb && c < kb) A[(size_t)(o + r) * n + o + c] = a[j];
  }
}

template <int E, bool PIV>
__global__ void __launch_bounds__(kB * kB / E) diag_inverse(double* __restrict__ Aall, int n, int K, int kb,
                                                            int* __restrict__ flag,
                                                            const unsigned long long* __restrict__ gmax2) {
  const int w = blockIdx.x;
  if constexpr (PIV)
    diag_block_lu<E>(reinterpret_cast<z*>(Aall) + (size_t)w * n * n, n, K, kb, w, flag, gmax2);
  else
    diag_block_pairs<E>(reinterpret_cast<z*>(Aall) + (size_t)w * n * n, n, K, kb, w, flag);
}
constexpr int kDiagE = 8;  // entries per thread of diag_inverse (512 threads: two waves per SIMD)

// Tile product acc = L R over m < kb (L: 16 RU rows x kb, leading dimension LL; R: kb x 16 RV
// columns, leading dimension LR; both in LDS). Thread t owns rows t / 16 + 16 u and columns
// t % 16 + 16 v: a wave reads four rows of L (broadcast) and 16 consecutive entries of R.
template <int RU, int RV, int LL, int LR>
__device__ __forceinline__ void tile_product(const z* __restrict__ L, const z* __restrict__ R, int kb,
                                             z (&acc)[RU][RV]) {
  const int t = threadIdx.x, rr0 = t >> 4, cc0 = t & 15;
#pragma unroll
  for (int u = 0; u < RU; ++u)
#pragma unroll
    for (int v = 0; v < RV; ++v) acc[u][v] = z{0.0, 0.0};
  for (int m = 0; m < kb; ++m) {
    z l[RU], rr[RV];
#pragma unroll
    for (int u = 0; u < RU; ++u) l[u] = L[(rr0 + 16 * u) * LL + m];
#pragma unroll
    for (int v = 0; v < RV; ++v) rr[v] = R[m * LR + cc0 + 16 * v];
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int v = 0; v < RV; ++v) cfma(acc[u][v], l[u], rr[v]);
  }
}

// Panel of block column K, each 64-wide tile in two halves (twice the workgroups of whole
// tiles: the panel is small and latency-bound). blockIdx.x = 2 * tile + half.
// Row tiles (tile < nt): A_Kj <- P A_Kj for the 32 columns of half h of tile j != K.
// Column tiles (tile >= nt): S_iK <- A_iK, A_iK <- -A_iK P for the 32 rows of half h of
// tile i != K (a row's 64 pivot columns stay in one workgroup: it reads them all before
// writing any). S: [nw][n][kB].
constexpr int kH = kB / 2;
__global__ void __launch_bounds__(256) row_col(double* __restrict__ Aall, int n, int K, int kb, int nt,
                                              double* __restrict__ Sall) {
  extern __shared__ unsigned char smem[];
  z* P = reinterpret_cast<z*>(smem);   // [kB][kB + 1]: the inverted diagonal block
  z* T = P + kB * (kB + 1);            // row tile: [kB][kH + 1]; column tile: [kH][kB + 1]
  const int w = blockIdx.y;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  z* S = reinterpret_cast<z*>(Sall) + (size_t)w * n * kB;
  const int tb = (int)blockIdx.x >> 1, h = (int)blockIdx.x & 1;
  const bool rowt = tb < nt;
  const int tile = rowt ? tb : tb - nt;
  if (tile == K) return;
  const int o = K * kB, x0 = tile * kB + h * kH;
  {
    // every load of both operands in flight before the LDS stores
    z vp[16], vt[8];
#pragma unroll
    for (int f = 0; f < 16; ++f) {
      const int e = threadIdx.x + 256 * f, i = e >> 6, j = e & 63;
      vp[f] = (i < kb && j < kb) ? A[(size_t)(o + i) * n + o + j] : z{0.0, 0.0};
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = threadIdx.x + 256 * f;
      if (rowt) {  // T[m][c] = A[o + m][x0 + c], 64 x 32
        const int i = e >> 5, j = e & 31;
        vt[f] = (i < kb && x0 + j < n) ? A[(size_t)(o + i) * n + x0 + j] : z{0.0, 0.0};
      } else {     // T[r][m] = A[x0 + r][o + m], 32 x 64
        const int i = e >> 6, j = e & 63;
        vt[f] = (x0 + i < n && j < kb) ? A[(size_t)(x0 + i) * n + o + j] : z{0.0, 0.0};
      }
    }
#pragma unroll
    for (int f = 0; f < 16; ++f) {
      const int e = threadIdx.x + 256 * f;
      P[(e >> 6) * (kB + 1) + (e & 63)] = vp[f];
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = threadIdx.x + 256 * f;
      if (rowt)
        T[(e >> 5) * (kH + 1) + (e & 31)] = vt[f];
      else
        T[(e >> 6) * (kB + 1) + (e & 63)] = vt[f];
    }
  }
  __syncthreads();
  const int t = threadIdx.x, rr0 = t >> 4, cc0 = t & 15;
  if (rowt) {
    z acc[4][2];
    tile_product<4, 2, kB + 1, kH + 1>(P, T, kb, acc);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int r = rr0 + 16 * u, c = x0 + cc0 + 16 * v;
        if (r < kb && c < n) A[(size_t)(o + r) * n + c] = acc[u][v];
      }
  } else {
    z acc[2][4];
    tile_product<2, 4, kB + 1, kB + 1>(T, P, kb, acc);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rr0 + 16 * u, m = cc0 + 16 * v;
        if (x0 + r < n && m < kb) {
          const size_t i = x0 + r;
          S[i * kB + m] = T[r * (kB + 1) + m];
          A[i * n + o + m] = z{-acc[u][v].x, -acc[u][v].y};
        }
      }
  }
}

// Rank-kb update of one 32 x 32 tile outside row block K and column block K:
//   A_ij -= S_iK A_Kj   (S old column, A_Kj new row).
// Thread t owns rows t / 16 + 16 u and columns t % 16 + 16 v (u, v < 2). Ends with a barrier,
// so a workgroup may update several tiles in a row.
constexpr int kT = 32;
__device__ __forceinline__ void update_tile(z* __restrict__ A, const z* __restrict__ S, int n, int o, int kb, int i0,
                                            int j0) {
  __shared__ z L[kT][kB + 1];
  __shared__ z R[kB][kT + 1];
  {
    z vl[8], vr[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = threadIdx.x + 256 * f;
      const int li = e >> 6, lj = e & 63;   // L: 32 rows x 64
      const int ri = e >> 5, rj = e & 31;   // R: 64 rows x 32
      vl[f] = (i0 + li < n && lj < kb) ? S[(size_t)(i0 + li) * kB + lj] : z{0.0, 0.0};
      vr[f] = (ri < kb && j0 + rj < n) ? A[(size_t)(o + ri) * n + j0 + rj] : z{0.0, 0.0};
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = threadIdx.x + 256 * f;
      L[e >> 6][e & 63] = vl[f];
      R[e >> 5][e & 31] = vr[f];
    }
  }
  __syncthreads();
  const int t = threadIdx.x, rr0 = t >> 4, cc0 = t & 15;
  z acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = z{0.0, 0.0};
  for (int m = 0; m < kb; ++m) {
    const z l0 = L[rr0][m], l1 = L[rr0 + 16][m], r0 = R[m][cc0], r1 = R[m][cc0 + 16];
    cfma(acc[0][0], l0, r0);
    cfma(acc[0][1], l0, r1);
    cfma(acc[1][0], l1, r0);
    cfma(acc[1][1], l1, r1);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = i0 + rr0 + 16 * u, j = j0 + cc0 + 16 * v;
      if (i < n && j < n) {
        z& x = A[(size_t)i * n + j];
        x = z{x.x - acc[u][v].x, x.y - acc[u][v].y};
      }
    }
  __syncthreads();
}

// The rank update of block step K: one workgroup per 32 x 32 tile (blockIdx.x = tile row,
// blockIdx.y = tile column) outside row block K and column block K.
__global__ void __launch_bounds__(256) rank_update(double* __restrict__ Aall, int n, int K, int kb,
                                                  const double* __restrict__ Sall) {
  const int w = blockIdx.z;
  const int o = K * kB;
  const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
  if ((i0 >= o && i0 < o + kB) || (j0 >= o && j0 < o + kB)) return;  // 32-tiles sit inside 64-blocks
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const z* S = reinterpret_cast<const z*>(Sall) + (size_t)w * n * kB;
  update_tile(A, S, n, o, kb, i0, j0);
}

// The rank update on FP64 matrix cores (v_mfma_f64_16x16x4f64): one workgroup per 32 x 32 tile
// outside row and column block K; wave (wr, wc) owns its 16 x 16 block (wr, wc) with a real
// and an imaginary accumulator. The complex product is taken in real arithmetic, two m per
// instruction: lane (i, k) (i = lane % 16, k = lane / 16) supplies A[i][k] = Re or Im (k even
// or odd) of S[row i][m + k / 2], and B[k][j] = (Re B, -Im B) for the real accumulator and
// (Im B, Re B) for the imaginary one, B = A_Kj[m + k / 2][column j]; the instruction leaves
// D[lane / 16 + 4 r][lane % 16] in register r (the FP64 form's own order, unlike the FP32
// 16 x 16 forms). The kb pivot rows are staged through LDS in two halves of 32 (34 KB, 72
// registers: four workgroups per CU), the next half's loads issued before the current half's
// products; entries past kb and past n are staged as zero. (64 x 64 tiles with four blocks per
// wave, two workgroups per CU, measured slower at every size.)
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kMT = 32;   // tile edge
constexpr int kUK = 32;   // pivot rows per LDS stage
__global__ void __launch_bounds__(256) rank_update_mfma(double* __restrict__ Aall, int n, int K, int kb, int nw,
                                                       const double* __restrict__ Sall) {
  constexpr int FL = kMT * kUK / 256;  // staged entries per thread, each operand
  // XCD-aware order: workgroup b runs on XCD b % 8, which takes a contiguous range of the
  // (tile row, tile column, frequency) space, tile row fastest: the tiles in flight on an
  // XCD share their pivot rows and neighbouring S rows in its L2
  const int nt = (n + kMT - 1) / kMT, ntiles = nt * nt * nw;
  const int per = (ntiles + 7) >> 3;
  const int L0 = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (L0 >= ntiles) return;
  const int ti = L0 % nt, tj = (L0 / nt) % nt, w = L0 / (nt * nt);
  if (ti * kMT / kB == K || tj * kMT / kB == K) return;  // 32-tiles sit inside 64-blocks
  __shared__ z L[kMT][kUK + 1];   // S rows of the tile, this stage's pivot columns
  __shared__ z R[kUK][kMT + 1];   // this stage's pivot rows, the tile's columns
  const int o = K * kB, i0 = ti * kMT, j0 = tj * kMT;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  const z* S = reinterpret_cast<const z*>(Sall) + (size_t)w * n * kB;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, r0 = 16 * (wave >> 1), c0 = 16 * (wave & 1);
  const int li = lane & 15, lk = lane >> 4, half = lk >> 1, part = lk & 1;
  d4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  // stage loads: the next stage's are issued before the current stage's products
  z vl[FL], vr[FL];
  auto load_stage = [&](int m0) {
#pragma unroll
    for (int f = 0; f < FL; ++f) {
      const int e = t + 256 * f, er = e / kUK, ec = e % kUK;  // L: 32 rows x 32; R: 32 rows x 32
      vl[f] = (i0 + er < n && m0 + ec < kb) ? S[(size_t)(i0 + er) * kB + m0 + ec] : z{0.0, 0.0};
      vr[f] = (m0 + er < kb && j0 + ec < n) ? A[(size_t)(o + m0 + er) * n + j0 + ec] : z{0.0, 0.0};
    }
  };
  load_stage(0);
  for (int m0 = 0; m0 < kb; m0 += kUK) {
    if (m0 > 0) __syncthreads();  // the previous stage's reads are done
#pragma unroll
    for (int f = 0; f < FL; ++f) {
      const int e = t + 256 * f;
      L[e / kUK][e % kUK] = vl[f];
      R[e / kUK][e % kUK] = vr[f];
    }
    __syncthreads();
    if (m0 + kUK < kb) load_stage(m0 + kUK);
    const int mk = min(kUK, kb - m0);
    for (int m = 0; m < mk; m += 2) {
      const z l = L[r0 + li][m + half], r = R[m + half][c0 + li];
      const double av = part ? l.y : l.x, br = part ? -r.y : r.x, bi = part ? r.x : r.y;
      re = __builtin_amdgcn_mfma_f64_16x16x4f64(av, br, re, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bi, im, 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + r0 + lk + 4 * q, j = j0 + c0 + li;
    if (i < n && j < n) {
      z& x = A[(size_t)i * n + j];
      x = z{x.x - re[q], x.y - im[q]};
    }
  }
}

// Panel of block column K on FP64 matrix cores, in strips of 16 (rows or columns) so that the
// small, latency-bound launch has many workgroups. blockIdx.x = strip (row strips first).
// Row strip s (columns x0 = 16 s .. + 15, outside block K): A_Kj <- P A_Kj over all kb rows of
//   the panel, wave v computing rows 16 v .. + 15 (a strip's rows are read whole before any
//   is written, and no other workgroup touches its columns).
// Column strip s (rows x0 .. x0 + 15 outside block K): S_iK <- A_iK, A_iK <- -A_iK P over all kb
//   pivot columns, wave v computing columns 16 v .. + 15.
// Both are C = X Y with X (row strip: P, 64 rows; column strip: the strip's A_iK, 16 rows) and
// Y (A_Kj, 16 columns; -P, 64 columns), taken as in rank_update_mfma: two m per instruction,
// halves of 32 m staged through LDS (42.5 KB: three workgroups per CU).
constexpr int kPS16 = 16;  // strip width
__global__ void __launch_bounds__(256) panel_mfma(double* __restrict__ Aall, int n, int K, int kb, int ns,
                                                 double* __restrict__ Sall) {
  const int w = blockIdx.y;
  const bool rowt = (int)blockIdx.x < ns;
  const int sidx = rowt ? (int)blockIdx.x : (int)blockIdx.x - ns;
  const int x0 = sidx * kPS16;
  if (x0 / kB == K) return;  // strips sit inside 64-blocks
  __shared__ z buf[64 * (kUK + 1) + kUK * (kPS16 + 1)];
  // row strip: Xs [64][33] (P), Ys [32][17] (A_Kj); column strip: Xs [16][33] (A_iK), Ys [32][65] (P)
  const int XL = kUK + 1, YL = rowt ? kPS16 + 1 : kB + 1;
  z* Xs = buf;
  z* Ys = buf + (rowt ? 64 : kPS16) * XL;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  z* S = reinterpret_cast<z*>(Sall) + (size_t)w * n * kB;
  const int o = K * kB;
  const int t = threadIdx.x, lane = t & 63, v = t >> 6;
  const int li = lane & 15, lk = lane >> 4, half = lk >> 1, part = lk & 1;
  const int ax = rowt ? 16 * v : 0, by = rowt ? 0 : 16 * v;  // this wave's X rows and Y columns
  const double sg = rowt ? 1.0 : -1.0;
  d4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  // per stage and thread: 8 entries of the 64-wide operand (P), 2 of the 16-wide one
  z vp[8], vq[2];
  auto load_stage = [&](int m0) {
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = t + 256 * f;
      if (rowt) {  // P[r][m0 + c], 64 x 32
        const int r = e >> 5, c = e & 31;
        vp[f] = (r < kb && m0 + c < kb) ? A[(size_t)(o + r) * n + o + m0 + c] : z{0.0, 0.0};
      } else {     // P[m0 + r][c], 32 x 64
        const int r = e >> 6, c = e & 63;
        vp[f] = (m0 + r < kb && c < kb) ? A[(size_t)(o + m0 + r) * n + o + c] : z{0.0, 0.0};
      }
    }
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int e = t + 256 * f;
      if (rowt) {  // A_Kj[m0 + r][x0 + c], 32 x 16
        const int r = e >> 4, c = e & 15;
        vq[f] = (m0 + r < kb && x0 + c < n) ? A[(size_t)(o + m0 + r) * n + x0 + c] : z{0.0, 0.0};
      } else {     // A_iK[x0 + r][m0 + c], 16 x 32
        const int r = e >> 5, c = e & 31;
        vq[f] = (x0 + r < n && m0 + c < kb) ? A[(size_t)(x0 + r) * n + o + m0 + c] : z{0.0, 0.0};
      }
    }
  };
  load_stage(0);
  for (int m0 = 0; m0 < kb; m0 += kUK) {
    if (m0 > 0) __syncthreads();  // the previous stage's reads are done
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int e = t + 256 * f;
      if (rowt)
        Xs[(e >> 5) * XL + (e & 31)] = vp[f];
      else
        Ys[(e >> 6) * YL + (e & 63)] = vp[f];
    }
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int e = t + 256 * f;
      if (rowt) {
        Ys[(e >> 4) * YL + (e & 15)] = vq[f];
      } else {
        const int r = e >> 5, c = e & 31;
        Xs[r * XL + c] = vq[f];
        if (x0 + r < n && m0 + c < kb) S[(size_t)(x0 + r) * kB + m0 + c] = vq[f];  // the old column
      }
    }
    __syncthreads();
    if (m0 + kUK < kb) load_stage(m0 + kUK);
    const int mk = min(kUK, kb - m0);
    for (int m = 0; m < mk; m += 2) {
      const z l = Xs[(ax + li) * XL + m + half], r = Ys[(m + half) * YL + by + li];
      const double av = part ? l.y : l.x;
      const double br = sg * (part ? -r.y : r.x), bi = sg * (part ? r.x : r.y);
      re = __builtin_amdgcn_mfma_f64_16x16x4f64(av, br, re, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bi, im, 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ax + lk + 4 * q, c = by + li;  // row and column of C
    if (rowt) {
      if (r < kb && x0 + c < n) A[(size_t)(o + r) * n + x0 + c] = z{re[q], im[q]};
    } else {
      if (x0 + r < n && c < kb) A[(size_t)(x0 + r) * n + o + c] = z{re[q], im[q]};
    }
  }
}

// Hermitian positive definite diagonal block on FP64 matrix cores: the two-pivot sweep of
// diag_block_pairs with the rank-2 update of the whole 64 x 64 block as matrix-core products.
// Wave v holds block row v (rows 16 v .. + 15) in the instruction's output layout: one 16 x 16
// block per block column c, real and imaginary accumulators; lane (i, g), register q holds row
// 16 v + g + 4 q, column 16 c + i. Every entry takes one update per pivot pair P = (k, k + 1):
//   A <- A - G R,   G = A[:, P] Q outside the pivot rows, G = I - Q in them,
//   R = A[P, :] + E  (E: ones at A[P_p][P_p]),
// which leaves Q A[P, :] in the pivot rows, -A[r, P] Q in the pivot columns and Q at A[P, P]:
// the pair's Gauss-Jordan step as one uniform product. G enters as the left operand (lane
// (i, k): Re or Im of G[16 v + i][k / 2]), R as the right one ((Re, -Im) for the real
// accumulator, (Im, Re) for the imaginary one), G negated. Per pair the owners publish the
// pivot columns and rows (values before the pair) in LDS, double buffered, one barrier; the
// pivots p00 and det P / p00 are flagged as in diag_block_pairs. Loops unrolled so that the
// block column and register of every pivot are compile-time.
__global__ void __launch_bounds__(256) diag_mfma(double* __restrict__ Aall, int n, int K, int kb,
                                                int* __restrict__ flag) {
  const int w = blockIdx.x;
  z* A = reinterpret_cast<z*>(Aall) + (size_t)w * n * n;
  __shared__ z pc[2][2][kB];  // [buffer][pivot column k, k + 1][row]
  __shared__ z pr[2][2][kB];  // [buffer][pivot row k, k + 1][column]
  const int o = K * kB;
  const int t = threadIdx.x, lane = t & 63, v = t >> 6;
  const int li = lane & 15, lg = lane >> 4;
  d4 re[4], im[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * v + lg + 4 * q, col = 16 * c + li;
      const z a = (row < kb && col < kb) ? A[(size_t)(o + row) * n + o + col] : z{row == col ? 1.0 : 0.0, 0.0};
      re[c][q] = a.x;
      im[c][q] = a.y;
    }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 16 * c + 2 * j;
      if (k >= kb) break;
      const int b = j & 1;
      // pivot columns k, k + 1: block column c, lane columns 2 j and 2 j + 1
      if ((li >> 1) == j) {
#pragma unroll
        for (int q = 0; q < 4; ++q) pc[b][li & 1][16 * v + lg + 4 * q] = z{re[c][q], im[c][q]};
      }
      // pivot rows k, k + 1: wave c, lane groups 2 (j & 1) and 2 (j & 1) + 1, register j / 2
      if (v == c && (lg >> 1) == (j & 1)) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) pr[b][lg & 1][16 * cc + li] = z{re[cc][j >> 1], im[cc][j >> 1]};
      }
      __syncthreads();
      const z p00 = pc[b][0][k], p01 = pc[b][1][k], p10 = pc[b][0][k + 1], p11 = pc[b][1][k + 1];
      const z pp = cmul(p00, p11), qq = cmul(p01, p10);
      const z det = z{pp.x - qq.x, pp.y - qq.y};
      if (t == 0) {
        if (!(p00.x > 0.0))
          atomicCAS(flag + w, 0, o + k + 1);  // first bad pivot of this frequency
        else if (!(det.x * p00.x + det.y * p00.y > 0.0))
          atomicCAS(flag + w, 0, o + k + 2);
      }
      const double den = det.x * det.x + det.y * det.y;
      const double rd = den > 0.0 ? 1.0 / den : 0.0;
      const z id = z{det.x * rd, -det.y * rd};
      const z q00 = cmul(p11, id), q11 = cmul(p00, id);
      const z m01 = cmul(p01, id), m10 = cmul(p10, id);
      const z q01 = z{-m01.x, -m01.y}, q10 = z{-m10.x, -m10.y};
      // left operand: G of row 16 v + i, component k / 2, Re or Im
      const int row = 16 * v + li;
      const z c0v = pc[b][0][row], c1v = pc[b][1][row];
      z g0 = cmul(c0v, q00), g1 = cmul(c0v, q01);
      cfma(g0, c1v, q10);
      cfma(g1, c1v, q11);
      if (row == k) {
        g0 = z{1.0 - q00.x, -q00.y};
        g1 = z{-q01.x, -q01.y};
      }
      if (row == k + 1) {
        g0 = z{-q10.x, -q10.y};
        g1 = z{1.0 - q11.x, -q11.y};
      }
      const z gs = (lg >> 1) ? g1 : g0;
      const double av = (lg & 1) ? -gs.y : -gs.x;
      const int p = lg >> 1;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int col = 16 * cc + li;
        z r = pr[b][p][col];
        if (col == k + p) r.x += 1.0;
        const double br = (lg & 1) ? -r.y : r.x, bi = (lg & 1) ? r.x : r.y;
        re[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, br, re[cc], 0, 0, 0);
        im[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bi, im[cc], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * v + lg + 4 * q, col = 16 * c + li;
      if (row < kb && col < kb) A[(size_t)(o + row) * n + o + col] = z{re[c][q], im[c][q]};
    }
}

__global__ void unsymmetrise(double* __restrict__ A, const double* __restrict__ qpg, int n) {
  const size_t w = blockIdx.y;
  const size_t nn = (size_t)n * n;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / n), j = (int)(e - (e / n) * n);
  const double f = coulomb_s(qpg, i) / coulomb_s(qpg, j);
  double* o = A + (w * nn + e) * 2;
  o[0] *= f;
  o[1] *= f;
}

}  // namespace
}  // namespace xo

namespace xo {
namespace {
// Diagonal-block (positive definite form), panel and rank-update kernels: FP64 matrix cores
// (default) or, with the environment variable XO_EPS_RANK=valu, the VALU forms (kept as a
// second implementation; the tests run both).
int rank_form() {
  const char* e = std::getenv("XO_EPS_RANK");
  return (e && !std::strcmp(e, "valu")) ? 2 : 1;
}

// Workspace of one call: the pivot flags and, with more than one block, the saved column panel.
size_t eps_head_bytes(int nw) { return align_up(sizeof(int) * nw, 256) + align_up(sizeof(double) * nw, 256); }
size_t eps_ws_bytes(int n, int nw) {
  const int nblk = (n + kB - 1) / kB;
  return eps_head_bytes(nw) + (nblk > 1 ? (size_t)nw * n * kB * sizeof(z) : 0);
}
}  // namespace
}  // namespace xo

extern "C" int xo_epsinv_workspace_size(const xo_eps_args* a, size_t* bytes) {
  using namespace xo;
  clear_error();
  XO_ARG(a && bytes, "xo_epsinv_workspace_size: null argument");
  XO_ARG(a->ng > 0 && a->nw > 0, "xo_epsinv_workspace_size: sizes must be positive (ng=%d nw=%d)", a->ng, a->nw);
  *bytes = eps_ws_bytes(a->ng, a->nw);
  return XO_OK;
}

namespace xo {
namespace {

// Static scratch of the no-allocation entry point (xo_epsinv_noalloc): the pivot flags,
// the per-frequency scales, |q+G| and the saved column panel. Each device holds its own
// copy for the life of the process; host code uses only the device address obtained from
// hipGetSymbolAddress, kept per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

int scratch_address(void** out) {
  int dev = 0;
  XO_TRY_HIP(hipGetDevice(&dev));
  XO_ARG(dev >= 0 && dev < kMaxDevices, "xo_epsinv_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("xo_epsinv_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return XO_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return XO_OK;
}

size_t noalloc_bytes(int n, int nw) { return eps_ws_bytes(n, nw) + align_up(sizeof(double) * n, 256); }
constexpr int kNoallocHostFlags = 1024;  // frequencies whose flags the no-allocation call reads back

// noalloc = false: workspace and |q+G| table from the library caches (may allocate);
// noalloc = true: everything in the static scratch, no allocation of any kind.
int epsinv_run(const xo_eps_args* a, hipStream_t st, bool noalloc) {
  const char* who = noalloc ? "xo_epsinv_noalloc" : "xo_epsinv";
  XO_ARG(a, "%s: null argument block", who);
  XO_ARG(a->ng > 0 && a->nw > 0, "%s: sizes must be positive (ng=%d nw=%d)", who, a->ng, a->nw);
  XO_ARG(a->qpg && a->chi0 && a->out, "%s: null pointer", who);
  XO_ARG((a->flags & ~(XO_EPS_NONSYM | XO_EPS_LU_FALLBACK)) == 0, "%s: unknown flags 0x%x", who, a->flags);
  XO_ARG(a->chi0 != a->out, "%s: chi0 and out must not alias", who);
  if (a->ng > 16384 || (size_t)a->ng * a->ng * a->nw > ((size_t)1 << 31)) {
    set_error("%s: ng=%d x nw=%d is beyond the supported size", who, a->ng, a->nw);
    return XO_ERR_UNSUPPORTED;
  }
  const int n = a->ng;
  for (int i = 0; i < n; ++i)
    XO_ARG(a->qpg[i] > 0.0 && std::isfinite(a->qpg[i]), "%s: |q+G| at %d must be positive", who, i);
  if (noalloc) {
    if (noalloc_bytes(n, a->nw) > kScratchBytes) {
      set_error("%s: ng=%d x nw=%d needs %zu bytes of scratch, more than its %zu", who, a->ng, a->nw,
                noalloc_bytes(n, a->nw), kScratchBytes);
      return XO_ERR_UNSUPPORTED;
    }
    if (!a->info && a->nw > kNoallocHostFlags) {
      set_error("%s: more than %d frequencies need a device info array", who, kNoallocHostFlags);
      return XO_ERR_UNSUPPORTED;
    }
  }
  const int nblk = (n + kB - 1) / kB;
  const size_t fbytes = align_up(sizeof(int) * a->nw, 256);
  char* ws = nullptr;
  const double* dq = nullptr;
  if (noalloc) {
    void* base = nullptr;
    XO_RET(scratch_address(&base));
    ws = static_cast<char*>(base);
    double* q = reinterpret_cast<double*>(ws + eps_ws_bytes(n, a->nw));
    XO_TRY_HIP(hipMemcpyAsync(q, a->qpg, sizeof(double) * n, hipMemcpyHostToDevice, st));
    dq = q;
  } else {
    const void* t = nullptr;
    XO_RET(device_table(a->qpg, sizeof(double) * n, st, &t));
    dq = static_cast<const double*>(t);
    void* w = nullptr;
    XO_RET(workspace(st, 2, eps_ws_bytes(n, a->nw), &w));
    ws = static_cast<char*>(w);
  }
  // pivot flags: the caller's info array (deferred check) or the call's own
  int* flag = a->info ? a->info : reinterpret_cast<int*>(ws);
  unsigned long long* gmax2 = reinterpret_cast<unsigned long long*>(ws + fbytes);
  double* S = reinterpret_cast<double*>(ws + eps_head_bytes(a->nw));
  hipLaunchKernelGGL(zero_flags, dim3((a->nw + 255) / 256), dim3(256), 0, st, flag, gmax2, a->nw);
  XO_CHECK_LAUNCH();
  const size_t nn = (size_t)n * n;
  {
    KernelTimer kt_("eps_build", st);
    hipLaunchKernelGGL(build_eps, dim3((unsigned)((nn + 255) / 256), a->nw), dim3(256), 0, st, a->chi0, dq, n,
                       a->out);
  }
  XO_CHECK_LAUNCH();
  const int check_sign = (a->flags & XO_EPS_LU_FALLBACK) ? 0 : 1;
  if (!check_sign) {
    {
      KernelTimer kt_("eps_absmax", st);
      hipLaunchKernelGGL(eps_absmax, dim3((unsigned)std::min<size_t>(256, (nn + 4095) / 4096), a->nw), dim3(256),
                         0, st, a->out, n, gmax2);
    }
    XO_CHECK_LAUNCH();
  }
  const size_t lds2 = ((size_t)kB * (kB + 1) + (size_t)kB * (kH + 1) + kH) * sizeof(z);
  static bool attr = false;
  if (!attr) {
    XO_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&row_col),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
    attr = true;
  }
  for (int K = 0; K < nblk; ++K) {
    const int kb = std::min(kB, n - K * kB);
    {
      KernelTimer kt_("eps_diag_inverse", st);
      if (check_sign && rank_form() != 2)
        hipLaunchKernelGGL(diag_mfma, dim3(a->nw), dim3(256), 0, st, a->out, n, K, kb, flag);
      else if (check_sign)
        hipLaunchKernelGGL((diag_inverse<kDiagE, false>), dim3(a->nw), dim3(kB * kB / kDiagE), 0, st, a->out, n,
                           K, kb, flag, gmax2);
      else
        hipLaunchKernelGGL((diag_inverse<kDiagE, true>), dim3(a->nw), dim3(kB * kB / kDiagE), 0, st, a->out, n,
                           K, kb, flag, gmax2);
    }
    XO_CHECK_LAUNCH();
    if (nblk > 1) {
      {
        KernelTimer kt_("eps_row_col", st);
        const int ns = (n + kPS16 - 1) / kPS16;
        if (rank_form() == 2)
          hipLaunchKernelGGL(row_col, dim3(4 * nblk, a->nw), dim3(256), lds2, st, a->out, n, K, kb, nblk, S);
        else
          hipLaunchKernelGGL(panel_mfma, dim3(2 * ns, a->nw), dim3(256), 0, st, a->out, n, K, kb, ns, S);
      }
      XO_CHECK_LAUNCH();
      {
        KernelTimer kt_("eps_rank_update", st);
        const unsigned nt32 = (n + 31) / 32;
        if (rank_form() == 2)
          hipLaunchKernelGGL(rank_update, dim3(nt32, nt32, a->nw), dim3(256), 0, st, a->out, n, K, kb,
                             static_cast<const double*>(S));
        else
          hipLaunchKernelGGL(rank_update_mfma, dim3(8 * ((nt32 * nt32 * a->nw + 7) / 8)), dim3(256), 0, st, a->out,
                             n, K, kb, a->nw, static_cast<const double*>(S));
      }
      XO_CHECK_LAUNCH();
    }
  }
  if (a->flags & XO_EPS_NONSYM) {
    {
      KernelTimer kt_("eps_unsymmetrise", st);
      hipLaunchKernelGGL(unsymmetrise, dim3((unsigned)((nn + 255) / 256), a->nw), dim3(256), 0, st, a->out, dq, n);
    }
    XO_CHECK_LAUNCH();
  }
  if (a->info) return XO_OK;  // the caller reads the flags when it needs them
  int local[kNoallocHostFlags];
  int* hf = local;
  if (!noalloc) XO_RET(host_flags(st, sizeof(int) * a->nw, reinterpret_cast<void**>(&hf)));
  XO_TRY_HIP(hipMemcpyAsync(hf, flag, sizeof(int) * a->nw, hipMemcpyDeviceToHost, st));
  XO_TRY_HIP(hipStreamSynchronize(st));
  for (int w = 0; w < a->nw; ++w) {
    if (hf[w]) {
      if (check_sign) {
        set_error("%s: eps~ is not positive definite at frequency %d (pivot %d)", who, w, hf[w] - 1);
        return XO_ERR_NOTPD;
      }
      set_error("%s: a diagonal block of the elimination is numerically singular at frequency %d (pivot %d)",
                who, w, hf[w] - 1);
      return XO_ERR_SINGULAR;
    }
  }
  return XO_OK;
}

}  // namespace
}  // namespace xo

extern "C" int xo_epsinv(const xo_eps_args* a, void* stream) {
  xo::clear_error();
  return xo::epsinv_run(a, static_cast<hipStream_t>(stream), false);
}

extern "C" int xo_epsinv_noalloc(const xo_eps_args* a, void* stream) {
  xo::clear_error();
  return xo::epsinv_run(a, static_cast<hipStream_t>(stream), true);
}
