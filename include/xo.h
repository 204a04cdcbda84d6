/*
 * xo -- independent-particle response chi0 and inverse dielectric matrix on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Yambo 2019 (arXiv:1902.03837), Linear Response section.
 *   rho_{cv k}(q,G) = < c k | exp(i(q+G).r) | v k-q >                 Eq. (rhotw)
 *   chi0_GG'(q, i w) = -pref sum_t [2 D_t/(w^2 + D_t^2)] rho_t(G) rho_t*(G')
 *                                                   Eq. (X_IP), App. A split
 *   eps~ = I - s chi0 s,  s_G = sqrt(4 pi)/|q+G|     Eq. (X_rpa_inv), Eq. (W_def)
 *
 * Conventions shared by every call
 * --------------------------------
 * - Array arguments marked [device] are device pointers allocated and owned by
 *   the caller. The library never frees them and keeps no reference to them
 *   after the call returns. Arguments marked [host] are host memory, read
 *   during the call only.
 * - Every compute call is asynchronous on the given stream (hipStream_t passed
 *   as void*; NULL means the default stream) unless its comment says it
 *   synchronises.
 * - Complex numbers are interleaved (re, im). Precision XO_FP64 uses complex128
 *   (two doubles); XO_FP32, XO_BF16X3 and XO_BF16 use complex64 (two floats) for
 *   rho and orbital coefficients. chi0 and eps^-1 are always complex128.
 * - Miller triples are int32 [n][3]; the reciprocal vector is m . (b1,b2,b3).
 *   The FFT index of m on an N1 x N2 x N3 grid is m mod N.
 * - Return values: XO_OK or an error code; xo_last_error() then holds a
 *   thread-local message. No call aborts or exits. Arguments are validated on
 *   the host before anything is launched; on an argument error nothing is
 *   enqueued.
 * - Library workspace is device memory cached per (device, stream) and grown
 *   on demand; xo_release_workspace() frees it (synchronising the device).
 *   Calls on distinct streams may run concurrently from distinct threads.
 */
#ifndef XO_H
#define XO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  XO_OK = 0,
  XO_ERR_ARG = 1,          /* invalid argument (message says which)            */
  XO_ERR_ALLOC = 2,        /* device allocation failed                         */
  XO_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed       */
  XO_ERR_NOTPD = 4,        /* eps~ not positive definite at some frequency     */
  XO_ERR_UNSUPPORTED = 5,  /* size or option outside what the kernels handle   */
  XO_ERR_SINGULAR = 6      /* xo_epsinv, general eps~: a diagonal block of the
                              elimination is numerically singular            */
};

/* Arithmetic of rho and chi0 (eps^-1 is FP64 in every form):
 *   XO_FP64   FP64 throughout (complex128 rho and orbitals);
 *   XO_FP32   FP32 MFMA / VALU (complex64);
 *   XO_BF16X3 complex64 data, each MFMA operand split into bf16 hi + lo and
 *             three products hi*hi + hi*lo + lo*hi, FP32 accumulation;
 *   XO_BF16   complex64 data, each MFMA operand rounded to bf16 (at most 2^-8 relative)
 *             and one product, FP32 accumulation. A throughput form, not one of
 *             the split-precision forms: it has no correction term, and its eps^-1
 *             error is not held to the 1e-4 of the split forms (relative
 *             Frobenius against FP64: about 4e-4 with a few hundred transitions,
 *             2e-5 with 2e5 on the imaginary axis, 9e-4 at real frequencies near
 *             poles). Its rho and chi0 obey element-wise rounding bounds; callers
 *             check eps^-1 against an FP64 run of their workload. */
enum { XO_FP64 = 0, XO_FP32 = 1, XO_BF16X3 = 2, XO_BF16 = 3 };

/* Thread-local message describing the last error of this thread ("" if none). */
const char* xo_last_error(void);
/* Library version string. */
const char* xo_version(void);
/* Free all cached workspace and geometry tables on every device (synchronises). */
int xo_release_workspace(void);

/* Kernel timing for benchmarks: with timing on, every kernel the library launches
 * is bracketed by HIP events recorded on its launch stream. xo_timing_report
 * synchronises those events, writes one line "name launches total_ms" per kernel
 * into buf (NUL-terminated, truncated to len bytes) and clears the counters. */
int xo_timing_enable(int on);
int xo_timing_report(char* buf, int len);

/* ------------------------------------------------------------------------- */
/* Oscillator strengths, Eq. (rhotw): the Fourier transform of the real-space
 * product conj(psi_c,k(r)) psi_v,k-q(r), evaluated for one k-pair and all
 * (v, c) of the given band sets.
 *
 * The conduction (empty) states c are at k; the valence (occupied) states v at
 * k - q = k' + G0 are stored at k' with Miller lists relative to k'. Output
 *   rho[v][c][g] = rho_{c v k}(q, G_g),  transition index t = v*nc + c,
 *   dE[v][c]     = e_c - e_v  (the pole energy of Eq. X_IP, Ha).
 * For q0 != 0 (q = 0 exactly, k' = k, G0 = 0) the G = 0 column holds the q -> 0
 * limit divided by |q| along qhat from velocity matrix elements (Eq. dip, the
 * G-space v approach for a local Hamiltonian):
 *   rho^_cv = qhat . sum_G conj(c_c(G)) (k+G) c_v(G) / (e_c - e_v),
 * and requires |e_c - e_v| >= 1e-8 Ha for every pair (checked on the device
 * data only by the caller; the library does not read device energies).
 *
 * Layout: coef_c [nc][npw_c], coef_v [nv][npw_v] complex (precision per prec);
 * rho [nv][nc][ng] complex of the same precision.
 * Errors (XO_ERR_ARG): sizes <= 0; a Miller list that wraps onto itself on the
 * grid; a grid too small for an alias-free product (per axis the reach
 * max|m_c - m_v - (m_G - G0)| must stay below N); q0 set with G = 0 missing
 * from the G-set. XO_ERR_UNSUPPORTED: grid axis > 128, or a plane-wave sphere
 * wider than 32 Miller steps along z.
 */
typedef struct {
  int n[3];                 /* FFT grid                                        */
  double bvec[9];           /* [host] rows b1,b2,b3 in 1/bohr (q0 velocities)  */
  int prec;                 /* XO_FP64 / XO_FP32 / XO_BF16X3 / XO_BF16 (see xo_rho_batch) */
  /* bra: conduction bands at k */
  int npw_c;
  const int32_t* mill_c;    /* [host] [npw_c][3]                               */
  int nc;
  const void* coef_c;       /* [device] [nc][npw_c] complex                    */
  const double* e_c;        /* [device] [nc] band energies, Ha                 */
  double kcart[3];          /* k in 1/bohr (q0 velocities only)                */
  /* ket: valence bands at k' (k - q = k' + G0) */
  int npw_v;
  const int32_t* mill_v;    /* [host] [npw_v][3]                               */
  int nv;
  const void* coef_v;       /* [device] [nv][npw_v] complex                    */
  const double* e_v;        /* [device] [nv]                                   */
  int g0[3];                /* umklapp G0 (Miller)                             */
  /* chi0 G-set */
  int ng;
  const int32_t* mill_g;    /* [host] [ng][3]                                  */
  int q0;                   /* nonzero: q = 0 head from velocities             */
  double qhat[3];           /* Cartesian direction of q -> 0                   */
  /* outputs */
  void* rho;                /* [device] [nv][nc][ng] complex                   */
  double* dE;               /* [device] [nv][nc] or NULL                       */
} xo_rho_args;

int xo_rho(const xo_rho_args* a, void* stream);

/* Several k-pairs in one call, with the same semantics as calling xo_rho on each
 * pair in order (each pair's output slice is written exactly as xo_rho writes
 * it). pairs: [host] array of npairs argument blocks. Pairs of one precision
 * that share the grid's x axis and the G-set run in one MFMA launch of the
 * direct plane-wave sum rho_cv(G) = sum_a conj(c_c(a)) c_v(a - G + G0) as a
 * gathered matrix product (equal to the transform on the alias-free grids that
 * validation requires), when every pair's gather box and the valence bands of a
 * workgroup fit in LDS: FP64 and FP32 on the 16x16x4 MFMAs of their precision,
 * XO_BF16X3 as split bf16 (hi + lo, three products, FP32 accumulation), XO_BF16
 * as plain bf16 (one product, FP32 accumulation).
 * Otherwise XO_BF16X3 and XO_BF16 batches take the axis-factorised split-bf16
 * transform on MFMA (orbitals real-space along x, y-z correlation of Miller
 * spectra, x-DFT in FP32) and FP64 / FP32 pairs the VALU transform, pair by pair. The environment
 * variable XO_RHO_KERNEL=gemm or =transform, read on each call, restricts the
 * choice to one of the two. q0 pairs take the same kernels; their G = 0 column
 * is then written from the velocity sum (accumulated in FP64). */
int xo_rho_batch(const xo_rho_args* pairs, int npairs, void* stream);

/* ------------------------------------------------------------------------- */
/* chi0 at imaginary frequencies, Eq. (X_IP) with the App. A split into the
 * frequency-free outer products and one frequency factor per transition:
 *   chi0[w][G][G'] (+)= -pref sum_t [2 dE_t / (w^2 + dE_t^2)] rho[t][G] conj(rho[t][G'])
 * A weighted Hermitian rank-nt update; only G-blocks i <= j are computed and
 * the lower triangle is written as the conjugate, so the result is exactly
 * Hermitian with a real diagonal.
 *
 * rho: [device] [nt][ng] complex (complex128 for XO_FP64, complex64 otherwise).
 * dE:  [device] [nt] pole energies, must be > 0 (with check_dE set the call
 *      synchronises the stream and returns XO_ERR_ARG if any is <= 0 or NaN).
 * w:   [host] [nw] imaginary frequencies (Ha), w >= 0, nw <= 64.
 * chi0: [device] [nw][ng][ng] complex128; accumulate = 0 overwrites, 1 adds
 *      (so chunks of transitions can be streamed).
 * prec: XO_FP64 (FP64 MFMA), XO_FP32 (FP32 MFMA, FP32 accumulation within a
 *      transition chunk, FP64 across chunks), XO_BF16X3 (each operand split
 *      into bf16 hi + lo, three bf16 MFMA products hi*hi + hi*lo + lo*hi,
 *      FP32 accumulation within a chunk, FP64 across chunks), XO_BF16 (each
 *      operand rounded to bf16, one product, FP32 accumulation within a chunk,
 *      FP64 across chunks).
 */
typedef struct {
  int nt, ng, nw;
  int prec;
  const void* rho;
  const double* dE;
  const double* w;
  double pref;
  int accumulate;
  int check_dE;
  double* chi0;
} xo_chi0_args;

int xo_chi0(const xo_chi0_args* a, void* stream);

/* Independent-particle response at real frequencies, Eq. (X_IP) with the
 * time-ordered poles (every transition its own pole group: the split of
 * Appendix A with the degeneracy threshold at zero):
 *   chi0[w][G][G'] (+)= pref sum_t F_t(w) rho[t][G] conj(rho[t][G']),
 *   F_t(w) = 1/(w - dE_t + i eta) - 1/(w + dE_t - i eta).
 * Not Hermitian. It is formed as A + i B, A and B the Hermitian updates with
 * the real weights Re F and Im F, each run by the kernels of xo_chi0 in the
 * given precision (so XO_BF16X3 / XO_BF16 / XO_FP32 accumulate in FP32 within a
 * transition chunk and in FP64 across chunks, as there); frequencies go in
 * chunks of 32 (64 weight slots). The Dyson step for these matrices is
 * xo_epsinv with XO_EPS_LU_FALLBACK (eps~ is not Hermitian off the imaginary
 * axis).
 * rho: [device] [nt][ng] complex (complex128 for XO_FP64, complex64 otherwise);
 * dE:  [device] [nt] pole energies > 0 (check_dE as for xo_chi0);
 * w:   [host] [nw] real frequencies (Ha), finite and >= 0, any count;
 * eta: broadening (Ha), > 0; chi0: [device] [nw][ng][ng] complex128.
 * Errors: XO_ERR_ARG for bad sizes, pointers, frequencies, eta or precision. */
typedef struct {
  int nt, ng, nw;
  int prec;
  const void* rho;
  const double* dE;
  const double* w;
  double eta;
  double pref;
  int accumulate;
  int check_dE;
  double* chi0;
} xo_chi0_real_args;

int xo_chi0_real(const xo_chi0_real_args* a, void* stream);

/* Many chi0 problems (q-points with their own G-set size, transitions and
 * output) sharing precision and frequencies, in one persistent launch: the
 * problems are cut into units (problem, block of the upper triangle, group of
 * frequencies, transition slice of kper), queued longest-first, and taken by
 * num_CUs * wg_per_cu workgroups from an atomic counter until the queue is
 * empty; partials are reduced per block in a fixed order, so the result does
 * not depend on the schedule and equals xo_chi0 on each item up to the order
 * of the FP64 partial sums. Blocks: nt_tiles 1 or 2 gives 16-row x 16*nt_tiles-
 * column blocks with up to 8 frequencies per unit, one wave per transition
 * quarter; nt_tiles 4 (XO_BF16X3 and XO_BF16 only) gives 64 x 64 blocks with 4
 * frequencies per unit, two units of one block and slice per eight-wave
 * workgroup (their rho strips staged once) and the right operand converted once
 * per workgroup in LDS; nt_tiles 8 (same forms) gives 64 x 128 strips with 2 frequencies per unit
 * (half the left-operand conversion per product, twice the right-operand reads).
 * With nt_tiles 0 the bf16 forms take the 64 x 64 form when there are at least
 * four frequencies, every other case 16 x 16. items: [host] array. */
typedef struct {
  int nt_tiles;   /* 0 (default), 1, 2, or 4 / 8 (XO_BF16X3 / XO_BF16 only)       */
  int kper;       /* transitions per unit; 0 = chosen to fill the chip            */
  int wg_per_cu;  /* persistent four-wave workgroups per compute unit (the 64 x 64
                     form runs half as many eight-wave ones); 0 = 2 (64 x 64), 4   */
} xo_tune;

int xo_chi0_batch(const xo_chi0_args* items, int n, const xo_tune* tune, void* stream);
/* Times a grid of xo_tune candidates on the given batch (each after a warm-up
 * run; results overwrite the outputs) and returns the fastest with its time in
 * milliseconds. Synchronises the stream. Items with accumulate set are rejected
 * (XO_ERR_ARG): every candidate run would add its update again. */
int xo_chi0_autotune(const xo_chi0_args* items, int n, xo_tune* best, double* best_ms, void* stream);

/* ------------------------------------------------------------------------- */
/* Inverse dielectric matrix by the Dyson equation in matrix form, Eq. (X_rpa_inv):
 *   eps~ = I - diag(s) chi0 diag(s),  s_G = sqrt(4 pi)/|q+G|,
 *   out  = eps~^-1                       (XO_EPS_SYM, default; the matrix that
 *                                          Eq. (W_def) scales by 4pi/(|q+G||q+G'|))
 *   out  = (I - v chi0)^-1 = diag(s) eps~^-1 diag(1/s)   (XO_EPS_NONSYM)
 * Always FP64. eps~ is Hermitian positive definite at imaginary frequencies;
 * the inversion is a blocked Gauss-Jordan (64-wide blocks) without pivoting
 * whose pivots are the LDL^H diagonal, so a non-positive pivot proves eps~ is
 * not PD: the call then returns XO_ERR_NOTPD naming the first such frequency.
 * XO_EPS_LU_FALLBACK is the form for general (non-Hermitian) eps~, e.g. at real
 * frequencies: each diagonal block is inverted with partial pivoting inside the
 * block, and a pivot below 1e-13 of the block's largest entry (a numerically
 * singular block: the elimination does not pivot across blocks) returns
 * XO_ERR_SINGULAR instead of an inaccurate inverse. With info NULL the call
 * synchronises the stream to read the pivot flags; with info set it does not
 * synchronise and leaves them to the caller. The diagonal-block sweeps (positive
 * definite form), panel products and trailing rank-64 updates run on FP64 matrix
 * cores; the environment variable
 * XO_EPS_RANK=valu, read on each call, runs them on VALU instead (results agree
 * to FP64 rounding).
 * qpg: [host] [ng] |q+G| (at q = 0 the G = 0 entry is 1 and chi0's G = 0 row and
 *      column are the q-normalised head and wings).
 * chi0: [device] [nw][ng][ng] complex128 (read only); out: [device] same shape.
 * info: [device] [nw] int32 or NULL. When set, info[w] receives 0 if frequency w
 *      passed and 1 + the index of its first failing pivot otherwise, written
 *      in stream order; the call then returns XO_OK without waiting for the
 *      kernels, and out is valid only where info[w] == 0.
 */
enum { XO_EPS_SYM = 0, XO_EPS_NONSYM = 1, XO_EPS_LU_FALLBACK = 2 };

typedef struct {
  int ng, nw;
  const double* qpg;
  const double* chi0;
  int flags;
  double* out;
  int* info;
} xo_eps_args;

int xo_epsinv(const xo_eps_args* a, void* stream);

/* xo_epsinv for callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same arguments,
 * results and errors as xo_epsinv, but the call allocates nothing (no hipMalloc,
 * no host or device workspace, no table cache). Its flags, scales, |q+G| copy and
 * saved column panel live in a static device array of 64 MiB that every GPU the
 * library runs on holds until the process ends; (align_up(4 nw, 256) +
 * align_up(8 nw, 256) + align_up(8 ng, 256) + 1024 nw ng bytes when ng > 64) must
 * fit in it, and without info nw <= 1024 (the flags are read back into a fixed host
 * array); larger calls return XO_ERR_UNSUPPORTED before anything is enqueued.
 * Every call on a GPU shares that GPU's array and leaves its contents behind (the
 * flags and scales are cleared by each call): calls that overlap on one GPU, on any
 * streams, race and must be ordered by the caller. |q+G| is copied from the host
 * array with hipMemcpyAsync, and without info the call synchronises the stream as
 * xo_epsinv does. */
int xo_epsinv_noalloc(const xo_eps_args* a, void* stream);


/* ------------------------------------------------------------------------- */
/* Learned empty-band tail (not in the paper: it takes the place of the
 * extrapolar X-terminator of Eq. (X_term_def) / Appendix B). A small MLP maps
 * features of the truncated band sum to the missing tail of chi0; the full band
 * sum stays available as fallback and as the reference for its error.
 *
 * MLP layout: nl layers with widths dims[0..nl] ([host]); SiLU after every layer
 * but the last. params [device] FP32: per layer W [dims[l+1]][dims[l]] row-major
 * then b [dims[l+1]]; grads has the same layout. X [n][dims[0]], Y [n][dims[nl]].
 * acts [device] holds, per hidden layer, the pre-activation Z [n][w] followed by
 * H = silu(Z) [n][w]; size sum_{l<nl} 2 n dims[l+1] floats.
 * work [device] for backward: 2 n max(dims) floats. dX may be NULL. */
int xo_mlp_forward(int nl, const int* dims, const float* params, const float* X, int n, float* acts,
                   float* Y, void* stream);
int xo_mlp_backward(int nl, const int* dims, const float* params, const float* X, int n, const float* acts,
                    const float* dY, float* grads, float* work, float* dX, void* stream);
/* Mean squared error over n elements: loss[0] = mean (Y - T)^2 and, if dY is not
 * NULL, dY = 2 (Y - T) / n. partial [device]: 256 floats of scratch. */
int xo_mse(const float* Y, const float* T, long n, float* dY, float* loss, float* partial, void* stream);
/* Adam (Kingma and Ba) with bias correction for step >= 1, in place on n parameters. */
int xo_adam_step(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                 int step, void* stream);
/* Column statistics of X [n][F] (device): out [device] [F][4] = mean, standard
 * deviation, min, max (FP64, fixed-order reduction). */
int xo_col_stats(const float* X, long n, int F, double* out, void* stream);
/* dst[r][:] = src[idx[r]][:] for n rows of F floats (minibatch assembly). */
int xo_gather_rows(const float* src, const int* idx, int n, int F, float* dst, void* stream);

/* Tail features per (w, G, G'), 9 per element, normalised as (f - mu) * isd:
 * Re, Im of s_G chi_t s_G'; Re, Im of s_G (chi_t - chi_h) s_G'; |q+G|, |q+G'|,
 * |G - G'|, w, delta_GG' (s_G = sqrt(4 pi)/|q+G|). chi_t: truncated sum; chi_h:
 * the sum over the lower part of the same bands (its difference is the
 * contribution of the last block). When chi_f and T are given, also writes the
 * target T [n][2] = tsc * s_G (chi_f - chi_t) s_G'. |G - G'| is taken from the
 * Cartesian G = sum_k m_k b_k (FP64). Device: chi_*, X, T; host: qpg [ng],
 * mill_g [ng][3], bvec [3][3] (rows b_1, b_2, b_3), w [nw], mu [9], isd [9]. */
typedef struct {
  const double* chi_t;
  const double* chi_h;
  const double* chi_f;
  const double* qpg;
  const int32_t* mill_g;
  const double* bvec;
  const double* w;
  int ng, nw;
  const float* mu;
  const float* isd;
  double tsc;
  float* X;
  float* T;
} xo_tail_args;

int xo_tail_features(const xo_tail_args* a, void* stream);

/* Fused inference of the learned tail: for every element e = (w, G, G') of
 * [nw][ng][ng], the features of xo_tail_features (from chi_t and chi_h, normalised
 * with mu and isd) go through each ensemble member's MLP
 *   dims = [F <= 16, 256, ..., 256, 2] (nl = len(dims) - 1 >= 2 layers, SiLU between),
 * and Y[e] = the members' mean output. The layer products run on bf16 matrix cores
 * (weights and activations rounded to nearest even, FP32 accumulation, biases and
 * SiLU in FP32). Guard statistics, as xo_tail_guard computes them over the same
 * features and member outputs (two members; with one, stats[1] = 0 and stats[2] =
 * sum |Y|^2): stats[0] = features outside [lo - m, hi + m], stats[1] = sum |Y1 - Y2|^2,
 * stats[2] = sum |(Y1 + Y2)/2|^2. The corrected chi0 is then xo_tail_apply(chi_t, Y).
 * Errors: XO_ERR_ARG for null pointers or bad sizes, XO_ERR_UNSUPPORTED for other
 * widths. params [device] [nmem][P] FP32 flat parameters (W_l [out][in] row-major then
 * b_l, layer by layer), nmem 1 or 2; chi_t, chi_h, Y [n][2], stats [3]: device; qpg,
 * mill_g, bvec, w, mu, isd, lo, hi, dims: host. */
typedef struct {
  const double* chi_t;
  const double* chi_h;
  const double* qpg;
  const int32_t* mill_g;
  const double* bvec;
  const double* w;
  int ng, nw;
  const float* mu;
  const float* isd;
  const float* lo;
  const float* hi;
  int nl;
  const int* dims;
  int nmem;
  const float* params;
  float* Y;
  double* stats;
} xo_tail_predict_args;

int xo_tail_predict(const xo_tail_predict_args* a, void* stream);
/* out = chi_t + Hermitian part of Y / (tsc s_G s_G'), Y = Y1 or (Y1 + Y2)/2 when Y2
 * is not NULL; Y1, Y2 [device] [nw][ng][ng][2]; qpg [host] [ng]; out must not alias chi_t. */
int xo_tail_apply(const double* chi_t, const float* Y1, const float* Y2, const double* qpg, int ng, int nw,
                  double tsc, double* out, void* stream);
/* Fallback test inputs: stats[0] = number of features outside the training range
 * widened by 10 % of its span (at least 1e-6: a feature that is zero up to
 * rounding in training, as Im chi0 of a centrosymmetric crystal, does not reject
 * data for its rounding); stats[1] = sum |Y1 - Y2|^2 and stats[2] =
 * sum |(Y1 + Y2)/2|^2 for two ensemble members. lo, hi [host] [F]; stats [device] [3]. */
int xo_tail_guard(const float* X, long n, int F, const float* lo, const float* hi, const float* Y1,
                  const float* Y2, int ny, double* stats, void* stream);

/* ------------------------------------------------------------------------- */
/* Bruneval-Gonze extrapolar correction of chi0 (the X-terminator; Eq. X_term_def,
 * Appendix B Eq. X-term) for one k-pair at imaginary frequencies, added to out:
 *   out[w][G][G'] += -pref sum_v W(w, ebar - e_v) [ <v| e^{i(G-G').r} |v>
 *                                                   - sum_{n < nn} rho_nv(G) conj(rho_nv(G')) ],
 *   W(w, D) = 2 D / (w^2 + D^2).
 * The empty states above the nn explicit bands at k get the single energy ebar
 * (the paper's default: the highest explicit band energy + 1.5 Ha), so their sum
 * closes over all states at k: the density element of each occupied v at k'
 * minus the explicit bands, occupied ones included. rho holds rho_nv(G) of the
 * nn explicit bands at k against the nv occupied bands at k', as written by
 * xo_rho with the conduction side set to bands 0 .. nn-1 (rows t = v nn + n).
 * Passing the truncated chi0 as out yields the corrected chi0. The density
 * elements are plane-wave sums in FP64; the explicit-band update runs in prec
 * (XO_FP64: complex128 coef_v and rho; the other precisions: complex64, with the
 * products of xo_chi0 in that precision). q = 0 (head and wings) is not treated.
 * Errors: XO_ERR_ARG for bad sizes or an ebar not above every e_v (checked on the
 * device; the call then synchronises).
 *   mill_v [host] [npw_v][3]; coef_v [device] [nv][npw_v];
 *   e_v [device] [nv]; mill_g [host] [ng][3]; w [host] [nw];
 *   rho [device] [nv*nn][ng]; out [device] [nw][ng][ng] complex128. */
typedef struct {
  int npw_v;
  const int32_t* mill_v;
  int nv;
  const void* coef_v;
  const double* e_v;
  double ebar;
  int ng;
  const int32_t* mill_g;
  int nw;
  const double* w;
  double pref;
  int nn;
  const void* rho;
  double* out;
  int prec;
} xo_xterm_args;

int xo_xterm(const xo_xterm_args* a, void* stream);

/* ------------------------------------------------------------------------- */
/* Godby-Needs plasmon-pole model of the screened interaction (Quasi-particle
 * corrections section, plasmon-pole paragraph; Eq. W_def). Every element of
 * X = eps~^-1 - 1 (eps~^-1 as written by xo_epsinv with XO_EPS_SYM) gets one
 * pole pair X(w) = R [1/(w - Om) - 1/(w + Om)], fixed by X(0) and X(i omega_p):
 *   Om = omega_p sqrt(Xp / (X0 - Xp))  (principal root),  R = -X0 Om / 2,
 * where Re(Xp conj(X0 - Xp)) > 0 (evaluated without fused operations); any
 * other element keeps its static value: Om = omega_p, R = -X0 omega_p / 2.
 * Output is the residue of the screened part of W, Wr = R v^1/2_G v^1/2_G', and
 * Om. The library forms the Coulomb factors (Coulomb interaction subsection):
 * v^1/2_G = sqrt(4 pi)/|q+G|; at q = 0 (q0 = 1, G = 0 the first entry of the
 * G-set) v^1/2_0 = 0 (the wings, odd in q, average to zero over the small cell
 * around q = 0) and the (0, 0) element takes the mean of 4 pi/q^2 over the sphere
 * of volume (2 pi)^3/(N_k Omega), 12 pi/q_c^2, q_c = (6 pi^2/(N_k Omega))^(1/3)
 * (a reading: the paper leaves the q = 0 treatment to the Coulomb options). FP64.
 *   einv0, einvp: [device] [ng][ng] complex128 (eps~^-1 at 0 and i omega_p)
 *   qpg: [host] [ng] |q+G| in 1/bohr, positive and finite (entry 0 not read when q0)
 *   nk_omega: N_k Omega in bohr^3 (read when q0)
 *   wr, om: [device] [ng][ng] complex128, written (may not alias the inputs).
 * Errors: XO_ERR_ARG for ng <= 0, null pointers, omega_p <= 0, a bad |q+G|, or
 * nk_omega <= 0 at q = 0. */
typedef struct {
  int ng;
  const void* einv0;
  const void* einvp;
  double omega_p;
  const double* qpg;
  int q0;
  double nk_omega;
  void* wr;
  void* om;
} xo_ppa_args;

int xo_ppa_fit(const xo_ppa_args* a, void* stream);

/* Diagonal GW self-energy matrix elements of one q (Eq. sigma_c with the
 * plasmon-pole W, whose frequency integral is done in closed form; Eq. I_c
 * for the index order):
 *   sigc[n][j] (+)= pref sum_m sum_{G,G'} rho_nm(G) conj(rho_nm(G')) Wr_GG'
 *                   [ f_m / (z_nj - e_m + Om_GG' - i eta) + (1 - f_m) / (z_nj - e_m - Om_GG' + i eta) ]
 *   sigx[n]    (+)= -pref sum_m f_m sum_G |rho_nm(G)|^2 v_G,  v_G = 4 pi/|q+G|^2 (q = 0: the head
 *                   mean of 4 pi/q^2 at G = 0, as in xo_ppa_fit)
 * rho_nm(G) = <n k| e^{i(q+G).r} |m k-q> as written by xo_rho with the states n
 * on the conduction side (at k) and the bands m on the valence side (at k-q).
 * pref = 1/(N_k Omega) from nk_omega = N_k Omega (bohr^3); e_m in Ha on the scale
 * of z; f_m in [0, 1] per spin.
 * Sum over q by calling once per q with accumulate = 1 after the first.
 * rho_swapped = 1: rho holds instead the mirrored strengths
 * <m k-q| e^{i(-q+G').r} |n k> for G' = -G, which equal conj(rho_nm(G)), in
 * [nn][nm][ng], as xo_rho writes them with the bands m on the conduction side
 * (at k-q), the states on the valence side, G0 negated and the G-set negated
 * (the wide side on the conduction side suits the gathered-product kernel).
 *   rho: [device] [nm][nn][ng] complex128 ([nn][nm][ng] when swapped); wr, om: [device] [ng][ng] complex128
 *   (from xo_ppa_fit); e_m, f_m: [device] [nm]; z: [device] [nn][nz] complex128
 *   (nz <= 4; z may be complex, e.g. i nu with eta = 0 on the imaginary axis);
 *   qpg: [host] [ng] |q+G| (needed when sigx is set; q0 as in xo_ppa_fit); sigx: [device] [nn] or NULL;
 *   sigc: [device] [nn][nz] complex128 (unused when nz = 0).
 * Errors: XO_ERR_ARG for bad sizes, nz > 4, null pointers, nk_omega <= 0, eta < 0,
 * a bad |q+G|. */
typedef struct {
  int nm, nn, ng, nz;
  const void* rho;
  const void* wr;
  const void* om;
  const double* e_m;
  const double* f_m;
  const void* z;
  double eta;
  double nk_omega;
  const double* qpg;
  int q0;
  double* sigx;
  void* sigc;
  int accumulate;
  int rho_swapped;
} xo_sigma_args;

int xo_sigma(const xo_sigma_args* a, void* stream);

/* ------------------------------------------------------------------------- */
/* Workspace size queries. Each returns in *bytes the device workspace that the
 * matching call with the same arguments takes from the library's per-stream
 * cache (before the cache's own rounding), so that a caller can budget device
 * memory ahead of the call. Small constant tables (Coulomb factors, gather
 * tables, launch plans) are cached apart and not counted. Host computation
 * only: no device work, no allocation, no GPU needed. Errors: the argument
 * errors of the matching call (XO_ERR_ARG), and XO_ERR_UNSUPPORTED where the
 * call would return it.
 *   xo_rho_workspace_size:   xo_rho_batch over npairs pairs (xo_rho: npairs = 1);
 *                            the kernel path is chosen as the call chooses it.
 *   xo_chi0_workspace_size:  xo_chi0_batch over n items with tune (xo_chi0: n = 1,
 *                            tune NULL).
 *   xo_epsinv_workspace_size: xo_epsinv (only ng and nw are read). */
int xo_rho_workspace_size(const xo_rho_args* pairs, int npairs, size_t* bytes);
int xo_chi0_workspace_size(const xo_chi0_args* items, int n, const xo_tune* tune, size_t* bytes);
int xo_epsinv_workspace_size(const xo_eps_args* a, size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* XO_H */
