/*
 * ufss.h -- C ABI of libufss: the matrix-free Fourier-subsampled pulse-echo
 * operator A, its adjoint A^H and the FISTA / ISTA l1 solver on MI355X (gfx950).
 *
 * The operator (paper Sec. II, eq. of the frequency-domain A-scan model,
 * discretised on the G2D / G3D grids; Sec. II-B compression Phi = S F Sigma with
 * Sigma = I):
 *
 *   A[(p, m), v] = H_k * 1[|p_x - v_x| <= W_x, |p_y - v_y| <= W_y]
 *                      * exp(-j 2 pi f_k (tau(p - v, z_v) - t0)),
 *   k = k_m(p) (the m-th selected DFT bin of scan position p), f_k = k f_s / N_t,
 *   tau(d, z) = (2 / c) sqrt((d_x dx)^2 + (d_y dy)^2 + z^2),  z_v = z_start + j_z dz,
 *   H_k = f_s sqrt(2 pi) sigma_t exp(-(f_k - f_c)^2 / (2 sigma_f^2)),
 *   sigma_f = frac_bw f_c / (2 sqrt(2 ln 2)), sigma_t = 1 / (2 pi sigma_f).
 *
 * Conventions shared by every call:
 *   - Every call returns UFSS_OK (0) or a negative UFSS_ERR_* code and never
 *     throws; ufss_last_error() then describes the failure (thread-local).
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - Complex buffers are interleaved float pairs (re, im), i.e. complex64.
 *   - x (reflectivity) is laid out [ny][nx][nz] (depth fastest);
 *     y (measurements) is [ny][nx][m] (bin fastest).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     is asynchronous unless the comment says the call synchronises.
 *   - The caller owns x, y and every buffer it passes; a plan owns its own
 *     device tables and workspace.  A plan is not thread-safe: use one plan per
 *     host thread / stream.
 */
#ifndef UFSS_H
#define UFSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define UFSS_OK                  0
#define UFSS_ERR_INVALID_ARG    -1  /* bad size, pointer or option            */
#define UFSS_ERR_BAND_TOO_SMALL -2  /* m exceeds the number of band bins      */
#define UFSS_ERR_HIP            -3  /* a HIP runtime call failed              */
#define UFSS_ERR_OOM            -4  /* device allocation failed               */
#define UFSS_ERR_UNSUPPORTED    -5  /* valid request the library cannot serve  */
#define UFSS_ERR_DIVERGED       -6  /* non-finite or exploding FISTA iterates */

/* ---- operator precision ------------------------------------------------ */
#define UFSS_F32  0   /* FP32 phasors and operands, FP32 accumulation           */
#define UFSS_BF16 1   /* BF16 phasors and operands, FP32 accumulation           */

/* ---- operator algorithm -------------------------------------------------- */
#define UFSS_ALGO_AUTO   0  /* GEMM, except FP32 per-position subsets whose
                               union holds at least 5 times the bins of one
                               position: phasor path (measured faster there)  */
#define UFSS_ALGO_GEMM   1  /* windowed complex GEMM over (offset, depth) on MFMA;
                               per-position subsets run over their union of bins
                               and are gathered / scattered                    */
#define UFSS_ALGO_PHASOR 2  /* per-position on-the-fly phasors (VALU); FP32 only */
#define UFSS_ALGO_FFT    3  /* transform domain (Sec. IV-B, Alg. 2): the windowed
                               correlation as a cyclic lateral transform of size
                               L >= N + W per axis, contracted over depth / bins
                               with a precomputed transformed kernel table
                               ((ly/2+1)(lx/2+1) nz (union bins) complex, built
                               in FP64, stored FP32, or BF16 for BF16 plans with
                               transforms and sums still in FP32); shared or
                               per-position (over the union) subsets; no grouped
                               (batched) launches */

/* Scan and pulse geometry (SI units).  Paper Sec. II-A (grids, delay, pulse),
 * Sec. VI (Gabor pulse).  t0 = NaN selects the window that centres the delay
 * span of the aperture: t0 = (tau_min + tau_max)/2 - nt/(2 fs).  ny = 1 is a
 * B-scan.  win_x / win_y < 0 means the full grid.  theta > 0 adds the Gaussian
 * beam of Sec. VI / VII: every entry of A is scaled by
 * g = exp(-r^2 / (z tan theta)^2), r the lateral distance between position and
 * voxel, z the voxel depth (the form whose x-derivative the paper prints);
 * theta = 0: g = 1.  The window applies either way. */
typedef struct ufss_geom {
    int32_t nx, ny, nz, nt;
    double dx, dy, dz, z_start, t0, c, fs, fc, frac_bw, band_db;
    int32_t win_x, win_y;
    int32_t dtype;      /* UFSS_F32 or UFSS_BF16 */
    int32_t algo;       /* UFSS_ALGO_* */
    double theta;       /* beam half-angle in radians, [0, pi/2); 0 = none */
} ufss_geom;

typedef struct ufss_plan_s* ufss_plan_t;
typedef void* ufss_stream_t;

/* Derived plan quantities (host struct filled by ufss_plan_info). */
typedef struct ufss_plan_info {
    double t0;            /* window start actually used (s)                    */
    double lipschitz;     /* cached L from ufss_lipschitz, 0 if not computed   */
    int32_t band_lo, band_hi, band_size;  /* pulse band [lo, hi] and its size   */
    int32_t win_x, win_y; /* effective aperture half-widths                    */
    int32_t m, per_position, dtype, algo; /* algo actually used                */
    int32_t union_size;   /* bins in the union of per-position subsets         */
    int64_t workspace_bytes;              /* device memory owned by the plan    */
    int32_t fwd_split, adj_split;         /* split-K factors of the GEMM path   */
    int32_t fwd_waves, fwd_zsplit;       /* FP32 forward: waves per workgroup;
                                            GEMM forward: depth split (1 for
                                            phasor and transform plans)        */
    int32_t fwd_tile, adj_tile;          /* FP32 GEMMs: 16-position sub-tiles
                                            per wave; BF16 adjoint (adj_tile):
                                            16-depth sub-tiles per wave (0
                                            elsewhere)                         */
    int32_t fwd_rows, adj_rows;          /* BF16 GEMMs: rows of waves in a
                                            tile (0 elsewhere)                 */
    int32_t fwd_chunk, adj_chunk;        /* FP32 GEMMs: staged depth / bin
                                            chunk (0 elsewhere)                */
    int32_t phasor_tables;               /* 1: BF16 phasor tables in use       */
    int32_t adj_waves;                   /* FP32 GEMM adjoint: waves per
                                            workgroup (0 elsewhere)            */
} ufss_plan_info;

/* Per-iteration FISTA statistics, FP64, written to HOST arrays of length
 * `iters` (each pointer may be NULL).  obj[k] = 1/2 ||A gamma_k - y||^2 +
 * lambda ||gamma_k||_1 (objective at the extrapolated point), res[k] =
 * ||A gamma_k - y||, rel_change[k] = ||a_k - a_{k-1}|| / ||a_k||, err_ref[k] =
 * ||a_k - a_ref|| / ||a_ref|| (only if a_ref was given). */
typedef struct ufss_fista_stats {
    double* obj;
    double* res;
    double* rel_change;
    double* err_ref;
    int32_t iters_done;   /* out: iterations executed                           */
    double lambda;        /* out: lambda used                                   */
} ufss_fista_stats;

/* Resumable FISTA state.  gamma is a caller-owned DEVICE buffer [ny][nx][nz]
 * complex64 holding the extrapolated point; k_done counts completed
 * iterations (0 = start from x).  The momentum sequence t_k depends on k only,
 * so (x = a_k, gamma, k_done) is the whole state. */
typedef struct ufss_fista_state {
    void* gamma;
    int32_t k_done;
} ufss_fista_state;

/* Message for the last failing call on this thread ("" if none). */
const char* ufss_last_error(void);

/* Select m DFT bins inside the pulse band from a seeded random draw.
 * Paper Sec. III-A (random sampling, and the per-A-scan variants of Table I).
 * The band is {k in [0, nt/2] : exp(-(f_k - f_c)^2 / (2 sigma_f^2)) >=
 * 10^(-band_db/20)}.  Generator: SplitMix64; key = seed for a shared subset,
 * seed XOR mix64(p + 1) for position p = ix + nx*iy; partial Fisher-Yates over
 * the ascending band with multiply-high bounds; each subset sorted ascending.
 *   bins_out      HOST int32 [m] (shared) or [ny][nx][m] (per_position != 0)
 *   band_size_out HOST, optional (may be NULL)
 * Errors: INVALID_ARG, BAND_TOO_SMALL (m > band size). */
int ufss_select_freqs(const ufss_geom* g, int32_t m, int32_t per_position,
                      uint64_t seed, int32_t* bins_out, int32_t* band_size_out);

/* ---- frequency sampling strategies (paper Sec. III-A, Table I) ---------- */
#define UFSS_SAMPLE_RND   0  /* uniform over the band, shared (Sigma = I)        */
#define UFSS_SAMPLE_RND_F 1  /* uniform over the band, one subset per position   */
#define UFSS_SAMPLE_MAX   2  /* the m bins of largest |H_k| (maximal sampling)   */
#define UFSS_SAMPLE_NRG   3  /* energy-based: drawn with probability |H_k| /
                                ||H||_1 without replacement, shared             */
#define UFSS_SAMPLE_NRG_F 4  /* energy-based, one subset per position           */

/* Select m DFT bins by one of the strategies of Sec. III-A.  RND / RND_F are
 * ufss_select_freqs.  MAX, NRG and NRG_F take their candidates from bins
 * 0..nt/2 (the complex Gabor pulse has no energy at negative frequencies) with
 * weights w_k = exp(-(f_k - f_c)^2 / (2 sigma_f^2)), proportional to |H_k|.
 * MAX keeps the m largest weights, ties to the lower bin.  NRG draws m times
 * without replacement: a draw takes u = (next() >> 11) 2^-53 from the
 * SplitMix64 stream, scales it by the FP64 sum of the remaining weights in
 * ascending bin order, and takes the first remaining bin whose running sum
 * exceeds it; the bin is then removed (the remaining weights renormalise).
 * NRG_F keys position p = ix + nx*iy with seed XOR mix64(p + 1).  Subsets are
 * sorted ascending.
 *   bins_out          HOST int32 [m] (RND, MAX, NRG) or [ny][nx][m] (RND_F,
 *                     NRG_F)
 *   per_position_out  HOST, optional: 1 for the per-position strategies
 * Errors: INVALID_ARG, BAND_TOO_SMALL (m above the candidates). */
int ufss_sample_bins(const ufss_geom* g, int32_t m, int32_t strategy, uint64_t seed,
                     int32_t* bins_out, int32_t* per_position_out);

/* Estimate of the largest singular value of A from its Frobenius norm (paper
 * Sec. IV-C, estimation by the geometric mean of the Frobenius bounds).  Host
 * only, FP64, no device work.
 *   fro_sq            ||A||_F^2, exact: sum over positions p and bins of
 *                     H_k^2 times the sum of g^2 over the voxels inside the
 *                     window of p (their count without a Gaussian beam)
 *   fro_sq_central    the paper's approximation: N_x N_y times the squared
 *                     norms of the columns of voxel ((nx-1)/2, (ny-1)/2),
 *                     summed over depth
 *   n                 N = N_x N_y min(m, N_z), a bound on the rank of A
 *   sigma_hat         sqrt(fro_sq) / N^(1/4)
 *   sigma_hat_central sqrt(fro_sq_central) / N^(1/4)
 * sigma_hat^2 can stand in for L in ufss_fista; it is not guaranteed to bound
 * the true L from above, and FISTA reports UFSS_ERR_DIVERGED when it does not
 * suffice. */
typedef struct ufss_sigma_est {
    double fro_sq, fro_sq_central;
    int64_t n;
    double sigma_hat, sigma_hat_central;
} ufss_sigma_est;

/*   bins  HOST int32 [m] or [ny][nx][m], as for ufss_plan_create
 *   out   HOST
 * Errors: INVALID_ARG. */
int ufss_sigma_estimate(const ufss_geom* g, int32_t m, int32_t per_position,
                        const int32_t* bins, ufss_sigma_est* out);

/* One point scatterer for ufss_crb: position (x, y) in metres on the scan grid
 * (position (ix, iy) sits at (ix dx, iy dy)), depth z (> 0), amplitude amp
 * (> 0), phase (rad; the bound does not depend on it) and the noise variance
 * sigma2 (> 0) of each measured coefficient. */
typedef struct ufss_crb_point {
    double x, y, z, amp, phase, sigma2;
} ufss_crb_point;

/* Cramer-Rao bound on the scatterer's position for `trials` bin selections
 * at once (paper Sec. VI: Slepian-Bangs Fisher information of the measured
 * coefficients, position block of its inverse by the Schur complement of the
 * amplitude / phase block).  The measurement of bin k at position i is
 * a e^{j phase} H_k g_i exp(-j 2 pi f_k (tau_i - t0)), with the operator's
 * H_k, delay and Gaussian beam; positions outside the aperture window of the
 * scatterer do not measure it.  Derivatives: d tau / d x = (2/c)(x - x_i)/R,
 * d g / d x = -2 (x - x_i) / (z tan theta)^2 g, d g / d z =
 * 2 r^2 / (z^3 tan^2 theta) g.  Sums in FP64 on the device (one workgroup per
 * selection, fixed order); the 5 x 5 algebra on the host in FP64.
 *   bins      HOST int32 [trials][m] (shared) or [trials][ny][nx][m], each
 *             subset as for ufss_plan_create
 *   fim_out   HOST double [trials][5][5] or NULL: J, parameters (x, y, z,
 *             amp, phase)
 *   crb_out   HOST double [trials][3]: (C_x, C_y, C_z) in m^2
 * Synchronises `stream`.  Allocates and frees two device buffers.
 * Errors: INVALID_ARG (also for a singular information matrix), HIP, OOM. */
int ufss_crb(const ufss_geom* g, int32_t m, int32_t per_position, int32_t trials,
             const int32_t* bins, const ufss_crb_point* pt, double* fim_out, double* crb_out,
             ufss_stream_t stream);

/* The same bound for randomly mixed measurements (Rademacher Sigma, as
 * ufss_plan_create_mixed): position i measures M_i B_i with M_i the rows
 * xih_i[(k_m - j) mod nt] over every DFT index j of the spectrum B_i, so the
 * derivative rows are M_i D_i over all nt signed bins and
 * J = (2 / sigma^2) Re{sum_i (M_i D_i)^H (M_i D_i)}.  FP64 on the device: the
 * rows D_i once per call, the transformed signs of every trial, then one
 * workgroup per trial.
 *   bins   HOST int32 [trials][m] or [trials][ny][nx][m], in [0, nt), ascending
 *   signs  HOST int8 [trials][nt] or [trials][ny][nx][nt] (per_position_signs),
 *          +1 / -1
 * nt must be a power of two, at most 4096.  Other arguments as ufss_crb.
 * Errors: INVALID_ARG, UNSUPPORTED (nt), HIP, OOM. */
int ufss_crb_mixed(const ufss_geom* g, int32_t m, int32_t per_position, int32_t trials,
                   const int32_t* bins, int32_t per_position_signs, const int8_t* signs,
                   const ufss_crb_point* pt, double* fim_out, double* crb_out,
                   ufss_stream_t stream);

/* Build a plan: derived geometry (FP64 on the host), the integer-turn delay
 * table, H_k and the device workspace.  Paper Sec. IV-B: the operator is block
 * 2-level Toeplitz in the lateral offset, which the kernels exploit.
 *   bins  HOST int32 [m] or [ny][nx][m]; each subset strictly ascending and in
 *         [0, nt/2] (normally from ufss_select_freqs)
 *   out   HOST, receives the plan handle
 * Errors: INVALID_ARG, UNSUPPORTED (e.g. BF16 with ALGO_PHASOR), OOM, HIP. */
int ufss_plan_create(const ufss_geom* g, int32_t m, int32_t per_position,
                     const int32_t* bins, ufss_plan_t* out);

/* A plan whose measurements are randomly mixed (paper Sec. II-B compression
 * Phi_i = S_i F Sigma_i with the random sampling strategy of Sec. III-A:
 * Sigma_i = Diag(xi_i), xi_i Rademacher; Table I Phi_rnd, Phi_rnd,m and
 * Phi_rnd,m,f).  The measurement of position i is y_i = S_i F Sigma_i b_i with
 * b_i the sampled A-scan, i.e. y_i[m] = sum_j xih_i[(k_m - j) mod nt] B_i[j]
 * with B_i = F b_i over every DFT index j (the signed bin j or j - nt: the
 * Gabor spectrum's small negative-frequency part is kept) and
 * xih_i = F xi_i / nt (FP64 on the host, stored FP32).  The operator core
 * (FP32 GEMM or transform, g->algo) runs over all nt indices; the mixing and
 * its adjoint replace the bin gather / scatter.  Every other call (forward,
 * adjoint, lipschitz, fista, backtracking, the unrolled network) takes the plan
 * as usual; batched FISTA refuses it.
 *   bins   HOST int32 [m] or [ny][nx][m] (per_position): strictly ascending in
 *          [0, nt) (any DFT coefficient of the mixed A-scan)
 *   signs  HOST int8 [nt] or [ny][nx][nt] (per_position_signs) of +1 / -1
 * nt must be a power of two with 8 nt + 12 m <= 65536 (LDS rows of the mixing).
 * Errors: INVALID_ARG, UNSUPPORTED (BF16, phasor path, nt, m), OOM, HIP. */
int ufss_plan_create_mixed(const ufss_geom* g, int32_t m, int32_t per_position,
                           const int32_t* bins, int32_t per_position_signs,
                           const int8_t* signs, ufss_plan_t* out);

/* Release a plan and its device memory (synchronises the device). */
int ufss_plan_destroy(ufss_plan_t plan);

/* Fill a HOST ufss_plan_info. */
int ufss_plan_info_get(ufss_plan_t plan, ufss_plan_info* info);

/* Forward projection y = A x (paper Sec. IV-A, phi mapping).
 *   x  DEVICE complex64 [ny][nx][nz], read only
 *   y  DEVICE complex64 [ny][nx][m], overwritten
 * Asynchronous on `stream`.  x and y must not overlap. */
int ufss_forward(ufss_plan_t plan, const void* x, void* y, ufss_stream_t stream);

/* Backward projection x = A^H y (paper Sec. IV-A, beta mapping; with a delta
 * pulse and no compression it is the SAFT image of the Remark on SAFT).
 *   y  DEVICE complex64 [ny][nx][m], read only
 *   x  DEVICE complex64 [ny][nx][nz], overwritten
 * Asynchronous on `stream`. */
int ufss_adjoint(ufss_plan_t plan, const void* y, void* x, ufss_stream_t stream);

/* Lipschitz constant L = margin_factor * rho of grad 1/2||Ax - y||^2, where rho
 * is the power-iteration Rayleigh quotient ||A v||^2 / ||v||^2 of A^H A
 * (paper Sec. IV-C: sigma_max^2, estimated iteratively; an under-estimate makes
 * FISTA diverge, so L = (1 + margin) rho).  Vectors in the plan's operator
 * precision, norms and quotient in FP64.  Start vector CN(0, I) from SplitMix64
 * keyed by `seed`.  Stops when |rho_k - rho_{k-1}| <= rtol rho_k or after
 * max_iters; iterations run in blocks of 8 between host checks and rho is the
 * first quotient that meets the test.  Synchronises `stream`; caches L in the
 * plan.
 *   L_out  HOST double */
int ufss_lipschitz(ufss_plan_t plan, int32_t max_iters, double rtol,
                   double margin, uint64_t seed, double* L_out,
                   ufss_stream_t stream);

/* FISTA (accel = 1) or ISTA (accel = 0) for min 1/2||A a - y||^2 + lambda||a||_1
 * (paper Alg. 1 with step 1/L, threshold lambda/L, complex soft threshold
 * z max(0, 1 - alpha/|z|), Beck-Teboulle momentum; lambda rule of Sec. VII).
 *   y       DEVICE complex64 [ny][nx][m]
 *   lambda  > 0: used as is; < 0: lambda = (-lambda) * max|A^H y|
 *   L       > 0: Lipschitz constant; <= 0: the plan's cached value (error if none)
 *   iters   number of iterations (>= 0)
 *   tol     > 0: stop early once ||a_k - a_{k-1}|| <= tol ||a_k|| (checked every
 *           8 iterations); 0: run exactly `iters`
 *   accel   bit 0: 1 = FISTA momentum, 0 = ISTA; bit 1: real reflectivity (the
 *           Re{H} comparison of Sec. VII: the gradient step keeps its real part
 *           before the threshold, so every iterate is real; the imaginary part
 *           of a_0 is dropped by the first step); other bits: INVALID_ARG
 *   x       DEVICE complex64 [ny][nx][nz]: in = a_0 (ignored when resuming), out = a_K
 *   a_ref   DEVICE complex64 [ny][nx][nz] or NULL (enables stats->err_ref)
 *   stats   HOST or NULL; state HOST or NULL (see the struct comments)
 * Synchronises `stream` before returning.  Returns UFSS_ERR_DIVERGED if an
 * iterate or residual becomes non-finite or the residual exceeds 1e6 times its
 * first value; x then holds the last iterate. */
int ufss_fista(ufss_plan_t plan, const void* y, double lambda, double L,
               int32_t iters, double tol, int32_t accel, void* x,
               const void* a_ref, ufss_fista_stats* stats,
               ufss_fista_state* state, ufss_stream_t stream);

/* FISTA with backtracking (paper Sec. IV-C, backtracking, after Beck and
 * Teboulle): needs no Lipschitz constant, only a start value L0 and a growth
 * factor eta.  At the extrapolated point gamma_k the constants L_{k-1} eta^i,
 * i = 0, 1, ..., are tried until p = soft(gamma - A^H(A gamma - y)/L, lambda/L)
 * satisfies
 *   f(p) <= f(gamma) + Re<p - gamma, grad f(gamma)> + L/2 ||p - gamma||^2 + s,
 * f = 1/2 ||A . - y||^2, s = eps * 1/2 ||y||^2, a margin for the rounding of
 * the residuals: eps = 1e-6 (FP32 plans) or 2^-8 (BF16 plans, whose input
 * rounding makes f noisy at that level); p is a_k and L_k = L.  Momentum as ufss_fista.
 * Sums and the test are FP64 on the host, one synchronisation per trial.  The
 * residual at gamma_{k+1} is formed from the two accepted residuals (A is
 * linear), so an iteration costs one adjoint and one forward per trial.
 *   lambda, y, x, a_ref, tol   as ufss_fista (tol is checked every iteration)
 *   L0     > 0; eta > 1
 *   stats  HOST or NULL: obj[k] = F(a_k) (at the iterate, not at gamma_k),
 *          res[k] = ||A a_k - y||, rel_change, err_ref (0 without a_ref)
 *   L_out  HOST double [iters] or NULL: accepted L_k
 *   trials_out HOST int32 [iters] or NULL: trials of iteration k (>= 1)
 * Errors: INVALID_ARG, DIVERGED (non-finite residual, or no acceptable step in
 * 100 trials).  Synchronises `stream`.  Does not resume. */
int ufss_fista_backtracking(ufss_plan_t plan, const void* y, double lambda, double L0,
                            double eta, int32_t iters, double tol, void* x, const void* a_ref,
                            ufss_fista_stats* stats, double* L_out, int32_t* trials_out,
                            ufss_stream_t stream);

/* Fused proximal-gradient update, standalone (paper Alg. 1, threshold and
 * momentum lines; ISTA is beta = 0).  For each of n complex entries:
 *   a_new = soft(gamma - step * g, thresh),  gamma <- a_new + beta (a_new - a),
 *   a <- a_new.
 *   gamma, a  DEVICE complex64 [n], updated in place;  g DEVICE complex64 [n]
 *   a_ref     DEVICE complex64 [n] or NULL
 *   norms_out HOST double [5] or NULL: ||a_new||_1, ||gamma_new||_1,
 *             ||a_new - a||^2, ||a_new||^2, ||a_new - a_ref||^2 (FP64, fixed-order
 *             reduction, bitwise reproducible).  Synchronises only if norms_out. */
int ufss_shrink_update(int64_t n, void* gamma, const void* g, void* a,
                       double step, double thresh, double beta,
                       const void* a_ref, double* norms_out,
                       ufss_stream_t stream);

/* max_v |x_v| over n complex entries (FP32 values, exact max), for the lambda
 * rule.  out HOST double.  Synchronises `stream`. */
int ufss_absmax(int64_t n, const void* x, double* out, ufss_stream_t stream);

/* ufss_shrink_update without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as ufss_shrink_update.
 * Its FP64 partials live in a fixed 41 KB device array that each GPU holds
 * until the process ends: every n is accepted (the update's grid is capped), no
 * hipMalloc / hipFree is called, and the library looks the array's address up
 * once per device on the first call there.  Calls on one GPU share that array:
 * calls that overlap on one GPU (several streams or host threads) race, so the
 * caller serialises them.  Synchronises `stream` only if norms_out. */
int ufss_shrink_update_noalloc(int64_t n, void* gamma, const void* g, void* a,
                               double step, double thresh, double beta,
                               const void* a_ref, double* norms_out,
                               ufss_stream_t stream);

/* Batched FISTA over n independent scans of uneven size (each with its own
 * plan), paper Alg. 1 applied to every scan.  Each phase of an iteration runs
 * as ONE grouped launch over all scans (forward GEMM, residual epilogue,
 * adjoint pre pass, adjoint GEMM, update fused with the adjoint's split sums,
 * FP64 reductions),
 * and the `iters` iterations are captured in one hipGraph and launched once on
 * `stream`.  Plans must use the GEMM algorithm (any dtype); a plan may appear
 * only once.
 *   ys[i]      DEVICE complex64 [ny][nx][m] of plan i
 *   xs[i]      DEVICE complex64 [ny][nx][nz]: in = a_0, out = a_iters
 *   lambdas[i] > 0 used as is; < 0: -lambdas[i] * max|A_i^H y_i|   (HOST array)
 *   Ls[i]      > 0 used as is; <= 0: the plan's cached constant      (HOST array)
 *   res_out    HOST double [n] or NULL: final ||A gamma - y|| per scan
 * Synchronises `stream`.  Returns UFSS_ERR_DIVERGED if any scan diverges. */
int ufss_fista_batched(int32_t n, const ufss_plan_t* plans, const void* const* ys,
                       void* const* xs, const double* lambdas, const double* Ls,
                       int32_t iters, double* res_out, ufss_stream_t stream);

/* Synthetic data on the device (training and evaluation scenes of the learned
 * solver; the scenes follow the simulated point-scatterer specimens of Sec.
 * VII).  Random numbers: SplitMix64 (Steele, Lea & Flood 2014) keyed `seed`,
 * whose k-th output is mix64(seed + k 0x9E3779B97F4A7C15).
 * ufss_synth_scene: x (DEVICE complex64 [ny][nx][nz]) = n_scat distinct point
 *   scatterers at voxels with depth index < max_depth, real amplitudes
 *   amp_lo + (amp_hi - amp_lo) u, plus (back_wall >= 0) amplitude 1 at every
 *   voxel of depth index back_wall.  Draw: scatterer j takes voxel index
 *   floor(next() N / 2^64) of the N = ny nx max_depth allowed ones (y, then x,
 *   then depth; redrawn while it repeats an earlier index), then the n_scat
 *   amplitudes with u = (next() >> 11) 2^-53.  n_scat <= 4096.
 * ufss_synth_measure: y (DEVICE complex64 [ny][nx][m]) = A x + n with
 *   n_i ~ CN(0, s^2), s^2 = ||A x||^2 / (ny nx m 10^(snr_db/10)) (||A x||^2 in
 *   FP64 on the device, no host round trip); value i reads outputs 2i + 1 and
 *   2i + 2: u1 = ((out >> 11) + 1) 2^-53, u2 = (out >> 11) 2^-53,
 *   n_i = s sqrt(-log u1) (cos 2 pi u2 + j sin 2 pi u2) (FP64).  snr_db = +inf:
 *   no noise.  Both are asynchronous on `stream`. */
int ufss_synth_scene(const ufss_geom* g, int32_t n_scat, double amp_lo, double amp_hi,
                     int32_t max_depth, int32_t back_wall, uint64_t seed, void* x,
                     ufss_stream_t stream);
int ufss_synth_measure(ufss_plan_t plan, const void* x, double snr_db, uint64_t seed, void* y,
                       ufss_stream_t stream);

/* Persistent batch (paper Alg. 1 on every scan of an uneven batch): the same
 * grouped launches as ufss_fista_batched, with the start state (gamma = x,
 * ||gamma||_1) and `iters` iterations captured ONCE into a hipGraph at
 * creation; every ufss_batch_run replays that graph on `stream` (no capture,
 * no host round trip inside the iterations) from the current contents of the
 * xs buffers (a_0) with the current contents of the ys buffers.  The batch
 * keeps the buffer pointers given at creation; the caller keeps them alive
 * and may overwrite their contents between runs (new scans of the same
 * shapes).  While a batch exists its plans are held: ufss_plan_destroy,
 * ufss_plan_set_tiling, ufss_autotune and ufss_plan_set_phasor_tables on
 * them fail with UFSS_ERR_INVALID_ARG, and a plan can be held by one batch.
 * Arguments as ufss_fista_batched; lambdas with the mu rule are resolved from
 * the ys contents at creation and again by ufss_batch_set_lambdas (they are
 * read from device memory at run time, so no new capture is needed).
 * create: synchronises `stream`; out HOST. */
typedef struct ufss_batch_s* ufss_batch_t;
int ufss_batch_create(int32_t n, const ufss_plan_t* plans, const void* const* ys,
                      void* const* xs, const double* lambdas, const double* Ls,
                      int32_t iters, ufss_stream_t stream, ufss_batch_t* out);
/* Replays the captured iterations; res_out / lambdas_out HOST double [n] or
 * NULL (final ||A gamma - y|| and the lambda used, per scan).  Synchronises
 * `stream`; UFSS_ERR_DIVERGED if any scan diverges. */
int ufss_batch_run(ufss_batch_t batch, double* res_out, double* lambdas_out, ufss_stream_t stream);
/* New lambdas (HOST double [n], same convention as at creation). */
int ufss_batch_set_lambdas(ufss_batch_t batch, const double* lambdas, ufss_stream_t stream);
int ufss_batch_destroy(ufss_batch_t batch);

/* Autotuner for the GEMM path: times candidate tilings (d_y and depth splits,
 * waves per workgroup, sub-tiles per wave, BF16 wave rows, then the smaller
 * FP32 staged chunk at the best of those; see ufss_plan_set_tiling) of the
 * forward and adjoint GEMMs of this plan's shape with HIP events, keeps the
 * fastest in the plan and, with flags bit 1, appends it to the JSON cache file
 * `cache_path` (keyed by the shape class); with flags bit 0 a cached entry is
 * used without timing; flags bit 2 restricts the search to d_y splits and two
 * depth splits at the default tile shape (about 9x fewer trials).  Overwrites
 * the plan's internal workspace; no effect for phasor and transform plans.  Synchronises
 * `stream`.
 *   fwd_split_out, adj_split_out  HOST, optional */
int ufss_autotune(ufss_plan_t plan, const char* cache_path, int32_t flags,
                  int32_t* fwd_split_out, int32_t* adj_split_out, ufss_stream_t stream);

/* Tiling of the GEMM path (what ufss_autotune chooses by timing).  In
 * ufss_plan_set_tiling a field of 0 keeps the plan's current value.
 *   fwd_split   parts of the forward GEMM's d_y range, 1..64
 *   adj_split   parts of the adjoint GEMM's d_y range, 1..64
 *   fwd_waves   FP32 forward: 16-bin sub-tiles (waves) per workgroup, 1..8
 *   fwd_zsplit  forward: parts of the depth range, 1..64 (FP32 and BF16)
 *   fwd_tile, adj_tile    FP32: 16-position sub-tiles per wave, 2 or 4;
 *               BF16 (adj_tile only): 16-depth sub-tiles per adjoint wave, 2
 *               or 4 (2: half-height depth tiles, twice the workgroups)
 *   fwd_rows, adj_rows    BF16: rows of waves in a tile, 1 or 2 (2: half as
 *               wide and twice as tall; C-scans only)
 *   fwd_chunk, adj_chunk  FP32: depths (forward) or bins (adjoint) staged in
 *               LDS per step, 16 or 8 (8 halves the halo and admits more
 *               workgroups per CU; shrunk further if the window needs it)
 *   adj_waves   FP32 adjoint with 2 sub-tiles per wave: waves (16 depths
 *               each) per workgroup, 4 or 8 (8: one staged halo serves 128
 *               depths, so more waves fit a CU's LDS; the bin chunk shrinks
 *               if the twice longer delay rows need it); with 4 sub-tiles
 *               per wave the adjoint runs 4 waves whatever this says
 * Any valid setting computes the same operator; parts that receive no rows
 * contribute zeros.  BF16 plans ignore the FP32-only fields; FP32 plans
 * ignore the rows.  Reallocates the plan's
 * split workspace (synchronises the device).  Errors: INVALID_ARG for values
 * out of range or NULL, UNSUPPORTED for phasor plans or a BF16 tile shape that
 * does not fit in LDS. */
typedef struct ufss_tiling {
    int32_t fwd_split, adj_split;
    int32_t fwd_waves, fwd_zsplit;
    int32_t fwd_tile, adj_tile;
    int32_t fwd_rows, adj_rows;
    int32_t fwd_chunk, adj_chunk;
    int32_t adj_waves;
} ufss_tiling;
int ufss_plan_set_tiling(ufss_plan_t plan, const ufss_tiling* tiling);

/* BF16 GEMM plans: the BF16 phasors exp(-j 2 pi k tau f_s / N_t) of every
 * (|d_y|, |d_x|, z, selected bin) (paper Sec. IV-B: the operator depends on the
 * lateral offset only through |d|) are kept in two precomputed HBM tables, one
 * per kernel layout, when they fit in 4 GiB together (the default at plan
 * creation); otherwise the kernels generate them.  enable = 0 frees the tables
 * (phasors generated), 1 builds them (if they fit).  Both settings compute the
 * same values up to BF16 rounding of the generation's angle-addition steps.
 *   active_out  HOST, optional: 1 if the tables are in use afterwards
 * Synchronises the device.  Errors: UNSUPPORTED for other plans. */
int ufss_plan_set_phasor_tables(ufss_plan_t plan, int32_t enable, int32_t* active_out);

/* ---- learned unrolled solver ---------------------------------------------
 * An S-stage unrolling of FISTA (paper Alg. 1) with learned step sizes and
 * thresholds and a 3x3x3 convolutional correction (2 -> channels -> 2 real
 * channels = Re/Im, ReLU, zero padding); the plan's A / A^H are fixed layers.
 * Stage i: gamma = x_i + beta_i (x_i - x_{i-1}) (FISTA momentum, beta_0 =
 * beta_1 = 0); z = gamma - exp(rho_i)/L A^H(A gamma - y); u = soft(z,
 * exp(kappa_i) lam / L) with lam = mu max|A^H y|; x_{i+1} = u +
 * c conv2(relu(conv1(u / c))) with c = lam / L, so the correction scales with
 * the data (the network is positively homogeneous in y).
 * Parameters per stage, flat FP32: rho, kappa, W1[ch][2][27], b1[ch],
 * W2[2][ch][27], b2[2] (offset e = 9(e_y+1) + 3(e_x+1) + e_z+1 over
 * [ny][nx][nz]).  Initial rho = kappa = 0, W2 = b2 = 0, so the untrained
 * network is exactly S FISTA iterations.  The network keeps a reference to the
 * plan (destroy the network first) and owns its activations and Adam state. */
typedef struct ufss_net_s* ufss_net_t;

/* Create a network on `plan` (stages >= 1, 1 <= channels <= 8, L > 0, mu > 0).
 * W1 ~ N(0, 0.01) from SplitMix64 keyed by `seed`.  out: HOST handle. */
int ufss_unrolled_create(ufss_plan_t plan, int32_t stages, int32_t channels, double L,
                         double mu, uint64_t seed, ufss_net_t* out);
int ufss_unrolled_destroy(ufss_net_t net);

/* Get (get_out HOST float[count] or NULL) and/or set (set_in HOST or NULL) the
 * flat parameters; count_out HOST (optional) receives their number. */
int ufss_unrolled_params(ufss_net_t net, float* get_out, const float* set_in, int64_t* count_out);

/* Inference: x = x_S for measurements y (DEVICE complex64).  Asynchronous. */
int ufss_unrolled_forward(ufss_net_t net, const void* y, void* x, ufss_stream_t stream);

/* Loss ||x_S - target||^2 / ||target||^2 and its gradient w.r.t. every
 * parameter (accumulate != 0 adds to the stored gradient).  grads_out HOST
 * float[count] or NULL.  Synchronises `stream`. */
int ufss_unrolled_grad(ufss_net_t net, const void* y, const void* target, int32_t accumulate,
                       double* loss_out, float* grads_out, ufss_stream_t stream);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean gradient of
 * `batch` samples (ys[b], targets[b] DEVICE).  loss_out HOST: mean loss before
 * the step.  Synchronises `stream`. */
int ufss_unrolled_train_step(ufss_net_t net, int32_t batch, const void* const* ys,
                             const void* const* targets, double lr, double* loss_out,
                             ufss_stream_t stream);

/* Checkpoint (parameters, Adam moments and step, L, mu) to / from a file. */
int ufss_unrolled_save(ufss_net_t net, const char* path);
int ufss_unrolled_load(ufss_net_t net, const char* path);

/* Kernel timing mode.  While enabled, every forward / adjoint core kernel
 * launch of this plan (the windowed GEMM, the phasor kernel or the transform
 * path's contraction, without the gather, scatter, mixing, lateral transform
 * and split-sum passes) is bracketed by two HIP events
 * recorded on its launch stream; enabling clears earlier records, at most 4096
 * launches per direction are kept.  Not for use under graph capture.
 * ufss_plan_kernel_times synchronises on the recorded events and returns the
 * average duration (ms) and the number of timed launches per direction
 * (0 where none); all outputs HOST, optional. */
int ufss_plan_kernel_timing(ufss_plan_t plan, int32_t enable);
int ufss_plan_kernel_times(ufss_plan_t plan, double* fwd_ms, double* adj_ms, int32_t* fwd_n,
                           int32_t* adj_n);

/* Diagnostic: average duration (ms) of the operator's core kernel, launched
 * `reps` times back to back between two HIP events recorded on `stream`.
 * which = 0: forward core (windowed GEMM, phasor forward, or the transform
 * path's contraction), 1: adjoint core (the GEMM kernel alone: its split-K
 * partials are not summed; the transform path's adjoint contraction).
 * The kernel reads the plan's own workspace (its last operands), so call it
 * after at least one ufss_forward / ufss_adjoint.  Synchronises `stream`.
 *   ms_out HOST double */
int ufss_time_kernel(ufss_plan_t plan, int32_t which, int32_t reps, double* ms_out,
                     ufss_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* UFSS_H */
