// Operator drivers, solvers and the C ABI entry points of libufss.
//
// FISTA (paper Alg. 1, Sec. IV-A) with step 1/L, threshold lambda/L and
// Beck-Teboulle momentum; lambda rule of Sec. VII; Lipschitz constant by power
// iteration on A^H A with FP64 norms (Sec. IV-C, iterative approximation).
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ufss {

Plan* plan_create(const ufss_geom* g, int m, int per_position, const int32_t* bins,
                  const MixSpec* mix = nullptr);
void plan_destroy(Plan* P);
void plan_info(const Plan* P, ufss_plan_info* info);
void select_freqs(const ufss_geom* g, int m, int per_position, uint64_t seed, int32_t* out,
                  int32_t* band_size);
void sample_bins(const ufss_geom* g, int m, int strategy, uint64_t seed, int32_t* out,
                 int32_t* per_position_out);
void sigma_estimate(const ufss_geom* g, int m, int per_position, const int32_t* bins,
                    ufss_sigma_est* out);
void crb(const ufss_geom* g, int m, int per_position, int trials, const int32_t* bins,
         const ufss_crb_point* pt, double* fim_out, double* crb_out, hipStream_t s);
void crb_mixed(const ufss_geom* g, int m, int per_position, int trials, const int32_t* bins,
               int per_position_signs, const int8_t* signs, const ufss_crb_point* pt,
               double* fim_out, double* crb_out, hipStream_t s);
const char* last_error();
int phasor_forward_blocks(const Plan& P);
int fista_batched(int n, Plan* const* plans, const cf32* const* ys, cf32* const* xs,
                  const double* lambdas, const double* Ls, int iters, hipStream_t stream,
                  double* res_out);
void synth_scene(const ufss_geom* g, int n, double lo, double hi, int max_depth, int back_wall,
                 uint64_t seed, cf32* x, hipStream_t s);
void synth_measure(Plan& P, const cf32* x, double snr_db, uint64_t seed, cf32* y, hipStream_t s);
struct BatchRun;
BatchRun* batch_create(int n, Plan* const* plans, const cf32* const* ys, cf32* const* xs,
                       const double* lambdas, const double* Ls, int iters, hipStream_t stream);
void batch_set_lambdas(BatchRun& R, const double* lambdas, hipStream_t stream);
void batch_run(BatchRun& R, double* res_out, double* lambdas_out, hipStream_t stream);
void batch_destroy(BatchRun* R);
int autotune(Plan& P, const char* cache_path, int flags, hipStream_t s, int32_t* fs_out,
             int32_t* as_out);
struct Net;
Net* net_create(Plan* P, int S, int ch, double L, double mu, uint64_t seed);
void net_destroy(Net* N);
void net_forward_out(Net& N, const cf32* y, cf32* x, hipStream_t s);
double net_grad(Net& N, const cf32* y, const cf32* aref, int accumulate, hipStream_t s);
double net_train_step(Net& N, int batch, const cf32* const* ys, const cf32* const* refs, double lr,
                      hipStream_t s);
void net_params(Net& N, float* get, const float* set, int64_t* count);
void net_grads(Net& N, float* get);
void net_save(Net& N, const char* path);
void net_load(Net& N, const char* path);

// y = A x (ymeas == NULL) or y = A x - ymeas.  If res2_out != NULL it receives
// ||y||^2 (FP64, device scalar).
// Kernel timing mode: an event pair around one core kernel launch.
static constexpr int kMaxTimed = 4096;        // pairs kept per direction
static void ktime_begin(Plan& P, int w, hipStream_t s) {
    if (!P.ktime || P.kev_used[w] >= kMaxTimed) return;
    auto& ev = P.kev[w];
    while ((int)ev.size() < 2 * (P.kev_used[w] + 1)) {
        hipEvent_t e;
        UFSS_HIP(hipEventCreate(&e));
        ev.push_back(e);
    }
    UFSS_HIP(hipEventRecord(ev[2 * P.kev_used[w]], s));
}
static void ktime_end(Plan& P, int w, hipStream_t s) {
    if (!P.ktime || P.kev_used[w] >= kMaxTimed) return;
    UFSS_HIP(hipEventRecord(P.kev[w][2 * P.kev_used[w] + 1], s));
    ++P.kev_used[w];
}

int op_forward_partials(Plan& P, const cf32* x, cf32* y, const cf32* ymeas, double* part,
                        hipStream_t s) {
    if (P.algo == UFSS_ALGO_PHASOR) {
        ktime_begin(P, 0, s);
        launch_forward_phasor(P, x, y, ymeas, part, s);
        ktime_end(P, 0, s);
        return phasor_forward_blocks(P);
    }
    if (P.algo == UFSS_ALGO_FFT) {
        fft_fwd_transform(P, x, s);
        ktime_begin(P, 0, s);
        fft_fwd_contract(P, s);
        ktime_end(P, 0, s);
        fft_fwd_inverse(P, s);
    } else if (P.dtype == UFSS_BF16) {
        launch_to_bf16(x, P.d_xop, P.nvox, s);
        ktime_begin(P, 0, s);
        launch_forward_gemm_bf16(P, s);
        ktime_end(P, 0, s);
    } else {
        ktime_begin(P, 0, s);
        launch_forward_gemm(P, x, s);
        ktime_end(P, 0, s);
    }
    return P.mix ? launch_mix_post(P, y, ymeas, part, s) : launch_forward_post(P, y, ymeas, part, s);
}

void op_forward(Plan& P, const cf32* x, cf32* y, const cf32* ymeas, double* res2_out,
                hipStream_t s) {
    const int nb = op_forward_partials(P, x, y, ymeas, P.d_part, s);
    if (res2_out) launch_reduce(P.d_part, nb, 1, res2_out, s);
}

int op_adjoint(Plan& P, const cf32* y, cf32* x, hipStream_t s, bool defer_sum) {
    if (P.mix)
        launch_mix_pre(P, y, s);
    else
        launch_adjoint_pre(P, y, s);
    if (P.algo == UFSS_ALGO_FFT) {
        fft_adj_transform(P, s);
        ktime_begin(P, 1, s);
        fft_adj_contract(P, s);
        ktime_end(P, 1, s);
        fft_adj_inverse(P, x, s);
        return 1;
    }
    ktime_begin(P, 1, s);
    if (P.algo == UFSS_ALGO_PHASOR) {
        launch_adjoint_phasor(P, x, s);
        ktime_end(P, 1, s);
        return 1;
    }
    if (P.dtype == UFSS_BF16)
        launch_adjoint_gemm_bf16(P, x, s, false);
    else
        launch_adjoint_gemm(P, x, s, false);
    ktime_end(P, 1, s);
    if (P.adj_split > 1 && !defer_sum) launch_sum_parts(P.d_gpart, P.adj_split, P.nvox, x, s);
    return (defer_sum && P.adj_split > 1) ? P.adj_split : 1;
}

static void sync(hipStream_t s) { UFSS_HIP(hipStreamSynchronize(s)); }

static double read_scalar(const double* d, hipStream_t s) {
    double h = 0.0;
    UFSS_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
    sync(s);
    return h;
}

static uint64_t sm_next(uint64_t& st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double lipschitz(Plan& P, int max_iters, double rtol, double margin, uint64_t seed, hipStream_t s) {
    if (max_iters < 1) fail(UFSS_ERR_INVALID_ARG, "max_iters must be >= 1");
    if (!(rtol >= 0) || !(margin >= 0)) fail(UFSS_ERR_INVALID_ARG, "rtol and margin must be >= 0");
    // CN(0, I) start vector by Box-Muller on SplitMix64 uniforms
    std::vector<cf32> v0(P.nvox);
    uint64_t st = seed;
    for (int64_t i = 0; i < P.nvox; ++i) {
        double u1 = ((sm_next(st) >> 11) + 1.0) * 0x1.0p-53;
        double u2 = (sm_next(st) >> 11) * 0x1.0p-53;
        double rad = std::sqrt(-std::log(u1));
        v0[i] = cf32{(float)(rad * std::cos(2 * M_PI * u2)), (float)(rad * std::sin(2 * M_PI * u2))};
    }
    UFSS_HIP(hipMemcpyAsync(P.d_v, v0.data(), P.nvox * sizeof(cf32), hipMemcpyHostToDevice, s));
    double* nrm = P.d_scalars + 32;
    int nb = launch_norm2(P.nvox, P.d_v, P.d_part, s);
    launch_reduce(P.d_part, nb, 2, nrm, s);
    launch_scale(P.nvox, P.d_v, nrm, s);
    // Iterations run in blocks of 8 without a host round trip; the quotients
    // of a block are then read and tested in order, and the first one that
    // meets the test is the result (the extra iterations of the block only
    // move the internal vector).
    constexpr int kBlock = 8;
    double* rho_dev = P.d_scalars + 48;                 // [kBlock]
    double rho = 0.0, rho_old = 0.0;
    bool done = false;
    for (int it0 = 1; it0 <= max_iters && !done; it0 += kBlock) {
        const int nit = std::min(kBlock, max_iters - it0 + 1);
        for (int j = 0; j < nit; ++j) {
            op_forward(P, P.d_v, P.d_r, nullptr, rho_dev + j, s);      // rho = ||A v||^2
            op_adjoint(P, P.d_r, P.d_g, s);
            nb = launch_norm2(P.nvox, P.d_g, P.d_part, s);
            launch_reduce(P.d_part, nb, 2, nrm, s);
            launch_copy(P.nvox, P.d_g, P.d_v, s);
            launch_scale(P.nvox, P.d_v, nrm, s);
        }
        double h[kBlock];
        UFSS_HIP(hipMemcpyAsync(h, rho_dev, nit * sizeof(double), hipMemcpyDeviceToHost, s));
        sync(s);
        for (int j = 0; j < nit; ++j) {
            rho = h[j];
            if (!std::isfinite(rho)) fail(UFSS_ERR_DIVERGED, "non-finite Rayleigh quotient");
            if (rho_old > 0 && std::fabs(rho - rho_old) <= rtol * rho) {
                done = true;
                break;
            }
            rho_old = rho;
        }
    }
    P.lipschitz = (1.0 + margin) * rho;
    return P.lipschitz;
}

static double absmax_dev(int64_t n, const cf32* x, double* part, double* out, hipStream_t s) {
    int nb = launch_absmax(n, x, part, s);
    launch_reduce_max(part, nb, out, s);
    return read_scalar(out, s);
}

int fista(Plan& P, const cf32* y, double lambda, double L, int iters, double tol, int flags,
          cf32* x, const cf32* aref, ufss_fista_stats* stats, ufss_fista_state* state,
          hipStream_t s) {
    if (!y || !x) fail(UFSS_ERR_INVALID_ARG, "y and x must be device pointers");
    if (flags & ~3) fail(UFSS_ERR_INVALID_ARG, "unknown FISTA flag bits");
    const int accel = flags & 1, real = (flags >> 1) & 1;
    if (iters < 0) fail(UFSS_ERR_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0)) fail(UFSS_ERR_INVALID_ARG, "tol must be >= 0");
    if (!(L > 0)) L = P.lipschitz;
    if (!(L > 0)) fail(UFSS_ERR_INVALID_ARG, "no Lipschitz constant given or cached");
    if (lambda == 0 || std::isnan(lambda)) fail(UFSS_ERR_INVALID_ARG, "lambda must be non-zero");
    if (lambda < 0) {
        op_adjoint(P, y, P.d_g, s);
        lambda = -lambda * absmax_dev(P.nvox, P.d_g, P.d_part, P.d_scalars + 40, s);
    }
    cf32* gamma = (state && state->gamma) ? static_cast<cf32*>(state->gamma) : P.d_gamma;
    const int k0 = state ? state->k_done : 0;
    if (k0 < 0) fail(UFSS_ERR_INVALID_ARG, "state->k_done must be >= 0");
    if (k0 > 0 && !(state && state->gamma))
        fail(UFSS_ERR_INVALID_ARG, "resuming needs state->gamma");
    if (k0 == 0) launch_copy(P.nvox, x, gamma, s);
    double tk = 1.0;
    for (int i = 0; i < k0; ++i) tk = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tk * tk));
    double ref2 = 0.0;
    if (aref) {
        int nb = launch_norm2(P.nvox, aref, P.d_part, s);
        launch_reduce(P.d_part, nb, 2, P.d_scalars + 44, s);
        ref2 = read_scalar(P.d_scalars + 44, s);
        if (!(ref2 > 0)) fail(UFSS_ERR_INVALID_ARG, "a_ref is zero");
    }
    if (P.stats_cap < iters) {
        if (P.d_stats) UFSS_HIP(hipFree(P.d_stats));
        P.d_stats = nullptr;
        P.stats_cap = 0;
        UFSS_HIP(hipMalloc(&P.d_stats, (size_t)std::max(iters, 1) * 4 * sizeof(double)));
        P.stats_cap = std::max(iters, 1);
    }
    // ||gamma_k0||_1 for the first objective value
    double* g1 = P.d_scalars + 16;
    {
        int nb = launch_norm2(P.nvox, gamma, P.d_part, s);
        double* tmp = P.d_scalars + 20;
        launch_reduce(P.d_part, nb, 2, tmp, s);
        UFSS_HIP(hipMemcpyAsync(g1, tmp + 1, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    const float step = (float)(1.0 / L), thresh = (float)(lambda / L);
    int done = 0;
    for (int k = 0; k < iters; ++k) {
        // the residual's partials wait in their own buffer for the statistics kernel
        const int nbr = op_forward_partials(P, gamma, P.d_r, y, P.d_part_res, s);
        // the adjoint's split-K partials are summed inside the update (its epilogue)
        const int ns = op_adjoint(P, P.d_r, P.d_g, s, true);
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tk * tk));
        const double beta = accel ? (tk - 1.0) / tn : 0.0;
        int nb = launch_update(P.nvox, gamma, ns > 1 ? P.d_gpart : P.d_g, ns, x, step, thresh,
                               (float)beta, aref, P.d_part, s, real);
        launch_reduce_fista_stats(P.d_part_res, nbr, P.d_scalars + 0, P.d_part, nb, P.d_scalars + 8,
                                  P.d_stats, k, g1, lambda, aref ? 1 : 0, ref2, s);
        tk = tn;
        done = k + 1;
        if (tol > 0 && (done % 8 == 0)) {
            double rc = read_scalar(P.d_stats + 4 * (int64_t)k + 2, s);
            if (rc <= tol) break;
        }
    }
    std::vector<double> h((size_t)std::max(done, 1) * 4);
    if (done > 0)
        UFSS_HIP(hipMemcpyAsync(h.data(), P.d_stats, (size_t)done * 4 * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    sync(s);
    if (state) state->k_done = k0 + done;
    if (stats) {
        stats->iters_done = done;
        stats->lambda = lambda;
        for (int k = 0; k < done; ++k) {
            if (stats->obj) stats->obj[k] = h[4 * k + 0];
            if (stats->res) stats->res[k] = h[4 * k + 1];
            if (stats->rel_change) stats->rel_change[k] = h[4 * k + 2];
            if (stats->err_ref) stats->err_ref[k] = h[4 * k + 3];
        }
    }
    for (int k = 0; k < done; ++k) {
        if (!std::isfinite(h[4 * k + 0]) || !std::isfinite(h[4 * k + 1]) ||
            !std::isfinite(h[4 * k + 2]) || h[4 * k + 1] > 1e6 * h[1] + 1e-300)
            fail(UFSS_ERR_DIVERGED, "FISTA diverged at iteration " + std::to_string(k0 + k) +
                                        " (non-finite or exploding residual); check L");
    }
    return UFSS_OK;
}

// FISTA with backtracking (Sec. IV-C; Beck & Teboulle 2009).  Trial constants
// L = L_{k-1} eta^i are tried at the extrapolated point gamma_k until
//   f(p) <= f(gamma) + Re<p - gamma, grad f(gamma)> + L/2 ||p - gamma||^2 + slack,
// f = 1/2 ||A . - y||^2, slack = eps * 1/2 ||y||^2 with eps = 1e-6 for the FP32
// operator and 2^-8 (one BF16 unit in the last place) for the BF16 operator,
// whose input rounding makes f(p) - f(gamma) noisy at that level: with a
// smaller margin no constant passes once the iterates settle.  A is linear, so the residual at the next extrapolated point
// is (1 + beta) r_k - beta r_{k-1} of the two accepted residuals: an iteration
// costs one adjoint plus one forward per trial (two operator applications when
// the first trial is accepted, as plain FISTA).
static constexpr double kBtSlackF32 = 1e-6;
static constexpr double kBtSlackBF16 = 0.00390625;
static constexpr int kBtMaxTrials = 100;

int fista_backtracking(Plan& P, const cf32* y, double lambda, double L0, double eta, int iters,
                       double tol, cf32* x, const cf32* aref, ufss_fista_stats* stats,
                       double* L_out, int32_t* trials_out, hipStream_t s) {
    if (!y || !x) fail(UFSS_ERR_INVALID_ARG, "y and x must be device pointers");
    if (iters < 0) fail(UFSS_ERR_INVALID_ARG, "iters must be >= 0");
    if (!(tol >= 0)) fail(UFSS_ERR_INVALID_ARG, "tol must be >= 0");
    if (!(L0 > 0) || !std::isfinite(L0)) fail(UFSS_ERR_INVALID_ARG, "L0 must be > 0");
    if (!(eta > 1) || !std::isfinite(eta)) fail(UFSS_ERR_INVALID_ARG, "eta must be > 1");
    if (lambda == 0 || std::isnan(lambda)) fail(UFSS_ERR_INVALID_ARG, "lambda must be non-zero");
    if (lambda < 0) {
        op_adjoint(P, y, P.d_g, s);
        lambda = -lambda * absmax_dev(P.nvox, P.d_g, P.d_part, P.d_scalars + 40, s);
    }
    const int64_t nv = P.nvox, nm = (int64_t)P.npos * P.m;
    if (!P.d_bt) {
        UFSS_HIP(hipMalloc(&P.d_bt, (size_t)(3 * nv + 3 * nm) * sizeof(cf32)));
        UFSS_HIP(hipMalloc(&P.d_bt_scal, 16 * sizeof(double)));
        P.ws_bytes += (3 * nv + 3 * nm) * sizeof(cf32) + 16 * sizeof(double);
    }
    cf32* X[3] = {P.d_bt, P.d_bt + nv, P.d_bt + 2 * nv};
    cf32* R[3] = {P.d_bt + 3 * nv, P.d_bt + 3 * nv + nm, P.d_bt + 3 * nv + 2 * nm};
    int cur = 0, prev = 1, cand = 2;
    double* sc = P.d_bt_scal;   // [0] ||r_p||^2, [1..6] trial sums, [8] ||r_gamma||^2, [10] ||y||^2
    double ref2 = 0.0;
    if (aref) {
        int nb = launch_norm2(nv, aref, P.d_part, s);
        launch_reduce(P.d_part, nb, 2, P.d_scalars + 44, s);
        ref2 = read_scalar(P.d_scalars + 44, s);
        if (!(ref2 > 0)) fail(UFSS_ERR_INVALID_ARG, "a_ref is zero");
    }
    {
        int nb = launch_norm2(nm, y, P.d_part, s);
        launch_reduce(P.d_part, nb, 2, sc + 10, s);
    }
    const double eps = P.dtype == UFSS_BF16 ? kBtSlackBF16 : kBtSlackF32;
    const double slack = eps * 0.5 * read_scalar(sc + 10, s);
    launch_copy(nv, x, X[cur], s);
    launch_copy(nv, x, P.d_gamma, s);
    op_forward(P, X[cur], R[cur], y, sc + 8, s);
    launch_copy(nm, R[cur], P.d_r, s);
    double tk = 1.0, L = L0;
    int done = 0;
    double h[9];
    for (int k = 0; k < iters; ++k) {
        op_adjoint(P, P.d_r, P.d_g, s);
        int trials = 0;
        for (;;) {
            if (++trials > kBtMaxTrials)
                fail(UFSS_ERR_DIVERGED, "backtracking found no step in " +
                                            std::to_string(kBtMaxTrials) + " trials");
            int nb = launch_bt_prox(nv, P.d_gamma, P.d_g, (float)(1.0 / L), (float)(lambda / L),
                                    X[cand], X[cur], aref, P.d_part, s);
            launch_reduce(P.d_part, nb, 6, sc + 1, s);
            op_forward(P, X[cand], R[cand], y, sc + 0, s);
            UFSS_HIP(hipMemcpyAsync(h, sc, 9 * sizeof(double), hipMemcpyDeviceToHost, s));
            sync(s);
            if (!std::isfinite(h[0]) || !std::isfinite(h[8]) || !std::isfinite(h[1]))
                fail(UFSS_ERR_DIVERGED, "non-finite residual at iteration " + std::to_string(k));
            const double model = 0.5 * h[8] + h[1] + 0.5 * L * h[2];
            if (0.5 * h[0] <= model + slack) break;
            L *= eta;
            if (!(L < 1e300)) fail(UFSS_ERR_DIVERGED, "backtracking constant overflowed");
        }
        const double rel = h[5] > 0 ? std::sqrt(h[4] / h[5]) : 0.0;
        if (stats) {
            if (stats->obj) stats->obj[k] = 0.5 * h[0] + lambda * h[3];
            if (stats->res) stats->res[k] = std::sqrt(h[0]);
            if (stats->rel_change) stats->rel_change[k] = rel;
            if (stats->err_ref) stats->err_ref[k] = aref ? std::sqrt(h[6] / ref2) : 0.0;
        }
        if (L_out) L_out[k] = L;
        if (trials_out) trials_out[k] = trials;
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tk * tk));
        const float beta = (float)((tk - 1.0) / tn);
        const int old_prev = prev;
        prev = cur;
        cur = cand;
        cand = old_prev;
        launch_extrap(nv, X[cur], X[prev], beta, P.d_gamma, P.d_part, s);
        int nb = launch_extrap(nm, R[cur], R[prev], beta, P.d_r, P.d_part, s);
        launch_reduce(P.d_part, nb, 1, sc + 8, s);
        tk = tn;
        done = k + 1;
        if (tol > 0 && rel <= tol) break;
    }
    launch_copy(nv, X[cur], x, s);
    sync(s);
    if (stats) {
        stats->iters_done = done;
        stats->lambda = lambda;
    }
    return done;
}

}  // namespace ufss

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
using ufss::Error;
using ufss::Plan;

#define UFSS_GUARD_BEGIN \
    try {                \
        ufss::set_last_error("");
#define UFSS_GUARD_END                                   \
    }                                                    \
    catch (const Error& e) {                             \
        ufss::set_last_error(e.msg);                     \
        return e.code;                                   \
    }                                                    \
    catch (const std::bad_alloc&) {                      \
        ufss::set_last_error("host allocation failed");  \
        return UFSS_ERR_OOM;                             \
    }                                                    \
    catch (...) {                                        \
        ufss::set_last_error("unexpected exception");    \
        return UFSS_ERR_INVALID_ARG;                     \
    }                                                    \
    return UFSS_OK;

static Plan* as_plan(ufss_plan_t p) {
    if (!p) ufss::fail(UFSS_ERR_INVALID_ARG, "plan is NULL");
    return reinterpret_cast<Plan*>(p);
}

// A persistent batch's captured graph holds pointers into the plan's workspace:
// calls that free or reallocate it are refused until the batch is destroyed.
static Plan* as_unpinned_plan(ufss_plan_t p) {
    Plan* P = as_plan(p);
    if (P->batch_refs > 0)
        ufss::fail(UFSS_ERR_INVALID_ARG, "plan is held by a persistent batch (destroy the batch first)");
    return P;
}

extern "C" {

const char* ufss_last_error(void) { return ufss::last_error(); }

int ufss_select_freqs(const ufss_geom* g, int32_t m, int32_t per_position, uint64_t seed,
                      int32_t* bins_out, int32_t* band_size_out) {
    UFSS_GUARD_BEGIN
    ufss::select_freqs(g, m, per_position, seed, bins_out, band_size_out);
    UFSS_GUARD_END
}

int ufss_sample_bins(const ufss_geom* g, int32_t m, int32_t strategy, uint64_t seed,
                     int32_t* bins_out, int32_t* per_position_out) {
    UFSS_GUARD_BEGIN
    ufss::sample_bins(g, m, strategy, seed, bins_out, per_position_out);
    UFSS_GUARD_END
}

int ufss_sigma_estimate(const ufss_geom* g, int32_t m, int32_t per_position,
                        const int32_t* bins, ufss_sigma_est* out) {
    UFSS_GUARD_BEGIN
    ufss::sigma_estimate(g, m, per_position, bins, out);
    UFSS_GUARD_END
}

int ufss_crb(const ufss_geom* g, int32_t m, int32_t per_position, int32_t trials,
             const int32_t* bins, const ufss_crb_point* pt, double* fim_out, double* crb_out,
             ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::crb(g, m, per_position, trials, bins, pt, fim_out, crb_out,
              static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_crb_mixed(const ufss_geom* g, int32_t m, int32_t per_position, int32_t trials,
                   const int32_t* bins, int32_t per_position_signs, const int8_t* signs,
                   const ufss_crb_point* pt, double* fim_out, double* crb_out,
                   ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::crb_mixed(g, m, per_position, trials, bins, per_position_signs, signs, pt, fim_out,
                    crb_out, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_plan_create(const ufss_geom* g, int32_t m, int32_t per_position, const int32_t* bins,
                     ufss_plan_t* out) {
    UFSS_GUARD_BEGIN
    if (!out) ufss::fail(UFSS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    *out = reinterpret_cast<ufss_plan_t>(ufss::plan_create(g, m, per_position, bins));
    UFSS_GUARD_END
}

int ufss_plan_create_mixed(const ufss_geom* g, int32_t m, int32_t per_position, const int32_t* bins,
                           int32_t per_position_signs, const int8_t* signs, ufss_plan_t* out) {
    UFSS_GUARD_BEGIN
    if (!out) ufss::fail(UFSS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    ufss::MixSpec mix;
    mix.per_sign = per_position_signs ? 1 : 0;
    mix.signs = signs;
    *out = reinterpret_cast<ufss_plan_t>(ufss::plan_create(g, m, per_position, bins, &mix));
    UFSS_GUARD_END
}

int ufss_plan_destroy(ufss_plan_t plan) {
    UFSS_GUARD_BEGIN
    ufss::plan_destroy(as_unpinned_plan(plan));
    UFSS_GUARD_END
}

int ufss_plan_info_get(ufss_plan_t plan, ufss_plan_info* info) {
    UFSS_GUARD_BEGIN
    ufss::plan_info(as_plan(plan), info);
    UFSS_GUARD_END
}

int ufss_forward(ufss_plan_t plan, const void* x, void* y, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    if (!x || !y) ufss::fail(UFSS_ERR_INVALID_ARG, "x and y must be device pointers");
    Plan* P = as_plan(plan);
    ufss::op_forward(*P, static_cast<const ufss::cf32*>(x), static_cast<ufss::cf32*>(y), nullptr,
                     nullptr, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_adjoint(ufss_plan_t plan, const void* y, void* x, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    if (!x || !y) ufss::fail(UFSS_ERR_INVALID_ARG, "x and y must be device pointers");
    Plan* P = as_plan(plan);
    ufss::op_adjoint(*P, static_cast<const ufss::cf32*>(y), static_cast<ufss::cf32*>(x),
                     static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_lipschitz(ufss_plan_t plan, int32_t max_iters, double rtol, double margin, uint64_t seed,
                   double* L_out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    double L = ufss::lipschitz(*P, max_iters, rtol, margin, seed, static_cast<hipStream_t>(stream));
    if (L_out) *L_out = L;
    UFSS_GUARD_END
}

int ufss_fista(ufss_plan_t plan, const void* y, double lambda, double L, int32_t iters,
               double tol, int32_t accel, void* x, const void* a_ref, ufss_fista_stats* stats,
               ufss_fista_state* state, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    return ufss::fista(*P, static_cast<const ufss::cf32*>(y), lambda, L, iters, tol, accel,
                       static_cast<ufss::cf32*>(x), static_cast<const ufss::cf32*>(a_ref), stats,
                       state, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_fista_backtracking(ufss_plan_t plan, const void* y, double lambda, double L0,
                            double eta, int32_t iters, double tol, void* x, const void* a_ref,
                            ufss_fista_stats* stats, double* L_out, int32_t* trials_out,
                            ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    ufss::fista_backtracking(*P, static_cast<const ufss::cf32*>(y), lambda, L0, eta, iters, tol,
                             static_cast<ufss::cf32*>(x), static_cast<const ufss::cf32*>(a_ref),
                             stats, L_out, trials_out, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_shrink_update(int64_t n, void* gamma, const void* g, void* a, double step, double thresh,
                       double beta, const void* a_ref, double* norms_out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    if (n < 0 || (n > 0 && (!gamma || !g || !a)))
        ufss::fail(UFSS_ERR_INVALID_ARG, "bad size or NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = nullptr;
    double* out = nullptr;
    UFSS_HIP(hipMalloc(&part, (size_t)ufss::max_blocks_vec() * 5 * sizeof(double) + 64));
    UFSS_HIP(hipMalloc(&out, 8 * sizeof(double)));
    try {
        int nb = ufss::launch_update(n, static_cast<ufss::cf32*>(gamma),
                                     static_cast<const ufss::cf32*>(g), 1, static_cast<ufss::cf32*>(a),
                                     (float)step, (float)thresh, (float)beta,
                                     static_cast<const ufss::cf32*>(a_ref), part, s);
        ufss::launch_reduce(part, nb, 5, out, s);
        if (norms_out) {
            UFSS_HIP(hipMemcpyAsync(norms_out, out, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        UFSS_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipFree(part);
        (void)hipFree(out);
        throw;
    }
    UFSS_HIP(hipFree(part));
    UFSS_HIP(hipFree(out));
    UFSS_GUARD_END
}

int ufss_fista_batched(int32_t n, const ufss_plan_t* plans, const void* const* ys, void* const* xs,
                       const double* lambdas, const double* Ls, int32_t iters, double* res_out,
                       ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    if (n < 1 || !plans || !ys || !xs) ufss::fail(UFSS_ERR_INVALID_ARG, "bad batch arrays");
    std::vector<Plan*> ps(n);
    for (int i = 0; i < n; ++i) ps[i] = as_plan(plans[i]);
    return ufss::fista_batched(n, ps.data(), reinterpret_cast<const ufss::cf32* const*>(ys),
                               reinterpret_cast<ufss::cf32* const*>(xs), lambdas, Ls, iters,
                               static_cast<hipStream_t>(stream), res_out);
    UFSS_GUARD_END
}

int ufss_synth_scene(const ufss_geom* g, int32_t n_scat, double amp_lo, double amp_hi,
                     int32_t max_depth, int32_t back_wall, uint64_t seed, void* x,
                     ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::synth_scene(g, n_scat, amp_lo, amp_hi, max_depth, back_wall, seed,
                      static_cast<ufss::cf32*>(x), static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_synth_measure(ufss_plan_t plan, const void* x, double snr_db, uint64_t seed, void* y,
                       ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::synth_measure(*as_plan(plan), static_cast<const ufss::cf32*>(x), snr_db, seed,
                        static_cast<ufss::cf32*>(y), static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

static ufss::BatchRun* as_batch(ufss_batch_t b) {
    if (!b) ufss::fail(UFSS_ERR_INVALID_ARG, "batch is NULL");
    return reinterpret_cast<ufss::BatchRun*>(b);
}

int ufss_batch_create(int32_t n, const ufss_plan_t* plans, const void* const* ys, void* const* xs,
                      const double* lambdas, const double* Ls, int32_t iters, ufss_stream_t stream,
                      ufss_batch_t* out) {
    UFSS_GUARD_BEGIN
    if (!out) ufss::fail(UFSS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !plans || !ys || !xs) ufss::fail(UFSS_ERR_INVALID_ARG, "bad batch arrays");
    std::vector<Plan*> ps(n);
    for (int i = 0; i < n; ++i) ps[i] = as_plan(plans[i]);
    *out = reinterpret_cast<ufss_batch_t>(ufss::batch_create(
        n, ps.data(), reinterpret_cast<const ufss::cf32* const*>(ys),
        reinterpret_cast<ufss::cf32* const*>(xs), lambdas, Ls, iters, static_cast<hipStream_t>(stream)));
    UFSS_GUARD_END
}

int ufss_batch_run(ufss_batch_t batch, double* res_out, double* lambdas_out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::batch_run(*as_batch(batch), res_out, lambdas_out, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_batch_set_lambdas(ufss_batch_t batch, const double* lambdas, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::batch_set_lambdas(*as_batch(batch), lambdas, static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_batch_destroy(ufss_batch_t batch) {
    UFSS_GUARD_BEGIN
    ufss::batch_destroy(as_batch(batch));
    UFSS_GUARD_END
}

int ufss_autotune(ufss_plan_t plan, const char* cache_path, int32_t flags, int32_t* fwd_split_out,
                  int32_t* adj_split_out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    Plan* P = as_unpinned_plan(plan);
    ufss::autotune(*P, cache_path, flags, static_cast<hipStream_t>(stream), fwd_split_out,
                   adj_split_out);
    UFSS_GUARD_END
}

int ufss_plan_set_tiling(ufss_plan_t plan, const ufss_tiling* t) {
    UFSS_GUARD_BEGIN
    Plan* P = as_unpinned_plan(plan);
    if (!t) ufss::fail(UFSS_ERR_INVALID_ARG, "tiling is NULL");
    if (P->algo != UFSS_ALGO_GEMM) ufss::fail(UFSS_ERR_UNSUPPORTED, "tiling applies to GEMM plans only");
    auto in = [](int v, int hi) { return v >= 0 && v <= hi; };
    auto one_of = [](int v, int a, int b) { return v == 0 || v == a || v == b; };
    if (!in(t->fwd_split, 64) || !in(t->adj_split, 64) || !in(t->fwd_waves, 8) || !in(t->fwd_zsplit, 64) ||
        !one_of(t->fwd_tile, 2, 4) || !one_of(t->adj_tile, 2, 4) || !in(t->fwd_rows, 2) ||
        !in(t->adj_rows, 2) || !one_of(t->fwd_chunk, 8, 16) || !one_of(t->adj_chunk, 8, 16) ||
        !one_of(t->adj_waves, 4, 8))
        ufss::fail(UFSS_ERR_INVALID_ARG, "tiling value out of range");
    if (P->dtype == UFSS_F32) {
        if (t->fwd_waves > 0) P->fwd_nw = t->fwd_waves;
        if (t->fwd_tile > 0) P->fwd_np = t->fwd_tile;
        if (t->adj_tile > 0) P->adj_np = t->adj_tile;
        if (t->fwd_chunk > 0) P->fwd_zc = t->fwd_chunk;
        if (t->adj_chunk > 0) P->adj_kc = t->adj_chunk;
        if (t->adj_waves > 0) P->adj_nw = t->adj_waves;
    } else {
        if (t->adj_tile > 0) P->bf_adj_nz = t->adj_tile;
    }
    if (P->dtype == UFSS_BF16 && (t->fwd_rows > 0 || t->adj_rows > 0)) {
        const int fr = t->fwd_rows > 0 ? t->fwd_rows : P->bf_fwd_rows;
        const int ar = t->adj_rows > 0 ? t->adj_rows : P->bf_adj_rows;
        if (!ufss::bf16_rows_ok(*P, fr, ar))
            ufss::fail(UFSS_ERR_UNSUPPORTED, "this BF16 tile shape does not fit the grid or LDS");
        P->bf_fwd_rows = fr;
        P->bf_adj_rows = ar;
    }
    ufss::plan_set_splits(*P, t->fwd_split > 0 ? t->fwd_split : P->fwd_split,
                          t->adj_split > 0 ? t->adj_split : P->adj_split,
                          t->fwd_zsplit > 0 ? t->fwd_zsplit : P->fwd_zsplit);
    UFSS_GUARD_END
}

int ufss_plan_set_phasor_tables(ufss_plan_t plan, int32_t enable, int32_t* active_out) {
    UFSS_GUARD_BEGIN
    Plan* P = as_unpinned_plan(plan);
    if (P->algo != UFSS_ALGO_GEMM || P->dtype != UFSS_BF16)
        ufss::fail(UFSS_ERR_UNSUPPORTED, "phasor tables apply to BF16 GEMM plans only");
    ufss::bf16_set_tables(*P, enable != 0);
    if (active_out) *active_out = P->d_ptab_f != nullptr;
    UFSS_GUARD_END
}

static ufss::Net* as_net(ufss_net_t n) {
    if (!n) ufss::fail(UFSS_ERR_INVALID_ARG, "net is NULL");
    return reinterpret_cast<ufss::Net*>(n);
}

int ufss_unrolled_create(ufss_plan_t plan, int32_t stages, int32_t channels, double L, double mu,
                         uint64_t seed, ufss_net_t* out) {
    UFSS_GUARD_BEGIN
    if (!out) ufss::fail(UFSS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    *out = reinterpret_cast<ufss_net_t>(ufss::net_create(as_plan(plan), stages, channels, L, mu, seed));
    UFSS_GUARD_END
}

int ufss_unrolled_destroy(ufss_net_t net) {
    UFSS_GUARD_BEGIN
    ufss::net_destroy(as_net(net));
    UFSS_GUARD_END
}

int ufss_unrolled_params(ufss_net_t net, float* get_out, const float* set_in, int64_t* count_out) {
    UFSS_GUARD_BEGIN
    ufss::net_params(*as_net(net), get_out, set_in, count_out);
    UFSS_GUARD_END
}

int ufss_unrolled_forward(ufss_net_t net, const void* y, void* x, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::net_forward_out(*as_net(net), static_cast<const ufss::cf32*>(y), static_cast<ufss::cf32*>(x),
                          static_cast<hipStream_t>(stream));
    UFSS_GUARD_END
}

int ufss_unrolled_grad(ufss_net_t net, const void* y, const void* target, int32_t accumulate,
                       double* loss_out, float* grads_out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    ufss::Net& N = *as_net(net);
    double l = ufss::net_grad(N, static_cast<const ufss::cf32*>(y), static_cast<const ufss::cf32*>(target),
                              accumulate, static_cast<hipStream_t>(stream));
    if (loss_out) *loss_out = l;
    ufss::net_grads(N, grads_out);
    UFSS_GUARD_END
}

int ufss_unrolled_train_step(ufss_net_t net, int32_t batch, const void* const* ys,
                             const void* const* targets, double lr, double* loss_out,
                             ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    double l = ufss::net_train_step(*as_net(net), batch, reinterpret_cast<const ufss::cf32* const*>(ys),
                                    reinterpret_cast<const ufss::cf32* const*>(targets), lr,
                                    static_cast<hipStream_t>(stream));
    if (loss_out) *loss_out = l;
    UFSS_GUARD_END
}

int ufss_unrolled_save(ufss_net_t net, const char* path) {
    UFSS_GUARD_BEGIN
    ufss::net_save(*as_net(net), path);
    UFSS_GUARD_END
}

int ufss_unrolled_load(ufss_net_t net, const char* path) {
    UFSS_GUARD_BEGIN
    ufss::net_load(*as_net(net), path);
    UFSS_GUARD_END
}

int ufss_plan_kernel_timing(ufss_plan_t plan, int32_t enable) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    if (enable) P->kev_used[0] = P->kev_used[1] = 0;
    P->ktime = enable != 0;
    UFSS_GUARD_END
}

int ufss_plan_kernel_times(ufss_plan_t plan, double* fwd_ms, double* adj_ms, int32_t* fwd_n,
                           int32_t* adj_n) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    double avg[2] = {0.0, 0.0};
    for (int w = 0; w < 2; ++w) {
        const int n = P->kev_used[w];
        double tot = 0.0;
        for (int i = 0; i < n; ++i) {
            UFSS_HIP(hipEventSynchronize(P->kev[w][2 * i + 1]));
            float ms = 0.f;
            UFSS_HIP(hipEventElapsedTime(&ms, P->kev[w][2 * i], P->kev[w][2 * i + 1]));
            tot += ms;
        }
        avg[w] = n > 0 ? tot / n : 0.0;
    }
    if (fwd_ms) *fwd_ms = avg[0];
    if (adj_ms) *adj_ms = avg[1];
    if (fwd_n) *fwd_n = P->kev_used[0];
    if (adj_n) *adj_n = P->kev_used[1];
    UFSS_GUARD_END
}

int ufss_time_kernel(ufss_plan_t plan, int32_t which, int32_t reps, double* ms_out,
                     ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    Plan* P = as_plan(plan);
    if (which < 0 || which > 1 || reps < 1 || !ms_out)
        ufss::fail(UFSS_ERR_INVALID_ARG, "which must be 0 or 1, reps >= 1, ms_out non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    UFSS_HIP(hipEventCreate(&e0));
    UFSS_HIP(hipEventCreate(&e1));
    try {
        auto launch = [&]() {
            if (P->algo == UFSS_ALGO_FFT) {    // the contraction (transform inputs as left)
                if (which == 0)
                    ufss::fft_fwd_contract(*P, s);
                else
                    ufss::fft_adj_contract(*P, s);
            } else if (which == 0) {
                if (P->algo == UFSS_ALGO_PHASOR)
                    ufss::launch_forward_phasor(*P, P->d_gamma, P->d_r, nullptr, P->d_part, s);
                else if (P->dtype == UFSS_BF16)
                    ufss::launch_forward_gemm_bf16(*P, s);
                else
                    ufss::launch_forward_gemm(*P, P->d_gamma, s);
            } else {
                if (P->algo == UFSS_ALGO_PHASOR)
                    ufss::launch_adjoint_phasor(*P, P->d_g, s);
                else if (P->dtype == UFSS_BF16)   // the GEMM alone, split partials not summed
                    ufss::launch_adjoint_gemm_bf16(*P, P->d_g, s, false);
                else
                    ufss::launch_adjoint_gemm(*P, P->d_g, s, false);
            }
        };
        launch();   // warm
        UFSS_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) launch();
        UFSS_HIP(hipEventRecord(e1, s));
        UFSS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        UFSS_HIP(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = (double)ms / reps;
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    UFSS_HIP(hipEventDestroy(e0));
    UFSS_HIP(hipEventDestroy(e1));
    UFSS_GUARD_END
}

int ufss_absmax(int64_t n, const void* x, double* out, ufss_stream_t stream) {
    UFSS_GUARD_BEGIN
    if (n < 1 || !x || !out) ufss::fail(UFSS_ERR_INVALID_ARG, "bad size or NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = nullptr;
    UFSS_HIP(hipMalloc(&part, (size_t)(ufss::max_blocks_vec() + 8) * sizeof(double)));
    try {
        *out = ufss::absmax_dev(n, static_cast<const ufss::cf32*>(x), part,
                                part + ufss::max_blocks_vec(), s);
    } catch (...) {
        (void)hipFree(part);
        throw;
    }
    UFSS_HIP(hipFree(part));
    UFSS_GUARD_END
}

}  // extern "C"
