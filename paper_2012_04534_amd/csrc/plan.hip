// Plan construction: derived geometry (FP64, host), bin selection, the
// integer-turn delay table and device workspace.
//
// Paper sources: Sec. II-A (delay tau, grids, frequency-domain A-scan model),
// Sec. III-A (random bin subsets, shared or per A-scan), Sec. IV-B (block
// 2-level Toeplitz structure: A depends on the lateral offset p - v only, so one
// table indexed by (|d_x|, |d_y|, z) serves every position).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace ufss {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    int code = (e == hipErrorOutOfMemory) ? UFSS_ERR_OOM : UFSS_ERR_HIP;
    fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Derived geometry.  Pulse: complex Gabor with -6 dB fractional bandwidth
// frac_bw, so sigma_f = frac_bw f_c / (2 sqrt(2 ln 2)) and sigma_t = 1/(2 pi
// sigma_f); its sampled echo has DFT H_k exp(-j 2 pi f_k (tau - t0)) with H_k as
// in ufss.h.  Band: bins 0..nt/2 whose Gaussian envelope is within band_db of
// the peak.  Window start: centre of the aperture's delay span.
// ---------------------------------------------------------------------------
static double delay(const ufss_geom& g, double ddx, double ddy, double z) {
    return (2.0 / g.c) * std::sqrt(ddx * ddx + ddy * ddy + z * z);
}

Derived derive(const ufss_geom& g) {
    Derived d;
    d.wx = g.win_x < 0 ? g.nx - 1 : std::min(g.win_x, g.nx - 1);
    d.wy = g.win_y < 0 ? g.ny - 1 : std::min(g.win_y, g.ny - 1);
    d.sigma_f = g.frac_bw * g.fc / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    d.sigma_t = 1.0 / (2.0 * M_PI * d.sigma_f);
    if (std::isnan(g.t0)) {
        double tmin = delay(g, 0.0, 0.0, g.z_start);
        double tmax = delay(g, d.wx * g.dx, d.wy * g.dy, g.z_start + (g.nz - 1) * g.dz);
        d.t0 = 0.5 * (tmin + tmax) - g.nt / (2.0 * g.fs);
    } else {
        d.t0 = g.t0;
    }
    double floor_amp = std::pow(10.0, -g.band_db / 20.0);
    for (int k = 0; k <= g.nt / 2; ++k) {
        double f = (double)k * g.fs / g.nt;
        double env = std::exp(-(f - g.fc) * (f - g.fc) / (2.0 * d.sigma_f * d.sigma_f));
        if (env >= floor_amp) d.band.push_back(k);
    }
    if (!d.band.empty()) {
        d.band_lo = d.band.front();
        d.band_hi = d.band.back();
    }
    return d;
}

double pulse_spectrum(const ufss_geom& g, const Derived& d, int k) {
    double f = (double)k * g.fs / g.nt;
    return g.fs * std::sqrt(2.0 * M_PI) * d.sigma_t *
           std::exp(-(f - g.fc) * (f - g.fc) / (2.0 * d.sigma_f * d.sigma_f));
}

static void validate_geom(const ufss_geom* g) {
    if (!g) fail(UFSS_ERR_INVALID_ARG, "geometry pointer is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nt < 2)
        fail(UFSS_ERR_INVALID_ARG, "grid sizes must be positive (nt >= 2)");
    if ((int64_t)g->nx * g->ny > (1 << 24) || g->nz > (1 << 16) || g->nt > (1 << 20))
        fail(UFSS_ERR_INVALID_ARG, "grid too large");
    if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !(g->c > 0) || !(g->fs > 0) ||
        !(g->fc > 0) || !(g->frac_bw > 0) || !(g->band_db > 0) || !(g->z_start >= 0))
        fail(UFSS_ERR_INVALID_ARG, "physical parameters must be positive");
    if (g->dtype != UFSS_F32 && g->dtype != UFSS_BF16)
        fail(UFSS_ERR_INVALID_ARG, "dtype must be UFSS_F32 or UFSS_BF16");
    if (g->algo < UFSS_ALGO_AUTO || g->algo > UFSS_ALGO_FFT)
        fail(UFSS_ERR_INVALID_ARG, "unknown algo");
    if (!(g->theta >= 0) || !(g->theta < 0.5 * M_PI))
        fail(UFSS_ERR_INVALID_ARG, "theta must be in [0, pi/2)");
}

// Gaussian beam amplitude g = exp(-r^2 / (z tan theta)^2) at lateral offset
// (ix dx, iy dy) and depth index z (Sec. VI); 1 without a beam.
static double beam(const ufss_geom& g, int ix, int iy, int z) {
    if (!(g.theta > 0)) return 1.0;
    double w = (g.z_start + z * g.dz) * std::tan(g.theta);
    double rx = ix * g.dx, ry = iy * g.dy;
    return std::exp(-(rx * rx + ry * ry) / (w * w));
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) and the seeded subset draw.
// ---------------------------------------------------------------------------
static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ull;
        return mix64(s);
    }
};

static void draw(const std::vector<int>& band, int m, uint64_t key, int32_t* out) {
    std::vector<int> pool(band);
    const uint64_t n = pool.size();
    SplitMix64 rng(key);
    for (int i = 0; i < m; ++i) {
        uint64_t span = n - (uint64_t)i;
        uint64_t j = (uint64_t)i + (uint64_t)(((unsigned __int128)rng.next() * span) >> 64);
        std::swap(pool[i], pool[j]);
    }
    std::sort(pool.begin(), pool.begin() + m);
    for (int i = 0; i < m; ++i) out[i] = pool[i];
}

void select_freqs(const ufss_geom* g, int m, int per_position, uint64_t seed, int32_t* out,
                  int32_t* band_size) {
    validate_geom(g);
    if (!out) fail(UFSS_ERR_INVALID_ARG, "bins_out is NULL");
    if (m < 1) fail(UFSS_ERR_INVALID_ARG, "m must be >= 1");
    Derived d = derive(*g);
    if (band_size) *band_size = (int32_t)d.band.size();
    if ((size_t)m > d.band.size())
        fail(UFSS_ERR_BAND_TOO_SMALL, "m = " + std::to_string(m) + " exceeds the band size " +
                                          std::to_string(d.band.size()));
    if (!per_position) {
        draw(d.band, m, seed, out);
        return;
    }
    for (int iy = 0; iy < g->ny; ++iy)
        for (int ix = 0; ix < g->nx; ++ix) {
            int64_t p = ix + (int64_t)g->nx * iy;
            draw(d.band, m, seed ^ mix64((uint64_t)p + 1), out + p * m);
        }
}

// Knowledge-based strategies (Sec. III-A maximal / energy-based sampling,
// Table I per-A-scan variant).  Candidates are bins 0..nt/2 weighted by the
// Gaussian envelope of |H_k|; energy-based draws go without replacement, each
// from the running sum of the remaining weights in ascending bin order, FP64.
static std::vector<double> energy_weights(const ufss_geom& g, const Derived& d) {
    std::vector<double> w(g.nt / 2 + 1);
    for (int k = 0; k <= g.nt / 2; ++k) {
        double f = (double)k * g.fs / g.nt;
        double e = f - g.fc;
        w[k] = std::exp(-(e * e) / (2.0 * d.sigma_f * d.sigma_f));
    }
    return w;
}

static void take_max(const std::vector<double>& w, int m, int32_t* out) {
    std::vector<int> idx(w.size());
    for (size_t k = 0; k < w.size(); ++k) idx[k] = (int)k;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::sort(idx.begin(), idx.begin() + m);
    for (int i = 0; i < m; ++i) out[i] = idx[i];
}

static void draw_energy(const std::vector<double>& w, int m, uint64_t key, int32_t* out) {
    std::vector<char> left(w.size());
    for (size_t k = 0; k < w.size(); ++k) left[k] = w[k] > 0.0;
    SplitMix64 rng(key);
    for (int i = 0; i < m; ++i) {
        double total = 0.0;
        for (size_t k = 0; k < w.size(); ++k)
            if (left[k]) total += w[k];
        double target = (double)(rng.next() >> 11) * (1.0 / 9007199254740992.0) * total;
        double run = 0.0;
        int pick = -1;
        for (size_t k = 0; k < w.size(); ++k) {
            if (!left[k]) continue;
            run += w[k];
            pick = (int)k;
            if (run > target) break;
        }
        left[pick] = 0;
        out[i] = pick;
    }
    std::sort(out, out + m);
}

void sample_bins(const ufss_geom* g, int m, int strategy, uint64_t seed, int32_t* out,
                 int32_t* per_position_out) {
    validate_geom(g);
    if (!out) fail(UFSS_ERR_INVALID_ARG, "bins_out is NULL");
    if (m < 1) fail(UFSS_ERR_INVALID_ARG, "m must be >= 1");
    if (strategy < UFSS_SAMPLE_RND || strategy > UFSS_SAMPLE_NRG_F)
        fail(UFSS_ERR_INVALID_ARG, "unknown sampling strategy");
    const bool per = strategy == UFSS_SAMPLE_RND_F || strategy == UFSS_SAMPLE_NRG_F;
    if (per_position_out) *per_position_out = per ? 1 : 0;
    if (strategy == UFSS_SAMPLE_RND || strategy == UFSS_SAMPLE_RND_F) {
        select_freqs(g, m, per ? 1 : 0, seed, out, nullptr);
        return;
    }
    Derived d = derive(*g);
    std::vector<double> w = energy_weights(*g, d);
    int positive = 0;
    for (double v : w) positive += v > 0.0;
    if (m > positive)
        fail(UFSS_ERR_BAND_TOO_SMALL, "m = " + std::to_string(m) + " exceeds the " +
                                          std::to_string(positive) + " bins with energy");
    if (strategy == UFSS_SAMPLE_MAX) {
        take_max(w, m, out);
    } else if (strategy == UFSS_SAMPLE_NRG) {
        draw_energy(w, m, seed, out);
    } else {
        for (int iy = 0; iy < g->ny; ++iy)
            for (int ix = 0; ix < g->nx; ++ix) {
                int64_t p = ix + (int64_t)g->nx * iy;
                draw_energy(w, m, seed ^ mix64((uint64_t)p + 1), out + p * m);
            }
    }
}

// ---------------------------------------------------------------------------
// Plan.
// ---------------------------------------------------------------------------
template <class T>
static T* dalloc(Plan& P, size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    UFSS_HIP(hipMalloc(&p, count * sizeof(T)));
    P.ws_bytes += count * sizeof(T);
    return static_cast<T*>(p);
}

template <class T>
static void upload(T* dst, const T* src, size_t count) {
    UFSS_HIP(hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice));
}

static void free_plan(Plan* P) {
    if (!P) return;
    void* ptrs[] = {P->d_bins, P->d_ubins, P->d_map, P->d_hsel, P->d_u, P->d_yraw,
                    P->d_rop, P->d_xop, P->d_part, P->d_part_res, P->d_scalars, P->d_r, P->d_g,
                    P->d_gamma, P->d_v, P->d_stats, P->d_gpart, P->d_ptab_f, P->d_ptab_a,
                    P->d_bt, P->d_bt_scal, P->d_amp, P->d_xih, P->d_khat, P->d_khat_t, P->d_tw_fx, P->d_tw_fy,
                    P->d_tw_ix, P->d_tw_iy, P->d_fa, P->d_fb, P->d_ft};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& v : P->kev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    delete P;
}

// Subsets must be strictly ascending inside [0, nt/2].
static void validate_bins(const ufss_geom* g, int m, int per_position, const int32_t* bins) {
    const int nrows = per_position ? g->nx * g->ny : 1;
    for (int r = 0; r < nrows; ++r) {
        const int32_t* b = bins + (int64_t)r * m;
        for (int i = 0; i < m; ++i) {
            if (b[i] < 0 || b[i] > g->nt / 2)
                fail(UFSS_ERR_INVALID_ARG, "bin index outside [0, nt/2]");
            if (i > 0 && b[i] <= b[i - 1])
                fail(UFSS_ERR_INVALID_ARG, "bins of a position must be strictly ascending");
        }
    }
}

void validate_geom_public(const ufss_geom* g) { validate_geom(g); }

void validate_bins_public(const ufss_geom* g, int m, int per_position, const int32_t* bins) {
    validate_geom(g);
    validate_bins(g, m, per_position, bins);
}

// Sec. IV-C estimate of sigma_max from the Frobenius norm.  Every non-zero
// entry of A has modulus H_k g, so ||A||_F^2 = sum_p sum_m H_{k_m(p)}^2 times
// the sum of g^2 over the voxels in the window of p; the paper's cheaper form
// takes N_x N_y times the squared norms of the columns below the grid centre,
// summed over depth.  N = min(rows, cols)
// bounds the rank, and sigma_hat = ||A||_F / N^(1/4) is the geometric mean of
// ||A||_F / sqrt(N) <= sigma_max <= ||A||_F.  Host only, FP64.
void sigma_estimate(const ufss_geom* g, int m, int per_position, const int32_t* bins,
                    ufss_sigma_est* out) {
    validate_geom(g);
    if (!bins || !out) fail(UFSS_ERR_INVALID_ARG, "bins or out is NULL");
    if (m < 1) fail(UFSS_ERR_INVALID_ARG, "m must be >= 1");
    validate_bins(g, m, per_position, bins);
    Derived d = derive(*g);
    auto hsq = [&](int py, int px) {
        const int32_t* b = bins + (per_position ? ((int64_t)py * g->nx + px) * m : 0);
        double s = 0.0;
        for (int i = 0; i < m; ++i) {
            double h = pulse_spectrum(*g, d, b[i]);
            s += h * h;
        }
        return s;
    };
    // S[|dy|][|dx|] = sum over depth of g^2 (N_z without a beam)
    std::vector<double> S((size_t)(d.wy + 1) * (d.wx + 1), 0.0);
    for (int iy = 0; iy <= d.wy; ++iy)
        for (int ix = 0; ix <= d.wx; ++ix) {
            double acc = 0.0;
            for (int z = 0; z < g->nz; ++z) {
                double b = beam(*g, ix, iy, z);
                acc += b * b;
            }
            S[(size_t)iy * (d.wx + 1) + ix] = acc;
        }
    auto wsum = [&](int py, int px) {
        double acc = 0.0;
        for (int vy = std::max(py - d.wy, 0); vy <= std::min(py + d.wy, g->ny - 1); ++vy)
            for (int vx = std::max(px - d.wx, 0); vx <= std::min(px + d.wx, g->nx - 1); ++vx)
                acc += S[(size_t)std::abs(vy - py) * (d.wx + 1) + std::abs(vx - px)];
        return acc;
    };
    double fro = 0.0;
    for (int py = 0; py < g->ny; ++py)
        for (int px = 0; px < g->nx; ++px) fro += hsq(py, px) * wsum(py, px);
    const int vx = (g->nx - 1) / 2, vy = (g->ny - 1) / 2;
    double col = 0.0;
    for (int py = std::max(vy - d.wy, 0); py <= std::min(vy + d.wy, g->ny - 1); ++py)
        for (int px = std::max(vx - d.wx, 0); px <= std::min(vx + d.wx, g->nx - 1); ++px)
            col += hsq(py, px) * S[(size_t)std::abs(py - vy) * (d.wx + 1) + std::abs(px - vx)];
    const double npos = (double)g->nx * g->ny;
    out->fro_sq = fro;
    out->fro_sq_central = npos * col;
    out->n = (int64_t)g->nx * g->ny * std::min(m, g->nz);
    const double q = std::pow((double)out->n, 0.25);
    out->sigma_hat = std::sqrt(out->fro_sq) / q;
    out->sigma_hat_central = std::sqrt(out->fro_sq_central) / q;
}

// F xi / nt of one row of signs, FP64 radix-2 FFT (nt a power of two).
static void signs_dft(const int8_t* xi, int nt, std::vector<double>& re, std::vector<double>& im) {
    re.assign(nt, 0.0);
    im.assign(nt, 0.0);
    int bits = 0;
    while ((1 << bits) < nt) ++bits;
    for (int i = 0; i < nt; ++i) {
        int r = 0;
        for (int b = 0; b < bits; ++b)
            if (i & (1 << b)) r |= 1 << (bits - 1 - b);
        re[r] = xi[i];
    }
    for (int len = 2; len <= nt; len <<= 1) {
        for (int i = 0; i < nt; i += len)
            for (int j = 0; j < len / 2; ++j) {
                const double a = -2.0 * M_PI * j / len;
                const double wr = std::cos(a), wi = std::sin(a);
                const int u = i + j, v = i + j + len / 2;
                const double tr = re[v] * wr - im[v] * wi, ti = re[v] * wi + im[v] * wr;
                re[v] = re[u] - tr;
                im[v] = im[u] - ti;
                re[u] += tr;
                im[u] += ti;
            }
    }
    for (int i = 0; i < nt; ++i) {
        re[i] /= nt;
        im[i] /= nt;
    }
}

Plan* plan_create(const ufss_geom* g, int m, int per_position, const int32_t* bins,
                  const MixSpec* mix) {
    validate_geom(g);
    if (!bins) fail(UFSS_ERR_INVALID_ARG, "bins is NULL");
    if (m < 1 || m > 4096) fail(UFSS_ERR_INVALID_ARG, "m must be in [1, 4096]");
    Derived d = derive(*g);
    const int npos = g->nx * g->ny;
    const int64_t nsel = per_position ? (int64_t)npos * m : m;
    int algo = g->algo;
    if (algo == UFSS_ALGO_AUTO) algo = UFSS_ALGO_GEMM;
    if (mix) {
        // bins anywhere in [0, nt), signs +-1; FP32 GEMM or transform core
        if (!mix->signs) fail(UFSS_ERR_INVALID_ARG, "signs is NULL");
        if (g->nt > 4096 || (g->nt & (g->nt - 1)))
            fail(UFSS_ERR_UNSUPPORTED, "mixing needs nt a power of two, at most 4096");
        if (g->dtype != UFSS_F32 || algo == UFSS_ALGO_PHASOR)
            fail(UFSS_ERR_UNSUPPORTED, "mixing runs on the FP32 GEMM or transform path");
        // the mixing passes stage a position's rows in LDS (64 KiB)
        if (8 * (int64_t)g->nt + 12 * (int64_t)m > 65536)
            fail(UFSS_ERR_UNSUPPORTED, "mixing: 8 nt + 12 m must not exceed 65536");
        const int nrows = per_position ? npos : 1;
        for (int r = 0; r < nrows; ++r)
            for (int i = 0; i < m; ++i) {
                const int32_t k = bins[(int64_t)r * m + i];
                if (k < 0 || k >= g->nt) fail(UFSS_ERR_INVALID_ARG, "bin index outside [0, nt)");
                if (i > 0 && k <= bins[(int64_t)r * m + i - 1])
                    fail(UFSS_ERR_INVALID_ARG, "bins of a position must be strictly ascending");
            }
        const int64_t ns = (int64_t)(mix->per_sign ? npos : 1) * g->nt;
        for (int64_t i = 0; i < ns; ++i)
            if (mix->signs[i] != 1 && mix->signs[i] != -1)
                fail(UFSS_ERR_INVALID_ARG, "signs must be +1 or -1");
    } else {
        validate_bins(g, m, per_position, bins);
    }
    if (g->algo == UFSS_ALGO_AUTO && per_position && !mix && g->dtype == UFSS_F32) {
        // per-position subsets: the phasor path costs about one phasor per
        // selected bin and term, the union-GEMM one MFMA slot per union bin
        // (padded) at several times the rate; measured on the 50x50x50
        // replica the phasor path wins while the union has at least ~5x the
        // bins of one position (n_f = 1, 2, 5 of a 37-bin union), the GEMM above
        std::vector<int> uu(bins, bins + nsel);
        std::sort(uu.begin(), uu.end());
        const int64_t nu = std::unique(uu.begin(), uu.end()) - uu.begin();
        if (5 * (int64_t)m <= nu) algo = UFSS_ALGO_PHASOR;
    }
    if (algo == UFSS_ALGO_PHASOR && g->dtype == UFSS_BF16)
        fail(UFSS_ERR_UNSUPPORTED, "the phasor path is FP32 only");
    if (algo == UFSS_ALGO_PHASOR && !per_position) algo = UFSS_ALGO_GEMM;

    Plan* P = new (std::nothrow) Plan();
    if (!P) fail(UFSS_ERR_OOM, "host allocation failed");
    try {
        P->g = *g;
        P->d = d;
        P->m = m;
        P->per_position = per_position ? 1 : 0;
        P->algo = algo;
        P->dtype = g->dtype;
        P->npos = npos;
        P->nvox = (int64_t)npos * g->nz;
        P->bins_h.assign(bins, bins + nsel);
        // union of bins (GEMM path over per-position subsets); a mixed plan runs
        // over every DFT index as a signed bin: j (j <= nt/2) or j - nt
        std::vector<int> u(P->bins_h);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        if (mix) {
            u.resize(g->nt);
            for (int j = 0; j < g->nt; ++j) u[j] = j <= g->nt / 2 ? j : j - g->nt;
        }
        P->ubins_h = u;
        const int mu = (int)u.size();
        const int opw = (algo == UFSS_ALGO_PHASOR) ? m : mu;   // operand row width
        std::vector<int> map(mix ? 1 : nsel, 0);
        std::vector<float> hsel(mix ? mu : nsel);
        if (mix) {
            for (int j = 0; j < mu; ++j) hsel[j] = (float)pulse_spectrum(*g, d, u[j]);
        } else {
            for (int64_t i = 0; i < nsel; ++i) {
                int k = P->bins_h[i];
                map[i] = (algo == UFSS_ALGO_PHASOR)
                             ? (int)(i % m)
                             : (int)(std::lower_bound(u.begin(), u.end(), k) - u.begin());
                hsel[i] = (float)pulse_spectrum(*g, d, k);
            }
        }
        // integer-turn delay table: u(|dx|, |dy|, z) = round(2^32 frac((tau - t0) fs / nt))
        const int wx = d.wx, wy = d.wy;
        std::vector<uint32_t> ut((size_t)(wy + 1) * (wx + 1) * g->nz);
        for (int j = 0; j <= wy; ++j)
            for (int i = 0; i <= wx; ++i)
                for (int z = 0; z < g->nz; ++z) {
                    double t = delay(*g, i * g->dx, j * g->dy, g->z_start + z * g->dz);
                    double ph = (t - d.t0) * g->fs / g->nt;
                    double fr = ph - std::floor(ph);
                    double q = std::nearbyint(fr * 4294967296.0);
                    uint64_t qi = (uint64_t)q & 0xFFFFFFFFull;
                    ut[((size_t)j * (wx + 1) + i) * g->nz + z] = (uint32_t)qi;
                }
        P->d_bins = dalloc<int>(*P, nsel);
        upload(P->d_bins, P->bins_h.data(), nsel);
        P->d_ubins = dalloc<int>(*P, mu);
        upload(P->d_ubins, u.data(), mu);
        P->d_map = dalloc<int>(*P, map.size());
        upload(P->d_map, map.data(), map.size());
        P->d_hsel = dalloc<float>(*P, hsel.size());
        upload(P->d_hsel, hsel.data(), hsel.size());
        if (mix) {
            const int nrow = mix->per_sign ? npos : 1;
            std::vector<cf32> xh((size_t)nrow * g->nt);
            std::vector<double> re, im;
            for (int r = 0; r < nrow; ++r) {
                signs_dft(mix->signs + (int64_t)r * g->nt, g->nt, re, im);
                for (int j = 0; j < g->nt; ++j)
                    xh[(size_t)r * g->nt + j] = cf32{(float)re[j], (float)im[j]};
            }
            P->d_xih = dalloc<cf32>(*P, xh.size());
            upload(static_cast<cf32*>(P->d_xih), xh.data(), xh.size());
            P->mix = 1;
            P->mix_per_sign = mix->per_sign ? 1 : 0;
        }
        P->d_u = dalloc<uint32_t>(*P, ut.size());
        upload(P->d_u, ut.data(), ut.size());
        if (g->theta > 0) {
            // beam amplitude table, same layout as the delay table
            std::vector<float> at(ut.size());
            for (int j = 0; j <= wy; ++j)
                for (int i = 0; i <= wx; ++i)
                    for (int z = 0; z < g->nz; ++z)
                        at[((size_t)j * (wx + 1) + i) * g->nz + z] = (float)beam(*g, i, j, z);
            P->d_amp = dalloc<float>(*P, at.size());
            upload(P->d_amp, at.data(), at.size());
        }
        if (algo == UFSS_ALGO_GEMM && P->dtype == UFSS_BF16) {
            if (!bf16_supported(*P))
                fail(UFSS_ERR_UNSUPPORTED, "aperture window too wide for the BF16 GEMM path");
            P->fwd_split = bf16_fwd_split(*P);
            P->adj_split = bf16_adj_split(*P);
        } else {
            P->fwd_split = (algo == UFSS_ALGO_GEMM) ? gemm_split(*P) : 1;
            P->adj_split = (algo == UFSS_ALGO_GEMM) ? adj_split(*P) : 1;
        }
        if (P->adj_split > 1) P->d_gpart = dalloc<cf32>(*P, (size_t)P->adj_split * P->nvox);
        P->d_yraw = dalloc<cf32>(*P, (size_t)P->fwd_split * npos * mu);
        P->d_rop = dalloc<cf32>(*P, (size_t)npos * opw);
        if (algo == UFSS_ALGO_GEMM && P->dtype == UFSS_BF16) P->d_xop = dalloc<cf32>(*P, (size_t)(P->nvox + 1) / 2 + 1);
        if (algo == UFSS_ALGO_GEMM && P->dtype == UFSS_BF16) bf16_set_tables(*P, 1);
        if (algo == UFSS_ALGO_FFT) fft_setup(*P);
        P->part_cap = 65536;
        P->d_part = dalloc<double>(*P, P->part_cap);
        P->d_part_res = dalloc<double>(*P, P->part_cap);
        P->d_scalars = dalloc<double>(*P, 64);
        P->d_r = dalloc<cf32>(*P, (size_t)npos * m);
        P->d_g = dalloc<cf32>(*P, P->nvox);
        P->d_gamma = dalloc<cf32>(*P, P->nvox);
        P->d_v = dalloc<cf32>(*P, P->nvox);
        UFSS_HIP(hipMemset(P->d_scalars, 0, 64 * sizeof(double)));
        UFSS_HIP(hipDeviceSynchronize());
    } catch (...) {
        free_plan(P);
        throw;
    }
    return P;
}

// Change the split-K factors of the GEMM path (reallocating their partials).
void plan_set_splits(Plan& P, int fs, int as, int zs) {
    if (fs < 1 || as < 1 || zs < 1) fail(UFSS_ERR_INVALID_ARG, "split factors must be >= 1");
    const size_t mu = P.ubins_h.size();
    if (fs * zs != P.fwd_split * P.fwd_zsplit) {
        UFSS_HIP(hipDeviceSynchronize());
        if (P.d_yraw) UFSS_HIP(hipFree(P.d_yraw));
        P.ws_bytes -= (int64_t)P.fwd_split * P.fwd_zsplit * P.npos * mu * sizeof(cf32);
        P.d_yraw = nullptr;
        P.d_yraw = dalloc<cf32>(P, (size_t)fs * zs * P.npos * mu);
    }
    P.fwd_split = fs;
    P.fwd_zsplit = zs;
    if (as != P.adj_split) {
        UFSS_HIP(hipDeviceSynchronize());
        if (P.d_gpart) {
            UFSS_HIP(hipFree(P.d_gpart));
            P.ws_bytes -= (int64_t)P.adj_split * P.nvox * sizeof(cf32);
        }
        P.d_gpart = nullptr;
        if (as > 1) P.d_gpart = dalloc<cf32>(P, (size_t)as * P.nvox);
        P.adj_split = as;
    }
}

void plan_destroy(Plan* P) {
    if (!P) fail(UFSS_ERR_INVALID_ARG, "plan is NULL");
    UFSS_HIP(hipDeviceSynchronize());
    free_plan(P);
}

void plan_info(const Plan* P, ufss_plan_info* info) {
    if (!P || !info) fail(UFSS_ERR_INVALID_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->t0 = P->d.t0;
    info->lipschitz = P->lipschitz;
    info->band_lo = P->d.band_lo;
    info->band_hi = P->d.band_hi;
    info->band_size = (int32_t)P->d.band.size();
    info->win_x = P->d.wx;
    info->win_y = P->d.wy;
    info->m = P->m;
    info->per_position = P->per_position;
    info->dtype = P->dtype;
    info->algo = P->algo;
    info->union_size = (int32_t)P->ubins_h.size();
    info->workspace_bytes = P->ws_bytes;
    info->fwd_split = P->fwd_split;
    info->adj_split = P->adj_split;
    const bool f32_gemm = P->algo == UFSS_ALGO_GEMM && P->dtype == UFSS_F32;
    info->fwd_waves = f32_gemm ? std::max(1, std::min(P->fwd_nw, ((int)P->ubins_h.size() + 15) / 16)) : 1;
    info->fwd_zsplit = P->algo == UFSS_ALGO_GEMM ? P->fwd_zsplit : 1;
    info->phasor_tables = P->d_ptab_f != nullptr;
    info->fwd_tile = f32_gemm ? fwd_tile_np(*P) : 0;
    info->adj_tile = f32_gemm ? adj_tile_np(*P) : 0;
    if (P->algo == UFSS_ALGO_GEMM && P->dtype == UFSS_BF16) info->adj_tile = P->bf_adj_nz;
    const bool bf_gemm = P->algo == UFSS_ALGO_GEMM && P->dtype == UFSS_BF16;
    info->fwd_rows = bf_gemm ? P->bf_fwd_rows : 0;
    info->adj_rows = bf_gemm ? P->bf_adj_rows : 0;
    info->fwd_chunk = f32_gemm ? fwd_chunk(*P) : 0;
    info->adj_chunk = f32_gemm ? adj_chunk(*P) : 0;
    info->adj_waves = f32_gemm ? adj_waves(*P) : 0;
}

}  // namespace ufss
