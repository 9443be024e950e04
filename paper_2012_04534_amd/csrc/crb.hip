// Cramer-Rao bound for locating one scatterer under a bin selection (paper
// Sec. VI, Slepian-Bangs Fisher information), for many selections at once.
//
// With b_{i,k} = a e^{j phi} H_k g_i exp(-j 2 pi f_k (tau_i - t0)) every
// derivative is b times a factor, d b / d u_n = b c_n with
//   c_x = gx - j w_k tx,  c_y = gy - j w_k ty,  c_z = gz - j w_k tz,
//   c_a = 1 / a,          c_phi = j,
// (t. = d tau / d., g. = (d g / d.) / g, w_k = 2 pi f_k), so
// Re{conj(d b_m) d b_n} = |b|^2 Re{conj(c_m) c_n} carries no phase.  Per scan
// position the bins enter only through S0 = sum H_k^2, S1 = sum H_k^2 w_k and
// S2 = sum H_k^2 w_k^2 over its selected bins.  One workgroup per selection
// sums the 15 distinct entries over positions in FP64 (fixed order); the host
// scales by 2 / sigma^2 and takes the position block of J^{-1} by the Schur
// complement of the (a, phi) block.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace ufss {

static constexpr int kCrbThreads = 256;

struct CrbArgs {
    const int* bins;        // [trials][npos][m] or [trials][m]
    double* out;            // [trials][15]
    int nx, ny, nt, m, per_pos, wx, wy;
    double dx, dy, c, fs, fc, sigma_f, sigma_t, tan_theta;
    double x1, y1, z1, amp;
};

// The 15 distinct entries, in this order: xx xy xz yy yz zz, then (x,a)
// (x,phi) (y,a) (y,phi) (z,a) (z,phi), then aa, (a,phi), (phi,phi).
__global__ __launch_bounds__(kCrbThreads) void crb_fim_kernel(CrbArgs a) {
    const int trial = blockIdx.x;
    const int npos = a.nx * a.ny;
    const int* tb = a.bins + (int64_t)trial * (a.per_pos ? (int64_t)npos * a.m : a.m);
    double acc[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) acc[e] = 0.0;
    const double kpi2 = 2.0 * M_PI;
    const double hs = a.fs * sqrt(2.0 * M_PI) * a.sigma_t;
    for (int p = threadIdx.x; p < npos; p += kCrbThreads) {
        const int ix = p % a.nx, iy = p / a.nx;
        const double dxm = a.x1 - ix * a.dx, dym = a.y1 - iy * a.dy;
        if (fabs(dxm) > a.wx * a.dx + 1e-12 || fabs(dym) > a.wy * a.dy + 1e-12) continue;
        const double R = sqrt(dxm * dxm + dym * dym + a.z1 * a.z1);
        const double k2c = 2.0 / a.c;
        const double tx = k2c * dxm / R, ty = k2c * dym / R, tz = k2c * a.z1 / R;
        double gx = 0.0, gy = 0.0, gz = 0.0, gb = 1.0;
        if (a.tan_theta > 0.0) {
            const double w = a.z1 * a.tan_theta, w2 = w * w, r2 = dxm * dxm + dym * dym;
            gb = exp(-r2 / w2);
            gx = -2.0 * dxm / w2;
            gy = -2.0 * dym / w2;
            gz = 2.0 * r2 / (w2 * a.z1);
        }
        const int* kb = tb + (a.per_pos ? (int64_t)p * a.m : 0);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < a.m; ++i) {
            const double f = (double)kb[i] * a.fs / a.nt;
            const double e = f - a.fc;
            const double h = hs * exp(-(e * e) / (2.0 * a.sigma_f * a.sigma_f));
            const double h2 = h * h, om = kpi2 * f;
            s0 += h2;
            s1 += h2 * om;
            s2 += h2 * om * om;
        }
        // |b|^2 = a^2 H_k^2 g^2 (H_k^2 already inside s0, s1, s2)
        const double wgt = a.amp * a.amp * gb * gb;
        const double al[3] = {gx, gy, gz}, ta[3] = {tx, ty, tz};
        int e = 0;
#pragma unroll
        for (int mi = 0; mi < 3; ++mi)
#pragma unroll
            for (int ni = mi; ni < 3; ++ni) acc[e++] += wgt * (al[mi] * al[ni] * s0 + ta[mi] * ta[ni] * s2);
#pragma unroll
        for (int mi = 0; mi < 3; ++mi) {
            acc[e++] += wgt * al[mi] * s0 / a.amp;     // (m, a)
            acc[e++] += -wgt * ta[mi] * s1;            // (m, phi)
        }
        acc[e++] += wgt * s0 / (a.amp * a.amp);        // (a, a)
        acc[e++] += 0.0;                               // (a, phi)
        acc[e++] += wgt * s0;                          // (phi, phi)
    }
    // block sum in fixed order
    __shared__ double red[15][kCrbThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 15; ++e) {
        double v = acc[e];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[e][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 15) {
        double s = 0.0;
        for (int w = 0; w < kCrbThreads / 64; ++w) s += red[threadIdx.x][w];
        a.out[(int64_t)trial * 15 + threadIdx.x] = s;
    }
}

// ---- mixed measurements (Rademacher Sigma) ----------------------------------
// Derivative rows over every signed bin j (DFT index order) of every position:
// BC[p][j][n] = b_{p,j} c_{p,j,n}, b = a e^{j phi} H_j g_p exp(-j 2 pi f_j (tau_p - t0)).
struct CrbMixArgs {
    CrbArgs base;
    double t0, phase;
};

__global__ __launch_bounds__(256) void crb_bc_kernel(CrbMixArgs m, double2* __restrict__ bc) {
    const CrbArgs& a = m.base;
    const int64_t n = (int64_t)a.nx * a.ny * a.nt;
    const double hs = a.fs * sqrt(2.0 * M_PI) * a.sigma_t;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / a.nt;
        const int j = (int)(t - p * a.nt);
        const int ix = (int)(p % a.nx), iy = (int)(p / a.nx);
        const double dxm = a.x1 - ix * a.dx, dym = a.y1 - iy * a.dy;
        double2* out = bc + t * 5;
        if (fabs(dxm) > a.wx * a.dx + 1e-12 || fabs(dym) > a.wy * a.dy + 1e-12) {
            for (int q = 0; q < 5; ++q) out[q] = double2{0.0, 0.0};
            continue;
        }
        const double R = sqrt(dxm * dxm + dym * dym + a.z1 * a.z1);
        const double k2c = 2.0 / a.c;
        const double tx = k2c * dxm / R, ty = k2c * dym / R, tz = k2c * a.z1 / R;
        double gx = 0.0, gy = 0.0, gz = 0.0, gb = 1.0;
        if (a.tan_theta > 0.0) {
            const double w = a.z1 * a.tan_theta, w2 = w * w, r2 = dxm * dxm + dym * dym;
            gb = exp(-r2 / w2);
            gx = -2.0 * dxm / w2;
            gy = -2.0 * dym / w2;
            gz = 2.0 * r2 / (w2 * a.z1);
        }
        const int k = j <= a.nt / 2 ? j : j - a.nt;
        const double f = (double)k * a.fs / a.nt, e = f - a.fc;
        const double h = hs * exp(-(e * e) / (2.0 * a.sigma_f * a.sigma_f));
        const double ang = m.phase - 2.0 * M_PI * f * (k2c * R - m.t0);
        double sn, cs;
        sincos(ang, &sn, &cs);
        const double br = a.amp * h * gb * cs, bi = a.amp * h * gb * sn;
        const double om = 2.0 * M_PI * f;
        // c = (g. - j om t.) for x, y, z; 1/a; j
        const double cr[5] = {gx, gy, gz, 1.0 / a.amp, 0.0};
        const double ci[5] = {-om * tx, -om * ty, -om * tz, 0.0, 1.0};
        for (int q = 0; q < 5; ++q) out[q] = double2{br * cr[q] - bi * ci[q], br * ci[q] + bi * cr[q]};
    }
}

// xih[r][k] = (1/nt) sum_n xi[r][n] exp(-j 2 pi k n / nt)  (nt a power of two)
__global__ __launch_bounds__(256) void crb_signs_dft_kernel(const int8_t* __restrict__ xi, int64_t rows,
                                                            int nt, double2* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    double2* w = reinterpret_cast<double2*>(smem);     // [nt] twiddles
    for (int n = threadIdx.x; n < nt; n += blockDim.x) {
        double sn, cs;
        sincos(-2.0 * M_PI * n / nt, &sn, &cs);
        w[n] = double2{cs, sn};
    }
    __syncthreads();
    const int mask = nt - 1;
    const int64_t total = rows * nt;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / nt;
        const int k = (int)(t - r * nt);
        const int8_t* x = xi + r * nt;
        double re = 0.0, im = 0.0;
        for (int n = 0; n < nt; ++n) {
            const double2 tw = w[(k * n) & mask];
            re += x[n] * tw.x;
            im += x[n] * tw.y;
        }
        out[t] = double2{re / nt, im / nt};
    }
}

// One workgroup per trial, threads over positions: z_m = sum_j xih[(k_m - j) mod nt] BC[p][j],
// J += Re{z_m^H z_m} (the 15 distinct entries in the order of crb_fim_kernel).
__global__ __launch_bounds__(256) void crb_fim_mixed_kernel(const double2* __restrict__ bc,
                                                            const double2* __restrict__ xih,
                                                            const int* __restrict__ bins, int npos,
                                                            int nt, int m, int per_pos, int per_sign,
                                                            double* __restrict__ out) {
    const int trial = blockIdx.x;
    const int mask = nt - 1;
    const int* tb = bins + (int64_t)trial * (per_pos ? (int64_t)npos * m : m);
    const double2* tx = xih + (int64_t)trial * (per_sign ? (int64_t)npos * nt : nt);
    double acc[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) acc[e] = 0.0;
    const int pr[15][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}, {0, 3}, {0, 4},
                           {1, 3}, {1, 4}, {2, 3}, {2, 4}, {3, 3}, {3, 4}, {4, 4}};
    for (int p = threadIdx.x; p < npos; p += blockDim.x) {
        const double2* row = bc + (int64_t)p * nt * 5;
        const double2* xs = tx + (per_sign ? (int64_t)p * nt : 0);
        const int* kb = tb + (per_pos ? (int64_t)p * m : 0);
        for (int m0 = 0; m0 < m; m0 += 4) {
            const int mb = min(4, m - m0);
            double zr[4][5], zi[4][5];
            for (int i = 0; i < 4; ++i)
                for (int q = 0; q < 5; ++q) zr[i][q] = zi[i][q] = 0.0;
            for (int j = 0; j < nt; ++j) {
                double2 v[5];
                for (int q = 0; q < 5; ++q) v[q] = row[(int64_t)j * 5 + q];
                for (int i = 0; i < 4; ++i) {
                    if (i >= mb) break;
                    const double2 w = xs[(kb[m0 + i] - j) & mask];
                    for (int q = 0; q < 5; ++q) {
                        zr[i][q] += w.x * v[q].x - w.y * v[q].y;
                        zi[i][q] += w.x * v[q].y + w.y * v[q].x;
                    }
                }
            }
            for (int i = 0; i < mb; ++i)
                for (int e = 0; e < 15; ++e) {
                    const int q = pr[e][0], r = pr[e][1];
                    acc[e] += zr[i][q] * zr[i][r] + zi[i][q] * zi[i][r];
                }
        }
    }
    __shared__ double red[15][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = 0; e < 15; ++e) {
        double v = acc[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[e][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 15) {
        double sm = 0.0;
        for (int w2 = 0; w2 < 4; ++w2) sm += red[threadIdx.x][w2];
        out[(int64_t)trial * 15 + threadIdx.x] = sm;
    }
}

// Gauss-Jordan inverse with partial pivoting of a small row-major matrix.
static void small_inverse(int n, const double* A, double* out) {
    std::vector<double> M((size_t)n * 2 * n, 0.0);
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) M[(size_t)r * 2 * n + c] = A[r * n + c];
        M[(size_t)r * 2 * n + n + r] = 1.0;
    }
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::fabs(A[i]));
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[(size_t)r * 2 * n + c]) > std::fabs(M[(size_t)piv * 2 * n + c])) piv = r;
        // a pivot at rounding level of the largest entry: numerically singular
        if (!(std::fabs(M[(size_t)piv * 2 * n + c]) > 1e-13 * scale))
            fail(UFSS_ERR_INVALID_ARG, "singular Fisher information: these measurements do not "
                                       "determine the scatterer");
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) std::swap(M[(size_t)c * 2 * n + k], M[(size_t)piv * 2 * n + k]);
        const double d = M[(size_t)c * 2 * n + c];
        for (int k = 0; k < 2 * n; ++k) M[(size_t)c * 2 * n + k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = M[(size_t)r * 2 * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < 2 * n; ++k) M[(size_t)r * 2 * n + k] -= f * M[(size_t)c * 2 * n + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) out[r * n + c] = M[(size_t)r * 2 * n + n + c];
}

// 15 distinct entries (kernel order) -> symmetric 5 x 5, scaled by s.
static void unpack_fim(const double* e, double s, double* J) {
    // kernel order: xx xy xz yy yz zz | xa xphi ya yphi za zphi | aa aphi phiphi
    const int pos[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int i = 0; i < 25; ++i) J[i] = 0.0;
    for (int q = 0; q < 6; ++q) {
        J[pos[q][0] * 5 + pos[q][1]] = J[pos[q][1] * 5 + pos[q][0]] = s * e[q];
    }
    for (int mi = 0; mi < 3; ++mi) {
        J[mi * 5 + 3] = J[3 * 5 + mi] = s * e[6 + 2 * mi];
        J[mi * 5 + 4] = J[4 * 5 + mi] = s * e[7 + 2 * mi];
    }
    J[3 * 5 + 3] = s * e[12];
    J[3 * 5 + 4] = J[4 * 5 + 3] = s * e[13];
    J[4 * 5 + 4] = s * e[14];
}

// Position block of J^{-1} by the Schur complement of the nuisance block:
// C_p = Jp^-1 + Jp^-1 Jpn Q^-1 Jpn^T Jp^-1,  Q = Jn - Jpn^T Jp^-1 Jpn.
static void crb_from_fim(const double* J, double* c3) {
    double Jp[9], Jpn[6], Jn[4], Jpi[9], Q[4], Qi[4];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Jp[r * 3 + c] = J[r * 5 + c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 2; ++c) Jpn[r * 2 + c] = J[r * 5 + 3 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) Jn[r * 2 + c] = J[(3 + r) * 5 + 3 + c];
    small_inverse(3, Jp, Jpi);
    double T[6];   // Jp^-1 Jpn  [3][2]
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 2; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Jpi[r * 3 + k] * Jpn[k * 2 + c];
            T[r * 2 + c] = s;
        }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Jpn[k * 2 + r] * T[k * 2 + c];
            Q[r * 2 + c] = Jn[r * 2 + c] - s;
        }
    small_inverse(2, Q, Qi);
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) s += T[d * 2 + r] * Qi[r * 2 + c] * T[d * 2 + c];
        c3[d] = Jpi[d * 3 + d] + s;
    }
}

void crb(const ufss_geom* g, int m, int per_position, int trials, const int32_t* bins,
         const ufss_crb_point* pt, double* fim_out, double* crb_out, hipStream_t s) {
    if (!g || !bins || !pt || !crb_out) fail(UFSS_ERR_INVALID_ARG, "NULL argument");
    if (m < 1 || trials < 1) fail(UFSS_ERR_INVALID_ARG, "m and trials must be >= 1");
    if (!(pt->z > 0) || !(pt->amp > 0) || !(pt->sigma2 > 0) || !std::isfinite(pt->x) ||
        !std::isfinite(pt->y) || !std::isfinite(pt->phase))
        fail(UFSS_ERR_INVALID_ARG, "need z > 0, amp > 0, sigma2 > 0 and finite x, y, phase");
    const int64_t per = per_position ? (int64_t)g->nx * g->ny * m : m;
    for (int t = 0; t < trials; ++t) validate_bins_public(g, m, per_position, bins + t * per);
    Derived d = derive(*g);
    CrbArgs a{};
    a.nx = g->nx;
    a.ny = g->ny;
    a.nt = g->nt;
    a.m = m;
    a.per_pos = per_position ? 1 : 0;
    a.wx = d.wx;
    a.wy = d.wy;
    a.dx = g->dx;
    a.dy = g->dy;
    a.c = g->c;
    a.fs = g->fs;
    a.fc = g->fc;
    a.sigma_f = d.sigma_f;
    a.sigma_t = d.sigma_t;
    a.tan_theta = g->theta > 0 ? std::tan(g->theta) : 0.0;
    a.x1 = pt->x;
    a.y1 = pt->y;
    a.z1 = pt->z;
    a.amp = pt->amp;
    int* dbins = nullptr;
    double* dout = nullptr;
    std::vector<double> h((size_t)trials * 15);
    try {
        UFSS_HIP(hipMalloc(&dbins, (size_t)trials * per * sizeof(int)));
        UFSS_HIP(hipMalloc(&dout, (size_t)trials * 15 * sizeof(double)));
        UFSS_HIP(hipMemcpyAsync(dbins, bins, (size_t)trials * per * sizeof(int), hipMemcpyHostToDevice, s));
        a.bins = dbins;
        a.out = dout;
        hipLaunchKernelGGL(crb_fim_kernel, dim3(trials), dim3(kCrbThreads), 0, s, a);
        UFSS_HIP(hipGetLastError());
        UFSS_HIP(hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        UFSS_HIP(hipStreamSynchronize(s));
    } catch (...) {
        if (dbins) (void)hipFree(dbins);
        if (dout) (void)hipFree(dout);
        throw;
    }
    (void)hipFree(dbins);
    (void)hipFree(dout);
    const double scale = 2.0 / pt->sigma2;
    for (int t = 0; t < trials; ++t) {
        double J[25];
        unpack_fim(h.data() + (size_t)t * 15, scale, J);
        if (fim_out)
            for (int i = 0; i < 25; ++i) fim_out[(size_t)t * 25 + i] = J[i];
        crb_from_fim(J, crb_out + (size_t)t * 3);
    }
}

void crb_mixed(const ufss_geom* g, int m, int per_position, int trials, const int32_t* bins,
               int per_position_signs, const int8_t* signs, const ufss_crb_point* pt,
               double* fim_out, double* crb_out, hipStream_t s) {
    if (!g || !bins || !signs || !pt || !crb_out) fail(UFSS_ERR_INVALID_ARG, "NULL argument");
    if (m < 1 || trials < 1) fail(UFSS_ERR_INVALID_ARG, "m and trials must be >= 1");
    if (!(pt->z > 0) || !(pt->amp > 0) || !(pt->sigma2 > 0) || !std::isfinite(pt->x) ||
        !std::isfinite(pt->y) || !std::isfinite(pt->phase))
        fail(UFSS_ERR_INVALID_ARG, "need z > 0, amp > 0, sigma2 > 0 and finite x, y, phase");
    validate_geom_public(g);
    const int nt = g->nt, npos = g->nx * g->ny;
    if (nt > 4096 || (nt & (nt - 1))) fail(UFSS_ERR_UNSUPPORTED, "mixing needs nt a power of two, at most 4096");
    const int64_t per = per_position ? (int64_t)npos * m : m;
    for (int t = 0; t < trials; ++t)
        for (int64_t r = 0; r < (per_position ? npos : 1); ++r)
            for (int i = 0; i < m; ++i) {
                const int32_t k = bins[t * per + r * m + i];
                if (k < 0 || k >= nt) fail(UFSS_ERR_INVALID_ARG, "bin index outside [0, nt)");
                if (i > 0 && k <= bins[t * per + r * m + i - 1])
                    fail(UFSS_ERR_INVALID_ARG, "bins of a position must be strictly ascending");
            }
    const int64_t srow = per_position_signs ? npos : 1;
    const int64_t ns = (int64_t)trials * srow * nt;
    for (int64_t i = 0; i < ns; ++i)
        if (signs[i] != 1 && signs[i] != -1) fail(UFSS_ERR_INVALID_ARG, "signs must be +1 or -1");
    Derived d = derive(*g);
    CrbMixArgs a{};
    a.base.nx = g->nx;
    a.base.ny = g->ny;
    a.base.nt = nt;
    a.base.wx = d.wx;
    a.base.wy = d.wy;
    a.base.dx = g->dx;
    a.base.dy = g->dy;
    a.base.c = g->c;
    a.base.fs = g->fs;
    a.base.fc = g->fc;
    a.base.sigma_f = d.sigma_f;
    a.base.sigma_t = d.sigma_t;
    a.base.tan_theta = g->theta > 0 ? std::tan(g->theta) : 0.0;
    a.base.x1 = pt->x;
    a.base.y1 = pt->y;
    a.base.z1 = pt->z;
    a.base.amp = pt->amp;
    a.t0 = d.t0;
    a.phase = pt->phase;
    int* dbins = nullptr;
    int8_t* dsig = nullptr;
    double2 *dbc = nullptr, *dxih = nullptr;
    double* dout = nullptr;
    std::vector<double> h((size_t)trials * 15);
    auto release = [&]() {
        if (dbins) (void)hipFree(dbins);
        if (dsig) (void)hipFree(dsig);
        if (dbc) (void)hipFree(dbc);
        if (dxih) (void)hipFree(dxih);
        if (dout) (void)hipFree(dout);
    };
    try {
        UFSS_HIP(hipMalloc(&dbins, (size_t)trials * per * sizeof(int)));
        UFSS_HIP(hipMalloc(&dsig, (size_t)ns));
        UFSS_HIP(hipMalloc(&dbc, (size_t)npos * nt * 5 * sizeof(double2)));
        UFSS_HIP(hipMalloc(&dxih, (size_t)ns * sizeof(double2)));
        UFSS_HIP(hipMalloc(&dout, (size_t)trials * 15 * sizeof(double)));
        UFSS_HIP(hipMemcpyAsync(dbins, bins, (size_t)trials * per * sizeof(int), hipMemcpyHostToDevice, s));
        UFSS_HIP(hipMemcpyAsync(dsig, signs, (size_t)ns, hipMemcpyHostToDevice, s));
        const int64_t nbc = (int64_t)npos * nt;
        hipLaunchKernelGGL(crb_bc_kernel, dim3((unsigned)std::min<int64_t>((nbc + 255) / 256, 65536)),
                           dim3(256), 0, s, a, dbc);
        UFSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(crb_signs_dft_kernel, dim3((unsigned)std::min<int64_t>((ns + 255) / 256, 65536)),
                           dim3(256), (size_t)nt * sizeof(double2), s, dsig, (int64_t)trials * srow, nt, dxih);
        UFSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(crb_fim_mixed_kernel, dim3(trials), dim3(256), 0, s, dbc, dxih, dbins, npos, nt,
                           m, per_position ? 1 : 0, per_position_signs ? 1 : 0, dout);
        UFSS_HIP(hipGetLastError());
        UFSS_HIP(hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        UFSS_HIP(hipStreamSynchronize(s));
    } catch (...) {
        release();
        throw;
    }
    release();
    const double scale = 2.0 / pt->sigma2;
    for (int t = 0; t < trials; ++t) {
        double J[25];
        unpack_fim(h.data() + (size_t)t * 15, scale, J);
        if (fim_out)
            for (int i = 0; i < 25; ++i) fim_out[(size_t)t * 25 + i] = J[i];
        crb_from_fim(J, crb_out + (size_t)t * 3);
    }
}

}  // namespace ufss
