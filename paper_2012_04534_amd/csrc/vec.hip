// Elementwise and reduction kernels: the operator's pre/post passes, the fused
// FISTA update, and FP64 block reductions.
//
// All reductions are deterministic: a fixed grid of at most kMaxBlocks blocks
// walks the data in a fixed order, each block writes FP64 partials to its own
// slot, and a single-block kernel sums the slots in a fixed order.  No float
// atomics anywhere, so results are bitwise reproducible run to run.
#include <algorithm>

#include "internal.h"

namespace ufss {

static constexpr int kThreads = 256;
static constexpr int kMaxBlocks = 1024;

int max_blocks_vec() { return kMaxBlocks; }

static int blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    return (int)(b > kMaxBlocks ? kMaxBlocks : b);
}

// Block-wide FP64 sum of W values per thread; thread 0 writes part[blk*W + w].
template <int W>
__device__ void block_sum_write(double (&v)[W], double* part) {
    __shared__ double red[W][kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        double x = v[w];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[w][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            double s = 0.0;
            for (int i = 0; i < kThreads / 64; ++i) s += red[w][i];
            part[(int64_t)blockIdx.x * W + w] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward post pass: y[p][m] = H_sel * sum_s yraw[s][p][map(p, m)] (- ymeas),
// plus FP64 partials of ||y||^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void fwd_post_kernel(
    const cf32* __restrict__ yraw, int split, int64_t npos, int mu, int m, int per_pos,
    const int* __restrict__ map, const float* __restrict__ hsel, const cf32* __restrict__ ymeas,
    cf32* __restrict__ y, double* __restrict__ part) {
    double acc[1] = {0.0};
    const int64_t n = npos * m;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        int64_t p = i / m;
        int mi = (int)(i - p * m);
        int64_t sel = per_pos ? i : mi;
        int j = map[sel];
        float h = hsel[sel];
        const cf32 sum = sum_parts_ordered(yraw + p * mu + j, npos * mu, split);
        float re = sum.re * h, im = sum.im * h;
        if (ymeas) {
            cf32 q = ymeas[i];
            re -= q.re;
            im -= q.im;
        }
        y[i] = cf32{re, im};
        acc[0] += (double)re * re + (double)im * im;
    }
    block_sum_write<1>(acc, part);
}

int launch_forward_post(const Plan& P, cf32* y, const cf32* ymeas, double* part, hipStream_t s) {
    const int64_t n = (int64_t)P.npos * P.m;
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(fwd_post_kernel, dim3(nb), dim3(kThreads), 0, s, P.d_yraw,
                       P.fwd_split * std::max(1, P.fwd_zsplit),
                       (int64_t)P.npos, (int)P.ubins_h.size(), P.m, P.per_position, P.d_map,
                       P.d_hsel, ymeas, y, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

// ---------------------------------------------------------------------------
// Adjoint pre pass: one block per scan position writes the row
// rop[p][0..w) = 0 except rop[p][map(p, m)] = H_sel * r[p][m].
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ __launch_bounds__(128) void adj_pre_kernel(const cf32* __restrict__ r, int m, int w,
                                                      int per_pos, const int* __restrict__ map,
                                                      const float* __restrict__ hsel,
                                                      void* __restrict__ rop) {
    const int64_t p = blockIdx.x;
    if (BF16) {
        cbf16* row = static_cast<cbf16*>(rop) + p * w;
        for (int j = threadIdx.x; j < w; j += blockDim.x) row[j] = to_cbf16(0.f, 0.f);
        __syncthreads();
        for (int mi = threadIdx.x; mi < m; mi += blockDim.x) {
            int64_t sel = per_pos ? p * m + mi : mi;
            cf32 v = r[p * m + mi];
            float h = hsel[sel];
            row[map[sel]] = to_cbf16(h * v.re, h * v.im);
        }
    } else {
        cf32* row = static_cast<cf32*>(rop) + p * w;
        for (int j = threadIdx.x; j < w; j += blockDim.x) row[j] = cf32{0.f, 0.f};
        __syncthreads();
        for (int mi = threadIdx.x; mi < m; mi += blockDim.x) {
            int64_t sel = per_pos ? p * m + mi : mi;
            cf32 v = r[p * m + mi];
            float h = hsel[sel];
            row[map[sel]] = cf32{h * v.re, h * v.im};
        }
    }
}

void launch_adjoint_pre(const Plan& P, const cf32* r, hipStream_t s) {
    const int w = (P.algo == UFSS_ALGO_PHASOR) ? P.m : (int)P.ubins_h.size();
    if (P.dtype == UFSS_BF16 && P.algo == UFSS_ALGO_GEMM)     // BF16 operand of the BF16 GEMM
        hipLaunchKernelGGL(adj_pre_kernel<true>, dim3(P.npos), dim3(128), 0, s, r, P.m, w,
                           P.per_position, P.d_map, P.d_hsel, P.d_rop);
    else
        hipLaunchKernelGGL(adj_pre_kernel<false>, dim3(P.npos), dim3(128), 0, s, r, P.m, w,
                           P.per_position, P.d_map, P.d_hsel, P.d_rop);
    UFSS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kThreads) void to_bf16_kernel(const cf32* __restrict__ x,
                                                           cbf16* __restrict__ out,
                                                           int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 v = x[i];
        out[i] = to_cbf16(v.re, v.im);
    }
}

void launch_to_bf16(const cf32* x, void* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, x,
                       static_cast<cbf16*>(out), n);
    UFSS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Fused proximal-gradient update (FISTA / ISTA step), in place:
//   z = gamma - step g;  a_new = z max(0, 1 - thresh/|z|);
//   gamma <- a_new + beta (a_new - a);  a <- a_new.
// With nsplit > 1, g is the adjoint GEMM's split-K partials [nsplit][n], summed
// here in the same fixed order as sum_parts_kernel (the adjoint's epilogue).
// Partials: ||a_new||_1, ||gamma_new||_1, ||a_new - a||^2, ||a_new||^2,
// ||a_new - a_ref||^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void update_kernel(int64_t n, cf32* __restrict__ gamma,
                                                          const cf32* __restrict__ g, int nsplit,
                                                          cf32* __restrict__ a, float step,
                                                          float thresh, float beta, int real,
                                                          const cf32* __restrict__ aref,
                                                          double* __restrict__ part) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 gm = gamma[i], aa = a[i];
        cf32 gg = g[i];
        if (nsplit > 1) gg = sum_parts_ordered(g + i, n, nsplit);
        // real: the reflectivity is real, the gradient step keeps Re (Re{H} model)
        float zr = gm.re - step * gg.re, zi = real ? 0.f : gm.im - step * gg.im;
        float mag = sqrtf(zr * zr + zi * zi);
        float sc = mag > thresh ? 1.0f - thresh / mag : 0.0f;
        float ar = zr * sc, ai = zi * sc;
        float gr = ar + beta * (ar - aa.re), gi = ai + beta * (ai - aa.im);
        a[i] = cf32{ar, ai};
        gamma[i] = cf32{gr, gi};
        double dr = (double)ar - aa.re, di = (double)ai - aa.im;
        acc[0] += sqrt((double)ar * ar + (double)ai * ai);
        acc[1] += sqrt((double)gr * gr + (double)gi * gi);
        acc[2] += dr * dr + di * di;
        acc[3] += (double)ar * ar + (double)ai * ai;
        if (aref) {
            cf32 q = aref[i];
            double er = (double)ar - q.re, ei = (double)ai - q.im;
            acc[4] += er * er + ei * ei;
        }
    }
    block_sum_write<5>(acc, part);
}

int launch_update(int64_t n, cf32* gamma, const cf32* g, int nsplit, cf32* a, float step,
                  float thresh, float beta, const cf32* aref, double* part, hipStream_t s, int real) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(kThreads), 0, s, n, gamma, g, nsplit, a, step,
                       thresh, beta, real, aref, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

// ---------------------------------------------------------------------------
// Random mixing (Rademacher Sigma, Sec. III-A).  The plan's union holds every
// DFT index j of the A-scan spectrum B (signed bins), so y_raw[p][j] is B_p[j] / H_j.
//   post:  y[p][m] = sum_j xih[(k_m - j) mod nt] H_j y_raw[p][j]  (- ymeas)
//   pre:   rop[p][j] = H_j sum_m conj(xih[(k_m - j) mod nt]) r[p][m]
// with xih = F xi / nt the transformed signs of the position's row (nt is a
// power of two).  One workgroup per position at a time stages its rows in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void mix_post_kernel(
    const cf32* __restrict__ yraw, int split, int64_t npos, int nt, int m, int per_bins,
    const int* __restrict__ bins, const float* __restrict__ hu, const cf32* __restrict__ xih,
    int per_sign, const cf32* __restrict__ ymeas, cf32* __restrict__ y, double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char smem[];
    cf32* v = reinterpret_cast<cf32*>(smem);       // [nt] H_j y_raw[p][j]
    cf32* xr = v + nt;                             // [nt] transformed signs
    double acc[1] = {0.0};
    const int mask = nt - 1;
    for (int64_t p = blockIdx.x; p < npos; p += gridDim.x) {
        __syncthreads();
        const cf32* xs = xih + (per_sign ? p * nt : 0);
        for (int j = threadIdx.x; j < nt; j += kThreads) {
            const cf32 sum = sum_parts_ordered(yraw + p * nt + j, npos * nt, split);
            const float h = hu[j];
            v[j] = cf32{h * sum.re, h * sum.im};
            xr[j] = xs[j];
        }
        __syncthreads();
        const int* kb = bins + (per_bins ? p * m : 0);
        for (int mi = threadIdx.x; mi < m; mi += kThreads) {
            const int k = kb[mi];
            float re = 0.f, im = 0.f;
            for (int j = 0; j < nt; ++j) {
                const cf32 a = xr[(k - j) & mask], b = v[j];
                re += a.re * b.re - a.im * b.im;
                im += a.re * b.im + a.im * b.re;
            }
            const int64_t o = p * m + mi;
            if (ymeas) {
                re -= ymeas[o].re;
                im -= ymeas[o].im;
            }
            y[o] = cf32{re, im};
            acc[0] += (double)re * re + (double)im * im;
        }
    }
    block_sum_write<1>(acc, part);
}

int launch_mix_post(const Plan& P, cf32* y, const cf32* ymeas, double* part, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(P.npos, kMaxBlocks);
    const int nt = P.g.nt;
    hipLaunchKernelGGL(mix_post_kernel, dim3(nb), dim3(kThreads), (size_t)2 * nt * sizeof(cf32), s,
                       P.d_yraw, P.fwd_split * std::max(1, P.fwd_zsplit), (int64_t)P.npos, nt, P.m,
                       P.per_position, P.d_bins, P.d_hsel, static_cast<const cf32*>(P.d_xih),
                       P.mix_per_sign, ymeas, y, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

__global__ __launch_bounds__(kThreads) void mix_pre_kernel(
    const cf32* __restrict__ r, int64_t npos, int nt, int m, int per_bins,
    const int* __restrict__ bins, const float* __restrict__ hu, const cf32* __restrict__ xih,
    int per_sign, cf32* __restrict__ rop) {
    extern __shared__ __align__(16) unsigned char smem[];
    cf32* xr = reinterpret_cast<cf32*>(smem);      // [nt]
    cf32* rr = xr + nt;                            // [m]
    int* kk = reinterpret_cast<int*>(rr + m);      // [m]
    const int mask = nt - 1;
    for (int64_t p = blockIdx.x; p < npos; p += gridDim.x) {
        __syncthreads();
        const cf32* xs = xih + (per_sign ? p * nt : 0);
        for (int j = threadIdx.x; j < nt; j += kThreads) xr[j] = xs[j];
        const int* kb = bins + (per_bins ? p * m : 0);
        for (int mi = threadIdx.x; mi < m; mi += kThreads) {
            rr[mi] = r[p * m + mi];
            kk[mi] = kb[mi];
        }
        __syncthreads();
        for (int j = threadIdx.x; j < nt; j += kThreads) {
            float re = 0.f, im = 0.f;
            for (int mi = 0; mi < m; ++mi) {
                const cf32 a = xr[(kk[mi] - j) & mask], b = rr[mi];
                // conj(a) * b
                re += a.re * b.re + a.im * b.im;
                im += a.re * b.im - a.im * b.re;
            }
            const float h = hu[j];
            rop[p * nt + j] = cf32{h * re, h * im};
        }
    }
}

void launch_mix_pre(const Plan& P, const cf32* r, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(P.npos, kMaxBlocks);
    const int nt = P.g.nt;
    hipLaunchKernelGGL(mix_pre_kernel, dim3(nb), dim3(kThreads),
                       (size_t)nt * sizeof(cf32) + (size_t)P.m * (sizeof(cf32) + sizeof(int)), s, r,
                       (int64_t)P.npos, nt, P.m, P.per_position, P.d_bins, P.d_hsel,
                       static_cast<const cf32*>(P.d_xih), P.mix_per_sign, static_cast<cf32*>(P.d_rop));
    UFSS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Backtracking FISTA (Sec. IV-C): the proximal trial step at one constant L,
// p = soft(gamma - g / L, lam / L), with FP64 partials of
//   Re<p - gamma, g>, ||p - gamma||^2, ||p||_1, ||p - prev||^2, ||p||^2,
//   ||p - aref||^2 (0 without aref)
// for the sufficient-decrease test and the iteration statistics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void bt_prox_kernel(int64_t n,
                                                           const cf32* __restrict__ gamma,
                                                           const cf32* __restrict__ g, float step,
                                                           float thresh, cf32* __restrict__ p,
                                                           const cf32* __restrict__ prev,
                                                           const cf32* __restrict__ aref,
                                                           double* __restrict__ part) {
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 gm = gamma[i], gg = g[i], pv = prev[i];
        float zr = gm.re - step * gg.re, zi = gm.im - step * gg.im;
        float mag = sqrtf(zr * zr + zi * zi);
        float sc = mag > thresh ? 1.0f - thresh / mag : 0.0f;
        float ar = zr * sc, ai = zi * sc;
        p[i] = cf32{ar, ai};
        double dr = (double)ar - gm.re, di = (double)ai - gm.im;
        acc[0] += dr * gg.re + di * gg.im;
        acc[1] += dr * dr + di * di;
        acc[2] += sqrt((double)ar * ar + (double)ai * ai);
        double er = (double)ar - pv.re, ei = (double)ai - pv.im;
        acc[3] += er * er + ei * ei;
        acc[4] += (double)ar * ar + (double)ai * ai;
        if (aref) {
            cf32 q = aref[i];
            double fr = (double)ar - q.re, fi = (double)ai - q.im;
            acc[5] += fr * fr + fi * fi;
        }
    }
    block_sum_write<6>(acc, part);
}

int launch_bt_prox(int64_t n, const cf32* gamma, const cf32* g, float step, float thresh,
                   cf32* p, const cf32* prev, const cf32* aref, double* part, hipStream_t s) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(bt_prox_kernel, dim3(nb), dim3(kThreads), 0, s, n, gamma, g, step, thresh,
                       p, prev, aref, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

// out = a + beta (a - b) (FISTA extrapolation; by linearity also of residuals),
// with FP64 partials of ||out||^2.
__global__ __launch_bounds__(kThreads) void extrap_kernel(int64_t n, const cf32* __restrict__ a,
                                                          const cf32* __restrict__ b, float beta,
                                                          cf32* __restrict__ out,
                                                          double* __restrict__ part) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 u = a[i], v = b[i];
        float re = u.re + beta * (u.re - v.re), im = u.im + beta * (u.im - v.im);
        out[i] = cf32{re, im};
        acc[0] += (double)re * re + (double)im * im;
    }
    block_sum_write<1>(acc, part);
}

int launch_extrap(int64_t n, const cf32* a, const cf32* b, float beta, cf32* out, double* part,
                  hipStream_t s) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(extrap_kernel, dim3(nb), dim3(kThreads), 0, s, n, a, b, beta, out, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

// ---------------------------------------------------------------------------
// Fixed-order reductions.
// ---------------------------------------------------------------------------
// out[w] = sum over b of part[b][w] for w < width <= kRedW, one workgroup of
// kThreads, fixed order: thread t sums b = t, t + kThreads, ... per column,
// then one tree over the threads carries all columns at once (the same pairs
// as a tree per column, with one barrier per level for all of them).  Thread
// w < width writes out[w] (and keep[w] when given); every thread returns after
// the last barrier.
static constexpr int kRedW = 8;

__device__ __forceinline__ void block_reduce_cols(const double* __restrict__ part, int nblk,
                                                  int width, double* __restrict__ out,
                                                  double* red, double* keep) {
    double acc[kRedW];
#pragma unroll
    for (int w = 0; w < kRedW; ++w) acc[w] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
#pragma unroll
        for (int w = 0; w < kRedW; ++w)
            if (w < width) acc[w] += part[(int64_t)b * width + w];
    }
#pragma unroll
    for (int w = 0; w < kRedW; ++w)
        if (w < width) red[w * kThreads + threadIdx.x] = acc[w];
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int w = 0; w < width; ++w) red[w * kThreads + threadIdx.x] += red[w * kThreads + threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < width) {
        out[threadIdx.x] = red[threadIdx.x * kThreads];
        if (keep) keep[threadIdx.x] = red[threadIdx.x * kThreads];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ part,
                                                          int nblk, int width,
                                                          double* __restrict__ out) {
    __shared__ double red[kRedW * kThreads];
    block_reduce_cols(part, nblk, width, out, red, nullptr);
}

void launch_reduce(const double* part, int nblk, int width, double* out, hipStream_t s) {
    if (width < 1 || width > kRedW) fail(UFSS_ERR_INVALID_ARG, "reduction width must be in [1, 8]");
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, part, nblk, width, out);
    UFSS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kThreads) void absmax_kernel(int64_t n, const cf32* __restrict__ x,
                                                          double* __restrict__ part) {
    __shared__ double red[kThreads];
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 v = x[i];
        mx = fmax(mx, sqrt((double)v.re * v.re + (double)v.im * v.im));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int launch_absmax(int64_t n, const cf32* x, double* part, hipStream_t s) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(absmax_kernel, dim3(nb), dim3(kThreads), 0, s, n, x, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

__global__ __launch_bounds__(kThreads) void reduce_max_kernel(const double* __restrict__ part,
                                                              int nblk, double* __restrict__ out) {
    __shared__ double red[kThreads];
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) mx = fmax(mx, part[b]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

void launch_reduce_max(const double* part, int nblk, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_max_kernel, dim3(1), dim3(kThreads), 0, s, part, nblk, out);
    UFSS_HIP(hipGetLastError());
}

// Partials of ||x||^2 and ||x||_1.
__global__ __launch_bounds__(kThreads) void norm2_kernel(int64_t n, const cf32* __restrict__ x,
                                                         double* __restrict__ part) {
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 v = x[i];
        double q = (double)v.re * v.re + (double)v.im * v.im;
        acc[0] += q;
        acc[1] += sqrt(q);
    }
    block_sum_write<2>(acc, part);
}

int launch_norm2(int64_t n, const cf32* x, double* part, hipStream_t s) {
    const int nb = blocks_for(n);
    hipLaunchKernelGGL(norm2_kernel, dim3(nb), dim3(kThreads), 0, s, n, x, part);
    UFSS_HIP(hipGetLastError());
    return nb;
}

__global__ __launch_bounds__(kThreads) void scale_kernel(int64_t n, cf32* __restrict__ x,
                                                         const double* __restrict__ norm2) {
    const float inv = (float)(1.0 / sqrt(norm2[0]));
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        cf32 v = x[i];
        x[i] = cf32{v.re * inv, v.im * inv};
    }
}

void launch_scale(int64_t n, cf32* x, const double* norm2, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, x, norm2);
    UFSS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kThreads) void sum_parts_kernel(const cf32* __restrict__ part,
                                                             int nsplit, int64_t n,
                                                             cf32* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        out[i] = sum_parts_ordered(part + i, n, nsplit);
    }
}

void launch_sum_parts(const cf32* part, int nsplit, int64_t n, cf32* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, part, nsplit,
                       n, out);
    UFSS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kThreads) void copy_kernel(int64_t n, const cf32* __restrict__ src,
                                                        cf32* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

void launch_copy(int64_t n, const cf32* src, cf32* dst, hipStream_t s) {
    hipLaunchKernelGGL(copy_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, src, dst);
    UFSS_HIP(hipGetLastError());
}

// The residual's partials and the update's five partial columns reduced (each
// as reduce_kernel, same order) and the iteration's statistics, in one launch:
// res2_out <- ||A gamma_k - y||^2, upd_out <- the five sums
// {l1a, l1g, dA2, a2, ref2diff}, then with g1 = ||gamma_k||_1
//   stats[k] = {1/2 res2 + lam g1, sqrt(res2), sqrt(dA2 / a2), sqrt(ref2diff / ref2)}
// and g1 <- ||gamma_new||_1 for the next iteration.
__global__ __launch_bounds__(kThreads) void reduce_fista_stats_kernel(
    const double* __restrict__ res_part, int res_nblk, double* __restrict__ res2_out,
    const double* __restrict__ part, int nblk, double* __restrict__ upd_out, double* stats, int k,
    double* g1, double lam, int have_ref, double ref2) {
    __shared__ double red[kRedW * kThreads];
    __shared__ double upd[6];
    block_reduce_cols(res_part, res_nblk, 1, res2_out, red, upd + 5);
    block_reduce_cols(part, nblk, 5, upd_out, red, upd);
    if (threadIdx.x != 0) return;
    const double r2 = upd[5];
    double* st = stats + 4 * (int64_t)k;
    st[0] = 0.5 * r2 + lam * g1[0];
    st[1] = sqrt(r2);
    st[2] = upd[3] > 0.0 ? sqrt(upd[2] / upd[3]) : 0.0;
    st[3] = have_ref ? sqrt(upd[4] / ref2) : 0.0;
    g1[0] = upd[1];
}

void launch_reduce_fista_stats(const double* res_part, int res_nblk, double* res2_out,
                               const double* part, int nblk, double* upd_out, double* stats, int k,
                               double* g1, double lam, int have_ref, double ref2, hipStream_t s) {
    hipLaunchKernelGGL(reduce_fista_stats_kernel, dim3(1), dim3(kThreads), 0, s, res_part, res_nblk,
                       res2_out, part, nblk, upd_out, stats, k, g1, lam, have_ref, ref2);
    UFSS_HIP(hipGetLastError());
}

}  // namespace ufss
