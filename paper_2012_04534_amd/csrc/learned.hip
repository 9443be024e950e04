// Learned unrolled shrinkage network: forward, backward, training and inference.
//
// The network unrolls FISTA (paper Alg. 1) into S stages with learned step and
// threshold and a small 3-D convolutional correction; the operator A / A^H of
// the plan is a fixed layer.  Stage i (FISTA iteration i + 1):
//
//   gamma_i = x_i + beta_i (x_i - x_{i-1})           beta_0 = beta_1 = 0, then FISTA's
//   z_i     = gamma_i - s_i A^H (A gamma_i - y)      s_i = exp(rho_i) / L
//   u_i     = soft(z_i, theta_i)                      theta_i = exp(kappa_i) lam / L
//   x_{i+1} = u_i + c conv2(relu(conv1([Re u_i, Im u_i] / c))),  c = lam / L
//
// lam = mu max|A^H y| per measurement.  3x3x3 convolutions with zero padding
// over the [ny][nx][nz] grid, offset e = (e_y, e_x, e_z) indexed 9 (e_y + 1) +
// 3 (e_x + 1) + e_z + 1.  The scale c makes the network homogeneous in y; in
// the backward pass the c factors cancel except on the W2, b2 and b1
// gradients, which carry one factor c.  Backward: the linear layers are transposed
// (z = gamma - s A^H A gamma + const has the self-adjoint Jacobian
// I - s A^H A, run with the same A and A^H kernels), the complex soft
// threshold on R^2 has Jacobian I - theta (I/|z| - z z^T/|z|^3) for |z| > theta
// and 0 otherwise, d/dtheta = -z/|z|.  Parameter gradients are reduced in FP64
// in a fixed order (deterministic); Adam (Kingma & Ba) updates the FP32
// master weights.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace ufss {

static constexpr int kLT = 256;
static constexpr int kMaxCh = 8;

struct Dims {
    int nx, ny, nz;
    int64_t n;
};

static int nblk(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + kLT - 1) / kLT)); }

// Grid coordinates of voxel v, computed once per voxel in 32-bit arithmetic
// (a network's grid holds fewer than 2^31 voxels).
struct VoxC {
    int z, x, y;
};
__device__ __forceinline__ VoxC vox_coords(const Dims& d, int64_t v) {
    const int vi = (int)v, t = vi / d.nz;
    return VoxC{vi - t * d.nz, t % d.nx, t / d.nx};
}

// Neighbour w = v + e of voxel v (coordinates p) for offset index e; false
// outside the grid.  With the offset loops unrolled, e is a constant.
__device__ __forceinline__ bool nb(const Dims& d, const VoxC& p, int64_t v, int e, int64_t& w) {
    const int ez = e % 3 - 1, ex = (e / 3) % 3 - 1, ey = e / 9 - 1;
    if ((unsigned)(p.y + ey) >= (unsigned)d.ny || (unsigned)(p.x + ex) >= (unsigned)d.nx ||
        (unsigned)(p.z + ez) >= (unsigned)d.nz)
        return false;
    w = v + ((int64_t)ey * d.nx + ex) * d.nz + ez;
    return true;
}

// --- forward kernels ---------------------------------------------------------
__global__ __launch_bounds__(kLT) void k_momentum(int64_t n, const cf32* __restrict__ x,
                                                  const cf32* __restrict__ xp, float beta,
                                                  cf32* __restrict__ gam) {
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        cf32 a = x[i], b = xp[i];
        gam[i] = cf32{a.re + beta * (a.re - b.re), a.im + beta * (a.im - b.im)};
    }
}

// stage parameters at par: [rho, kappa, ...]
__global__ __launch_bounds__(kLT) void k_prox(int64_t n, const cf32* __restrict__ gam,
                                              const cf32* __restrict__ g, const float* __restrict__ par,
                                              float invL, const double* __restrict__ lam,
                                              cf32* __restrict__ z, cf32* __restrict__ u) {
    const float s = expf(par[0]) * invL;
    const float th = expf(par[1]) * (float)lam[0] * invL;
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        const cf32 a = gam[i], b = g[i];
        const float zr = a.re - s * b.re, zi = a.im - s * b.im;
        const float mag = sqrtf(zr * zr + zi * zi);
        const float sc = mag > th ? 1.0f - th / mag : 0.0f;
        z[i] = cf32{zr, zi};
        u[i] = cf32{zr * sc, zi * sc};
    }
}

// h[co][v] = relu(b1[co] + sum_{c, e} W1[co][c][e] u_c(v + e) / c),  c = lam / L
__global__ __launch_bounds__(kLT) void k_conv1(Dims d, int ch, const cf32* __restrict__ u,
                                               const float* __restrict__ W1, const float* __restrict__ b1,
                                               const double* __restrict__ lam, float invL,
                                               float* __restrict__ h) {
    const float ic = 1.0f / ((float)lam[0] * invL);
    __shared__ float w[kMaxCh * 54 + kMaxCh];
    for (int t = threadIdx.x; t < ch * 54; t += kLT) w[t] = W1[t];
    for (int t = threadIdx.x; t < ch; t += kLT) w[ch * 54 + t] = b1[t];
    __syncthreads();
    const float* uf = reinterpret_cast<const float*>(u);
    for (int64_t v = (int64_t)blockIdx.x * kLT + threadIdx.x; v < d.n; v += (int64_t)gridDim.x * kLT) {
        float acc[kMaxCh];
        for (int o = 0; o < ch; ++o) acc[o] = w[ch * 54 + o];
        const VoxC pc = vox_coords(d, v);
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            int64_t q;
            if (!nb(d, pc, v, e, q)) continue;
            const float ur = uf[2 * q] * ic, ui = uf[2 * q + 1] * ic;
            for (int o = 0; o < ch; ++o) acc[o] += w[o * 54 + e] * ur + w[o * 54 + 27 + e] * ui;
        }
        for (int o = 0; o < ch; ++o) h[(int64_t)o * d.n + v] = fmaxf(acc[o], 0.f);
    }
}

// xout = u + c (b2 + sum_{c, e} W2[o][c][e] h_c(v + e)) as complex (o = re, im)
__global__ __launch_bounds__(kLT) void k_conv2(Dims d, int ch, const float* __restrict__ h,
                                               const float* __restrict__ W2, const float* __restrict__ b2,
                                               const double* __restrict__ lam, float invL,
                                               const cf32* __restrict__ u, cf32* __restrict__ xout) {
    const float cs = (float)lam[0] * invL;
    __shared__ float w[2 * kMaxCh * 27 + 2];
    for (int t = threadIdx.x; t < 2 * ch * 27; t += kLT) w[t] = W2[t];
    if (threadIdx.x < 2) w[2 * ch * 27 + threadIdx.x] = b2[threadIdx.x];
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kLT + threadIdx.x; v < d.n; v += (int64_t)gridDim.x * kLT) {
        float ar = w[2 * ch * 27], ai = w[2 * ch * 27 + 1];
        const VoxC pc = vox_coords(d, v);
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            int64_t q;
            if (!nb(d, pc, v, e, q)) continue;
            for (int c = 0; c < ch; ++c) {
                const float hv = h[(int64_t)c * d.n + q];
                ar += w[c * 27 + e] * hv;
                ai += w[(ch + c) * 27 + e] * hv;
            }
        }
        const cf32 uu = u[v];
        xout[v] = cf32{uu.re + cs * ar, uu.im + cs * ai};
    }
}

// --- backward kernels ---------------------------------------------------------
__global__ __launch_bounds__(kLT) void k_loss_grad(int64_t n, const cf32* __restrict__ x,
                                                   const cf32* __restrict__ aref, const double* __restrict__ ref2,
                                                   cf32* __restrict__ dx, double* __restrict__ part) {
    __shared__ double red[kLT];
    const float sc = (float)(2.0 / ref2[0]);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        const cf32 a = x[i], b = aref[i];
        const float er = a.re - b.re, ei = a.im - b.im;
        dx[i] = cf32{sc * er, sc * ei};
        acc += (double)er * er + (double)ei * ei;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kLT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dh[c][v] = (h[c][v] > 0) * sum_{o, e} W2[o][c][e] dx_o(v - e)
__global__ __launch_bounds__(kLT) void k_conv2_bwd(Dims d, int ch, const cf32* __restrict__ dx,
                                                   const float* __restrict__ W2, const float* __restrict__ h,
                                                   float* __restrict__ dh) {
    __shared__ float w[2 * kMaxCh * 27];
    for (int t = threadIdx.x; t < 2 * ch * 27; t += kLT) w[t] = W2[t];
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kLT + threadIdx.x; v < d.n; v += (int64_t)gridDim.x * kLT) {
        float acc[kMaxCh];
        for (int c = 0; c < ch; ++c) acc[c] = 0.f;
        const VoxC pc = vox_coords(d, v);
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            int64_t q;
            if (!nb(d, pc, v, 26 - e, q)) continue;     // v - e
            const cf32 g = dx[q];
            for (int c = 0; c < ch; ++c) acc[c] += w[c * 27 + e] * g.re + w[(ch + c) * 27 + e] * g.im;
        }
        for (int c = 0; c < ch; ++c)
            dh[(int64_t)c * d.n + v] = h[(int64_t)c * d.n + v] > 0.f ? acc[c] : 0.f;
    }
}

// du = dx + sum_{o, e} W1[o][c][e] dh_o(v - e)
__global__ __launch_bounds__(kLT) void k_conv1_bwd(Dims d, int ch, const float* __restrict__ dh,
                                                   const float* __restrict__ W1, const cf32* __restrict__ dx,
                                                   cf32* __restrict__ du) {
    __shared__ float w[kMaxCh * 54];
    for (int t = threadIdx.x; t < ch * 54; t += kLT) w[t] = W1[t];
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * kLT + threadIdx.x; v < d.n; v += (int64_t)gridDim.x * kLT) {
        float ar = 0.f, ai = 0.f;
        const VoxC pc = vox_coords(d, v);
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            int64_t q;
            if (!nb(d, pc, v, 26 - e, q)) continue;
            for (int o = 0; o < ch; ++o) {
                const float gv = dh[(int64_t)o * d.n + q];
                ar += w[o * 54 + e] * gv;
                ai += w[o * 54 + 27 + e] * gv;
            }
        }
        const cf32 g = dx[v];
        du[v] = cf32{g.re + ar, g.im + ai};
    }
}

// Weight-gradient partials: block (r, oc) with oc = o * cin + c sums, over its
// voxel range r, dout_o(v) in_c(v + e) for the 27 offsets e and dout_o(v) (slot
// 27, the bias), into part[(oc * nsplit + r) * 28 + slot] in FP64.
// Channel accessors: value = base[c * cstride + v * vstride].
__global__ __launch_bounds__(kLT) void k_wgrad(Dims d, const float* __restrict__ dout, int64_t ocs,
                                               int ovs, const float* __restrict__ in, int64_t ics,
                                               int ivs, int cin, int nsplit, double* __restrict__ part) {
    __shared__ double red[28][kLT / 64];
    const int oc = blockIdx.y, o = oc / cin, c = oc % cin;
    const int64_t chunk = (d.n + nsplit - 1) / nsplit;
    const int64_t v0 = (int64_t)blockIdx.x * chunk, v1 = std::min<int64_t>(d.n, v0 + chunk);
    float acc[28];
    for (int e = 0; e < 28; ++e) acc[e] = 0.f;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += kLT) {
        const float g = dout[o * ocs + v * ovs];
        if (g == 0.f) continue;
        const VoxC pc = vox_coords(d, v);
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            int64_t q;
            if (nb(d, pc, v, e, q)) acc[e] += g * in[c * ics + q * ivs];
        }
        acc[27] += g;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = 0; e < 28; ++e) {
        double x = acc[e];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[e][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 28) {
        double s = 0.0;
        for (int i = 0; i < kLT / 64; ++i) s += red[threadIdx.x][i];
        part[((int64_t)oc * nsplit + blockIdx.x) * 28 + threadIdx.x] = s;
    }
}

// grad[(o * cin + c) * 27 + e] += sum over the ranges of the partials (fixed
// order); bias[o] += the slot-27 sum of channel 0; each optionally times
// c = lam / L (the correction's scale, see the stage definition).
__global__ void k_wgrad_sum(const double* __restrict__ part, int nsplit, int cin,
                            float* __restrict__ gW, float* __restrict__ gb,
                            const double* __restrict__ lam, float invL, int scale_w, int scale_b) {
    const int oc = blockIdx.x, o = oc / cin, c = oc % cin, e = threadIdx.x;
    if (e >= 28) return;
    const double cs = lam[0] * (double)invL;
    double s = 0.0;
    for (int r = 0; r < nsplit; ++r) s += part[((int64_t)oc * nsplit + r) * 28 + e];
    if (e < 27) gW[oc * 27 + e] += (float)(scale_w ? cs * s : s);
    else if (c == 0) gb[o] += (float)(scale_b ? cs * s : s);
}

// Voxel ranges per weight-gradient launch: about 16 voxels per thread, at
// most kWgSplit ranges (with 2 ch <= 16 (o, c) pairs, up to 2048 workgroups).
static constexpr int kWgSplit = 128;
static int wgrad_split(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kWgSplit, (n + 16 * kLT - 1) / (16 * kLT)));
}

// Soft-threshold backward and the step-size gradient partials.
__global__ __launch_bounds__(kLT) void k_soft_bwd(int64_t n, const cf32* __restrict__ z,
                                                  const cf32* __restrict__ du, const cf32* __restrict__ g,
                                                  const float* __restrict__ par, float invL,
                                                  const double* __restrict__ lam, cf32* __restrict__ dz,
                                                  double* __restrict__ part) {
    __shared__ double red[2][kLT];
    const float th = expf(par[1]) * (float)lam[0] * invL;
    double a_th = 0.0, a_s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        const cf32 zz = z[i], d = du[i];
        const float mag = sqrtf(zz.re * zz.re + zz.im * zz.im);
        cf32 o{0.f, 0.f};
        if (mag > th) {
            const float inv = 1.0f / mag;
            const float zd = zz.re * d.re + zz.im * d.im;
            const float k3 = th * zd * inv * inv * inv;
            o.re = d.re - th * inv * d.re + k3 * zz.re;
            o.im = d.im - th * inv * d.im + k3 * zz.im;
            a_th += -(double)zd * inv;
        }
        dz[i] = o;
        const cf32 gg = g[i];
        a_s += -((double)o.re * gg.re + (double)o.im * gg.im);
    }
    red[0][threadIdx.x] = a_th;
    red[1][threadIdx.x] = a_s;
    __syncthreads();
    for (int off = kLT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

// d gamma = dz - s (A^H A dz); dx_i += (1 + beta) d gamma; dx_{i-1} -= beta d gamma
__global__ __launch_bounds__(kLT) void k_dgamma(int64_t n, const cf32* __restrict__ dz,
                                                const cf32* __restrict__ ahadz, const float* __restrict__ par,
                                                float invL, float beta, cf32* __restrict__ dxi,
                                                cf32* __restrict__ dxim1) {
    const float s = expf(par[0]) * invL;
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        const cf32 a = dz[i], b = ahadz[i];
        const float gr = a.re - s * b.re, gi = a.im - s * b.im;
        cf32 x = dxi[i];
        dxi[i] = cf32{x.re + (1.f + beta) * gr, x.im + (1.f + beta) * gi};
        if (dxim1) {
            cf32 y = dxim1[i];
            dxim1[i] = cf32{y.re - beta * gr, y.im - beta * gi};
        }
    }
}

// grad[rho] += s * ds, grad[kappa] += theta * dtheta (sums of the partials, fixed order)
__global__ void k_scalar_grads(const double* __restrict__ part, int nb, const float* __restrict__ par,
                               float invL, const double* __restrict__ lam, float* __restrict__ grad) {
    __shared__ double red[2][kLT];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += kLT) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = kLT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = exp((double)par[0]) * invL;
        const double th = exp((double)par[1]) * lam[0] * invL;
        grad[0] += (float)(red[1][0] * s);
        grad[1] += (float)(red[0][0] * th);
    }
}

__global__ __launch_bounds__(kLT) void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr,
                                              float gscale, float b1t, float b2t, int64_t t) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t i = (int64_t)blockIdx.x * kLT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLT) {
        const float gg = g[i] * gscale;
        const float mm = b1 * m[i] + (1.f - b1) * gg;
        const float vv = b2 * v[i] + (1.f - b2) * gg * gg;
        m[i] = mm;
        v[i] = vv;
        p[i] -= lr * (mm / b1t) / (sqrtf(vv / b2t) + eps);
    }
    (void)t;
}

__global__ void k_mul_scalar(double* x, double f) {
    if (threadIdx.x == 0) x[0] *= f;
}

// --- network object -----------------------------------------------------------
struct Net {
    Plan* P = nullptr;
    int S = 0, ch = 0, sn = 0;
    double L = 0, mu = 0;
    int64_t np = 0;
    float *d_par = nullptr, *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
    int64_t adam_t = 0;
    std::vector<cf32*> x, gam, g, z, u, dxs;
    std::vector<float*> h;
    cf32 *du = nullptr, *dz = nullptr, *tmp = nullptr, *rtmp = nullptr;
    float* dh = nullptr;
    double *d_lam = nullptr, *d_part = nullptr, *d_sc = nullptr, *d_wpart = nullptr;
    std::vector<float> beta;
    std::vector<void*> owned;
};

template <class T>
static T* nalloc(Net& N, size_t count) {
    void* p = nullptr;
    UFSS_HIP(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
    N.owned.push_back(p);
    return static_cast<T*>(p);
}

static void net_free(Net* N) {
    if (!N) return;
    for (void* p : N->owned) (void)hipFree(p);
    delete N;
}

static int stage_size(int ch) { return 2 + ch * 54 + ch + 2 * ch * 27 + 2; }

Net* net_create(Plan* P, int S, int ch, double L, double mu, uint64_t seed) {
    if (!P) fail(UFSS_ERR_INVALID_ARG, "plan is NULL");
    if (S < 1 || S > 256 || ch < 1 || ch > kMaxCh) fail(UFSS_ERR_INVALID_ARG, "stages in [1,256], channels in [1,8]");
    if (P->nvox >= (int64_t(1) << 31)) fail(UFSS_ERR_UNSUPPORTED, "the network needs fewer than 2^31 voxels");
    if (!(L > 0) || !(mu > 0)) fail(UFSS_ERR_INVALID_ARG, "L and mu must be positive");
    Net* N = new Net();
    try {
        N->P = P;
        N->S = S;
        N->ch = ch;
        N->sn = stage_size(ch);
        N->L = L;
        N->mu = mu;
        N->np = (int64_t)S * N->sn;
        const int64_t nv = P->nvox, nm = (int64_t)P->npos * P->m;
        N->d_par = nalloc<float>(*N, N->np);
        N->d_grad = nalloc<float>(*N, N->np);
        N->d_m = nalloc<float>(*N, N->np);
        N->d_v = nalloc<float>(*N, N->np);
        for (int i = 0; i <= S; ++i) {
            N->x.push_back(nalloc<cf32>(*N, nv));
            N->dxs.push_back(nalloc<cf32>(*N, nv));
        }
        for (int i = 0; i < S; ++i) {
            N->gam.push_back(nalloc<cf32>(*N, nv));
            N->g.push_back(nalloc<cf32>(*N, nv));
            N->z.push_back(nalloc<cf32>(*N, nv));
            N->u.push_back(nalloc<cf32>(*N, nv));
            N->h.push_back(nalloc<float>(*N, (size_t)ch * nv));
        }
        N->du = nalloc<cf32>(*N, nv);
        N->dz = nalloc<cf32>(*N, nv);
        N->tmp = nalloc<cf32>(*N, nv);
        N->rtmp = nalloc<cf32>(*N, nm);
        N->dh = nalloc<float>(*N, (size_t)ch * nv);
        N->d_lam = nalloc<double>(*N, 4);
        N->d_part = nalloc<double>(*N, 4096);
        N->d_sc = nalloc<double>(*N, 16);
        N->d_wpart = nalloc<double>(*N, (size_t)2 * kMaxCh * kWgSplit * 28);
        // FISTA momentum weights (stage i = iteration i + 1)
        double t = 1.0;
        for (int i = 0; i < S; ++i) {
            double b = 0.0;
            if (i > 0) {
                const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
                b = (t - 1.0) / tn;
                t = tn;
            }
            N->beta.push_back((float)b);
        }
        // initial parameters: rho = kappa = 0, W1 ~ N(0, 0.1^2) (SplitMix64 + Box-Muller), rest 0
        std::vector<float> h((size_t)N->np, 0.f);
        uint64_t st = seed;
        auto next = [&]() {
            st += 0x9E3779B97F4A7C15ull;
            uint64_t zz = st;
            zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ull;
            zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBull;
            return zz ^ (zz >> 31);
        };
        for (int i = 0; i < S; ++i)
            for (int k = 0; k < ch * 54; ++k) {
                const double u1 = ((next() >> 11) + 1.0) * 0x1.0p-53, u2 = (next() >> 11) * 0x1.0p-53;
                h[(size_t)i * N->sn + 2 + k] = (float)(0.1 * std::sqrt(-2.0 * std::log(u1)) * std::cos(2 * M_PI * u2));
            }
        UFSS_HIP(hipMemcpy(N->d_par, h.data(), N->np * sizeof(float), hipMemcpyHostToDevice));
        UFSS_HIP(hipMemset(N->d_grad, 0, N->np * sizeof(float)));
        UFSS_HIP(hipMemset(N->d_m, 0, N->np * sizeof(float)));
        UFSS_HIP(hipMemset(N->d_v, 0, N->np * sizeof(float)));
        UFSS_HIP(hipMemset(N->x[0], 0, nv * sizeof(cf32)));
    } catch (...) {
        net_free(N);
        throw;
    }
    return N;
}

void net_destroy(Net* N) {
    if (!N) fail(UFSS_ERR_INVALID_ARG, "net is NULL");
    UFSS_HIP(hipDeviceSynchronize());
    net_free(N);
}

static Dims dims_of(const Net& N) {
    return Dims{N.P->g.nx, N.P->g.ny, N.P->g.nz, N.P->nvox};
}

// Forward pass; activations kept for the backward pass.  Result in N.x[S].
static void net_forward(Net& N, const cf32* y, hipStream_t s) {
    Plan& P = *N.P;
    const int64_t n = P.nvox;
    const float invL = (float)(1.0 / N.L);
    // lam = mu max |A^H y|
    op_adjoint(P, y, N.tmp, s);
    int nb = launch_absmax(n, N.tmp, N.d_part, s);
    launch_reduce_max(N.d_part, nb, N.d_lam, s);
    hipLaunchKernelGGL(k_mul_scalar, dim3(1), dim3(64), 0, s, N.d_lam, N.mu);
    const Dims d = dims_of(N);
    const int ch = N.ch;
    for (int i = 0; i < N.S; ++i) {
        const float* par = N.d_par + (int64_t)i * N.sn;
        const cf32* xprev = i > 0 ? N.x[i - 1] : N.x[0];
        hipLaunchKernelGGL(k_momentum, dim3(nblk(n)), dim3(kLT), 0, s, n, N.x[i], xprev, N.beta[i], N.gam[i]);
        op_forward(P, N.gam[i], P.d_r, y, nullptr, s);
        op_adjoint(P, P.d_r, N.g[i], s);
        hipLaunchKernelGGL(k_prox, dim3(nblk(n)), dim3(kLT), 0, s, n, N.gam[i], N.g[i], par, invL,
                           N.d_lam, N.z[i], N.u[i]);
        hipLaunchKernelGGL(k_conv1, dim3(nblk(n)), dim3(kLT), 0, s, d, ch, N.u[i], par + 2,
                           par + 2 + ch * 54, N.d_lam, invL, N.h[i]);
        hipLaunchKernelGGL(k_conv2, dim3(nblk(n)), dim3(kLT), 0, s, d, ch, N.h[i],
                           par + 2 + ch * 54 + ch, par + 2 + ch * 54 + ch + 2 * ch * 27, N.d_lam, invL,
                           N.u[i], N.x[i + 1]);
    }
    UFSS_HIP(hipGetLastError());
}

// Backward pass for one sample; accumulates into d_grad; loss into d_sc[0].
static void net_backward(Net& N, const cf32* aref, hipStream_t s) {
    Plan& P = *N.P;
    const int64_t n = P.nvox;
    const float invL = (float)(1.0 / N.L);
    const Dims d = dims_of(N);
    const int ch = N.ch;
    const int nsp = wgrad_split(n);
    int nb = launch_norm2(n, aref, P.d_part, s);
    launch_reduce(P.d_part, nb, 2, N.d_sc + 2, s);   // [2] = ||a_ref||^2
    for (int i = 0; i <= N.S; ++i) UFSS_HIP(hipMemsetAsync(N.dxs[i], 0, n * sizeof(cf32), s));
    const int nbl = nblk(n);
    hipLaunchKernelGGL(k_loss_grad, dim3(nbl), dim3(kLT), 0, s, n, N.x[N.S], aref, N.d_sc + 2,
                       N.dxs[N.S], N.d_part);
    launch_reduce(N.d_part, nbl, 1, N.d_sc + 0, s);   // [0] = ||x - a_ref||^2
    for (int i = N.S - 1; i >= 0; --i) {
        const float* par = N.d_par + (int64_t)i * N.sn;
        float* gpar = N.d_grad + (int64_t)i * N.sn;
        const float* W1 = par + 2;
        const float* W2 = par + 2 + ch * 54 + ch;
        float* gW1 = gpar + 2;
        float* gb1 = gpar + 2 + ch * 54;
        float* gW2 = gb1 + ch;
        float* gb2 = gW2 + 2 * ch * 27;
        // conv correction backward
        hipLaunchKernelGGL(k_conv2_bwd, dim3(nbl), dim3(kLT), 0, s, d, ch, N.dxs[i + 1], W2, N.h[i], N.dh);
        hipLaunchKernelGGL(k_wgrad, dim3(nsp, 2 * ch), dim3(kLT), 0, s, d,
                           reinterpret_cast<const float*>(N.dxs[i + 1]), (int64_t)1, 2, N.h[i], (int64_t)n, 1,
                           ch, nsp, N.d_wpart);
        hipLaunchKernelGGL(k_wgrad_sum, dim3(2 * ch), dim3(64), 0, s, N.d_wpart, nsp, ch, gW2, gb2,
                           N.d_lam, invL, 1, 1);
        hipLaunchKernelGGL(k_wgrad, dim3(nsp, ch * 2), dim3(kLT), 0, s, d, N.dh, (int64_t)n, 1,
                           reinterpret_cast<const float*>(N.u[i]), (int64_t)1, 2, 2, nsp, N.d_wpart);
        hipLaunchKernelGGL(k_wgrad_sum, dim3(ch * 2), dim3(64), 0, s, N.d_wpart, nsp, 2, gW1, gb1,
                           N.d_lam, invL, 0, 1);
        hipLaunchKernelGGL(k_conv1_bwd, dim3(nbl), dim3(kLT), 0, s, d, ch, N.dh, W1, N.dxs[i + 1], N.du);
        // soft threshold backward, theta / step partials
        hipLaunchKernelGGL(k_soft_bwd, dim3(nbl), dim3(kLT), 0, s, n, N.z[i], N.du, N.g[i], par, invL,
                           N.d_lam, N.dz, N.d_part);
        hipLaunchKernelGGL(k_scalar_grads, dim3(1), dim3(kLT), 0, s, N.d_part, nbl, par, invL, N.d_lam, gpar);
        // gamma backward through I - s A^H A
        op_forward(P, N.dz, N.rtmp, nullptr, nullptr, s);
        op_adjoint(P, N.rtmp, N.tmp, s);
        hipLaunchKernelGGL(k_dgamma, dim3(nbl), dim3(kLT), 0, s, n, N.dz, N.tmp, par, invL, N.beta[i],
                           N.dxs[i], i >= 1 ? N.dxs[i - 1] : nullptr);
    }
    UFSS_HIP(hipGetLastError());
}

void net_forward_out(Net& N, const cf32* y, cf32* x, hipStream_t s) {
    if (!y || !x) fail(UFSS_ERR_INVALID_ARG, "NULL buffer");
    net_forward(N, y, s);
    launch_copy(N.P->nvox, N.x[N.S], x, s);
}

double net_grad(Net& N, const cf32* y, const cf32* aref, int accumulate, hipStream_t s) {
    if (!y || !aref) fail(UFSS_ERR_INVALID_ARG, "NULL buffer");
    if (!accumulate) UFSS_HIP(hipMemsetAsync(N.d_grad, 0, N.np * sizeof(float), s));
    net_forward(N, y, s);
    net_backward(N, aref, s);
    double h[3];
    UFSS_HIP(hipMemcpyAsync(h, N.d_sc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    UFSS_HIP(hipStreamSynchronize(s));
    return h[0] / h[2];
}

double net_train_step(Net& N, int batch, const cf32* const* ys, const cf32* const* refs, double lr,
                      hipStream_t s) {
    if (batch < 1 || !ys || !refs) fail(UFSS_ERR_INVALID_ARG, "bad batch");
    UFSS_HIP(hipMemsetAsync(N.d_grad, 0, N.np * sizeof(float), s));
    double loss = 0.0;
    for (int b = 0; b < batch; ++b) loss += net_grad(N, ys[b], refs[b], 1, s);
    N.adam_t += 1;
    const double b1t = 1.0 - std::pow(0.9, (double)N.adam_t), b2t = 1.0 - std::pow(0.999, (double)N.adam_t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(N.np)), dim3(kLT), 0, s, N.np, N.d_par, N.d_grad, N.d_m, N.d_v,
                       (float)lr, (float)(1.0 / batch), (float)b1t, (float)b2t, N.adam_t);
    UFSS_HIP(hipGetLastError());
    UFSS_HIP(hipStreamSynchronize(s));
    return loss / batch;
}

void net_params(Net& N, float* get, const float* set, int64_t* count) {
    if (count) *count = N.np;
    if (set) UFSS_HIP(hipMemcpy(N.d_par, set, N.np * sizeof(float), hipMemcpyHostToDevice));
    if (get) UFSS_HIP(hipMemcpy(get, N.d_par, N.np * sizeof(float), hipMemcpyDeviceToHost));
}

void net_grads(Net& N, float* get) {
    if (get) UFSS_HIP(hipMemcpy(get, N.d_grad, N.np * sizeof(float), hipMemcpyDeviceToHost));
}

// Checkpoint: magic, stages, channels, L, mu, adam step, params, m, v.
void net_save(Net& N, const char* path) {
    if (!path) fail(UFSS_ERR_INVALID_ARG, "path is NULL");
    std::vector<float> p(N.np), m(N.np), v(N.np);
    UFSS_HIP(hipMemcpy(p.data(), N.d_par, N.np * 4, hipMemcpyDeviceToHost));
    UFSS_HIP(hipMemcpy(m.data(), N.d_m, N.np * 4, hipMemcpyDeviceToHost));
    UFSS_HIP(hipMemcpy(v.data(), N.d_v, N.np * 4, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) fail(UFSS_ERR_INVALID_ARG, std::string("cannot write ") + path);
    const char magic[8] = {'U', 'F', 'S', 'S', 'N', 'E', 'T', '1'};
    int32_t hdr[2] = {N.S, N.ch};
    double dd[2] = {N.L, N.mu};
    int64_t t = N.adam_t;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
              std::fwrite(dd, 8, 2, f) == 2 && std::fwrite(&t, 8, 1, f) == 1 &&
              std::fwrite(p.data(), 4, N.np, f) == (size_t)N.np &&
              std::fwrite(m.data(), 4, N.np, f) == (size_t)N.np &&
              std::fwrite(v.data(), 4, N.np, f) == (size_t)N.np;
    std::fclose(f);
    if (!ok) fail(UFSS_ERR_INVALID_ARG, "short write");
}

void net_load(Net& N, const char* path) {
    if (!path) fail(UFSS_ERR_INVALID_ARG, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) fail(UFSS_ERR_INVALID_ARG, std::string("cannot read ") + path);
    char magic[8];
    int32_t hdr[2];
    double dd[2];
    int64_t t;
    std::vector<float> p(N.np), m(N.np), v(N.np);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "UFSSNET1", 8) == 0 &&
              std::fread(hdr, 4, 2, f) == 2 && hdr[0] == N.S && hdr[1] == N.ch &&
              std::fread(dd, 8, 2, f) == 2 && std::fread(&t, 8, 1, f) == 1 &&
              std::fread(p.data(), 4, N.np, f) == (size_t)N.np &&
              std::fread(m.data(), 4, N.np, f) == (size_t)N.np &&
              std::fread(v.data(), 4, N.np, f) == (size_t)N.np;
    std::fclose(f);
    if (!ok) fail(UFSS_ERR_INVALID_ARG, "not a checkpoint of this network shape");
    UFSS_HIP(hipMemcpy(N.d_par, p.data(), N.np * 4, hipMemcpyHostToDevice));
    UFSS_HIP(hipMemcpy(N.d_m, m.data(), N.np * 4, hipMemcpyHostToDevice));
    UFSS_HIP(hipMemcpy(N.d_v, v.data(), N.np * 4, hipMemcpyHostToDevice));
    N.adam_t = t;
    N.L = dd[0];
    N.mu = dd[1];
}

}  // namespace ufss
