// Synthetic scenes and measurements generated on the device (training and
// evaluation data of the learned solver: a scene and its noisy measurements
// never leave HBM).
//
// Scene: n distinct on-grid point scatterers with real amplitudes U[lo, hi]
// (drawn above `max_depth`), plus an optional back wall of amplitude 1 at one
// depth index.  Noise: circular complex Gaussian CN(0, s^2) per measured value
// with s^2 = ||A x||^2 / (count 10^(snr/10)), ||A x||^2 reduced in FP64 on the
// device.  Random numbers come from SplitMix64 (Steele, Lea & Flood 2014): the
// k-th output of the stream keyed `seed` is mix64(seed + k gamma), so element i
// of the noise reads outputs 2i + 1 and 2i + 2 independently of every other
// element (Box-Muller in FP64).  The scene draw is sequential: index j of
// scatterer j is floor(next() N / 2^64) over the N = ny nx max_depth allowed
// voxels, redrawn while it repeats an earlier one, then the amplitudes.
#include <cmath>

#include "internal.h"

namespace ufss {

static constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
static constexpr int kMaxScat = 4096;

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void zero_kernel(cf32* __restrict__ x, int64_t n, int nz, int back_wall) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % nz);
        x[i] = cf32{z == back_wall ? 1.0f : 0.0f, 0.0f};
    }
}

// One thread: the sequential draw (n <= kMaxScat; duplicates redrawn).
__global__ void scene_kernel(cf32* __restrict__ x, int nx, int nz, int max_depth, uint64_t nallow,
                             int n, double lo, double hi, uint64_t seed) {
    __shared__ uint64_t idx[kMaxScat];
    if (threadIdx.x != 0) return;
    uint64_t st = seed;
    for (int j = 0; j < n; ++j) {
        uint64_t v;
        bool dup;
        do {
            st += kGamma;
            v = __umul64hi(sm_mix(st), nallow);
            dup = false;
            for (int q = 0; q < j; ++q) dup = dup || idx[q] == v;
        } while (dup);
        idx[j] = v;
    }
    for (int j = 0; j < n; ++j) {
        st += kGamma;
        const double u = (double)(sm_mix(st) >> 11) * 0x1.0p-53;
        const uint64_t v = idx[j];
        const uint64_t per_row = (uint64_t)nx * max_depth;
        const uint64_t iy = v / per_row, rem = v - iy * per_row;
        const uint64_t ix = rem / max_depth, iz = rem - ix * max_depth;
        x[(iy * nx + ix) * nz + iz] = cf32{(float)(lo + (hi - lo) * u), 0.0f};
    }
}

// y += s n_i with s^2 = e2[0] / (count 10^(snr/10)); n_i ~ CN(0, 1) by Box-Muller.
__global__ void noise_kernel(cf32* __restrict__ y, int64_t count, const double* __restrict__ e2,
                             double snr_lin, uint64_t seed) {
    const double s = sqrt(e2[0] / ((double)count * snr_lin)) * 0.70710678118654752440;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = 2 * (uint64_t)i;
        const double u1 = ((double)(sm_mix(seed + (k + 1) * kGamma) >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
        const double u2 = (double)(sm_mix(seed + (k + 2) * kGamma) >> 11) * 0x1.0p-53;         // [0, 1)
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        const cf32 v = y[i];
        y[i] = cf32{(float)((double)v.re + s * r * cs), (float)((double)v.im + s * r * sn)};
    }
}

void synth_scene(const ufss_geom* g, int n, double lo, double hi, int max_depth, int back_wall,
                 uint64_t seed, cf32* x, hipStream_t s) {
    validate_geom_public(g);
    if (!x) fail(UFSS_ERR_INVALID_ARG, "x is NULL");
    if (n < 0 || n > kMaxScat) fail(UFSS_ERR_INVALID_ARG, "scatterer count must be in [0, 4096]");
    if (max_depth < 1 || max_depth > g->nz) fail(UFSS_ERR_INVALID_ARG, "max_depth must be in [1, nz]");
    if (back_wall >= g->nz) fail(UFSS_ERR_INVALID_ARG, "back wall below the grid");
    if (!(lo <= hi)) fail(UFSS_ERR_INVALID_ARG, "amplitude range must satisfy lo <= hi");
    const uint64_t nallow = (uint64_t)g->ny * g->nx * max_depth;
    if ((uint64_t)n > nallow) fail(UFSS_ERR_INVALID_ARG, "more scatterers than allowed voxels");
    const int64_t nv = (int64_t)g->ny * g->nx * g->nz;
    const int blocks = (int)std::min<int64_t>((nv + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, x, nv, g->nz, back_wall);
    hipLaunchKernelGGL(scene_kernel, dim3(1), dim3(64), 0, s, x, g->nx, g->nz, max_depth, nallow, n, lo,
                       hi, seed);
    UFSS_HIP(hipGetLastError());
}

void synth_measure(Plan& P, const cf32* x, double snr_db, uint64_t seed, cf32* y, hipStream_t s) {
    if (!x || !y) fail(UFSS_ERR_INVALID_ARG, "x and y must be device pointers");
    if (std::isnan(snr_db)) fail(UFSS_ERR_INVALID_ARG, "snr_db is NaN");
    double* e2 = P.d_scalars + 56;           // ||A x||^2 (FP64, device)
    op_forward(P, x, y, nullptr, e2, s);
    if (std::isinf(snr_db) && snr_db > 0) return;   // noise free
    const int64_t count = (int64_t)P.npos * P.m;
    const int blocks = (int)std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(noise_kernel, dim3(blocks), dim3(256), 0, s, y, count, e2,
                       std::pow(10.0, snr_db / 10.0), seed);
    UFSS_HIP(hipGetLastError());
}

}  // namespace ufss
