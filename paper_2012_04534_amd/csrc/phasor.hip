// Per-position frequency subsets: on-the-fly phasor path (FP32, VALU).
//
// When every A-scan keeps its own bins (the "f" strategies of the paper's
// Table I, Sec. III-A) the phase matrix differs per position, so the GEMM
// structure is lost; each term is generated where it is used:
//
//   forward  y[p, m] = H_{k_m(p)} sum_{v in W(p)} sum_z exp(-j 2 pi k_m(p) u(p - v, z)) x[v, z]
//   adjoint  x[v, z] = sum_{p in W(v)} sum_m exp(+j 2 pi k_m(p) u(p - v, z)) R[p, m]
//
// with R = H r prepared by the adjoint pre pass.  Forward: one workgroup per
// (position, group of bins: the selection's size rounded up to a power of two,
// at most 32); lanes stride the (voxel, depth) terms of the window with
// depth-contiguous, coalesced loads of x and of the delay table, the bins are
// wave-uniform scalars, and the per-lane sums are reduced across the wavefront
// with shuffles and across waves in LDS.  Adjoint: each lane owns one depth of
// one voxel column (64, 128 or 256 lanes per column), so no cross-lane
// reduction over depths is needed (the window's rows are split over the
// workgroup's waves), and the bins and operands of each position are
// wave-uniform scalar loads.
#include "internal.h"

namespace ufss {

static constexpr float kTwoM32 = 2.3283064365386963e-10f;

__device__ __forceinline__ void phasor_p(uint32_t ku, float& c, float& s) {
    float ph = (float)(int32_t)ku * kTwoM32;
    c = __builtin_amdgcn_cosf(ph);
    s = __builtin_amdgcn_sinf(ph);
}

// Bins per forward workgroup: the smallest power of two >= m, at most 32
// (a plan with more bins runs several groups of 32), so a position with one
// selected bin evaluates one phasor per term, not 32.
static constexpr int kMBMax = 32;
static int fwd_mb(int m) {
    int mb = 1;
    while (mb < m && mb < kMBMax) mb *= 2;
    return mb;
}

template <int MB>
__global__ __launch_bounds__(256) void fwd_phasor_kernel(
    const cf32* __restrict__ x, const uint32_t* __restrict__ ut, const float* __restrict__ amp,
    const int* __restrict__ bins, const float* __restrict__ hsel, const cf32* __restrict__ ymeas,
    cf32* __restrict__ y,
    double* __restrict__ part, int nx, int ny, int nz, int wx, int wy, int m, int ngroups) {
    __shared__ float red[2 * MB][4];
    const int p = blockIdx.x / ngroups, grp = blockIdx.x - p * ngroups;
    const int px = p % nx, py = p / nx;
    const int mb0 = grp * MB;
    uint32_t kb[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) kb[j] = (mb0 + j < m) ? (uint32_t)bins[(int64_t)p * m + mb0 + j] : 0u;

    const int vx_lo = max(px - wx, 0), vx_hi = min(px + wx, nx - 1);
    const int vy_lo = max(py - wy, 0), vy_hi = min(py + wy, ny - 1);
    const int nvx = vx_hi - vx_lo + 1;
    const int total = nvx * (vy_hi - vy_lo + 1) * nz;   // < 2^31 (host check)

    float acc_re[MB], acc_im[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) acc_re[j] = acc_im[j] = 0.f;

    // walk t = w * nz + z over the window's columns w = (cy, cx), updating
    // (cx, cy, z) incrementally: a step of 256 terms moves dcol columns and dz
    // depths (divided once), plus one column when the depth wraps.  The offset
    // of x moves by 256 per step plus (nx - nvx) nz per wrap to the next window
    // row; the delay-table row of |d_y| changes only on such a wrap.
    const int dcol = 256 / nz, dz = 256 - dcol * nz;
    const int rowjump = (nx - nvx) * nz, ustride = (wx + 1) * nz;
    int z = threadIdx.x % nz, cx = threadIdx.x / nz, cy = 0;
    while (cx >= nvx) { cx -= nvx; ++cy; }
    int xoff = ((vy_lo + cy) * nx + vx_lo + cx) * nz + z;
    int urow = (py > vy_lo + cy ? py - vy_lo - cy : vy_lo + cy - py) * ustride;
    const int pxr = px - vx_lo;                      // window column of the position
    for (int t = threadIdx.x; t < total; t += 256) {
        cf32 xv = x[xoff];
        const int adx = pxr > cx ? pxr - cx : cx - pxr;
        const int o = urow + adx * nz + z;
        const uint32_t u = ut[o];
        if (amp) {                       // Gaussian beam: g scales every bin's term
            const float gb = amp[o];
            xv.re *= gb;
            xv.im *= gb;
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            float c, s;
            phasor_p(kb[j] * u, c, s);
            // (xr + j xi)(c - j s)
            acc_re[j] += xv.re * c + xv.im * s;
            acc_im[j] += xv.im * c - xv.re * s;
        }
        xoff += 256;
        z += dz;
        cx += dcol;
        if (z >= nz) { z -= nz; ++cx; }
        if (cx >= nvx) {
            do {
                cx -= nvx;
                ++cy;
                xoff += rowjump;
            } while (cx >= nvx);
            const int vy = vy_lo + cy;
            urow = (py > vy ? py - vy : vy - py) * ustride;
        }
    }
    // reduce over the block
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        float a = acc_re[j], b = acc_im[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        if (lane == 0) {
            red[2 * j][wave] = a;
            red[2 * j + 1][wave] = b;
        }
    }
    __syncthreads();
    double r2 = 0.0;
    if (threadIdx.x < MB) {
        const int j = threadIdx.x, mi = mb0 + j;
        if (mi < m) {
            float re = (red[2 * j][0] + red[2 * j][1]) + (red[2 * j][2] + red[2 * j][3]);
            float im = (red[2 * j + 1][0] + red[2 * j + 1][1]) + (red[2 * j + 1][2] + red[2 * j + 1][3]);
            const int64_t o = (int64_t)p * m + mi;
            const float h = hsel[o];
            re *= h;
            im *= h;
            if (ymeas) {
                re -= ymeas[o].re;
                im -= ymeas[o].im;
            }
            y[o] = cf32{re, im};
            r2 = (double)re * re + (double)im * im;
        }
    }
    // partial |y|^2 of this block (threads >= MB contribute 0); fixed order
    if (threadIdx.x < 64) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off, 64);
        if (threadIdx.x == 0) part[blockIdx.x] = r2;
    }
}

void launch_forward_phasor(const Plan& P, const cf32* x, cf32* y, const cf32* ymeas,
                           double* part, hipStream_t s) {
    const int mb = fwd_mb(P.m);
    const int ngroups = (P.m + mb - 1) / mb;
    const int nblk = P.npos * ngroups;
    if (nblk > P.part_cap) fail(UFSS_ERR_UNSUPPORTED, "too many positions for the phasor path");
    // the forward walks the volume and the delay table with 32-bit offsets
    if ((int64_t)(P.npos + P.g.nx + 1) * P.g.nz + 256 > INT32_MAX ||
        (int64_t)(P.d.wy + 1) * (P.d.wx + 1) * P.g.nz > INT32_MAX)
        fail(UFSS_ERR_UNSUPPORTED, "volume too large for the phasor path");
#define UFSS_PF(MBV)                                                                              \
    hipLaunchKernelGGL(fwd_phasor_kernel<MBV>, dim3(nblk), dim3(256), 0, s, x, P.d_u, P.d_amp,    \
                       P.d_bins, P.d_hsel, ymeas, y, part, P.g.nx, P.g.ny, P.g.nz, P.d.wx, P.d.wy, \
                       P.m, ngroups)
    switch (mb) {
        case 1: UFSS_PF(1); break;
        case 2: UFSS_PF(2); break;
        case 4: UFSS_PF(4); break;
        case 8: UFSS_PF(8); break;
        case 16: UFSS_PF(16); break;
        default: UFSS_PF(32); break;
    }
#undef UFSS_PF
    UFSS_HIP(hipGetLastError());
}

int phasor_forward_blocks(const Plan& P) { return P.npos * ((P.m + fwd_mb(P.m) - 1) / fwd_mb(P.m)); }

// Adjoint lanes per voxel column: 64, 128 or 256 (the smallest that covers the
// depths, else 256 with several depth chunks).  A workgroup of 256 threads owns
// one (column, depth chunk); its 256 / lanes groups of lanes split the window's
// position rows between them and meet in LDS (fixed order), so a shallow grid
// still launches four waves per column to hide the load latency of the
// per-position operands.  Every wave stays on one column, so its bins and
// operands are uniform scalar loads.
static int adj_lanes(int nz) { return nz <= 64 ? 64 : (nz <= 128 ? 128 : 256); }

__global__ __launch_bounds__(256) void adj_phasor_kernel(
    const cf32* __restrict__ rop, const uint32_t* __restrict__ ut, const float* __restrict__ amp,
    const int* __restrict__ bins, cf32* __restrict__ out, int nx, int ny, int nz, int wx, int wy,
    int m, int nzc, int lanes) {
    __shared__ cf32 red[256];
    const int nsplit = 256 / lanes;                       // row splits per column
    const int64_t v = blockIdx.x / nzc;
    const int zc = (int)(blockIdx.x - v * nzc);
    const int vx = (int)(v % nx), vy = (int)(v / nx);
    // a wave never straddles two row splits (lanes is a multiple of 64): the
    // split index is wave-uniform
    const int sidx = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / lanes));
    const int zl0 = (int)(threadIdx.x % lanes);
    const int z = zc * lanes + zl0;
    const int zl = z < nz ? z : nz - 1;      // clamp for loads; store is guarded
    const int px_lo = max(vx - wx, 0), px_hi = min(vx + wx, nx - 1);
    const int py_lo = max(vy - wy, 0), py_hi = min(vy + wy, ny - 1);
    const int nrow = py_hi - py_lo + 1, rows_per = (nrow + nsplit - 1) / nsplit;
    const int r_lo = py_lo + sidx * rows_per, r_hi = min(py_hi, r_lo + rows_per - 1);
    float acc_re = 0.f, acc_im = 0.f;
    // one position's bins: (rr + j ri)(c + j s) summed over its selection
    auto position = [&](const int64_t prow, const uint32_t u, float& in_re, float& in_im) {
        // unrolled so that the scalar loads of two bins are requested together
#pragma unroll 2
        for (int mi = 0; mi < m; ++mi) {
            const uint32_t k = (uint32_t)bins[prow + mi];
            const cf32 rv = rop[prow + mi];
            float c, s;
            phasor_p(k * u, c, s);
            in_re += rv.re * c - rv.im * s;
            in_im += rv.re * s + rv.im * c;
        }
    };
    for (int py = r_lo; py <= r_hi; ++py) {
        const int ady = py > vy ? py - vy : vy - py;
        const int64_t obase = (int64_t)ady * (wx + 1) * nz + zl;
        const int64_t prow0 = (int64_t)py * nx * m;
        int px = px_lo;
        // four positions at a time: their delays and beams (vector loads) and,
        // with one bin per position, their bins and operands (scalar loads)
        // are all requested before the first is used
        for (; px + 3 <= px_hi; px += 4) {
            uint32_t u4[4];
            float g4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int adx = px + t > vx ? px + t - vx : vx - px - t;
                const int64_t o = obase + (int64_t)adx * nz;
                u4[t] = ut[o];
                g4[t] = amp ? amp[o] : 1.f;
            }
            if (m == 1) {
                uint32_t k4[4];
                cf32 r4[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    k4[t] = (uint32_t)bins[prow0 + px + t];
                    r4[t] = rop[prow0 + px + t];
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    float c, s;
                    phasor_p(k4[t] * u4[t], c, s);
                    const float in_re = r4[t].re * c - r4[t].im * s;
                    const float in_im = r4[t].re * s + r4[t].im * c;
                    acc_re += g4[t] * in_re;
                    acc_im += g4[t] * in_im;
                }
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    float in_re = 0.f, in_im = 0.f;
                    position(prow0 + (int64_t)(px + t) * m, u4[t], in_re, in_im);
                    acc_re += g4[t] * in_re;
                    acc_im += g4[t] * in_im;
                }
            }
        }
        for (; px <= px_hi; ++px) {
            const int adx = px > vx ? px - vx : vx - px;
            const int64_t o = obase + (int64_t)adx * nz;
            float in_re = 0.f, in_im = 0.f;
            position(prow0 + (int64_t)px * m, ut[o], in_re, in_im);
            const float gb = amp ? amp[o] : 1.f;
            acc_re += gb * in_re;
            acc_im += gb * in_im;
        }
    }
    if (nsplit > 1) {
        red[threadIdx.x] = cf32{acc_re, acc_im};
        __syncthreads();
        if (sidx != 0) return;
        for (int q = 1; q < nsplit; ++q) {
            const cf32 w = red[q * lanes + zl0];
            acc_re += w.re;
            acc_im += w.im;
        }
    }
    if (z < nz) out[v * nz + z] = cf32{acc_re, acc_im};
}

void launch_adjoint_phasor(const Plan& P, cf32* out, hipStream_t s) {
    const int lanes = adj_lanes(P.g.nz);
    const int nzc = (P.g.nz + lanes - 1) / lanes;
    const int64_t nblk = (int64_t)P.npos * nzc;
    if (nblk > 0x7fffffff) fail(UFSS_ERR_UNSUPPORTED, "too many voxel columns for the phasor path");
    hipLaunchKernelGGL(adj_phasor_kernel, dim3((unsigned)nblk), dim3(256), 0, s,
                       static_cast<const cf32*>(P.d_rop), P.d_u, P.d_amp, P.d_bins, out, P.g.nx, P.g.ny,
                       P.g.nz, P.d.wx, P.d.wy, P.m, nzc, lanes);
    UFSS_HIP(hipGetLastError());
}

}  // namespace ufss
