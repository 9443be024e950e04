// Windowed complex GEMM kernels for shared frequency subsets, FP32 on MFMA.
//
// The operator is block 2-level Toeplitz in the lateral offset d = p - v
// (paper Sec. IV-B, theorem on the structure of H): for one offset d it is a
// dense complex product between the phase matrix P_d[k, z] and the depth
// profiles of the voxels at p - d.  Instead of the paper's FFT-based
// correlation (Alg. 2) the window is summed directly, one small GEMM per
// offset, which puts the work on the matrix cores:
//
//   forward  Y[p, k] = sum_{d in W} sum_z  P_d[k, z] x[p - d, z]
//   adjoint  G[v, z] = sum_{d in W} sum_k  conj(P_d[k, z]) R[v + d, k]
//
// with P_d[k, z] = exp(-j 2 pi (k * u(|d|, z) mod 2^32) / 2^32), u the
// integer-turn delay table built by the plan.  H_k scaling, gathers for
// per-position subsets and residuals live in the small pre/post kernels.
//
// MFMA: v_mfma_f32_16x16x4_f32.  Lane l holds A[i = l%16][k = l/16],
// B[k = l/16][j = l%16] and D[i = 4(l/16) + r][j = l%16] for r = 0..3.
// Complex products use three real MFMAs on split real / imaginary parts
// (Gauss's form: one product of sums, two products with combined phasors).
//
// Tiling (both kernels): a workgroup of 4 waves owns one lateral tile of
// NP sub-tiles of 16 positions (sw x 16/sw each, sw = 4 for C-scans, 16 for
// B-scans).  Forward: each wave owns 16 bins, the 4 waves cover 64 bins.
// Adjoint: each wave owns NZ x 16 depths.  The shifted input rows for one d_y
// and one chunk of the reduction axis are staged in LDS (zero outside the
// grid); phasors are generated per lane in registers.  Accumulation is two
// level (per d_y in MFMA registers, then into an outer FP32 sum) to keep the
// FP32 error of ~1e5-term sums near 1e-6.
#include <type_traits>

#include "internal.h"

namespace ufss {

typedef float f4 __attribute__((ext_vector_type(4)));

static constexpr float kTwoM32 = 2.3283064365386963e-10f;   // 2^-32

// exp(-j 2 pi phi) components for the integer phase k*u (mod 2^32) in turns.
__device__ __forceinline__ void phasor(uint32_t ku, float& c, float& s) {
    float ph = (float)(int32_t)ku * kTwoM32;     // [-0.5, 0.5) turns
    c = __builtin_amdgcn_cosf(ph);              // cos(2 pi ph)
    s = __builtin_amdgcn_sinf(ph);              // sin(2 pi ph)
}

// Stages rows x hc cells of `chunk` consecutive complex values into LDS
// (cell stride cs, row pitch `pitch` cells), zero outside the grid or past
// `ilim` along the inner axis.  Grid row gy = ybase + r lands in row slot
// gy & slot_mask, so a window of slot_mask + 1 consecutive rows that moves by
// one row only needs the entering row staged:
//   halo[((gy & slot_mask) * pitch + c) * cs + e] = src[(gy * nx + xbase + c) * ld + i0 + e].
// `chunk` is a power of two dividing blockDim.x, so each thread keeps one inner
// index and walks the cells with a fixed step; UNR independent loads are in
// flight per thread before their LDS stores.
template <int UNR>
__device__ __forceinline__ void stage_halo(cf32* __restrict__ halo, int cs, int rows, int hc, int pitch, int slot_mask, int chunk,
                                           const cf32* __restrict__ src, int ny, int nx, int64_t ld,
                                           int ybase, int xbase, int i0, int ilim) {
    const int e = threadIdx.x & (chunk - 1);
    const int step = blockDim.x / chunk;
    const int total = rows * hc;
    int cell = threadIdx.x / chunk;
    int r = cell / hc, c = cell - r * hc;
    const bool eok = i0 + e < ilim;
    for (; cell < total; cell += UNR * step) {
        cf32 v[UNR];
        int dst[UNR];
        int rr = r, cc = c;
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            v[u] = cf32{0.f, 0.f};
            const int gy = ybase + rr, gx = xbase + cc;
            dst[u] = ((gy & slot_mask) * pitch + cc) * cs + e;
            if (cell + u * step < total && eok && gy >= 0 && gy < ny && gx >= 0 && gx < nx)
                v[u] = src[((int64_t)gy * nx + gx) * ld + i0 + e];
            cc += step;
            while (cc >= hc) { cc -= hc; ++rr; }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (cell + u * step < total) halo[dst[u]] = v[u];
        r = rr;
        c = cc;
    }
}

struct FwdArgs {
    const cf32* x;
    cf32* yraw;            // [split][npos][mu]
    const uint32_t* u;     // [wy+1][wx+1][nz]
    const float* amp;      // beam amplitude, same layout (DIR kernels only)
    const int* kb;         // [mu]
    int nx, ny, nz, wx, wy, mu;
    int sw;                // sub-tile width (4 or 16)
    int ntx, nty;          // lateral tiles
    int nbt;               // bin tiles of 16 * nw
    int nw;                // waves with a bin sub-tile (<= blockDim / 64)
    int ft;                // bins past the last full tile (1..4) folded into it, else 0
    int zc;                // depth chunk (multiple of 4)
    int split;             // split of the d_y range
    int zsplit;            // split of the depth range (partials = split * zsplit)
    int64_t npos;
    int nblk;              // blocks of this plan's grid
};

// ZC: the depth chunk a.zc as a compile-time constant (16, 8 or 4).
// DIR: scale each phasor by the beam amplitude g(|d_x|, |d_y|, z) (staged in
// LDS beside the delay table).
// FOLD: the plan folds a.ft tail bins into its last bin tile (below).
template <int NP, int ZC, bool DIR = false, bool FOLD = false>
__device__ __forceinline__ void fwd_f32_body(const FwdArgs& a, int b, const int nblk, unsigned char* smem) {
    constexpr int zc = ZC;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int sw = a.sw, sh = 16 / sw;
    const int tpx = sw * NP, tpy = sh;
    const int hc = tpx + 2 * a.wx;            // halo columns
    const int cs = zc + 1;                  // padded cell stride (complex)
    cf32* halo = reinterpret_cast<cf32*>(smem);
    uint32_t* ulds = reinterpret_cast<uint32_t*>(halo + (size_t)tpy * hc * cs);
    float* glds = reinterpret_cast<float*>(ulds + (size_t)(a.wx + 1) * zc);

    // block -> (split, bin tile, lateral tile); consecutive tiles of one split
    // and bin tile stay on one XCD (blocks are dealt round-robin to 8 XCDs).
    int per_xcd = nblk / 8;
    if (per_xcd * 8 == nblk) b = (b % 8) * per_xcd + b / 8;
    const int ntile = a.ntx * a.nty;
    const int tile = b % ntile;
    const int bt = (b / ntile) % a.nbt;
    const int sp_all = b / (ntile * a.nbt);          // partial index: (d_y part, depth part)
    const int sp = sp_all % a.split, spz = sp_all / a.split;
    const int px0 = (tile % a.ntx) * tpx, py0 = (tile / a.ntx) * tpy;
    const int zper = ((a.nz + zc * a.zsplit - 1) / (zc * a.zsplit)) * zc;
    const int z_lo = spz * zper, z_hi = min(a.nz, z_lo + zper);

    // d_y range of this split (rows that hit the grid for some tile row)
    int dy_lo = max(-a.wy, py0 - (a.ny - 1));
    int dy_hi = min(a.wy, py0 + tpy - 1);
    const int ndy = dy_hi - dy_lo + 1;
    const int chunk = (ndy + a.split - 1) / a.split;
    dy_lo += sp * chunk;
    dy_hi = min(dy_hi, dy_lo + chunk - 1);
    const int dx_lo = max(-a.wx, px0 - (a.nx - 1));
    const int dx_hi = min(a.wx, px0 + tpx - 1);

    const int bin0 = bt * 16 * a.nw + wave * 16;               // this wave's first bin
    const bool wave_active = wave < a.nw && bin0 < a.mu;
    const int i = lane & 15, ix = i % sw, iy = i / sw;
    const int kq = lane >> 4;
    // A wave left with at most 4 bins (the short last one of a union such as
    // 66 = 4 x 16 + 2) runs v_mfma_f32_4x4x1_16b_f32 instead: 16 blocks of a
    // 4 x 4 product with one depth each, the same rate per flop, a quarter of
    // the 16 x 16 x 4 cycles.  Its A operand is the same (lane l: position
    // l % 16, depth l / 16), its B operand takes bin l % 4 (block l / 4 =
    // (position group, depth)), and the four depth blocks of a position group
    // are summed across lanes at the end.
    const bool tail = wave_active && a.mu - bin0 <= 4;
    // Folded tail (four waves, a.ft bins past the last full bin tile, e.g. the
    // 2 of 66 = 64 + 2): the last tile's waves share those bins' products on the
    // same 4 x 4 x 1 form, wave w at the offsets d_x = w (mod 4), reusing the
    // A operands of their own products; the four partial sums meet in LDS at
    // the end.  Every wave keeps the same work per offset range, where a fifth
    // wave for the tail shares a SIMD with another wave.
    const bool fold = FOLD && bt == a.nbt - 1;
    const int tb = FOLD ? a.nbt * 16 * a.nw + (lane & 3) : 0;   // this lane's folded bin
    auto run = [&](auto tailc) {
        constexpr bool TAIL = decltype(tailc)::value;
        const int mb = bin0 + (TAIL ? (lane & 3) : (lane & 15));   // this lane's bin column
        const uint32_t kbin = (mb < a.mu) ? (uint32_t)a.kb[mb] : 0u;
        uint32_t kbt = 0u;
        if constexpr (FOLD) kbt = (fold && tb < a.mu) ? (uint32_t)a.kb[tb] : 0u;
        auto mfma = [](float av, float bv, f4 acc) {
            if constexpr (TAIL) return __builtin_amdgcn_mfma_f32_4x4x1f32(av, bv, acc, 0, 0, 0);
            else return __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
        };

        f4 out_re[NP], out_im[NP], t_re[FOLD ? NP : 1], t_im[FOLD ? NP : 1];
#pragma unroll
        for (int s = 0; s < NP; ++s) out_re[s] = out_im[s] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < (FOLD ? NP : 1); ++s) t_re[s] = t_im[s] = f4{0.f, 0.f, 0.f, 0.f};

        for (int z0 = z_lo; z0 < z_hi; z0 += zc) {
            for (int dy = dy_lo; dy <= dy_hi; ++dy) {
                __syncthreads();
                // stage x rows (py0 + r - dy), columns (px0 - wx + c), depths z0..z0+zc
                // rows live in slot (grid row mod tpy): after the first d_y only the row
                // entering the window is loaded
                stage_halo<8>(halo, cs, dy == dy_lo ? tpy : 1, hc, hc, tpy - 1, zc, a.x, a.ny, a.nx, a.nz,
                              py0 - dy, px0 - a.wx, z0, a.nz);
                const int ady = dy < 0 ? -dy : dy;
                for (int t = threadIdx.x; t < (a.wx + 1) * zc; t += blockDim.x) {
                    int adx = t / zc, zz = t - adx * zc;
                    int z = z0 + zz;
                    const int64_t o = ((int64_t)ady * (a.wx + 1) + adx) * a.nz + z;
                    ulds[t] = z < a.nz ? a.u[o] : 0u;
                    if (DIR) glds[t] = z < a.nz ? a.amp[o] : 0.f;
                }
                __syncthreads();
                if (!wave_active) continue;
                // Gauss's three-product form of (xr + j xi)(c - j s):
                //   m1 = c (xr + xi), m2 = xr (-s - c), m3 = xi (c - s);
                //   Re = m1 - m3 = xr c + xi s,  Im = m1 + m2 = xi c - xr s
                f4 m1[NP], m2[NP], m3[NP];
#pragma unroll
                for (int s = 0; s < NP; ++s) m1[s] = m2[s] = m3[s] = f4{0.f, 0.f, 0.f, 0.f};
                for (int dx = dx_lo; dx <= dx_hi; ++dx) {
                    const int adx = dx < 0 ? -dx : dx;
                    const uint32_t* urow = ulds + adx * zc;
                    const cf32* hrow = halo + ((((py0 + iy - dy) & (tpy - 1)) * hc) + ix + a.wx - dx) * cs;
                    // sub-tiles whose shifted columns all fall outside the grid add
                    // exact zeros: skip their MFMAs (wave-uniform test)
                    bool act[NP];
#pragma unroll
                    for (int s = 0; s < NP; ++s) {
                        const int c0 = px0 + s * sw - dx;
                        act[s] = c0 + sw - 1 >= 0 && c0 <= a.nx - 1;
                    }
                    float cz[zc / 4], bmz[zc / 4], bpz[zc / 4];
#pragma unroll
                    for (int j = 0; j < zc / 4; ++j) {
                        float c, sn;
                        phasor(kbin * urow[4 * j + kq], c, sn);
                        if (DIR) {
                            const float gv = glds[adx * zc + 4 * j + kq];
                            c *= gv;
                            sn *= gv;
                        }
                        cz[j] = c;
                        bmz[j] = -sn - c;
                        bpz[j] = c - sn;
                    }
#pragma unroll
                    for (int s = 0; s < NP; ++s) {
                        if (!act[s]) continue;
#pragma unroll
                        for (int j = 0; j < zc / 4; ++j) {
                            cf32 xv = hrow[s * sw * cs + 4 * j + kq];
                            m1[s] = mfma(xv.re + xv.im, cz[j], m1[s]);
                            m2[s] = mfma(xv.re, bmz[j], m2[s]);
                            m3[s] = mfma(xv.im, bpz[j], m3[s]);
                        }
                    }
                    if constexpr (FOLD && !TAIL) {
                        if (fold && (dx & 3) == wave) {
                            // (xr + j xi)(c - j s) for the folded bins, four real products;
                            // the wave's 4 bins x zc depths are one phasor per lane (bin
                            // l % 4, depth l / 4), handed to the lanes that take them
                            const int dz = min(lane >> 2, zc - 1);
                            float c0, s0;
                            phasor(kbt * urow[dz], c0, s0);
                            if (DIR) {
                                const float gv = glds[adx * zc + dz];
                                c0 *= gv;
                                s0 *= gv;
                            }
#pragma unroll
                            for (int j = 0; j < zc / 4; ++j) {
                                const int src = 4 * (4 * j + kq) + (lane & 3);
                                const float c = __shfl(c0, src, 64), sn = __shfl(s0, src, 64);
#pragma unroll
                                for (int s = 0; s < NP; ++s) {
                                    if (!act[s]) continue;
                                    const cf32 xv = hrow[s * sw * cs + 4 * j + kq];
                                    t_re[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(xv.re, c, t_re[s], 0, 0, 0);
                                    t_re[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(xv.im, sn, t_re[s], 0, 0, 0);
                                    t_im[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(xv.im, c, t_im[s], 0, 0, 0);
                                    t_im[s] = __builtin_amdgcn_mfma_f32_4x4x1f32(xv.re, -sn, t_im[s], 0, 0, 0);
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < NP; ++s) {
                    out_re[s] += m1[s] - m3[s];
                    out_im[s] += m1[s] + m2[s];
                }
            }
        }
        if constexpr (FOLD && !TAIL) {
            if (fold) {
                cf32* yo = a.yraw + (int64_t)sp_all * a.npos * a.mu;
                // the four waves' folded sums, added in wave order, then the four
                // depth blocks of each position group as in the tail wave below
                float* red = reinterpret_cast<float*>(smem);     // [4][NP][8][64]
                __syncthreads();                                 // halo reads done
                if (wave < 4) {
#pragma unroll
                    for (int s = 0; s < NP; ++s)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            red[((wave * NP + s) * 8 + r) * 64 + lane] = t_re[s][r];
                            red[((wave * NP + s) * 8 + 4 + r) * 64 + lane] = t_im[s][r];
                        }
                }
                __syncthreads();
                if (wave == 0) {
#pragma unroll
                    for (int s = 0; s < NP; ++s)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float vr = red[(s * 8 + r) * 64 + lane], vi = red[(s * 8 + 4 + r) * 64 + lane];
#pragma unroll
                            for (int w = 1; w < 4; ++w) {
                                vr += red[((w * NP + s) * 8 + r) * 64 + lane];
                                vi += red[((w * NP + s) * 8 + 4 + r) * 64 + lane];
                            }
                            vr += __shfl_xor(vr, 16, 64);
                            vi += __shfl_xor(vi, 16, 64);
                            vr += __shfl_xor(vr, 32, 64);
                            vi += __shfl_xor(vi, 32, 64);
                            const int irow = 4 * (lane >> 2) + r;
                            const int px = px0 + s * sw + irow % sw, py = py0 + irow / sw;
                            if (lane < 16 && tb < a.mu && px < a.nx && py < a.ny)
                                yo[((int64_t)py * a.nx + px) * a.mu + tb] = cf32{vr, vi};
                        }
                }
            }
        }
        if (!wave_active) return;
        cf32* yo = a.yraw + (int64_t)sp_all * a.npos * a.mu;
        if constexpr (TAIL) {
            // lane l holds rows r = 0..3 (positions 4 (l / 4 % 4) + r) of column
            // l % 4 of block l / 4; the blocks of depths 0..3 (lanes l, l ^ 16,
            // l ^ 32, l ^ 48) are summed in a fixed order
#pragma unroll
            for (int s = 0; s < NP; ++s)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    out_re[s][r] += __shfl_xor(out_re[s][r], 16, 64);
                    out_im[s][r] += __shfl_xor(out_im[s][r], 16, 64);
                    out_re[s][r] += __shfl_xor(out_re[s][r], 32, 64);
                    out_im[s][r] += __shfl_xor(out_im[s][r], 32, 64);
                }
            if (lane >= 16 || mb >= a.mu) return;
#pragma unroll
            for (int s = 0; s < NP; ++s) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int irow = 4 * (lane >> 2) + r;
                    const int px = px0 + s * sw + irow % sw, py = py0 + irow / sw;
                    if (px < a.nx && py < a.ny)
                        yo[((int64_t)py * a.nx + px) * a.mu + mb] = cf32{out_re[s][r], out_im[s][r]};
                }
            }
        } else {
            if (mb >= a.mu) return;
#pragma unroll
            for (int s = 0; s < NP; ++s) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int irow = 4 * kq + r;
                    int px = px0 + s * sw + irow % sw, py = py0 + irow / sw;
                    if (px < a.nx && py < a.ny)
                        yo[((int64_t)py * a.nx + px) * a.mu + mb] = cf32{out_re[s][r], out_im[s][r]};
                }
            }
        }
    };
    if (tail) run(std::true_type{});
    else run(std::false_type{});
}

template <int NP, int ZC, bool DIR = false, bool FOLD = false>
__global__ __launch_bounds__(512) void fwd_gemm_f32_kernel(FwdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    fwd_f32_body<NP, ZC, DIR, FOLD>(a, blockIdx.x, gridDim.x, smem);
}

// Grouped launch: block -> (plan index, block index inside that plan's grid).
template <int NP>
__global__ __launch_bounds__(512) void fwd_gemm_f32_kernel_grouped(const FwdArgs* __restrict__ descs,
                                                 const int2* __restrict__ blk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 sb = blk[blockIdx.x];
    const FwdArgs a = descs[sb.x];
    // scans of one batch may differ in depth chunk
    if (a.zc == 16) fwd_f32_body<NP, 16>(a, sb.y, a.nblk, smem);
    else if (a.zc == 8) fwd_f32_body<NP, 8>(a, sb.y, a.nblk, smem);
    else fwd_f32_body<NP, 4>(a, sb.y, a.nblk, smem);
}

struct AdjArgs {
    const cf32* r;         // H-scaled operand [npos][mu]
    cf32* out;             // [ny][nx][nz]
    const uint32_t* u;
    const float* amp;      // beam amplitude, same layout as u (DIR kernels only)
    const int* kb;
    int nx, ny, nz, wx, wy, mu;
    int sw, ntx, nty, nzt; // lateral tiles, depth tiles (of 64 * NZ)
    int kc;                // bin chunk (multiple of 4)
    int kcons;             // 1: the union's bins are consecutive integers (phasor rotation)
    int split;             // split of the d_y range; split > 1 writes partials
    cf32* part;            // [split][ny][nx][nz] when split > 1
    int64_t nvox;
    int nblk;              // blocks of this plan's grid
};

// KC: the bin chunk a.kc as a compile-time constant (16, 8 or 4).
// DIR: scale each phasor by the beam amplitude (staged in LDS after the bins).
// NW: waves per workgroup, each on its own 16 x NZ depths; the staged halo
// (positions x bins) is the same for every depth, so 8 waves share one halo
// over 128 depths where 4 waves cover 64.
template <int NP, int NZ, int KC, bool DIR = false, int NW = 4>
__device__ __forceinline__ void adj_f32_body(const AdjArgs& a, int b, const int nblk, unsigned char* smem) {
    constexpr int kc = KC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sw = a.sw, sh = 16 / sw;
    const int tpx = sw * NP, tpy = sh;
    const int hc = tpx + 2 * a.wx;
    const int cs = kc + 1;
    const int zspan = 16 * NW * NZ;                  // depths per workgroup
    cf32* halo = reinterpret_cast<cf32*>(smem);
    uint32_t* ulds = reinterpret_cast<uint32_t*>(halo + (size_t)tpy * hc * cs);
    int* klds = reinterpret_cast<int*>(ulds + (size_t)(a.wx + 1) * zspan);
    float* glds = reinterpret_cast<float*>(klds + kc);

    int per_xcd = nblk / 8;
    if (per_xcd * 8 == nblk) b = (b % 8) * per_xcd + b / 8;
    const int ntile = a.ntx * a.nty;
    const int tile = b % ntile;
    const int zt = (b / ntile) % a.nzt;
    const int sp = b / (ntile * a.nzt);
    const int vx0 = (tile % a.ntx) * tpx, vy0 = (tile / a.ntx) * tpy;
    const int zw0 = zt * zspan;                      // first depth of the workgroup

    // d with v + d inside the grid for some voxel of the tile, split in chunks
    int dy_lo = max(-a.wy, -(vy0 + tpy - 1));
    int dy_hi = min(a.wy, a.ny - 1 - vy0);
    const int chunk = (dy_hi - dy_lo + 1 + a.split - 1) / a.split;
    dy_lo += sp * chunk;
    dy_hi = min(dy_hi, dy_lo + chunk - 1);
    const int dx_lo = max(-a.wx, -(vx0 + tpx - 1)), dx_hi = min(a.wx, a.nx - 1 - vx0);

    const int i = lane & 15, ix = i % sw, iy = i / sw;
    const int kq = lane >> 4;
    const bool wave_active = zw0 + wave * NZ * 16 < a.nz;

    f4 out_re[NP][NZ], out_im[NP][NZ];
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
        for (int q = 0; q < NZ; ++q) out_re[s][q] = out_im[s][q] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < a.mu; k0 += kc) {
        const int kcur = min(kc, (a.mu - k0 + 3) & ~3);   // last chunk: valid bins, rounded to 4
        const bool pair = a.mu - k0 <= 2;                 // at most 2 bins left: two offsets per product
        for (int dy = dy_lo; dy <= dy_hi; ++dy) {
            __syncthreads();
            stage_halo<8>(halo, cs, dy == dy_lo ? tpy : 1, hc, hc, tpy - 1, kc, a.r, a.ny, a.nx, a.mu,
                          dy == dy_lo ? vy0 + dy : vy0 + dy + tpy - 1, vx0 - a.wx, k0, a.mu);
            const int ady = dy < 0 ? -dy : dy;
            for (int t = threadIdx.x; t < (a.wx + 1) * zspan; t += 64 * NW) {
                int adx = t / zspan, zz = t - adx * zspan;
                int z = zw0 + zz;
                const int64_t o = ((int64_t)ady * (a.wx + 1) + adx) * a.nz + z;
                ulds[t] = z < a.nz ? a.u[o] : 0u;
                if (DIR) glds[t] = z < a.nz ? a.amp[o] : 0.f;
            }
            for (int t = threadIdx.x; t < kc; t += 64 * NW)
                klds[t] = (k0 + t < a.mu) ? a.kb[k0 + t] : 0;
            __syncthreads();
            if (!wave_active) continue;
            // Gauss's three-product form of (rr + j ri)(c + j s):
            //   m1 = c (rr + ri), m2 = rr (s - c), m3 = ri (c + s);
            //   Re = m1 - m3 = rr c - ri s,  Im = m1 + m2 = rr s + ri c
            f4 m1[NP][NZ], m2[NP][NZ], m3[NP][NZ];
#pragma unroll
            for (int s = 0; s < NP; ++s)
#pragma unroll
                for (int q = 0; q < NZ; ++q) m1[s][q] = m2[s][q] = m3[s][q] = f4{0.f, 0.f, 0.f, 0.f};
            // the offsets of [d0, d1] with the sub-tiles of MASK active: with two
            // sub-tiles the range splits into (second only, both, first only),
            // and a sub-tile whose shifted columns all leave the grid runs no
            // MFMAs (compile-time masks keep the products branch-free); FULL: a
            // whole chunk of kc bins, so the offset step is one basic block whose
            // LDS reads and products the compiler can interleave (8-wave
            // workgroups only: with 4 waves the second copy of the offset loops
            // costs registers and measured 3% slower on the 64 x 64 C-scan and
            // in grouped launches)
            auto dxloop = [&](auto maskc, auto fullc, auto consc, const int d0, const int d1) {
                constexpr int MASK = decltype(maskc)::value;
                constexpr bool FULL = decltype(fullc)::value;
                constexpr bool CONS = decltype(consc)::value;
            for (int dx = d0; dx <= d1; ++dx) {
                const int adx = dx < 0 ? -dx : dx;
                uint32_t uz[NZ];
                float gz[NZ];
#pragma unroll
                for (int q = 0; q < NZ; ++q) {
                    uz[q] = ulds[adx * zspan + wave * NZ * 16 + q * 16 + i];
                    gz[q] = DIR ? glds[adx * zspan + wave * NZ * 16 + q * 16 + i] : 1.f;
                }
                const cf32* hrow = halo + ((((vy0 + iy + dy) & (tpy - 1)) * hc) + ix + a.wx + dx) * cs;
                // CONS (consecutive bins, whole chunk): lane group kq takes bins
                // k0 + kq + 4 j, so its phasor steps by exp(-j 2 pi 4 u) from one
                // bin step to the next: one rotation (4 FMAs) instead of a cos/sin
                // pair, whose issue does not hide under the products; the chain
                // restarts from cos/sin at every offset (3 rotations at most)
                float pc[NZ], ps[NZ], rc[NZ], rsn[NZ];
                if constexpr (CONS) {
                    const uint32_t k0l = (uint32_t)klds[kq];
#pragma unroll
                    for (int q = 0; q < NZ; ++q) {
                        phasor(k0l * uz[q], pc[q], ps[q]);
                        phasor(uz[q] << 2, rc[q], rsn[q]);
                    }
                }
#pragma unroll
                for (int kk = 0; kk < kc; kk += 4) {
                    if (!FULL && kk >= kcur) break;
                    const uint32_t k = (uint32_t)klds[kk + kq];
                    cf32 rv[NP];
                    float rs[NP];
#pragma unroll
                    for (int s = 0; s < NP; ++s) {
                        rv[s] = hrow[s * sw * cs + kk + kq];
                        rs[s] = rv[s].re + rv[s].im;
                    }
#pragma unroll
                    for (int q = 0; q < NZ; ++q) {
                        float c, sn;
                        if constexpr (CONS) {
                            c = pc[q];
                            sn = ps[q];
                            if (kk + 4 < kc) {
                                pc[q] = c * rc[q] - sn * rsn[q];
                                ps[q] = sn * rc[q] + c * rsn[q];
                            }
                        } else {
                            phasor(k * uz[q], c, sn);
                        }
                        if (DIR) {
                            c *= gz[q];
                            sn *= gz[q];
                        }
                        const float bm = sn - c, bp = c + sn;
#pragma unroll
                        for (int s = 0; s < NP; ++s) {
                            if (!((MASK >> s) & 1)) continue;
                            m1[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rs[s], c, m1[s][q], 0, 0, 0);
                            m2[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[s].re, bm, m2[s][q], 0, 0, 0);
                            m3[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[s].im, bp, m3[s][q], 0, 0, 0);
                        }
                    }
                }
            }
            };
            if (pair) {
                // a last chunk of at most 2 bins: the K = 4 of one product takes
                // those bins at two offsets, lane groups kq = 0, 1 at d_x and
                // kq = 2, 3 at d_x + 1 (zero past dx_hi), so the chunk runs half
                // the offset steps and no product lane carries a padding bin
                // (every sub-tile, out-of-grid cells are staged as zeros)
                const uint32_t k = (uint32_t)klds[kq & 1];
                for (int dx = dx_lo; dx <= dx_hi; dx += 2) {
                    const bool ok = dx + (kq >> 1) <= dx_hi;
                    const int dl = ok ? dx + (kq >> 1) : dx;
                    const int adl = dl < 0 ? -dl : dl;
                    const cf32* hrow = halo + ((((vy0 + iy + dy) & (tpy - 1)) * hc) + ix + a.wx + dl) * cs + (kq & 1);
                    cf32 rv[NP];
                    float rs[NP];
#pragma unroll
                    for (int s = 0; s < NP; ++s) {
                        rv[s] = ok ? hrow[s * sw * cs] : cf32{0.f, 0.f};
                        rs[s] = rv[s].re + rv[s].im;
                    }
#pragma unroll
                    for (int q = 0; q < NZ; ++q) {
                        float c, sn;
                        phasor(k * ulds[adl * zspan + wave * NZ * 16 + q * 16 + i], c, sn);
                        if (DIR) {
                            const float gv = glds[adl * zspan + wave * NZ * 16 + q * 16 + i];
                            c *= gv;
                            sn *= gv;
                        }
                        const float bm = sn - c, bp = c + sn;
#pragma unroll
                        for (int s = 0; s < NP; ++s) {
                            m1[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rs[s], c, m1[s][q], 0, 0, 0);
                            m2[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[s].re, bm, m2[s][q], 0, 0, 0);
                            m3[s][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[s].im, bp, m3[s][q], 0, 0, 0);
                        }
                    }
                }
            } else if constexpr (NP == 2) {
                // column ranges of the two sub-tiles' shifted voxels inside the grid
                const int a0 = -(vx0 + sw - 1), b1 = a.nx - 1 - vx0 - sw;
                auto segs = [&](auto fullc, auto consc) {
                    dxloop(std::integral_constant<int, 2>{}, fullc, consc, dx_lo, min(min(a0 - 1, b1), dx_hi));
                    dxloop(std::integral_constant<int, 3>{}, fullc, consc, max(dx_lo, a0), min(b1, dx_hi));
                    dxloop(std::integral_constant<int, 1>{}, fullc, consc, max(max(a0, b1 + 1), dx_lo), dx_hi);
                };
                if constexpr (NW == 8) {
                    if (kcur == kc) {                         // every chunk but a short last one
                        if (a.kcons) segs(std::true_type{}, std::true_type{});
                        else segs(std::true_type{}, std::false_type{});
                    } else {
                        segs(std::false_type{}, std::false_type{});
                    }
                } else {
                    segs(std::false_type{}, std::false_type{});
                }
            } else {
                dxloop(std::integral_constant<int, (1 << NP) - 1>{}, std::false_type{}, std::false_type{}, dx_lo, dx_hi);
            }
#pragma unroll
            for (int s = 0; s < NP; ++s)
#pragma unroll
                for (int q = 0; q < NZ; ++q) {
                    out_re[s][q] += m1[s][q] - m3[s][q];
                    out_im[s][q] += m1[s][q] + m2[s][q];
                }
        }
    }
    if (!wave_active) return;
    cf32* dst = a.split > 1 ? a.part + (int64_t)sp * a.nvox : a.out;
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
        for (int q = 0; q < NZ; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int irow = 4 * kq + r;
                int vx = vx0 + s * sw + irow % sw, vy = vy0 + irow / sw;
                int z = zw0 + wave * NZ * 16 + q * 16 + i;
                if (vx < a.nx && vy < a.ny && z < a.nz)
                    dst[((int64_t)vy * a.nx + vx) * a.nz + z] = cf32{out_re[s][q][r], out_im[s][q][r]};
            }
}

template <int NP, int NZ, int KC, bool DIR = false>
__global__ __launch_bounds__(256) void adj_gemm_f32_kernel(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    adj_f32_body<NP, NZ, KC, DIR>(a, blockIdx.x, gridDim.x, smem);
}

// Two sub-tiles per wave: registers capped for 6 waves per SIMD, which pays
// when a small LDS chunk admits that many workgroups per CU (measured on the
// 32 x 32 and 64 x 64 C-scans).  NW = 8: one halo for 128 depths, so the
// LDS of 8 waves is the halo plus twice the delay rows instead of twice both
// (on the 32 x 32 C-scan 3 workgroups per CU: 6 waves per SIMD, not 3).
template <int NZ, int KC, bool DIR = false, int NW = 4>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(6, 8)))
void adj_gemm_f32_kernel_np2(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    adj_f32_body<2, NZ, KC, DIR, NW>(a, blockIdx.x, gridDim.x, smem);
}

// Grouped launch: block -> (plan index, block index inside that plan's grid).
template <int NP, int NZ>
__global__ __launch_bounds__(256) void adj_gemm_f32_kernel_grouped(const AdjArgs* __restrict__ descs,
                                                 const int2* __restrict__ blk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 sb = blk[blockIdx.x];
    const AdjArgs a = descs[sb.x];
    if (a.kc == 16) adj_f32_body<NP, NZ, 16>(a, sb.y, a.nblk, smem);
    else if (a.kc == 8) adj_f32_body<NP, NZ, 8>(a, sb.y, a.nblk, smem);
    else adj_f32_body<NP, NZ, 4>(a, sb.y, a.nblk, smem);
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static constexpr int kGroupNP = 2;   // grouped (batched) launches: one shape for every scan

int fwd_tile_np(const Plan& P) { return P.fwd_np == 4 ? 4 : 2; }
int adj_tile_np(const Plan& P) { return P.adj_np == 4 ? 4 : 2; }
int adj_waves(const Plan& P) { return adj_tile_np(P) == 2 && P.adj_nw == 8 ? 8 : 4; }

static int fwd_args(const Plan& P, const cf32* x, FwdArgs& a, size_t& lds, int np, bool fold = true);
static int adj_args(const Plan& P, cf32* out, AdjArgs& a, size_t& lds, int np, int nw = 4);

int fwd_chunk(const Plan& P) {
    FwdArgs a;
    size_t lds;
    fwd_args(P, nullptr, a, lds, fwd_tile_np(P));
    return a.zc;
}

int adj_chunk(const Plan& P) {
    AdjArgs a;
    size_t lds;
    adj_args(P, nullptr, a, lds, adj_tile_np(P), adj_waves(P));
    return a.kc;
}
static constexpr int kAdjNZ = 1;
static constexpr size_t kLdsMax = 64 * 1024;

static int sub_width(const Plan& P) { return P.g.ny == 1 ? 16 : 4; }

int gemm_split(const Plan& P) {
    const int sw = sub_width(P), tpx = sw * fwd_tile_np(P), tpy = 16 / sw;
    const int ntx = (P.g.nx + tpx - 1) / tpx, nty = (P.g.ny + tpy - 1) / tpy;
    const int mu = (int)P.ubins_h.size();
    const int nbt = (mu + 63) / 64;
    const int nw = std::max(1, std::min(P.fwd_nw, (mu + 15) / 16));
    const int active_waves = ntx * nty * ((mu + 16 * nw - 1) / (16 * nw)) * nw;
    const int ndy_max = std::min(2 * P.d.wy + 1, P.g.ny + tpy - 1);
    int split = (2048 + active_waves - 1) / active_waves;
    split = std::max(1, std::min(split, std::min(ndy_max, 16)));
    const int chunk = (ndy_max + split - 1) / split;
    (void)nbt;
    return (ndy_max + chunk - 1) / chunk;      // no split left without rows
}

// Split of the adjoint's d_y range: enough workgroups to fill 256 CUs twice.
int adj_split(const Plan& P) {
    const int sw = sub_width(P), tpx = sw * adj_tile_np(P), tpy = 16 / sw;
    const int ntx = (P.g.nx + tpx - 1) / tpx, nty = (P.g.ny + tpy - 1) / tpy;
    const int nzt = (P.g.nz + 64 * kAdjNZ - 1) / (64 * kAdjNZ);
    const int wgs = ntx * nty * nzt;
    const int ndy_max = std::min(2 * P.d.wy + 1, P.g.ny + tpy - 1);
    int split = (512 + wgs - 1) / wgs;
    split = std::max(1, std::min(split, std::min(ndy_max, 8)));
    const int chunk = (ndy_max + split - 1) / split;
    return (ndy_max + chunk - 1) / chunk;
}

// Descriptor of one plan's forward GEMM launch; returns the block count.
// `fold`: allow the folded tail (single-plan launches; grouped launches keep
// one kernel body for every plan).
static int fwd_args(const Plan& P, const cf32* x, FwdArgs& a, size_t& lds, int np, bool fold) {
    a = FwdArgs{};
    a.x = x;
    a.yraw = P.d_yraw;
    a.u = P.d_u;
    a.amp = P.d_amp;
    a.kb = P.d_ubins;
    a.nx = P.g.nx;
    a.ny = P.g.ny;
    a.nz = P.g.nz;
    a.wx = P.d.wx;
    a.wy = P.d.wy;
    a.mu = (int)P.ubins_h.size();
    a.sw = sub_width(P);
    const int tpx = a.sw * np, tpy = 16 / a.sw;
    a.ntx = (a.nx + tpx - 1) / tpx;
    a.nty = (a.ny + tpy - 1) / tpy;
    a.nw = std::max(1, std::min(P.fwd_nw, (a.mu + 15) / 16));
    a.nbt = (a.mu + 16 * a.nw - 1) / (16 * a.nw);
    // four waves and at most 4 bins past the last full tile: fold them into it
    const int rem = a.mu % (16 * a.nw);
    a.ft = (fold && a.nw == 4 && a.mu > 64 && rem >= 1 && rem <= 4) ? rem : 0;
    if (a.ft) a.nbt = a.mu / 64;
    a.split = P.fwd_split;
    a.npos = P.npos;
    const int hc = tpx + 2 * a.wx;
    int zc = P.fwd_zc == 8 ? 8 : 16;
    const size_t tab = P.d_amp ? 8 : 4;      // delay (+ beam) table bytes per entry
    auto lds_of = [&](int z) {
        return (size_t)tpy * hc * (z + 1) * sizeof(cf32) + (size_t)(a.wx + 1) * z * tab;
    };
    while (zc > 4 && lds_of(zc) > kLdsMax) zc /= 2;   // powers of two: the staging needs zc | blockDim
    lds = lds_of(zc);
    if (lds > kLdsMax) fail(UFSS_ERR_UNSUPPORTED, "aperture window too wide for the GEMM path");
    if (a.ft) lds = std::max(lds, (size_t)4 * np * 8 * 64 * sizeof(float));   // the folded sums
    a.zc = zc;
    a.zsplit = std::max(1, P.fwd_zsplit);
    a.nblk = a.ntx * a.nty * a.nbt * a.split * a.zsplit;
    return a.nblk;
}

// nw: waves per workgroup (4, or 8 with two sub-tiles per wave), 16 depths each.
static int adj_args(const Plan& P, cf32* out, AdjArgs& a, size_t& lds, int np, int nw) {
    a = AdjArgs{};
    a.r = static_cast<const cf32*>(P.d_rop);
    a.out = out;
    a.u = P.d_u;
    a.amp = P.d_amp;
    a.kb = P.d_ubins;
    a.nx = P.g.nx;
    a.ny = P.g.ny;
    a.nz = P.g.nz;
    a.wx = P.d.wx;
    a.wy = P.d.wy;
    a.mu = (int)P.ubins_h.size();
    a.sw = sub_width(P);
    const int tpx = a.sw * np, tpy = 16 / a.sw;
    a.ntx = (a.nx + tpx - 1) / tpx;
    a.nty = (a.ny + tpy - 1) / tpy;
    const int zspan = 16 * nw * kAdjNZ;
    a.nzt = (a.nz + zspan - 1) / zspan;
    const int hc = tpx + 2 * a.wx;
    int kc = P.adj_kc == 8 ? 8 : 16;
    const size_t tab = P.d_amp ? 8 : 4;      // delay (+ beam) table bytes per entry
    auto lds_of = [&](int k) {
        return (size_t)tpy * hc * (k + 1) * sizeof(cf32) + (size_t)(a.wx + 1) * zspan * tab +
               (size_t)k * 4;
    };
    while (kc > 4 && lds_of(kc) > kLdsMax) kc /= 2;   // powers of two (staging)
    if (lds_of(kc) > kLdsMax) fail(UFSS_ERR_UNSUPPORTED, "aperture window too wide for the GEMM path");
    a.kc = kc;
    a.kcons = 1;                              // a band without gaps (the C-scan unions)
    for (size_t t = 1; t < P.ubins_h.size(); ++t)
        if (P.ubins_h[t] != P.ubins_h[t - 1] + 1) a.kcons = 0;
    lds = lds_of(kc);
    a.split = P.adj_split;
    a.part = P.d_gpart;
    a.nvox = P.nvox;
    a.nblk = a.ntx * a.nty * a.nzt * a.split;
    return a.nblk;
}

void launch_forward_gemm(const Plan& P, const cf32* x, hipStream_t s) {
    FwdArgs a;
    size_t lds;
    const int np = fwd_tile_np(P);
    fwd_args(P, x, a, lds, np);
    const dim3 grid(a.nblk), block(64 * a.nw);
#define UFSS_FWD(NPV, ZCV)                                                                                   \
    do {                                                                                                     \
        if (a.ft) hipLaunchKernelGGL((fwd_gemm_f32_kernel<NPV, ZCV, false, true>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((fwd_gemm_f32_kernel<NPV, ZCV>), grid, block, lds, s, a);                   \
    } while (0)
#define UFSS_FWDG(NPV, ZCV)                                                                                 \
    do {                                                                                                    \
        if (a.ft) hipLaunchKernelGGL((fwd_gemm_f32_kernel<NPV, ZCV, true, true>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((fwd_gemm_f32_kernel<NPV, ZCV, true>), grid, block, lds, s, a);            \
    } while (0)
    if (a.amp) {
        if (np == 4) {
            if (a.zc == 16) UFSS_FWDG(4, 16); else if (a.zc == 8) UFSS_FWDG(4, 8); else UFSS_FWDG(4, 4);
        } else {
            if (a.zc == 16) UFSS_FWDG(2, 16); else if (a.zc == 8) UFSS_FWDG(2, 8); else UFSS_FWDG(2, 4);
        }
    } else if (np == 4) {
        if (a.zc == 16) UFSS_FWD(4, 16); else if (a.zc == 8) UFSS_FWD(4, 8); else UFSS_FWD(4, 4);
    } else {
        if (a.zc == 16) UFSS_FWD(2, 16); else if (a.zc == 8) UFSS_FWD(2, 8); else UFSS_FWD(2, 4);
    }
#undef UFSS_FWDG
#undef UFSS_FWD
    UFSS_HIP(hipGetLastError());
}

void launch_adjoint_gemm(const Plan& P, cf32* out, hipStream_t s, bool sum) {
    AdjArgs a;
    size_t lds;
    const int np = adj_tile_np(P);
    const int nw = adj_waves(P);
    adj_args(P, out, a, lds, np, nw);
    const dim3 grid(a.nblk), block(64 * nw);
#define UFSS_ADJ(NPV, KCV) hipLaunchKernelGGL((adj_gemm_f32_kernel<NPV, kAdjNZ, KCV>), grid, block, lds, s, a)
#define UFSS_ADJ2(KCV)                                                                                       \
    do {                                                                                                     \
        if (nw == 8) hipLaunchKernelGGL((adj_gemm_f32_kernel_np2<kAdjNZ, KCV, false, 8>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((adj_gemm_f32_kernel_np2<kAdjNZ, KCV>), grid, block, lds, s, a);              \
    } while (0)
#define UFSS_ADJG(NPV, KCV) hipLaunchKernelGGL((adj_gemm_f32_kernel<NPV, kAdjNZ, KCV, true>), grid, block, lds, s, a)
#define UFSS_ADJ2G(KCV)                                                                                      \
    do {                                                                                                     \
        if (nw == 8) hipLaunchKernelGGL((adj_gemm_f32_kernel_np2<kAdjNZ, KCV, true, 8>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((adj_gemm_f32_kernel_np2<kAdjNZ, KCV, true>), grid, block, lds, s, a);        \
    } while (0)
    if (a.amp) {
        if (np == 4) {
            if (a.kc == 16) UFSS_ADJG(4, 16); else if (a.kc == 8) UFSS_ADJG(4, 8); else UFSS_ADJG(4, 4);
        } else {
            if (a.kc == 16) UFSS_ADJ2G(16); else if (a.kc == 8) UFSS_ADJ2G(8); else UFSS_ADJ2G(4);
        }
    } else if (np == 4) {
        if (a.kc == 16) UFSS_ADJ(4, 16); else if (a.kc == 8) UFSS_ADJ(4, 8); else UFSS_ADJ(4, 4);
    } else {
        if (a.kc == 16) UFSS_ADJ2(16); else if (a.kc == 8) UFSS_ADJ2(8); else UFSS_ADJ2(4);
    }
#undef UFSS_ADJ2G
#undef UFSS_ADJG
#undef UFSS_ADJ2
#undef UFSS_ADJ
    UFSS_HIP(hipGetLastError());
    if (a.split > 1 && sum) launch_sum_parts(P.d_gpart, a.split, P.nvox, out, s);
}

// Grouped launches (one grid for many plans).  Descriptors are opaque bytes.
size_t desc_size(GemmKind k) {
    switch (k) {
        case GemmKind::FwdF32: return sizeof(FwdArgs);
        case GemmKind::AdjF32: return sizeof(AdjArgs);
        default: return bf16_desc_size(k);
    }
}

int make_desc(GemmKind k, const Plan& P, const void* in, void* out, void* desc, size_t* lds, int* threads) {
    if (P.d_amp) fail(UFSS_ERR_UNSUPPORTED, "grouped launches do not take a Gaussian beam");
    if (P.mix) fail(UFSS_ERR_UNSUPPORTED, "grouped launches do not take mixed plans");
    switch (k) {
        case GemmKind::FwdF32: {
            FwdArgs& a = *static_cast<FwdArgs*>(desc);
            const int nb = fwd_args(P, static_cast<const cf32*>(in), a, *lds, kGroupNP, false);
            *threads = 64 * a.nw;                   // the waves with a bin sub-tile
            return nb;
        }
        case GemmKind::AdjF32:
            *threads = 256;
            return adj_args(P, static_cast<cf32*>(out), *static_cast<AdjArgs*>(desc), *lds, kGroupNP);
        default:
            *threads = 256;
            return bf16_make_desc(k, P, in, out, desc, lds);
    }
}

void launch_grouped(GemmKind k, const void* descs, const int2* blk, int nblocks, size_t lds, int threads,
                    hipStream_t s) {
    if (nblocks <= 0) return;
    switch (k) {
        case GemmKind::FwdF32:
            if (threads < 64 || threads > 512 || threads % 64)
                fail(UFSS_ERR_INVALID_ARG, "grouped forward: workgroup size must be 64 to 512 in steps of 64");
            hipLaunchKernelGGL(fwd_gemm_f32_kernel_grouped<kGroupNP>, dim3(nblocks), dim3(threads), lds, s,
                               static_cast<const FwdArgs*>(descs), blk);
            break;
        case GemmKind::AdjF32:
            hipLaunchKernelGGL((adj_gemm_f32_kernel_grouped<kGroupNP, kAdjNZ>), dim3(nblocks), dim3(256),
                               lds, s, static_cast<const AdjArgs*>(descs), blk);
            break;
        default: bf16_launch_grouped(k, descs, blk, nblocks, lds, s); return;
    }
    UFSS_HIP(hipGetLastError());
}

}  // namespace ufss
