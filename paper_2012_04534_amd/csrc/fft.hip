// Transform-domain operator (paper Sec. IV-B, Alg. 2): the block two-level
// Toeplitz structure makes A a lateral 2-D correlation, which a cyclic
// transform of size L >= N + W per axis evaluates exactly on the scan grid.
//
//   forward  X^[q][z] = DFT_2(x)              (separable twiddle products)
//            Y^[q][k] = sum_z K^[q][z][k] X^[q][z]
//            y[p][k]  = IDFT_2(Y^) on the N x N grid positions, then H_k
//   adjoint  R^[q][k] = DFT_2(H r)
//            X'[q][z] = sum_k conj(K^[q][z][k]) R^[q][k]
//            x[v][z]  = IDFT_2(X') on the grid voxels
//
// K^[q][z][k] = sum_{|d| <= W} P_d[k][z] exp(-j 2 pi (q_x d_x / L_x + q_y d_y / L_y))
// with P_d the windowed, beam-weighted phasor of the other paths (same
// integer-turn delays).  P_d is even in d_x and in d_y, so K^ is a cosine
// transform, even in q_x and q_y: only the quadrant q_x <= L_x / 2,
// q_y <= L_y / 2 is stored, and each stored entry serves up to four q.
// K^ is built once per plan in FP64 and stored in FP32, also as a transposed
// copy [q][k][z] so that both contractions read rows in order; the applies run
// in FP32.  The contraction streams K^ once per apply and is bound by HBM (or by
// the last-level cache when K^ fits there); the lateral transforms are small
// products with twiddle tables.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace ufss {

static constexpr int kTwT = 256;   // threads of the twiddle products (channels)

// out[b][i][c] = sum_j W[i][j] in[b][j][c]  (complex, FP32; c contiguous).  TI
// outputs per thread along the transformed axis; the launch picks TI so the
// product has enough threads to cover the chip.  The walk over j loads kTwJ
// inputs before using them, so that many loads are in flight per thread; the
// twiddle rows in LDS are padded with zeros to a multiple of kTwJ.
static constexpr int kTwJ = 8;

__host__ __device__ static inline int tw_stride(int J) { return (J + kTwJ - 1) / kTwJ * kTwJ; }

template <int TI>
__global__ __launch_bounds__(kTwT) void twiddle_kernel(cf32* __restrict__ out,
                                                      const cf32* __restrict__ in,
                                                      const cf32* __restrict__ W, int I, int J,
                                                      int C, int64_t sib, int64_t sij,
                                                      int64_t sob, int64_t soi) {
    extern __shared__ __align__(16) unsigned char smem[];
    cf32* wl = reinterpret_cast<cf32*>(smem);          // [TI][Jp]
    const int Jp = tw_stride(J);
    const int c = blockIdx.x * kTwT + threadIdx.x;
    const int i0 = blockIdx.y * TI;
    const int b = blockIdx.z;
    for (int t = threadIdx.x; t < TI * Jp; t += kTwT) {
        const int ii = t / Jp, j = t - ii * Jp;
        wl[t] = (i0 + ii < I && j < J) ? W[(int64_t)(i0 + ii) * J + j] : cf32{0.f, 0.f};
    }
    __syncthreads();
    if (c >= C) return;
    float ar[TI], ai[TI];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii) ar[ii] = ai[ii] = 0.f;
    const cf32* src = in + (int64_t)b * sib + c;
    for (int j0 = 0; j0 < J; j0 += kTwJ) {
        cf32 v[kTwJ];
#pragma unroll
        for (int t = 0; t < kTwJ; ++t)
            v[t] = (j0 + t < J) ? src[(int64_t)(j0 + t) * sij] : cf32{0.f, 0.f};
#pragma unroll
        for (int t = 0; t < kTwJ; ++t) {
#pragma unroll
            for (int ii = 0; ii < TI; ++ii) {
                // four FMAs per complex product (no separate multiplies and adds)
                const cf32 w = wl[ii * Jp + j0 + t];
                ar[ii] = fmaf(w.re, v[t].re, ar[ii]);
                ar[ii] = fmaf(-w.im, v[t].im, ar[ii]);
                ai[ii] = fmaf(w.re, v[t].im, ai[ii]);
                ai[ii] = fmaf(w.im, v[t].re, ai[ii]);
            }
        }
    }
    cf32* dst = out + (int64_t)b * sob + c;
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
        if (i0 + ii < I) dst[(int64_t)(i0 + ii) * soi] = cf32{ar[ii], ai[ii]};
}

// The same product on the FP32 matrix cores (v_mfma_f32_16x16x4f32: rows i,
// columns c, reduction over j four at a time; four real products per complex
// one, the imaginary part of W negated for the real accumulator).  A workgroup
// is 4 waves on 4 consecutive 16-column tiles of one b and one block of 16 NI
// rows.  The plan keeps each twiddle table also in operand order,
//   Wop[(T ks + s) 64 + lane] = W[16 T + lane % 16][4 s + lane / 16]
// (row tile T, reduction step s, ks = ceil(J / 4) steps, zero outside I x J),
// so a block's tiles are one contiguous range: it is copied to LDS with 16-byte
// loads and each lane then reads 8 contiguous bytes per operand.  Each lane
// streams its column of the input kTmPK reduction steps ahead.
typedef float f4v __attribute__((ext_vector_type(4)));
static constexpr int kTmMaxNI = 8;
static constexpr int kTmPK = 4;
static constexpr size_t kTmLds = 64 * 1024;   // bytes of staged twiddles per workgroup

template <int NI>
__global__ __launch_bounds__(256) void twiddle_mfma_kernel(cf32* __restrict__ out,
                                                           const cf32* __restrict__ in,
                                                           const cf32* __restrict__ Wop, int I, int J,
                                                           int C, int64_t sib, int64_t sij,
                                                           int64_t sob, int64_t soi) {
    extern __shared__ __align__(16) unsigned char smem[];
    cf32* wl = reinterpret_cast<cf32*>(smem);            // [NI][ks][64]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ks = (J + 3) / 4;
    const int tiles = (I + 15) / 16;
    const int t0 = blockIdx.y * NI, i0 = 16 * t0;
    const int b = blockIdx.z;
    {
        // this block's tiles: a contiguous run of 32-byte pairs of entries,
        // zero past the last tile of W
        const int nvalid = min(NI, tiles - t0) * ks * 32;   // 16-byte units present
        const int nall = NI * ks * 32;
        const float4* src4 = reinterpret_cast<const float4*>(Wop + (int64_t)t0 * ks * 64);
        float4* dst4 = reinterpret_cast<float4*>(wl);
        for (int t = threadIdx.x; t < nall; t += 256)
            dst4[t] = t < nvalid ? src4[t] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const int c0 = (blockIdx.x * 4 + wave) * 16;
    if (c0 >= C) return;                                  // wave-uniform
    const int c = c0 + (lane & 15), kq = lane >> 4;
    const bool cok = c < C;
    const cf32* src = in + (int64_t)b * sib + (cok ? c : 0);
    f4v ar[NI], ai[NI];
#pragma unroll
    for (int t = 0; t < NI; ++t) ar[t] = ai[t] = f4v{0.f, 0.f, 0.f, 0.f};
    cf32 cur[kTmPK];
#pragma unroll
    for (int p = 0; p < kTmPK; ++p) {
        const int j = 4 * p + kq;
        cur[p] = (cok && j < J) ? src[(int64_t)j * sij] : cf32{0.f, 0.f};
    }
    for (int s0 = 0; s0 < ks; s0 += kTmPK) {
        cf32 nxt[kTmPK];
#pragma unroll
        for (int p = 0; p < kTmPK; ++p) {
            const int j = 4 * (s0 + kTmPK + p) + kq;
            nxt[p] = (cok && j < J) ? src[(int64_t)j * sij] : cf32{0.f, 0.f};
        }
#pragma unroll
        for (int p = 0; p < kTmPK; ++p) {
            const int st = s0 + p;
            if (st >= ks) break;                          // wave-uniform
            const cf32 bv = cur[p];
#pragma unroll
            for (int t = 0; t < NI; ++t) {
                const cf32 a = wl[(t * ks + st) * 64 + lane];
                ar[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, bv.re, ar[t], 0, 0, 0);
                ar[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, bv.im, ar[t], 0, 0, 0);
                ai[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, bv.im, ai[t], 0, 0, 0);
                ai[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, bv.re, ai[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < kTmPK; ++p) cur[p] = nxt[p];
    }
    if (!cok) return;
    cf32* dst = out + (int64_t)b * sob + c;
#pragma unroll
    for (int t = 0; t < NI; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * t + 4 * kq + r;
            if (i < I) dst[(int64_t)i * soi] = cf32{ar[t][r], ai[t][r]};
        }
}

// Row tiles per wave for the matrix-core product: enough to cover I (at most
// kTmMaxNI), no more than the LDS budget holds; 0 when not even one fits.
static int tm_tiles(int I, int J) {
    const int ks = (J + 3) / 4;
    const int by_lds = (int)(kTmLds / ((size_t)ks * 64 * sizeof(cf32)));
    return std::min(std::min(kTmMaxNI, (I + 15) / 16), by_lds);
}

static void twiddle(cf32* out, const cf32* in, const cf32* W, int B, int I, int J, int C,
                    int64_t sib, int64_t sij, int64_t sob, int64_t soi, hipStream_t s) {
    // row tiles per wave: as many as fit, then fewer (more waves, each input
    // column read by more of them) while the launch has under 2048 waves
    int ni = tm_tiles(I, J);
    {
        const int64_t tiles = (I + 15) / 16, col_waves = (int64_t)((C + 15) / 16) * B;
        while (ni > 1 && col_waves * ((tiles + ni - 1) / ni) < 2048) --ni;
    }
    if (ni >= 1) {
        const dim3 grid((C + 63) / 64, (I + 16 * ni - 1) / (16 * ni), B);
        const size_t lds = (size_t)((J + 3) / 4) * ni * 64 * sizeof(cf32);
        const cf32* Wop = W + (((int64_t)I * J + 1) & ~(int64_t)1);   // operand-order copy (16-byte aligned)
#define UFSS_TM(T) hipLaunchKernelGGL(twiddle_mfma_kernel<T>, grid, dim3(256), lds, s, out, in, Wop, I, J, C, sib, sij, sob, soi)
        switch (ni) {
            case 1: UFSS_TM(1); break;
            case 2: UFSS_TM(2); break;
            case 3: UFSS_TM(3); break;
            case 4: UFSS_TM(4); break;
            case 5: UFSS_TM(5); break;
            case 6: UFSS_TM(6); break;
            case 7: UFSS_TM(7); break;
            default: UFSS_TM(8); break;
        }
#undef UFSS_TM
        UFSS_HIP(hipGetLastError());
        return;
    }
    // vector-ALU product for twiddle blocks too large for LDS
    // outputs per thread: as many as keep at least ~64K threads in flight
    const int64_t base = (int64_t)B * C;
    int ti = 8;
    while (ti > 1 && base * ((I + ti - 1) / ti) < 65536) ti /= 2;
    const dim3 grid((C + kTwT - 1) / kTwT, (I + ti - 1) / ti, B);
    const size_t lds = (size_t)ti * tw_stride(J) * sizeof(cf32);
#define UFSS_TW(T) hipLaunchKernelGGL(twiddle_kernel<T>, grid, dim3(kTwT), lds, s, out, in, W, I, J, C, sib, sij, sob, soi)
    if (ti == 8) UFSS_TW(8); else if (ti == 4) UFSS_TW(4); else if (ti == 2) UFSS_TW(2); else UFSS_TW(1);
#undef UFSS_TW
    UFSS_HIP(hipGetLastError());
}

// The up-to-four transform indices (q_y, q_x) of quadrant entry (oy, ox),
// enumerated as q = a nx2 + b with q_y = oy or ly - oy (a) and q_x = ox or
// lx - ox (b); nx2 (ny2) is 1 on the axis's self-mirrored entries.  Computed
// per use (no per-thread arrays, which would live in scratch memory).
struct Orbit {
    int oy, ox, ly, lx, nx2, n;
    __device__ Orbit(int oy_, int ox_, int ly_, int lx_) : oy(oy_), ox(ox_), ly(ly_), lx(lx_) {
        const int ny2 = (oy == 0 || 2 * oy == ly) ? 1 : 2;
        nx2 = (ox == 0 || 2 * ox == lx) ? 1 : 2;
        n = ny2 * nx2;
    }
    // row index q_y lx + q_x of member q
    __device__ int64_t row(int q) const {
        const int a = q / nx2, b = q - a * nx2;
        return (int64_t)(a ? ly - oy : oy) * lx + (b ? lx - ox : ox);
    }
};

// Contraction, both directions: one workgroup per quadrant entry (its up to
// four transform indices q), out[q][c] = sum_r T[o][r][c] in[q][r] (CONJ:
// conj(T)).  Forward: c = bin, r = depth, T = K^[o][z][k]; adjoint: c = depth,
// r = bin, T = the transposed copy K^t[o][k][z].  Consecutive threads take
// consecutive c (coalesced rows of T); when C is below the workgroup size NT
// the reduction range is split over G = NT / C thread groups whose partial
// sums meet in LDS in a fixed order.
//
// The table is streamed kPF rows ahead: each thread holds the current block of
// kPF entries of its column while the next block is in flight, and the first
// block is requested before the input rows are staged.  Four rows ahead keep
// the kernel within 64 registers, so eight waves fit per SIMD (four
// 512-thread workgroups per CU): more workgroups in flight and fewer rounds
// over the chip than eight rows ahead at six waves (measured on the 32 x 32
// and 64 x 64 C-scans).
static constexpr int kPF = 4;

// Table entries as FP32 pairs (FP32 plans) or BF16 pairs (BF16 plans: the table
// rounded to nearest even once at plan time, products and sums in FP32).
__device__ __forceinline__ cf32 entry(const cf32& v) { return v; }
__device__ __forceinline__ cf32 entry(const cbf16& v) { return cf32{(float)v.re, (float)v.im}; }

template <bool CONJ, int NT, typename TT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void contract_kernel(const TT* __restrict__ tab,
                                                      const cf32* __restrict__ in,
                                                      cf32* __restrict__ out, int ly, int lx,
                                                      int nox, int C, int R) {
    // rows ahead: BF16 entries are half the bytes, so two more rows (as many
    // as fit the 64 registers of eight waves per SIMD) keep more bytes in flight
    constexpr int PF = sizeof(TT) == sizeof(cf32) ? kPF : kPF + 2;
    extern __shared__ __align__(16) unsigned char smem[];
    cf32* vs = reinterpret_cast<cf32*>(smem);                 // [4][R] input rows
    float* red = reinterpret_cast<float*>(vs + 4 * R);        // [G][4][C][2] partials
    const int o = blockIdx.x, oy = o / nox, ox = o - oy * nox;
    const Orbit orb(oy, ox, ly, lx);
    const int nq = orb.n;
    const TT* tb = tab + (int64_t)o * R * C;
    const int W = C >= NT ? NT : C;                           // threads per group (c stride)
    const int G = C >= NT ? 1 : NT / C;
    const int grp = threadIdx.x / W;
    const int lane_c = threadIdx.x - grp * W;
    const int rper = (R + G - 1) / G;
    const int r0 = grp * rper, r1 = min(R, r0 + rper);
    const bool active = grp < G;
    TT cur[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t)
        cur[t] = (active && lane_c < C && r0 + t < r1) ? tb[(int64_t)(r0 + t) * C + lane_c] : TT{};
    for (int t = threadIdx.x; t < nq * R; t += blockDim.x) {
        const int q = t / R, r = t - q * R;
        vs[t] = in[orb.row(q) * R + r];
    }
    __syncthreads();
    for (int c = lane_c; c < C && active; c += W) {
        const TT* col = tb + c;
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
        for (int rb = r0; rb < r1; rb += PF) {
            TT nxt[PF];
#pragma unroll
            for (int t = 0; t < PF; ++t) {
                const int r = rb + PF + t;
                nxt[t] = r < r1 ? col[(int64_t)r * C] : TT{};
            }
#pragma unroll
            for (int t = 0; t < PF; ++t) {
                if (rb + t >= r1) break;
                const cf32 kv = entry(cur[t]);
                const float ki = CONJ ? -kv.im : kv.im;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q >= nq) break;
                    const cf32 v = vs[q * R + rb + t];
                    ar[q] = fmaf(kv.re, v.re, ar[q]);
                    ar[q] = fmaf(-ki, v.im, ar[q]);
                    ai[q] = fmaf(kv.re, v.im, ai[q]);
                    ai[q] = fmaf(ki, v.re, ai[q]);
                }
            }
#pragma unroll
            for (int t = 0; t < PF; ++t) cur[t] = nxt[t];
        }
        if (G == 1) {
            for (int q = 0; q < nq; ++q)
                out[orb.row(q) * C + c] = cf32{ar[q], ai[q]};
        } else {
            for (int q = 0; q < nq; ++q) {
                red[((grp * 4 + q) * C + c) * 2] = ar[q];
                red[((grp * 4 + q) * C + c) * 2 + 1] = ai[q];
            }
        }
        // first block of this thread's next column (C > NT only)
        const int cn = c + W;
#pragma unroll
        for (int t = 0; t < PF; ++t)
            cur[t] = (cn < C && r0 + t < r1) ? tb[(int64_t)(r0 + t) * C + cn] : TT{};
    }
    if (G == 1) return;
    __syncthreads();
    for (int t = threadIdx.x; t < nq * C; t += blockDim.x) {
        const int q = t / C, c = t - q * C;
        float sr = 0.f, si = 0.f;
        for (int g2 = 0; g2 < G; ++g2) {
            sr += red[((g2 * 4 + q) * C + c) * 2];
            si += red[((g2 * 4 + q) * C + c) * 2 + 1];
        }
        out[orb.row(q) * C + c] = cf32{sr, si};
    }
}

// Threads per workgroup: 512 when the contiguous index is short (more groups
// over the reduction, more loads in flight) or long enough to give every
// thread one column of its own, else 256 (measured on the 32 x 32 and 64 x 64
// C-scans).
static int contract_threads(int C) { return (C <= 128 || C >= 512) ? 512 : 256; }

static size_t contract_lds(int C, int R) {
    const int NT = contract_threads(C);
    const int G = C >= NT ? 1 : NT / C;
    return (size_t)4 * R * sizeof(cf32) + (G > 1 ? (size_t)G * 4 * C * 2 * sizeof(float) : 0);
}

// Plan time: T[o][b][a] = S[o][a][b] for S of shape [A][B] per entry (the
// transposed copy of K^: A = nz, B = mu).
__global__ void transpose_kernel(const cf32* __restrict__ src, cf32* __restrict__ dst, int A, int B) {
    const int o = blockIdx.y;
    const cf32* s = src + (int64_t)o * A * B;
    cf32* d = dst + (int64_t)o * A * B;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < A * B; t += gridDim.x * blockDim.x) {
        const int b = t / A, a = t - b * A;
        d[t] = s[(int64_t)a * B + b];
    }
}

// ---- plan-time construction of K^ (FP64) -------------------------------------
// P64[dy][dx][z][k] = g(dx, dy, z) exp(-j 2 pi (kb[k] u(dy, dx, z) mod 2^32) / 2^32)
__global__ void phasor64_kernel(const uint32_t* __restrict__ u, const float* __restrict__ amp,
                                const int* __restrict__ kb, int64_t ncell, int mu,
                                double2* __restrict__ out) {
    const int64_t n = ncell * mu;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cell = t / mu;
        const int k = (int)(t - cell * mu);
        const uint32_t ph = (uint32_t)kb[k] * u[cell];
        const double turns = (double)ph * (1.0 / 4294967296.0);
        double sn, cs;
        sincos(2.0 * M_PI * turns, &sn, &cs);
        const double g = amp ? (double)amp[cell] : 1.0;
        out[t] = double2{g * cs, -g * sn};
    }
}

// out[b][i][c] = sum_j C[i][j] in[b][j][c] with a real FP64 weight table
// (the cosine transforms of the build); OUTF: FP32 output.
template <bool OUTF>
__global__ __launch_bounds__(256) void cos_kernel(void* __restrict__ out, const double2* __restrict__ in,
                                                  const double* __restrict__ Cw, int I, int J,
                                                  int64_t C, int64_t sib, int64_t sij,
                                                  int64_t sob, int64_t soi) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y, b = blockIdx.z;
    if (c >= C || i >= I) return;
    double re = 0.0, im = 0.0;
    const double2* src = in + (int64_t)b * sib + c;
    for (int j = 0; j < J; ++j) {
        const double w = Cw[(int64_t)i * J + j];
        const double2 v = src[(int64_t)j * sij];
        re += w * v.x;
        im += w * v.y;
    }
    const int64_t o = (int64_t)b * sob + (int64_t)i * soi + c;
    if (OUTF)
        static_cast<cf32*>(out)[o] = cf32{(float)re, (float)im};
    else
        static_cast<double2*>(out)[o] = double2{re, im};
}

// Cyclic transform size per axis: the smallest L >= N + W (and >= 1).
static int fft_len(int n, int w) { return std::max(1, n + w); }

int64_t fft_table_bytes(const Plan& P) {
    const int lx = fft_len(P.g.nx, P.d.wx), ly = fft_len(P.g.ny, P.d.wy);
    return (int64_t)(ly / 2 + 1) * (lx / 2 + 1) * P.g.nz * (int64_t)P.ubins_h.size() * 8;
}

static constexpr int64_t kFftTableMax = int64_t(32) << 30;

void fft_setup(Plan& P) {
    const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz, wx = P.d.wx, wy = P.d.wy;
    const int mu = (int)P.ubins_h.size();
    const int lx = fft_len(nx, wx), ly = fft_len(ny, wy);
    const int nox = lx / 2 + 1, noy = ly / 2 + 1;
    if (fft_table_bytes(P) > kFftTableMax)
        fail(UFSS_ERR_UNSUPPORTED, "transform table larger than 32 GiB");
    // LDS staging: twiddle rows (8 x L) and four transform rows (4 x nz or mu)
    if (std::max(lx, ly) > 1024 || std::max(nz, mu) > 1536)
        fail(UFSS_ERR_UNSUPPORTED, "grid too large for the transform path (L <= 1024, nz and bins <= 1536)");
    P.fft_lx = lx;
    P.fft_ly = ly;
    // twiddle tables (FP64 angles from exact integer products, stored FP32)
    auto tw = [](int rows, int cols, int L, double sign, double scale) {
        std::vector<cf32> t((size_t)rows * cols);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                const double a = 2.0 * M_PI * (double)(((int64_t)r * c) % L) / L;
                t[(size_t)r * cols + c] = cf32{(float)(scale * std::cos(a)), (float)(scale * sign * std::sin(a))};
            }
        return t;
    };
    auto up = [&](const std::vector<cf32>& h) {
        void* d = nullptr;
        UFSS_HIP(hipMalloc(&d, h.size() * sizeof(cf32)));
        UFSS_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(cf32), hipMemcpyHostToDevice));
        P.ws_bytes += h.size() * sizeof(cf32);
        return static_cast<cf32*>(d);
    };
    // each table [rows][cols] is followed, from the next even entry (16-byte
    // alignment), by its copy in matrix-core operand order
    // [ceil(rows/16)][ceil(cols/4)][64] (see twiddle_mfma_kernel)
    auto with_op = [](std::vector<cf32> t, int rows, int cols) {
        const int tiles = (rows + 15) / 16, ks = (cols + 3) / 4;
        const size_t base = (t.size() + 1) & ~(size_t)1;
        t.resize(base + (size_t)tiles * ks * 64, cf32{0.f, 0.f});
        for (int T = 0; T < tiles; ++T)
            for (int st = 0; st < ks; ++st)
                for (int l = 0; l < 64; ++l) {
                    const int r = 16 * T + (l & 15), c = 4 * st + (l >> 4);
                    if (r < rows && c < cols)
                        t[base + ((size_t)T * ks + st) * 64 + l] = t[(size_t)r * cols + c];
                }
        return t;
    };
    P.d_tw_fx = up(with_op(tw(lx, nx, lx, -1.0, 1.0), lx, nx));          // [qx][nx]
    P.d_tw_fy = up(with_op(tw(ly, ny, ly, -1.0, 1.0), ly, ny));          // [qy][ny]
    P.d_tw_ix = up(with_op(tw(nx, lx, lx, +1.0, 1.0 / lx), nx, lx));     // [px][qx]
    P.d_tw_iy = up(with_op(tw(ny, ly, ly, +1.0, 1.0 / ly), ny, ly));     // [py][qy]
    const int64_t cmax = std::max(nz, mu);
    const int64_t wbytes = (int64_t)ly * lx * cmax * sizeof(cf32);
    const int64_t tbytes = (int64_t)std::max((int64_t)ny * lx, (int64_t)ly * nx) * cmax * sizeof(cf32);
    UFSS_HIP(hipMalloc(&P.d_fa, wbytes));
    UFSS_HIP(hipMalloc(&P.d_fb, wbytes));
    UFSS_HIP(hipMalloc(&P.d_ft, tbytes));
    P.ws_bytes += 2 * wbytes + tbytes;

    // K^ in FP64: phasors, cosine transform over d_x, then over d_y
    const int64_t ncell = (int64_t)(wy + 1) * (wx + 1) * nz;
    const int64_t zc = (int64_t)nz * mu;                 // channels (z, k)
    double2 *p64 = nullptr, *s64 = nullptr;
    double *cx = nullptr, *cy = nullptr;
    std::vector<double> hx((size_t)nox * (wx + 1)), hy((size_t)noy * (wy + 1));
    for (int q = 0; q < nox; ++q)
        for (int d = 0; d <= wx; ++d)
            hx[(size_t)q * (wx + 1) + d] = (d == 0 ? 1.0 : 2.0) * std::cos(2.0 * M_PI * (double)(((int64_t)q * d) % lx) / lx);
    for (int q = 0; q < noy; ++q)
        for (int d = 0; d <= wy; ++d)
            hy[(size_t)q * (wy + 1) + d] = (d == 0 ? 1.0 : 2.0) * std::cos(2.0 * M_PI * (double)(((int64_t)q * d) % ly) / ly);
    try {
        UFSS_HIP(hipMalloc(&p64, ncell * mu * sizeof(double2)));
        UFSS_HIP(hipMalloc(&s64, (int64_t)(wy + 1) * nox * zc * sizeof(double2)));
        UFSS_HIP(hipMalloc(&cx, hx.size() * sizeof(double)));
        UFSS_HIP(hipMalloc(&cy, hy.size() * sizeof(double)));
        UFSS_HIP(hipMalloc(&P.d_khat, (int64_t)noy * nox * zc * sizeof(cf32)));
        UFSS_HIP(hipMalloc(&P.d_khat_t, (int64_t)noy * nox * zc * sizeof(cf32)));
        P.ws_bytes += 2 * (int64_t)noy * nox * zc * sizeof(cf32);
        UFSS_HIP(hipMemcpy(cx, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice));
        UFSS_HIP(hipMemcpy(cy, hy.data(), hy.size() * sizeof(double), hipMemcpyHostToDevice));
        const int64_t n = ncell * mu;
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(phasor64_kernel, dim3(blocks), dim3(256), 0, nullptr, P.d_u, P.d_amp,
                           P.d_ubins, ncell, mu, p64);
        UFSS_HIP(hipGetLastError());
        // S[dy][qx][z][k] = sum_dx hx[qx][dx] P[dy][dx][z][k]
        hipLaunchKernelGGL(cos_kernel<false>, dim3((unsigned)((zc + 255) / 256), nox, wy + 1), dim3(256),
                           0, nullptr, (void*)s64, p64, cx, nox, wx + 1, zc, (int64_t)(wx + 1) * zc, zc,
                           (int64_t)nox * zc, zc);
        UFSS_HIP(hipGetLastError());
        // K^[qy][qx][z][k] = sum_dy hy[qy][dy] S[dy][qx][z][k]
        hipLaunchKernelGGL(cos_kernel<true>, dim3((unsigned)((zc + 255) / 256), noy, nox), dim3(256),
                           0, nullptr, (void*)P.d_khat, s64, cy, noy, wy + 1, zc, zc, (int64_t)nox * zc,
                           zc, (int64_t)nox * zc);
        UFSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)std::min<int64_t>((zc + 255) / 256, 1024), noy * nox),
                           dim3(256), 0, nullptr, static_cast<const cf32*>(P.d_khat),
                           static_cast<cf32*>(P.d_khat_t), nz, mu);
        UFSS_HIP(hipGetLastError());
        if (P.dtype == UFSS_BF16) {
            // BF16 plans stream both copies of the table in BF16 (rounded to
            // nearest even once, here); the FP32 copies are released
            const int64_t n = (int64_t)noy * nox * zc;
            void* k16 = nullptr;
            void* kt16 = nullptr;
            try {
                UFSS_HIP(hipMalloc(&k16, n * sizeof(cbf16)));
                UFSS_HIP(hipMalloc(&kt16, n * sizeof(cbf16)));
            } catch (...) {
                if (k16) (void)hipFree(k16);
                throw;
            }
            launch_to_bf16(static_cast<const cf32*>(P.d_khat), k16, n, nullptr);
            launch_to_bf16(static_cast<const cf32*>(P.d_khat_t), kt16, n, nullptr);
            UFSS_HIP(hipDeviceSynchronize());
            (void)hipFree(P.d_khat);
            (void)hipFree(P.d_khat_t);
            P.d_khat = k16;
            P.d_khat_t = kt16;
            P.ws_bytes -= 2 * n * (int64_t)(sizeof(cf32) - sizeof(cbf16));
        }
        UFSS_HIP(hipDeviceSynchronize());
    } catch (...) {
        if (p64) (void)hipFree(p64);
        if (s64) (void)hipFree(s64);
        if (cx) (void)hipFree(cx);
        if (cy) (void)hipFree(cy);
        throw;
    }
    (void)hipFree(p64);
    (void)hipFree(s64);
    (void)hipFree(cx);
    (void)hipFree(cy);
}

// Forward, in three steps (the contraction is the core kernel):
//   x[ny][nx][nz] -> T[ny][lx][nz] -> X^[ly][lx][nz]
void fft_fwd_transform(const Plan& P, const cf32* x, hipStream_t s) {
    const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz, lx = P.fft_lx, ly = P.fft_ly;
    twiddle(P.d_ft, x, P.d_tw_fx, ny, lx, nx, nz, (int64_t)nx * nz, nz, (int64_t)lx * nz, nz, s);
    twiddle(P.d_fa, P.d_ft, P.d_tw_fy, lx, ly, ny, nz, nz, (int64_t)lx * nz, nz, (int64_t)lx * nz, s);
}

//   Y^[q][k] = sum_z K^[q][z][k] X^[q][z]
void fft_fwd_contract(const Plan& P, hipStream_t s) {
    const int lx = P.fft_lx, ly = P.fft_ly, nox = lx / 2 + 1, noy = ly / 2 + 1;
    const int mu = (int)P.ubins_h.size(), nz = P.g.nz;
    const size_t lds = contract_lds(mu, nz);
    const dim3 grid(noy * nox);
    if (P.dtype == UFSS_BF16) {
        const cbf16* t = static_cast<const cbf16*>(P.d_khat);
        if (contract_threads(mu) == 512)
            hipLaunchKernelGGL((contract_kernel<false, 512, cbf16>), grid, dim3(512), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, mu, nz);
        else
            hipLaunchKernelGGL((contract_kernel<false, 256, cbf16>), grid, dim3(256), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, mu, nz);
    } else {
        const cf32* t = static_cast<const cf32*>(P.d_khat);
        if (contract_threads(mu) == 512)
            hipLaunchKernelGGL((contract_kernel<false, 512, cf32>), grid, dim3(512), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, mu, nz);
        else
            hipLaunchKernelGGL((contract_kernel<false, 256, cf32>), grid, dim3(256), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, mu, nz);
    }
    UFSS_HIP(hipGetLastError());
}

//   Y^[ly][lx][mu] -> U[ly][nx][mu] -> y_raw[ny][nx][mu]
void fft_fwd_inverse(const Plan& P, hipStream_t s) {
    const int nx = P.g.nx, ny = P.g.ny, lx = P.fft_lx, ly = P.fft_ly, mu = (int)P.ubins_h.size();
    twiddle(P.d_ft, P.d_fb, P.d_tw_ix, ly, nx, lx, mu, (int64_t)lx * mu, mu, (int64_t)nx * mu, mu, s);
    twiddle(P.d_yraw, P.d_ft, P.d_tw_iy, nx, ny, ly, mu, mu, (int64_t)nx * mu, mu, (int64_t)nx * mu, s);
}

// Adjoint, in three steps; the operand is the H-scaled union-bin rows in P.d_rop.
void fft_adj_transform(const Plan& P, hipStream_t s) {
    const int nx = P.g.nx, ny = P.g.ny, lx = P.fft_lx, ly = P.fft_ly, mu = (int)P.ubins_h.size();
    const cf32* r = static_cast<const cf32*>(P.d_rop);
    twiddle(P.d_ft, r, P.d_tw_fx, ny, lx, nx, mu, (int64_t)nx * mu, mu, (int64_t)lx * mu, mu, s);
    twiddle(P.d_fa, P.d_ft, P.d_tw_fy, lx, ly, ny, mu, mu, (int64_t)lx * mu, mu, (int64_t)lx * mu, s);
}

void fft_adj_contract(const Plan& P, hipStream_t s) {
    const int lx = P.fft_lx, ly = P.fft_ly, nox = lx / 2 + 1, noy = ly / 2 + 1;
    const int mu = (int)P.ubins_h.size();
    const int nz = P.g.nz;
    const size_t lds = contract_lds(nz, mu);
    const dim3 grid(noy * nox);
    if (P.dtype == UFSS_BF16) {
        const cbf16* t = static_cast<const cbf16*>(P.d_khat_t);
        if (contract_threads(nz) == 512)
            hipLaunchKernelGGL((contract_kernel<true, 512, cbf16>), grid, dim3(512), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, nz, mu);
        else
            hipLaunchKernelGGL((contract_kernel<true, 256, cbf16>), grid, dim3(256), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, nz, mu);
    } else {
        const cf32* t = static_cast<const cf32*>(P.d_khat_t);
        if (contract_threads(nz) == 512)
            hipLaunchKernelGGL((contract_kernel<true, 512, cf32>), grid, dim3(512), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, nz, mu);
        else
            hipLaunchKernelGGL((contract_kernel<true, 256, cf32>), grid, dim3(256), lds, s, t, P.d_fa, P.d_fb, ly, lx, nox, nz, mu);
    }
    UFSS_HIP(hipGetLastError());
}

void fft_adj_inverse(const Plan& P, cf32* out, hipStream_t s) {
    const int nx = P.g.nx, ny = P.g.ny, nz = P.g.nz, lx = P.fft_lx, ly = P.fft_ly;
    twiddle(P.d_ft, P.d_fb, P.d_tw_ix, ly, nx, lx, nz, (int64_t)lx * nz, nz, (int64_t)nx * nz, nz, s);
    twiddle(out, P.d_ft, P.d_tw_iy, nx, ny, ly, nz, nz, (int64_t)nx * nz, nz, (int64_t)nx * nz, s);
}

}  // namespace ufss
