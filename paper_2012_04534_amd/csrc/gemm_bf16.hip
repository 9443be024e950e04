// Windowed complex GEMM kernels, BF16 operands with FP32 accumulation.
//
// Same products as the FP32 kernels (paper Sec. IV-B: one small complex GEMM
// per lateral offset d of the block 2-level Toeplitz operator):
//
//   forward  Y[p, k] = sum_d sum_z  P_d[k, z] x[p - d, z]
//   adjoint  G[v, z] = sum_d sum_k  conj(P_d[k, z]) R[v + d, k]
//
// with the phasors P and the operands x (forward) and R = H r (adjoint) rounded
// to BF16 (round to nearest even); accumulation and everything in HBM stay FP32.
//
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l holds A[i = l%16][k = 8(l/16) + e],
// B[k = 8(l/16) + e][j = l%16] for e = 0..7, D[i = 4(l/16) + r][j = l%16].
// The adjoint's folded short bin chunk uses v_mfma_f32_4x4x4_16b_bf16 (half
// the cycles of the 16 x 16 x 32 form on gfx950, the 16 x 16 x 16 form costs
// as much as the 16 x 16 x 32 one): block b = l/4 holds A_b[i = l%4][k = e],
// B_b[k = e][j = l%4] for e = 0..3 and D_b[i = r][j = l%4].
//
// At BF16 rates a phasor costs far more VALU time than the MFMA work one wave
// does with it, so the four waves of a workgroup share one phasor tile: it is
// generated cooperatively in LDS for each offset d (double buffered, the next
// offset's tile is written while the current one is consumed) and each wave
// applies it to its own positions.  Along the bin axis the phasors of
// consecutive bins are produced by one complex multiplication (angle addition)
// from the previous one; non-consecutive bins take a fresh sin/cos.  Operand
// halos are stored planar (8 real then 8 imaginary values contiguous) so one
// 16-byte LDS read fills a BF16 MFMA operand; columns outside the grid map to a
// single zero cell.
#include "internal.h"

namespace ufss {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef short s4v __attribute__((ext_vector_type(4)));

static constexpr float kTwoM32b = 2.3283064365386963e-10f;
static constexpr int ZCB = 32;             // reduction chunk = one MFMA K
static constexpr int CELL = 2 * ZCB + 8;   // bf16 per halo cell (re, im, pad)
static constexpr int PROW = ZCB + 8;       // bf16 per phasor-tile row
// Adjoint with a short last bin chunk (at most ZX bins past the last full
// one, e.g. 66 = 2 x 32 + 2): those bins ride along with the previous chunk in
// the padding of its cells (re at 2 ZCB, im at 2 ZCB + ZX) and tile rows (at ZCB)
static constexpr int ZX = 4;

__device__ __forceinline__ void sincos_turns(uint32_t ku, float& c, float& s) {
    float ph = (float)(int32_t)ku * kTwoM32b;
    c = __builtin_amdgcn_cosf(ph);
    s = __builtin_amdgcn_sinf(ph);
}

__device__ __forceinline__ bf8 lds_bf8(const __bf16* p) {
    return *reinterpret_cast<const bf8*>(p);
}

__device__ __forceinline__ bf8 neg_bf8(bf8 v) {
    u4 w = __builtin_bit_cast(u4, v);
    w ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(bf8, w);
}

// Stages rows x ncol cells of W complex BF16 values into planar LDS cells of
// CELL bf16 (real parts at re0, imaginary parts at im0; row pitch `pitch` cells;
// grid row gy = ybase + r in row slot gy & slot_mask, so a window of
// consecutive rows that moves by one row only needs the entering row staged):
//   cell (gy & slot_mask, c) <- src[(gy * nx + xbase + c) * ld + i0 + e], e < W,
// zero for rows outside the grid or past `ilim` along the inner axis (columns
// are inside the grid by construction).  Each thread keeps one e and walks the
// cells with a fixed step, with UNR loads in flight before the LDS stores.
template <int UNR, int W = ZCB>
__device__ __forceinline__ void stage_planar(__bf16* __restrict__ halo, int rows, int ncol, int pitch, int slot_mask,
                                             const cbf16* __restrict__ src, int ny, int nx, int64_t ld,
                                             int ybase, int xbase, int i0, int ilim, int re0 = 0, int im0 = ZCB) {
    const int e = threadIdx.x & (W - 1);
    const int step = blockDim.x / W;
    const int total = rows * ncol;
    int cell = threadIdx.x / W;
    int r = cell / ncol, c = cell - r * ncol;
    const bool eok = i0 + e < ilim;
    for (; cell < total; cell += UNR * step) {
        cbf16 v[UNR];
        int dst[UNR];
        int rr = r, cc = c;
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            v[u] = to_cbf16(0.f, 0.f);
            dst[u] = ((ybase + rr) & slot_mask) * pitch + cc;
            const int gy = ybase + rr;
            if (cell + u * step < total && eok && gy >= 0 && gy < ny)
                v[u] = src[((int64_t)gy * nx + xbase + cc) * ld + i0 + e];
            cc += step;
            while (cc >= ncol) { cc -= ncol; ++rr; }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (cell + u * step < total) {
                halo[(size_t)dst[u] * CELL + re0 + e] = v[u].re;
                halo[(size_t)dst[u] * CELL + im0 + e] = v[u].im;
            }
        r = rr;
        c = cc;
    }
}

// Phasor tiles read from the precomputed tables: a tile is `nrows` rows of
// 2 planes x 32 BF16 values (128 contiguous bytes per row in the table), copied
// to pc / ps rows of PROW.  256 threads move 16 bytes each per pass, two passes
// cover 64 rows; rows at or past `rows_valid` are zero.  Loads are issued into
// registers first (tab_load) so they overlap the MFMA work of the current tile,
// and written to LDS afterwards (tab_store).
struct TabRegs {
    u4 v[2];
    u2 x;                  // folded short chunk: the first ZX bins of the next table chunk
};

__device__ __forceinline__ void tab_load(TabRegs& R, const __bf16* __restrict__ src, int rows_valid) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int t = threadIdx.x + p * 256, row = t >> 3, part = t & 7;
        R.v[p] = u4{0u, 0u, 0u, 0u};
        if (row < rows_valid) R.v[p] = *reinterpret_cast<const u4*>(src + (size_t)row * 64 + part * 8);
    }
}

__device__ __forceinline__ void tab_store(const TabRegs& R, __bf16* pc, __bf16* ps, int nrows) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int t = threadIdx.x + p * 256, row = t >> 3, part = t & 7;
        if (row < nrows)
            *reinterpret_cast<u4*>((part < 4 ? pc : ps) + row * PROW + (part & 3) * 8) = R.v[p];
    }
}

// The folded bins' part of a tile: per row the first ZX cos and ZX sin values
// of the next table chunk (2 x 8 bytes, one per thread, threads 0..127),
// stored in columns ZCB .. ZCB + ZX - 1 of the rows.
__device__ __forceinline__ void tab_load_x(TabRegs& R, const __bf16* __restrict__ src, int rows_valid) {
    const int t = threadIdx.x, row = t >> 1, part = t & 1;
    R.x = u2{0u, 0u};
    if (t < 128 && row < rows_valid) R.x = *reinterpret_cast<const u2*>(src + (size_t)row * 64 + part * ZCB);
}

__device__ __forceinline__ void tab_store_x(const TabRegs& R, __bf16* pc, __bf16* ps, int nrows) {
    const int t = threadIdx.x, row = t >> 1, part = t & 1;
    if (t < 128 && row < nrows) *reinterpret_cast<u2*>((part ? ps : pc) + row * PROW + ZCB) = R.x;
}

__device__ __forceinline__ s4v lds_s4(const __bf16* p) {
    return __builtin_bit_cast(s4v, *reinterpret_cast<const u2*>(p));
}

__device__ __forceinline__ s4v neg_s4(s4v v) {
    const u2 w = __builtin_bit_cast(u2, v);
    return __builtin_bit_cast(s4v, u2{w.x ^ 0x80008000u, w.y ^ 0x80008000u});
}

// Cooperative phasor generation: `rows` x ZCB entries of cos / sin(2 pi k u)
// for the tile rows' bins.  Thread t takes one reduction index and a run of
// `run` consecutive rows.  kidx(row) gives the bin, uval(col) the delay.
//   layout: pc[row * PROW + col], ps[row * PROW + col]
template <class KF, class UF>
__device__ __forceinline__ void gen_tile(__bf16* pc, __bf16* ps, int rows, int ncol, int run,
                                         KF kidx, UF uval) {
    const int groups = (rows + run - 1) / run;
    for (int t = threadIdx.x; t < groups * ncol; t += blockDim.x) {
        const int col = t % ncol, g = t / ncol;
        const uint32_t u = uval(col);
        float wc, ws;
        sincos_turns(u, wc, ws);
        int kprev = -2;
        float c = 0.f, s = 0.f;
        const int r_end = min(rows, (g + 1) * run);
        for (int r = g * run; r < r_end; ++r) {
            const int k = kidx(r);
            if (k == kprev + 1) {
                // angle addition: e^{j 2 pi (k-1) u} e^{j 2 pi u}
                float c2 = c * wc - s * ws;
                s = s * wc + c * ws;
                c = c2;
            } else {
                sincos_turns((uint32_t)k * u, c, s);
            }
            kprev = k;
            pc[r * PROW + col] = (__bf16)c;
            ps[r * PROW + col] = (__bf16)s;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
struct FwdB {
    const cbf16* x;        // [ny][nx][nz] bf16 complex
    cf32* yraw;            // [split][npos][mu]
    const uint32_t* u;
    const int* kb;
    int nx, ny, nz, wx, wy, mu;
    int sw, ntx, nty, nbt, split;
    int zsplit;            // depth-chunk split (partials [split * zsplit])
    int bt0, tile_bins;    // first bin tile of this launch, bins per (full) bin tile
    int64_t npos;
    int nblk;              // blocks of this plan's grid
    const __bf16* tab;     // phasor tiles [wy+1][wx+1][nzc][mu][2][32] or null
};

// WR: rows of waves in a tile (1: the 4 waves side by side along x; 2: a 2 x 2
// arrangement, half as wide and twice as tall, which needs fewer offsets per
// useful one when the aperture covers the whole grid).
template <int NP, int NB, int WR>
__device__ __forceinline__ void fwd_bf16_body(const FwdB& a, int b, const int nblk, unsigned char* smem) {
    static_assert(NB * 16 <= 64, "table tiles are copied in two passes of 256 x 16 bytes");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int sw = a.sw, sh = 16 / sw;
    constexpr int WC = 4 / WR;                   // waves per tile row
    const int tpx = WC * NP * sw, tpy = WR * sh;
    const int wave_x = wave % WC, wave_y = wave / WC;

    int per_xcd = nblk / 8;
    if (per_xcd * 8 == nblk) b = (b % 8) * per_xcd + b / 8;
    const int ntile = a.ntx * a.nty;
    const int tile = b % ntile;
    const int bt = a.bt0 + (b / ntile) % a.nbt;
    const int sp = b / (ntile * a.nbt);           // partial slot: d_y part + split * depth part
    const int dsp = sp % a.split, zsp = sp / a.split;
    const int px0 = (tile % a.ntx) * tpx, py0 = (tile / a.ntx) * tpy;
    const int cx_lo = max(0, px0 - a.wx), cx_hi = min(a.nx - 1, px0 + tpx - 1 + a.wx);
    const int ncol = cx_hi - cx_lo + 1;

    const int pitch = ncol;
    __bf16* halo = reinterpret_cast<__bf16*>(smem);                    // [tpy*pitch + 1][CELL]
    const int zero_cell = tpy * pitch;
    __bf16* ptile = halo + (size_t)(zero_cell + 1) * CELL;               // [2][2][NB*16][PROW]
    // delay slab [wx+1][ZCB] (phasor generation only: absent with tables), then bins [NB*16]
    uint32_t* ulds = reinterpret_cast<uint32_t*>(ptile + 2 * 2 * NB * 16 * PROW);
    int* klds = reinterpret_cast<int*>(ulds + (a.tab ? 0 : (a.wx + 1) * ZCB));

    int dy_lo = max(-a.wy, py0 - (a.ny - 1));
    int dy_hi = min(a.wy, py0 + tpy - 1);
    const int chunk = (dy_hi - dy_lo + 1 + a.split - 1) / a.split;
    dy_lo += dsp * chunk;
    dy_hi = min(dy_hi, dy_lo + chunk - 1);
    const int dx_lo = max(-a.wx, px0 - (a.nx - 1));
    const int dx_hi = min(a.wx, px0 + tpx - 1);
    // offsets at which this wave's own positions see a voxel column inside
    // the grid (wave-uniform; outside them its products would only read the
    // zero cell, so it skips them and leaves the matrix cores to other waves)
    const int wpx0 = px0 + wave_x * NP * sw, wpy0 = py0 + wave_y * sh;
    const int wdx_lo = wpx0 - (a.nx - 1), wdx_hi = min(wpx0 + NP * sw, a.nx) - 1;
    const int wdy_lo = wpy0 - (a.ny - 1), wdy_hi = min(wpy0 + sh, a.ny) - 1;
    // this block's depth chunks (an empty range leaves zeros in its partial slot)
    const int nzc_all = (a.nz + ZCB - 1) / ZCB;
    const int zc_per = (nzc_all + a.zsplit - 1) / a.zsplit;
    const int z_lo = zsp * zc_per * ZCB, z_hi = min(a.nz, (zsp + 1) * zc_per * ZCB);

    const int mb0 = bt * a.tile_bins;
    const int nbins = min(NB * 16, a.mu - mb0);          // valid bins of this tile
    const int nb_act = (nbins + 15) / 16;                // active bin sub-tiles
    const int i = lane & 15, kq = lane >> 4;

    for (int t = threadIdx.x; t < NB * 16; t += 256) klds[t] = t < nbins ? a.kb[mb0 + t] : 0;
    for (int t = threadIdx.x; t < CELL; t += 256) halo[(size_t)zero_cell * CELL + t] = (__bf16)0.f;

    f4 acc_re[NP][NB], acc_im[NP][NB];
#pragma unroll
    for (int s = 0; s < NP; ++s)
#pragma unroll
        for (int q = 0; q < NB; ++q) acc_re[s][q] = acc_im[s][q] = f4{0.f, 0.f, 0.f, 0.f};

    const int prow_count = nb_act * 16;
    for (int z0 = z_lo; z0 < z_hi; z0 += ZCB) {
        for (int dy = dy_lo; dy <= dy_hi; ++dy) {
            __syncthreads();
            // stage x rows (planar bf16) and the delay slab of |dy|
            // rows live in slot (grid row mod tpy): after the first d_y only the
            // row entering the window is loaded
            stage_planar<8>(halo, dy == dy_lo ? tpy : 1, ncol, pitch, tpy - 1, a.x, a.ny, a.nx, a.nz, py0 - dy,
                            cx_lo, z0, a.nz);
            const int ady = dy < 0 ? -dy : dy;
            if (!a.tab)
                for (int t = threadIdx.x; t < (a.wx + 1) * ZCB; t += 256) {
                    const int adx = t / ZCB, zz = t - adx * ZCB, z = z0 + zz;
                    ulds[t] = z < a.nz ? a.u[((int64_t)ady * (a.wx + 1) + adx) * a.nz + z] : 0u;
                }
            __syncthreads();
            auto gen = [&](int dx, int buf) {
                const int adx = dx < 0 ? -dx : dx;
                __bf16* pc = ptile + (size_t)buf * 2 * NB * 16 * PROW;
                __bf16* ps = pc + NB * 16 * PROW;
                gen_tile(pc, ps, prow_count, ZCB, (prow_count * ZCB + 255) / 256,
                         [&](int r) { return klds[r]; },
                         [&](int col) { return ulds[adx * ZCB + col]; });
            };
            // table tiles of this (|d_y|, depth chunk, bin tile), one per |d_x|
            const int nzc = (a.nz + ZCB - 1) / ZCB;
            const __bf16* tsrc = a.tab ? a.tab + (((int64_t)ady * (a.wx + 1) * nzc + z0 / ZCB) * a.mu + mb0) * 64
                                       : nullptr;
            const int64_t tstep = (int64_t)nzc * a.mu * 64;
            auto tile_at = [&](int dx) { return tsrc + (dx < 0 ? -dx : dx) * tstep; };
            // P_d depends on |d_x| only, so one staged tile serves d_x = +|d_x|
            // and -|d_x| (twice the products per tile and per barrier).  Table
            // path: tile |d_x| + 1 waits in registers (Rn) while |d_x| is
            // consumed and |d_x| + 2 is being loaded, so a load has two steps
            // to arrive.
            const int adx_hi = max(dx_hi, -dx_lo);
            const int adx_lo = (dx_lo <= 0 && dx_hi >= 0) ? 0 : min(dx_lo < 0 ? -dx_lo : dx_lo, dx_hi < 0 ? -dx_hi : dx_hi);
            const bool wy_ok = dy >= wdy_lo && dy <= wdy_hi;
            // this lane's halo column and byte address at d_x = 0 per sub-tile:
            // at d_x the cell is column - d_x when that column is staged, else
            // the zero cell (an add, a compare and a select per step)
            int hcol[NP], hadr[NP];
#pragma unroll
            for (int s = 0; s < NP; ++s) {
                hcol[s] = px0 + (wave_x * NP + s) * sw + i % sw - cx_lo;
                hadr[s] = (((py0 + wave_y * sh + i / sw - dy) & (tpy - 1)) * pitch + hcol[s]) * (CELL * 2);
            }
            TabRegs Ra, Rb;
            if (dx_lo <= dx_hi) {
                if (a.tab) {
                    TabRegs R0;
                    tab_load(R0, tile_at(adx_lo), nbins);
                    if (adx_lo < adx_hi) tab_load(Ra, tile_at(adx_lo + 1), nbins);
                    tab_store(R0, ptile, ptile + NB * 16 * PROW, prow_count);
                } else {
                    gen(adx_lo, 0);
                }
            }
            __syncthreads();
            // one offset step on LDS tile buffer BUF: tile |d_x| + 1 waits in
            // Rs (stored into the other buffer at the end of the step) while
            // tile |d_x| + 2 is loaded into Rl
            auto step = [&](const int adx, const int BUF, TabRegs& Rs, TabRegs& Rl) {
                const bool more = adx < adx_hi;
                if (a.tab) {
                    if (adx + 2 <= adx_hi) tab_load(Rl, tile_at(adx + 2), nbins);
                } else if (more) {
                    gen(adx + 1, BUF ^ 1);
                }
                const __bf16* pc = ptile + (size_t)BUF * 2 * NB * 16 * PROW;
                const __bf16* ps = pc + NB * 16 * PROW;
                // every bin sub-tile runs (no data-dependent exit), so the
                // 4 NP NB products issue in four independent passes; a last
                // bin tile with fewer sub-tiles is a launch of its own with a
                // smaller NB (host), else (grouped launches) the sub-tiles past
                // nb_act read stale LDS rows into accumulators never stored
                // -sin once for both signs of d_x, unless the registers it
                // needs would cost a wave per SIMD (the widest tiles)
                constexpr bool neg_once = NP * NB < 16;
                bf8 c8[NB], s8[NB], ns8[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    c8[nb] = lds_bf8(pc + (nb * 16 + i) * PROW + 8 * kq);
                    s8[nb] = lds_bf8(ps + (nb * 16 + i) * PROW + 8 * kq);
                    if constexpr (neg_once) ns8[nb] = neg_bf8(s8[nb]);
                }
                auto apply = [&](const int dx) {
                    // A operands: x at (p - d) for this lane's position of each sub-tile
                    bf8 xr[NP], xi[NP];
#pragma unroll
                    for (int s = 0; s < NP; ++s) {
                        const int ab = (unsigned)(hcol[s] - dx) < (unsigned)ncol ? hadr[s] - dx * (CELL * 2) : zero_cell * (CELL * 2);
                        const __bf16* hp = reinterpret_cast<const __bf16*>(reinterpret_cast<const unsigned char*>(halo) + ab);
                        xr[s] = lds_bf8(hp + 8 * kq);
                        xi[s] = lds_bf8(hp + ZCB + 8 * kq);
                    }
                    // (xr + j xi)(c - j s) = xr c + xi s + j (xi c - xr s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int s = 0; s < NP; ++s)
                            acc_re[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr[s], c8[nb], acc_re[s][nb], 0, 0, 0);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int s = 0; s < NP; ++s)
                            acc_im[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xi[s], c8[nb], acc_im[s][nb], 0, 0, 0);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int s = 0; s < NP; ++s)
                            acc_re[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xi[s], s8[nb], acc_re[s][nb], 0, 0, 0);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int s = 0; s < NP; ++s)
                            acc_im[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                xr[s], neg_once ? ns8[nb] : neg_bf8(s8[nb]), acc_im[s][nb], 0, 0, 0);
                };
                if (wy_ok && adx <= dx_hi && adx >= wdx_lo && adx <= wdx_hi) apply(adx);   // d_x = +|d_x|
                if (wy_ok && adx > 0 && -adx >= dx_lo && -adx >= wdx_lo && -adx <= wdx_hi)
                    apply(-adx);                                                          // d_x = -|d_x|
                if (more && a.tab) {
                    __bf16* pn = ptile + (size_t)(BUF ^ 1) * 2 * NB * 16 * PROW;
                    tab_store(Rs, pn, pn + NB * 16 * PROW, prow_count);
                }
                __syncthreads();
            };
            if (dx_lo <= dx_hi) {
                if constexpr (NP * NB < 16) {
                    // steps in pairs with the register sets and buffers
                    // swapped: nothing is copied between steps and the buffer
                    // offsets are constants
                    for (int adx = adx_lo; adx <= adx_hi; adx += 2) {
                        step(adx, 0, Ra, Rb);
                        if (adx + 1 > adx_hi) break;
                        step(adx + 1, 1, Rb, Ra);
                    }
                } else {
                    // the widest tiles: one step per iteration (the doubled
                    // loop body measured 2% slower there)
                    int buf = 0;
                    for (int adx = adx_lo; adx <= adx_hi; ++adx) {
                        step(adx, buf, Ra, Rb);
                        buf ^= 1;
                        Ra = Rb;
                    }
                }
            }
        }
    }
    cf32* yo = a.yraw + (int64_t)sp * a.npos * a.mu;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int q = wave_x * NP + s;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int mb = mb0 + nb * 16 + i;
            if (nb >= nb_act || mb >= a.mu) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int irow = 4 * kq + r;
                const int px = px0 + q * sw + irow % sw, py = py0 + wave_y * sh + irow / sw;
                if (px < a.nx && py < a.ny)
                    yo[((int64_t)py * a.nx + px) * a.mu + mb] = cf32{acc_re[s][nb][r], acc_im[s][nb][r]};
            }
        }
    }
}

template <int NP, int NB, int WR>
__global__ __launch_bounds__(256) void fwd_gemm_bf16_kernel(FwdB a) {
    extern __shared__ __align__(16) unsigned char smem[];
    fwd_bf16_body<NP, NB, WR>(a, blockIdx.x, gridDim.x, smem);
}

// Grouped launch: block -> (plan index, block index inside that plan's grid).
template <int NP, int NB>
__global__ __launch_bounds__(256) void fwd_gemm_bf16_kernel_grouped(const FwdB* __restrict__ descs,
                                                 const int2* __restrict__ blk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 sb = blk[blockIdx.x];
    const FwdB a = descs[sb.x];
    fwd_bf16_body<NP, NB, 1>(a, sb.y, a.nblk, smem);
}

// ---------------------------------------------------------------------------
// Adjoint.
// ---------------------------------------------------------------------------
struct AdjB {
    const cbf16* r;        // H-scaled operand [npos][mu] bf16 complex
    cf32* out;
    cf32* part;
    const uint32_t* u;
    const int* kb;
    int nx, ny, nz, wx, wy, mu;
    int sw, ntx, nty, nzt, split;
    int64_t nvox;
    int nblk;              // blocks of this plan's grid
    const __bf16* tab;     // phasor tiles [wy+1][wx+1][nkc][nz][2][32] or null
};

// EXT: the plan's last chunk holds at most ZX bins; they are folded into the
// previous chunk (phasors from the tables only).
template <int NV, int NZ, int WR, bool EXT = false>
__device__ __forceinline__ void adj_bf16_body(const AdjB& a, int b, const int nblk, unsigned char* smem) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int sw = a.sw, sh = 16 / sw;
    constexpr int WC = 4 / WR;                   // waves per tile row
    const int tvx = WC * NV * sw, tvy = WR * sh;
    const int wave_x = wave % WC, wave_y = wave / WC;
    const int zspan = NZ * 16;
    static_assert(NZ * 16 <= 64, "table tiles are copied in two passes of 256 x 16 bytes");

    int per_xcd = nblk / 8;
    if (per_xcd * 8 == nblk) b = (b % 8) * per_xcd + b / 8;
    const int ntile = a.ntx * a.nty;
    const int tile = b % ntile;
    const int zt = (b / ntile) % a.nzt;
    const int sp = b / (ntile * a.nzt);
    const int vx0 = (tile % a.ntx) * tvx, vy0 = (tile / a.ntx) * tvy;
    const int zw0 = zt * zspan;
    const int cx_lo = max(0, vx0 - a.wx), cx_hi = min(a.nx - 1, vx0 + tvx - 1 + a.wx);
    const int ncol = cx_hi - cx_lo + 1;

    const int pitch = ncol;
    __bf16* halo = reinterpret_cast<__bf16*>(smem);                  // [tvy*pitch + 1][CELL]
    const int zero_cell = tvy * pitch;
    __bf16* ptile = halo + (size_t)(zero_cell + 1) * CELL;               // [2][2][zspan][PROW]
    // delay slab [wx+1][zspan] (phasor generation only: absent with tables), then bins [ZCB]
    uint32_t* ulds = reinterpret_cast<uint32_t*>(ptile + 2 * 2 * zspan * PROW);
    int* klds = reinterpret_cast<int*>(ulds + (a.tab ? 0 : (a.wx + 1) * zspan));

    int dy_lo = max(-a.wy, -(vy0 + tvy - 1));
    int dy_hi = min(a.wy, a.ny - 1 - vy0);
    const int chunk = (dy_hi - dy_lo + 1 + a.split - 1) / a.split;
    dy_lo += sp * chunk;
    dy_hi = min(dy_hi, dy_lo + chunk - 1);
    const int dx_lo = max(-a.wx, -(vx0 + tvx - 1)), dx_hi = min(a.wx, a.nx - 1 - vx0);
    // offsets at which this wave's own voxels see a position inside the grid
    // (wave-uniform; the others are skipped, as in the forward)
    const int wvx0 = vx0 + wave_x * NV * sw, wvy0 = vy0 + wave_y * sh;
    const int wdx_lo = -(min(wvx0 + NV * sw, a.nx) - 1), wdx_hi = a.nx - 1 - wvx0;
    const int wdy_lo = -(min(wvy0 + sh, a.ny) - 1), wdy_hi = a.ny - 1 - wvy0;

    const int i = lane & 15, kq = lane >> 4;
    const int nz_act = min(NZ, (a.nz - zw0 + 15) / 16);   // active depth sub-tiles
    for (int t = threadIdx.x; t < CELL; t += 256) halo[(size_t)zero_cell * CELL + t] = (__bf16)0.f;

    f4 acc_re[NV][NZ], acc_im[NV][NZ];
#pragma unroll
    for (int s = 0; s < NV; ++s)
#pragma unroll
        for (int q = 0; q < NZ; ++q) acc_re[s][q] = acc_im[s][q] = f4{0.f, 0.f, 0.f, 0.f};

    const int nkm = EXT ? a.mu / ZCB : (a.mu + ZCB - 1) / ZCB;          // chunks run
    for (int kc = 0; kc < nkm; ++kc) {
        const int k0 = kc * ZCB;
        const bool ext = EXT && kc == nkm - 1;            // this chunk carries the folded bins
        for (int dy = dy_lo; dy <= dy_hi; ++dy) {
            __syncthreads();
            stage_planar<8>(halo, dy == dy_lo ? tvy : 1, ncol, pitch, tvy - 1, a.r, a.ny, a.nx, a.mu,
                            dy == dy_lo ? vy0 + dy : vy0 + dy + tvy - 1, cx_lo, k0, a.mu);
            if (ext)
                stage_planar<4, ZX>(halo, dy == dy_lo ? tvy : 1, ncol, pitch, tvy - 1, a.r, a.ny, a.nx, a.mu,
                                    dy == dy_lo ? vy0 + dy : vy0 + dy + tvy - 1, cx_lo, k0 + ZCB, a.mu,
                                    2 * ZCB, 2 * ZCB + ZX);
            const int ady = dy < 0 ? -dy : dy;
            if (!a.tab)
                for (int t = threadIdx.x; t < (a.wx + 1) * zspan; t += 256) {
                    const int adx = t / zspan, zz = t - adx * zspan, z = zw0 + zz;
                    ulds[t] = z < a.nz ? a.u[((int64_t)ady * (a.wx + 1) + adx) * a.nz + z] : 0u;
                }
            for (int t = threadIdx.x; t < ZCB; t += 256) klds[t] = (k0 + t < a.mu) ? a.kb[k0 + t] : 0;
            __syncthreads();
            auto gen = [&](int dx, int buf) {
                const int adx = dx < 0 ? -dx : dx;
                __bf16* pc = ptile + (size_t)buf * 2 * zspan * PROW;
                __bf16* ps = pc + zspan * PROW;
                // rows = depths, columns = bins: the recurrence runs along the bins
                // of one depth, so generate transposed: thread -> (depth, run of bins)
                const int runs = 4;                       // bins per thread run
                const int nruns = ZCB / runs;
                for (int t = threadIdx.x; t < zspan * nruns; t += blockDim.x) {
                    const int zz = t % zspan, g = t / zspan;
                    const uint32_t uu = ulds[adx * zspan + zz];
                    float wc, ws;
                    sincos_turns(uu, wc, ws);
                    int kprev = -2;
                    float c = 0.f, s = 0.f;
                    for (int j = g * runs; j < (g + 1) * runs; ++j) {
                        const int k = klds[j];
                        if (k == kprev + 1) {
                            float c2 = c * wc - s * ws;
                            s = s * wc + c * ws;
                            c = c2;
                        } else {
                            sincos_turns((uint32_t)k * uu, c, s);
                        }
                        kprev = k;
                        pc[zz * PROW + j] = (__bf16)c;
                        ps[zz * PROW + j] = (__bf16)s;
                    }
                }
            };
            // table tiles of this (|d_y|, bin chunk, depth tile), one per |d_x|
            const int nkc = (a.mu + ZCB - 1) / ZCB;
            const __bf16* tsrc = a.tab ? a.tab + (((int64_t)ady * (a.wx + 1) * nkc + k0 / ZCB) * a.nz + zw0) * 64
                                       : nullptr;
            const int64_t tstep = (int64_t)nkc * a.nz * 64;
            const int zrows = min(zspan, a.nz - zw0);
            auto tile_at = [&](int dx) { return tsrc + (dx < 0 ? -dx : dx) * tstep; };
            // the folded bins: the same rows of the next table chunk
            auto load = [&](TabRegs& R, int adx) {
                tab_load(R, tile_at(adx), zrows);
                if (ext) tab_load_x(R, tile_at(adx) + (int64_t)a.nz * 64, zrows);
            };
            auto store = [&](const TabRegs& R, __bf16* pn) {
                tab_store(R, pn, pn + zspan * PROW, zspan);
                if (ext) tab_store_x(R, pn, pn + zspan * PROW, zspan);
            };
            // as in the forward: one staged tile serves d_x = +|d_x| and -|d_x|,
            // with two steps of prefetch
            const int adx_hi = max(dx_hi, -dx_lo);
            const int adx_lo = (dx_lo <= 0 && dx_hi >= 0) ? 0 : min(dx_lo < 0 ? -dx_lo : dx_lo, dx_hi < 0 ? -dx_hi : dx_hi);
            const bool wy_ok = dy >= wdy_lo && dy <= wdy_hi;
            // as in the forward: halo column and byte address at d_x = 0 per
            // sub-tile (the cell at d_x is column + d_x), for the lane's voxel
            // i of the 16 x 16 products and voxel 4 kq + l % 4 of the folded ones
            int hcol[NV], hadr[NV], xcol[EXT ? NV : 1], xadr[EXT ? NV : 1];
#pragma unroll
            for (int s = 0; s < NV; ++s) {
                hcol[s] = vx0 + (wave_x * NV + s) * sw + i % sw - cx_lo;
                hadr[s] = (((vy0 + wave_y * sh + i / sw + dy) & (tvy - 1)) * pitch + hcol[s]) * (CELL * 2);
                if constexpr (EXT) {
                    const int iv = 4 * kq + (lane & 3);
                    xcol[s] = vx0 + (wave_x * NV + s) * sw + iv % sw - cx_lo;
                    xadr[s] = (((vy0 + wave_y * sh + iv / sw + dy) & (tvy - 1)) * pitch + xcol[s]) * (CELL * 2);
                }
            }
            TabRegs Ra, Rb;
            if (dx_lo <= dx_hi) {
                if (a.tab) {
                    TabRegs R0;
                    load(R0, adx_lo);
                    if (adx_lo < adx_hi) load(Ra, adx_lo + 1);
                    store(R0, ptile);
                } else {
                    gen(adx_lo, 0);
                }
            }
            __syncthreads();
            // steps in pairs with swapped register sets and buffers, as in the forward
            auto step = [&](const int adx, const int BUF, TabRegs& Rs, TabRegs& Rl) {
                const bool more = adx < adx_hi;
                if (a.tab) {
                    if (adx + 2 <= adx_hi) load(Rl, adx + 2);
                } else if (more) {
                    gen(adx + 1, BUF ^ 1);
                }
                const __bf16* pc = ptile + (size_t)BUF * 2 * zspan * PROW;
                const __bf16* ps = pc + zspan * PROW;
                // all NZ depth sub-tiles in four independent passes (inactive
                // ones are never stored)
                constexpr bool neg_once = NV * NZ < 16;     // as in the forward
                bf8 c8[NZ], s8[NZ], ns8[NZ];
#pragma unroll
                for (int q = 0; q < NZ; ++q) {
                    c8[q] = lds_bf8(pc + (q * 16 + i) * PROW + 8 * kq);
                    s8[q] = lds_bf8(ps + (q * 16 + i) * PROW + 8 * kq);
                    if constexpr (neg_once) ns8[q] = neg_bf8(s8[q]);
                }
                auto apply = [&](const int dx) {
                    bf8 rr8[NV], ri8[NV];
#pragma unroll
                    for (int s = 0; s < NV; ++s) {
                        const int ab = (unsigned)(hcol[s] + dx) < (unsigned)ncol ? hadr[s] + dx * (CELL * 2) : zero_cell * (CELL * 2);
                        const __bf16* hp = reinterpret_cast<const __bf16*>(reinterpret_cast<const unsigned char*>(halo) + ab);
                        rr8[s] = lds_bf8(hp + 8 * kq);
                        ri8[s] = lds_bf8(hp + ZCB + 8 * kq);
                    }
                    // (rr + j ri)(c + j s) = rr c - ri s + j (rr s + ri c)
#pragma unroll
                    for (int q = 0; q < NZ; ++q)
#pragma unroll
                        for (int s = 0; s < NV; ++s)
                            acc_re[s][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rr8[s], c8[q], acc_re[s][q], 0, 0, 0);
#pragma unroll
                    for (int q = 0; q < NZ; ++q)
#pragma unroll
                        for (int s = 0; s < NV; ++s)
                            acc_im[s][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(rr8[s], s8[q], acc_im[s][q], 0, 0, 0);
#pragma unroll
                    for (int q = 0; q < NZ; ++q)
#pragma unroll
                        for (int s = 0; s < NV; ++s)
                            acc_im[s][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ri8[s], c8[q], acc_im[s][q], 0, 0, 0);
#pragma unroll
                    for (int q = 0; q < NZ; ++q)
#pragma unroll
                        for (int s = 0; s < NV; ++s)
                            acc_re[s][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                ri8[s], neg_once ? ns8[q] : neg_bf8(s8[q]), acc_re[s][q], 0, 0, 0);
                    if constexpr (EXT) {
                        if (ext) {
                            // the folded bins: v_mfma_f32_4x4x4_16b_bf16, 16 blocks of
                            // 4 voxels x 4 depths with K = the ZX bins; block l / 4
                            // takes voxels 4 (l / 16) .. + 3 and depths 4 (l / 4 % 4)
                            // .. + 3, so lane l supplies voxel 4 kq + l % 4 (A) and depth
                            // i (B) and the result lands in the 16 x 16 accumulator layout
                            s4v rr4[NV], ri4[NV];
#pragma unroll
                            for (int s = 0; s < NV; ++s) {
                                const int ab = (unsigned)(xcol[s] + dx) < (unsigned)ncol ? xadr[s] + dx * (CELL * 2) : zero_cell * (CELL * 2);
                                const __bf16* hp = reinterpret_cast<const __bf16*>(reinterpret_cast<const unsigned char*>(halo) + ab);
                                rr4[s] = lds_s4(hp + 2 * ZCB);
                                ri4[s] = lds_s4(hp + 2 * ZCB + ZX);
                            }
#pragma unroll
                            for (int q = 0; q < NZ; ++q) {
                                const s4v c4 = lds_s4(pc + (q * 16 + i) * PROW + ZCB);
                                const s4v s4 = lds_s4(ps + (q * 16 + i) * PROW + ZCB);
                                const s4v n4 = neg_s4(s4);
#pragma unroll
                                for (int s = 0; s < NV; ++s) {
                                    acc_re[s][q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(rr4[s], c4, acc_re[s][q], 0, 0, 0);
                                    acc_im[s][q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(rr4[s], s4, acc_im[s][q], 0, 0, 0);
                                    acc_im[s][q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ri4[s], c4, acc_im[s][q], 0, 0, 0);
                                    acc_re[s][q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ri4[s], n4, acc_re[s][q], 0, 0, 0);
                                }
                            }
                        }
                    }
                };
                if (wy_ok && adx <= dx_hi && adx >= wdx_lo && adx <= wdx_hi) apply(adx);   // d_x = +|d_x|
                if (wy_ok && adx > 0 && -adx >= dx_lo && -adx >= wdx_lo && -adx <= wdx_hi)
                    apply(-adx);                                                          // d_x = -|d_x|
                if (more && a.tab) store(Rs, ptile + (size_t)(BUF ^ 1) * 2 * zspan * PROW);
                __syncthreads();
            };
            if (dx_lo <= dx_hi)
                for (int adx = adx_lo; adx <= adx_hi; adx += 2) {
                    step(adx, 0, Ra, Rb);
                    if (adx + 1 > adx_hi) break;
                    step(adx + 1, 1, Rb, Ra);
                }
        }
    }
    cf32* dst = a.split > 1 ? a.part + (int64_t)sp * a.nvox : a.out;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        const int q = wave_x * NV + s;
#pragma unroll
        for (int qz = 0; qz < NZ; ++qz) {
            if (qz >= nz_act) continue;
            const int z = zw0 + qz * 16 + i;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int irow = 4 * kq + r;
                const int vx = vx0 + q * sw + irow % sw, vy = vy0 + wave_y * sh + irow / sw;
                if (vx < a.nx && vy < a.ny && z < a.nz)
                    dst[((int64_t)vy * a.nx + vx) * a.nz + z] = cf32{acc_re[s][qz][r], acc_im[s][qz][r]};
            }
        }
    }
}

template <int NV, int NZ, int WR, bool EXT>
__global__ __launch_bounds__(256) void adj_gemm_bf16_kernel(AdjB a) {
    extern __shared__ __align__(16) unsigned char smem[];
    adj_bf16_body<NV, NZ, WR, EXT>(a, blockIdx.x, gridDim.x, smem);
}

// Grouped launch: block -> (plan index, block index inside that plan's grid).
template <int NV, int NZ>
__global__ __launch_bounds__(256) void adj_gemm_bf16_kernel_grouped(const AdjB* __restrict__ descs,
                                                 const int2* __restrict__ blk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 sb = blk[blockIdx.x];
    const AdjB a = descs[sb.x];
    adj_bf16_body<NV, NZ, 1>(a, sb.y, a.nblk, smem);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static constexpr int kBfNB = 4;     // forward: 4 x 16 bins per wave
static constexpr int kBfNZ = 4;     // adjoint: 4 x 16 depths per wave (default; 2 also built)
static constexpr size_t kLdsMaxB = 64 * 1024;

static int bf_sw(const Plan& P) { return P.g.ny == 1 ? 16 : 4; }

// Lateral sub-tiles of 16 per wave: 4 when the grid is wide enough that a
// 64-position tile row does not overhang it by much, else 2.  Batched
// (grouped) launches always use 2 and one wave row so one kernel fits every scan.
static int bf_np(const Plan& P) { return (P.g.ny > 1 && P.g.nx >= 48) ? 4 : 2; }

// Bin sub-tiles per forward tile: at most 4, spread evenly over the bin tiles
// (a 66-bin union takes 3 + 2 sub-tiles rather than 4 + 1: every bin tile pays
// the same staging and barriers per offset; measured 14% faster on the 32 x 32
// C-scan).  Tiles of 6 sub-tiles, one tile for 66 bins, measured slower.
static int bf_nb(const Plan& P, int) {
    const int nsub = ((int)P.ubins_h.size() + 15) / 16, ntile = (nsub + kBfNB - 1) / kBfNB;
    return std::max(1, (nsub + ntile - 1) / ntile);
}

// Tile of np sub-tiles per wave, 4 waves in wr rows.
static void bf_tile(const Plan& P, int np, int wr, int& tx, int& ty) {
    const int sw = bf_sw(P);
    tx = (4 / wr) * np * sw;
    ty = wr * (16 / sw);
}

// LDS bytes; `tables`: phasors copied from the tables (no delay slab needed).
static size_t fwd_bf16_lds(const Plan& P, int np, int nb, int wr, bool tables) {
    int tpx, tpy;
    bf_tile(P, np, wr, tpx, tpy);
    const int ncol = std::min(P.g.nx, tpx + 2 * P.d.wx);
    return (size_t)(tpy * ncol + 1) * CELL * 2 + (size_t)2 * 2 * nb * 16 * PROW * 2 +
           (tables ? 0 : (size_t)(P.d.wx + 1) * ZCB * 4) + nb * 16 * 4;
}

static size_t adj_bf16_lds(const Plan& P, int nv, int wr, bool tables, int nzs = kBfNZ) {
    int tvx, tvy;
    bf_tile(P, nv, wr, tvx, tvy);
    const int ncol = std::min(P.g.nx, tvx + 2 * P.d.wx);
    return (size_t)(tvy * ncol + 1) * CELL * 2 + (size_t)2 * 2 * nzs * 16 * PROW * 2 +
           (tables ? 0 : (size_t)(P.d.wx + 1) * nzs * 16 * 4) + ZCB * 4;
}

// The adjoint folds the last bin chunk into the previous one when it holds at
// most ZX bins and the phasors come from the tables.
static bool adj_bf16_ext(const Plan& P) {
    const int mu = (int)P.ubins_h.size(), rem = mu % ZCB;
    return P.d_ptab_a != nullptr && mu > ZCB && rem >= 1 && rem <= ZX;
}

// One-row tiles must fit with in-kernel phasor generation (the fallback).
bool bf16_supported(const Plan& P) {
    for (int np : {2, bf_np(P)})
        if (fwd_bf16_lds(P, np, bf_nb(P, np), 1, false) > kLdsMaxB ||
            adj_bf16_lds(P, np, 1, false) > kLdsMaxB)
            return false;
    return true;
}

bool bf16_rows_ok(const Plan& P, int fwd_rows, int adj_rows) {
    const int np = bf_np(P);
    if (P.g.ny == 1 && (fwd_rows > 1 || adj_rows > 1)) return false;   // B-scans: one row
    return fwd_bf16_lds(P, np, bf_nb(P, np), fwd_rows, P.d_ptab_f != nullptr) <= kLdsMaxB &&
           adj_bf16_lds(P, np, adj_rows, P.d_ptab_a != nullptr) <= kLdsMaxB;
}

int bf16_fwd_split(const Plan& P) {
    int tpx, tpy;
    bf_tile(P, bf_np(P), P.bf_fwd_rows, tpx, tpy);
    const int ntx = (P.g.nx + tpx - 1) / tpx, nty = (P.g.ny + tpy - 1) / tpy;
    const int mu = (int)P.ubins_h.size();
    const int nb = bf_nb(P, bf_np(P));
    const int nbt = (mu + nb * 16 - 1) / (nb * 16);
    const int wgs = ntx * nty * nbt;
    const int ndy_max = std::min(2 * P.d.wy + 1, P.g.ny + tpy - 1);
    int split = (1024 + wgs - 1) / wgs;
    split = std::max(1, std::min(split, std::min(ndy_max, 16)));
    const int chunk = (ndy_max + split - 1) / split;
    return (ndy_max + chunk - 1) / chunk;
}

int bf16_adj_split(const Plan& P) {
    int tvx, tvy;
    bf_tile(P, bf_np(P), P.bf_adj_rows, tvx, tvy);
    const int ntx = (P.g.nx + tvx - 1) / tvx, nty = (P.g.ny + tvy - 1) / tvy;
    const int nzt = (P.g.nz + kBfNZ * 16 - 1) / (kBfNZ * 16);
    const int wgs = ntx * nty * nzt;
    const int ndy_max = std::min(2 * P.d.wy + 1, P.g.ny + tvy - 1);
    int split = (1024 + wgs - 1) / wgs;
    split = std::max(1, std::min(split, std::min(ndy_max, 8)));
    const int chunk = (ndy_max + split - 1) / split;
    return (ndy_max + chunk - 1) / chunk;
}

static int fwdb_args(const Plan& P, FwdB& a, size_t& lds, int np, int nb, int wr) {
    a = FwdB{};
    a.x = static_cast<const cbf16*>(P.d_xop);
    a.yraw = P.d_yraw;
    a.u = P.d_u;
    a.kb = P.d_ubins;
    a.nx = P.g.nx;
    a.ny = P.g.ny;
    a.nz = P.g.nz;
    a.wx = P.d.wx;
    a.wy = P.d.wy;
    a.mu = (int)P.ubins_h.size();
    a.sw = bf_sw(P);
    int tpx, tpy;
    bf_tile(P, np, wr, tpx, tpy);
    a.ntx = (a.nx + tpx - 1) / tpx;
    a.nty = (a.ny + tpy - 1) / tpy;
    a.nbt = (a.mu + nb * 16 - 1) / (nb * 16);
    a.bt0 = 0;
    a.tile_bins = nb * 16;
    a.split = P.fwd_split;
    a.zsplit = std::max(1, P.fwd_zsplit);
    a.npos = P.npos;
    a.tab = static_cast<const __bf16*>(P.d_ptab_f);
    lds = fwd_bf16_lds(P, np, nb, wr, a.tab != nullptr);
    if (lds > kLdsMaxB) fail(UFSS_ERR_UNSUPPORTED, "aperture window too wide for the BF16 GEMM path");
    a.nblk = a.ntx * a.nty * a.nbt * a.split * a.zsplit;
    return a.nblk;
}

// nzs: 16-depth sub-tiles per wave (4, or 2 for twice the workgroups on
// shallow grids / small windows).
static int adjb_args(const Plan& P, cf32* out, AdjB& a, size_t& lds, int nv, int wr, int nzs) {
    a = AdjB{};
    a.r = static_cast<const cbf16*>(P.d_rop);
    a.out = out;
    a.part = P.d_gpart;
    a.u = P.d_u;
    a.kb = P.d_ubins;
    a.nx = P.g.nx;
    a.ny = P.g.ny;
    a.nz = P.g.nz;
    a.wx = P.d.wx;
    a.wy = P.d.wy;
    a.mu = (int)P.ubins_h.size();
    a.sw = bf_sw(P);
    int tvx, tvy;
    bf_tile(P, nv, wr, tvx, tvy);
    a.ntx = (a.nx + tvx - 1) / tvx;
    a.nty = (a.ny + tvy - 1) / tvy;
    a.nzt = (a.nz + nzs * 16 - 1) / (nzs * 16);
    a.split = P.adj_split;
    a.nvox = P.nvox;
    a.tab = static_cast<const __bf16*>(P.d_ptab_a);
    lds = adj_bf16_lds(P, nv, wr, a.tab != nullptr, nzs);
    if (lds > kLdsMaxB) fail(UFSS_ERR_UNSUPPORTED, "aperture window too wide for the BF16 GEMM path");
    a.nblk = a.ntx * a.nty * a.nzt * a.split;
    return a.nblk;
}

void launch_forward_gemm_bf16(const Plan& P, hipStream_t s) {
    FwdB a;
    size_t lds;
    const int np = bf_np(P), nb = bf_nb(P, np), wr = P.bf_fwd_rows == 2 ? 2 : 1;
    fwdb_args(P, a, lds, np, nb, wr);
    // bin tiles with all nb sub-tiles, then (if shorter) the last tile as a
    // launch of its own with exactly its active sub-tiles (no MFMA on padding)
    const int mu = (int)P.ubins_h.size();
    const int nb_last = (mu - (a.nbt - 1) * nb * 16 + 15) / 16;
    const int ntile = a.ntx * a.nty, nsplit = a.split * a.zsplit;
#define UFSS_FB(NPV, NBV, WRV) hipLaunchKernelGGL((fwd_gemm_bf16_kernel<NPV, NBV, WRV>), dim3(b.nblk), dim3(256), lds, s, b)
#define UFSS_FBN(NBRT, NPV, WRV)                                                  \
    do {                                                                          \
        if (NBRT == 4) UFSS_FB(NPV, 4, WRV);                                      \
        else if (NBRT == 3) UFSS_FB(NPV, 3, WRV);                                 \
        else if (NBRT == 2) UFSS_FB(NPV, 2, WRV);                                 \
        else UFSS_FB(NPV, 1, WRV);                                                \
    } while (0)
    auto launch = [&](const FwdB& b, int nbr) {
        if (np == 4) {
            if (wr == 2) UFSS_FBN(nbr, 4, 2); else UFSS_FBN(nbr, 4, 1);
        } else {
            if (wr == 2) UFSS_FBN(nbr, 2, 2); else UFSS_FBN(nbr, 2, 1);
        }
    };
    if (nb_last == nb) {
        launch(a, nb);
    } else {
        FwdB full = a, last = a;
        full.nbt = a.nbt - 1;
        full.nblk = ntile * full.nbt * nsplit;
        last.bt0 = a.nbt - 1;
        last.nbt = 1;
        last.nblk = ntile * nsplit;
        if (full.nbt > 0) launch(full, nb);
        launch(last, nb_last);
    }
#undef UFSS_FBN
#undef UFSS_FB
    UFSS_HIP(hipGetLastError());
}

void launch_adjoint_gemm_bf16(const Plan& P, cf32* out, hipStream_t s, bool sum) {
    AdjB a;
    size_t lds;
    const int nv = bf_np(P), wr = P.bf_adj_rows == 2 ? 2 : 1, nzs = P.bf_adj_nz == 2 ? 2 : 4;
    adjb_args(P, out, a, lds, nv, wr, nzs);
    const bool ext = adj_bf16_ext(P);
    const dim3 grid(a.nblk), block(256);
#define UFSS_AB(NVV, NZV, WRV)                                                                              \
    do {                                                                                                    \
        if (ext) hipLaunchKernelGGL((adj_gemm_bf16_kernel<NVV, NZV, WRV, true>), grid, block, lds, s, a);  \
        else hipLaunchKernelGGL((adj_gemm_bf16_kernel<NVV, NZV, WRV, false>), grid, block, lds, s, a);     \
    } while (0)
#define UFSS_ABZ(NVV, WRV)                                  \
    do {                                                    \
        if (nzs == 2) UFSS_AB(NVV, 2, WRV);                 \
        else UFSS_AB(NVV, 4, WRV);                          \
    } while (0)
    if (nv == 4) {
        if (wr == 2) UFSS_ABZ(4, 2); else UFSS_ABZ(4, 1);
    } else {
        if (wr == 2) UFSS_ABZ(2, 2); else UFSS_ABZ(2, 1);
    }
#undef UFSS_ABZ
#undef UFSS_AB
    UFSS_HIP(hipGetLastError());
    if (a.split > 1 && sum) launch_sum_parts(P.d_gpart, a.split, P.nvox, out, s);
}

// Phasor tables: entry (|d_y|, |d_x|, z, k) = cos / sin(2 pi kb[k] u(|d_y|, |d_x|, z))
// times the beam amplitude (when there is one), rounded to BF16, zero past nz
// or mu, written in both kernels' tile layouts.
__global__ void build_ptab_kernel(const uint32_t* __restrict__ u, const float* __restrict__ amp,
                                  const int* __restrict__ kb, int wx,
                                  int wy, int nz, int mu, int nzc, int nkc, __bf16* __restrict__ tf,
                                  __bf16* __restrict__ ta) {
    const int kw = nkc * ZCB, zw = nzc * ZCB;
    const int64_t n = (int64_t)(wy + 1) * (wx + 1) * zw * kw;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % kw);
        const int64_t r = t / kw;
        const int z = (int)(r % zw);
        const int64_t dxy = r / zw;                   // |d_y| * (wx + 1) + |d_x|
        float c = 0.f, sn = 0.f;
        if (z < nz && k < mu) {
            sincos_turns((uint32_t)kb[k] * u[dxy * nz + z], c, sn);
            if (amp) {
                const float gb = amp[dxy * nz + z];
                c *= gb;
                sn *= gb;
            }
        }
        if (k < mu) {
            __bf16* f = tf + ((dxy * nzc + z / ZCB) * mu + k) * 64 + z % ZCB;
            f[0] = (__bf16)c;
            f[ZCB] = (__bf16)sn;
        }
        if (z < nz) {
            __bf16* q = ta + ((dxy * nkc + k / ZCB) * nz + z) * 64 + k % ZCB;
            q[0] = (__bf16)c;
            q[ZCB] = (__bf16)sn;
        }
    }
}

static constexpr int64_t kPtabMax = int64_t(4) << 30;   // both tables together

static void bf16_build_tables(Plan& P) {
    const int mu = (int)P.ubins_h.size();
    const int nzc = (P.g.nz + ZCB - 1) / ZCB, nkc = (mu + ZCB - 1) / ZCB;
    const int64_t dxy = (int64_t)(P.d.wy + 1) * (P.d.wx + 1);
    const int64_t fb = dxy * nzc * mu * 64 * 2, ab = dxy * nkc * P.g.nz * 64 * 2;
    if (fb + ab > kPtabMax) return;                 // phasors generated in the kernels
    void *tf = nullptr, *ta = nullptr;
    if (hipMalloc(&tf, fb) != hipSuccess || hipMalloc(&ta, ab) != hipSuccess) {
        (void)hipGetLastError();                    // no room: generated in the kernels
        if (tf) (void)hipFree(tf);
        return;
    }
    const int64_t n = dxy * nzc * ZCB * nkc * ZCB;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(build_ptab_kernel, dim3(blocks), dim3(256), 0, nullptr, P.d_u, P.d_amp,
                       P.d_ubins, P.d.wx,
                       P.d.wy, P.g.nz, mu, nzc, nkc, static_cast<__bf16*>(tf), static_cast<__bf16*>(ta));
    UFSS_HIP(hipGetLastError());
    UFSS_HIP(hipDeviceSynchronize());
    P.d_ptab_f = tf;
    P.d_ptab_a = ta;
    P.ptab_bytes = fb + ab;
    P.ws_bytes += P.ptab_bytes;
}

void bf16_set_tables(Plan& P, int enable) {
    const bool bf_gemm = P.dtype == UFSS_BF16 && P.algo == UFSS_ALGO_GEMM;
    // the in-kernel phasor generation has no beam amplitude: a Gaussian beam
    // needs the tables
    if (bf_gemm && P.d_amp && !enable)
        fail(UFSS_ERR_UNSUPPORTED, "a BF16 plan with a Gaussian beam needs its phasor tables");
    UFSS_HIP(hipDeviceSynchronize());
    if (P.d_ptab_f) UFSS_HIP(hipFree(P.d_ptab_f));
    if (P.d_ptab_a) UFSS_HIP(hipFree(P.d_ptab_a));
    P.d_ptab_f = P.d_ptab_a = nullptr;
    P.ws_bytes -= P.ptab_bytes;
    P.ptab_bytes = 0;
    if (P.dtype != UFSS_BF16 || P.algo != UFSS_ALGO_GEMM) return;
    if (enable) bf16_build_tables(P);
    if (P.d_amp && !P.d_ptab_f)
        fail(UFSS_ERR_UNSUPPORTED, "BF16 phasor tables do not fit; a Gaussian beam needs them");
    // without tables the kernels also stage the delay slab: fall back to one-row
    // tiles where two rows no longer fit
    if (!bf16_rows_ok(P, P.bf_fwd_rows, P.bf_adj_rows)) P.bf_fwd_rows = P.bf_adj_rows = 1;
}

size_t bf16_desc_size(GemmKind k) { return k == GemmKind::FwdBF16 ? sizeof(FwdB) : sizeof(AdjB); }

int bf16_make_desc(GemmKind k, const Plan& P, const void* in, void* out, void* desc, size_t* lds) {
    (void)in;
    if (k == GemmKind::FwdBF16) return fwdb_args(P, *static_cast<FwdB*>(desc), *lds, 2, kBfNB, 1);
    return adjb_args(P, static_cast<cf32*>(out), *static_cast<AdjB*>(desc), *lds, 2, 1, kBfNZ);
}

void bf16_launch_grouped(GemmKind k, const void* descs, const int2* blk, int nblocks, size_t lds,
                         hipStream_t s) {
    if (k == GemmKind::FwdBF16)
        hipLaunchKernelGGL((fwd_gemm_bf16_kernel_grouped<2, kBfNB>), dim3(nblocks), dim3(256), lds,
                           s, static_cast<const FwdB*>(descs), blk);
    else
        hipLaunchKernelGGL((adj_gemm_bf16_kernel_grouped<2, kBfNZ>), dim3(nblocks), dim3(256), lds,
                           s, static_cast<const AdjB*>(descs), blk);
    UFSS_HIP(hipGetLastError());
}

}  // namespace ufss
