// Internal declarations of libufss (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ufss.h"

namespace ufss {

// Error handling: C-ABI entry points catch ufss::Error and return its code.
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define UFSS_HIP(call) ::ufss::check_hip((call), #call)
void set_last_error(const std::string& msg);

// Complex value as stored in device memory (interleaved re, im).
struct cf32 {
    float re, im;
};

// Complex BF16 (round-to-nearest-even from FP32), used by BF16 plans.
struct cbf16 {
    __bf16 re, im;
};
__host__ __device__ inline cbf16 to_cbf16(float re, float im) {
    return cbf16{(__bf16)re, (__bf16)im};
}

// sum_{s < count} v[s * stride], added in order s = 0, 1, ... (the result
// does not depend on the grouping), with eight loads in flight: the split-K
// partials of the GEMMs are summed this way by every epilogue.
__device__ __forceinline__ cf32 sum_parts_ordered(const cf32* __restrict__ v, int64_t stride, int count) {
    float re = 0.f, im = 0.f;
    int s = 0;
    for (; s + 8 <= count; s += 8) {
        cf32 q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = v[(int64_t)(s + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            re += q[u].re;
            im += q[u].im;
        }
    }
    for (; s < count; ++s) {
        const cf32 q = v[(int64_t)s * stride];
        re += q.re;
        im += q.im;
    }
    return cf32{re, im};
}

// Host-side derived geometry, computed in FP64.
struct Derived {
    int wx = 0, wy = 0;                 // effective aperture half-widths
    double t0 = 0, sigma_f = 0, sigma_t = 0;
    int band_lo = 0, band_hi = -1;      // inclusive bin range of the band
    std::vector<int> band;              // ascending band bins
};
Derived derive(const ufss_geom& g);
// Random mixing of a plan: the Rademacher signs, one row or one per position.
struct MixSpec {
    int per_sign = 0;
    const int8_t* signs = nullptr;   // [1 or npos][nt] of +-1
};
// Geometry and bin-subset checks of ufss_plan_create (throws INVALID_ARG).
void validate_bins_public(const ufss_geom* g, int m, int per_position, const int32_t* bins);
void validate_geom_public(const ufss_geom* g);
double pulse_spectrum(const ufss_geom& g, const Derived& d, int k);

// Launch description of the operator kernels.  Everything a kernel needs is in
// these POD structs, passed by value.
struct OpDims {
    int nx, ny, nz;
    int wx, wy;         // window half-widths
    int mu;             // number of bins the GEMM runs over (M or union size)
};

// Plan: owns device tables and workspace.
struct Plan {
    ufss_geom g{};
    Derived d;
    int m = 0, per_position = 0, algo = 0, dtype = 0;
    int npos = 0;
    int64_t nvox = 0;
    int fwd_split = 1;             // split of the forward GEMM's d_y range
    int fwd_nw = 4;                // waves (16-bin sub-tiles) per forward FP32 workgroup
    int fwd_zsplit = 1;            // split of the forward FP32 GEMM's depth range
                                   // (raw output holds fwd_split * fwd_zsplit partials)
    int fwd_np = 2, adj_np = 2;    // FP32 GEMMs: 16-position sub-tiles per wave (2 or 4)
    int bf_fwd_rows = 1, bf_adj_rows = 1;   // BF16 GEMMs: rows of waves in a tile (1 or 2)
    int bf_adj_nz = 4;             // BF16 adjoint: 16-depth sub-tiles per wave (2 or 4)
    int fwd_zc = 16, adj_kc = 16;  // FP32 GEMMs: preferred staged depth / bin chunk (16 or 8)
    int adj_nw = 4;                // FP32 adjoint with 2 sub-tiles: waves per workgroup (4 or 8)
    int adj_split = 1;             // split of the adjoint GEMM's d_y range
    cf32* d_gpart = nullptr;       // adjoint partials [adj_split][nvox] (adj_split > 1)
    std::vector<int> bins_h;       // [m] or [npos*m]
    std::vector<int> ubins_h;      // union of bins (GEMM path), ascending
    // device tables
    int* d_bins = nullptr;         // selected bins [m] or [npos*m]
    int* d_ubins = nullptr;        // union bins [mu]
    int* d_map = nullptr;          // per (p, m): index into the union list
    float* d_hsel = nullptr;       // H_k per selection entry [m] or [npos*m]
    uint32_t* d_u = nullptr;       // integer-turn delay table [wy+1][wx+1][nz]
    float* d_amp = nullptr;        // Gaussian beam amplitude, same layout (theta > 0)
    // random mixing (Rademacher signs): the union is every DFT index (signed
    // bins), d_hsel holds H over the union and d_xih the transformed signs
    // [1 or npos][nt]
    int mix = 0, mix_per_sign = 0;
    void* d_xih = nullptr;
    // transform path (UFSS_ALGO_FFT): sizes, K^ quadrant [ly/2+1][lx/2+1][nz][mu],
    // twiddle tables and three work buffers
    int fft_lx = 0, fft_ly = 0;
    void* d_khat = nullptr;
    void* d_khat_t = nullptr;      // the same, transposed per entry: [..][mu][nz]
    cf32 *d_tw_fx = nullptr, *d_tw_fy = nullptr, *d_tw_ix = nullptr, *d_tw_iy = nullptr;
    cf32 *d_fa = nullptr, *d_fb = nullptr, *d_ft = nullptr;
    // device workspace
    cf32* d_yraw = nullptr;        // GEMM output over union bins [npos][mu]
    void* d_rop = nullptr;         // adjoint operand (H-scaled), [npos][mu] f32 or bf16
    void* d_xop = nullptr;         // forward operand in BF16 [nvox] (BF16 plans)
    // BF16 GEMM plans: precomputed phasor tiles (cos, sin of 2 pi k u) in BF16,
    // laid out as the kernels' LDS tiles; null = generated inside the kernels.
    //   forward [wy+1][wx+1][ceil(nz/32)][mu][2][32 depths]
    //   adjoint [wy+1][wx+1][ceil(mu/32)][nz][2][32 bins]
    void* d_ptab_f = nullptr;
    void* d_ptab_a = nullptr;
    int64_t ptab_bytes = 0;
    double* d_part = nullptr;      // FP64 block partials
    double* d_part_res = nullptr;  // FP64 partials of the residual norm, kept for a later reduction
    int part_cap = 0;
    double* d_scalars = nullptr;   // small FP64 results
    cf32* d_r = nullptr;           // residual [npos*m]
    cf32* d_g = nullptr;           // gradient [nvox]
    cf32* d_gamma = nullptr;       // FISTA extrapolated point [nvox]
    cf32* d_v = nullptr;           // power-iteration vector [nvox]
    double* d_stats = nullptr;     // FISTA per-iteration statistics
    // backtracking FISTA workspace (allocated on first use): three iterate
    // buffers [nvox], three residual buffers [npos*m], 16 FP64 results
    cf32* d_bt = nullptr;
    double* d_bt_scal = nullptr;
    int stats_cap = 0;
    int batch_refs = 0;            // persistent batches whose graph holds this plan's workspace
    double lipschitz = 0.0;
    int64_t ws_bytes = 0;
    hipStream_t cap_stream = nullptr;
    // kernel timing mode: HIP event pairs around each core kernel launch
    // (index 0 forward, 1 adjoint), recorded on the launch stream
    bool ktime = false;
    std::vector<hipEvent_t> kev[2];
    int kev_used[2] = {0, 0};
};

// Kernel launchers (kernels_*.hip).  All asynchronous on `s`.
void launch_forward_gemm(const Plan& P, const cf32* x, hipStream_t s);   // -> P.d_yraw
// P.d_rop -> out; with sum = false and a split > 1 the partials stay in P.d_gpart.
void launch_adjoint_gemm(const Plan& P, cf32* out, hipStream_t s, bool sum = true);
void launch_forward_phasor(const Plan& P, const cf32* x, cf32* y, const cf32* ymeas,
                           double* part, hipStream_t s);
void launch_adjoint_phasor(const Plan& P, cf32* out, hipStream_t s);     // P.d_rop -> out
// y[p][m] = H * yraw[p][map(p,m)] (- ymeas), FP64 partial sums of |y|^2 per block.
int launch_forward_post(const Plan& P, cf32* y, const cf32* ymeas, double* part, hipStream_t s);
// rop[p][j] = sum over m with map(p,m) = j of H * r[p][m] (zero elsewhere).
void launch_adjoint_pre(const Plan& P, const cf32* r, hipStream_t s);
void launch_to_bf16(const cf32* x, void* out, int64_t n, hipStream_t s);
int gemm_split(const Plan& P);
int adj_split(const Plan& P);
// Sets the split factors (and reallocates the split workspace when they change).
void plan_set_splits(Plan& P, int fs, int as, int zs);
// Lateral tile shape of the FP32 GEMMs (sub-tiles per wave, 2 or 4).
int fwd_tile_np(const Plan& P);
int adj_tile_np(const Plan& P);
// Waves per FP32 adjoint workgroup the GEMM actually uses (8 only with 2 sub-tiles).
int adj_waves(const Plan& P);
// The staged chunk the FP32 GEMMs actually use (the preference, halved until LDS fits).
int fwd_chunk(const Plan& P);
int adj_chunk(const Plan& P);
// Grouped GEMM launches: one grid runs the tiles of many plans.  A descriptor
// is the kernel's argument block for one plan (opaque bytes of desc_size);
// blk[b] = {plan index, block index inside that plan's own grid}.
enum class GemmKind { FwdF32 = 0, AdjF32 = 1, FwdBF16 = 2, AdjBF16 = 3 };
size_t desc_size(GemmKind k);
// Fills `desc` for plan P (in: forward input; out: adjoint output), the LDS
// bytes and the threads per workgroup it needs; returns the plan's block count.
int make_desc(GemmKind k, const Plan& P, const void* in, void* out, void* desc, size_t* lds, int* threads);
// One grid over many plans' blocks; `threads`: the most any of them needs.
void launch_grouped(GemmKind k, const void* descs, const int2* blk, int nblocks, size_t lds, int threads,
                    hipStream_t s);
size_t bf16_desc_size(GemmKind k);
int bf16_make_desc(GemmKind k, const Plan& P, const void* in, void* out, void* desc, size_t* lds);
void bf16_launch_grouped(GemmKind k, const void* descs, const int2* blk, int nblocks, size_t lds,
                         hipStream_t s);
bool bf16_supported(const Plan& P);
bool bf16_rows_ok(const Plan& P, int fwd_rows, int adj_rows);   // tile shapes fit in LDS
// Builds (enable != 0, if within the size limit) or frees the BF16 phasor tables.
void bf16_set_tables(Plan& P, int enable);
int bf16_fwd_split(const Plan& P);
int bf16_adj_split(const Plan& P);
void launch_forward_gemm_bf16(const Plan& P, hipStream_t s);
void launch_adjoint_gemm_bf16(const Plan& P, cf32* out, hipStream_t s, bool sum = true);
// out[i] = sum_{s < nsplit} part[s][i] in fixed order.
void launch_sum_parts(const cf32* part, int nsplit, int64_t n, cf32* out, hipStream_t s);

// Vector kernels.
// g: the gradient [n], or with nsplit > 1 the adjoint's split partials [nsplit][n].
int launch_update(int64_t n, cf32* gamma, const cf32* g, int nsplit, cf32* a, float step,
                  float thresh, float beta, const cf32* aref, double* part, hipStream_t s, int real = 0);
// Sums nblk partial blocks of `width` doubles in fixed order into out[width].
void launch_reduce(const double* part, int nblk, int width, double* out, hipStream_t s);
int launch_absmax(int64_t n, const cf32* x, double* part, hipStream_t s);
void launch_reduce_max(const double* part, int nblk, double* out, hipStream_t s);
int launch_norm2(int64_t n, const cf32* x, double* part, hipStream_t s);
void launch_scale(int64_t n, cf32* x, const double* norm2, hipStream_t s);   // x /= sqrt(norm2)
void launch_copy(int64_t n, const cf32* src, cf32* dst, hipStream_t s);
// the residual's partials reduced into res2_out and the update's five partial
// columns into upd_out, then the FISTA statistics of iteration k (objective,
// residual, relative change, error vs a reference) and the next ||gamma||_1,
// in one launch
void launch_reduce_fista_stats(const double* res_part, int res_nblk, double* res2_out,
                               const double* part, int nblk, double* upd_out, double* stats, int k,
                               double* g1, double lam, int have_ref, double ref2, hipStream_t s);

// Transform path (fft.hip).
void fft_setup(Plan& P);
int64_t fft_table_bytes(const Plan& P);
void fft_fwd_transform(const Plan& P, const cf32* x, hipStream_t s);
void fft_fwd_contract(const Plan& P, hipStream_t s);
void fft_fwd_inverse(const Plan& P, hipStream_t s);
void fft_adj_transform(const Plan& P, hipStream_t s);
void fft_adj_contract(const Plan& P, hipStream_t s);
void fft_adj_inverse(const Plan& P, cf32* out, hipStream_t s);

// Random mixing passes (vec.hip): they replace launch_forward_post and
// launch_adjoint_pre on mixed plans.
int launch_mix_post(const Plan& P, cf32* y, const cf32* ymeas, double* part, hipStream_t s);
void launch_mix_pre(const Plan& P, const cf32* r, hipStream_t s);

// Backtracking FISTA: trial step p = soft(gamma - step g, thresh) with six
// FP64 partials per block (see vec.hip); out = a + beta (a - b) with ||out||^2.
int launch_bt_prox(int64_t n, const cf32* gamma, const cf32* g, float step, float thresh,
                   cf32* p, const cf32* prev, const cf32* aref, double* part, hipStream_t s);
int launch_extrap(int64_t n, const cf32* a, const cf32* b, float beta, cf32* out, double* part,
                  hipStream_t s);

int max_blocks_vec();

// Operator drivers (operator.cpp).
// The forward operator with its residual epilogue, the FP64 block partials of
// ||y - ymeas||^2 left in part (capacity part_cap); returns their count.
int op_forward_partials(Plan& P, const cf32* x, cf32* y, const cf32* ymeas, double* part,
                        hipStream_t s);
void op_forward(Plan& P, const cf32* x, cf32* y, const cf32* ymeas, double* res2_out,
                hipStream_t s);
// Returns 1 when x holds A^H y; with defer_sum, the number of split partials
// left in P.d_gpart instead (> 1) for a consumer that sums them itself.
int op_adjoint(Plan& P, const cf32* y, cf32* x, hipStream_t s, bool defer_sum = false);

}  // namespace ufss
