// Batched FISTA over many uneven scans: one grid per phase, K iterations
// captured in one hipGraph, and a split-K autotuner with a JSON cache.
//
// Every phase of a FISTA iteration (forward GEMM, residual epilogue, adjoint
// pre pass, adjoint GEMM, update fused with the adjoint's split sums, FP64
// reductions, stats)
// runs as ONE grouped launch that covers all scans of the batch: block b reads
// blk[b] = {scan, local block} and the scan's descriptor, then executes the
// same tile code as the single-scan kernels.  The momentum weights depend on
// the iteration index only (paper Alg. 1), so they are baked into the captured
// launches and the graph runs K iterations with no host round trip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <vector>

#include "internal.h"

namespace ufss {

static constexpr int kT = 256;

// Per-scan descriptor of the elementwise phases.
struct ScanDesc {
    const cf32* y;
    cf32* x;          // a_k (caller's buffer)
    cf32* gamma;
    cf32* r;
    cf32* g;
    const cf32* yraw;
    void* rop;
    void* xop;
    const cf32* gpart;
    const int* map;
    const float* hsel;
    double* part;     // FP64 partials
    double* scal;     // scalars: [0] res2, [8..12] update norms, [16] ||gamma||_1
    double* stats;    // [K][4]
    int64_t npos, nvox;
    int m, mu, fsplit, asplit, per_pos, bf16, opw;
    float step, thresh;
    double lam;
    int nb_post, nb_upd, nb_vox;   // local grid sizes
};

// --- grouped elementwise kernels -------------------------------------------
__device__ __forceinline__ void wave_block_sum(double* v, int W, double* part, int slot_block,
                                               double (*red)[kT / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < W; ++w) {
        double x = v[w];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[w][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 0; w < W; ++w) {
            double s = 0.0;
            for (int i = 0; i < kT / 64; ++i) s += red[w][i];
            part[(int64_t)slot_block * W + w] = s;
        }
}

__global__ __launch_bounds__(kT) void g_to_bf16(const ScanDesc* __restrict__ d, const int2* __restrict__ blk) {
    const int2 sb = blk[blockIdx.x];
    const ScanDesc& a = d[sb.x];
    cbf16* out = static_cast<cbf16*>(a.xop);
    for (int64_t i = (int64_t)sb.y * kT + threadIdx.x; i < a.nvox; i += (int64_t)a.nb_vox * kT) {
        cf32 v = a.gamma[i];
        out[i] = to_cbf16(v.re, v.im);
    }
}

__global__ __launch_bounds__(kT) void g_post(const ScanDesc* __restrict__ d, const int2* __restrict__ blk) {
    __shared__ double red[1][kT / 64];
    const int2 sb = blk[blockIdx.x];
    const ScanDesc& a = d[sb.x];
    double acc = 0.0;
    const int64_t n = a.npos * a.m;
    for (int64_t i = (int64_t)sb.y * kT + threadIdx.x; i < n; i += (int64_t)a.nb_post * kT) {
        const int64_t p = i / a.m;
        const int mi = (int)(i - p * a.m);
        const int64_t sel = a.per_pos ? i : mi;
        const int j = a.map[sel];
        const float h = a.hsel[sel];
        const cf32 sum = sum_parts_ordered(a.yraw + p * a.mu + j, a.npos * a.mu, a.fsplit);
        const float re = sum.re * h - a.y[i].re;
        const float im = sum.im * h - a.y[i].im;
        a.r[i] = cf32{re, im};
        acc += (double)re * re + (double)im * im;
    }
    wave_block_sum(&acc, 1, a.part, sb.y, red);
}

// one block per (scan, position)
__global__ __launch_bounds__(128) void g_pre(const ScanDesc* __restrict__ d, const int2* __restrict__ blk) {
    const int2 sb = blk[blockIdx.x];
    const ScanDesc& a = d[sb.x];
    const int64_t p = sb.y;
    const int w = a.opw;
    if (a.bf16) {
        cbf16* row = static_cast<cbf16*>(a.rop) + p * w;
        for (int j = threadIdx.x; j < w; j += blockDim.x) row[j] = to_cbf16(0.f, 0.f);
        __syncthreads();
        for (int mi = threadIdx.x; mi < a.m; mi += blockDim.x) {
            const int64_t sel = a.per_pos ? p * a.m + mi : mi;
            const cf32 v = a.r[p * a.m + mi];
            const float h = a.hsel[sel];
            row[a.map[sel]] = to_cbf16(h * v.re, h * v.im);
        }
    } else {
        cf32* row = static_cast<cf32*>(a.rop) + p * w;
        for (int j = threadIdx.x; j < w; j += blockDim.x) row[j] = cf32{0.f, 0.f};
        __syncthreads();
        for (int mi = threadIdx.x; mi < a.m; mi += blockDim.x) {
            const int64_t sel = a.per_pos ? p * a.m + mi : mi;
            const cf32 v = a.r[p * a.m + mi];
            const float h = a.hsel[sel];
            row[a.map[sel]] = cf32{h * v.re, h * v.im};
        }
    }
}

__global__ __launch_bounds__(kT) void g_update(const ScanDesc* __restrict__ d, const int2* __restrict__ blk,
                                               float beta) {
    __shared__ double red[4][kT / 64];
    const int2 sb = blk[blockIdx.x];
    const ScanDesc& a = d[sb.x];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)sb.y * kT + threadIdx.x; i < a.nvox; i += (int64_t)a.nb_upd * kT) {
        const cf32 gm = a.gamma[i], aa = a.x[i];
        cf32 gg;
        if (a.asplit > 1) {
            // the adjoint's split-K partials, summed in fixed order (its epilogue)
            gg = sum_parts_ordered(a.gpart + i, a.nvox, a.asplit);
        } else {
            gg = a.g[i];
        }
        const float zr = gm.re - a.step * gg.re, zi = gm.im - a.step * gg.im;
        const float mag = sqrtf(zr * zr + zi * zi);
        const float sc = mag > a.thresh ? 1.0f - a.thresh / mag : 0.0f;
        const float ar = zr * sc, ai = zi * sc;
        const float gr = ar + beta * (ar - aa.re), gi = ai + beta * (ai - aa.im);
        a.x[i] = cf32{ar, ai};
        a.gamma[i] = cf32{gr, gi};
        const double dr = (double)ar - aa.re, di = (double)ai - aa.im;
        acc[0] += sqrt((double)ar * ar + (double)ai * ai);
        acc[1] += sqrt((double)gr * gr + (double)gi * gi);
        acc[2] += dr * dr + di * di;
        acc[3] += (double)ar * ar + (double)ai * ai;
    }
    wave_block_sum(acc, 4, a.part + 8192, sb.y, red);
}

// one block per scan: fixed-order sums of the partials, then the stats row
__global__ __launch_bounds__(kT) void g_finish(const ScanDesc* __restrict__ d, int k) {
    __shared__ double red[kT];
    const ScanDesc& a = d[blockIdx.x];
    double vals[5];
    for (int w = 0; w < 5; ++w) {
        const double* src = (w == 0) ? a.part : a.part + 8192;
        const int width = (w == 0) ? 1 : 4;
        const int col = (w == 0) ? 0 : w - 1;
        const int nb = (w == 0) ? a.nb_post : a.nb_upd;
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kT) s += src[(int64_t)b * width + col];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int off = kT / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        vals[w] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* st = a.stats + 4 * (int64_t)k;
        st[0] = 0.5 * vals[0] + a.lam * a.scal[16];
        st[1] = sqrt(vals[0]);
        st[2] = vals[4] > 0 ? sqrt(vals[3] / vals[4]) : 0.0;
        st[3] = 0.0;
        a.scal[16] = vals[2];
    }
}

// --- batch object -----------------------------------------------------------
struct Batch {
    std::vector<Plan*> plans;
    std::vector<int> gemm_idx;                         // scans on the grouped GEMM path
    void* d_desc = nullptr;                            // ScanDesc[n]
    std::map<int, std::pair<void*, size_t>> gdesc;     // GemmKind -> (device descs, lds)
    std::map<int, int> gthreads;                       // GemmKind -> threads per workgroup
    std::map<int, int> gcount;                         // GemmKind -> total blocks
    std::map<int, int2*> gblk;                         // GemmKind -> block table
    int2 *blk_post = nullptr, *blk_pre = nullptr, *blk_vox = nullptr, *blk_upd = nullptr,
         *blk_bf = nullptr;
    int n_post = 0, n_pre = 0, n_vox = 0, n_upd = 0, n_bf = 0;
    std::vector<void*> owned;
};

template <class T>
static T* upload_vec(Batch& B, const std::vector<T>& v) {
    void* p = nullptr;
    UFSS_HIP(hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T)));
    B.owned.push_back(p);
    if (!v.empty()) UFSS_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return static_cast<T*>(p);
}

static void free_batch(Batch& B) {
    for (void* p : B.owned) (void)hipFree(p);
    B.owned.clear();
}

int launch_absmax(int64_t n, const cf32* x, double* part, hipStream_t s);
void launch_reduce_max(const double* part, int nblk, double* out, hipStream_t s);
void op_forward(Plan& P, const cf32* x, cf32* y, const cf32* ymeas, double* res2_out, hipStream_t s);

// Persistent batch: descriptors built and K iterations captured in one hipGraph
// at creation; every run replays that graph (no capture, no host round trip
// inside the K iterations).  A run starts from the caller's x buffers (gamma =
// x and ||gamma||_1 are computed inside the graph), so replays with new
// measurements in the same y buffers solve the new problems.  The descriptors
// live in device memory and are read at run time: new lambdas need no capture.
struct BatchRun {
    Batch B;
    std::vector<Plan*> plans;
    std::vector<const cf32*> ys;
    std::vector<cf32*> xs;
    std::vector<double> L;
    std::vector<ScanDesc> sd;
    double* d_stats = nullptr;      // [n][iters][4], owned by the batch
    int n = 0, iters = 0;
    bool pinned = false;            // the plans' batch_refs were raised
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// x -> gamma and FP64 partials of ||gamma||_1 (in part + 8192, one column)
__global__ __launch_bounds__(kT) void g_init(const ScanDesc* __restrict__ d, const int2* __restrict__ blk) {
    __shared__ double red[1][kT / 64];
    const int2 sb = blk[blockIdx.x];
    const ScanDesc& a = d[sb.x];
    double acc = 0.0;
    for (int64_t i = (int64_t)sb.y * kT + threadIdx.x; i < a.nvox; i += (int64_t)a.nb_upd * kT) {
        const cf32 v = a.x[i];
        a.gamma[i] = v;
        acc += sqrt((double)v.re * v.re + (double)v.im * v.im);
    }
    wave_block_sum(&acc, 1, a.part + 8192, sb.y, red);
}

// one block per scan: ||gamma_0||_1 into scal[16], in fixed order
__global__ __launch_bounds__(kT) void g_init_finish(const ScanDesc* __restrict__ d) {
    __shared__ double red[kT];
    const ScanDesc& a = d[blockIdx.x];
    double s = 0.0;
    for (int b = threadIdx.x; b < a.nb_upd; b += kT) s += a.part[8192 + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.scal[16] = red[0];
}

static double resolve_lambda(Plan& P, const cf32* y, double lam, hipStream_t stream) {
    if (lam == 0 || std::isnan(lam)) fail(UFSS_ERR_INVALID_ARG, "lambda must be non-zero");
    if (lam > 0) return lam;
    op_adjoint(P, y, P.d_g, stream);
    int nb = launch_absmax(P.nvox, P.d_g, P.d_part, stream);
    launch_reduce_max(P.d_part, nb, P.d_scalars + 40, stream);
    double mx = 0;
    UFSS_HIP(hipMemcpyAsync(&mx, P.d_scalars + 40, 8, hipMemcpyDeviceToHost, stream));
    UFSS_HIP(hipStreamSynchronize(stream));
    return -lam * mx;
}

static void batch_free(BatchRun* R) {
    if (!R) return;
    if (R->exec) (void)hipGraphExecDestroy(R->exec);
    if (R->graph) (void)hipGraphDestroy(R->graph);
    free_batch(R->B);
    if (R->pinned)
        for (Plan* P : R->plans) --P->batch_refs;
    delete R;
}

BatchRun* batch_create(int n, Plan* const* plans, const cf32* const* ys, cf32* const* xs,
                       const double* lambdas, const double* Ls, int iters, hipStream_t stream) {
    if (n < 1) fail(UFSS_ERR_INVALID_ARG, "n must be >= 1");
    if (iters < 1) fail(UFSS_ERR_INVALID_ARG, "iters must be >= 1");
    if (!plans || !ys || !xs || !lambdas || !Ls) fail(UFSS_ERR_INVALID_ARG, "NULL array");
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !ys[i] || !xs[i]) fail(UFSS_ERR_INVALID_ARG, "NULL plan or buffer");
        if (plans[i]->algo != UFSS_ALGO_GEMM)
            fail(UFSS_ERR_UNSUPPORTED, "batched FISTA needs GEMM-path plans");
        if (plans[i]->d_amp)
            fail(UFSS_ERR_UNSUPPORTED, "batched FISTA does not take a Gaussian beam");
        if (plans[i]->mix)
            fail(UFSS_ERR_UNSUPPORTED, "batched FISTA does not take mixed plans");
        if (plans[i]->batch_refs > 0)
            fail(UFSS_ERR_INVALID_ARG, "a plan is already held by another persistent batch");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) fail(UFSS_ERR_INVALID_ARG, "a plan appears twice in the batch");
    }
    BatchRun* R = new BatchRun();
    Batch& B = R->B;
    try {
        R->n = n;
        R->iters = iters;
        R->plans.assign(plans, plans + n);
        R->ys.assign(ys, ys + n);
        R->xs.assign(xs, xs + n);
        // lambda (mu rule) and L per scan, resolved before capture
        std::vector<double> lam(n);
        R->L.resize(n);
        for (int i = 0; i < n; ++i) {
            Plan& P = *plans[i];
            R->L[i] = Ls[i] > 0 ? Ls[i] : P.lipschitz;
            if (!(R->L[i] > 0)) fail(UFSS_ERR_INVALID_ARG, "scan without a Lipschitz constant");
            lam[i] = resolve_lambda(P, ys[i], lambdas[i], stream);
        }
        {
            void* p = nullptr;
            UFSS_HIP(hipMalloc(&p, (size_t)n * iters * 4 * sizeof(double)));
            B.owned.push_back(p);
            R->d_stats = static_cast<double*>(p);
        }
        // descriptors
        std::vector<ScanDesc>& sd = R->sd;
        sd.resize(n);
        std::vector<int2> bpost, bpre, bupd, bbf;
        auto blocks_for = [](int64_t cnt) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (cnt + kT - 1) / kT)); };
        for (int i = 0; i < n; ++i) {
            Plan& P = *plans[i];
            ScanDesc& a = sd[i];
            a = ScanDesc{};
            a.y = ys[i];
            a.x = xs[i];
            a.gamma = P.d_gamma;
            a.r = P.d_r;
            a.g = P.d_g;
            a.yraw = P.d_yraw;
            a.rop = P.d_rop;
            a.xop = P.d_xop;
            a.gpart = P.d_gpart;
            a.map = P.d_map;
            a.hsel = P.d_hsel;
            a.part = P.d_part;
            a.scal = P.d_scalars;
            a.stats = R->d_stats + (size_t)i * iters * 4;
            a.npos = P.npos;
            a.nvox = P.nvox;
            a.m = P.m;
            a.mu = (int)P.ubins_h.size();
            a.fsplit = P.fwd_split * std::max(1, P.fwd_zsplit);
            a.asplit = P.adj_split;
            a.per_pos = P.per_position;
            a.bf16 = P.dtype == UFSS_BF16;
            a.opw = a.mu;
            a.step = (float)(1.0 / R->L[i]);
            a.thresh = (float)(lam[i] / R->L[i]);
            a.lam = lam[i];
            a.nb_post = blocks_for(P.npos * (int64_t)P.m);
            a.nb_upd = blocks_for(P.nvox);
            a.nb_vox = blocks_for(P.nvox);
            if (a.nb_post > 8192 || a.nb_upd * 4 > P.part_cap - 8192)
                fail(UFSS_ERR_UNSUPPORTED, "scan too large for the batched partial buffers");
            for (int b = 0; b < a.nb_post; ++b) bpost.push_back(int2{i, b});
            for (int b = 0; b < (int)P.npos; ++b) bpre.push_back(int2{i, b});
            for (int b = 0; b < a.nb_upd; ++b) bupd.push_back(int2{i, b});
            if (a.bf16)
                for (int b = 0; b < a.nb_vox; ++b) bbf.push_back(int2{i, b});
        }
        B.d_desc = upload_vec(B, sd);
        B.blk_post = upload_vec(B, bpost);
        B.n_post = (int)bpost.size();
        B.blk_pre = upload_vec(B, bpre);
        B.n_pre = (int)bpre.size();
        B.blk_upd = upload_vec(B, bupd);
        B.n_upd = (int)bupd.size();
        B.blk_bf = upload_vec(B, bbf);
        B.n_bf = (int)bbf.size();
        // grouped GEMM descriptors per kind
        for (int kind = 0; kind < 4; ++kind) {
            const GemmKind K = (GemmKind)kind;
            const bool want_bf16 = (K == GemmKind::FwdBF16 || K == GemmKind::AdjBF16);
            const bool fwd = (K == GemmKind::FwdF32 || K == GemmKind::FwdBF16);
            const size_t dsz = desc_size(K);
            std::vector<unsigned char> bytes;
            std::vector<int2> blk;
            size_t lds_max = 0;
            int threads_max = 64;
            int idx = 0;
            for (int i = 0; i < n; ++i) {
                Plan& P = *plans[i];
                if ((P.dtype == UFSS_BF16) != want_bf16) continue;
                std::vector<unsigned char> one(dsz);
                size_t lds = 0;
                int threads = 256;
                int nb = make_desc(K, P, fwd ? (const void*)P.d_gamma : nullptr,
                                   fwd ? nullptr : (P.adj_split > 1 ? (void*)P.d_gpart : (void*)P.d_g),
                                   one.data(), &lds, &threads);
                bytes.insert(bytes.end(), one.begin(), one.end());
                lds_max = std::max(lds_max, lds);
                threads_max = std::max(threads_max, threads);
                for (int b = 0; b < nb; ++b) blk.push_back(int2{idx, b});
                ++idx;
            }
            if (idx == 0) continue;
            B.gdesc[kind] = {upload_vec(B, bytes), lds_max};
            B.gthreads[kind] = threads_max;
            B.gblk[kind] = upload_vec(B, blk);
            B.gcount[kind] = (int)blk.size();
        }
        UFSS_HIP(hipStreamSynchronize(stream));

        // capture: start state, then K iterations
        hipStream_t cs;
        UFSS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        try {
            UFSS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            const ScanDesc* D = static_cast<const ScanDesc*>(B.d_desc);
            hipLaunchKernelGGL(g_init, dim3(B.n_upd), dim3(kT), 0, cs, D, B.blk_upd);
            hipLaunchKernelGGL(g_init_finish, dim3(n), dim3(kT), 0, cs, D);
            double t = 1.0;
            for (int k = 0; k < iters; ++k) {
                const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
                const float beta = (float)((t - 1.0) / tn);
                t = tn;
                if (B.n_bf) hipLaunchKernelGGL(g_to_bf16, dim3(B.n_bf), dim3(kT), 0, cs, D, B.blk_bf);
                for (int kind : {0, 2})
                    if (B.gcount.count(kind))
                        launch_grouped((GemmKind)kind, B.gdesc[kind].first, B.gblk[kind], B.gcount[kind],
                                       B.gdesc[kind].second, B.gthreads[kind], cs);
                hipLaunchKernelGGL(g_post, dim3(B.n_post), dim3(kT), 0, cs, D, B.blk_post);
                hipLaunchKernelGGL(g_pre, dim3(B.n_pre), dim3(128), 0, cs, D, B.blk_pre);
                for (int kind : {1, 3})
                    if (B.gcount.count(kind))
                        launch_grouped((GemmKind)kind, B.gdesc[kind].first, B.gblk[kind], B.gcount[kind],
                                       B.gdesc[kind].second, B.gthreads[kind], cs);
                hipLaunchKernelGGL(g_update, dim3(B.n_upd), dim3(kT), 0, cs, D, B.blk_upd, beta);
                hipLaunchKernelGGL(g_finish, dim3(n), dim3(kT), 0, cs, D, k);
            }
            UFSS_HIP(hipStreamEndCapture(cs, &R->graph));
            UFSS_HIP(hipGraphInstantiate(&R->exec, R->graph, nullptr, nullptr, 0));
        } catch (...) {
            hipStreamCaptureStatus st;
            if (hipStreamIsCapturing(cs, &st) == hipSuccess && st == hipStreamCaptureStatusActive) {
                hipGraph_t g2 = nullptr;
                (void)hipStreamEndCapture(cs, &g2);
                if (g2) (void)hipGraphDestroy(g2);
            }
            (void)hipStreamDestroy(cs);
            throw;
        }
        UFSS_HIP(hipStreamDestroy(cs));
        for (Plan* P : R->plans) ++P->batch_refs;
        R->pinned = true;
    } catch (...) {
        batch_free(R);
        throw;
    }
    return R;
}

void batch_set_lambdas(BatchRun& R, const double* lambdas, hipStream_t stream) {
    if (!lambdas) fail(UFSS_ERR_INVALID_ARG, "lambdas is NULL");
    std::vector<double> lam(R.n);
    for (int i = 0; i < R.n; ++i) lam[i] = resolve_lambda(*R.plans[i], R.ys[i], lambdas[i], stream);
    for (int i = 0; i < R.n; ++i) {
        R.sd[i].lam = lam[i];
        R.sd[i].thresh = (float)(lam[i] / R.L[i]);
    }
    UFSS_HIP(hipMemcpyAsync(R.B.d_desc, R.sd.data(), R.sd.size() * sizeof(ScanDesc),
                            hipMemcpyHostToDevice, stream));
    UFSS_HIP(hipStreamSynchronize(stream));
}

void batch_run(BatchRun& R, double* res_out, double* lambdas_out, hipStream_t stream) {
    UFSS_HIP(hipGraphLaunch(R.exec, stream));
    std::vector<double> h((size_t)R.n * R.iters * 4);
    UFSS_HIP(hipMemcpyAsync(h.data(), R.d_stats, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    UFSS_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < R.n; ++i) {
        const double* st = h.data() + (size_t)i * R.iters * 4;
        if (res_out) res_out[i] = st[4 * (R.iters - 1) + 1];
        if (lambdas_out) lambdas_out[i] = R.sd[i].lam;
        for (int k = 0; k < R.iters; ++k)
            if (!std::isfinite(st[4 * k]) || !std::isfinite(st[4 * k + 1]) || st[4 * k + 1] > 1e6 * st[1] + 1e-300)
                fail(UFSS_ERR_DIVERGED, "scan " + std::to_string(i) + " diverged at iteration " +
                                            std::to_string(k));
    }
}

void batch_destroy(BatchRun* R) {
    if (!R) fail(UFSS_ERR_INVALID_ARG, "batch is NULL");
    UFSS_HIP(hipDeviceSynchronize());
    batch_free(R);
}

int fista_batched(int n, Plan* const* plans, const cf32* const* ys, cf32* const* xs,
                  const double* lambdas, const double* Ls, int iters, hipStream_t stream,
                  double* res_out) {
    BatchRun* R = batch_create(n, plans, ys, xs, lambdas, Ls, iters, stream);
    try {
        batch_run(*R, res_out, nullptr, stream);
    } catch (...) {
        batch_free(R);
        throw;
    }
    batch_free(R);
    return UFSS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: split-K factors of the forward and adjoint GEMMs per shape class,
// chosen by timing every candidate with HIP events; results cached as JSON.
// ---------------------------------------------------------------------------

// Waves per forward workgroup the autotuner tries (FP32 kernel): 4, and one
// wave per 16-bin sub-tile of the whole bin list when that fits in 8.
static std::vector<int> nw_candidates(const Plan& P) {
    std::vector<int> c{4};
    const int all = ((int)P.ubins_h.size() + 15) / 16;
    if (P.dtype == UFSS_F32 && all > 4 && all <= 8) c.push_back(all);
    return c;
}

static std::string shape_key(const Plan& P) {
    std::ostringstream o;
    o << "gfx950/nx" << P.g.nx << "/ny" << P.g.ny << "/nz" << P.g.nz << "/mu" << P.ubins_h.size()
      << "/m" << P.m << "/wx" << P.d.wx << "/wy" << P.d.wy << "/" << (P.dtype == UFSS_BF16 ? "bf16" : "f32");
    if (P.d_amp) o << "/beam";       // beam plans run other kernel variants
    return o.str();
}

static std::map<std::string, std::vector<double>> read_cache(const std::string& path) {
    std::map<std::string, std::vector<double>> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        size_t q1 = line.find('"'), q2 = line.find('"', q1 + 1), b1 = line.find('['), b2 = line.find(']');
        if (q1 == std::string::npos || q2 == std::string::npos || b1 == std::string::npos || b2 == std::string::npos)
            continue;
        std::vector<double> v;
        std::stringstream ss(line.substr(b1 + 1, b2 - b1 - 1));
        std::string tok;
        while (std::getline(ss, tok, ',')) v.push_back(std::atof(tok.c_str()));
        if (v.size() >= 2) out[line.substr(q1 + 1, q2 - q1 - 1)] = v;
    }
    return out;
}

static void write_cache(const std::string& path, const std::map<std::string, std::vector<double>>& c) {
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (auto& kv : c) {
        f << "  \"" << kv.first << "\": [";
        for (size_t j = 0; j < kv.second.size(); ++j) f << (j ? ", " : "") << kv.second[j];
        f << "]" << (++i < c.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

static double time_ms(const std::function<void()>& fn, int reps, hipStream_t s) {
    fn();
    hipEvent_t e0, e1;
    UFSS_HIP(hipEventCreate(&e0));
    UFSS_HIP(hipEventCreate(&e1));
    UFSS_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) fn();
    UFSS_HIP(hipEventRecord(e1, s));
    UFSS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    UFSS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

int autotune(Plan& P, const char* cache_path, int flags, hipStream_t s, int32_t* fs_out, int32_t* as_out) {
    if (P.algo != UFSS_ALGO_GEMM) {
        if (fs_out) *fs_out = 1;
        if (as_out) *as_out = 1;
        return UFSS_OK;
    }
    const std::string key = shape_key(P);
    std::map<std::string, std::vector<double>> cache;
    if (cache_path && (flags & 1)) cache = read_cache(cache_path);
    if (cache.count(key) && cache[key].size() >= 12) {
        P.fwd_nw = (int)cache[key][4];
        P.fwd_np = (int)cache[key][6];
        P.adj_np = (int)cache[key][7];
        P.bf_fwd_rows = (int)cache[key][8];
        P.bf_adj_rows = (int)cache[key][9];
        P.fwd_zc = (int)cache[key][10];
        P.adj_kc = (int)cache[key][11];
        if (cache[key].size() >= 13) P.bf_adj_nz = (int)cache[key][12];
        if (cache[key].size() >= 14) P.adj_nw = (int)cache[key][13];
        plan_set_splits(P, (int)cache[key][0], (int)cache[key][1], (int)cache[key][5]);
    } else {
        const int tpy = P.g.ny == 1 ? 1 : 4;
        const int ndy = std::min(2 * P.d.wy + 1, P.g.ny + tpy - 1);
        std::vector<int> cand;
        for (int c : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
            if (c <= ndy) cand.push_back(c);
        // inputs: the plan's own workspace vectors hold finite values
        UFSS_HIP(hipMemsetAsync(P.d_gamma, 0, P.nvox * sizeof(cf32), s));
        UFSS_HIP(hipMemsetAsync(P.d_r, 0, (size_t)P.npos * P.m * sizeof(cf32), s));
        double best_f = 1e30, best_a = 1e30;
        int bf = P.fwd_split, ba = P.adj_split, bnw = P.fwd_nw, bz = P.fwd_zsplit;
        int bnp = P.fwd_np, bnpa = P.adj_np, bfr = P.bf_fwd_rows, bar = P.bf_adj_rows;
        // flags bit 2: quick search (d_y splits and two depth splits at the default tile shape)
        const bool quick = (flags & 4) != 0;
        // BF16 C-scans: one or two rows of waves per tile
        std::vector<int> rows{1};
        if (P.dtype == UFSS_BF16 && !quick && bf16_rows_ok(P, 2, 2)) rows.push_back(2);
        // FP32: 2 or 4 position sub-tiles per wave; BF16 picks its own tile width
        const std::vector<int> npc =
            (P.dtype == UFSS_F32 && !quick) ? std::vector<int>{2, 4} : std::vector<int>{2};
        std::vector<int> zcand{1};
        for (int z : {2, 4, 8})
            if (P.g.nz >= 32 * z) zcand.push_back(z);
        if (quick && zcand.size() > 2) zcand = {1, zcand[2]};
        const std::vector<int> nwc = quick ? std::vector<int>{P.fwd_nw} : nw_candidates(P);
        for (int wr : rows)
            for (int np : npc)
                for (int nw : nwc)
                    for (int zs : zcand)
                        for (int c : cand) {
                            if (c * zs > 96) continue;          // bounds the partial-sum workspace
                            P.fwd_nw = nw;
                            P.fwd_np = np;
                            P.bf_fwd_rows = wr;
                            plan_set_splits(P, c, P.adj_split, zs);
                            double t = time_ms([&]() { op_forward(P, P.d_gamma, P.d_r, nullptr, nullptr, s); }, 3, s);
                            if (t < best_f) { best_f = t; bf = c; bnw = nw; bz = zs; bnp = np; bfr = wr; }
                        }
        P.fwd_nw = bnw;
        P.fwd_np = bnp;
        P.bf_fwd_rows = bfr;
        // then the smaller depth chunk at that shape (FP32)
        int bzc = 16;
        if (P.dtype == UFSS_F32 && !quick) {
            for (int c : cand) {
                if (c * bz > 96) continue;
                P.fwd_zc = 8;
                plan_set_splits(P, c, P.adj_split, bz);
                double t = time_ms([&]() { op_forward(P, P.d_gamma, P.d_r, nullptr, nullptr, s); }, 3, s);
                if (t < best_f) { best_f = t; bf = c; bzc = 8; }
            }
        }
        P.fwd_zc = bzc;
        // BF16 adjoint: 4 or 2 depth sub-tiles per wave (2: twice the workgroups)
        const std::vector<int> nzc = P.dtype == UFSS_BF16 ? std::vector<int>{4, 2} : std::vector<int>{4};
        // FP32 adjoint with 2 sub-tiles per wave: 4 or 8 waves per workgroup
        const std::vector<int> awc =
            (P.dtype == UFSS_F32 && !quick) ? std::vector<int>{4, 8} : std::vector<int>{P.adj_nw};
        int bnz = P.bf_adj_nz, baw = P.adj_nw;
        for (int wr : rows)
            for (int np : npc)
                for (int nzs : nzc)
                    for (int aw : awc) {
                        if (aw == 8 && np != 2) continue;
                        for (int c : cand) {
                            P.adj_np = np;
                            P.bf_adj_rows = wr;
                            P.bf_adj_nz = nzs;
                            P.adj_nw = aw;
                            plan_set_splits(P, bf, c, bz);
                            double t = time_ms([&]() { op_adjoint(P, P.d_r, P.d_g, s); }, 3, s);
                            if (t < best_a) { best_a = t; ba = c; bnpa = np; bar = wr; bnz = nzs; baw = aw; }
                        }
                    }
        P.adj_np = bnpa;
        P.bf_adj_rows = bar;
        P.bf_adj_nz = bnz;
        P.adj_nw = baw;
        // then the smaller bin chunk at that shape (FP32)
        int bkc = 16;
        if (P.dtype == UFSS_F32 && !quick) {
            for (int c : cand) {
                P.adj_kc = 8;
                plan_set_splits(P, bf, c, bz);
                double t = time_ms([&]() { op_adjoint(P, P.d_r, P.d_g, s); }, 3, s);
                if (t < best_a) { best_a = t; ba = c; bkc = 8; }
            }
        }
        P.adj_kc = bkc;
        plan_set_splits(P, bf, ba, bz);
        if (cache_path && (flags & 2)) {
            cache = read_cache(cache_path);
            cache[key] = {(double)bf, (double)ba, best_f, best_a, (double)bnw, (double)bz, (double)bnp,
                          (double)bnpa, (double)bfr, (double)bar, (double)bzc, (double)bkc,
                          (double)P.bf_adj_nz, (double)P.adj_nw};
            write_cache(cache_path, cache);
        }
    }
    if (fs_out) *fs_out = P.fwd_split;
    if (as_out) *as_out = P.adj_split;
    return UFSS_OK;
}

}  // namespace ufss
