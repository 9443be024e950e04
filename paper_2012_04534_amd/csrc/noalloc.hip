// Allocation-free variant of the standalone fused update (ufss_shrink_update_noalloc).
//
// The update's FP64 block partials and their reduced norms live in `scratch`, a
// file-scope device array every GPU holds for the life of the process, instead
// of a buffer allocated per call.  Host code never passes the array's name to a
// kernel or a copy: the name is only a host-side stand-in.  The device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and kept in `g_scratch_ptr`; every kernel argument and copy uses it.
//
// Capacity: 41 KB.  The update kernel's grid is capped at max_blocks_vec()
// blocks (grid-stride loop), so the array covers every n; the entry point
// refuses to launch if that cap ever exceeded the array's capacity.
//
// Every call on one GPU shares that GPU's array and leaves its contents behind;
// each call writes all partials it reads, so nothing needs clearing.  Calls that
// overlap on one GPU (two streams, or two host threads) race on the array.
#include <mutex>

#include "internal.h"

namespace ufss {

static constexpr int kScratchBlocks = 1024;                        // = max_blocks_vec()
static constexpr int kScratchDoubles = kScratchBlocks * 5 + 8;     // partials + 5 norms (+pad)

__device__ __align__(256) double scratch[kScratchDoubles];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
static double* scratch_on_current_device() {
    int dev = -1;
    UFSS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(UFSS_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        UFSS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(UFSS_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace ufss

extern "C" int ufss_shrink_update_noalloc(int64_t n, void* gamma, const void* g, void* a,
                                          double step, double thresh, double beta,
                                          const void* a_ref, double* norms_out,
                                          ufss_stream_t stream) {
    try {
        ufss::set_last_error("");
        if (n < 0 || (n > 0 && (!gamma || !g || !a)))
            ufss::fail(UFSS_ERR_INVALID_ARG, "bad size or NULL buffer");
        if (ufss::max_blocks_vec() > ufss::kScratchBlocks)
            ufss::fail(UFSS_ERR_UNSUPPORTED, "update grid exceeds the scratch array's capacity");
        hipStream_t s = static_cast<hipStream_t>(stream);
        double* part = ufss::scratch_on_current_device();
        double* out = part + (size_t)ufss::kScratchBlocks * 5;
        int nb = ufss::launch_update(n, static_cast<ufss::cf32*>(gamma),
                                     static_cast<const ufss::cf32*>(g), 1, static_cast<ufss::cf32*>(a),
                                     (float)step, (float)thresh, (float)beta,
                                     static_cast<const ufss::cf32*>(a_ref), part, s);
        ufss::launch_reduce(part, nb, 5, out, s);
        if (norms_out) {
            UFSS_HIP(hipMemcpyAsync(norms_out, out, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
            UFSS_HIP(hipStreamSynchronize(s));
        }
    } catch (const ufss::Error& e) {
        ufss::set_last_error(e.msg);
        return e.code;
    } catch (...) {
        ufss::set_last_error("unexpected exception");
        return UFSS_ERR_INVALID_ARG;
    }
    return UFSS_OK;
}
