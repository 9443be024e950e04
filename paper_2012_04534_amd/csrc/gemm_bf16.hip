// BF16 variants of the windowed GEMM kernels (placeholder until implemented).
#include "internal.h"

namespace ufss {

void launch_forward_gemm_bf16(const Plan&, hipStream_t) {
    fail(UFSS_ERR_UNSUPPORTED, "BF16 operator not built yet");
}

void launch_adjoint_gemm_bf16(const Plan&, cf32*, hipStream_t) {
    fail(UFSS_ERR_UNSUPPORTED, "BF16 operator not built yet");
}

}  // namespace ufss
