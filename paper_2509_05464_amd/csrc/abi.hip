// Library-wide pieces of the C ABI: error text, version, a fill kernel.
#include "fq_common.hpp"

namespace fq {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {
__global__ void zero_kernel(uint32_t* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}
}  // namespace

// Zero n_bytes (multiple of 4) with a kernel rather than a memset node, so that the
// call behaves the same inside a captured graph.
int zero_async(void* p, size_t n_bytes, hipStream_t s) {
    if (n_bytes == 0) return FQ_OK;
    size_t n = n_bytes / 4;
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), n);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

}  // namespace fq

extern "C" int fq_version(void) { return 1; }

extern "C" const char* fq_last_error(void) { return fq::g_err; }

// One dispatching query over the per-call workspace sizes (pure host arithmetic).
extern "C" size_t fq_workspace_size(int32_t which, const void* params) {
    if (!params) return 0;
    const fq_ws_query& q = *static_cast<const fq_ws_query*>(params);
    switch (which) {
        case FQ_WS_DAS:
        case FQ_WS_DAS_MIN:
            if (!q.probe || !q.tx) return 0;
            return das_workspace_size(q.probe, q.tx, q.n_t, q.n_samples, which == FQ_WS_DAS_MIN ? 1 : 0);
        case FQ_WS_GRAM:
            return gram_workspace_size(q.n, q.n_t, q.gram_mode);
        case FQ_WS_SVD:
            return svd_workspace_size(q.n, q.n_t);
        case FQ_WS_SSM:
            return ssm_workspace_size(q.n, q.n_t);
        case FQ_WS_FD:
            if (!q.probe || !q.tx || !q.pulse || !q.fd) return 0;
            return fd_workspace_size(q.probe, q.tx, q.pulse, q.fd, q.n_samples, q.n);
        case FQ_WS_DISPLAY:
            return display_workspace_size(q.n);
        case FQ_WS_FALLBACK:
            return fallback_workspace_size(q.n);
        case FQ_WS_LCF_ACT:
            return lcf_act_size(q.n, q.n_t);
        default:
            return 0;
    }
}
