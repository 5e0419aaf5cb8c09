// Learned slow-time clutter filter (placeholder until the BF16 kernels land).
#include "fq_common.hpp"

using namespace fq;

extern "C" size_t lcf_act_size(int64_t, int32_t) { return 0; }
extern "C" int lcf_forward(const float*, const uint16_t*, const float*, int64_t, int32_t, float, uint16_t*, float*,
                           float*, void*) {
    set_error("lcf_forward: not built");
    return FQ_E_INVALID;
}
extern "C" int lcf_backward(const float*, const uint16_t*, const float*, const float*, int64_t, int32_t, float,
                            const uint16_t*, float*, float*, void*) {
    set_error("lcf_backward: not built");
    return FQ_E_INVALID;
}
extern "C" int lcf_adam_step(float*, uint16_t*, float*, float*, const float*, int32_t, float, float, float, float,
                             int32_t, void*) {
    set_error("lcf_adam_step: not built");
    return FQ_E_INVALID;
}
extern "C" int lcf_gather(const float*, int64_t, int32_t, int64_t, const int64_t*, int64_t, float*, void*) {
    set_error("lcf_gather: not built");
    return FQ_E_INVALID;
}
extern "C" size_t fallback_workspace_size(int64_t) { return 0; }
extern "C" int lcf_fallback(const float*, const float*, int64_t, float, void*, size_t, float*, int32_t*, float*,
                            void*) {
    set_error("lcf_fallback: not built");
    return FQ_E_INVALID;
}
