// roof_probe: microbenchmarks of the on-chip ceilings the kernels are priced against
// (gfx950): the LDS read bandwidth (16-byte reads, every lane a distinct 16-byte slot,
// conflict-free) and the FP32 FMA issue rate (8 independent chains per lane).  Every
// access stays inside the workgroup's 64 KB LDS buffer; the results are folded into one
// value per thread so the work is not dropped.
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_LDS_F4 = 4096;   // 64 KB

__global__ void __launch_bounds__(PROBE_THREADS) lds_read_probe(int iters, float* out) {
    __shared__ float4 buf[PROBE_LDS_F4];
    const int tid = threadIdx.x;
    for (int i = tid; i < PROBE_LDS_F4; i += PROBE_THREADS)
        buf[i] = make_float4((float)i, (float)(i + 1), (float)(i + 2), (float)(i + 3));
    __syncthreads();
    unsigned int a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int base = tid;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 v = buf[(base + u * PROBE_THREADS) & (PROBE_LDS_F4 - 1)];
            a0 ^= __float_as_uint(v.x);
            a1 ^= __float_as_uint(v.y);
            a2 ^= __float_as_uint(v.z);
            a3 ^= __float_as_uint(v.w);
        }
        base = (base + 8 * PROBE_THREADS + 1) & (PROBE_LDS_F4 - 1);
    }
    out[(size_t)blockIdx.x * PROBE_THREADS + tid] = __uint_as_float(a0 ^ a1 ^ a2 ^ a3);
}

__global__ void __launch_bounds__(PROBE_THREADS) fma_probe(int iters, float* out) {
    const int tid = threadIdx.x;
    float c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = (float)(tid + q) * 1e-3f;
    const float m = 0.999999f, s = 1e-7f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = fmaf(c[q], m, s);
    }
    float r = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) r += c[q];
    out[(size_t)blockIdx.x * PROBE_THREADS + tid] = r;
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" int roof_probe(int32_t which, int32_t n_blocks, int32_t iters, float* out, void* stream) {
    FQ_REQUIRE(which == FQ_PROBE_LDS_READ || which == FQ_PROBE_FP32_FMA, "bad probe");
    FQ_REQUIRE(n_blocks >= 1 && iters >= 1, "bad probe sizes");
    FQ_REQUIRE(out && aligned16(out), "null or misaligned pointer");
    hipStream_t s = as_stream(stream);
    if (which == FQ_PROBE_LDS_READ)
        hipLaunchKernelGGL(lds_read_probe, dim3(n_blocks), dim3(PROBE_THREADS), 0, s, iters, out);
    else
        hipLaunchKernelGGL(fma_probe, dim3(n_blocks), dim3(PROBE_THREADS), 0, s, iters, out);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
