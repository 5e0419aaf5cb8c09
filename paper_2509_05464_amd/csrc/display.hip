// display_db and mip: log-compressed display of B-mode and power-Doppler volumes over a
// dynamic range, and their maximum-intensity projections (Section 2.4.2; the results
// show B-mode over 75 dB, power Doppler over 60 dB, and MIPs onto the x-y, x-z and y-z
// planes).  All passes are HBM-bound streams.
//
//   displayed power p = PD (power) or |IQ|^2 (complex IQ; 20 log10 |IQ| = 10 log10 |IQ|^2)
//   out = max(-dr, 10 log10(p / max p));  max p == 0 shows everything at -dr;
//   or, as grey levels, 1 + out / dr in [0, 1].
// The reference max p comes from a two-pass reduction (block maxima, then one block); a
// maximum does not depend on the order of its operands, so the result is exact and
// deterministic.  The logarithms use the hardware log2 (error far below 1e-4 dB).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int DISP_THREADS = 256;
constexpr int DISP_MAX_BLOCKS = 1024;
constexpr float TEN_LOG10_2 = 3.0102999566398120f;   // 10 log10(2)

__device__ __forceinline__ float wave_max(float m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    return m;
}

// max over the block of 256 threads (4 waves); valid in thread 0
__device__ __forceinline__ float block_max(float m, float* s) {
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(s[0], s[1]), fmaxf(s[2], s[3]));
}

template <bool IQ>
__device__ __forceinline__ float power_at(const float* in, int64_t i) {
    if (IQ) {
        const float2 z = reinterpret_cast<const float2*>(in)[i];
        return z.x * z.x + z.y * z.y;
    }
    return in[i];
}

template <bool IQ>
__global__ void __launch_bounds__(DISP_THREADS) peak_partial_kernel(const float* in, int64_t n, float* part) {
    __shared__ float s[4];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * DISP_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * DISP_THREADS)
        m = fmaxf(m, power_at<IQ>(in, i));
    m = block_max(m, s);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(DISP_THREADS) peak_final_kernel(const float* part, int nb, float* peak) {
    __shared__ float s[4];
    float m = 0.0f;
    for (int i = threadIdx.x; i < nb; i += DISP_THREADS) m = fmaxf(m, part[i]);
    m = block_max(m, s);
    if (threadIdx.x == 0) *peak = m;
}

template <bool IQ>
__global__ void __launch_bounds__(DISP_THREADS) db_kernel(const float* in, int64_t n, const float* peak, float neg_dr,
                                                          int unit, float* out) {
    const float pk = *peak;
    const float lpk = __builtin_amdgcn_logf(pk);   // log2
    for (int64_t i = (int64_t)blockIdx.x * DISP_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * DISP_THREADS) {
        const float p = power_at<IQ>(in, i);
        float d = neg_dr;
        if (pk > 0.0f && p > 0.0f) d = fmaxf(neg_dr, TEN_LOG10_2 * (__builtin_amdgcn_logf(p) - lpk));
        // grey level (d + dr) / dr: exactly 0 at the floor and 1 at the peak
        out[i] = unit ? (d - neg_dr) / -neg_dr : d;
    }
}

// MIP onto x-y (max over z) or x-z (max over y): one thread per output pixel, the
// reduction runs along a strided axis while neighbouring threads read neighbouring x.
__global__ void __launch_bounds__(DISP_THREADS) mip_strided_kernel(const float* vol, int nx, int ny, int nz,
                                                                   int over_z, float* out) {
    const int64_t idx = (int64_t)blockIdx.x * DISP_THREADS + threadIdx.x;
    const int64_t n_out = over_z ? (int64_t)nx * ny : (int64_t)nx * nz;
    if (idx >= n_out) return;
    const int ix = (int)(idx % nx);
    const int o = (int)(idx / nx);   // iy (over z) or iz (over y)
    float m = -INFINITY;
    if (over_z) {
        for (int iz = 0; iz < nz; ++iz) m = fmaxf(m, vol[((int64_t)iz * ny + o) * nx + ix]);
    } else {
        for (int iy = 0; iy < ny; ++iy) m = fmaxf(m, vol[((int64_t)o * ny + iy) * nx + ix]);
    }
    out[idx] = m;
}

// MIP onto y-z (max over x): one wave per row of x.
__global__ void __launch_bounds__(DISP_THREADS) mip_rows_kernel(const float* vol, int nx, int64_t n_rows, float* out) {
    const int64_t row = (int64_t)blockIdx.x * (DISP_THREADS / 64) + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const int l = threadIdx.x & 63;
    const float* r = vol + row * nx;
    float m = -INFINITY;
    for (int ix = l; ix < nx; ix += 64) m = fmaxf(m, r[ix]);
    m = wave_max(m);
    if (l == 0) out[row] = m;
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(DISP_MAX_BLOCKS, (n + DISP_THREADS - 1) / DISP_THREADS)); }

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t display_workspace_size(int64_t n) {
    (void)n;
    return sizeof(float) * (DISP_MAX_BLOCKS + 64);
}

extern "C" int display_db(const float* in, int64_t n, int32_t kind, float dr_db, void* ws, size_t ws_bytes, float* out,
                          float* peak, void* stream) {
    FQ_REQUIRE(n >= 1, "n must be >= 1");
    const bool unit = (kind & FQ_DISP_UNIT) != 0;
    kind &= ~FQ_DISP_UNIT;
    FQ_REQUIRE(kind == FQ_DISP_POWER || kind == FQ_DISP_IQ, "kind must be FQ_DISP_POWER or FQ_DISP_IQ (| FQ_DISP_UNIT)");
    FQ_REQUIRE(dr_db > 0.0f && dr_db < 1000.0f, "dr_db must be in (0, 1000)");
    FQ_REQUIRE(in && out && ws && aligned16(in) && aligned16(out) && aligned16(ws), "null or misaligned pointer");
    if (ws_bytes < display_workspace_size(n)) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, display_workspace_size(n));
        return FQ_E_WORKSPACE;
    }
    hipStream_t s = as_stream(stream);
    float* part = reinterpret_cast<float*>(ws);
    float* pk = peak ? peak : part + DISP_MAX_BLOCKS;
    const int nb = blocks_for(n);
    if (kind == FQ_DISP_IQ)
        hipLaunchKernelGGL(peak_partial_kernel<true>, dim3(nb), dim3(DISP_THREADS), 0, s, in, n, part);
    else
        hipLaunchKernelGGL(peak_partial_kernel<false>, dim3(nb), dim3(DISP_THREADS), 0, s, in, n, part);
    FQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(peak_final_kernel, dim3(1), dim3(DISP_THREADS), 0, s, part, nb, pk);
    FQ_LAUNCH_CHECK();
    if (kind == FQ_DISP_IQ)
        hipLaunchKernelGGL(db_kernel<true>, dim3(nb), dim3(DISP_THREADS), 0, s, in, n, pk, -dr_db, unit ? 1 : 0, out);
    else
        hipLaunchKernelGGL(db_kernel<false>, dim3(nb), dim3(DISP_THREADS), 0, s, in, n, pk, -dr_db, unit ? 1 : 0, out);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

extern "C" int mip(const float* vol, int32_t nx, int32_t ny, int32_t nz, int32_t plane, float* out, void* stream) {
    FQ_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, "bad volume size");
    FQ_REQUIRE(plane == FQ_MIP_XY || plane == FQ_MIP_XZ || plane == FQ_MIP_YZ, "bad plane");
    FQ_REQUIRE(vol && out && aligned16(vol) && aligned16(out), "null or misaligned pointer");
    hipStream_t s = as_stream(stream);
    if (plane == FQ_MIP_YZ) {
        const int64_t rows = (int64_t)ny * nz;
        const unsigned nb = (unsigned)((rows + DISP_THREADS / 64 - 1) / (DISP_THREADS / 64));
        hipLaunchKernelGGL(mip_rows_kernel, dim3(nb), dim3(DISP_THREADS), 0, s, vol, nx, rows, out);
    } else {
        const int over_z = plane == FQ_MIP_XY ? 1 : 0;
        const int64_t n_out = over_z ? (int64_t)nx * ny : (int64_t)nx * nz;
        const unsigned nb = (unsigned)((n_out + DISP_THREADS - 1) / DISP_THREADS);
        hipLaunchKernelGGL(mip_strided_kernel, dim3(nb), dim3(DISP_THREADS), 0, s, vol, nx, ny, nz, over_z, out);
    }
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
