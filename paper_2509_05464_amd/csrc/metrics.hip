// image_quality: MSE, PSNR and SSIM of an image against its ground truth (Section 2.4.3;
// the paper applies them to maximum-intensity projections).  SSIM after Wang, Bovik,
// Sheikh and Simoncelli (IEEE TIP 2004): 11 x 11 Gaussian window (sigma 1.5, weights
// summing to 1), K1 = 0.01, K2 = 0.03, window-weighted moments, averaged over the
// positions where the window lies inside the image.  The images are small (projections),
// so one workgroup computes everything in FP64 and reduces in a fixed order
// (deterministic).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int IQM_THREADS = 1024;
constexpr int IQM_WIN = 11;

struct IqmArgs {
    const float* a;
    const float* b;
    double* out;      // [3]: MSE, PSNR, SSIM
    int nx, ny;
    double c1, c2, range2;
    double w[IQM_WIN];
};

__global__ void __launch_bounds__(IQM_THREADS) image_quality_kernel(const IqmArgs p) {
    __shared__ double s_mse[IQM_THREADS];
    __shared__ double s_ssim[IQM_THREADS];
    const int tid = threadIdx.x;
    const int64_t n = (int64_t)p.nx * p.ny;
    double m = 0.0;
    for (int64_t i = tid; i < n; i += IQM_THREADS) {
        const double d = (double)p.a[i] - (double)p.b[i];
        m = fma(d, d, m);
    }
    const int ox = p.nx - IQM_WIN + 1, oy = p.ny - IQM_WIN + 1;
    const int64_t npos = (int64_t)ox * oy;
    double ss = 0.0;
    for (int64_t q = tid; q < npos; q += IQM_THREADS) {
        const int y = (int)(q / ox), x = (int)(q % ox);
        double ma = 0.0, mb = 0.0, eaa = 0.0, ebb = 0.0, eab = 0.0;
        for (int dy = 0; dy < IQM_WIN; ++dy) {
            const float* ra = p.a + (int64_t)(y + dy) * p.nx + x;
            const float* rb = p.b + (int64_t)(y + dy) * p.nx + x;
#pragma unroll
            for (int dx = 0; dx < IQM_WIN; ++dx) {
                const double w = p.w[dy] * p.w[dx];
                const double va = ra[dx], vb = rb[dx];
                ma = fma(w, va, ma);
                mb = fma(w, vb, mb);
                eaa = fma(w * va, va, eaa);
                ebb = fma(w * vb, vb, ebb);
                eab = fma(w * va, vb, eab);
            }
        }
        const double sa = eaa - ma * ma, sb = ebb - mb * mb, sab = eab - ma * mb;
        ss += ((2.0 * ma * mb + p.c1) * (2.0 * sab + p.c2)) / ((ma * ma + mb * mb + p.c1) * (sa + sb + p.c2));
    }
    s_mse[tid] = m;
    s_ssim[tid] = ss;
    __syncthreads();
    for (int o = IQM_THREADS / 2; o > 0; o >>= 1) {
        if (tid < o) {
            s_mse[tid] += s_mse[tid + o];
            s_ssim[tid] += s_ssim[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double mse = s_mse[0] / (double)n;
        p.out[0] = mse;
        p.out[1] = mse > 0.0 ? 10.0 * log10(p.range2 / mse) : __builtin_inf();
        p.out[2] = s_ssim[0] / (double)npos;
    }
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" int image_quality(const float* img, const float* ref, int32_t nx, int32_t ny, double data_range,
                             double* out, void* stream) {
    FQ_REQUIRE(nx >= IQM_WIN && ny >= IQM_WIN, "images must be at least %d x %d (SSIM window)", IQM_WIN, IQM_WIN);
    FQ_REQUIRE((int64_t)nx * ny <= ((int64_t)1 << 24), "image larger than 2^24 pixels");
    FQ_REQUIRE(data_range > 0.0, "data_range must be > 0");
    FQ_REQUIRE(img && ref && out, "null pointer");
    IqmArgs p{};
    p.a = img;
    p.b = ref;
    p.out = out;
    p.nx = nx;
    p.ny = ny;
    p.c1 = (0.01 * data_range) * (0.01 * data_range);
    p.c2 = (0.03 * data_range) * (0.03 * data_range);
    p.range2 = data_range * data_range;
    double sum = 0.0;
    for (int i = 0; i < IQM_WIN; ++i) {
        const double t = i - 0.5 * (IQM_WIN - 1);
        p.w[i] = std::exp(-t * t / (2.0 * 1.5 * 1.5));
        sum += p.w[i];
    }
    for (int i = 0; i < IQM_WIN; ++i) p.w[i] /= sum;
    hipLaunchKernelGGL(image_quality_kernel, dim3(1), dim3(IQM_THREADS), 0, as_stream(stream), p);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
