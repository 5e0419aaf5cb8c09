// rf_synth: analytic RF of point scatterers under tilted plane-wave transmits (gfx950).
//
// One workgroup is one wavefront and owns one trace (frame, transmit, receive element),
// held in LDS, so no two waves ever touch the same LDS word and small workgroups keep
// many waves resident to hide LDS latency.  The wave sweeps the scatterers in batches of
// 64: lane l computes, for scatterer l of the batch, in FP64 a small record:
// the first sample n0 of the truncated pulse, the offset u0 = n0 - x of that sample
// from the two-way delay x (FP64, in samples), the amplitude and cos/sin(theta u0).
// The wave then walks the 64 records one by one with lane k computing pulse sample
// n0 + k directly:
//     g = amp * exp(-(u0 + k)^2 / 2s^2) * (cos(theta k) cos(theta u0) - sin(theta k) sin(theta u0))
// and adding it to the trace word n0 + k.  The lanes of one record address distinct,
// consecutive words, and each trace belongs to one wave, so plain LDS read-add-write
// is race-free: no atomics, and the result is bitwise reproducible.  The whole trace is
// written (or added) to global memory once at the end, and for static scatterers to
// every frame (Algorithm 1 reuses the static tissue RF for all frames).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int RF_THREADS = 64;       // one wave per workgroup, one trace per wave
constexpr int RF_LDS_FLOATS = 16384;  // per-trace budget (64 KiB)
constexpr int RF_MAX_SPAN = 64;       // pulse samples per record (one per lane)

struct RfArgs {
    const float* pos;
    const float* amp;
    float* rf;
    int64_t n_scat;
    int n_frames, n_angles, n_elem, T;
    int nx_el;
    int accumulate;
    double pitch_x, pitch_y;
    double fs_c;            // fs / c (samples per metre)
    double half;            // pulse half-support, samples
    float kexp;             // -log2(e) / (2 s^2), s in samples
    float theta;            // 2 pi fc / fs
    float r_ref;
    float ck[RF_MAX_SPAN], sk[RF_MAX_SPAN];   // cos(theta k), sin(theta k)
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES], t0s[FQ_MAX_ANGLES];  // t0s = t0 * fs
};

struct Rec {
    float u0, amp, cu, su;
};

template <bool STATIC>
__global__ void __launch_bounds__(RF_THREADS) rf_synth_kernel(const RfArgs a) {
    extern __shared__ float tr[];  // [T]
    __shared__ Rec rec[64];
    __shared__ int rnc[64];        // n0 * 64 + count
    const int e = blockIdx.x;
    const int f = STATIC ? 0 : blockIdx.y;
    const int an = blockIdx.z;
    const int l = threadIdx.x;
    for (int i = l; i < a.T; i += RF_THREADS) tr[i] = 0.0f;
    __builtin_amdgcn_wave_barrier();

    const double pex = ((e % a.nx_el) - 0.5 * (a.nx_el - 1)) * a.pitch_x;
    const double pey = ((e / a.nx_el) - 0.5 * ((a.n_elem / a.nx_el) - 1)) * a.pitch_y;
    const float* posf = a.pos + (STATIC ? 0 : (int64_t)f * a.n_scat * 3);
    const float ckl = a.ck[l], skl = a.sk[l];
    const float kf = (float)l;
    const double ux = a.ux[an], uy = a.uy[an], uz = a.uz[an], t0s = a.t0s[an];

    for (int64_t s0 = 0; s0 < a.n_scat; s0 += 64) {
        const int64_t s = s0 + l;
        const bool valid = s < a.n_scat;
        double px = 0.0, py = 0.0, pz = 1.0;
        float am = 0.0f;
        if (valid) {
            px = posf[3 * s];
            py = posf[3 * s + 1];
            pz = posf[3 * s + 2];
            am = a.amp[s];
        }
        const double dx = px - pex, dy = py - pey;
        const double rho = sqrt(dx * dx + dy * dy + pz * pz);
        const double x = (ux * px + uy * py + uz * pz) * a.fs_c - t0s + rho * a.fs_c;
        const double lo = ceil(x - a.half), hi = floor(x + a.half);
        const float u0 = (float)(lo - x);
        float sn, cs;
        sincosf(a.theta * u0, &sn, &cs);
        rec[l] = Rec{u0, (float)((double)am * a.r_ref / rho), cs, sn};
        rnc[l] = (int)lo * 64 + (valid ? (int)(hi - lo) + 1 : 0);
        __builtin_amdgcn_wave_barrier();
        const int nrec = (int)min<int64_t>(64, a.n_scat - s0);
        for (int r = 0; r < nrec; ++r) {
            const Rec R = rec[r];
            const int nc = rnc[r];
            const int n = (nc >> 6) + l;     // arithmetic shift: n0 may be negative
            if (l < (nc & 63) && (unsigned)n < (unsigned)a.T) {
                const float u = R.u0 + kf;
                const float g = R.amp * exp2f(a.kexp * u * u) * (ckl * R.cu - skl * R.su);
                tr[n] += g;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();

    const int nf = STATIC ? a.n_frames : 1;
    for (int ff = 0; ff < nf; ++ff) {
        const int fo = STATIC ? ff : f;
        float* dst = a.rf + (((int64_t)fo * a.n_angles + an) * a.n_elem + e) * a.T;
        for (int i = l; i < a.T; i += RF_THREADS) dst[i] = a.accumulate ? dst[i] + tr[i] : tr[i];
    }
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" int rf_synth(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse, int32_t n_frames,
                        int64_t n_scat, const float* pos, int32_t pos_static, const float* amp,
                        int32_t n_samples, int32_t accumulate, float* rf, void* stream) {
    int st = check_probe_tx(probe, tx);
    if (st != FQ_OK) return st;
    FQ_REQUIRE(pulse != nullptr, "pulse must not be NULL");
    FQ_REQUIRE(pulse->n_cycles > 0 && pulse->trunc_sigmas > 0 && pulse->trunc_sigmas <= 8 && pulse->r_ref_m > 0,
               "bad pulse parameters");
    FQ_REQUIRE(n_frames >= 1 && n_samples >= 1 && n_samples <= 8192, "bad n_frames / n_samples");
    FQ_REQUIRE(n_scat >= 0, "n_scat must be >= 0");
    FQ_REQUIRE(rf != nullptr && aligned16(rf), "rf must be a 16-byte aligned device pointer");
    FQ_REQUIRE(n_scat == 0 || (pos && amp), "pos/amp must not be NULL");
    FQ_REQUIRE(n_samples <= RF_LDS_FLOATS, "n_samples too large");
    const int E = probe->nx_el * probe->ny_el;
    const int A = tx->n_angles;
    hipStream_t s = as_stream(stream);
    if (n_scat == 0) {
        return accumulate ? FQ_OK : zero_async(rf, sizeof(float) * (size_t)n_frames * A * E * n_samples, s);
    }
    TxHost th = make_tx(*probe, *tx);
    RfArgs a{};
    a.pos = pos;
    a.amp = amp;
    a.rf = rf;
    a.n_scat = n_scat;
    a.n_frames = n_frames;
    a.n_angles = A;
    a.n_elem = E;
    a.T = n_samples;
    a.nx_el = probe->nx_el;
    a.accumulate = accumulate ? 1 : 0;
    a.pitch_x = probe->pitch_x;
    a.pitch_y = probe->pitch_y;
    a.fs_c = probe->fs_hz / probe->c_mps;
    const double sig = pulse->n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * probe->fc_hz) * probe->fs_hz;
    a.half = pulse->trunc_sigmas * sig;
    FQ_REQUIRE(2.0 * a.half + 1.0 < RF_MAX_SPAN, "pulse longer than %d samples", RF_MAX_SPAN);
    a.kexp = (float)(-1.0 / (2.0 * sig * sig) / std::log(2.0));
    const double theta = 2.0 * M_PI * probe->fc_hz / probe->fs_hz;
    a.theta = (float)theta;
    for (int k = 0; k < RF_MAX_SPAN; ++k) {
        a.ck[k] = (float)std::cos(theta * k);
        a.sk[k] = (float)std::sin(theta * k);
    }
    a.r_ref = (float)pulse->r_ref_m;
    for (int i = 0; i < A; ++i) {
        a.ux[i] = th.ux[i];
        a.uy[i] = th.uy[i];
        a.uz[i] = th.uz[i];
        a.t0s[i] = th.t0[i] * probe->fs_hz;
    }
    const size_t lds = sizeof(float) * (size_t)n_samples;
    if (pos_static) {
        hipLaunchKernelGGL(rf_synth_kernel<true>, dim3(E, 1, A), dim3(RF_THREADS), lds, s, a);
    } else {
        hipLaunchKernelGGL(rf_synth_kernel<false>, dim3(E, n_frames, A), dim3(RF_THREADS), lds, s, a);
    }
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
