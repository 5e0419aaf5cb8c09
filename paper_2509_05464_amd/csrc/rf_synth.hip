// rf_synth: analytic RF of point scatterers under tilted plane-wave transmits (gfx950).
//
// One workgroup is one wavefront and owns one trace (frame, transmit, receive element)
// held in LDS, so no two waves ever touch the same LDS word and the small workgroups
// keep many waves resident.  Each lane takes a scatterer, computes its two-way delay x
// in FP64 (samples) and runs the truncated Gaussian pulse through recurrences on the
// sample grid (see the kernel).  The whole trace is written (or added) to global memory
// once at the end, and for static scatterers to every frame (Algorithm 1 reuses the
// static tissue RF for all frames).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int RF_THREADS = 64;       // one wave per workgroup, one trace per wave
constexpr int RF_LDS_FLOATS = 16384;  // per-trace budget (64 KiB)
constexpr int RF_MAX_SPAN = 64;       // longest pulse, samples

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
    float q;                // exp(-1 / s^2)
    float theta;            // 2 pi fc / fs
    float two_cos_theta;
    float r_ref;
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES], t0s[FQ_MAX_ANGLES];  // t0s = t0 * fs
};

// Lanes = scatterers variant.  Each lane runs the pulse of its own record through
// two exact recurrences on the sample grid u_k = u0 + k:
//   Gaussian  G_{k+1} = G_k R_k, R_{k+1} = R_k Q, Q = exp(-1/s^2)
//   carrier   C_{k+1} = 2 cos(theta) C_k - C_{k-1}
// (one FMA and three multiplies per sample).  In one round only lanes whose first
// samples n0 differ modulo 64 write (a 64-slot LDS claim table, last writer wins); at
// step k those lanes touch n0 + k, distinct words in distinct banks, so the
// read-add-write is race- and conflict-free.  Losing lanes keep their record for the
// next round; winners load the next scatterers (wave prefix sum over the free lanes).
template <bool STATIC>
__global__ void __launch_bounds__(RF_THREADS) rf_synth_claim_kernel(const RfArgs a) {
    extern __shared__ float tr[];  // [T]
    __shared__ int claim[64];
    const int e = blockIdx.x;
    const int f = STATIC ? 0 : blockIdx.y;
    const int an = blockIdx.z;
    const int l = threadIdx.x;
    for (int i = l; i < a.T; i += RF_THREADS) tr[i] = 0.0f;
    claim[l] = -1;
    __builtin_amdgcn_wave_barrier();

    const double pex = ((e % a.nx_el) - 0.5 * (a.nx_el - 1)) * a.pitch_x;
    const double pey = ((e / a.nx_el) - 0.5 * ((a.n_elem / a.nx_el) - 1)) * a.pitch_y;
    const float* posf = a.pos + (STATIC ? 0 : (int64_t)f * a.n_scat * 3);
    const double ux = a.ux[an], uy = a.uy[an], uz = a.uz[an], t0s = a.t0s[an];
    const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));

    bool has = false;
    int n0 = 0, cnt = 0;
    float g = 0.f, r = 0.f, c0 = 0.f, cm = 0.f;
    int64_t next = 0;
    for (int epoch = 1;; ++epoch) {
        // refill the free lanes with the next scatterers
        const uint64_t need = __ballot(!has);
        if (!has) {
            const int64_t s = next + __popcll(need & below);
            if (s < a.n_scat) {
                const double px = posf[3 * s], py = posf[3 * s + 1], pz = posf[3 * s + 2];
                const double dx = px - pex, dy = py - pey;
                const double rho = sqrt(dx * dx + dy * dy + pz * pz);
                const double x = (ux * px + uy * py + uz * pz) * a.fs_c - t0s + rho * a.fs_c;
                const double lo = ceil(x - a.half), hi = floor(x + a.half);
                const float u0 = (float)(lo - x);
                const float scale = (float)((double)a.amp[s] * a.r_ref / rho);
                n0 = (int)lo;
                cnt = (int)(hi - lo) + 1;
                g = scale * exp2f(a.kexp * u0 * u0);
                r = exp2f(a.kexp * (2.0f * u0 + 1.0f));
                c0 = cosf(a.theta * u0);
                cm = cosf(a.theta * (u0 - 1.0f));
                has = true;
            }
        }
        next += __popcll(need);
        if (!__ballot(has)) break;
        // claim: one winner per residue of n0 modulo 64
        const int slot = n0 & 63;
        const int tag = (epoch << 6) | l;
        if (has) claim[slot] = tag;
        __builtin_amdgcn_wave_barrier();
        const bool win = has && claim[slot] == tag;
        __builtin_amdgcn_wave_barrier();
        if (win) {
            for (int k = 0; k < cnt; ++k) {
                const int n = n0 + k;
                if ((unsigned)n < (unsigned)a.T) tr[n] += g * c0;
                const float cn = a.two_cos_theta * c0 - cm;
                cm = c0;
                c0 = cn;
                g *= r;
                r *= a.q;
            }
            has = false;
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
    a.two_cos_theta = (float)(2.0 * std::cos(theta));
    a.q = (float)std::exp(-1.0 / (sig * sig));
    a.r_ref = (float)pulse->r_ref_m;
    for (int i = 0; i < A; ++i) {
        a.ux[i] = th.ux[i];
        a.uy[i] = th.uy[i];
        a.uz[i] = th.uz[i];
        a.t0s[i] = th.t0[i] * probe->fs_hz;
    }
    const size_t lds = sizeof(float) * (size_t)n_samples;
    if (pos_static) {
        hipLaunchKernelGGL(rf_synth_claim_kernel<true>, dim3(E, 1, A), dim3(RF_THREADS), lds, s, a);
    } else {
        hipLaunchKernelGGL(rf_synth_claim_kernel<false>, dim3(E, n_frames, A), dim3(RF_THREADS), lds, s, a);
    }
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
