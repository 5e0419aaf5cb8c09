// rf_synth: analytic RF of point scatterers under tilted plane-wave transmits (gfx950).
//
// One workgroup is one wavefront and owns one trace (frame, transmit, receive element)
// held in LDS, with a zero guard band on both sides so that pulse taps falling off the
// record need no bounds test.  Each lane takes a scatterer, computes its two-way delay
// x (in samples) in FP64, and adds the truncated Gaussian pulse on the sample grid into
// the LDS trace.  The whole trace is written (or added) to global memory once at the
// end, and for static scatterers to every frame (Algorithm 1 computes the static tissue
// RF once and reuses it for all frames).
//
// Pulse samples.  With nb = floor(x), f = x - nb and tap j at sample nb + j (u = j - f),
//   g(u) = A exp(-u^2 / (2 s^2)) cos(theta u),   theta = 2 pi fc / fs,  s in samples,
// splits as  g = F_j * e_j  with the lane-independent Gaussian factor
//   F_j = exp(-j^2 / (2 s^2))
// and  e_j = Gc rho^j cos(theta (j - f)),  Gc = A exp(-f^2/(2 s^2)),  rho = exp(f / s^2).
// e_j is the real part of a geometric sequence with ratio rho e^{i theta}, so it obeys
//   e_{j+1} = 2 rho cos(theta) e_j - rho^2 e_{j-1}        (forward)
//   e_{j-1} = (2 cos(theta) / rho) e_j - rho^-2 e_{j+1}   (backward)
// Both chains start at the centre (e_0, e_1: cosines of arguments below a quarter
// turn), so |rho^j| stays within exp(+-J/s^2) and nothing over- or underflows.  A tap
// costs one multiply, one FMA, one multiply by F_j (a scalar register) and one LDS
// read-add-write.
//
// Tap window.  The pulse is kept where |u| <= half (half = truncation x s).  With
// J = floor(half) and h = half - J, taps j = -J+1 .. J are always inside, tap -J is
// inside iff f <= h and tap J+1 iff f >= 1 - h; J is a compile-time constant so the
// 2J+2 taps unroll into straight-line code with immediate LDS offsets.
//
// Lanes of one instruction must not update the same word, and lanes whose words fall in
// the same LDS bank serialise.  The LDS serves a 64-lane access as two 32-lane halves
// over 32 banks, so each round only one lane per residue of nb modulo 32 within each
// half adds its taps (a 2 x 32-slot claim table in LDS, last writer wins), and a winner
// of the upper half stands down if the lower half's winner of the same residue has the
// same nb.  The taps of one instruction then hit distinct words and, per half, distinct
// banks.  (LDS float atomics would remove the claim but run at a small fraction of the
// plain access rate.)  Lanes that lose keep their scatterer for the next round and the
// others load new ones (wave prefix sum over the free lanes).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int RF_THREADS = 64;        // one wave per workgroup, one trace per wave
constexpr int RF_PAD = 64;            // guard band (floats) on each side of the LDS trace
constexpr int RF_MAX_J = 31;          // floor(half) limit: 2J+2 <= RF_PAD taps
constexpr int RF_LDS_FLOATS = 16384;  // trace + guard bands budget (64 KiB)

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
    double h;               // half - J
    float kexp2;            // -log2(e) / (2 s^2)
    float nu;               // fc / fs (carrier cycles per sample)
    float two_cos_theta;
    float r_ref;
    float F[2 * RF_MAX_J + 2];   // F[J + j] = exp(-j^2 / (2 s^2)), j = -J .. J+1
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES], t0s[FQ_MAX_ANGLES];  // t0s = t0 * fs
};

// State of one scatterer record held by a lane between rounds.
struct Rec {
    int nb;
    float e0, e1;     // e_0, e_1
    float af, bf;     // forward coefficients 2 rho cos(theta), rho^2
    float ab, bb;     // backward coefficients 2 cos(theta) / rho, rho^-2
    float mlo, mhi;   // inclusion of taps -J and J+1 (0 or 1)
};

// Delay and pulse set-up of scatterer s for element (pex, pey) and transmit an.
// Returns false when no tap of the pulse falls inside the record.
template <int J>
__device__ __forceinline__ bool make_rec(const RfArgs& a, const float* posf, int64_t s, double pex, double pey,
                                         double ux, double uy, double uz, double t0s, Rec& r) {
    const double px = posf[3 * s], py = posf[3 * s + 1], pz = posf[3 * s + 2];
    const double dx = px - pex, dy = py - pey;
    // receive distance (relative error ~1e-14, i.e. ~1e-11 samples of delay)
    const double rho = sqrt_nr(dx * dx + dy * dy + pz * pz);
    const double x = (ux * px + uy * py + uz * pz) * a.fs_c - t0s + rho * a.fs_c;
    if (!(x > -(double)(J + 2) && x < (double)(a.T + J + 1))) return false;   // also rejects NaN
    const double fl = floor(x);
    const double fd = x - fl;
    r.nb = (int)fl;
    r.mlo = fd <= a.h ? 1.0f : 0.0f;
    r.mhi = fd >= 1.0 - a.h ? 1.0f : 0.0f;
    const float f = (float)fd;
    const float scale = a.amp[s] * a.r_ref * __builtin_amdgcn_rcpf((float)rho);
    // exponent arguments lie in [-1/(2 s^2 ln 2), 1/(s^2 ln 2)], far from over/underflow:
    // the bare hardware exp2 is enough
    const float gc = scale * __builtin_amdgcn_exp2f(a.kexp2 * f * f);
    const float rh = __builtin_amdgcn_exp2f(-2.0f * a.kexp2 * f);   // rho = exp(f / s^2) >= 1
    const float rhi = __builtin_amdgcn_exp2f(2.0f * a.kexp2 * f);   // 1 / rho
    r.e0 = gc * __builtin_amdgcn_cosf(a.nu * f);                 // cos(theta f), argument in turns
    r.e1 = gc * rh * __builtin_amdgcn_cosf(a.nu * (1.0f - f));   // rho cos(theta (1 - f))
    r.af = a.two_cos_theta * rh;
    r.bf = rh * rh;
    r.ab = a.two_cos_theta * rhi;
    r.bb = rhi * rhi;
    return true;
}

// Adds the 2J+2 taps of one record into the trace (tr indexed by sample) with plain
// LDS read-add-write.  Within one instruction the lanes of a round touch distinct words
// (distinct nb), but the word a lane updates at one tap can be the word another lane
// reads at the next tap, so each tap's write must land before the next tap's read is
// issued: a wave barrier between taps keeps the compiler from hoisting the reads, and
// the LDS executes one wave's accesses in order.
__device__ __forceinline__ void add_tap(float* p, float v) {
    *p += v;
    __builtin_amdgcn_wave_barrier();
}

template <int J>
__device__ __forceinline__ void emit(const RfArgs& a, float* tr, const Rec& r) {
    float* p = tr + r.nb;
    // backward chain: j = -J .. -1 (values computed first, added in sample order below)
    float vb[J > 0 ? J : 1];
    {
        float em = r.e1, ec = r.e0;
#pragma unroll
        for (int j = -1; j >= -J; --j) {
            const float en = fmaf(r.ab, ec, -(r.bb * em));
            em = ec;
            ec = en;
            float v = a.F[J + j] * en;
            if (j == -J) v *= r.mlo;
            vb[-j - 1] = v;
        }
    }
#pragma unroll
    for (int j = -J; j <= -1; ++j) add_tap(p + j, vb[-j - 1]);
    // forward chain: j = 0 .. J+1
    add_tap(p, a.F[J] * r.e0 * (J == 0 ? r.mlo : 1.0f));
    add_tap(p + 1, a.F[J + 1] * r.e1 * (J == 0 ? r.mhi : 1.0f));
    float em = r.e0, ec = r.e1;
#pragma unroll
    for (int j = 2; j <= J + 1; ++j) {
        const float en = fmaf(r.af, ec, -(r.bf * em));
        em = ec;
        ec = en;
        float v = a.F[J + j] * en;
        if (j == J + 1) v *= r.mhi;
        add_tap(p + j, v);
    }
}

template <bool STATIC, int J>
__global__ void __launch_bounds__(RF_THREADS) rf_synth_kernel(const RfArgs a) {
    extern __shared__ float sh[];  // [RF_PAD + T + RF_PAD]
    __shared__ int claim[64];
    __shared__ int nbw[32];   // nb of each lower-half winner, by residue
    float* tr = sh + RF_PAD;
    const int e = blockIdx.x;
    const int f = STATIC ? 0 : blockIdx.y;
    const int an = blockIdx.z;
    const int l = threadIdx.x;
    for (int i = l; i < a.T + 2 * RF_PAD; i += RF_THREADS) sh[i] = 0.0f;
    claim[l] = -1;
    __syncthreads();

    const double pex = ((e % a.nx_el) - 0.5 * (a.nx_el - 1)) * a.pitch_x;
    const double pey = ((e / a.nx_el) - 0.5 * ((a.n_elem / a.nx_el) - 1)) * a.pitch_y;
    const float* posf = a.pos + (STATIC ? 0 : (int64_t)f * a.n_scat * 3);
    const double ux = a.ux[an], uy = a.uy[an], uz = a.uz[an], t0s = a.t0s[an];
    const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));

    bool has = false;
    Rec r{};
    int64_t next = 0;
    for (int epoch = 1;; ++epoch) {
        // refill the free lanes with the next scatterers
        const uint64_t need = __ballot(!has);
        if (!has) {
            const int64_t s = next + __popcll(need & below);
            if (s < a.n_scat) has = make_rec<J>(a, posf, s, pex, pey, ux, uy, uz, t0s, r);
        }
        next += __popcll(need);
        const bool more = next < a.n_scat;
        if (!__ballot(has)) {
            if (!more) break;
            continue;
        }
        // claim: one winner per residue of nb modulo 32 in each half of the wave
        const int slot = (r.nb & 31) | (l & 32);
        const int ep = epoch & 0x1ffffff;   // a stale tag can only make a lane yield
        const int tag = (ep << 6) | l;
        if (has) claim[slot] = tag;
        __builtin_amdgcn_wave_barrier();
        bool win = has && claim[slot] == tag;
        if (win && l < 32) nbw[slot] = r.nb;
        __builtin_amdgcn_wave_barrier();
        // same nb won in both halves: the upper half yields
        if (win && l >= 32 && (claim[slot & 31] >> 6) == ep && nbw[slot & 31] == r.nb) win = false;
        __builtin_amdgcn_wave_barrier();
        if (win) {
            emit<J>(a, tr, r);
            has = false;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    const int nf = STATIC ? a.n_frames : 1;
    for (int ff = 0; ff < nf; ++ff) {
        const int fo = STATIC ? ff : f;
        float* dst = a.rf + (((int64_t)fo * a.n_angles + an) * a.n_elem + e) * a.T;
        for (int i = l; i < a.T; i += RF_THREADS) dst[i] = a.accumulate ? dst[i] + tr[i] : tr[i];
    }
}

using RfFn = void (*)(const RfArgs);

template <int J>
RfFn rf_fn_j(bool stat, int j) {
    if constexpr (J > RF_MAX_J) {
        return nullptr;
    } else {
        if (j == J) return stat ? rf_synth_kernel<true, J> : rf_synth_kernel<false, J>;
        return rf_fn_j<J + 1>(stat, j);
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
    FQ_REQUIRE(n_samples + 2 * RF_PAD <= RF_LDS_FLOATS, "n_samples too large");
    const int E = probe->nx_el * probe->ny_el;
    const int A = tx->n_angles;
    hipStream_t s = as_stream(stream);
    if (n_scat == 0) {
        return accumulate ? FQ_OK : zero_async(rf, sizeof(float) * (size_t)n_frames * A * E * n_samples, s);
    }
    const double sig = pulse->n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * probe->fc_hz) * probe->fs_hz;
    const double half = pulse->trunc_sigmas * sig;
    const int J = (int)std::floor(half);
    FQ_REQUIRE(J <= RF_MAX_J, "pulse longer than %d samples", 2 * RF_MAX_J + 2);
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
    a.h = half - J;
    a.kexp2 = (float)(-1.0 / (2.0 * sig * sig) / std::log(2.0));
    a.nu = (float)(probe->fc_hz / probe->fs_hz);
    a.two_cos_theta = (float)(2.0 * std::cos(2.0 * M_PI * probe->fc_hz / probe->fs_hz));
    a.r_ref = (float)pulse->r_ref_m;
    for (int j = -J; j <= J + 1; ++j) a.F[J + j] = (float)std::exp(-(double)j * j / (2.0 * sig * sig));
    for (int i = 0; i < A; ++i) {
        a.ux[i] = th.ux[i];
        a.uy[i] = th.uy[i];
        a.uz[i] = th.uz[i];
        a.t0s[i] = th.t0[i] * probe->fs_hz;
    }
    const RfFn fn = rf_fn_j<0>(pos_static != 0, J);
    FQ_REQUIRE(fn != nullptr, "no kernel for a pulse half-support of %d samples", J);
    const size_t lds = sizeof(float) * (size_t)(n_samples + 2 * RF_PAD);
    hipLaunchKernelGGL(fn, dim3(E, pos_static ? 1 : n_frames, A), dim3(RF_THREADS), lds, s, a);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
