// rf_synth: analytic RF of point scatterers under tilted plane-wave transmits (gfx950).
//
// Two forms.  The direct form (this header) adds every pulse sample of every scatterer;
// it serves pulses cut below 5 sigma or narrower than ~3.3 samples.  The spreading form
// (further down) serves the others, the workloads' 2-cycle pulse among them: the pulse
// envelope is split into two Gaussians, scatterers are spread onto a half-rate complex
// trace with the narrow one, and the trace is filtered with the other.
//
// One workgroup is one wavefront and owns one trace (frame, transmit, receive element)
// held in LDS, with a zero guard band on both sides so that pulse taps falling off the
// record need no bounds test.  Each lane takes a scatterer, computes its two-way delay
// x (in samples) in FP64, and adds the truncated Gaussian pulse on the sample grid into
// the LDS trace.  The whole trace is written (or added) to global memory once at the
// end, and for static scatterers to every frame (Algorithm 1 computes the static tissue
// RF once and reuses it for all frames).
//
// Pulse samples.  With the even base sample b = 2 floor(x / 2), f = x - b in [0, 2) and
// tap j at sample b + j (u = j - f),
//   g(u) = A exp(-u^2 / (2 s^2)) cos(theta u),   theta = 2 pi fc / fs,  s in samples,
// splits as  g = F_j * e_j  with the lane-independent Gaussian factor
//   F_j = exp(-j^2 / (2 s^2))
// and  e_j = Gc rho^j cos(theta (j - f)),  Gc = A exp(-f^2/(2 s^2)),  rho = exp(f / s^2).
// e_j is the real part of a geometric sequence with ratio rho e^{i theta}, so it obeys
//   e_{j+1} = 2 rho cos(theta) e_j - rho^2 e_{j-1}        (forward)
//   e_{j-1} = (2 cos(theta) / rho) e_j - rho^-2 e_{j+1}   (backward)
// Both chains start at the centre (e_0, e_1: cosines of arguments below half a turn),
// so |rho^j| stays within exp(+-2(J+2)/s^2) and nothing over- or underflows.  A tap
// costs one multiply, one FMA and one FMA with F_j (a scalar register) into the trace.
//
// Tap window.  The pulse is kept where |u| <= half (half = truncation x s).  With
// J = floor(half) and h = half - J, taps j = -J+2 .. J are always inside, tap -J is
// inside iff f <= h, tap -J+1 iff f <= 1 + h, tap J+1 iff f >= 1 - h and tap J+2 iff
// f >= 2 - h.  The taps are added in aligned pairs of samples (b + j, b + j + 1), j
// even, with one 8-byte LDS read-add-write per pair: J + 2 pairs, so the chain of
// dependent LDS round trips per scatterer is half as long as with single samples.  J is
// a compile-time constant, so the pairs unroll into straight-line code with immediate
// LDS offsets.
//
// Lanes of one instruction must not update the same word, and lanes whose words fall in
// the same LDS bank serialise.  On gfx950 a 64-lane 8-byte LDS read is served as two
// 32-lane halves over 64 banks (32 bank pairs), an 8-byte write as four 16-lane quarters
// over 32 banks.  Each round only one lane per residue of the pair index b / 2 modulo 32
// within each half adds its taps (a 2 x 32-slot claim table in LDS, last writer wins), and
// a winner of the upper half stands down if the lower half's winner of the same residue
// has the same pair index.  The pairs of one instruction then hit distinct words, the
// reads distinct bank pairs; two winners of one quarter whose pair indices differ by 16
// (mod 32) share a bank pair on the write.  (Claims that also keep the writes apart, or
// one 4-byte plane per sample parity, cost more issue slots or LDS instructions than
// these write conflicts cost.)  (LDS float atomics would
// remove the claim but run at a small fraction of the plain access rate.)  Lanes that
// lose keep their scatterer for the next round and the others load new ones (wave prefix
// sum over the free lanes).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int RF_THREADS = 64;        // one wave per workgroup, one trace per wave
constexpr int RF_MAX_J = 31;          // floor(half) limit
// guard band (floats, even) on each side of the LDS trace: taps reach 2J + 5 samples out
__host__ __device__ constexpr int rf_pad(int J) { return 2 * J + 6; }
constexpr int RF_MAX_PAD = rf_pad(RF_MAX_J);
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
    float F[2 * RF_MAX_J + 6];   // F[J + 1 + j] = exp(-j^2 / (2 s^2)), j = -J-1 .. J+3
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES], t0s[FQ_MAX_ANGLES];  // t0s = t0 * fs
};

// State of one scatterer record held by a lane between rounds.
struct Rec {
    int nbp;          // pair index b / 2
    float e0, e1;     // e_0, e_1
    float af, bf;     // forward coefficients 2 rho cos(theta), rho^2
    float ab, bb;     // backward coefficients 2 cos(theta) / rho, rho^-2
    float m0, m1;     // inclusion of taps -J and -J+1 (0 or 1)
    float m2, m3;     // inclusion of taps J+1 and J+2 (0 or 1)
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
    const double fl = floor(0.5 * x);
    const double fd = x - 2.0 * fl;   // in [0, 2)
    r.nbp = (int)fl;
    r.m0 = fd <= a.h ? 1.0f : 0.0f;
    r.m1 = fd <= 1.0 + a.h ? 1.0f : 0.0f;
    r.m2 = fd >= 1.0 - a.h ? 1.0f : 0.0f;
    r.m3 = fd >= 2.0 - a.h ? 1.0f : 0.0f;
    const float f = (float)fd;
    const float scale = a.amp[s] * a.r_ref * __builtin_amdgcn_rcpf((float)rho);
    // exponent arguments lie in [-2/(s^2 ln 2), 2/(s^2 ln 2)], far from over/underflow:
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

// Adds the taps of one record into the trace (tr indexed by sample) as J + 2 aligned
// pairs with plain 8-byte LDS read-add-write.  Within one instruction the lanes of a
// round touch distinct pairs, but the pair a lane updates at one step can be the pair
// another lane reads at the next step, so each write must land before the next read is
// issued: a wave barrier between steps keeps the compiler from hoisting the reads, and
// the LDS executes one wave's accesses in order.
__device__ __forceinline__ void add_pair(float2* p, float lo, float hi) {
    float2 v = *p;
    v.x += lo;
    v.y += hi;
    *p = v;
    __builtin_amdgcn_wave_barrier();
}

// Inclusion mask of tap j (only the four edge taps can be outside the window).
template <int J>
__device__ __forceinline__ float tap_mask(const Rec& r, int j) {
    float m = 1.0f;
    if (j == -J) m *= r.m0;
    if (j == -J + 1) m *= r.m1;
    if (j == J + 1) m *= r.m2;
    if (j == J + 2) m *= r.m3;
    return m;
}

template <int J>
__device__ __forceinline__ void emit(const RfArgs& a, float* tr, const Rec& r) {
    float2* p = reinterpret_cast<float2*>(tr) + r.nbp;   // samples b, b + 1
    constexpr int P0 = (J & 1) ? -J - 1 : -J;              // first (even) pair start
    // backward chain: taps j = -1 .. -J (values first, added in sample order below)
    float vb[J > 0 ? J : 1];
    {
        float em = r.e1, ec = r.e0;
#pragma unroll
        for (int j = -1; j >= -J; --j) {
            const float en = fmaf(r.ab, ec, -(r.bb * em));
            em = ec;
            ec = en;
            vb[-j - 1] = a.F[J + 1 + j] * en * tap_mask<J>(r, j);
        }
    }
    // forward chain state: e_{q-2}, e_{q-1} for the pair starting at q = 2
    float em = r.e0, ec = r.e1;
#pragma unroll
    for (int q = P0; q <= J + 2; q += 2) {
        float lo, hi;
        if (q <= -2) {
            lo = q >= -J ? vb[-q - 1] : 0.0f;
            hi = vb[-q - 2];
        } else if (q == 0) {
            lo = a.F[J + 1] * r.e0 * tap_mask<J>(r, 0);
            hi = a.F[J + 2] * r.e1 * tap_mask<J>(r, 1);
        } else {
            const float e_lo = fmaf(r.af, ec, -(r.bf * em));
            lo = a.F[J + 1 + q] * e_lo * tap_mask<J>(r, q);
            hi = 0.0f;
            if (q + 1 <= J + 2) {
                const float e_hi = fmaf(r.af, e_lo, -(r.bf * ec));
                hi = a.F[J + 2 + q] * e_hi * tap_mask<J>(r, q + 1);
                em = e_lo;
                ec = e_hi;
            }
        }
        add_pair(p + q / 2, lo, hi);
    }
}

template <bool STATIC, int J>
__global__ void __launch_bounds__(RF_THREADS) rf_synth_kernel(const RfArgs a) {
    constexpr int PAD = rf_pad(J);
    extern __shared__ float sh[];  // [PAD + T + PAD]
    __shared__ int claim[64];
    __shared__ int nbw[32];   // pair index of each lower-half winner, by residue
    float* tr = sh + PAD;
    const int e = blockIdx.x;
    const int f = STATIC ? 0 : blockIdx.y;
    const int an = blockIdx.z;
    const int l = threadIdx.x;
    for (int i = l; i < a.T + 2 * PAD; i += RF_THREADS) sh[i] = 0.0f;
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
        // claim: one winner per residue of the pair index modulo 32 in each half of the wave
        const int slot = (r.nbp & 31) | (l & 32);
        const int ep = epoch & 0x1ffffff;   // a stale tag can only make a lane yield
        const int tag = (ep << 6) | l;
        if (has) claim[slot] = tag;
        __builtin_amdgcn_wave_barrier();
        bool win = has && claim[slot] == tag;
        if (win && l < 32) nbw[slot] = r.nbp;
        __builtin_amdgcn_wave_barrier();
        // same pair won in both halves: the upper half yields
        if (win && l >= 32 && (claim[slot & 31] >> 6) == ep && nbw[slot & 31] == r.nbp) win = false;
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


// ---------------------------------------------------------------- spreading form
//
// For a pulse kept to at least 5 sigma (the tail it drops is below 3.7e-6 of the peak)
// and at least ~3.3 samples wide, the trace is formed without evaluating the pulse at
// every sample.  The pulse is the real part of a carrier times a Gaussian envelope,
//   A g(n - x) = Re[ e^{i theta n} c env(n - x) ],  c = A e^{-i theta x},
// and the envelope, of variance s^2, is the convolution of two Gaussians phi and psi of
// variances alpha s^2 and (1 - alpha) s^2 (alpha ~1/3: the narrow phi needs few taps).  Each scatterer therefore adds c phi(2m - x) to a complex
// trace on every other sample (index m, sample 2m): NT taps around x / 2, with phi
// evaluated by the same split as above (a lane-independent factor F_j times a geometric
// sequence, here complex: one complex multiply by a real ratio and two FMAs per tap).
// After all scatterers, each output sample is
//   rf[n] = Re[ e^{i theta n} sum_m psi(n - 2m) B[m] ],
// psi including the factor 2 of the half-rate grid and the Gaussian normalisation.
// Errors against the pulse cut at 5 sigma: the dropped tail (< 3.7e-6 of each pulse
// peak), aliasing of the half-rate grid 2 exp(-pi^2 alpha (1 - alpha) s^2 / 2) (alpha is
// chosen on the host to keep it below 5e-6), and the cut ends of phi (taps to
// |2j - f| >= sqrt(24) sigma_phi) and psi (17 natural log units).  The claim scheme is the one of the direct form, on the half-rate index:
// one complex sample (8 bytes) per tap.
constexpr int SP_MAX_NT = 32;      // taps (even)
constexpr int SP_MAX_P = 48;       // half-width of psi, samples

struct SpArgs {
    const float* pos;
    const float* amp;
    float* rf;
    int64_t n_scat;
    int n_frames, n_angles, n_elem, T;
    int nx_el;
    int accumulate;
    int J;                  // acceptance: x in (-(J+2), T+J+1), as the direct form
    int guard;              // half-rate guard band (complex words) on each side
    int P;                  // psi half-width
    double pitch_x, pitch_y;
    double fs_c;            // fs / c
    double nu;              // fc / fs
    float kphi;             // -log2(e) / (2 sigma_phi^2)
    float r_ref;
    float F[SP_MAX_NT];     // F[j - j0] = exp(-2 j^2 / sigma_phi^2)
    float psiT[2 * SP_MAX_P + 2];   // psiT[t + P + 1], t = -P-1 .. P (psiT[0] = 0)
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES], t0s[FQ_MAX_ANGLES];
};

struct SpRec {
    int mb;            // half-rate index of tap 0
    float rr, ri;      // c scale G rho^j0: the first tap (j = j0) before its factor F_j0
    float rho;         // ratio of consecutive taps
};

template <int NT>
__device__ __forceinline__ bool make_sp(const SpArgs& a, const float* posf, int64_t s, double pex, double pey,
                                        double ux, double uy, double uz, double t0s, SpRec& r) {
    const double px = posf[3 * s], py = posf[3 * s + 1], pz = posf[3 * s + 2];
    const double dx = px - pex, dy = py - pey;
    const double rho = sqrt_nr(dx * dx + dy * dy + pz * pz);
    const double x = (ux * px + uy * py + uz * pz) * a.fs_c - t0s + rho * a.fs_c;
    if (!(x > -(double)(a.J + 2) && x < (double)(a.T + a.J + 1))) return false;   // also rejects NaN
    const double fl = floor(0.5 * x);
    r.mb = (int)fl;
    const float f = (float)(x - 2.0 * fl);   // in [0, 2)
    const float2 c = cis_cycles(-x * a.nu);   // e^{-i theta x}
    const float scale = a.amp[s] * a.r_ref * __builtin_amdgcn_rcpf((float)rho);
    // phi(2j - f) = F_j rho^j G, G = exp(-f^2 / (2 sigma_phi^2)), rho = exp(2 f / sigma_phi^2);
    // the taps run forward from j0 = 1 - NT/2, starting at G rho^j0 = exp2(kphi f (f - 4 j0));
    // the exponents stay within (4 - 8 j0) / (2 sigma_phi^2 ln 2) (~6 for the 2-cycle pulse):
    // the bare hardware exp2 is enough
    constexpr int J0 = 1 - NT / 2;
    const float g = scale * __builtin_amdgcn_exp2f(a.kphi * f * (f - 4.0f * (float)J0));
    r.rho = __builtin_amdgcn_exp2f(-4.0f * a.kphi * f);
    r.rr = g * c.x;
    r.ri = g * c.y;
    return true;
}

__device__ __forceinline__ void add_c(float2* p, float re, float im) {
    float2 v = *p;
    v.x += re;
    v.y += im;
    *p = v;
    __builtin_amdgcn_wave_barrier();
}

template <int NT>
__device__ __forceinline__ void emit_sp(const SpArgs& a, float2* tr, const SpRec& r) {
    constexpr int J0 = 1 - NT / 2;
    float2* p = tr + r.mb + J0;
    float vr = r.rr, vi = r.ri;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        if (k > 0) {
            vr *= r.rho;
            vi *= r.rho;
        }
        add_c(p + k, a.F[k] * vr, a.F[k] * vi);
    }
}

template <bool STATIC, int NT>
__global__ void __launch_bounds__(RF_THREADS) rf_spread_kernel(const SpArgs a) {
    extern __shared__ float2 shc[];   // [guard + (T+1)/2 + guard] complex
    __shared__ int claim[64];
    __shared__ int nbw[32];
    const int M = (a.T + 1) / 2 + 2 * a.guard;
    float2* tr = shc + a.guard;
    const int e = blockIdx.x;
    const int f = STATIC ? 0 : blockIdx.y;
    const int an = blockIdx.z;
    const int l = threadIdx.x;
    for (int i = l; i < M; i += RF_THREADS) shc[i] = make_float2(0.0f, 0.0f);
    claim[l] = -1;
    __syncthreads();

    const double pex = ((e % a.nx_el) - 0.5 * (a.nx_el - 1)) * a.pitch_x;
    const double pey = ((e / a.nx_el) - 0.5 * ((a.n_elem / a.nx_el) - 1)) * a.pitch_y;
    const float* posf = a.pos + (STATIC ? 0 : (int64_t)f * a.n_scat * 3);
    const double ux = a.ux[an], uy = a.uy[an], uz = a.uz[an], t0s = a.t0s[an];
    const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));

    bool has = false;
    SpRec r{};
    int64_t next = 0;
    for (int epoch = 1;; ++epoch) {
        const uint64_t need = __ballot(!has);
        if (!has) {
            const int64_t s = next + __popcll(need & below);
            if (s < a.n_scat) has = make_sp<NT>(a, posf, s, pex, pey, ux, uy, uz, t0s, r);
        }
        next += __popcll(need);
        const bool more = next < a.n_scat;
        if (!__ballot(has)) {
            if (!more) break;
            continue;
        }
        const int slot = (r.mb & 31) | (l & 32);
        const int ep = epoch & 0x1ffffff;   // a stale tag can only make a lane yield
        const int tag = (ep << 6) | l;
        if (has) claim[slot] = tag;
        __builtin_amdgcn_wave_barrier();
        bool win = has && claim[slot] == tag;
        if (win && l < 32) nbw[slot] = r.mb;
        __builtin_amdgcn_wave_barrier();
        if (win && l >= 32 && (claim[slot & 31] >> 6) == ep && nbw[slot & 31] == r.mb) win = false;
        __builtin_amdgcn_wave_barrier();
        if (win) {
            emit_sp<NT>(a, tr, r);
            has = false;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // rf[n] = Re[e^{i theta n} sum_m psi(n - 2m) B[m]], m = mlo .. mlo + P
    const int P = a.P;
    const int nf = STATIC ? a.n_frames : 1;
    for (int n = l; n < a.T; n += RF_THREADS) {
        const int mlo = (n - P + 1) >> 1;   // first m with n - 2m <= P
        const int odd = (n - P) & 1;        // n - 2 mlo = P - odd
        float br = 0.0f, bi = 0.0f;
        for (int k = 0; k <= P; ++k) {
            const float cf = odd ? a.psiT[2 * P - 2 * k] : a.psiT[2 * P + 1 - 2 * k];
            const float2 b = tr[mlo + k];
            br = fmaf(cf, b.x, br);
            bi = fmaf(cf, b.y, bi);
        }
        const float2 cs = cis_cycles((double)n * a.nu);
        const float v = cs.x * br - cs.y * bi;
        for (int ff = 0; ff < nf; ++ff) {
            const int fo = STATIC ? ff : f;
            float* dst = a.rf + (((int64_t)fo * a.n_angles + an) * a.n_elem + e) * a.T;
            dst[n] = a.accumulate ? dst[n] + v : v;
        }
    }
}

using SpFn = void (*)(const SpArgs);

template <int NT>
SpFn sp_fn(bool stat, int nt) {
    if constexpr (NT > SP_MAX_NT) {
        return nullptr;
    } else {
        if (nt == NT) return stat ? rf_spread_kernel<true, NT> : rf_spread_kernel<false, NT>;
        return sp_fn<NT + 2>(stat, nt);
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
    FQ_REQUIRE(n_samples + 2 * RF_MAX_PAD <= RF_LDS_FLOATS, "n_samples too large");
    const int E = probe->nx_el * probe->ny_el;
    const int A = tx->n_angles;
    hipStream_t s = as_stream(stream);
    if (n_scat == 0) {
        return accumulate ? FQ_OK : zero_async(rf, sizeof(float) * (size_t)n_frames * A * E * n_samples, s);
    }
    const double sig = pulse->n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * probe->fc_hz) * probe->fs_hz;
    const double half = pulse->trunc_sigmas * sig;
    const int J = (int)std::floor(half);
    TxHost th = make_tx(*probe, *tx);
    {
        // spreading form for a pulse kept to >= 5 sigma and at least 3.3 samples wide.  The
        // split sigma_phi^2 = alpha s^2, sigma_psi^2 = (1 - alpha) s^2 takes the smallest
        // alpha (fewest taps) whose half-rate aliasing, 2 exp(-pi^2 alpha (1 - alpha) s^2 / 2),
        // stays below 5e-6: alpha (1 - alpha) s^2 >= 2.614.
        const double s2 = sig * sig;
        const double q = 4.0 * 2.614 / s2;
        // (not below 1/3: a narrower phi would make psi longer than SP_MAX_P for wide pulses)
        const double alpha = q < 1.0 ? std::max(1.0 / 3.0, 0.5 * (1.0 - std::sqrt(1.0 - q))) : 0.5;
        const double aphi = alpha * s2, bpsi = s2 - aphi;
        const int nt = 2 * (int)std::ceil(0.5 * std::sqrt(24.0 * aphi));
        const int P = (int)std::ceil(std::sqrt(2.0 * bpsi * 17.0));
        if (pulse->trunc_sigmas >= 5.0 && sig >= 3.3 && q < 1.0 && nt >= 4 && nt <= SP_MAX_NT && P <= SP_MAX_P) {
            SpArgs a{};
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
            a.J = J;
            a.P = P;
            // taps reach half-rate index floor(x/2) + j, x in (-(J+2), T+J+1), j in [1 - nt/2, nt/2];
            // psi reads (n - P)/2 .. (n + P)/2 for n in [0, T)
            a.guard = std::max((J + 4) / 2 + nt / 2, (P + 1) / 2) + 2;
            a.pitch_x = probe->pitch_x;
            a.pitch_y = probe->pitch_y;
            a.fs_c = probe->fs_hz / probe->c_mps;
            a.nu = probe->fc_hz / probe->fs_hz;
            a.kphi = (float)(-1.0 / (2.0 * aphi) / std::log(2.0));
            a.r_ref = (float)pulse->r_ref_m;
            const int j0 = 1 - nt / 2;
            for (int j = j0; j < j0 + nt; ++j) a.F[j - j0] = (float)std::exp(-2.0 * (double)j * j / aphi);
            const double norm = 2.0 / std::sqrt(2.0 * M_PI * aphi * bpsi / s2);
            a.psiT[0] = 0.0f;
            for (int t = -P; t <= P; ++t) a.psiT[t + P + 1] = (float)(norm * std::exp(-(double)t * t / (2.0 * bpsi)));
            for (int i = 0; i < A; ++i) {
                a.ux[i] = th.ux[i];
                a.uy[i] = th.uy[i];
                a.uz[i] = th.uz[i];
                a.t0s[i] = th.t0[i] * probe->fs_hz;
            }
            const SpFn fn = sp_fn<4>(pos_static != 0, nt);
            FQ_REQUIRE(fn != nullptr, "no spreading kernel for %d taps", nt);
            const size_t lds = sizeof(float2) * (size_t)((n_samples + 1) / 2 + 2 * a.guard);
            hipLaunchKernelGGL(fn, dim3(E, pos_static ? 1 : n_frames, A), dim3(RF_THREADS), lds, s, a);
            FQ_LAUNCH_CHECK();
            return FQ_OK;
        }
    }
    FQ_REQUIRE(J <= RF_MAX_J, "pulse longer than %d samples", 2 * RF_MAX_J + 3);
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
    for (int j = -J - 1; j <= J + 3; ++j) a.F[J + 1 + j] = (float)std::exp(-(double)j * j / (2.0 * sig * sig));
    for (int i = 0; i < A; ++i) {
        a.ux[i] = th.ux[i];
        a.uy[i] = th.uy[i];
        a.uz[i] = th.uz[i];
        a.t0s[i] = th.t0[i] * probe->fs_hz;
    }
    const RfFn fn = rf_fn_j<0>(pos_static != 0, J);
    FQ_REQUIRE(fn != nullptr, "no kernel for a pulse half-support of %d samples", J);
    const size_t lds = sizeof(float) * (size_t)(n_samples + 2 * rf_pad(J));
    hipLaunchKernelGGL(fn, dim3(E, pos_static ? 1 : n_frames, A), dim3(RF_THREADS), lds, s, a);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
