// fd_synth: frequency-domain RF synthesis of point scatterers (Appendix D, Eq. 1 and
// Eq. 2; the scatterer-block partition and frequency stepping of Algorithm 2).
//
// Per frequency sample f_j = j df (k_j = 2 pi f_j / c), with the element response
//   H_e(s, f) = sum over the v sub-elements mu of element e (the coherent sub-element
//               sum of Eq. 2; Eq. 1 sums every transmitting sub-element) of
//               (r_ref / r) e^{(i k - alpha) r} sinc(k b_x u_x) sinc(k b_y u_y),
// the field of transmit a at scatterer s and the echo at receive element m are
//   T_a(s, f) = sum_e W_e e^{i 2 pi f dtau_ae} H_e(s, f),
//   P_a(m, f) = sum_s H_m(s, f) R_s T_a(s, f),
// and the RF is  rf_a(m, t) = 2 Re sum_j w_j P_a(m, f_j) e^{-i 2 pi j t / N},
// w_j = q_j S(f_j) df with S the Fourier transform of the Gaussian pulse (q = 1/2 at
// j = 0 and j = N/2).  Three kernels per scatterer block and frame:
//   fd_tx_kernel   lane = scatterer: T for a chunk of KC consecutive frequencies and up
//                  to AG transmits; elements are visited in LDS blocks holding
//                  W_e e^{i 2 pi f dtau_ae} for the chunk;
//   fd_rx_kernel   lane = receive element: P for the chunk, scatterers staged in LDS
//                  blocks with R_s T_a(s, f); scatterer ranges split over z for
//                  occupancy, partial sums kept apart and added in a fixed order;
//   fd_idft_kernel workgroup = (element, transmit): the weighted inverse transform of the
//                  band, the complex exponential stepped in frequency and re-anchored
//                  from an exact integer phase every 64 samples.
// Within a chunk e^{i k r} is stepped from frequency to frequency by one complex
// multiplication (the frequency-stepping propagation update of Algorithm 2); each chunk
// starts from phases taken in FP64 (cycles = j df r / c) so the error does not grow with
// j.  The directivity sines (a few cycles at most) come straight from the hardware sine.  Scatterer blocks bound the transmit-field buffer by the
// workspace (the memory partition of Algorithm 2); their echoes add up in P.
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int FD_THREADS = 256;
constexpr int KC = 4;         // frequencies per chunk
constexpr int AG = 9;         // transmits per launch group
constexpr int EB = 64;        // elements per LDS block (transmit field)
constexpr int SB = 64;        // scatterers per LDS block (echo)
constexpr int FD_MAX_K = 4096;
constexpr int FD_MIN_BLOCK = 256;
constexpr double TWO_PI = 6.283185307179586;

struct FdArgs {
    const float* pos;       // [S][3] of this frame
    const float* amp;       // [S]
    const float* apod;      // [E] or null
    float2* T;              // [K][nsb][AG]
    float2* P;              // [nsplit][K][E][AG]
    const float* w;         // [K] 2 w_j
    float* rf;              // output of the inverse transform
    int64_t s0, ns, nsb;    // scatterer block [s0, s0 + ns), T row stride nsb
    int n_elem, nx_el, K, j_lo, N;
    int vx, vy;
    int na;                 // transmits in this group (<= AG)
    int nsplit, p_acc;      // echo splits; P accumulates over scatterer blocks
    double pitch_x, pitch_y, hx, hy;   // element pitch; (n-1)/2 pitch offsets
    double wx, wy;          // element size
    double df_c;            // df / c: cycles per metre per frequency step
    double bx_df_c, by_df_c;   // directivity cycles per step per unit direction cosine (b df / c)
    double alpha_df;        // attenuation nepers per metre per frequency step
    double df;
    float r_ref;
    double ux[AG], uy[AG], t0[AG];   // transmit directions and first-firing offsets (s)
    double inv_c;
    // inverse transform
    int T_len, n_frames_out, frame0, n_angles_total, a0, accumulate;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ void elem_xy(const FdArgs& a, int e, double& ex, double& ey) {
    ex = (e % a.nx_el) * a.pitch_x - a.hx;
    ey = (e / a.nx_el) * a.pitch_y - a.hy;
}

// h[q] += (1/v) sum_mu (r_ref/r) e^{(i k - alpha) r} D for f = (j0 + q) df, q < KC.
__device__ __forceinline__ void elem_resp(const FdArgs& a, double ex, double ey, double sx, double sy, double sz,
                                          int j0, const float* invj, float2* h) {
#pragma unroll
    for (int q = 0; q < KC; ++q) h[q] = make_float2(0.f, 0.f);
    for (int mx = 0; mx < a.vx; ++mx) {
        const double px = ex + ((mx + 0.5) / a.vx - 0.5) * a.wx;
        for (int my = 0; my < a.vy; ++my) {
            const double py = ey + ((my + 0.5) / a.vy - 0.5) * a.wy;
            const double dx = sx - px, dy = sy - py;
            const double r = sqrt_nr(dx * dx + dy * dy + sz * sz);
            const double cyc = a.df_c * r;                        // phase cycles per frequency step
            float2 z = cis_cycles((double)j0 * cyc);
            float2 st = cis_cycles(cyc);
            float g = a.r_ref * __builtin_amdgcn_rcpf((float)r);
            if (a.alpha_df > 0.0) {
                const float ar = (float)(a.alpha_df * r);         // nepers per frequency step
                g *= __expf(-ar * (float)j0);
                const float ast = __expf(-ar);
                st.x *= ast;
                st.y *= ast;
            }
            z.x *= g;
            z.y *= g;
            // directivity sinc(2 pi j t) = sin(2 pi j t) / (2 pi j t), t = b df u / c cycles per
            // frequency step: the sine straight from the hardware (argument reduced to a turn)
            float dxq[KC], dyq[KC];
#pragma unroll
            for (int q = 0; q < KC; ++q) dxq[q] = dyq[q] = 1.0f;
            const float rinv = (float)(1.0 / r);
            if (a.wx > 0.0) {
                const float tx = (float)(a.bx_df_c * dx) * rinv;   // directivity cycles per step
                if (tx != 0.0f) {
                    const float ix = __builtin_amdgcn_rcpf((float)TWO_PI * tx);
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        const float c = tx * (float)(j0 + q);
                        dxq[q] = invj[q] > 0.0f ? __builtin_amdgcn_sinf(c - floorf(c)) * ix * invj[q] : 1.0f;
                    }
                }
            }
            if (a.wy > 0.0) {
                const float ty = (float)(a.by_df_c * dy) * rinv;
                if (ty != 0.0f) {
                    const float iy = __builtin_amdgcn_rcpf((float)TWO_PI * ty);
#pragma unroll
                    for (int q = 0; q < KC; ++q) {
                        const float c = ty * (float)(j0 + q);
                        dyq[q] = invj[q] > 0.0f ? __builtin_amdgcn_sinf(c - floorf(c)) * iy * invj[q] : 1.0f;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < KC; ++q) {
                const float d = dxq[q] * dyq[q];
                h[q].x = fmaf(z.x, d, h[q].x);
                h[q].y = fmaf(z.y, d, h[q].y);
                z = cmul(z, st);
            }
        }
    }
}

__device__ __forceinline__ void chunk_invj(const FdArgs& a, int j0, float* invj) {
#pragma unroll
    for (int q = 0; q < KC; ++q) invj[q] = (j0 + q) > 0 ? 1.0f / (float)(j0 + q) : 0.0f;
}

// Transmit field T_a(s, f) of one chunk of frequencies; lane = scatterer.
__global__ void __launch_bounds__(FD_THREADS) fd_tx_kernel(const FdArgs a) {
    __shared__ float2 etab[EB][AG][KC];
    const int kc0 = blockIdx.y * KC;
    const int j0 = a.j_lo + kc0;
    const int nq = min(KC, a.K - kc0);
    const int64_t sl = (int64_t)blockIdx.x * FD_THREADS + threadIdx.x;
    const bool valid = sl < a.ns;
    double sx = 0.0, sy = 0.0, sz = 1.0;
    if (valid) {
        const float* p = a.pos + 3 * (a.s0 + sl);
        sx = p[0];
        sy = p[1];
        sz = p[2];
    }
    const bool live = valid && sz > 0.0;
    if (!live) sz = 1.0;
    float invj[KC];
    chunk_invj(a, j0, invj);
    float2 acc[KC][AG];
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int g = 0; g < AG; ++g) acc[q][g] = make_float2(0.f, 0.f);

    for (int e0 = 0; e0 < a.n_elem; e0 += EB) {
        __syncthreads();
        for (int i = threadIdx.x; i < EB * AG * KC; i += FD_THREADS) {
            const int el = i / (AG * KC), g = (i / KC) % AG, q = i % KC;
            const int e = e0 + el;
            float2 v = make_float2(0.f, 0.f);
            if (e < a.n_elem && g < a.na && q < nq) {
                double ex, ey;
                elem_xy(a, e, ex, ey);
                const double dtau = (a.ux[g] * ex + a.uy[g] * ey) * a.inv_c - a.t0[g];
                v = cis_cycles((double)(j0 + q) * a.df * dtau);
                const float wgt = a.apod ? a.apod[e] : 1.0f;
                v.x *= wgt;
                v.y *= wgt;
            }
            etab[el][g][q] = v;
        }
        __syncthreads();
        const int ne = min(EB, a.n_elem - e0);
        for (int el = 0; el < ne; ++el) {
            double ex, ey;
            elem_xy(a, e0 + el, ex, ey);
            float2 h[KC];
            elem_resp(a, ex, ey, sx, sy, sz, j0, invj, h);
#pragma unroll
            for (int q = 0; q < KC; ++q)
#pragma unroll
                for (int g = 0; g < AG; ++g) {
                    const float2 E = etab[el][g][q];
                    acc[q][g].x = fmaf(h[q].x, E.x, fmaf(-h[q].y, E.y, acc[q][g].x));
                    acc[q][g].y = fmaf(h[q].x, E.y, fmaf(h[q].y, E.x, acc[q][g].y));
                }
        }
    }
    if (!valid) return;
#pragma unroll
    for (int q = 0; q < KC; ++q) {
        if (q < nq) {
            float2* dst = a.T + ((int64_t)(kc0 + q) * a.nsb + sl) * AG;
#pragma unroll
            for (int g = 0; g < AG; ++g) dst[g] = live ? acc[q][g] : make_float2(0.f, 0.f);
        }
    }
}

// Echo P_a(m, f) of one chunk of frequencies and one scatterer split; lane = element.
__global__ void __launch_bounds__(FD_THREADS) fd_rx_kernel(const FdArgs a) {
    __shared__ float4 spos[SB];
    __shared__ float2 xs[SB][KC][AG];
    const int kc0 = blockIdx.y * KC;
    const int j0 = a.j_lo + kc0;
    const int nq = min(KC, a.K - kc0);
    const int m = blockIdx.x * FD_THREADS + threadIdx.x;
    const int split = blockIdx.z;
    const int64_t per = (a.ns + a.nsplit - 1) / a.nsplit;
    const int64_t sb0 = split * per;
    const int64_t sb1 = a.ns < sb0 + per ? a.ns : sb0 + per;
    double ex = 0.0, ey = 0.0;
    if (m < a.n_elem) elem_xy(a, m, ex, ey);
    float invj[KC];
    chunk_invj(a, j0, invj);
    float2 acc[KC][AG];
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int g = 0; g < AG; ++g) acc[q][g] = make_float2(0.f, 0.f);

    for (int64_t b = sb0; b < sb1; b += SB) {
        const int nb = sb1 - b < SB ? (int)(sb1 - b) : SB;
        __syncthreads();
        for (int i = threadIdx.x; i < SB; i += FD_THREADS) {
            float4 v = make_float4(0.f, 0.f, -1.f, 0.f);
            if (i < nb) {
                const float* p = a.pos + 3 * (a.s0 + b + i);
                v = make_float4(p[0], p[1], p[2], a.amp[a.s0 + b + i]);
            }
            spos[i] = v;
        }
        for (int i = threadIdx.x; i < SB * KC * AG; i += FD_THREADS) {
            const int sl = i / (KC * AG), q = (i / AG) % KC, g = i % AG;
            float2 v = make_float2(0.f, 0.f);
            if (sl < nb && q < nq) {
                v = a.T[((int64_t)(kc0 + q) * a.nsb + b + sl) * AG + g];
                const float r = a.amp[a.s0 + b + sl];
                v.x *= r;
                v.y *= r;
            }
            xs[sl][q][g] = v;
        }
        __syncthreads();
        if (m < a.n_elem) {
            for (int sl = 0; sl < nb; ++sl) {
                const float4 p = spos[sl];
                if (!(p.z > 0.0f)) continue;
                float2 h[KC];
                elem_resp(a, ex, ey, p.x, p.y, p.z, j0, invj, h);
#pragma unroll
                for (int q = 0; q < KC; ++q)
#pragma unroll
                    for (int g = 0; g < AG; ++g) {
                        const float2 X = xs[sl][q][g];
                        acc[q][g].x = fmaf(h[q].x, X.x, fmaf(-h[q].y, X.y, acc[q][g].x));
                        acc[q][g].y = fmaf(h[q].x, X.y, fmaf(h[q].y, X.x, acc[q][g].y));
                    }
            }
        }
    }
    if (m >= a.n_elem) return;
#pragma unroll
    for (int q = 0; q < KC; ++q) {
        if (q < nq) {
            float2* dst = a.P + (((int64_t)split * a.K + kc0 + q) * a.n_elem + m) * AG;
#pragma unroll
            for (int g = 0; g < AG; ++g) {
                float2 v = acc[q][g];
                if (a.p_acc) {
                    v.x += dst[g].x;
                    v.y += dst[g].y;
                }
                dst[g] = v;
            }
        }
    }
}

// Inverse transform of one (element, transmit): rf(t) = sum_j Re(Q_j e^{-i 2 pi j t / N}),
// Q_j = 2 w_j sum_split P; written to n_frames_out consecutive frames from frame0.
__global__ void __launch_bounds__(FD_THREADS) fd_idft_kernel(const FdArgs a) {
    __shared__ float2 Q[FD_MAX_K];
    const int m = blockIdx.x, g = blockIdx.y;
    for (int kk = threadIdx.x; kk < a.K; kk += FD_THREADS) {
        float2 s = make_float2(0.f, 0.f);
        for (int sp = 0; sp < a.nsplit; ++sp) {
            const float2 v = a.P[(((int64_t)sp * a.K + kk) * a.n_elem + m) * AG + g];
            s.x += v.x;
            s.y += v.y;
        }
        const float wk = a.w[kk];
        Q[kk] = make_float2(s.x * wk, s.y * wk);
    }
    __syncthreads();
    const int an = a.a0 + g;
    for (int t = threadIdx.x; t < a.T_len; t += FD_THREADS) {
        // e^{-i 2 pi j t / N}, stepped in j; exact integer phase every 64 samples
        const float2 st = cis_cycles(-(double)t / a.N);
        float acc = 0.0f;
        float2 z = make_float2(1.f, 0.f);
        for (int kk = 0; kk < a.K; ++kk) {
            if ((kk & 63) == 0) {
                const int64_t ph = ((int64_t)(a.j_lo + kk) * t) % a.N;
                z = cis_cycles(-(double)ph / a.N);
            }
            const float2 q = Q[kk];
            acc = fmaf(q.x, z.x, fmaf(-q.y, z.y, acc));
            z = cmul(z, st);
        }
        for (int f = 0; f < a.n_frames_out; ++f) {
            float* dst = a.rf + (((int64_t)(a.frame0 + f) * a.n_angles_total + an) * a.n_elem + m) * a.T_len + t;
            *dst = a.accumulate ? *dst + acc : acc;
        }
    }
}

__global__ void fd_weights_kernel(float* w, int K, int j_lo, int N, double df, double fc, double sig) {
    const int kk = blockIdx.x * blockDim.x + threadIdx.x;
    if (kk >= K) return;
    const int j = j_lo + kk;
    const double f = j * df;
    const double aa = 2.0 * 3.141592653589793 * 3.141592653589793 * sig * sig;
    const double S = sig * 2.5066282746310002 / 2.0 * (exp(-aa * (f - fc) * (f - fc)) + exp(-aa * (f + fc) * (f + fc)));
    const double q = (j == 0 || 2 * j == N) ? 0.5 : 1.0;
    w[kk] = (float)(2.0 * q * S * df);
}

struct FdPlan {
    int N, j_lo, K, nsplit;
    int64_t nsb;
    size_t off_w, off_T, off_P, bytes;
};

double spectrum(double f, double fc, double sig) {
    const double aa = 2.0 * M_PI * M_PI * sig * sig;
    return sig * std::sqrt(2.0 * M_PI) / 2.0 * (std::exp(-aa * (f - fc) * (f - fc)) + std::exp(-aa * (f + fc) * (f + fc)));
}

FdPlan plan(const fq_probe& p, const fq_pulse& pl, const fq_fd_params& fd, int n_samples, int64_t nsb) {
    FdPlan r{};
    const double sig = pl.n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * p.fc_hz);
    r.N = n_samples + 2 * (int)std::ceil(6.0 * sig * p.fs_hz);
    const double df = p.fs_hz / r.N;
    double smax = 0.0;
    for (int j = 0; j <= r.N / 2; ++j) smax = std::max(smax, spectrum(j * df, p.fc_hz, sig));
    int lo = -1, hi = -1;
    for (int j = 0; j <= r.N / 2; ++j) {
        if (spectrum(j * df, p.fc_hz, sig) >= fd.spectral_floor * smax) {
            if (lo < 0) lo = j;
            hi = j;
        }
    }
    r.j_lo = lo;
    r.K = hi - lo + 1;
    const int E = p.nx_el * p.ny_el;
    r.nsb = nsb;
    const int wg0 = ((E + FD_THREADS - 1) / FD_THREADS) * ((r.K + KC - 1) / KC);
    r.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)8, (1024 + wg0 - 1) / wg0, (nsb + SB - 1) / SB}));
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o += round_up(b, 256);
        return at;
    };
    r.off_w = take(sizeof(float) * r.K);
    r.off_T = take(sizeof(float2) * (size_t)r.K * nsb * AG);
    r.off_P = take(sizeof(float2) * (size_t)r.nsplit * r.K * E * AG);
    r.bytes = o;
    return r;
}

int check_fd(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse, const fq_fd_params* fd, int n_samples) {
    int st = check_probe_tx(probe, tx);
    if (st != FQ_OK) return st;
    FQ_REQUIRE(pulse && fd, "pulse / fd parameters must not be NULL");
    FQ_REQUIRE(pulse->n_cycles > 0 && pulse->r_ref_m > 0, "bad pulse parameters");
    FQ_REQUIRE(fd->n_sub_x >= 1 && fd->n_sub_y >= 1 && fd->n_sub_x * fd->n_sub_y <= 64, "sub-elements must be 1..64");
    FQ_REQUIRE(fd->elem_width_x >= 0 && fd->elem_width_y >= 0 && fd->elem_width_x <= probe->pitch_x * 4 &&
                   fd->elem_width_y <= probe->pitch_y * 4,
               "bad element size");
    FQ_REQUIRE(fd->atten_db_cm_mhz >= 0 && fd->atten_db_cm_mhz < 100, "bad attenuation");
    FQ_REQUIRE(fd->spectral_floor > 0 && fd->spectral_floor < 1, "spectral_floor must be in (0, 1)");
    FQ_REQUIRE(n_samples >= 1 && n_samples <= 16384, "bad n_samples");
    return FQ_OK;
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t fd_workspace_size(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse,
                                    const fq_fd_params* fd, int32_t n_samples, int64_t scatterers_per_block) {
    if (check_fd(probe, tx, pulse, fd, n_samples) != FQ_OK) return 0;
    return plan(*probe, *pulse, *fd, n_samples, std::max<int64_t>(FD_MIN_BLOCK, scatterers_per_block)).bytes;
}

extern "C" int fd_synth(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse, const fq_fd_params* fd,
                        int32_t n_frames, int64_t n_scat, const float* pos, int32_t pos_static, const float* amp,
                        const float* apod, int32_t n_samples, int32_t accumulate, void* ws, size_t ws_bytes, float* rf,
                        void* stream) {
    int st = check_fd(probe, tx, pulse, fd, n_samples);
    if (st != FQ_OK) return st;
    FQ_REQUIRE(n_frames >= 1 && n_scat >= 0, "bad n_frames / n_scat");
    FQ_REQUIRE(rf && aligned16(rf) && ws && aligned16(ws), "null or misaligned rf / ws");
    FQ_REQUIRE(n_scat == 0 || (pos && amp), "pos/amp must not be NULL");
    const int E = probe->nx_el * probe->ny_el;
    const int A = tx->n_angles;
    hipStream_t s = as_stream(stream);
    if (n_scat == 0) return accumulate ? FQ_OK : zero_async(rf, sizeof(float) * (size_t)n_frames * A * E * n_samples, s);
    // largest scatterer block whose buffers fit the workspace (memory partition)
    const int64_t want = n_scat;
    FdPlan pl = plan(*probe, *pulse, *fd, n_samples, FD_MIN_BLOCK);
    if (ws_bytes < pl.bytes) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, pl.bytes);
        return FQ_E_WORKSPACE;
    }
    int64_t lo = FD_MIN_BLOCK, hi = std::max<int64_t>(FD_MIN_BLOCK, want);
    if (plan(*probe, *pulse, *fd, n_samples, hi).bytes <= ws_bytes) {
        lo = hi;
    } else {
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (plan(*probe, *pulse, *fd, n_samples, mid).bytes <= ws_bytes) lo = mid; else hi = mid;
        }
    }
    pl = plan(*probe, *pulse, *fd, n_samples, lo);
    FQ_REQUIRE(pl.K >= 1 && pl.K <= FD_MAX_K, "frequency band of %d samples (limit %d)", pl.K, FD_MAX_K);
    char* w = reinterpret_cast<char*>(ws);
    const TxHost th = make_tx(*probe, *tx);
    const double sig = pulse->n_cycles / (2.0 * std::sqrt(2.0 * std::log(2.0)) * probe->fc_hz);
    const double df = probe->fs_hz / pl.N;

    FdArgs a{};
    a.apod = apod;
    a.T = reinterpret_cast<float2*>(w + pl.off_T);
    a.P = reinterpret_cast<float2*>(w + pl.off_P);
    a.w = reinterpret_cast<const float*>(w + pl.off_w);
    a.rf = rf;
    a.nsb = pl.nsb;
    a.n_elem = E;
    a.nx_el = probe->nx_el;
    a.K = pl.K;
    a.j_lo = pl.j_lo;
    a.N = pl.N;
    a.vx = fd->n_sub_x;
    a.vy = fd->n_sub_y;
    a.nsplit = pl.nsplit;
    a.pitch_x = probe->pitch_x;
    a.pitch_y = probe->pitch_y;
    a.hx = 0.5 * (probe->nx_el - 1) * probe->pitch_x;
    a.hy = 0.5 * (probe->ny_el - 1) * probe->pitch_y;
    a.wx = fd->elem_width_x;
    a.wy = fd->elem_width_y;
    a.df = df;
    a.df_c = df / probe->c_mps;
    a.bx_df_c = 0.5 * fd->elem_width_x / fd->n_sub_x * df / probe->c_mps;
    a.by_df_c = 0.5 * fd->elem_width_y / fd->n_sub_y * df / probe->c_mps;
    a.alpha_df = fd->atten_db_cm_mhz / (20.0 * std::log10(std::exp(1.0))) * 100.0 * df / 1e6;
    a.r_ref = (float)pulse->r_ref_m;
    a.inv_c = 1.0 / probe->c_mps;
    a.T_len = n_samples;
    a.n_angles_total = A;
    a.accumulate = accumulate ? 1 : 0;

    hipLaunchKernelGGL(fd_weights_kernel, dim3((pl.K + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<float*>(w + pl.off_w), pl.K, pl.j_lo, pl.N, df, probe->fc_hz, sig);
    FQ_LAUNCH_CHECK();
    const int nfr = pos_static ? 1 : n_frames;
    const int kchunks = (pl.K + KC - 1) / KC;
    for (int f = 0; f < nfr; ++f) {
        a.pos = pos + (pos_static ? 0 : (int64_t)f * n_scat * 3);
        a.amp = amp;
        for (int a0 = 0; a0 < A; a0 += AG) {
            a.a0 = a0;
            a.na = std::min(AG, A - a0);
            for (int g = 0; g < AG; ++g) {
                const int an = std::min(a0 + g, A - 1);
                a.ux[g] = th.ux[an];
                a.uy[g] = th.uy[an];
                a.t0[g] = th.t0[an];
            }
            for (int64_t s0 = 0; s0 < n_scat; s0 += pl.nsb) {
                a.s0 = s0;
                a.ns = std::min<int64_t>(pl.nsb, n_scat - s0);
                a.p_acc = s0 > 0 ? 1 : 0;
                hipLaunchKernelGGL(fd_tx_kernel, dim3((unsigned)((a.ns + FD_THREADS - 1) / FD_THREADS), kchunks),
                                   dim3(FD_THREADS), 0, s, a);
                FQ_LAUNCH_CHECK();
                hipLaunchKernelGGL(fd_rx_kernel, dim3((E + FD_THREADS - 1) / FD_THREADS, kchunks, pl.nsplit),
                                   dim3(FD_THREADS), 0, s, a);
                FQ_LAUNCH_CHECK();
            }
            a.frame0 = pos_static ? 0 : f;
            a.n_frames_out = pos_static ? n_frames : 1;
            hipLaunchKernelGGL(fd_idft_kernel, dim3(E, a.na), dim3(FD_THREADS), 0, s, a);
            FQ_LAUNCH_CHECK();
        }
    }
    return FQ_OK;
}
