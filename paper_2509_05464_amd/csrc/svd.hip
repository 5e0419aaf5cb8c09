// svd_clutter_filter / hermitian_eig / power_doppler (gfx950).
//
// Eigendecomposition of the N_t x N_t Hermitian Gram in FP64 by parallel cyclic Jacobi
// in one workgroup: each round rotates N/2 disjoint index pairs (round-robin ordering),
// so the two-sided update J^H A J splits into independent 2x2 blocks and V <- V J into
// independent row pairs.  The complex rotation of a pair (p, q) with a = A_pp, d = A_qq,
// b = A_pq = |b| e^{i phi} is J = diag(1, e^{-i phi}) R(theta), which first makes the
// off-diagonal real and then annihilates it with a real Jacobi rotation
// (cot 2 theta = (d - a) / 2|b|, smaller root t = tan theta).  A pair is rotated while
// |b| > tol sqrt(a d) (relative criterion, suited to the graded spectrum of clutter).
// Eigenvalues are then ranked in descending order, clamped at zero (round-off of a PSD
// matrix), and the rank is chosen (fixed, or the knee of the dB spectrum).
//
// The projection S_f = S - (S V_K) V_K^H and the power Doppler are fused: one thread
// per voxel reads its slow-time series twice (coalesced across voxels), first to form
// the K projections, then to subtract them and accumulate |S_f|^2.  V_K is read through
// the scalar cache (uniform across the wavefront).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int EIG_THREADS = 1024;
constexpr int KMAX = 64;
// The knee rule floors the dB spectrum at -60 dB: eigenvalues of a Gram accumulated in
// FP32 or split-BF16 are exact only to ~1e-7 lambda_1, so the tail below is not used.
constexpr double KNEE_FLOOR = 1e-6;

struct EigArgs {
    const double2* G;
    double2* A;        // [m][m] work copy
    double2* V;        // [m][m]
    double* lam;       // [n] descending
    double* sigma;     // [n] or null
    double2* vecs;     // [n][n] or null
    int* status;       // or null
    int n, m, max_sweeps;
    double tol;
};

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

// slot j of the round-robin schedule in round r (m even): slot 0 fixed, others rotate
__device__ __forceinline__ int rr_slot(int j, int r, int m) { return j == 0 ? 0 : 1 + (j - 1 + r) % (m - 1); }

__global__ void __launch_bounds__(EIG_THREADS) jacobi_kernel(const EigArgs a) {
    __shared__ double rc[FQ_MAX_NT / 2 + 1], rs[FQ_MAX_NT / 2 + 1];
    __shared__ double2 re_[FQ_MAX_NT / 2 + 1];
    __shared__ int rp[FQ_MAX_NT / 2 + 1], rq[FQ_MAX_NT / 2 + 1];
    __shared__ double red[EIG_THREADS / 64];
    __shared__ int any_rot;
    const int n = a.n, m = a.m, h = m / 2, tid = threadIdx.x;

    double fro = 0.0;
    for (int idx = tid; idx < m * m; idx += EIG_THREADS) {
        const int i = idx / m, j = idx % m;
        double2 g = (i < n && j < n) ? a.G[i * n + j] : make_double2(0.0, 0.0);
        if (i == j) g.y = 0.0;
        a.A[idx] = g;
        a.V[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        fro += g.x * g.x + g.y * g.y;
    }
    for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o);
    if ((tid & 63) == 0) red[tid >> 6] = fro;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < EIG_THREADS / 64; ++w) tot += red[w];
    const double abs_tol = 1e-300 + 1e-18 * sqrt(tot);

    int sweep = 0;
    bool converged = false;
    for (; sweep < a.max_sweeps; ++sweep) {
        if (tid == 0) any_rot = 0;
        __syncthreads();
        for (int r = 0; r < m - 1; ++r) {
            if (tid < h) {
                int p = rr_slot(tid, r, m), q = rr_slot(m - 1 - tid, r, m);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double app = a.A[p * m + p].x, aqq = a.A[q * m + q].x;
                const double2 b = a.A[p * m + q];
                const double mag = sqrt(b.x * b.x + b.y * b.y);
                double c = 1.0, s = 0.0;
                double2 e = make_double2(1.0, 0.0);
                if (mag > fmax(a.tol * sqrt(fabs(app * aqq)), abs_tol)) {
                    const double tau = (aqq - app) / (2.0 * mag);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    e = make_double2(b.x / mag, -b.y / mag);   // e^{-i phi}
                    any_rot = 1;
                }
                rc[tid] = c;
                rs[tid] = s;
                re_[tid] = e;
                rp[tid] = p;
                rq[tid] = q;
            }
            __syncthreads();
            // A <- J^H A J, one 2x2 block per (row pair i, column pair j)
            for (int idx = tid; idx < h * h; idx += EIG_THREADS) {
                const int i = idx / h, j = idx % h;
                const int pi = rp[i], qi = rq[i], pj = rp[j], qj = rq[j];
                const double ci = rc[i], si = rs[i], cj = rc[j], sj = rs[j];
                const double2 ei = re_[i], ej = re_[j];
                const double2 a00 = a.A[pi * m + pj], a01 = a.A[pi * m + qj];
                const double2 a10 = a.A[qi * m + pj], a11 = a.A[qi * m + qj];
                // M = A_blk J_j,  J_j = [[c, s], [-s e, c e]]
                const double2 mse = zscale(-sj, ej), mce = zscale(cj, ej);
                const double2 m00 = zadd(zscale(cj, a00), zmul(a01, mse));
                const double2 m01 = zadd(zscale(sj, a00), zmul(a01, mce));
                const double2 m10 = zadd(zscale(cj, a10), zmul(a11, mse));
                const double2 m11 = zadd(zscale(sj, a10), zmul(a11, mce));
                // J_i^H = [[c, -s conj e], [s, c conj e]]
                const double2 ce = zconj(ei);
                const double2 nse = zscale(-si, ce), nce = zscale(ci, ce);
                double2 n00 = zadd(zscale(ci, m00), zmul(nse, m10));
                double2 n01 = zadd(zscale(ci, m01), zmul(nse, m11));
                double2 n10 = zadd(zscale(si, m00), zmul(nce, m10));
                double2 n11 = zadd(zscale(si, m01), zmul(nce, m11));
                if (i == j) {
                    n00.y = 0.0;
                    n11.y = 0.0;
                    if (si != 0.0) {
                        n01 = make_double2(0.0, 0.0);
                        n10 = make_double2(0.0, 0.0);
                    }
                }
                a.A[pi * m + pj] = n00;
                a.A[pi * m + qj] = n01;
                a.A[qi * m + pj] = n10;
                a.A[qi * m + qj] = n11;
            }
            // V <- V J
            for (int idx = tid; idx < m * h; idx += EIG_THREADS) {
                const int row = idx / h, j = idx % h;
                const double c = rc[j], s = rs[j];
                if (s == 0.0) continue;
                const double2 e = re_[j];
                const int p = rp[j], q = rq[j];
                const double2 vp = a.V[row * m + p], vq = a.V[row * m + q];
                a.V[row * m + p] = zadd(zscale(c, vp), zmul(zscale(-s, e), vq));
                a.V[row * m + q] = zadd(zscale(s, vp), zmul(zscale(c, e), vq));
            }
            __syncthreads();
        }
        __syncthreads();
        if (!any_rot) {
            converged = true;
            break;
        }
        __syncthreads();
    }

    // rank eigenvalues (descending, ties by index) and write outputs
    for (int i = tid; i < n; i += EIG_THREADS) {
        const double li = a.A[i * m + i].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double lj = a.A[j * m + j].x;
            rank += (lj > li) || (lj == li && j < i);
        }
        const double lc = li > 0.0 ? li : 0.0;
        a.lam[rank] = lc;
        if (a.sigma) a.sigma[rank] = sqrt(lc);
        if (a.vecs)
            for (int row = 0; row < n; ++row) a.vecs[row * n + rank] = a.V[row * m + i];
    }
    if (tid == 0 && a.status) *a.status = converged ? 0 : FQ_E_NUMERIC;
}

// K selection and FP32 copy of V_K (one workgroup).
struct RankArgs {
    const double* lam;
    const double2* vecs;   // [n][n]
    float2* vk;            // [n][KMAX]
    int* k_used;
    int* status;           // may be null
    int n, cutoff;
};

__global__ void rank_kernel(const RankArgs a) {
    __shared__ int Ks;
    const int n = a.n;
    if (threadIdx.x == 0) {
        int K;
        if (a.cutoff >= 0) {
            K = a.cutoff;
        } else if (n < 4 || !(a.lam[0] > 0.0)) {
            K = 1;
        } else {
            // chord rule on the dB spectrum (k is 1-based in the description)
            const double l1 = a.lam[0];
            const double d1 = 0.0;
            const double dN = 10.0 * log10(fmax(a.lam[n - 1], KNEE_FLOOR * l1) / l1);
            int best_k = 2;
            double best = -1.0 / 0.0;
            for (int k = 2; k <= n / 2; ++k) {
                const double dk = 10.0 * log10(fmax(a.lam[k - 1], KNEE_FLOOR * l1) / l1);
                const double chord = d1 + (dN - d1) * (double)(k - 1) / (double)(n - 1);
                const double gap = chord - dk;
                if (gap > best) {
                    best = gap;
                    best_k = k;
                }
            }
            K = min(max(best_k - 1, 1), n / 2 - 1);
            if (K > KMAX) {
                K = KMAX;
                if (a.status) *a.status = FQ_E_NUMERIC;
            }
        }
        Ks = K;
        *a.k_used = K;
    }
    __syncthreads();
    const int K = Ks;
    for (int idx = threadIdx.x; idx < n * KMAX; idx += blockDim.x) {
        const int f = idx / KMAX, k = idx % KMAX;
        float2 v = make_float2(0.f, 0.f);
        if (k < K) {
            const double2 d = a.vecs[f * n + k];
            v = make_float2((float)d.x, (float)d.y);
        }
        a.vk[idx] = v;
    }
}

struct PdArgs {
    const float2* iq;     // [nt][nv]
    const float2* vk;     // [nt][KMAX]
    const int* k_used;
    float2* out;          // [nt][nv] or null
    float* pd;            // [nv] or null
    int64_t nv;
    int nt;
    int k_lo;             // this instantiation serves k_lo < K <= KM (device-side dispatch)
    float inv_nt;
};

template <int KM>
__global__ void __launch_bounds__(256) project_pd_kernel(const PdArgs a) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nv) return;
    const int K = *a.k_used;
    if (K <= a.k_lo || K > KM) return;
    float2 p[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) p[k] = make_float2(0.f, 0.f);
    if (K > 0) {
        for (int f = 0; f < a.nt; ++f) {
            const float2 s = a.iq[(int64_t)f * a.nv + v];
            const float2* vr = a.vk + f * KMAX;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (k < K) {
                    const float2 w = vr[k];
                    p[k].x = fmaf(s.x, w.x, fmaf(-s.y, w.y, p[k].x));
                    p[k].y = fmaf(s.x, w.y, fmaf(s.y, w.x, p[k].y));
                }
            }
        }
    }
    float acc = 0.f;
    for (int f = 0; f < a.nt; ++f) {
        float2 r = a.iq[(int64_t)f * a.nv + v];
        const float2* vr = a.vk + f * KMAX;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            if (k < K) {
                const float2 w = vr[k];   // subtract p_k conj(w)
                r.x -= p[k].x * w.x + p[k].y * w.y;
                r.y -= p[k].y * w.x - p[k].x * w.y;
            }
        }
        if (a.out) a.out[(int64_t)f * a.nv + v] = r;
        acc = fmaf(r.x, r.x, fmaf(r.y, r.y, acc));
    }
    if (a.pd) a.pd[v] = acc * a.inv_nt;
}

__global__ void __launch_bounds__(256) pd_kernel(const float2* iq, int64_t nv, int nt, float inv_nt, float* pd) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    float acc = 0.f;
    for (int f = 0; f < nt; ++f) {
        const float2 s = iq[(int64_t)f * nv + v];
        acc = fmaf(s.x, s.x, fmaf(s.y, s.y, acc));
    }
    pd[v] = acc * inv_nt;
}

struct SvdWs {
    size_t off_A, off_V, off_lam, off_vecs, off_vk, off_k, total;
};

SvdWs svd_layout(int n) {
    const int m = n + (n & 1);
    SvdWs w{};
    size_t o = 0;
    w.off_A = o;
    o += round_up(sizeof(double2) * (size_t)m * m, 256);
    w.off_V = o;
    o += round_up(sizeof(double2) * (size_t)m * m, 256);
    w.off_lam = o;
    o += round_up(sizeof(double) * (size_t)n, 256);
    w.off_vecs = o;
    o += round_up(sizeof(double2) * (size_t)n * n, 256);
    w.off_vk = o;
    o += round_up(sizeof(float2) * (size_t)n * KMAX, 256);
    w.off_k = o;
    o += 256;
    w.total = o;
    return w;
}

int launch_eig(const double* gram, int n, char* ws, const SvdWs& L, double* lam, double* sigma, double* vecs,
               int* status, hipStream_t s) {
    EigArgs ea{};
    ea.G = reinterpret_cast<const double2*>(gram);
    ea.A = reinterpret_cast<double2*>(ws + L.off_A);
    ea.V = reinterpret_cast<double2*>(ws + L.off_V);
    ea.lam = lam;
    ea.sigma = sigma;
    ea.vecs = reinterpret_cast<double2*>(vecs);
    ea.status = status;
    ea.n = n;
    ea.m = n + (n & 1);
    ea.max_sweeps = 60;
    ea.tol = 1e-14;
    if (ea.m < 2) ea.m = 2;
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(EIG_THREADS), 0, s, ea);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

using PdFn = void (*)(const PdArgs);
PdFn pd_fn(int k) {
    if (k <= 4) return project_pd_kernel<4>;
    if (k <= 8) return project_pd_kernel<8>;
    if (k <= 16) return project_pd_kernel<16>;
    if (k <= 32) return project_pd_kernel<32>;
    return project_pd_kernel<64>;
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t svd_workspace_size(int64_t n_vox, int32_t n_t) {
    (void)n_vox;
    if (n_t < 1) return 0;
    return svd_layout(std::max(n_t, 2)).total;
}

extern "C" int hermitian_eig(const double* gram, int32_t n_t, void* ws, size_t ws_bytes, double* lam, double* vecs,
                             int32_t* status, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(gram && ws && lam && aligned16(gram) && aligned16(ws), "null or misaligned pointer");
    const SvdWs L = svd_layout(std::max(n_t, 2));
    if (ws_bytes < L.total) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, L.total);
        return FQ_E_WORKSPACE;
    }
    return launch_eig(gram, n_t, reinterpret_cast<char*>(ws), L, lam, nullptr, vecs, status, as_stream(stream));
}

extern "C" int svd_clutter_filter(const float* iq, int64_t n_vox, int32_t n_t, const double* gram, int32_t cutoff,
                                  void* ws, size_t ws_bytes, float* iq_filt, float* pd, double* sigma,
                                  int32_t* k_used, int32_t* status, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(cutoff >= -1 && cutoff <= n_t, "cutoff must be -1 (knee) or 0..n_t");
    FQ_REQUIRE(cutoff <= KMAX, "fixed cutoff above %d is not supported", KMAX);
    FQ_REQUIRE(iq && gram && ws && sigma && k_used && aligned16(iq) && aligned16(gram) && aligned16(ws),
               "null or misaligned pointer");
    FQ_REQUIRE(!iq_filt || aligned16(iq_filt), "misaligned iq_filt");
    const SvdWs L = svd_layout(std::max(n_t, 2));
    if (ws_bytes < L.total) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, L.total);
        return FQ_E_WORKSPACE;
    }
    hipStream_t s = as_stream(stream);
    char* w = reinterpret_cast<char*>(ws);
    double* lam = reinterpret_cast<double*>(w + L.off_lam);
    double* vecs = reinterpret_cast<double*>(w + L.off_vecs);
    int st = launch_eig(gram, n_t, w, L, lam, sigma, vecs, status, s);
    if (st != FQ_OK) return st;
    RankArgs ra{lam, reinterpret_cast<const double2*>(vecs), reinterpret_cast<float2*>(w + L.off_vk), k_used, status,
                n_t, cutoff};
    hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(256), 0, s, ra);
    FQ_LAUNCH_CHECK();
    if (!iq_filt && !pd) return FQ_OK;
    PdArgs pa{};
    pa.iq = reinterpret_cast<const float2*>(iq);
    pa.vk = reinterpret_cast<const float2*>(w + L.off_vk);
    pa.k_used = k_used;
    pa.out = reinterpret_cast<float2*>(iq_filt);
    pa.pd = pd;
    pa.nv = n_vox;
    pa.nt = n_t;
    pa.inv_nt = 1.0f / (float)n_t;
    const unsigned blocks = (unsigned)((n_vox + 255) / 256);
    if (cutoff >= 0) {
        pa.k_lo = -1;
        hipLaunchKernelGGL(pd_fn(cutoff), dim3(blocks), dim3(256), 0, s, pa);
        FQ_LAUNCH_CHECK();
    } else {
        // the knee's K is only known on the device: every size class is launched and
        // all but the one holding K return at once
        const int bounds[6] = {-1, 4, 8, 16, 32, 64};
        for (int c = 0; c < 5; ++c) {
            pa.k_lo = bounds[c];
            hipLaunchKernelGGL(pd_fn(bounds[c + 1]), dim3(blocks), dim3(256), 0, s, pa);
            FQ_LAUNCH_CHECK();
        }
    }
    return FQ_OK;
}

extern "C" int power_doppler(const float* iq, int64_t n_vox, int32_t n_t, float* pd, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_vox >= 1, "bad sizes");
    FQ_REQUIRE(iq && pd && aligned16(iq), "null or misaligned pointer");
    const unsigned blocks = (unsigned)((n_vox + 255) / 256);
    hipLaunchKernelGGL(pd_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), reinterpret_cast<const float2*>(iq),
                       n_vox, n_t, 1.0f / (float)n_t, pd);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
