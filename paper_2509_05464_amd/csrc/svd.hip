// svd_clutter_filter / hermitian_eig / power_doppler (gfx950).
//
// Eigendecomposition of the N_t x N_t Hermitian Gram G = S^H S in FP64, in four steps:
//  1. tridiagonalisation (one workgroup): for k = 0 .. n-2 a Householder reflector
//     H_k = I - tau_k v_k v_k^H (v_k[k+1] = 1) maps column k below the diagonal to
//     beta_k e_1 with beta_k real, and the trailing block is updated two-sided,
//     A22 <- H^H A22 H = A22 - (v w^H + w v^H),  w = tau A22 v - |tau|^2 (v^H A22 v) v / 2.
//     G = Q T Q^H with Q = H_0 H_1 ... and T real symmetric tridiagonal (d, e = beta).
//  2. implicit QL with Wilkinson shifts on T (one lane, on T scaled to unit size): the
//     eigenvalues, plus the log of every plane rotation in the order applied;
//  3. replay of the log on the identity, row by row (each lane owns a row of Z, held in
//     LDS), which gives T = Z diag(lambda) Z^T; columns are ranked by descending eigenvalue;
//  4. back-transformation of the wanted columns, V = Q Z, one wavefront per column.
// Eigenvalues are clamped at zero (round-off of a PSD matrix), and the rank is chosen
// (fixed, or the knee of the dB spectrum).
//
// The projection S_f = S - (S V_K) V_K^H and the power Doppler are fused: one thread
// per voxel reads its slow-time series twice (coalesced across voxels), first to form
// the K projections, then to subtract them and accumulate |S_f|^2.  V_K is read through
// the scalar cache (uniform across the wavefront).
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int TRI_THREADS = 1024;
constexpr int KMAX = 64;
constexpr int QL_MAX_ITER = 60;       // QL iterations per eigenvalue
constexpr int ROT_PER_N2 = 8;         // rotation log capacity, in units of n^2 (typical use ~1.2)
// The knee rule reads the dB spectrum down to -60 dB: the cutoff is marked by eye on the
// singular-value curve (Section 3.2) and power Doppler is shown over 60 dB (Sections 3.1,
// 3.3); eigen-energies further below the leading one are treated as one flat floor.
constexpr double KNEE_FLOOR = 1e-6;

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
// a * conj(b)
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// sum over the workgroup; every thread gets the total (red holds one slot per wave)
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += red[i];
    return t;
}

// ------------------------------------------------------------------ 1. tridiagonalisation
struct TriArgs {
    const double2* G;   // [n][n]
    double2* A;         // [n][n] work copy
    double2* vh;        // [n][n]: v_k in row k, entries k+1 .. n-1
    double2* tau;       // [n]
    double* d;          // [n]
    double* e;          // [n]
    int n;
};

__global__ void __launch_bounds__(TRI_THREADS) tridiag_kernel(const TriArgs a) {
    __shared__ double2 sv[FQ_MAX_NT], sy[FQ_MAX_NT];
    __shared__ double red[TRI_THREADS / 64];
    __shared__ double2 s_tau, s_scale;
    __shared__ int s_skip;
    const int n = a.n, tid = threadIdx.x;
    // Hermitian part of the input (the Gram is Hermitian up to its own rounding)
    for (int idx = tid; idx < n * n; idx += TRI_THREADS) {
        const int i = idx / n, j = idx - i * n;
        const double2 g = a.G[idx], gt = a.G[j * n + i];
        a.A[idx] = i == j ? make_double2(g.x, 0.0) : make_double2(0.5 * (g.x + gt.x), 0.5 * (g.y - gt.y));
    }
    __syncthreads();
    for (int k = 0; k < n - 1; ++k) {
        const int m = n - k - 1;            // length of the reflected part (rows k+1 .. n-1)
        double ps = 0.0;
        for (int i = k + 2 + tid; i < n; i += TRI_THREADS) {
            const double2 x = a.A[i * n + k];
            ps += x.x * x.x + x.y * x.y;
        }
        const double sigma = block_sum<TRI_THREADS>(ps, red);
        if (tid == 0) {
            const double2 alpha = a.A[(k + 1) * n + k];
            double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
            double beta = alpha.x;
            int skip = 1;
            if (sigma > 0.0 || alpha.y != 0.0) {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
                const double dd = den.x * den.x + den.y * den.y;
                scale = make_double2(den.x / dd, -den.y / dd);
                skip = 0;
            }
            a.tau[k] = tau;
            a.e[k] = beta;
            a.d[k] = a.A[k * n + k].x;
            s_tau = tau;
            s_scale = scale;
            s_skip = skip;
        }
        __syncthreads();
        const double2 tau = s_tau, scale = s_scale;
        const int skip = s_skip;
        for (int i = tid; i < m; i += TRI_THREADS) {
            const double2 v = i == 0 ? make_double2(1.0, 0.0) : zmul(a.A[(k + 1 + i) * n + k], scale);
            sv[i] = v;
            a.vh[k * n + k + 1 + i] = v;
        }
        __syncthreads();
        if (skip) continue;
        // y = A22 v, four threads per row
        for (int row = tid >> 2; row < m; row += TRI_THREADS / 4) {
            const double2* Ar = a.A + (size_t)(k + 1 + row) * n + (k + 1);
            double2 acc = make_double2(0.0, 0.0);
            for (int j = tid & 3; j < m; j += 4) {
                const double2 x = Ar[j], v = sv[j];
                acc.x += x.x * v.x - x.y * v.y;
                acc.y += x.x * v.y + x.y * v.x;
            }
            acc.x += __shfl_xor(acc.x, 1);
            acc.y += __shfl_xor(acc.y, 1);
            acc.x += __shfl_xor(acc.x, 2);
            acc.y += __shfl_xor(acc.y, 2);
            if ((tid & 3) == 0) sy[row] = acc;
        }
        __syncthreads();
        // r = v^H y (real for Hermitian A22)
        double pr = 0.0;
        for (int i = tid; i < m; i += TRI_THREADS) pr += sv[i].x * sy[i].x + sv[i].y * sy[i].y;
        const double r = block_sum<TRI_THREADS>(pr, red);
        const double hw = 0.5 * (tau.x * tau.x + tau.y * tau.y) * r;
        for (int i = tid; i < m; i += TRI_THREADS) {
            const double2 ty = zmul(tau, sy[i]);
            sy[i] = make_double2(ty.x - hw * sv[i].x, ty.y - hw * sv[i].y);
        }
        __syncthreads();
        // A22 -= v w^H + w v^H
        for (int idx = tid; idx < m * m; idx += TRI_THREADS) {
            const int i = idx / m, j = idx - i * m;
            const double2 p = zmulc(sv[i], sy[j]), q = zmulc(sy[i], sv[j]);
            double2* x = a.A + (size_t)(k + 1 + i) * n + (k + 1 + j);
            const double2 o = *x;
            *x = make_double2(o.x - p.x - q.x, o.y - p.y - q.y);
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.d[n - 1] = a.A[(n - 1) * n + (n - 1)].x;
        a.e[n - 1] = 0.0;
    }
}

// ------------------------------------------------------------------ 2. QL on T
struct QlArgs {
    const double* d;
    const double* e;
    int* rot_i;         // rotation log: plane (i, i+1), cos, sin
    double* rot_c;
    double* rot_s;
    int* rot_n;
    int cap;
    double* lam;        // [n] descending, clamped at 0
    double* sigma;      // [n] or null
    int* perm;          // [n]: column of Z holding the eigenvalue of rank j
    int* status;        // or null
    int n;
};

__global__ void __launch_bounds__(64) ql_kernel(const QlArgs a) {
    __shared__ double d[FQ_MAX_NT], e[FQ_MAX_NT];
    __shared__ double s_sc;
    const int n = a.n, l0 = threadIdx.x;
    for (int i = l0; i < n; i += 64) {
        d[i] = a.d[i];
        e[i] = a.e[i];
    }
    __syncthreads();
    if (l0 == 0) {
        // scale T to unit size (no overflow in squares, scale-free tolerances)
        double sc = 0.0;
        for (int i = 0; i < n; ++i) sc = fmax(sc, fabs(d[i]) + fabs(e[i]));
        const double isc = sc > 0.0 ? 1.0 / sc : 0.0;
        for (int i = 0; i < n; ++i) {
            d[i] *= isc;
            e[i] *= isc;
        }
        e[n - 1] = 0.0;
        s_sc = sc;
    }
    __syncthreads();
    const double eps = 2.220446049250313e-16;
    // The wave runs the iteration in lockstep: the search for the deflation point is
    // wave-parallel, each sweep of rotations runs on lane 0 (a dependent chain).
    int cnt = 0, bad = 0;
    for (int l = 0; l < n && !bad; ++l) {
        for (int it = 0;; ++it) {
            // m = the first index >= l with a negligible off-diagonal e[m], n - 1 if none
            int m = n - 1;
            for (int m0 = l; m0 < n - 1; m0 += 64) {
                const int mm = m0 + l0;
                bool small = false;
                if (mm < n - 1) small = fabs(e[mm]) <= eps * (fabs(d[mm]) + fabs(d[mm + 1]));
                const uint64_t b = __ballot(small);
                if (b) {
                    m = m0 + __ffsll((unsigned long long)b) - 1;
                    break;
                }
            }
            if (m == l) break;
            if (it >= QL_MAX_ITER || cnt + (m - l) > a.cap) {
                bad = 1;
                break;
            }
            int split = 0;
            if (l0 == 0) {
                // Wilkinson shift from the leading 2x2 block
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = sqrt(g * g + 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
                double s = 1.0, c = 1.0, p = 0.0;
                int i = m - 1;
                // d[i], d[i+1], e[i] of the current plane; the next plane's e and d are
                // read one step ahead (this step writes only e[i+1] and d[i+1])
                double ei = e[i], di = d[i], dip1 = d[i + 1];
                for (; i >= l; --i) {
                    const int inx = i > 0 ? i - 1 : 0;   // clamped: read unconditionally
                    const double e_nx = e[inx], d_nx = d[inx];
                    const double f = s * ei, b = c * ei;
                    const double x = f * f + g * g;
                    if (x == 0.0) {   // e[i] vanished: the block splits, restart
                        e[i + 1] = 0.0;
                        d[i + 1] = dip1 - p;
                        e[m] = 0.0;
                        split = 1;
                        break;
                    }
                    // 1/sqrt(x) from the hardware estimate and two Newton steps
                    double y = __builtin_amdgcn_rsq(x);
                    y = y * fma(-0.5 * x * y, y, 1.5);
                    y = y * fma(-0.5 * x * y, y, 1.5);
                    e[i + 1] = x * y;
                    s = f * y;
                    c = g * y;
                    g = dip1 - p;
                    r = (di - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    a.rot_i[cnt] = i;
                    a.rot_c[cnt] = c;
                    a.rot_s[cnt] = s;
                    ++cnt;
                    ei = e_nx;
                    dip1 = di;
                    di = d_nx;
                }
                if (!split) {
                    d[l] -= p;
                    e[l] = g;
                    e[m] = 0.0;
                }
            }
            cnt = __shfl(cnt, 0);
            __syncthreads();   // lane 0's updates of d and e before the next search
        }
    }
    if (l0 == 0) {
        const double sc = s_sc;
        for (int i = 0; i < n; ++i) d[i] *= sc;
        *a.rot_n = cnt;
        if (a.status) *a.status = bad ? FQ_E_NUMERIC : FQ_OK;
    }
    __syncthreads();
    // rank: descending, ties by index
    for (int i = l0; i < n; i += 64) {
        const double li = d[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += (d[j] > li) || (d[j] == li && j < i);
        const double lc = li > 0.0 ? li : 0.0;
        a.lam[rank] = lc;
        if (a.sigma) a.sigma[rank] = sqrt(lc);
        a.perm[rank] = i;
    }
}

// ------------------------------------------------------------------ 3. replay of the log
struct ReplayArgs {
    const int* rot_i;
    const double* rot_c;
    const double* rot_s;
    const int* rot_n;
    const int* perm;
    double* Zs;         // [n][n], columns in rank order
    int n, rows;        // rows per workgroup (= threads)
};

// Each lane owns one row of Z, stored column-major in LDS (word col * rows + lane).  The
// rotation log is staged through LDS in chunks and read two rotations ahead.  A QL sweep
// applies rotations on planes i, i-1, i-2, ...: the column shared by consecutive planes
// stays in a register, and the next plane's other column is loaded before the current
// plane's result is stored (it is a different column), so the LDS latency is off the
// dependency chain.
constexpr int RCH = 1024;   // rotations per staged chunk

__global__ void __launch_bounds__(64) replay_kernel(const ReplayArgs a) {
    extern __shared__ double zl[];
    __shared__ int ri_s[RCH + 2];   // two sentinel planes (-1) after the chunk
    __shared__ double rc_s[RCH + 2], rs_s[RCH + 2];
    const int n = a.n, R = a.rows, lane = threadIdx.x;
    const int row = blockIdx.x * R + lane;
    const bool live = lane < R && row < n;
    if (lane < R)
        for (int col = 0; col < n; ++col) zl[col * R + lane] = (col == row) ? 1.0 : 0.0;
    const int cnt = *a.rot_n;
    double* z = zl + (lane < R ? lane : 0);
    for (int base = 0; base < cnt; base += RCH) {
        const int nch = min(RCH, cnt - base);
        __syncthreads();
        for (int t = lane; t < nch + 2; t += 64) {
            const bool in = t < nch;
            ri_s[t] = in ? a.rot_i[base + t] : -1;
            rc_s[t] = in ? a.rot_c[base + t] : 1.0;
            rs_s[t] = in ? a.rot_s[base + t] : 0.0;
        }
        __syncthreads();
        if (lane >= R) continue;
        int i = ri_s[0];
        double c = rc_s[0], s = rs_s[0];
        int i1 = ri_s[1];
        double c1 = rc_s[1], s1 = rs_s[1];
        double av = z[i * R], bv = z[(i + 1) * R];
        for (int k = 0; k < nch; ++k) {
            // rotation k+2 is fetched now (sentinels past the end), k+1 is in registers
            const int i2 = ri_s[k + 2];
            const double c2 = rc_s[k + 2], s2 = rs_s[k + 2];
            const int i1c = i1 > 0 ? i1 : 0;
            const double pre = z[i1c * R];   // column i-1 when the sweep continues (untouched here)
            const double na = c * av - s * bv;
            const double nb = s * av + c * bv;
            z[(i + 1) * R] = nb;
            z[i * R] = na;
            if (i1 == i - 1) {   // same sweep: plane i-1 shares column i
                bv = na;
                av = pre;
            } else if (i1 >= 0) {   // new sweep: read both columns after the stores above
                av = z[i1 * R];
                bv = z[(i1 + 1) * R];
            }
            i = i1;
            c = c1;
            s = s1;
            i1 = i2;
            c1 = c2;
            s1 = s2;
        }
    }
    __syncthreads();
    if (live)
        for (int j = 0; j < n; ++j) a.Zs[(size_t)row * n + j] = zl[a.perm[j] * R + lane];
}

// ------------------------------------------------------------------ 4. back-transformation
struct BackArgs {
    const double* Zs;     // [n][n]
    const double2* vh;    // [n][n]
    const double2* tau;   // [n]
    double2* V;           // [n][n], columns 0 .. ncols-1 written
    int n;
};

constexpr int BT_PER_LANE = FQ_MAX_NT / 64;

__global__ void __launch_bounds__(64) back_kernel(const BackArgs a) {
    const int n = a.n, j = blockIdx.x, lane = threadIdx.x;
    double2 z[BT_PER_LANE];
#pragma unroll
    for (int t = 0; t < BT_PER_LANE; ++t) {
        const int i = lane + 64 * t;
        z[t] = make_double2(i < n ? a.Zs[(size_t)i * n + j] : 0.0, 0.0);
    }
    for (int k = n - 2; k >= 0; --k) {
        const double2 tau = a.tau[k];
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        const double2* v = a.vh + (size_t)k * n;
        double2 dot = make_double2(0.0, 0.0);   // v^H z over rows k+1 .. n-1
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) {
            const int i = lane + 64 * t;
            if (i > k && i < n) {
                const double2 vi = v[i];
                dot.x += vi.x * z[t].x + vi.y * z[t].y;
                dot.y += vi.x * z[t].y - vi.y * z[t].x;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            dot.x += __shfl_xor(dot.x, o);
            dot.y += __shfl_xor(dot.y, o);
        }
        const double2 td = zmul(tau, dot);
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) {
            const int i = lane + 64 * t;
            if (i > k && i < n) {
                const double2 u = zmul(v[i], td);
                z[t].x -= u.x;
                z[t].y -= u.y;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < BT_PER_LANE; ++t) {
        const int i = lane + 64 * t;
        if (i < n) a.V[(size_t)i * n + j] = z[t];
    }
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
        } else if (a.cutoff == FQ_CUTOFF_SSM) {
            K = *a.k_used;   // written by the spatial-similarity pass
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

// The V_K copy (vk) is zero beyond column K, so every instantiation runs all KM columns
// without a per-column test: the extra terms add exact zeros for finite data (a voxel
// with a non-finite sample has a non-finite PD either way).  Frames are unrolled by 4 so
// that several HBM loads of a voxel's series are in flight.
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
#pragma unroll 4
        for (int f = 0; f < a.nt; ++f) {
            const float2 s = a.iq[(int64_t)f * a.nv + v];
            const float2* vr = a.vk + f * KMAX;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const float2 w = vr[k];
                p[k].x = fmaf(s.x, w.x, fmaf(-s.y, w.y, p[k].x));
                p[k].y = fmaf(s.x, w.y, fmaf(s.y, w.x, p[k].y));
            }
        }
    }
    float acc = 0.f;
#pragma unroll 4
    for (int f = 0; f < a.nt; ++f) {
        float2 r = a.iq[(int64_t)f * a.nv + v];
        const float2* vr = a.vk + f * KMAX;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const float2 w = vr[k];   // subtract p_k conj(w)
            r.x -= p[k].x * w.x + p[k].y * w.y;
            r.y -= p[k].y * w.x - p[k].x * w.y;
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
    size_t off_A, off_vh, off_tau, off_d, off_e, off_ri, off_rc, off_rs, off_rn, off_perm, off_Zs;
    size_t off_lam, off_vecs, off_vk, off_k, total;
    int cap;
};

SvdWs svd_layout(int n) {
    SvdWs w{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += round_up(bytes, 256);
        return at;
    };
    const size_t nn = (size_t)n * n;
    w.cap = ROT_PER_N2 * n * n + 64;
    w.off_A = take(sizeof(double2) * nn);
    w.off_vh = take(sizeof(double2) * nn);
    w.off_tau = take(sizeof(double2) * n);
    w.off_d = take(sizeof(double) * n);
    w.off_e = take(sizeof(double) * n);
    w.off_ri = take(sizeof(int) * (size_t)w.cap);
    w.off_rc = take(sizeof(double) * (size_t)w.cap);
    w.off_rs = take(sizeof(double) * (size_t)w.cap);
    w.off_rn = take(sizeof(int));
    w.off_perm = take(sizeof(int) * n);
    w.off_Zs = take(sizeof(double) * nn);
    w.off_lam = take(sizeof(double) * n);
    w.off_vecs = take(sizeof(double2) * nn);
    w.off_vk = take(sizeof(float2) * (size_t)n * KMAX);
    w.off_k = take(sizeof(int));
    w.total = o;
    return w;
}

// Eigenvalues (descending, clamped) into lam/sigma; the leading ncols eigenvectors into
// vecs ([n][n] complex128, columns in rank order) unless vecs is null.
int launch_eig(const double* gram, int n, char* ws, const SvdWs& L, double* lam, double* sigma, double* vecs,
               int ncols, int* status, hipStream_t s) {
    double2* vh = reinterpret_cast<double2*>(ws + L.off_vh);
    double2* tau = reinterpret_cast<double2*>(ws + L.off_tau);
    double* d = reinterpret_cast<double*>(ws + L.off_d);
    double* e = reinterpret_cast<double*>(ws + L.off_e);
    int* ri = reinterpret_cast<int*>(ws + L.off_ri);
    double* rc = reinterpret_cast<double*>(ws + L.off_rc);
    double* rs = reinterpret_cast<double*>(ws + L.off_rs);
    int* rn = reinterpret_cast<int*>(ws + L.off_rn);
    int* perm = reinterpret_cast<int*>(ws + L.off_perm);
    double* Zs = reinterpret_cast<double*>(ws + L.off_Zs);

    TriArgs ta{reinterpret_cast<const double2*>(gram), reinterpret_cast<double2*>(ws + L.off_A), vh, tau, d, e, n};
    hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(TRI_THREADS), 0, s, ta);
    FQ_LAUNCH_CHECK();
    QlArgs qa{d, e, ri, rc, rs, rn, L.cap, lam, sigma, perm, status, n};
    hipLaunchKernelGGL(ql_kernel, dim3(1), dim3(64), 0, s, qa);
    FQ_LAUNCH_CHECK();
    if (!vecs || ncols < 1) return FQ_OK;
    const int rows = n <= 256 ? 64 : 32;   // LDS: rows x n doubles <= 128 KiB
    ReplayArgs pa{ri, rc, rs, rn, perm, Zs, n, rows};
    hipLaunchKernelGGL(replay_kernel, dim3((n + rows - 1) / rows), dim3(64), sizeof(double) * (size_t)rows * n, s, pa);
    FQ_LAUNCH_CHECK();
    BackArgs ba{Zs, vh, tau, reinterpret_cast<double2*>(vecs), n};
    hipLaunchKernelGGL(back_kernel, dim3(std::min(ncols, n)), dim3(64), 0, s, ba);
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
    if (n_t < 1 || n_vox < 1) return 0;
    return svd_layout(n_t).total + ssm_bytes(n_vox, n_t);
}

extern "C" int hermitian_eig(const double* gram, int32_t n_t, void* ws, size_t ws_bytes, double* lam, double* vecs,
                             int32_t* status, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(gram && ws && lam && aligned16(gram) && aligned16(ws), "null or misaligned pointer");
    const SvdWs L = svd_layout(n_t);
    if (ws_bytes < L.total) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, L.total);
        return FQ_E_WORKSPACE;
    }
    return launch_eig(gram, n_t, reinterpret_cast<char*>(ws), L, lam, nullptr, vecs, n_t, status, as_stream(stream));
}

extern "C" int svd_clutter_filter(const float* iq, int64_t n_vox, int32_t n_t, const double* gram, int32_t cutoff,
                                  void* ws, size_t ws_bytes, float* iq_filt, float* pd, double* sigma,
                                  int32_t* k_used, int32_t* status, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(cutoff >= FQ_CUTOFF_SSM && cutoff <= n_t, "cutoff must be -2 (SSM), -1 (knee) or 0..n_t");
    FQ_REQUIRE(cutoff != FQ_CUTOFF_SSM || n_t >= 2, "the SSM cutoff needs n_t >= 2");
    FQ_REQUIRE(cutoff <= KMAX, "fixed cutoff above %d is not supported", KMAX);
    FQ_REQUIRE(iq && gram && ws && sigma && k_used && aligned16(iq) && aligned16(gram) && aligned16(ws),
               "null or misaligned pointer");
    FQ_REQUIRE(!iq_filt || aligned16(iq_filt), "misaligned iq_filt");
    const SvdWs L = svd_layout(n_t);
    const size_t need = L.total + (cutoff == FQ_CUTOFF_SSM ? ssm_bytes(n_vox, n_t) : 0);
    if (ws_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
        return FQ_E_WORKSPACE;
    }
    hipStream_t s = as_stream(stream);
    char* w = reinterpret_cast<char*>(ws);
    double* lam = reinterpret_cast<double*>(w + L.off_lam);
    double* vecs = reinterpret_cast<double*>(w + L.off_vecs);
    int st = launch_eig(gram, n_t, w, L, lam, sigma, vecs, std::min(n_t, KMAX), status, s);
    if (st != FQ_OK) return st;
    if (cutoff == FQ_CUTOFF_SSM) {
        // the leading min(n_t, 64) eigenvectors are the ones back-transformed above
        st = launch_ssm(iq, n_vox, n_t, vecs, std::min(n_t, FQ_SSM_MAX_MODES), w + L.total, nullptr, k_used, s);
        if (st != FQ_OK) return st;
    }
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
