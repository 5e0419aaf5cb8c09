// svd_clutter_filter / hermitian_eig / power_doppler (gfx950).
//
// The clutter filter needs every eigenvalue of the N_t x N_t Hermitian Gram G = S^H S
// (the singular-value curve, the knee) but only the K <= 64 leading eigenvectors (the
// tissue subspace).  Its FP64 eigensolver therefore runs:
//  1. tridiagonalisation (one workgroup): for k = 0 .. n-2 a Householder reflector
//     H_k = I - tau_k v_k v_k^H (v_k[k+1] = 1) maps column k below the diagonal to
//     beta_k e_1 with beta_k real, and the trailing block is updated two-sided,
//     A22 <- H^H A22 H = A22 - (v w^H + w v^H),  w = tau A22 v - |tau|^2 (v^H A22 v) v / 2.
//     G = Q T Q^H with Q = H_0 H_1 ... and T real symmetric tridiagonal (d, e = beta).
//  2. eigenvalues of T by multisection on Sturm counts: the number of negative pivots of
//     the LDL^T factorisation of T - x I is the number of eigenvalues below x (Sylvester's
//     law of inertia); one wavefront per eigenvalue evaluates the count at 64 points of
//     its bracket at once and keeps the sub-interval where the count passes the
//     eigenvalue's index (a 65-fold narrowing per round), on T scaled to unit size;
//  3. the rank K (fixed, or the knee of the dB spectrum);
//  4. eigenvectors of T for the K leading eigenvalues by inverse iteration: a few solves
//     of (T - lambda I) z = x with a tridiagonal LU factorisation with partial pivoting,
//     one workgroup per eigenvalue, all in parallel; the vectors of eigenvalues closer
//     than 1e-6 of ||T|| (a cluster) are then made orthogonal by Gram-Schmidt, twice;
//  5. back-transformation of the K columns, V_K = Q Z_K, one wavefront per column.
// hermitian_eig (every eigenvector) keeps the implicit QL iteration with Wilkinson shifts
// (the EISPACK tql2 recurrence, Bowdler, Martin, Reinsch & Wilkinson 1968) on T, logging
// each plane rotation, and replays the log on the identity to form all of Z.
// Eigenvalues are clamped at zero (round-off of a PSD matrix).
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
constexpr int EV_THREADS = 256;       // four eigenvalues (one per wavefront) per workgroup
constexpr int EV_ROUNDS = 16;         // multisection rounds (65-fold narrowing each)
constexpr double CLUSTER_TOL = 1e-6;  // eigenvalues of the unit-scaled T this close form a cluster
constexpr int INVIT_ITERS = 4;        // inverse-iteration solves per eigenvector
constexpr double DBL_TINY = 2.2250738585072014e-308;

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

// The two-sided update of step k is applied lazily: step k+1 reads column k+1 through
// it (for its reflector) and then makes one pass over its trailing block that applies
// the update, stores the block and forms y = A22 v for its own reflector, so every step
// reads and writes the trailing block once.  Each wavefront owns every 16th row of the
// block (coalesced across columns, CT chunks of 64 columns per row) and loads its next
// row before storing the current one.
template <int CT>
__global__ void __launch_bounds__(TRI_THREADS) tridiag_kernel(const TriArgs a) {
    __shared__ double2 pv[FQ_MAX_NT], pw[FQ_MAX_NT];   // v, w of the previous step (pending update)
    __shared__ double2 sv[FQ_MAX_NT], sy[FQ_MAX_NT];   // v of this step; y = A22 v, then w
    __shared__ double2 col[FQ_MAX_NT];                 // column k with the pending update applied
    __shared__ double red[TRI_THREADS / 64];
    __shared__ double2 s_tau, s_scale;
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = TRI_THREADS / 64;
    // Hermitian part of the input (the Gram is Hermitian up to its own rounding)
    for (int idx = tid; idx < n * n; idx += TRI_THREADS) {
        const int i = idx / n, j = idx - i * n;
        const double2 g = a.G[idx], gt = a.G[j * n + i];
        a.A[idx] = i == j ? make_double2(g.x, 0.0) : make_double2(0.5 * (g.x + gt.x), 0.5 * (g.y - gt.y));
    }
    for (int i = tid; i < n; i += TRI_THREADS) {
        pv[i] = make_double2(0.0, 0.0);
        pw[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < n - 1; ++k) {
        // column k (rows k .. n-1) with the previous step's update, read as the conjugate
        // of row k (contiguous; A is kept Hermitian)
        double ps = 0.0;
        for (int i = k + tid; i < n; i += TRI_THREADS) {
            const double2 x0 = zconj(a.A[(size_t)k * n + i]);
            const double2 p = zmulc(pv[i], pw[k]), q = zmulc(pw[i], pv[k]);
            const double2 x = make_double2(x0.x - p.x - q.x, x0.y - p.y - q.y);
            col[i] = x;
            if (i >= k + 2) ps += x.x * x.x + x.y * x.y;
        }
        const double sigma = block_sum<TRI_THREADS>(ps, red);
        if (tid == 0) {
            const double2 alpha = col[k + 1];
            double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
            double beta = alpha.x;
            if (sigma > 0.0 || alpha.y != 0.0) {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                const double ib = 1.0 / beta;
                tau = make_double2((beta - alpha.x) * ib, -alpha.y * ib);
                const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
                const double idd = 1.0 / (den.x * den.x + den.y * den.y);
                scale = make_double2(den.x * idd, -den.y * idd);
            }
            a.tau[k] = tau;
            a.e[k] = beta;
            a.d[k] = col[k].x;
            s_tau = tau;
            s_scale = scale;
        }
        __syncthreads();
        const double2 tau = s_tau, scale = s_scale;
        for (int i = k + 1 + tid; i < n; i += TRI_THREADS) {
            const double2 v = i == k + 1 ? make_double2(1.0, 0.0) : zmul(col[i], scale);
            sv[i] = v;
            a.vh[(size_t)k * n + i] = v;
        }
        __syncthreads();
        // trailing block: apply the pending update, store, and y = A22 v; the wave's next
        // row is loaded before the current one is stored (no store-to-load wait in the chain)
        {
            double2 cur[CT], nxt[CT];
            int i = k + 1 + wv;
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int j = k + 1 + lane + 64 * t;
                cur[t] = i < n && j < n ? a.A[(size_t)i * n + j] : make_double2(0.0, 0.0);
            }
            for (; i < n; i += NW) {
                const int in = i + NW;
#pragma unroll
                for (int t = 0; t < CT; ++t) {
                    const int j = k + 1 + lane + 64 * t;
                    nxt[t] = in < n && j < n ? a.A[(size_t)in * n + j] : make_double2(0.0, 0.0);
                }
                double2* Ar = a.A + (size_t)i * n;
                const double2 pvi = pv[i], pwi = pw[i];
                double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                for (int t = 0; t < CT; ++t) {
                    const int j = k + 1 + lane + 64 * t;
                    if (j < n) {
                        const double2 x0 = cur[t];
                        const double2 p = zmulc(pvi, pw[j]), q = zmulc(pwi, pv[j]);
                        const double2 x = make_double2(x0.x - p.x - q.x, x0.y - p.y - q.y);
                        Ar[j] = x;
                        const double2 v = sv[j];
                        acc.x += x.x * v.x - x.y * v.y;
                        acc.y += x.x * v.y + x.y * v.x;
                    }
                    cur[t] = nxt[t];
                }
                for (int o = 32; o > 0; o >>= 1) {
                    acc.x += __shfl_xor(acc.x, o);
                    acc.y += __shfl_xor(acc.y, o);
                }
                if (lane == 0) sy[i] = acc;
            }
        }
        __syncthreads();
        // r = v^H y (real for Hermitian A22); w = tau y - |tau|^2 r v / 2 becomes the pending update
        double pr = 0.0;
        for (int i = k + 1 + tid; i < n; i += TRI_THREADS) pr += sv[i].x * sy[i].x + sv[i].y * sy[i].y;
        const double r = block_sum<TRI_THREADS>(pr, red);
        const double hw = 0.5 * (tau.x * tau.x + tau.y * tau.y) * r;
        for (int i = k + 1 + tid; i < n; i += TRI_THREADS) {
            const double2 ty = zmul(tau, sy[i]);
            pv[i] = sv[i];
            pw[i] = make_double2(ty.x - hw * sv[i].x, ty.y - hw * sv[i].y);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int m = n - 1;
        const double2 x0 = a.A[(size_t)m * n + m];
        const double2 p = zmulc(pv[m], pw[m]);
        a.d[m] = x0.x - 2.0 * p.x;
        a.e[m] = 0.0;
    }
}

// Register-resident form for n <= RT_N: the lower block triangle of A (the Hermitian
// matrix) is held in the registers of one workgroup for the whole reduction, so a step
// reads and writes no global memory.  It is cut into 16x16 blocks (I >= J; the diagonal
// blocks are held whole, both triangles), listed by block column J descending and I
// ascending and dealt to the 8 wavefronts in turn (a wavefront keeps blocks across the
// whole matrix, so the shrinking trailing block stays spread over all of them); in a
// block, lane l holds rows 4(l/16) .. 4(l/16)+3 of column l%16.  Step k:
//   1. the owners of column k put A[k..n-1][k] in LDS;
//   2. one wavefront forms the reflector (same formulas as the kernel above);
//   3. p = A22 v: each stored A_ij adds A_ij v_j to p_i and, in the blocks below the
//      diagonal, conj(A_ij) v_i to p_j: row sums are reduced over the block's 16 columns by
//      a halving butterfly (each exchange halves the values a lane carries), column sums
//      over its 4 row groups, both added into p with LDS atomics (each contribution rounded
//      to a grid on which the FP64 sums are exact: the reduction is deterministic);
//   4. every wavefront forms r = v^H p itself, and w = tau p - |tau|^2 r v / 2 on the fly;
//   5. A22 -= v w^H + w v^H on every stored element, with w_j taken as 0 in the columns
//      j <= k already reduced (v_j = 0 there too, so they are left as they are).
// Rows and columns past n start at zero and stay zero without a test: v is zero there, so
// their p and w are zero and the update adds nothing.
// v and p alternate between two buffers by step parity, so a step's writes never meet
// the previous step's reads (three barriers per step).
constexpr int RT_N = 208;                  // 13 block rows: 91 blocks, at most 12 per wavefront
constexpr int RT_THREADS = 512;            // 8 wavefronts, 2 per SIMD: 256 registers each
constexpr int RT_WAVES = RT_THREADS / 64;
constexpr int RT_BPW = 12;                 // blocks per wavefront
constexpr int RT_REG = 8;                  // of them in registers; the rest in LDS (lane-private)

__device__ __forceinline__ void rt_block(int b, int nbr, int& I, int& J) {
    I = J = -1;
    for (int jj = nbr - 1; jj >= 0; --jj) {
        const int cnt = nbr - jj;
        if (b < cnt) {
            J = jj;
            I = jj + b;
            return;
        }
        b -= cnt;
    }
}

// Lane exchanges inside a row of 16 lanes on the VALU (DPP), for FP64 values:
// row_ror:n gives lane x the value of lane (x - n) mod 16 of its row; quad_perm swaps.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_XOR1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int DPP_ROR4 = 0x124, DPP_ROR8 = 0x128, DPP_ROR12 = 0x12C;

// value of lane l (l uniform), the same in every lane
__device__ __forceinline__ double lane_f64(double x, int l) {
    const long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// x + x(lane ^ 16) and x + x(lane ^ 32), the same value in both lanes of each pair: the
// gfx950 row swaps (permlane16_swap of x with itself gives the even rows' values in the first
// result and the odd rows' in the second, permlane32_swap the lower and upper halves')
template <bool HALVES>
__device__ __forceinline__ double swap_sum(double x) {
    const long long u = __double_as_longlong(x);
    const int lo = (int)u, hi = (int)(u >> 32);
    auto l = HALVES ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false) : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto h = HALVES ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false) : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double a = __longlong_as_double(((long long)h[0] << 32) | (unsigned int)l[0]);
    const double b = __longlong_as_double(((long long)h[1] << 32) | (unsigned int)l[1]);
    return a + b;
}
// sum over a full wavefront, the same value in every lane: each row of 16 lanes summed by
// DPP (quad swaps, then rotations by 4 and 8), the four row totals read out in a fixed order
__device__ __forceinline__ double wave_total(double x) {
    x += dpp_f64<DPP_XOR1>(x);
    x += dpp_f64<DPP_XOR2>(x);
    x += dpp_f64<DPP_ROR4>(x);
    x += dpp_f64<DPP_ROR8>(x);
    return (lane_f64(x, 0) + lane_f64(x, 16)) + (lane_f64(x, 32) + lane_f64(x, 48));
}

// p = A22 v is summed in LDS by FP64 atomics from the blocks of every wavefront in the order
// they arrive.  Each contribution is first rounded to a multiple of delta = 1/scale: the
// contributions to p_i are the block pieces of one row of the Hermitian trailing matrix times v,
// so by Cauchy-Schwarz every partial sum of them is at most ||A_i|| ||v|| <= sqrt(2) ||A||_F
// (||v||^2 <= 2; the trailing block keeps ||A||_F), below 2^53 delta for the scale chosen; every
// FP64 addition is then exact and the sums do not depend on the order, so the reduction is
// deterministic.  delta <= 2^-51 ||A||_F, a few units in the last place of the products' sums.
__device__ __forceinline__ double quantize(double x, double scale, double inv_scale) {
    return rint(x * scale) * inv_scale;
}

// step 3 on one block (rows i0 .. i0+3 of column j in this lane); a diagonal block holds
// both triangles and adds its row sums only
template <bool DIAG>
__device__ __forceinline__ void rt_matvec(const double2 (&x)[4], int i0, int j, int n, int c, int lane,
                                          const double2* v, double2* p, double scale, double inv_scale) {
    const double2 vj = v[j];
    double d[8];
    double2 cs = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double2 r = zmul(x[q], vj);
        d[2 * q] = r.x;
        d[2 * q + 1] = r.y;
        if (!DIAG) {
            const double2 t = zmul(zconj(x[q]), v[i0 + q]);
            cs.x += t.x;
            cs.y += t.y;
        }
    }
    // row sums over the 16 lanes of this row group: halving butterfly on c, partners c ^ 8,
    // c ^ 4, c ^ 2, c ^ 1 (the row's lanes, exchanged by DPP: c ^ 8 is a rotation by 8, c ^ 4
    // a rotation by 4 for the lanes with bit 2 set and by 12 for the others)
    const bool b3 = c & 8, b2 = c & 4, b1 = c & 2;
    double e4[4], e2[2];
#pragma unroll
    for (int m = 0; m < 4; ++m) e4[m] = (b3 ? d[4 + m] : d[m]) + dpp_f64<DPP_ROR8>(b3 ? d[m] : d[4 + m]);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double snd = b2 ? e4[m] : e4[2 + m];
        const double a4 = dpp_f64<DPP_ROR4>(snd), a12 = dpp_f64<DPP_ROR12>(snd);
        e2[m] = (b2 ? e4[2 + m] : e4[m]) + (b2 ? a4 : a12);
    }
    double e1 = (b1 ? e2[1] : e2[0]) + dpp_f64<DPP_XOR2>(b1 ? e2[0] : e2[1]);
    e1 += dpp_f64<DPP_XOR1>(e1);
    if ((c & 1) == 0) {   // value 4 b3 + 2 b2 + b1: row q = 2 b3 + b2, part b1
        const int idx = (b3 ? 4 : 0) + (b2 ? 2 : 0) + (b1 ? 1 : 0);
        atomicAdd(reinterpret_cast<double*>(p + i0 + (idx >> 1)) + (idx & 1), quantize(e1, scale, inv_scale));
    }
    if (DIAG) return;
    // column sums over the block's 4 row groups
    cs.x = swap_sum<true>(swap_sum<false>(cs.x));
    cs.y = swap_sum<true>(swap_sum<false>(cs.y));
    if (lane < 16 && j < n) {
        atomicAdd(&p[j].x, quantize(cs.x, scale, inv_scale));
        atomicAdd(&p[j].y, quantize(cs.y, scale, inv_scale));
    }
}

// step 5 on one block: A -= v w^H + w v^H, w = tau p - hw v, for this lane's stored elements
// (w_j = 0 in a column j <= k: p_j there holds partial sums of reduced columns, not A22 v)
__device__ __forceinline__ void rt_update(double2 (&x)[4], int i0, int j, int k, const double2* v, const double2* p,
                                          double2 tau, double hw) {
    const double2 vj = v[j], tpj = zmul(tau, p[j]);
    const bool live = j > k;
    const double2 wj = make_double2(live ? tpj.x - hw * vj.x : 0.0, live ? tpj.y - hw * vj.y : 0.0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double2 vi = v[i0 + q], tpi = zmul(tau, p[i0 + q]);
        const double2 wi = make_double2(tpi.x - hw * vi.x, tpi.y - hw * vi.y);
        const double2 u1 = zmulc(vi, wj), u2 = zmulc(wi, vj);
        x[q].x -= u1.x + u2.x;
        x[q].y -= u1.y + u2.y;
    }
}

__global__ void __launch_bounds__(RT_THREADS) tridiag_reg_kernel(const TriArgs a) {
    __shared__ double2 col[RT_N];
    __shared__ double2 sv[2][RT_N], sp[2][RT_N];
    __shared__ double2 s_tau;
    __shared__ double fro2_w[RT_WAVES];
    // blocks RT_REG .. RT_BPW-1 of each wavefront: [wave][block][q][lane]
    __shared__ double2 AL[RT_WAVES * (RT_BPW - RT_REG) * 4 * 64];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: block bookkeeping in scalars
    const int nbr = (n + 15) / 16;
    const int c = lane & 15, rb = (lane >> 4) * 4;
    for (int i = tid; i < RT_N; i += RT_THREADS) {
        col[i] = sv[0][i] = sv[1][i] = sp[0][i] = sp[1][i] = make_double2(0.0, 0.0);
    }
    auto lds_blk = [&](int s, int q) -> double2& { return AL[((wv * (RT_BPW - RT_REG) + s - RT_REG) * 4 + q) * 64 + lane]; };
    int bI[RT_BPW], bJ[RT_BPW];
    double2 A[RT_REG][4];
    double fro2 = 0.0;   // this lane's part of ||A||_F^2
#pragma unroll
    for (int s = 0; s < RT_BPW; ++s) {
        rt_block(wv + RT_WAVES * s, nbr, bI[s], bJ[s]);
        const int j = 16 * bJ[s] + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 16 * bI[s] + rb + q;
            double2 x = make_double2(0.0, 0.0);
            if (bI[s] >= 0 && i < n && j < n) {
                // Hermitian part of the input (the Gram is Hermitian up to its own rounding)
                const double2 g = a.G[(size_t)i * n + j], gt = a.G[(size_t)j * n + i];
                x = i == j ? make_double2(g.x, 0.0) : make_double2(0.5 * (g.x + gt.x), 0.5 * (g.y - gt.y));
                fro2 += (bI[s] == bJ[s] ? 1.0 : 2.0) * (x.x * x.x + x.y * x.y);
            }
            if (s < RT_REG) A[s][q] = x;
            else lds_blk(s, q) = x;
        }
    }
    fro2 = wave_total(fro2);
    if (lane == 0) fro2_w[wv] = fro2;
    __syncthreads();
    // scale 2^(51 - e) with ||A||_F < 2^(e+1): partial sums of p_i below sqrt(2) 2^(e+1) + 13 delta
    // < 2^52.6 delta
    double fro = 0.0;
#pragma unroll
    for (int w = 0; w < RT_WAVES; ++w) fro += fro2_w[w];
    fro = sqrt(fro);
    const int fe = __builtin_amdgcn_readfirstlane(fro > 0.0 ? max(ilogb(fro), -900) : 0);
    const double scale = ldexp(1.0, 51 - fe), inv_scale = ldexp(1.0, fe - 51);
    for (int k = 0; k < n - 1; ++k) {
        double2* v = sv[k & 1];
        double2* p = sp[k & 1];
        // 1. column k, rows k .. n-1; clear p
        const int kb = k >> 4, kc = k & 15;
#pragma unroll
        for (int s = 0; s < RT_BPW; ++s) {
            if (bJ[s] == kb && c == kc) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 16 * bI[s] + rb + q;
                    if (i >= k && i < n) col[i] = s < RT_REG ? A[s < RT_REG ? s : 0][q] : lds_blk(s, q);
                }
            }
        }
        for (int i = tid; i < n; i += RT_THREADS) p[i] = make_double2(0.0, 0.0);
        __syncthreads();
        // 2. the reflector of column k
        if (wv == 0) {
            double ps = 0.0;
            for (int i = k + 2 + lane; i < n; i += 64) ps += col[i].x * col[i].x + col[i].y * col[i].y;
            const double sigma = wave_total(ps);
            const double2 alpha = col[k + 1];
            double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
            double beta = alpha.x;
            if (sigma > 0.0 || alpha.y != 0.0) {
                const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sigma);
                beta = alpha.x >= 0.0 ? -nrm : nrm;
                const double ib = 1.0 / beta;
                tau = make_double2((beta - alpha.x) * ib, -alpha.y * ib);
                const double2 den = make_double2(alpha.x - beta, alpha.y);   // 1 / (alpha - beta)
                const double idd = 1.0 / (den.x * den.x + den.y * den.y);
                scale = make_double2(den.x * idd, -den.y * idd);
            }
            if (lane == 0) {
                a.tau[k] = tau;
                a.e[k] = beta;
                a.d[k] = col[k].x;
                s_tau = tau;
            }
            for (int i = lane; i < n; i += 64) {
                double2 vi = make_double2(0.0, 0.0);
                if (i == k + 1) vi = make_double2(1.0, 0.0);
                else if (i > k + 1) vi = zmul(col[i], scale);
                v[i] = vi;
                if (i > k) a.vh[(size_t)k * n + i] = vi;
            }
        }
        __syncthreads();
        const double2 tau = s_tau;
        // 3. p = A22 v (blocks with a column beyond k)
#pragma unroll
        for (int s = 0; s < RT_BPW; ++s) {
            if (bI[s] < 0 || 16 * bJ[s] + 15 <= k) continue;
            const int j = 16 * bJ[s] + c, i0 = 16 * bI[s] + rb;
            if (s < RT_REG) {
                if (bI[s] == bJ[s]) rt_matvec<true>(A[s < RT_REG ? s : 0], i0, j, n, c, lane, v, p, scale, inv_scale);
                else rt_matvec<false>(A[s < RT_REG ? s : 0], i0, j, n, c, lane, v, p, scale, inv_scale);
            } else {
                double2 x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = lds_blk(s, q);
                if (bI[s] == bJ[s]) rt_matvec<true>(x, i0, j, n, c, lane, v, p, scale, inv_scale);
                else rt_matvec<false>(x, i0, j, n, c, lane, v, p, scale, inv_scale);
            }
        }
        __syncthreads();
        // 4. r = v^H p (real), in every wavefront
        double pr = 0.0;
        for (int i = k + 1 + lane; i < n; i += 64) pr += v[i].x * p[i].x + v[i].y * p[i].y;
        pr = wave_total(pr);
        const double hw = 0.5 * (tau.x * tau.x + tau.y * tau.y) * pr;
        // 5. the rank-2 update on columns beyond k
#pragma unroll
        for (int s = 0; s < RT_BPW; ++s) {
            if (bI[s] < 0 || 16 * bJ[s] + 15 <= k) continue;
            const int j = 16 * bJ[s] + c, i0 = 16 * bI[s] + rb;
            if (s < RT_REG) {
                rt_update(A[s < RT_REG ? s : 0], i0, j, k, v, p, tau, hw);
            } else {
                double2 x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = lds_blk(s, q);
                rt_update(x, i0, j, k, v, p, tau, hw);
#pragma unroll
                for (int q = 0; q < 4; ++q) lds_blk(s, q) = x[q];
            }
        }
    }
    // the last diagonal element
    const int m = n - 1;
#pragma unroll
    for (int s = 0; s < RT_BPW; ++s) {
        if (bJ[s] == (m >> 4) && bI[s] == (m >> 4) && c == (m & 15)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (16 * bI[s] + rb + q == m) {
                    a.d[m] = s < RT_REG ? A[s < RT_REG ? s : 0][q].x : lds_blk(s, q).x;
                    a.e[m] = 0.0;
                }
            }
        }
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

// ------------------------------------------------------------------ 2'. eigenvalues by multisection
struct EigvalArgs {
    const double* d;      // [n] diagonal of T
    const double* e;      // [n] off-diagonal: e[i] couples i and i+1 (e[n-1] = 0)
    double* ev;           // [n] eigenvalues of T / scale, descending, unclamped
    double* scale;        // [1] the scale: infinity norm of T
    double* lam;          // [n] eigenvalues of T, descending, clamped at 0
    double* sigma;        // [n] sqrt(lam), or null
    int* status;          // or null
    int n;
};

// Number of eigenvalues of the scaled T below x: the negative pivots of the LDL^T
// factorisation of T - x I.  A pivot smaller than pmin in magnitude is replaced by -pmin
// (the count of a nearby matrix; no division by zero).
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pmin) {
    double q = d[0] - x;
    if (fabs(q) < pmin) q = -pmin;
    int c = q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pmin) q = -pmin;
        c += q < 0.0;
    }
    return c;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ void __launch_bounds__(EV_THREADS) eigval_kernel(const EigvalArgs a) {
    constexpr int NW = EV_THREADS / 64;
    __shared__ double sd[FQ_MAX_NT], se2[FQ_MAX_NT];
    __shared__ double red[3][NW];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // infinity norm of T
    double nrm = 0.0;
    for (int i = tid; i < n; i += EV_THREADS)
        nrm = fmax(nrm, fabs(a.d[i]) + fabs(a.e[i]) + (i > 0 ? fabs(a.e[i - 1]) : 0.0));
    nrm = wave_max(nrm);
    if (lane == 0) red[0][w] = nrm;
    __syncthreads();
    double sc = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) sc = fmax(sc, red[0][k]);
    const double isc = sc > 0.0 ? 1.0 / sc : 0.0;
    // scaled T in LDS and its Gershgorin interval
    double glo = 0.0, ghi = 0.0, emax = 0.0;
    for (int i = tid; i < n; i += EV_THREADS) {
        const double di = a.d[i] * isc, ei = i + 1 < n ? a.e[i] * isc : 0.0;
        const double em = i > 0 ? a.e[i - 1] * isc : 0.0;
        sd[i] = di;
        se2[i] = ei * ei;
        const double r = fabs(ei) + fabs(em);
        glo = fmin(glo, di - r);
        ghi = fmax(ghi, di + r);
        emax = fmax(emax, ei * ei);
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    emax = wave_max(emax);
    __syncthreads();
    if (lane == 0) {
        red[0][w] = glo;
        red[1][w] = ghi;
        red[2][w] = emax;
    }
    __syncthreads();
    double gl = red[0][0], gu = red[1][0], e2max = red[2][0];
#pragma unroll
    for (int k = 1; k < NW; ++k) {
        gl = fmin(gl, red[0][k]);
        gu = fmax(gu, red[1][k]);
        e2max = fmax(e2max, red[2][k]);
    }
    const double eps = 2.220446049250313e-16;
    const double pmin = DBL_TINY * fmax(1.0, e2max);
    const double widen = 2.1 * eps * n * fmax(fabs(gl), fabs(gu)) + 4.0 * pmin;
    gl -= widen;
    gu += widen;
    if (blockIdx.x == 0 && tid == 0) {
        *a.scale = sc;
        if (a.status) *a.status = FQ_OK;
    }
    const int j = blockIdx.x * NW + w;   // index in ascending order
    if (j >= n) return;
    // bracket [lo, hi) with count(lo) <= j < count(hi), narrowed 65-fold per round
    double lo = gl, hi = gu;
    for (int r = 0; r < EV_ROUNDS; ++r) {
        const double x = lo + (hi - lo) * ((double)(lane + 1) * (1.0 / 65.0));
        const int c = sturm_count(sd, se2, n, x, pmin);
        const uint64_t b = __ballot(c > j);
        const int f = b ? __ffsll((unsigned long long)b) - 1 : 64;
        const double xf = __shfl(x, f < 64 ? f : 63);
        const double xp = __shfl(x, f > 0 ? f - 1 : 0);
        if (f > 0) lo = xp;
        if (f < 64) hi = xf;
        if (hi - lo <= fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), 1e-20)) break;
    }
    if (lane == 0) {
        const double ev = 0.5 * (lo + hi);
        const int rk = n - 1 - j;
        a.ev[rk] = ev;
        const double l = ev > 0.0 ? ev * sc : 0.0;
        a.lam[rk] = l;
        if (a.sigma) a.sigma[rk] = sqrt(l);
    }
}

// ------------------------------------------------------------------ 4'. inverse iteration
struct InvitArgs {
    const double* d;
    const double* e;
    const double* ev;       // [n] eigenvalues of T / scale, descending
    const double* scale;    // [1]
    const int* k_dev;       // vectors wanted (device word), or null: k_const
    int k_const;
    double* Z;              // [KMAX][n]: Z[j * n + i] = component i of the eigenvector of ev[j]
    int* status;            // or null
    int n;
};

// deterministic pseudo-random start vector in [-1, 1)
__device__ __forceinline__ double start_component(int i, int j) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)j * 0x85EBCA77u + 0x27D4EB2Fu);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// One workgroup (one wavefront) per wanted eigenvalue.  T - lambda I is factorised by
// Gaussian elimination with partial pivoting (rows i, i+1 exchanged when the sub-diagonal
// entry is the larger): U has a diagonal, a super-diagonal and a second super-diagonal
// (created by exchanges); pivots below eps of the unit-scaled T are raised to +-eps, which
// is what makes the nearly singular solve amplify the wanted eigenvector.  The serial
// factorisation and solves run on lane 0 with the next row's operands loaded one step
// ahead (the dependent chain is then arithmetic only); normalisation is wave-parallel.
// Vectors of eigenvalues closer than CLUSTER_TOL are made orthogonal afterwards
// (orth_kernel); farther apart, inverse iteration leaves them orthogonal to ~eps/gap.
__global__ void __launch_bounds__(64) invit_kernel(const InvitArgs a) {
    __shared__ double sd[FQ_MAX_NT], se[FQ_MAX_NT];
    __shared__ double ua[FQ_MAX_NT], ub[FQ_MAX_NT], uc[FQ_MAX_NT], lf[FQ_MAX_NT];
    __shared__ unsigned char sw[FQ_MAX_NT];
    __shared__ double x[FQ_MAX_NT];
    const int n = a.n, lane = threadIdx.x, j = blockIdx.x;
    const int K = a.k_dev ? *a.k_dev : a.k_const;
    if (j >= K) return;
    const double sc = *a.scale, isc = sc > 0.0 ? 1.0 / sc : 0.0;
    const double lam = a.ev[j];
    for (int i = lane; i < n; i += 64) {
        sd[i] = a.d[i] * isc - lam;
        se[i] = i + 1 < n ? a.e[i] * isc : 0.0;
        x[i] = start_component(i, j);
    }
    __syncthreads();
    const double tiny = 2.220446049250313e-16;
    if (lane == 0) {
        // elimination; (p, q) = diagonal and super-diagonal of the current row
        double p = sd[0], q = se[0];
        for (int i = 0; i + 1 < n; ++i) {
            const double sub = se[i];                           // entry (i+1, i)
            const double dn = sd[i + 1];                        // entry (i+1, i+1)
            const double en = i + 2 < n ? se[i + 1] : 0.0;      // entry (i+1, i+2)
            if (fabs(p) >= fabs(sub)) {
                const double l = sub / (p != 0.0 ? p : tiny);
                lf[i] = l;
                sw[i] = 0;
                ua[i] = p;
                ub[i] = q;
                uc[i] = 0.0;
                p = dn - l * q;
                q = en;
            } else {
                const double l = p / sub;
                lf[i] = l;
                sw[i] = 1;
                ua[i] = sub;
                ub[i] = dn;
                uc[i] = en;
                p = q - l * dn;
                q = -l * en;
            }
        }
        ua[n - 1] = p;
        ub[n - 1] = 0.0;
        uc[n - 1] = 0.0;
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        const double p = ua[i];
        ua[i] = 1.0 / (fabs(p) >= tiny ? p : (p < 0.0 ? -tiny : tiny));
    }
    __syncthreads();
    int bad = 0;
    for (int it = 0; it < INVIT_ITERS; ++it) {
        if (lane == 0) {
            // L y = P x: the carried value is x[i] as updated by step i-1
            double c = x[0];
            for (int i = 0; i + 1 < n; ++i) {
                const double nx = x[i + 1];
                const double l = lf[i];
                if (sw[i]) {
                    x[i] = nx;
                    c = c - l * nx;
                } else {
                    x[i] = c;
                    c = nx - l * c;
                }
            }
            x[n - 1] = c;
            // U z = y
            double z1 = 0.0, z2 = 0.0;   // z[i+1], z[i+2]
            for (int i = n - 1; i >= 0; --i) {
                const double zi = (x[i] - ub[i] * z1 - uc[i] * z2) * ua[i];
                x[i] = zi;
                z2 = z1;
                z1 = zi;
            }
        }
        __syncthreads();
        double ss = 0.0;
        for (int i = lane; i < n; i += 64) ss += x[i] * x[i];
        ss = wave_sum(ss);
        const bool ok = ss > 0.0 && ss < 1.0 / 0.0;
        bad |= !ok;
        const double inv = ok ? 1.0 / sqrt(ss) : 0.0;
        for (int i = lane; i < n; i += 64) x[i] = ok ? x[i] * inv : start_component(i, j + it + 1);
        __syncthreads();
    }
    for (int i = lane; i < n; i += 64) a.Z[(size_t)j * n + i] = x[i];
    if (bad && lane == 0 && a.status) *a.status = FQ_E_NUMERIC;
}

// Orthogonalisation inside clusters (one workgroup): for each wanted vector whose
// eigenvalue lies within CLUSTER_TOL of the previous one, classical Gram-Schmidt against
// the cluster's earlier vectors, applied twice, then normalisation.
constexpr int ORTH_THREADS = 256;

__global__ void __launch_bounds__(ORTH_THREADS) orth_kernel(const InvitArgs a) {
    __shared__ double zj[FQ_MAX_NT];
    __shared__ double dots[KMAX];
    __shared__ double red[ORTH_THREADS / 64];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int K = a.k_dev ? *a.k_dev : a.k_const;
    int c = 0;   // first index of the current cluster
    for (int j = 1; j < K; ++j) {
        if (a.ev[j - 1] - a.ev[j] > CLUSTER_TOL) {
            c = j;
            continue;
        }
        double* z = a.Z + (size_t)j * n;
        for (int i = tid; i < n; i += ORTH_THREADS) zj[i] = z[i];
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int p = c + wv; p < j; p += ORTH_THREADS / 64) {
                const double* zp = a.Z + (size_t)p * n;
                double d = 0.0;
                for (int i = lane; i < n; i += 64) d += zp[i] * zj[i];
                d = wave_sum(d);
                if (lane == 0) dots[p - c] = d;
            }
            __syncthreads();
            for (int i = tid; i < n; i += ORTH_THREADS) {
                double v = zj[i];
                for (int p = c; p < j; ++p) v -= dots[p - c] * a.Z[(size_t)p * n + i];
                zj[i] = v;
            }
            __syncthreads();
        }
        double ss = 0.0;
        for (int i = tid; i < n; i += ORTH_THREADS) ss += zj[i] * zj[i];
        ss = block_sum<ORTH_THREADS>(ss, red);
        const bool ok = ss > 0.0 && ss < 1.0 / 0.0;
        const double inv = ok ? 1.0 / sqrt(ss) : 0.0;
        for (int i = tid; i < n; i += ORTH_THREADS) z[i] = zj[i] * inv;
        if (!ok && tid == 0 && a.status) *a.status = FQ_E_NUMERIC;
        __threadfence();   // the next vectors of the cluster read this one back
        __syncthreads();
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
    const double* Z;      // eigenvectors of T: component i of vector j at Z[i * zr + j * zc]
    int zr, zc;
    const double2* vh;    // [n][n]
    const double2* tau;   // [n]
    double2* V;           // [n][n], columns j < K written
    const int* k_dev;     // K (device word), or null: k_const
    int k_const;
    int n;
};

constexpr int BT_PER_LANE = FQ_MAX_NT / 64;

__global__ void __launch_bounds__(64) back_kernel(const BackArgs a) {
    const int n = a.n, j = blockIdx.x, lane = threadIdx.x;
    if (j >= (a.k_dev ? *a.k_dev : a.k_const)) return;
    double2 z[BT_PER_LANE];
#pragma unroll
    for (int t = 0; t < BT_PER_LANE; ++t) {
        const int i = lane + 64 * t;
        z[t] = make_double2(i < n ? a.Z[(size_t)i * a.zr + (size_t)j * a.zc] : 0.0, 0.0);
    }
    // reflector k's tau and v (zero outside rows k+1 .. n-1), fetched one reflector ahead
    double2 vn[BT_PER_LANE], taun = make_double2(0.0, 0.0);
    auto fetch = [&](int k) {
        taun = a.tau[k];
        const double2* v = a.vh + (size_t)k * n;
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) {
            const int i = lane + 64 * t;
            vn[t] = i > k && i < n ? v[i] : make_double2(0.0, 0.0);
        }
    };
    if (n >= 2) fetch(n - 2);
    for (int k = n - 2; k >= 0; --k) {
        double2 v[BT_PER_LANE];
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) v[t] = vn[t];
        const double2 tau = taun;
        if (k > 0) fetch(k - 1);
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        double2 dot = make_double2(0.0, 0.0);   // v^H z over rows k+1 .. n-1
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) {
            dot.x += v[t].x * z[t].x + v[t].y * z[t].y;
            dot.y += v[t].x * z[t].y - v[t].y * z[t].x;
        }
        dot.x = wave_total(dot.x);
        dot.y = wave_total(dot.y);
        const double2 td = zmul(tau, dot);
#pragma unroll
        for (int t = 0; t < BT_PER_LANE; ++t) {
            const double2 u = zmul(v[t], td);
            z[t].x -= u.x;
            z[t].y -= u.y;
        }
    }
#pragma unroll
    for (int t = 0; t < BT_PER_LANE; ++t) {
        const int i = lane + 64 * t;
        if (i < n) a.V[(size_t)i * n + j] = z[t];
    }
}

// K selection (one thread).
struct RankArgs {
    const double* lam;
    int* k_used;
    int* status;           // may be null
    int n, cutoff;
};

__global__ void rank_kernel(const RankArgs a) {
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
        *a.k_used = K;
    }
}

// FP32 copy of V_K [n][KMAX] and FP64 copy of its first KN columns [n][KN], both zero
// beyond column K (the projections run whole size classes).
constexpr int KN = 16;
__global__ void vk_kernel(const double2* vecs, const int* k_used, float2* vk, double2* vk64, int n) {
    const int K = *k_used;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * KMAX; idx += gridDim.x * blockDim.x) {
        const int f = idx / KMAX, k = idx % KMAX;
        double2 d = make_double2(0.0, 0.0);
        if (k < K) d = vecs[(size_t)f * n + k];
        vk[idx] = make_float2((float)d.x, (float)d.y);
        if (k < KN) vk64[f * KN + k] = d;
    }
}

// Power Doppler alone (no filtered IQ) for K <= 16: V_K has orthonormal columns, so the
// filtered energy of a voxel's row s of S is ||s - s V_K V_K^H||^2 = ||s||^2 - ||s V_K||^2
// (Pythagoras), formed in FP64 (the clutter energy it cancels is up to ~1e6 times the
// result) from one read of S.
// One voxel per thread; V_K rows are uniform across the wavefront (scalar loads).  The
// difference is clamped at zero, the value it rounds around when K removes every mode.
struct PdNormArgs {
    const float2* iq;     // [nt][nv]
    const double2* vk64;  // [nt][KN]
    const int* k_used;
    float* pd;            // [nv]
    int64_t nv;
    int nt;
    int k_lo;             // this instantiation serves k_lo < K <= KM
};

template <int KM>
__global__ void __launch_bounds__(256) pd_norm_kernel(const PdNormArgs a) {
    const int K = *a.k_used;
    if (K <= a.k_lo || K > KM) return;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.nv) return;
    double cr[KM], ci[KM], nx = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) cr[k] = ci[k] = 0.0;
    const float2* sv = a.iq + v;
#pragma unroll 2
    for (int f = 0; f < a.nt; ++f) {
        const float2 x = sv[(int64_t)f * a.nv];
        const double xr = x.x, xi = x.y;
        nx = fma(xr, xr, fma(xi, xi, nx));
        const double2* w = a.vk64 + f * KN;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const double2 u = w[k];   // c_k = sum_f s_f V[f][k] (s V_K for the row s of S)
            cr[k] = fma(u.x, xr, fma(-u.y, xi, cr[k]));
            ci[k] = fma(u.x, xi, fma(u.y, xr, ci[k]));
        }
    }
    double c2 = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) c2 = fma(cr[k], cr[k], fma(ci[k], ci[k], c2));
    a.pd[v] = (float)(fmax(nx - c2, 0.0) / a.nt);
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

// Projection and power Doppler on the matrix cores.  A workgroup of four wavefronts
// stages V_K (FP32 copy, zero beyond column K and frame n_t) in LDS once; each wavefront
// then owns 16 voxels: P = S V_K (16 x KM) with v_mfma_f32_16x16x4_f32 over the frames
// (the four real products of the complex product, S read straight from HBM as MFMA
// operands), P staged in LDS, and R = S - P V_K^H formed 16 frames at a time with the
// same MFMA over the K columns, subtracted from S (read again: the wavefront's 16-voxel
// slice was just fetched, so this read is served by the L2), squared and summed per voxel.
// MFMA 16x16x4 (FP32) lane layout: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// holds D[4(l/16) + r][l%16], r = 0..3.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int PV = 16;             // voxels per wavefront
constexpr int PW = 4;              // wavefronts per workgroup

__host__ __device__ inline int vk_stride(int km) { return km + 2; }   // LDS row stride of V_K (float2)

// VL: V_K staged in LDS (when it fits beside the P staging), else read from the
// L2-resident table (rows beyond n_t are then masked).
template <int KM, bool VL>
__global__ void __launch_bounds__(64 * PW) project_mfma_kernel(const PdArgs a) {
    extern __shared__ float2 sm2[];
    const int K = *a.k_used;
    if (K <= a.k_lo || K > KM) return;
    constexpr int NKT = KM / 16;
    constexpr int VS = VL ? KM + 2 : KMAX;
    constexpr int PS = KM + 1;
    const int nt = a.nt, ntp = (nt + 15) & ~15;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float* Pr = reinterpret_cast<float*>(sm2 + (VL ? ntp * VS : 0)) + wv * 2 * PV * PS;   // [PV][PS]
    float* Pi = Pr + PV * PS;
    if (VL) {
        for (int idx = threadIdx.x; idx < ntp * KM; idx += 64 * PW) {
            const int f = idx / KM, k = idx % KM;
            sm2[f * VS + k] = f < nt ? a.vk[f * KMAX + k] : make_float2(0.f, 0.f);
        }
    }
    const float2* V = VL ? sm2 : a.vk;   // [ntp or n_t][VS]
    __syncthreads();
    const int li = lane & 15, lk = lane >> 4;
    const int64_t v0 = ((int64_t)blockIdx.x * PW + wv) * PV;
    if (v0 >= a.nv) return;
    const bool full = v0 + PV <= a.nv;
    const float2* S = a.iq;
    // P = S V_K: A[i][k] = S[voxel i][frame f0 + k], B[k][j] = V[frame f0 + k][column 16t + j]
    floatx4 rr[NKT], ii[NKT], ri[NKT], ir[NKT];
#pragma unroll
    for (int t = 0; t < NKT; ++t)
        for (int r = 0; r < 4; ++r) rr[t][r] = ii[t][r] = ri[t][r] = ir[t][r] = 0.f;
    const bool vin = full || v0 + li < a.nv;
#pragma unroll 4
    for (int f0 = 0; f0 < ntp; f0 += 4) {
        const int f = f0 + lk;
        const float2 x = (f < nt && vin) ? S[(int64_t)f * a.nv + v0 + li] : make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < NKT; ++t) {
            const float2 w = (VL || f < nt) ? V[f * VS + 16 * t + li] : make_float2(0.f, 0.f);
            rr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, w.x, rr[t], 0, 0, 0);
            ii[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, w.y, ii[t], 0, 0, 0);
            ri[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, w.y, ri[t], 0, 0, 0);
            ir[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, w.x, ir[t], 0, 0, 0);
        }
    }
    // P[voxel 4 lk + r][column 16 t + li]
#pragma unroll
    for (int t = 0; t < NKT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Pr[(4 * lk + r) * PS + 16 * t + li] = rr[t][r] - ii[t][r];
            Pi[(4 * lk + r) * PS + 16 * t + li] = ri[t][r] + ir[t][r];
        }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // R = S - P V_K^H, 16 frames at a time: A[i][k] = P[voxel i][k0 + k],
    // B[k][j] = conj(V[frame f0 + j][k0 + k]); lane holds R[voxel 4 lk + r][frame f0 + li]
    float pacc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int f0 = 0; f0 < ntp; f0 += 16) {
        const int f = f0 + li;
        floatx4 qa, qb, qc, qd;
        for (int r = 0; r < 4; ++r) qa[r] = qb[r] = qc[r] = qd[r] = 0.f;
#pragma unroll
        for (int k0 = 0; k0 < KM; k0 += 4) {
            const float pr = Pr[li * PS + k0 + lk], pi = Pi[li * PS + k0 + lk];
            const float2 w = (VL || f < nt) ? V[f * VS + k0 + lk] : make_float2(0.f, 0.f);
            qa = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, w.x, qa, 0, 0, 0);
            qb = __builtin_amdgcn_mfma_f32_16x16x4f32(pi, w.y, qb, 0, 0, 0);
            qc = __builtin_amdgcn_mfma_f32_16x16x4f32(pi, w.x, qc, 0, 0, 0);
            qd = __builtin_amdgcn_mfma_f32_16x16x4f32(pr, w.y, qd, 0, 0, 0);
        }
        float2 sv[4];
        if (f < nt && full) {
            const float4* sp = reinterpret_cast<const float4*>(S + (int64_t)f * a.nv + v0 + 4 * lk);
            const float4 s0 = sp[0], s1 = sp[1];
            sv[0] = make_float2(s0.x, s0.y);
            sv[1] = make_float2(s0.z, s0.w);
            sv[2] = make_float2(s1.x, s1.y);
            sv[3] = make_float2(s1.z, s1.w);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t v = v0 + 4 * lk + r;
                sv[r] = (f < nt && v < a.nv) ? S[(int64_t)f * a.nv + v] : make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // P conj(V) = (Pr Vr + Pi Vi) + i (Pi Vr - Pr Vi)
            const float xr = sv[r].x - (qa[r] + qb[r]);
            const float xi = sv[r].y - (qc[r] - qd[r]);
            pacc[r] = fmaf(xr, xr, fmaf(xi, xi, pacc[r]));
            const int64_t v = v0 + 4 * lk + r;
            if (a.out && f < nt && v < a.nv) a.out[(int64_t)f * a.nv + v] = make_float2(xr, xi);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float x = pacc[r];
        for (int o = 1; o < 16; o <<= 1) x += __shfl_xor(x, o);
        pacc[r] = x;
    }
    if (li == 0 && a.pd) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t v = v0 + 4 * lk + r;
            if (v < a.nv) a.pd[v] = pacc[r] * a.inv_nt;
        }
    }
}

constexpr size_t PROJ_LDS_MAX = 150 * 1024;

size_t project_mfma_lds(int nt, int km, bool vl) {
    const int ntp = (nt + 15) & ~15;
    return (vl ? sizeof(float2) * (size_t)ntp * vk_stride(km) : 0) + sizeof(float) * 2 * PW * PV * (size_t)(km + 1);
}
bool project_vl(int nt, int km) { return project_mfma_lds(nt, km, true) <= PROJ_LDS_MAX; }

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

using TriFn = void (*)(const TriArgs);
int tri_threads(int n) { return n <= RT_N ? RT_THREADS : TRI_THREADS; }
TriFn tri_fn(int n) {
    if (n <= RT_N) return tridiag_reg_kernel;
    if (n <= 256) return tridiag_kernel<4>;
    return tridiag_kernel<FQ_MAX_NT / 64>;
}

struct SvdWs {
    size_t off_A, off_vh, off_tau, off_d, off_e, off_ri, off_rc, off_rs, off_rn, off_perm, off_Zs;
    size_t off_lam, off_vecs, off_vk, off_vk64, off_k, off_ev, off_sc, off_zt, total;
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
    w.off_vk64 = take(sizeof(double2) * (size_t)n * KN);
    w.off_k = take(sizeof(int));
    w.off_ev = take(sizeof(double) * n);
    w.off_sc = take(sizeof(double));
    w.off_zt = take(sizeof(double) * (size_t)n * KMAX);
    w.total = o;
    return w;
}

// Every eigenpair by QL (hermitian_eig): eigenvalues (descending, clamped) into lam/sigma;
// the leading ncols eigenvectors into vecs ([n][n] complex128, columns in rank order)
// unless vecs is null.
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
    hipLaunchKernelGGL(tri_fn(n), dim3(1), dim3(tri_threads(n)), 0, s, ta);
    FQ_LAUNCH_CHECK();
    QlArgs qa{d, e, ri, rc, rs, rn, L.cap, lam, sigma, perm, status, n};
    hipLaunchKernelGGL(ql_kernel, dim3(1), dim3(64), 0, s, qa);
    FQ_LAUNCH_CHECK();
    if (!vecs || ncols < 1) return FQ_OK;
    const int rows = n <= 256 ? 64 : 32;   // LDS: rows x n doubles <= 128 KiB
    ReplayArgs pa{ri, rc, rs, rn, perm, Zs, n, rows};
    hipLaunchKernelGGL(replay_kernel, dim3((n + rows - 1) / rows), dim3(64), sizeof(double) * (size_t)rows * n, s, pa);
    FQ_LAUNCH_CHECK();
    BackArgs ba{Zs, n, 1, vh, tau, reinterpret_cast<double2*>(vecs), nullptr, std::min(ncols, n), n};
    hipLaunchKernelGGL(back_kernel, dim3(std::min(ncols, n)), dim3(64), 0, s, ba);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

// The clutter filter's eigensolver, first half: tridiagonalisation and every eigenvalue
// (lam, sigma, and the unit-scaled ev for the vectors).
int launch_eigvals(const double* gram, int n, char* ws, const SvdWs& L, double* lam, double* sigma, int* status,
                   hipStream_t s) {
    TriArgs ta{reinterpret_cast<const double2*>(gram), reinterpret_cast<double2*>(ws + L.off_A),
               reinterpret_cast<double2*>(ws + L.off_vh), reinterpret_cast<double2*>(ws + L.off_tau),
               reinterpret_cast<double*>(ws + L.off_d), reinterpret_cast<double*>(ws + L.off_e), n};
    hipLaunchKernelGGL(tri_fn(n), dim3(1), dim3(tri_threads(n)), 0, s, ta);
    FQ_LAUNCH_CHECK();
    EigvalArgs ea{reinterpret_cast<const double*>(ws + L.off_d), reinterpret_cast<const double*>(ws + L.off_e),
                  reinterpret_cast<double*>(ws + L.off_ev), reinterpret_cast<double*>(ws + L.off_sc), lam, sigma,
                  status, n};
    constexpr int per_block = EV_THREADS / 64;
    hipLaunchKernelGGL(eigval_kernel, dim3((n + per_block - 1) / per_block), dim3(EV_THREADS), 0, s, ea);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

// Second half: the K leading eigenvectors (K from the device word k_dev, else k_const),
// by inverse iteration on T and back-transformation, into vecs columns 0 .. K-1.
int launch_eigvecs(int n, char* ws, const SvdWs& L, const int* k_dev, int k_const, double* vecs, int* status,
                   hipStream_t s) {
    double* zt = reinterpret_cast<double*>(ws + L.off_zt);
    const int grid = k_dev ? KMAX : k_const;
    if (grid < 1) return FQ_OK;
    InvitArgs ia{reinterpret_cast<const double*>(ws + L.off_d), reinterpret_cast<const double*>(ws + L.off_e),
                 reinterpret_cast<const double*>(ws + L.off_ev), reinterpret_cast<const double*>(ws + L.off_sc),
                 k_dev, k_const, zt, status, n};
    hipLaunchKernelGGL(invit_kernel, dim3(grid), dim3(64), 0, s, ia);
    FQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(ORTH_THREADS), 0, s, ia);
    FQ_LAUNCH_CHECK();
    BackArgs ba{zt, 1, n, reinterpret_cast<const double2*>(ws + L.off_vh),
                reinterpret_cast<const double2*>(ws + L.off_tau), reinterpret_cast<double2*>(vecs), k_dev, k_const, n};
    hipLaunchKernelGGL(back_kernel, dim3(grid), dim3(64), 0, s, ba);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

using PdFn = void (*)(const PdArgs);
PdFn pd_fn(int k, bool vl) {
    if (k <= 16) return vl ? project_mfma_kernel<16, true> : project_mfma_kernel<16, false>;
    if (k <= 32) return vl ? project_mfma_kernel<32, true> : project_mfma_kernel<32, false>;
    return vl ? project_mfma_kernel<64, true> : project_mfma_kernel<64, false>;
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

// The filter's last stage on the V_K (FP32 and FP64 copies) and K that the eigendecomposition
// left in the workspace: the filtered IQ and/or the power Doppler.
static int launch_apply(const float* iq, int64_t n_vox, int n_t, char* w, const SvdWs& L, int cutoff,
                        const int32_t* k_used, float* iq_filt, float* pd, hipStream_t s) {
    PdArgs pa{};
    pa.iq = reinterpret_cast<const float2*>(iq);
    pa.vk = reinterpret_cast<const float2*>(w + L.off_vk);
    pa.k_used = k_used;
    pa.out = reinterpret_cast<float2*>(iq_filt);
    pa.pd = pd;
    pa.nv = n_vox;
    pa.nt = n_t;
    pa.inv_nt = 1.0f / (float)n_t;
    const unsigned blocks = (unsigned)((n_vox + PV * PW - 1) / (PV * PW));
    if (!iq_filt) {
        // power Doppler alone: the FP64 norm difference up to K = 16, the explicit
        // projection above; all but the class holding K return at once
        PdNormArgs na{pa.iq, reinterpret_cast<const double2*>(w + L.off_vk64), k_used, pd, n_vox, n_t, -1};
        const unsigned nb = (unsigned)((n_vox + 255) / 256);
        const int bounds[6] = {-1, 4, 8, 16, 32, 64};
        for (int c = 0; c < 5; ++c) {
            if (cutoff >= 0 && !(cutoff > bounds[c] && cutoff <= bounds[c + 1])) continue;
            if (c < 3) {
                na.k_lo = bounds[c];
                auto kern = c == 0 ? pd_norm_kernel<4> : (c == 1 ? pd_norm_kernel<8> : pd_norm_kernel<16>);
                hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s, na);
            } else {
                pa.k_lo = bounds[c];
                const bool vl = project_vl(n_t, bounds[c + 1]);
                hipLaunchKernelGGL(pd_fn(bounds[c + 1], vl), dim3(blocks), dim3(64 * PW),
                                   project_mfma_lds(n_t, bounds[c + 1], vl), s, pa);
            }
            FQ_LAUNCH_CHECK();
        }
        return FQ_OK;
    }
    if (cutoff >= 0) {
        const int km = cutoff <= 16 ? 16 : (cutoff <= 32 ? 32 : 64);
        pa.k_lo = -1;
        const bool vl = project_vl(n_t, km);
        hipLaunchKernelGGL(pd_fn(km, vl), dim3(blocks), dim3(64 * PW), project_mfma_lds(n_t, km, vl), s, pa);
        FQ_LAUNCH_CHECK();
    } else {
        // the knee's K is only known on the device: every size class is launched and
        // all but the one holding K return at once
        const int bounds[4] = {-1, 16, 32, 64};
        for (int c = 0; c < 3; ++c) {
            pa.k_lo = bounds[c];
            const bool vl = project_vl(n_t, bounds[c + 1]);
            hipLaunchKernelGGL(pd_fn(bounds[c + 1], vl), dim3(blocks), dim3(64 * PW),
                               project_mfma_lds(n_t, bounds[c + 1], vl), s, pa);
            FQ_LAUNCH_CHECK();
        }
    }
    return FQ_OK;
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
    int st = launch_eigvals(gram, n_t, w, L, lam, sigma, status, s);
    if (st != FQ_OK) return st;
    RankArgs ra{lam, k_used, status, n_t, cutoff};
    if (cutoff == FQ_CUTOFF_SSM) {
        // the rank is read from the leading min(n_t, 64) spatial modes
        const int M = std::min(n_t, FQ_SSM_MAX_MODES);
        st = launch_eigvecs(n_t, w, L, nullptr, M, vecs, status, s);
        if (st != FQ_OK) return st;
        st = launch_ssm(iq, n_vox, n_t, vecs, M, w + L.total, nullptr, k_used, s);
        if (st != FQ_OK) return st;
        hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(64), 0, s, ra);
        FQ_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(64), 0, s, ra);
        FQ_LAUNCH_CHECK();
        st = launch_eigvecs(n_t, w, L, k_used, 0, vecs, status, s);
        if (st != FQ_OK) return st;
    }
    hipLaunchKernelGGL(vk_kernel, dim3((n_t * KMAX + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(vecs), static_cast<const int*>(k_used),
                       reinterpret_cast<float2*>(w + L.off_vk), reinterpret_cast<double2*>(w + L.off_vk64), n_t);
    FQ_LAUNCH_CHECK();
    if (!iq_filt && !pd) return FQ_OK;
    return launch_apply(iq, n_vox, n_t, w, L, cutoff, k_used, iq_filt, pd, s);
}

extern "C" int svd_filter_apply(const float* iq, int64_t n_vox, int32_t n_t, const void* ws, size_t ws_bytes,
                                const int32_t* k_used, float* iq_filt, float* pd, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(iq && ws && k_used && aligned16(iq) && aligned16(ws), "null or misaligned pointer");
    FQ_REQUIRE(iq_filt || pd, "nothing to compute: iq_filt and pd are both null");
    FQ_REQUIRE(!iq_filt || aligned16(iq_filt), "misaligned iq_filt");
    const SvdWs L = svd_layout(n_t);
    if (ws_bytes < L.total) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, L.total);
        return FQ_E_WORKSPACE;
    }
    return launch_apply(iq, n_vox, n_t, reinterpret_cast<char*>(const_cast<void*>(ws)), L, -1, k_used, iq_filt, pd,
                        as_stream(stream));
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
