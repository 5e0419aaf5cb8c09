// spatial_similarity: the correlation-coefficient matrix of the magnitudes of the spatial
// modes U = S V (the singular-value analyses of Section 3 show it beside the singular-value
// curves; the scale 1/sigma_k of a column does not change a correlation coefficient), and
// the tissue rank read from it.
//
// One pass over the Casorati matrix, fused on the matrix cores:
//   1. a workgroup owns 128-voxel tiles; its four waves form U = S V for 32 voxels x 64
//      modes each with v_mfma_f32_32x32x2_f32 (Re U = Sr Vr - Si Vi, Im U = Sr Vi + Si Vr),
//      streaming 16-frame stages of S and of V (FP32 copy) through LDS;
//   2. |U| of the tile goes to LDS (never to HBM), its column sums are taken from the
//      accumulators, and the 64 x 64 product |U|^T |U| of the tile is formed with MFMA;
//   3. tile results are accumulated in FP64 per workgroup; the workgroup partials are
//      summed in a fixed order (deterministic) and the correlations are formed in FP64:
//        C_jk = (G_jk - s_j s_k / N) / sqrt((G_jj - s_j^2 / N)(G_kk - s_k^2 / N)),
//      clipped to [-1, 1]; a mode without spatial variation gets NaN.
// The rank rule: mode k >= 1 joins the tissue block while a_k > b_k, with
//   a_k = mean_{i<k} C_ik, b_k = mean_{k<j<M} C_kj; K is the first k in [1, min(M-2, M/2)]
//   that does not join (a NaN does not join), or max(1, M/2) when all join.
#include "fq_common.hpp"

namespace fq {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int TV = 128;               // voxels per tile
constexpr int MM = FQ_SSM_MAX_MODES;  // modes per tile (64, zero padded)
constexpr int KF = 16;                // frames per LDS stage
constexpr int LDS_V = TV + 4;         // row stride of an S stage row (floats)
constexpr int LDS_M = MM + 4;         // row stride of a V stage row and of the |U| tile
constexpr int SSM_THREADS = 256;
constexpr int SSM_MAX_WG = 512;
constexpr int PART = MM * MM + MM;    // doubles per workgroup partial: Gram, column sums

constexpr int STAGE_FLOATS = 2 * KF * LDS_V + 2 * KF * LDS_M;
constexpr int TILE_FLOATS = TV * LDS_M;
constexpr int LDS_FLOATS = STAGE_FLOATS > TILE_FLOATS ? STAGE_FLOATS : TILE_FLOATS;

struct VkArgs {
    const double2* vecs;  // [nt][nt]
    float2* vk;           // [rows][MM]
    int nt, rows, m;
};

__global__ void __launch_bounds__(256) ssm_vk_kernel(const VkArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.rows * MM) return;
    const int f = idx / MM, k = idx % MM;
    float2 v = make_float2(0.f, 0.f);
    if (f < a.nt && k < a.m) {
        const double2 d = a.vecs[(size_t)f * a.nt + k];
        v = make_float2((float)d.x, (float)d.y);
    }
    a.vk[idx] = v;
}

struct TileArgs {
    const float2* iq;     // [nt][nv]
    const float2* vk;     // [n_chunks * KF][MM]
    double* part;         // [nwg][PART]
    int64_t nv;
    int nt, n_chunks, ntiles, nwg;
};

__global__ void __launch_bounds__(SSM_THREADS) ssm_tile_kernel(const TileArgs a) {
    __shared__ __attribute__((aligned(16))) float lds[LDS_FLOATS];
    __shared__ double csum_s[4][MM];
    float* sSr = lds;
    float* sSi = sSr + KF * LDS_V;
    float* sVr = sSi + KF * LDS_V;
    float* sVi = sVr + KF * LDS_M;
    float* sA = lds;   // |U| tile, aliases the stage once a tile's last stage is consumed

    const int wg = blockIdx.x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int li = l & 31, lh = l >> 5;
    const int gJ = w >> 1, gK = w & 1;   // Gram quadrant of this wave

    // stage loader: S row fr = tid/16 holds voxels seg*8 .. +8; V row fr holds modes seg*4 .. +4
    const int fr = threadIdx.x >> 4, seg = threadIdx.x & 15;
    const bool even = (a.nv & 1) == 0;
    float4 ps[4], pv[2];
    auto load = [&](int t, int c) {
        const int f = c * KF + fr;
        const int64_t v = (int64_t)t * TV + seg * 8;
        if (f < a.nt && even && v + 8 <= a.nv) {
            const float4* src = reinterpret_cast<const float4*>(a.iq + (int64_t)f * a.nv + v);
#pragma unroll
            for (int q = 0; q < 4; ++q) ps[q] = src[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float2 p0 = make_float2(0.f, 0.f), p1 = make_float2(0.f, 0.f);
                if (f < a.nt && v + 2 * q < a.nv) p0 = a.iq[(int64_t)f * a.nv + v + 2 * q];
                if (f < a.nt && v + 2 * q + 1 < a.nv) p1 = a.iq[(int64_t)f * a.nv + v + 2 * q + 1];
                ps[q] = make_float4(p0.x, p0.y, p1.x, p1.y);
            }
        }
        const float4* vsrc = reinterpret_cast<const float4*>(a.vk + (size_t)f * MM + seg * 4);
        pv[0] = vsrc[0];
        pv[1] = vsrc[1];
    };

    floatx16 ur0, ui0, ur1, ui1;
    double g64[16];
    double cs64[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        ur0[r] = ui0[r] = ur1[r] = ui1[r] = 0.f;
        g64[r] = 0.0;
    }

    int t = wg, c = 0;
    if (t < a.ntiles) load(t, 0);
    while (t < a.ntiles) {
        __syncthreads();   // the previous stage / |U| tile is no longer read
        {
            float* dr = sSr + fr * LDS_V + seg * 8;
            float* di = sSi + fr * LDS_V + seg * 8;
            *reinterpret_cast<float4*>(dr) = make_float4(ps[0].x, ps[0].z, ps[1].x, ps[1].z);
            *reinterpret_cast<float4*>(dr + 4) = make_float4(ps[2].x, ps[2].z, ps[3].x, ps[3].z);
            *reinterpret_cast<float4*>(di) = make_float4(ps[0].y, ps[0].w, ps[1].y, ps[1].w);
            *reinterpret_cast<float4*>(di + 4) = make_float4(ps[2].y, ps[2].w, ps[3].y, ps[3].w);
            *reinterpret_cast<float4*>(sVr + fr * LDS_M + seg * 4) = make_float4(pv[0].x, pv[0].z, pv[1].x, pv[1].z);
            *reinterpret_cast<float4*>(sVi + fr * LDS_M + seg * 4) = make_float4(pv[0].y, pv[0].w, pv[1].y, pv[1].w);
        }
        __syncthreads();
        int tn = t, cn = c + 1;
        if (cn == a.n_chunks) {
            cn = 0;
            tn = t + a.nwg;
        }
        if (tn < a.ntiles) load(tn, cn);   // next stage in flight during the MFMAs

        if (c == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) ur0[r] = ui0[r] = ur1[r] = ui1[r] = 0.f;
        }
#pragma unroll
        for (int kk = 0; kk < KF; kk += 2) {
            const int f = kk + lh;
            const float ar = sSr[f * LDS_V + 32 * w + li];
            const float ai = sSi[f * LDS_V + 32 * w + li];
            const float nai = -ai;
            const float br0 = sVr[f * LDS_M + li], bi0 = sVi[f * LDS_M + li];
            const float br1 = sVr[f * LDS_M + 32 + li], bi1 = sVi[f * LDS_M + 32 + li];
            ur0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br0, ur0, 0, 0, 0);
            ur0 = __builtin_amdgcn_mfma_f32_32x32x2f32(nai, bi0, ur0, 0, 0, 0);
            ui0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi0, ui0, 0, 0, 0);
            ui0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br0, ui0, 0, 0, 0);
            ur1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br1, ur1, 0, 0, 0);
            ur1 = __builtin_amdgcn_mfma_f32_32x32x2f32(nai, bi1, ur1, 0, 0, 0);
            ui1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi1, ui1, 0, 0, 0);
            ui1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br1, ui1, 0, 0, 0);
        }

        if (c == a.n_chunks - 1) {
            __syncthreads();   // every wave is done with the stage that sA overwrites
            // accumulator layout: lane l holds column l%32, rows 8*(r/4) + 4*(l/32) + r%4
            float cs0 = 0.f, cs1 = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * w + 8 * (r >> 2) + 4 * lh + (r & 3);
                const float m0 = __builtin_sqrtf(ur0[r] * ur0[r] + ui0[r] * ui0[r]);
                const float m1 = __builtin_sqrtf(ur1[r] * ur1[r] + ui1[r] * ui1[r]);
                sA[row * LDS_M + li] = m0;
                sA[row * LDS_M + 32 + li] = m1;
                cs0 += m0;
                cs1 += m1;
            }
            cs64[0] += (double)cs0;
            cs64[1] += (double)cs1;
            __syncthreads();
            floatx16 g;
#pragma unroll
            for (int r = 0; r < 16; ++r) g[r] = 0.f;
#pragma unroll 8
            for (int vv = 0; vv < TV; vv += 2) {
                const float x = sA[(vv + lh) * LDS_M + 32 * gJ + li];
                const float y = sA[(vv + lh) * LDS_M + 32 * gK + li];
                g = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, g, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) g64[r] += (double)g[r];
        }
        t = tn;
        c = cn;
    }

    double* P = a.part + (size_t)wg * PART;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 32 * gJ + 8 * (r >> 2) + 4 * lh + (r & 3);
        P[row * MM + 32 * gK + li] = g64[r];
    }
    // column sums: lanes l and l^32 hold the two row halves of the same columns
    cs64[0] += __shfl_xor(cs64[0], 32);
    cs64[1] += __shfl_xor(cs64[1], 32);
    if (lh == 0) {
        csum_s[w][li] = cs64[0];
        csum_s[w][32 + li] = cs64[1];
    }
    __syncthreads();
    if (threadIdx.x < MM) {
        const int k = threadIdx.x;
        P[MM * MM + k] = ((csum_s[0][k] + csum_s[1][k]) + csum_s[2][k]) + csum_s[3][k];
    }
}

struct RedArgs {
    const double* part;
    double* red;          // [PART]
    int nwg;
};

__global__ void __launch_bounds__(256) ssm_reduce_kernel(const RedArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= PART) return;
    double s = 0.0;
    for (int g = 0; g < a.nwg; ++g) s += a.part[(size_t)g * PART + idx];
    a.red[idx] = s;
}

struct CorrArgs {
    const double* red;
    double* C;            // [m][m]
    int* k_out;           // may be null
    double inv_n;
    int m;
};

// One workgroup: correlations, then the rank rule on them.
__global__ void __launch_bounds__(256) ssm_corr_kernel(const CorrArgs a) {
    __shared__ double sd[MM];
    __shared__ double sC[MM * MM];
    __shared__ int stop[MM];
    const int m = a.m;
    const double* G = a.red;
    const double* s = a.red + MM * MM;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double var = G[j * MM + j] - s[j] * s[j] * a.inv_n;
        sd[j] = var > 0.0 ? sqrt(var) : 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int j = idx / m, k = idx % m;
        double cjk;
        if (sd[j] > 0.0 && sd[k] > 0.0) {
            // symmetric by construction: the pair (j, k) is read from the upper triangle
            const int lo = min(j, k), hi = max(j, k);
            const double cov = G[lo * MM + hi] - s[lo] * s[hi] * a.inv_n;
            cjk = cov / sd[j] / sd[k];
            cjk = cjk > 1.0 ? 1.0 : (cjk < -1.0 ? -1.0 : cjk);
        } else {
            cjk = __builtin_nan("");
        }
        sC[idx] = cjk;
        a.C[idx] = cjk;
    }
    __syncthreads();
    if (!a.k_out) return;
    const int cap = max(1, m / 2);
    const int kmax = min(m - 2, cap);
    if (threadIdx.x < MM) {
        const int k = threadIdx.x;
        int st = 0;
        if (k >= 1 && k <= kmax) {
            double sa = 0.0, sb = 0.0;
            for (int i = 0; i < k; ++i) sa += sC[k * m + i];
            for (int j = k + 1; j < m; ++j) sb += sC[k * m + j];
            const double am = sa / (double)k, bm = sb / (double)(m - k - 1);
            st = !(am > bm);
        }
        stop[k] = st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int K = cap;
        for (int k = 1; k <= kmax; ++k) {
            if (stop[k]) {
                K = k;
                break;
            }
        }
        *a.k_out = K;
    }
}

struct SsmWs {
    size_t off_vk, off_part, off_red, off_C, total;
    int rows, n_chunks, ntiles, nwg;
};

SsmWs ssm_layout(int64_t nv, int nt) {
    SsmWs w{};
    w.n_chunks = (nt + KF - 1) / KF;
    w.rows = w.n_chunks * KF;
    const int64_t nt_tiles = (nv + TV - 1) / TV;
    w.ntiles = (int)std::min<int64_t>(nt_tiles, (int64_t)1 << 30);
    w.nwg = std::max(1, std::min(w.ntiles, SSM_MAX_WG));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += round_up(bytes, 256);
        return at;
    };
    w.off_vk = take(sizeof(float2) * (size_t)w.rows * MM);
    w.off_part = take(sizeof(double) * (size_t)w.nwg * PART);
    w.off_red = take(sizeof(double) * PART);
    w.off_C = take(sizeof(double) * MM * MM);
    w.total = o;
    return w;
}

}  // namespace

size_t ssm_bytes(int64_t n_vox, int n_t) { return ssm_layout(n_vox, n_t).total; }

int launch_ssm(const float* iq, int64_t n_vox, int n_t, const double* vecs, int n_modes, char* ws, double* C,
               int* k_out, hipStream_t s) {
    const SsmWs L = ssm_layout(n_vox, n_t);
    float2* vk = reinterpret_cast<float2*>(ws + L.off_vk);
    double* part = reinterpret_cast<double*>(ws + L.off_part);
    double* red = reinterpret_cast<double*>(ws + L.off_red);
    if (!C) C = reinterpret_cast<double*>(ws + L.off_C);

    VkArgs va{reinterpret_cast<const double2*>(vecs), vk, n_t, L.rows, n_modes};
    hipLaunchKernelGGL(ssm_vk_kernel, dim3((L.rows * MM + 255) / 256), dim3(256), 0, s, va);
    FQ_LAUNCH_CHECK();
    TileArgs ta{reinterpret_cast<const float2*>(iq), vk, part, n_vox, n_t, L.n_chunks, L.ntiles, L.nwg};
    hipLaunchKernelGGL(ssm_tile_kernel, dim3(L.nwg), dim3(SSM_THREADS), 0, s, ta);
    FQ_LAUNCH_CHECK();
    RedArgs ra{part, red, L.nwg};
    hipLaunchKernelGGL(ssm_reduce_kernel, dim3((PART + 255) / 256), dim3(256), 0, s, ra);
    FQ_LAUNCH_CHECK();
    CorrArgs ca{red, C, k_out, 1.0 / (double)n_vox, n_modes};
    hipLaunchKernelGGL(ssm_corr_kernel, dim3(1), dim3(256), 0, s, ca);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

}  // namespace fq

using namespace fq;

extern "C" size_t ssm_workspace_size(int64_t n_vox, int32_t n_t) {
    if (n_vox < 1 || n_t < 1) return 0;
    return ssm_bytes(n_vox, n_t);
}

extern "C" int spatial_similarity(const float* iq, int64_t n_vox, int32_t n_t, const double* vecs, int32_t n_modes,
                                  void* ws, size_t ws_bytes, double* ssm, int32_t* k_tissue, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(n_modes >= 2 && n_modes <= n_t && n_modes <= FQ_SSM_MAX_MODES, "n_modes must be 2..min(n_t, %d)",
               FQ_SSM_MAX_MODES);
    FQ_REQUIRE(iq && vecs && ws && ssm && aligned16(iq) && aligned16(vecs) && aligned16(ws),
               "null or misaligned pointer");
    const size_t need = ssm_bytes(n_vox, n_t);
    if (ws_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, need);
        return FQ_E_WORKSPACE;
    }
    return launch_ssm(iq, n_vox, n_t, vecs, n_modes, reinterpret_cast<char*>(ws), ssm, k_tissue, as_stream(stream));
}
