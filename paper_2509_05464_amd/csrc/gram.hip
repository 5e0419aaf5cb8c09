// casorati_gram: G = S^H S of the Casorati matrix on the gfx950 matrix cores.
//
// With S = A + iB (voxels x frames), Re G = A^T A + B^T B and Im G = A^T B - B^T A.
// G is Hermitian, so only the 32x32 frame tiles (I, J) with I <= J are formed.  One
// workgroup owns one tile and one voxel range (split over the contraction dimension);
// its four waves form the four real products Re.Re, Im.Im, Re.Im and Im.Re of the tile
// with MFMA, reading 64-voxel slices of the 64 frames involved from LDS.
//   FP32 mode       : v_mfma_f32_32x32x2_f32.
//   split-BF16 mode : x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
//                     even); three v_mfma_f32_32x32x16_bf16 products hi.hi + hi.lo + lo.hi.
//   split-BF16 x4   : hi.hi + hi.lo + lo.hi + lo.lo.  The three-product form drops
//                     sum_v lo lo^H, a positive semi-definite term of about 2^-18 of the
//                     Gram's trace that biases every eigenvalue below that level; the
//                     fourth product removes it.
//   BF16 mode       : hi.hi only (negative control).
// Accumulation is FP32 inside each 64-voxel stage and FP64 across stages (a long FP32
// running sum of same-sign terms grows its rounding error with the sum; short blocks
// keep the Gram exact to ~1e-8 of lambda_1, which the clutter subspace near the cutoff
// needs); the partial tiles of all voxel ranges are then summed in FP64 in a fixed
// order (deterministic).
// Workgroups that share a voxel range are placed on the same XCD so the range is read
// from HBM once and served to the other tiles from that XCD's L2.
#include "fq_common.hpp"

namespace fq {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

constexpr int GT = 32;            // tile edge, frames
constexpr int KC = 64;            // voxels per LDS stage
constexpr int LDW = KC + 4;       // LDS row stride (floats)
constexpr int FLUSH = 1;          // stages per FP32 accumulation block (64 voxels)
constexpr int GRAM_THREADS = 256;
constexpr int NXCD = 8;

struct GramArgs {
    const float2* iq;     // [nt][nv]
    double* part;         // [nsplit][ntiles][4][GT*GT]
    int64_t nv;
    int64_t chunk;        // voxels per split
    int nt, nb, ntiles, nsplit;
};

__device__ __forceinline__ void tile_ij(int t, int nb, int& I, int& J) {
    int i = 0;
    while (t >= nb - i) {
        t -= nb - i;
        ++i;
    }
    I = i;
    J = i + t;
}

__device__ __forceinline__ unsigned short bf16_rne_bits(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }

template <int MODE>
__global__ void __launch_bounds__(GRAM_THREADS) gram_kernel(const GramArgs a) {
    __shared__ float sRe[2 * GT * LDW];
    __shared__ float sIm[2 * GT * LDW];

    // XCD-aware decode: workgroups id, id+8, ... run on one XCD; give them one voxel range.
    const int id = blockIdx.x;
    const int xcd = id % NXCD, loc = id / NXCD;
    const int t = loc % a.ntiles;
    const int split = (loc / a.ntiles) * NXCD + xcd;
    if (split >= a.nsplit) return;
    int I, J;
    tile_ij(t, a.nb, I, J);
    const int64_t v_begin = (int64_t)split * a.chunk;
    const int64_t v_end = min(a.nv, v_begin + a.chunk);

    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const float* X = (w == 0 || w == 2) ? sRe : sIm;          // rows of block I
    const float* Y = ((w == 0 || w == 3) ? sRe : sIm) + GT * LDW;   // rows of block J

    floatx16 acc;
    double acc64[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc[r] = 0.0f;
        acc64[r] = 0.0;
    }

    // loader mapping: 64 rows x 64 voxels; thread -> (row, 16-voxel quarter)
    const int lrow = threadIdx.x / 4, lq = threadIdx.x % 4;
    const int frame = lrow < GT ? I * GT + lrow : J * GT + (lrow - GT);
    const float4* src = reinterpret_cast<const float4*>(a.iq + (int64_t)frame * a.nv);

    int stage = 0;
    for (int64_t v0 = v_begin; v0 < v_end; v0 += KC, ++stage) {
        __syncthreads();
        {
            float re[16], im[16];
            const int64_t vb = v0 + lq * 16;
            if (frame < a.nt && vb + 16 <= v_end && (a.nv % 2) == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 p = src[(vb >> 1) + q];
                    re[2 * q] = p.x;
                    im[2 * q] = p.y;
                    re[2 * q + 1] = p.z;
                    im[2 * q + 1] = p.w;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    float2 p = make_float2(0.f, 0.f);
                    if (frame < a.nt && vb + q < v_end) p = a.iq[(int64_t)frame * a.nv + vb + q];
                    re[q] = p.x;
                    im[q] = p.y;
                }
            }
            float* dr = sRe + lrow * LDW + lq * 16;
            float* di = sIm + lrow * LDW + lq * 16;
#pragma unroll
            for (int q = 0; q < 16; q += 4) {
                *reinterpret_cast<float4*>(dr + q) = make_float4(re[q], re[q + 1], re[q + 2], re[q + 3]);
                *reinterpret_cast<float4*>(di + q) = make_float4(im[q], im[q + 1], im[q + 2], im[q + 3]);
            }
        }
        __syncthreads();
        const int i = l % 32, h = l / 32;
        if (MODE == FQ_GRAM_FP32) {
#pragma unroll
            for (int kk = 0; kk < KC; kk += 2) {
                const float av = X[i * LDW + kk + h];
                const float bv = Y[i * LDW + kk + h];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < KC; kk += 16) {
                const float4* xp = reinterpret_cast<const float4*>(X + i * LDW + kk + h * 8);
                const float4* yp = reinterpret_cast<const float4*>(Y + i * LDW + kk + h * 8);
                const float4 x0 = xp[0], x1 = xp[1], y0 = yp[0], y1 = yp[1];
                const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                const float ys[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
                ushortx8 xh, xl, yh, yl;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    xh[q] = bf16_rne_bits(xs[q]);
                    yh[q] = bf16_rne_bits(ys[q]);
                    xl[q] = bf16_rne_bits(xs[q] - bf16_to_f32(xh[q]));
                    yl[q] = bf16_rne_bits(ys[q] - bf16_to_f32(yh[q]));
                }
                const bf16x8 XH = __builtin_bit_cast(bf16x8, xh), YH = __builtin_bit_cast(bf16x8, yh);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XH, YH, acc, 0, 0, 0);
                if (MODE == FQ_GRAM_SPLIT_BF16 || MODE == FQ_GRAM_SPLIT4_BF16) {
                    const bf16x8 XL = __builtin_bit_cast(bf16x8, xl), YL = __builtin_bit_cast(bf16x8, yl);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XH, YL, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XL, YH, acc, 0, 0, 0);
                    if (MODE == FQ_GRAM_SPLIT4_BF16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XL, YL, acc, 0, 0, 0);
                }
            }
        }
        if ((stage + 1) % FLUSH == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc64[r] += (double)acc[r];
                acc[r] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc64[r] += (double)acc[r];

    // 32x32 accumulator layout: lane l holds column l%32, rows 8*(r/4) + 4*(l/32) + r%4
    double* out = a.part + (((int64_t)split * a.ntiles + t) * 4 + w) * (GT * GT);
    const int col = l % 32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * (l / 32) + (r % 4);
        out[row * GT + col] = acc64[r];
    }
}

struct ReduceArgs {
    const double* part;
    double2* gram;        // [nt][nt]
    int nt, nb, ntiles, nsplit;
};

__global__ void gram_reduce_kernel(const ReduceArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.nt * a.nt) return;
    const int f = idx / a.nt, g = idx % a.nt;
    const int lo = min(f, g), hi = max(f, g);
    const int I = lo / GT, J = hi / GT;
    // tile index of (I, J) in the row-major upper triangle
    const int t = I * a.nb - I * (I - 1) / 2 + (J - I);
    const int i = lo % GT, j = hi % GT;
    double rr = 0, ii = 0, ri = 0, ir = 0;
    for (int s = 0; s < a.nsplit; ++s) {
        const double* p = a.part + ((int64_t)s * a.ntiles + t) * 4 * GT * GT + i * GT + j;
        rr += p[0];
        ii += p[GT * GT];
        ri += p[2 * GT * GT];
        ir += p[3 * GT * GT];
    }
    double re = rr + ii, im = ri - ir;
    if (f == g) im = 0.0;
    if (f > g) im = -im;
    a.gram[idx] = make_double2(re, im);
}

struct Plan {
    int nb, ntiles, nsplit;
    int64_t chunk;
    size_t bytes;
};

Plan plan(int64_t nv, int nt) {
    Plan p{};
    p.nb = (nt + GT - 1) / GT;
    p.ntiles = p.nb * (p.nb + 1) / 2;
    // about 2048 workgroups; voxel ranges are whole multiples of the 4096-voxel block
    int64_t want = std::max<int64_t>(1, 2048 / p.ntiles);
    int64_t chunk = (nv + want - 1) / want;
    chunk = std::max<int64_t>(4096, round_up((size_t)chunk, 4096));
    int64_t ns = (nv + chunk - 1) / chunk;
    p.nsplit = (int)round_up((size_t)ns, NXCD);
    p.chunk = chunk;
    p.bytes = (size_t)p.nsplit * p.ntiles * 4 * GT * GT * sizeof(double);
    return p;
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t gram_workspace_size(int64_t n_vox, int32_t n_t, int32_t gram_mode) {
    (void)gram_mode;
    if (n_vox < 1 || n_t < 1) return 0;
    return plan(n_vox, n_t).bytes;
}

extern "C" int casorati_gram(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, void* ws, size_t ws_bytes,
                             double* gram, void* stream) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(gram_mode == FQ_GRAM_FP32 || gram_mode == FQ_GRAM_SPLIT_BF16 || gram_mode == FQ_GRAM_BF16 ||
                   gram_mode == FQ_GRAM_SPLIT4_BF16,
               "bad gram_mode");
    FQ_REQUIRE(iq && gram && ws && aligned16(iq) && aligned16(gram) && aligned16(ws), "null or misaligned pointer");
    const Plan p = plan(n_vox, n_t);
    if (ws_bytes < p.bytes) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, p.bytes);
        return FQ_E_WORKSPACE;
    }
    hipStream_t s = as_stream(stream);
    GramArgs ga{};
    ga.iq = reinterpret_cast<const float2*>(iq);
    ga.part = reinterpret_cast<double*>(ws);
    ga.nv = n_vox;
    ga.chunk = p.chunk;
    ga.nt = n_t;
    ga.nb = p.nb;
    ga.ntiles = p.ntiles;
    ga.nsplit = p.nsplit;
    const unsigned nwg = (unsigned)(p.ntiles * p.nsplit);
    switch (gram_mode) {
        case FQ_GRAM_FP32:
            hipLaunchKernelGGL(gram_kernel<FQ_GRAM_FP32>, dim3(nwg), dim3(GRAM_THREADS), 0, s, ga);
            break;
        case FQ_GRAM_SPLIT_BF16:
            hipLaunchKernelGGL(gram_kernel<FQ_GRAM_SPLIT_BF16>, dim3(nwg), dim3(GRAM_THREADS), 0, s, ga);
            break;
        case FQ_GRAM_SPLIT4_BF16:
            hipLaunchKernelGGL(gram_kernel<FQ_GRAM_SPLIT4_BF16>, dim3(nwg), dim3(GRAM_THREADS), 0, s, ga);
            break;
        default:
            hipLaunchKernelGGL(gram_kernel<FQ_GRAM_BF16>, dim3(nwg), dim3(GRAM_THREADS), 0, s, ga);
            break;
    }
    FQ_LAUNCH_CHECK();
    ReduceArgs ra{reinterpret_cast<const double*>(ws), reinterpret_cast<double2*>(gram), n_t, p.nb, p.ntiles,
                  p.nsplit};
    const int n2 = n_t * n_t;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((n2 + 255) / 256), dim3(256), 0, s, ra);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
