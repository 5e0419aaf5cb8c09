// casorati_gram: G = S^H S of the Casorati matrix on the gfx950 matrix cores.
//
// With S = A + iB (voxels x frames), Re G = A^T A + B^T B and Im G = A^T B - B^T A.
// G is Hermitian, so only the 32x32 frame tiles (I, J) with I <= J are formed.  A
// workgroup owns a 2x2 group of tiles (64 frames of I-blocks by 64 frames of J-blocks)
// and one voxel range (split over the contraction dimension): each 64-voxel stage of the
// 128 frames involved (64 on the group's diagonal) is staged in LDS once, and each of
// the four waves forms the four real products Re.Re, Im.Im, Re.Im and Im.Re of its own
// tile with MFMA, so every staged value feeds two tiles' products.
//   FP32 mode       : v_mfma_f32_32x32x2_f32.
//   split-BF16 mode : x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
//                     even), split once when the stage is written to LDS; three
//                     v_mfma_f32_32x32x16_bf16 products hi.hi + hi.lo + lo.hi.
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
// from HBM once and served to the other groups from that XCD's L2.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "fq_common.hpp"

namespace fq {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int GT = 32;            // tile edge, frames
constexpr int GR = 2 * GT;        // LDS stage: 4 frame blocks (2 GR rows)
constexpr int GMAX = 34;          // tile groups at n_t = 512 (136 tiles, 4 per group)
constexpr int KC = 64;            // voxels per LDS stage
constexpr int LDW = KC + 4;       // FP32 LDS row stride (floats)
constexpr int LDB = KC + 8;       // BF16 LDS row stride (bf16 values; 144-byte rows)
constexpr int GRAM_THREADS = 256;
constexpr int NXCD = 8;

// A workgroup's four tiles (one per wavefront; 255 = none) and the at most four frame
// blocks they read (255 = none): the blocks fill the LDS stage's four 32-row slots.
struct GroupTab {
    unsigned char ij[GMAX][4][2];
    unsigned char blk[GMAX][4];
};

struct GramArgs {
    const float2* iq;     // [nt][nv]
    double* part;         // [nsplit][ntiles][2][GT*GT]: Re G, Im G partial tiles
    int64_t nv;
    int64_t chunk;        // voxels per split
    int nt, nb, ntiles, nsplit;
    int ngroups;          // tile groups
    GroupTab tab;
};

// hi/lo pair of 8 values packed as two 16-byte vectors of bf16 bit patterns, with the
// hardware pair conversion (round to nearest even): hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split8(const float* x, uint4& hi, uint4& lo) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    unsigned int h[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x2 hv = {(__bf16)x[2 * q], (__bf16)x[2 * q + 1]};
        h[q] = __builtin_bit_cast(unsigned int, hv);
        const bf16x2 lv = {(__bf16)(x[2 * q] - __uint_as_float(h[q] << 16)),
                           (__bf16)(x[2 * q + 1] - __uint_as_float(h[q] & 0xffff0000u))};
        l[q] = __builtin_bit_cast(unsigned int, lv);
    }
    hi = make_uint4(h[0], h[1], h[2], h[3]);
    lo = make_uint4(l[0], l[1], l[2], l[3]);
}

// flip the sign bits of 8 packed bf16 values
__device__ __forceinline__ uint4 neg8(uint4 x) {
    return make_uint4(x.x ^ 0x80008000u, x.y ^ 0x80008000u, x.z ^ 0x80008000u, x.w ^ 0x80008000u);
}

template <int MODE>
__global__ void __launch_bounds__(GRAM_THREADS, 2) gram_kernel(const GramArgs a) {
    constexpr bool SPLIT = MODE != FQ_GRAM_FP32;
    // FP32: planes Re, Im of [2 GR][LDW] floats; BF16: planes Re.hi, Re.lo, Im.hi, Im.lo of [2 GR][LDB]
    constexpr int PLANE = SPLIT ? 2 * GR * LDB * 2 : 2 * GR * LDW * 4;   // bytes
    constexpr int NPLANE = SPLIT ? 4 : 2;
    __shared__ __align__(16) unsigned char lds[NPLANE * PLANE];

    // XCD-aware decode: workgroups id, id+8, ... run on one XCD; give them one voxel range.
    const int id = blockIdx.x;
    const int xcd = id % NXCD, loc = id / NXCD;
    const int grp = loc % a.ngroups;
    const int split = (loc / a.ngroups) * NXCD + xcd;
    if (split >= a.nsplit) return;
    const int64_t v_begin = (int64_t)split * a.chunk;
    const int64_t v_end = min(a.nv, v_begin + a.chunk);

    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int I = a.tab.ij[grp][w][0], J = a.tab.ij[grp][w][1];
    const bool active = I != 255;
    int xrow = 0, yrow = 0;   // stage rows of blocks I and J
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
        if (a.tab.blk[grp][sl] == I) xrow = sl * GT;
        if (a.tab.blk[grp][sl] == J) yrow = sl * GT;
    }

    // Re G = Re.Re + Im.Im and Im G = Re.Im - Im.Re accumulate directly (the second term of
    // Im G through a negated operand): FP32 within a stage, FP64 across stages
    floatx16 acc_re, acc_im;
    double sum_re[16], sum_im[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc_re[r] = acc_im[r] = 0.0f;
        sum_re[r] = sum_im[r] = 0.0;
    }

    // loader mapping: up to 128 rows x 64 voxels; thread -> (row, 32-voxel half).  The next
    // stage is loaded into registers while the current one is multiplied.
    const int lrow = threadIdx.x >> 1, lh = threadIdx.x & 1;
    const int lblk = a.tab.blk[grp][lrow / GT];
    const bool lact = lblk != 255;
    const int frame = lblk * GT + lrow % GT;
    const bool fvalid = lact && frame < a.nt;
    const float2* srow = a.iq + (int64_t)(fvalid ? frame : 0) * a.nv;
    float re[32], im[32];
    auto load = [&](int64_t v0) {
        const int64_t vb = v0 + lh * 32;
        if (fvalid && vb + 32 <= v_end && (a.nv % 2) == 0) {
            const float4* src = reinterpret_cast<const float4*>(srow + vb);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float4 p = src[q];
                re[2 * q] = p.x;
                im[2 * q] = p.y;
                re[2 * q + 1] = p.z;
                im[2 * q + 1] = p.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                float2 p = make_float2(0.f, 0.f);
                if (fvalid && vb + q < v_end) p = srow[vb + q];
                re[q] = p.x;
                im[q] = p.y;
            }
        }
    };
    if (lact && v_begin < v_end) load(v_begin);

    const int i = l % 32, h = l / 32;
    for (int64_t v0 = v_begin; v0 < v_end; v0 += KC) {
        __syncthreads();
        if (lact) {
            if (!SPLIT) {
                float* dr = reinterpret_cast<float*>(lds) + lrow * LDW + lh * 32;
                float* di = reinterpret_cast<float*>(lds + PLANE) + lrow * LDW + lh * 32;
#pragma unroll
                for (int q = 0; q < 32; q += 4) {
                    *reinterpret_cast<float4*>(dr + q) = make_float4(re[q], re[q + 1], re[q + 2], re[q + 3]);
                    *reinterpret_cast<float4*>(di + q) = make_float4(im[q], im[q + 1], im[q + 2], im[q + 3]);
                }
            } else {
                const int off = (lrow * LDB + lh * 32) * 2;   // bytes
#pragma unroll
                for (int q = 0; q < 32; q += 8) {
                    uint4 hi, lo;
                    split8(re + q, hi, lo);
                    *reinterpret_cast<uint4*>(lds + 0 * PLANE + off + q * 2) = hi;
                    *reinterpret_cast<uint4*>(lds + 1 * PLANE + off + q * 2) = lo;
                    split8(im + q, hi, lo);
                    *reinterpret_cast<uint4*>(lds + 2 * PLANE + off + q * 2) = hi;
                    *reinterpret_cast<uint4*>(lds + 3 * PLANE + off + q * 2) = lo;
                }
            }
        }
        __syncthreads();
        if (lact && v0 + KC < v_end) load(v0 + KC);
        if (!active) continue;
        if (!SPLIT) {
            const float* Re = reinterpret_cast<const float*>(lds);
            const float* Im = reinterpret_cast<const float*>(lds + PLANE);
            const int xo = (xrow + i) * LDW + h, yo = (yrow + i) * LDW + h;
#pragma unroll
            for (int kk = 0; kk < KC; kk += 2) {
                const float xr = Re[xo + kk], xi = Im[xo + kk], yr = Re[yo + kk], yi = Im[yo + kk];
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(xr, yr, acc_re, 0, 0, 0);
                acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(xi, yi, acc_re, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(xr, yi, acc_im, 0, 0, 0);
                acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(-xi, yr, acc_im, 0, 0, 0);
            }
        } else {
            const int xo = ((xrow + i) * LDB + h * 8) * 2, yo = ((yrow + i) * LDB + h * 8) * 2;   // bytes
#pragma unroll
            for (int kk = 0; kk < KC; kk += 16) {
                const int k2 = kk * 2;
                const uint4 xrh = *reinterpret_cast<const uint4*>(lds + 0 * PLANE + xo + k2);
                const uint4 xrl = *reinterpret_cast<const uint4*>(lds + 1 * PLANE + xo + k2);
                const uint4 xih = *reinterpret_cast<const uint4*>(lds + 2 * PLANE + xo + k2);
                const uint4 xil = *reinterpret_cast<const uint4*>(lds + 3 * PLANE + xo + k2);
                const uint4 yrh = *reinterpret_cast<const uint4*>(lds + 0 * PLANE + yo + k2);
                const uint4 yrl = *reinterpret_cast<const uint4*>(lds + 1 * PLANE + yo + k2);
                const uint4 yih = *reinterpret_cast<const uint4*>(lds + 2 * PLANE + yo + k2);
                const uint4 yil = *reinterpret_cast<const uint4*>(lds + 3 * PLANE + yo + k2);
                // (x, y) operand pairs: Re.Re and Im.Im into Re G; Re.Im and (-Im).Re into Im G
                const uint4 XH[4] = {xrh, xih, xrh, neg8(xih)}, XL[4] = {xrl, xil, xrl, neg8(xil)};
                const uint4 YH[4] = {yrh, yih, yih, yrh}, YL[4] = {yrl, yil, yil, yrl};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    floatx16& acc = p < 2 ? acc_re : acc_im;
                    const bf16x8 xh = __builtin_bit_cast(bf16x8, XH[p]), yh = __builtin_bit_cast(bf16x8, YH[p]);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yh, acc, 0, 0, 0);
                    if (MODE == FQ_GRAM_SPLIT_BF16 || MODE == FQ_GRAM_SPLIT4_BF16) {
                        const bf16x8 xl = __builtin_bit_cast(bf16x8, XL[p]), yl = __builtin_bit_cast(bf16x8, YL[p]);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl, yh, acc, 0, 0, 0);
                        if (MODE == FQ_GRAM_SPLIT4_BF16) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl, yl, acc, 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            sum_re[r] += (double)acc_re[r];
            sum_im[r] += (double)acc_im[r];
            acc_re[r] = acc_im[r] = 0.0f;
        }
    }
    if (!active) return;

    // 32x32 accumulator layout: lane l holds column l%32, rows 8*(r/4) + 4*(l/32) + r%4
    const int t = I * a.nb - I * (I - 1) / 2 + (J - I);
    const int col = l % 32;
    double* out = a.part + ((int64_t)split * a.ntiles + t) * 2 * (GT * GT);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * (l / 32) + (r % 4);
        out[row * GT + col] = sum_re[r];
        out[GT * GT + row * GT + col] = sum_im[r];
    }
}

struct ReduceArgs {
    const double* part;
    double2* gram;        // [nt][nt]
    int nt, nb, ntiles, nsplit;
};

// One thread per element of the partial tiles and per eighth of the voxel ranges (consecutive
// threads read consecutive words of each range's tiles); the eight part sums are added in a
// fixed order (deterministic).  Tile element (i, j) of tile (I, J) is G[f][g], f = 32 I + i,
// g = 32 J + j; elements with f < g are written with their mirror conj(G[f][g]) at G[g][f], the
// diagonal with a zero imaginary part, and the lower half of the diagonal tiles is not read.
constexpr int RED_GROUPS = 8;
__global__ void __launch_bounds__(256) gram_reduce_kernel(const ReduceArgs a) {
    __shared__ double sums[RED_GROUPS][32];
    const int le = threadIdx.x % 32, rg = threadIdx.x / 32;
    const int64_t per_split = (int64_t)a.ntiles * 2 * GT * GT;
    const int64_t e = (int64_t)blockIdx.x * 32 + le;
    double acc = 0.0;
    if (e < per_split)
        for (int sp = rg; sp < a.nsplit; sp += RED_GROUPS) acc += a.part[(int64_t)sp * per_split + e];
    sums[rg][le] = acc;
    __syncthreads();
    if (rg != 0 || e >= per_split) return;
    double tot = sums[0][le];
#pragma unroll
    for (int q = 1; q < RED_GROUPS; ++q) tot += sums[q][le];
    int t = (int)(e / (2 * GT * GT));
    const int rem = (int)(e % (2 * GT * GT));
    const int c = rem / (GT * GT), i = (rem % (GT * GT)) / GT, j = rem % GT;
    int I = 0;
    while (t >= a.nb - I) {   // tile t of the row-major upper triangle -> (I, J)
        t -= a.nb - I;
        ++I;
    }
    const int J = I + t;
    const int f = I * GT + i, g = J * GT + j;
    if (f >= a.nt || g >= a.nt || f > g) return;
    double* G = reinterpret_cast<double*>(a.gram);   // [nt][nt] x (Re, Im)
    if (f == g) {
        G[((int64_t)f * a.nt + g) * 2 + c] = c ? 0.0 : tot;
        return;
    }
    G[((int64_t)f * a.nt + g) * 2 + c] = tot;
    G[((int64_t)g * a.nt + f) * 2 + c] = c ? -tot : tot;
}

struct Plan {
    int nb, ntiles, ngroups, nsplit;
    int64_t chunk;
    size_t bytes;
    GroupTab tab;
};

// Tiles (I <= J) into groups of four that read at most four frame blocks: first every full
// 2x2 block of tiles off the diagonal between the block pairs (2a, 2a+1) and (2b, 2b+1), then
// the remaining tiles in row-major order, each group seeded with the first left and grown by
// the tile that adds the fewest new blocks.  This reaches ceil(ntiles / 4) groups for every
// nb <= 16 (a 2x2 tiling of the triangle needs up to 36% more, its diagonal and edge groups
// being partly empty).
void group_tiles(int nb, Plan& p) {
    std::memset(&p.tab, 255, sizeof(p.tab));
    std::vector<std::pair<int, int>> rest;
    std::vector<char> used(nb * nb, 0);
    int g = 0;
    auto put = [&](int gi, const std::vector<std::pair<int, int>>& ts) {
        int nbk = 0;
        for (size_t w = 0; w < ts.size(); ++w) {
            p.tab.ij[gi][w][0] = (unsigned char)ts[w].first;
            p.tab.ij[gi][w][1] = (unsigned char)ts[w].second;
            for (int x : {ts[w].first, ts[w].second}) {
                bool have = false;
                for (int k = 0; k < nbk; ++k) have |= p.tab.blk[gi][k] == x;
                if (!have) p.tab.blk[gi][nbk++] = (unsigned char)x;
            }
        }
    };
    for (int a2 = 0; a2 + 1 < nb; a2 += 2)
        for (int b2 = a2 + 2; b2 + 1 < nb; b2 += 2) {
            const std::vector<std::pair<int, int>> ts = {{a2, b2}, {a2, b2 + 1}, {a2 + 1, b2}, {a2 + 1, b2 + 1}};
            for (auto& t : ts) used[t.first * nb + t.second] = 1;
            put(g++, ts);
        }
    for (int I = 0; I < nb; ++I)
        for (int J = I; J < nb; ++J)
            if (!used[I * nb + J]) rest.push_back({I, J});
    while (!rest.empty()) {
        std::vector<std::pair<int, int>> ts = {rest.front()};
        rest.erase(rest.begin());
        std::vector<int> blocks = {ts[0].first};
        if (ts[0].second != ts[0].first) blocks.push_back(ts[0].second);
        while (ts.size() < 4) {
            int best = -1, best_add = 3;
            for (size_t c = 0; c < rest.size(); ++c) {
                int add = 0;
                for (int x : {rest[c].first, rest[c].second}) {
                    if (std::find(blocks.begin(), blocks.end(), x) == blocks.end()) ++add;
                }
                if (rest[c].first == rest[c].second && add == 2) add = 1;
                if ((int)blocks.size() + add <= 4 && add < best_add) {
                    best = (int)c;
                    best_add = add;
                }
            }
            if (best < 0) break;
            for (int x : {rest[best].first, rest[best].second})
                if (std::find(blocks.begin(), blocks.end(), x) == blocks.end()) blocks.push_back(x);
            ts.push_back(rest[best]);
            rest.erase(rest.begin() + best);
        }
        put(g++, ts);
    }
    p.ngroups = g;
}

Plan plan(int64_t nv, int nt, size_t max_bytes = 0) {
    Plan p{};
    p.nb = (nt + GT - 1) / GT;
    p.ntiles = p.nb * (p.nb + 1) / 2;
    group_tiles(p.nb, p);
    // about 16384 workgroups (short voxel ranges: the groups of one range stay close enough
    // in step to share its stages through the L2); ranges are whole multiples of 2048 voxels
    int64_t want = std::max<int64_t>(1, 16384 / p.ngroups);
    if (max_bytes) {
        // at most max_bytes of partial tiles: whole multiples of NXCD voxel ranges
        const size_t per_split = (size_t)p.ntiles * 2 * GT * GT * sizeof(double);
        const int64_t cap = (int64_t)(max_bytes / per_split) / NXCD * NXCD;
        want = std::max<int64_t>(1, std::min<int64_t>(want, cap));
    }
    int64_t chunk = (nv + want - 1) / want;
    chunk = std::max<int64_t>(2048, round_up((size_t)chunk, 2048));
    int64_t ns = (nv + chunk - 1) / chunk;
    p.nsplit = (int)round_up((size_t)ns, NXCD);
    p.chunk = chunk;
    p.bytes = (size_t)p.nsplit * p.ntiles * 2 * GT * GT * sizeof(double);
    return p;
}

}  // namespace
}  // namespace fq

// Partial tiles of casorati_gram_noalloc: a static device array (each GPU the library runs
// on holds its own copy until the process ends).  Host code never passes the symbol
// itself to a kernel: its device address is looked up once per device.
static __device__ __align__(256) unsigned char scratch[FQ_GRAM_SCRATCH_BYTES];

namespace fq {
namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mu;

int scratch_for_current_device(void** out) {
    int dev = -1;
    FQ_HIP(hipGetDevice(&dev));
    FQ_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        FQ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FQ_REQUIRE(ptr != nullptr, "no device address for the Gram scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FQ_OK;
}

int launch_gram(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, const Plan& p, void* ws,
                double* gram, hipStream_t s) {
    GramArgs ga{};
    ga.iq = reinterpret_cast<const float2*>(iq);
    ga.part = reinterpret_cast<double*>(ws);
    ga.nv = n_vox;
    ga.chunk = p.chunk;
    ga.nt = n_t;
    ga.nb = p.nb;
    ga.ntiles = p.ntiles;
    ga.nsplit = p.nsplit;
    ga.ngroups = p.ngroups;
    ga.tab = p.tab;
    const unsigned nwg = (unsigned)(p.ngroups * p.nsplit);
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
    const int64_t per_split = (int64_t)p.ntiles * 2 * GT * GT;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((per_split + 31) / 32)), dim3(256), 0, s, ra);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

int check_gram_args(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, double* gram) {
    FQ_REQUIRE(n_t >= 1 && n_t <= FQ_MAX_NT, "n_t must be 1..%d", FQ_MAX_NT);
    FQ_REQUIRE(n_vox >= 1, "n_vox must be >= 1");
    FQ_REQUIRE(gram_mode == FQ_GRAM_FP32 || gram_mode == FQ_GRAM_SPLIT_BF16 || gram_mode == FQ_GRAM_BF16 ||
                   gram_mode == FQ_GRAM_SPLIT4_BF16,
               "bad gram_mode");
    FQ_REQUIRE(iq && gram && aligned16(iq) && aligned16(gram), "null or misaligned pointer");
    return FQ_OK;
}
}  // namespace
}  // namespace fq

using namespace fq;

extern "C" int casorati_gram_noalloc(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, double* gram,
                                     void* stream) {
    int st = check_gram_args(iq, n_vox, n_t, gram_mode, gram);
    if (st != FQ_OK) return st;
    const Plan p = plan(n_vox, n_t, FQ_GRAM_SCRATCH_BYTES);
    if (p.bytes > FQ_GRAM_SCRATCH_BYTES) {
        set_error("n_t = %d needs %zu bytes of partial tiles, above the %zu-byte static scratch", n_t, p.bytes,
                  (size_t)FQ_GRAM_SCRATCH_BYTES);
        return FQ_E_INVALID;
    }
    void* ws = nullptr;
    if ((st = scratch_for_current_device(&ws)) != FQ_OK) return st;
    return launch_gram(iq, n_vox, n_t, gram_mode, p, ws, gram, as_stream(stream));
}

extern "C" size_t gram_workspace_size(int64_t n_vox, int32_t n_t, int32_t gram_mode) {
    (void)gram_mode;
    if (n_vox < 1 || n_t < 1) return 0;
    return plan(n_vox, n_t).bytes;
}

extern "C" int casorati_gram(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, void* ws, size_t ws_bytes,
                             double* gram, void* stream) {
    int st = check_gram_args(iq, n_vox, n_t, gram_mode, gram);
    if (st != FQ_OK) return st;
    FQ_REQUIRE(ws && aligned16(ws), "null or misaligned workspace");
    const Plan p = plan(n_vox, n_t);
    if (ws_bytes < p.bytes) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, p.bytes);
        return FQ_E_WORKSPACE;
    }
    return launch_gram(iq, n_vox, n_t, gram_mode, p, ws, gram, as_stream(stream));
}
