// Learned slow-time clutter filter on gfx950: BF16 matrix-core training and inference.
//
// Network (per voxel series, T frames): x = [Re, Im](s)/r, r = sqrt(mean |s|^2 + eps),
//   h1 = GELU(conv9(x; W1[32][2][9]) + b1), h2 = GELU(conv9(h1; W2) + b2),
//   h3 = GELU(conv9(h2; W3) + b3),          y  = W4[2][32] h3 + b4,
// blood estimate r (y0 + i y1).  conv9 has "same" zero padding (taps t-4..t+4).
//
// Each 32->32 conv is an implicit GEMM on v_mfma_f32_32x32x16_bf16:
//   C[o][t] = sum_kk A[o][kk] B[kk][t],  kk = k*32 + i (tap-major),
//   A = weights (held in registers as MFMA fragments for the whole kernel),
//   B[kk][t] = h[t + k - 4][i] read from a time-major LDS image h[row][32 channels]
//   (row = t + 4): the 8 consecutive kk a lane supplies are 8 consecutive channels of
//   one row, one 16-byte LDS read.  The 2-channel input layer uses an 8-channel image
//   (kk = k*8 + i, channels 2..7 zero).  Output C tiles are 32 channels x 32 frames.
// Backward: dgrad is the same conv on dz with the transposed, time-flipped kernel
// (A[i][k'*32+o] = W[o][i][8-k']); wgrad reduces over time,
//   dW[o][i][k] = sum_t dz[t][o] h[t+k-4][i],
// with K = time: its operands are gathered from the time-major images.
// Rounding points (round to nearest even): weights (BF16 copy kept by Adam), the
// network input, every stored activation (z and h of layers 1-3) and every dz; all
// accumulation, biases, GELU and the output layer are FP32.
#include "fq_common.hpp"

namespace fq {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32, KW = 9, PADT = 4;
constexpr int OFF_W1 = 0, OFF_B1 = 576, OFF_W2 = 608, OFF_B2 = 9824, OFF_W3 = 9856, OFF_B3 = 19072,
              OFF_W4 = 19104, OFF_B4 = 19168, NPAR = 19170;
constexpr int K1C = 2;    // layer-1 K chunks: 9 taps x 2 channels = 18 -> 32
constexpr int K2C = 18;   // 32->32 K chunks: 9 taps x 32 channels = 288
constexpr int NWB = 256;  // waves of the backward reduction kernels
constexpr int PART = 9216 + 32;   // partial gradient of one 32->32 layer (W then b)
constexpr int PART1 = 576 + 32;   // partial gradient of layer 1
constexpr int PART4 = 64 + 2 + 1; // partial gradient of layer 4 + loss

__device__ __forceinline__ unsigned short f2bf(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }
// GELU in its tanh form (Hendrycks & Gimpel): GELU(z) = z (1 + tanh u)/2, u = C (z + A z^3),
// C = sqrt(2/pi), A = 0.044715.  With (1 + tanh u)/2 = 1/(1 + exp(-2u)) and exp(-2u) =
// 2^(z (K1 + K3 z^2)), K1 = -2 C log2 e, K3 = -2 C A log2 e: three multiply/FMAs, one
// exponential, one add, one reciprocal and a product (z -> -inf: 2^y overflows, the
// reciprocal gives 0 and GELU -0; z -> +inf: GELU = z).
constexpr float GELU_K1 = -2.3022081982f, GELU_K3 = -0.10294324f;
__device__ __forceinline__ float gelu_fwd(float z) {
    const float y = z * fmaf(GELU_K3, z * z, GELU_K1);
    return z * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f);
}
// two floats to BF16 (round to nearest even) with the hardware pair conversion
__device__ __forceinline__ unsigned int f2bf2(float lo, float hi) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(unsigned int, v);
}
// d GELU / dz = s + 2 C z s (1 - s) (1 + 3 A z^2), s = (1 + tanh u)/2
__device__ __forceinline__ float gelu_grad(float z) {
    const float z2 = z * z;
    const float s = 1.0f / (1.0f + exp2f(z * fmaf(GELU_K3, z2, GELU_K1)));
    return s + 1.5957691216f * z * s * (1.0f - s) * fmaf(0.134145f, z2, 1.0f);
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ floatx16 mfma(const u16x8& a, const u16x8& b, const floatx16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

struct Geo {
    int T, TT, TP;   // frames, 32-frame tiles, image rows (32*TT + 8)
    __device__ Geo(int t) : T(t), TT((t + 31) / 32), TP(32 * ((t + 31) / 32) + 8) {}
};

// per-series activation record (u16): h0 [T][2] hi terms, [T][2] lo terms (padded to 8) |
// z1 h1 z2 h2 z3 h3 [T][32]; every slot starts on a 16-byte boundary
__host__ __device__ inline int64_t h0_len(int T) { return ((int64_t)4 * T + 7) / 8 * 8; }
__host__ __device__ inline int64_t act_stride(int T) { return h0_len(T) + (int64_t)6 * T * CH; }
__host__ __device__ inline int64_t act_off(int which, int T) {   // 0:h0 1:z1 2:h1 3:z2 4:h2 5:z3 6:h3
    return which == 0 ? 0 : h0_len(T) + (int64_t)(which - 1) * T * CH;
}

// ---------------------------------------------------------------- fragment loads
__device__ void frag_fwd32(const uint16_t* wb, int base, int l, u16x8* fr) {
    const int o = l % 32, h = l / 32;
#pragma unroll
    for (int c = 0; c < K2C; ++c) {
        const int k = c / 2, i0 = (c % 2) * 16 + 8 * h;
#pragma unroll
        for (int q = 0; q < 8; ++q) fr[c][q] = wb[base + o * 288 + (i0 + q) * 9 + k];
    }
}
// dgrad: A[i][k'*32 + o] = W[o][i][8 - k']
__device__ void frag_dgrad32(const uint16_t* wb, int base, int l, u16x8* fr) {
    const int i = l % 32, h = l / 32;
#pragma unroll
    for (int c = 0; c < K2C; ++c) {
        const int kp = c / 2, o0 = (c % 2) * 16 + 8 * h;
#pragma unroll
        for (int q = 0; q < 8; ++q) fr[c][q] = wb[base + (o0 + q) * 288 + i * 9 + (8 - kp)];
    }
}

// one 32x32 output tile (channels x frames t0..t0+31) of a 32-channel image conv
__device__ __forceinline__ floatx16 conv32(const unsigned short* img, int t0, const u16x8* fr, int l) {
    const int j = l % 32, h = l / 32;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int c = 0; c < K2C; ++c) {
        const int k = c / 2, ch0 = (c % 2) * 16 + 8 * h;
        const u16x8 b = *reinterpret_cast<const u16x8*>(img + (t0 + j + k) * CH + ch0);
        acc = mfma(fr[c], b, acc);
    }
    return acc;
}
// 32x32 accumulator layout: lane l holds frame column l%32 and channel rows
// 8*(r/4) + 4*(l/32) + r%4, r = 0..15 (four groups of four consecutive channels).
__device__ __forceinline__ int acc_row(int r, int l) { return 8 * (r / 4) + 4 * (l / 32) + (r % 4); }

// ---------------------------------------------------------------- forward
struct FwdArgs {
    const float* w;
    const uint16_t* wb;
    const float2* x;      // [T][N]
    uint16_t* act;        // or null
    float2* y;            // [T][N] or null
    float* pd;            // [N] or null
    int64_t N;
    int T;
    float eps;
};

// An FP32 bias enters the products exactly as three BF16 terms (hi + mid + lo = b: each
// split leaves a remainder with 8 fewer significant bits), each times a B entry of 1.
__device__ __forceinline__ void split3(float b, unsigned short* o) {
    o[0] = f2bf(b);
    const float r1 = b - bf2f(o[0]);
    o[1] = f2bf(r1);
    o[2] = f2bf(r1 - bf2f(o[1]));
}
constexpr unsigned int BF_ONE2 = 0x3F803F80u;   // two BF16 ones
// Row stride (elements) of the forward pass's 32-channel image: 80 bytes, so the 16-byte
// reads of consecutive rows by consecutive lanes fall in distinct banks (a 64-byte stride
// puts every other row, or every fourth, on the same banks).
constexpr int RS = 40;

// input layer: kk = 2k + i (tap-major over the 2 input channels), 18 used of 32; the bias
// terms sit at kk = 18, 19, 20 (chunk 1, lanes h = 0, elements 2..4)
__device__ void frag_fwd1(const uint16_t* wb, const float* w, int l, u16x8* fr) {
    const int o = l % 32, h = l / 32;
#pragma unroll
    for (int c = 0; c < K1C; ++c) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kk = 16 * c + 8 * h + q, k = kk / 2, i = kk % 2;
            fr[c][q] = k < KW ? wb[OFF_W1 + o * 18 + i * 9 + k] : (unsigned short)0;
        }
    }
    unsigned short bs[3];
    split3(w[OFF_B1 + o], bs);
    if (h == 0) {
        fr[1][2] = bs[0];
        fr[1][3] = bs[1];
        fr[1][4] = bs[2];
    }
}
// bias chunk of a 32->32 layer (kk = 288..290, lanes h = 0)
__device__ u16x8 frag_bias(const float* w, int off, int l) {
    u16x8 fr;
#pragma unroll
    for (int q = 0; q < 8; ++q) fr[q] = 0;
    unsigned short bs[3];
    split3(w[off + l % 32], bs);
    if (l < 32) {
        fr[0] = bs[0];
        fr[1] = bs[1];
        fr[2] = bs[2];
    }
    return fr;
}
// output layer as a 32-row product (rows 0, 1 used) over the 32 channels of h3 in the
// order the layer-3 accumulator holds them: chunk c, element e is channel
// 8 (2c + e/4) + 4h + e%4
__device__ void frag_out(const uint16_t* wb, int l, u16x8* fr) {
    const int o = l % 32, h = l / 32;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int ch = 8 * (2 * c + e / 4) + 4 * h + e % 4;
            fr[c][e] = o < 2 ? wb[OFF_W4 + o * CH + ch] : (unsigned short)0;
        }
    }
}

// the input layer's conv: 2-channel image, 4 bytes per row; a lane's 8 consecutive kk are
// taps 8c + 4h .. 8c + 4h + 3 of both channels, 16 contiguous bytes (4-byte aligned)
// The input is two BF16 terms per value (hi = bf16(x), lo = bf16(x - hi)): the same
// weights multiply the hi image and the lo image.
__device__ __forceinline__ floatx16 conv2(const unsigned short* img, const unsigned short* img_lo, int t0,
                                         const u16x8* fr, int l) {
    const int j = l % 32, h = l / 32;
    const unsigned int* im = reinterpret_cast<const unsigned int*>(img);
    const unsigned int* il = reinterpret_cast<const unsigned int*>(img_lo);
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int c = 0; c < K1C; ++c) {
        const int row = t0 + j + 8 * c + 4 * h;
        uint4 w = make_uint4(im[row], im[row + 1], im[row + 2], im[row + 3]);
        uint4 wl = make_uint4(il[row], il[row + 1], il[row + 2], il[row + 3]);
        if (c == 1 && h == 0) {   // B = 1 against the bias terms, once
            w.y = w.z = BF_ONE2;
            wl.y = wl.z = 0u;
        }
        acc = mfma(fr[c], __builtin_bit_cast(u16x8, w), acc);
        acc = mfma(fr[c], __builtin_bit_cast(u16x8, wl), acc);
    }
    return acc;
}
// a 32->32 conv tile with its bias chunk
__device__ __forceinline__ floatx16 conv32b(const unsigned short* img, int t0, const u16x8* fr, const u16x8& fb,
                                           int l) {
    const int j = l % 32, h = l / 32;
    u16x8 one;
#pragma unroll
    for (int q = 0; q < 8; ++q) one[q] = q < 3 ? (unsigned short)0x3F80 : (unsigned short)0;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    acc = mfma(fb, one, acc);
#pragma unroll
    for (int c = 0; c < K2C; ++c) {
        const int k = c / 2, ch0 = (c % 2) * 16 + 8 * h;
        const u16x8 b = *reinterpret_cast<const u16x8*>(img + (t0 + j + k) * RS + ch0);
        acc = mfma(fr[c], b, acc);
    }
    return acc;
}

// GELU of one 32x32 output tile (this lane: frame t, channels 8q + 4h + p), rounded to
// BF16 (zero for frames past the end: they are the next layer's padding).  With an
// activation record, z and h of the layer are stored too.
template <bool ACT>
__device__ __forceinline__ void gelu_tile(const floatx16& acc, uint16_t* actv, int layer, int t, int T, int h,
                                          uint2* hv) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float z[4] = {acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
        hv[q] = t < T ? make_uint2(f2bf2(gelu_fwd(z[0]), gelu_fwd(z[1])), f2bf2(gelu_fwd(z[2]), gelu_fwd(z[3])))
                      : make_uint2(0u, 0u);
        if (ACT && actv) {
            const int o = 8 * q + 4 * h;
            *reinterpret_cast<uint2*>(actv + act_off(2 * layer - 1, T) + t * CH + o) =
                make_uint2(f2bf2(z[0], z[1]), f2bf2(z[2], z[3]));
            *reinterpret_cast<uint2*>(actv + act_off(2 * layer, T) + t * CH + o) = hv[q];
        }
    }
}

// Layers 1-3 are streamed over 32-frame tiles: step s computes layer 1 on tile s, layer 2
// on tile s-1 and layer 3 on tile s-2, so each layer's output only needs a ring of three
// tile slots.  A slot holds its tile's 32 rows between 4 halo rows on each side (the taps
// reach 4 frames into the neighbouring tiles): a tile's first 4 rows are also written into
// the after-halo of the previous tile's slot and its last 4 into the before-halo of the
// next one, so a tile's products read one contiguous 40-row window.  The halos outside the
// series (before tile 0, after the last tile) are cleared.
constexpr int SLOT = 40;   // rows per ring slot
constexpr int RING_ELEMS = 3 * SLOT * RS;

__device__ __forceinline__ void ring_store(unsigned short* ring, int s, int j, int h, const uint2* hv) {
    const int cur = s % 3, prev = (s + 2) % 3, next = (s + 1) % 3;
    unsigned short* body = ring + (cur * SLOT + 4 + j) * RS + 4 * h;
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2*>(body + 8 * q) = hv[q];
    if (j < 4) {
        unsigned short* p = ring + (prev * SLOT + 36 + j) * RS + 4 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2*>(p + 8 * q) = hv[q];
    } else if (j >= 28) {
        unsigned short* p = ring + (next * SLOT + j - 28) * RS + 4 * h;
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2*>(p + 8 * q) = hv[q];
    }
}
__device__ __forceinline__ void ring_clear(unsigned short* ring, int first_row, int l) {
    for (int i = l; i < 4 * RS / 4; i += 64) reinterpret_cast<uint2*>(ring + first_row * RS)[i] = make_uint2(0u, 0u);
}

// One wave per series at a time (grid-stride), two waves per SIMD: one wave's GELU
// epilogue overlaps the other's matrix products.  Every layer, biases and the output
// layer included, runs on the matrix cores; the weights stay in registers as MFMA
// fragments.  The next series' samples are fetched into registers (XR per lane, frames
// l, l+64, ...) while the current one is processed.
// Up to 256 frames (XR = 4) one image of the whole series serves layers 1 and 2 (about
// 20 KB, eight workgroups per CU); longer series stream the layers over tile rings, whose
// size does not grow with the series.
template <int XR, bool ACT>
__global__ void __launch_bounds__(64, 2) lcf_fwd_kernel(const FwdArgs a) {
    constexpr bool STREAM = XR > 4;
    extern __shared__ float4 smem4[];
    const Geo g(a.T);
    const int l = threadIdx.x;
    // streamed: ring of layer-1 tiles, ring of layer-2 tiles, input images (hi, lo) [TP+8][2]
    // whole:    input images (hi, lo) [TP+8][2], image [TP][RS] of layer 1, then layer 2 in place
    unsigned short* ra = reinterpret_cast<unsigned short*>(smem4);
    unsigned short* rb = ra + RING_ELEMS;
    unsigned short* h0 = STREAM ? rb + RING_ELEMS : ra;
    unsigned short* hl = h0 + (g.TP + 8) * 2;   // lo terms of the input, [TP+8][2]
    unsigned short* hb = hl + (g.TP + 8) * 2;

    u16x8 f1[K1C], f2[K2C], f3[K2C], f4[2];
    frag_fwd1(a.wb, a.w, l, f1);
    frag_fwd32(a.wb, OFF_W2, l, f2);
    frag_fwd32(a.wb, OFF_W3, l, f3);
    frag_out(a.wb, l, f4);
    const u16x8 fb2 = frag_bias(a.w, OFF_B2, l), fb3 = frag_bias(a.w, OFF_B3, l);
    const float b40 = a.w[OFF_B4], b41 = a.w[OFF_B4 + 1];
    for (int i = l; i < (g.TP + 8) * 4 + (STREAM ? 0 : g.TP * RS); i += 64) h0[i] = 0;   // padding rows stay zero
    __builtin_amdgcn_wave_barrier();

    const int h = l / 32, j = l % 32;
    const int last = (g.TT - 1) % 3;   // slot of the last tile
    float2 xn[XR];
    auto fetch = [&](int64_t v) {
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const int t = l + 64 * q;
            xn[q] = (v < a.N && t < g.T) ? a.x[(int64_t)t * a.N + v] : make_float2(0.f, 0.f);
        }
    };
    fetch(blockIdx.x);
    for (int64_t v = blockIdx.x; v < a.N; v += gridDim.x) {
        float2 xc[XR];
#pragma unroll
        for (int q = 0; q < XR; ++q) xc[q] = xn[q];
        fetch(v + gridDim.x);
        float ss = 0.0f;
#pragma unroll
        for (int q = 0; q < XR; ++q) ss += xc[q].x * xc[q].x + xc[q].y * xc[q].y;
        const float r = sqrtf(wave_sum(ss) / (float)g.T + a.eps);
        const float ir = 1.0f / r;
        uint16_t* actv = ACT ? a.act + v * act_stride(g.T) : nullptr;
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const int t = l + 64 * q;
            if (t < g.T) {
                const float xr = xc[q].x * ir, xi = xc[q].y * ir;
                const unsigned int p = f2bf2(xr, xi);
                const unsigned int pl = f2bf2(xr - __uint_as_float(p << 16), xi - __uint_as_float(p & 0xffff0000u));
                *reinterpret_cast<unsigned int*>(h0 + (t + PADT) * 2) = p;
                *reinterpret_cast<unsigned int*>(hl + (t + PADT) * 2) = pl;
                if (ACT) {
                    *reinterpret_cast<unsigned int*>(actv + act_off(0, g.T) + 2 * t) = p;
                    *reinterpret_cast<unsigned int*>(actv + act_off(0, g.T) + 2 * g.T + 2 * t) = pl;
                }
            }
        }
        float pdacc = 0.0f;
        // layer 3 and the output layer on tile u of the image img (rows of tile u start at
        // row 0): y = W4 h3 (rows 0 and 1 of a 32-row product whose B operand is h3 as this
        // lane holds it) + b4
        auto layer3 = [&](const unsigned short* img, int u) {
            const floatx16 acc = conv32b(img, 0, f3, fb3, l);
            const int t = 32 * u + j;
            uint2 hv[4];
            gelu_tile<ACT>(acc, t < g.T ? actv : nullptr, 3, t, g.T, h, hv);
            floatx16 yo;
#pragma unroll
            for (int i = 0; i < 16; ++i) yo[i] = 0.0f;
            yo = mfma(f4[0], __builtin_bit_cast(u16x8, make_uint4(hv[0].x, hv[0].y, hv[1].x, hv[1].y)), yo);
            yo = mfma(f4[1], __builtin_bit_cast(u16x8, make_uint4(hv[2].x, hv[2].y, hv[3].x, hv[3].y)), yo);
            if (h == 0 && t < g.T) {   // rows 0 and 1 of column j
                const float y0 = yo[0] + b40, y1 = yo[1] + b41;
                pdacc += y0 * y0 + y1 * y1;
                if (a.y) a.y[(int64_t)t * a.N + v] = make_float2(r * y0, r * y1);
            }
        };
        if (STREAM) {
            ring_clear(ra, 0, l);   // before tile 0
            ring_clear(rb, 0, l);
            __builtin_amdgcn_wave_barrier();
            for (int s = 0; s < g.TT + 2; ++s) {
                if (s < g.TT) {   // layer 1, tile s
                    const floatx16 acc = conv2(h0, hl, 32 * s, f1, l);
                    const int t = 32 * s + j;
                    uint2 hv[4];
                    gelu_tile<ACT>(acc, t < g.T ? actv : nullptr, 1, t, g.T, h, hv);
                    ring_store(ra, s, j, h, hv);
                } else if (s == g.TT) {
                    ring_clear(ra, last * SLOT + 36, l);   // after the last tile
                }
                if (s >= 1 && s <= g.TT) {   // layer 2, tile s - 1
                    const int u = s - 1;
                    const floatx16 acc = conv32b(ra + (u % 3) * SLOT * RS, 0, f2, fb2, l);
                    const int t = 32 * u + j;
                    uint2 hv[4];
                    gelu_tile<ACT>(acc, t < g.T ? actv : nullptr, 2, t, g.T, h, hv);
                    ring_store(rb, u, j, h, hv);
                } else if (s == g.TT + 1) {
                    ring_clear(rb, last * SLOT + 36, l);
                }
                if (s >= 2) layer3(rb + ((s - 2) % 3) * SLOT * RS, s - 2);
            }
        } else {
            __builtin_amdgcn_wave_barrier();
            // layer 1 -> hb; layer 2 -> hb in place: the output of a 32-frame tile is
            // stored only after the next tile's products have read their inputs (the taps
            // reach 4 frames into the neighbouring tiles)
            for (int tt = 0; tt < g.TT; ++tt) {
                const floatx16 acc = conv2(h0, hl, 32 * tt, f1, l);
                const int t = 32 * tt + j;
                uint2 hv[4];
                gelu_tile<ACT>(acc, t < g.T ? actv : nullptr, 1, t, g.T, h, hv);
#pragma unroll
                for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2*>(hb + (t + PADT) * RS + 8 * q + 4 * h) = hv[q];
            }
            __builtin_amdgcn_wave_barrier();
            uint2 pend[4];
            for (int tt = 0; tt < g.TT; ++tt) {
                const floatx16 acc = conv32b(hb, 32 * tt, f2, fb2, l);
                if (tt > 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<uint2*>(hb + (32 * tt - 32 + j + PADT) * RS + 8 * q + 4 * h) = pend[q];
                }
                const int t = 32 * tt + j;
                gelu_tile<ACT>(acc, t < g.T ? actv : nullptr, 2, t, g.T, h, pend);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint2*>(hb + (32 * g.TT - 32 + j + PADT) * RS + 8 * q + 4 * h) = pend[q];
            __builtin_amdgcn_wave_barrier();
            for (int tt = 0; tt < g.TT; ++tt) layer3(hb + 32 * tt * RS, tt);
        }
        pdacc = wave_sum(pdacc);
        if (a.pd && l == 0) a.pd[v] = r * r * pdacc / (float)g.T;
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- backward, per series
struct BwdArgs {
    const float* w;
    const uint16_t* wb;
    const float2* x;      // [T][N]
    const float2* tgt;    // [T][N]
    uint16_t* act;
    float* part4;         // [NWB][PART4]: dW4 (64), db4 (2), loss sum (1)
    int64_t N;
    int T;
    float eps;
    float inv_count;      // 1 / (N * 2 * T)
};

// Output-layer gradient, then dz of layers 3, 2, 1 through the transposed convs.
// Each dz overwrites the pre-activation z of its layer in the activation record
// (z is read for GELU' by the same lane immediately before).
__global__ void __launch_bounds__(64) lcf_bwd_series_kernel(const BwdArgs a) {
    extern __shared__ float4 smem4[];
    const Geo g(a.T);
    const int l = threadIdx.x, h = l / 32, j = l % 32;
    float* par = reinterpret_cast<float*>(smem4);      // w4 (64) b4 (2) pad -> 68
    float2* xs = reinterpret_cast<float2*>(par + 68);  // [T]
    float2* ts = xs + g.T;                              // [T]
    unsigned short* d3 = reinterpret_cast<unsigned short*>(ts + g.T);   // [TP][32]
    unsigned short* d2 = d3 + g.TP * CH;                                 // [TP][32]

    u16x8 fd3[K2C], fd2[K2C];
    frag_dgrad32(a.wb, OFF_W3, l, fd3);
    frag_dgrad32(a.wb, OFF_W2, l, fd2);
    for (int i = l; i < 68; i += 64) par[i] = i < 64 ? bf2f(a.wb[OFF_W4 + i]) : (i < 66 ? a.w[OFF_B4 + i - 64] : 0.f);
    for (int i = l; i < 2 * g.TP * CH; i += 64) d3[i] = 0;
    __builtin_amdgcn_wave_barrier();

    float dw4[2 * CH];
#pragma unroll
    for (int i = 0; i < 2 * CH; ++i) dw4[i] = 0.0f;
    float db40 = 0.0f, db41 = 0.0f, lossacc = 0.0f;

    for (int64_t v = blockIdx.x; v < a.N; v += gridDim.x) {
        for (int t = l; t < g.T; t += 64) {
            xs[t] = a.x[(int64_t)t * a.N + v];
            ts[t] = a.tgt[(int64_t)t * a.N + v];
        }
        __builtin_amdgcn_wave_barrier();
        float ss = 0.0f;
        for (int t = l; t < g.T; t += 64) ss += xs[t].x * xs[t].x + xs[t].y * xs[t].y;
        const float ir = 1.0f / sqrtf(wave_sum(ss) / (float)g.T + a.eps);
        uint16_t* av = a.act + v * act_stride(g.T);
        // output layer and dz3: one frame per lane
        for (int t = l; t < g.T; t += 64) {
            unsigned short* h3 = av + act_off(6, g.T) + t * CH;
            unsigned short* z3 = av + act_off(5, g.T) + t * CH;
            float hv[CH];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const u16x8 hh = *reinterpret_cast<const u16x8*>(h3 + 8 * q);
#pragma unroll
                for (int p = 0; p < 8; ++p) hv[8 * q + p] = bf2f(hh[p]);
            }
            float y0 = par[64], y1 = par[65];
#pragma unroll
            for (int o = 0; o < CH; ++o) {
                y0 = fmaf(par[o], hv[o], y0);
                y1 = fmaf(par[32 + o], hv[o], y1);
            }
            const float e0 = y0 - ts[t].x * ir, e1 = y1 - ts[t].y * ir;
            lossacc += e0 * e0 + e1 * e1;
            const float g0 = 2.0f * e0 * a.inv_count, g1 = 2.0f * e1 * a.inv_count;
            db40 += g0;
            db41 += g1;
#pragma unroll
            for (int o = 0; o < CH; ++o) {
                dw4[o] = fmaf(g0, hv[o], dw4[o]);
                dw4[CH + o] = fmaf(g1, hv[o], dw4[CH + o]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const u16x8 zz = *reinterpret_cast<const u16x8*>(z3 + 8 * q);
                u16x8 ob;
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const int o = 8 * q + p;
                    const float dh = par[o] * g0 + par[32 + o] * g1;
                    ob[p] = f2bf(dh * gelu_grad(bf2f(zz[p])));
                }
                *reinterpret_cast<u16x8*>(d3 + (t + PADT) * CH + 8 * q) = ob;
                *reinterpret_cast<u16x8*>(z3 + 8 * q) = ob;          // dz3 replaces z3
            }
        }
        __builtin_amdgcn_wave_barrier();
        // dgrad through layer 3: dz2 = conv(dz3; W3 transposed, flipped) * GELU'(z2)
        for (int tt = 0; tt < g.TT; ++tt) {
            const floatx16 acc = conv32(d3, 32 * tt, fd3, l);
            const int t = 32 * tt + j;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 8 * q + 4 * h;
                u16x4 ob = {0, 0, 0, 0};
                if (t < g.T) {
                    u16x4* zp = reinterpret_cast<u16x4*>(av + act_off(3, g.T) + t * CH + i);
                    const u16x4 z = *zp;
#pragma unroll
                    for (int p = 0; p < 4; ++p) ob[p] = f2bf(acc[4 * q + p] * gelu_grad(bf2f(z[p])));
                    *zp = ob;                                         // dz2 replaces z2
                }
                *reinterpret_cast<u16x4*>(d2 + (t + PADT) * CH + i) = ob;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // dgrad through layer 2: dz1 = conv(dz2; W2 transposed, flipped) * GELU'(z1)
        for (int tt = 0; tt < g.TT; ++tt) {
            const floatx16 acc = conv32(d2, 32 * tt, fd2, l);
            const int t = 32 * tt + j;
            if (t < g.T) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 8 * q + 4 * h;
                    u16x4* zp = reinterpret_cast<u16x4*>(av + act_off(1, g.T) + t * CH + i);
                    const u16x4 z = *zp;
                    u16x4 ob;
#pragma unroll
                    for (int p = 0; p < 4; ++p) ob[p] = f2bf(acc[4 * q + p] * gelu_grad(bf2f(z[p])));
                    *zp = ob;                                         // dz1 replaces z1
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // wave reduction of the output-layer partials
    float* out = a.part4 + (int64_t)blockIdx.x * PART4;
#pragma unroll
    for (int i = 0; i < 2 * CH; ++i) {
        const float s = wave_sum(dw4[i]);
        if (l == 0) out[i] = s;
    }
    db40 = wave_sum(db40);
    db41 = wave_sum(db41);
    lossacc = wave_sum(lossacc);
    if (l == 0) {
        out[64] = db40;
        out[65] = db41;
        out[66] = lossacc;
    }
}

// ---------------------------------------------------------------- weight gradients
struct WgArgs {
    const uint16_t* act;
    float* part;          // [NWB][PART] (layers 2, 3) or [NWB][PART1] (layer 1)
    int64_t N;
    int T;
    int layer;            // 1, 2 or 3
};

// dW[o][i][k] = sum_series sum_t dz[t][o] h_prev[t + k - 4][i], db[o] = sum dz[t][o]:
// a GEMM over K = time.  A[o][t] = dz (gathered from the time-major record), B[t][n] =
// h_prev shifted by the tap k of column block n.  Each wave accumulates over its series.
template <int LAYER>
__global__ void __launch_bounds__(64) lcf_wgrad_kernel(const WgArgs a) {
    extern __shared__ float4 smem4[];
    const Geo g(a.T);
    const int T16 = (a.T + 15) / 16 * 16;
    constexpr int HC = LAYER == 1 ? 2 : CH;            // channels of h_prev
    constexpr int NTILE = LAYER == 1 ? 1 : KW;
    const int l = threadIdx.x, h = l / 32, n = l % 32;
    unsigned short* dz = reinterpret_cast<unsigned short*>(smem4);   // [T16][32]
    unsigned short* hp = dz + T16 * CH;                              // [TP][HC]
    unsigned short* hq = hp + g.TP * HC;                             // layer 1: lo terms [TP][2]
    for (int i = l; i < T16 * CH + g.TP * HC * (LAYER == 1 ? 2 : 1); i += 64) dz[i] = 0;
    __builtin_amdgcn_wave_barrier();
    const int zslot = 2 * LAYER - 1;                          // dz_L sits in z_L's slot
    const int hslot = LAYER == 1 ? 0 : 2 * (LAYER - 1);       // h_{L-1}

    floatx16 acc[NTILE];
#pragma unroll
    for (int k = 0; k < NTILE; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.0f;
    float dbacc = 0.0f;

    for (int64_t v = blockIdx.x; v < a.N; v += gridDim.x) {
        const uint16_t* av = a.act + v * act_stride(g.T);
        for (int t = l; t < g.T; t += 64) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<u16x8*>(dz + t * CH + 8 * q) =
                    *reinterpret_cast<const u16x8*>(av + act_off(zslot, g.T) + t * CH + 8 * q);
            if (LAYER == 1) {
                hp[(t + PADT) * 2] = av[act_off(0, g.T) + 2 * t];
                hp[(t + PADT) * 2 + 1] = av[act_off(0, g.T) + 2 * t + 1];
                hq[(t + PADT) * 2] = av[act_off(0, g.T) + 2 * g.T + 2 * t];
                hq[(t + PADT) * 2 + 1] = av[act_off(0, g.T) + 2 * g.T + 2 * t + 1];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *reinterpret_cast<u16x8*>(hp + (t + PADT) * CH + 8 * q) =
                        *reinterpret_cast<const u16x8*>(av + act_off(hslot, g.T) + t * CH + 8 * q);
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int t0 = 0; t0 < T16; t0 += 16) {
            u16x8 A;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                A[q] = dz[(t0 + 8 * h + q) * CH + n];
                dbacc += bf2f(A[q]);
            }
#pragma unroll
            for (int k = 0; k < NTILE; ++k) {
                u16x8 B;
                if (LAYER == 1) {   // dz (hi + lo): the hi product here, the lo one below
                    const int kk = min(n / 2, KW - 1), ii = n % 2;
                    u16x8 Bl;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        B[q] = n < 18 ? hp[(t0 + 8 * h + q + kk) * 2 + ii] : (unsigned short)0;
                        Bl[q] = n < 18 ? hq[(t0 + 8 * h + q + kk) * 2 + ii] : (unsigned short)0;
                    }
                    acc[k] = mfma(A, Bl, acc[k]);
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) B[q] = hp[(t0 + 8 * h + q + k) * CH + n];
                }
                acc[k] = mfma(A, B, acc[k]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    const int stride = LAYER == 1 ? PART1 : PART;
    float* out = a.part + (int64_t)blockIdx.x * stride;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int o = acc_row(r, l);
        if (LAYER == 1) {
            if (n < 18) out[o * 18 + (n % 2) * 9 + n / 2] = acc[0][r];
        } else {
#pragma unroll
            for (int k = 0; k < NTILE; ++k) out[o * 288 + n * 9 + k] = acc[k][r];
        }
    }
    dbacc += __shfl_xor(dbacc, 32);
    if (h == 0) out[(LAYER == 1 ? 576 : 9216) + n] = dbacc;
}

struct RedArgs {
    const float* p1;   // [NWB][PART1]
    const float* p2;   // [NWB][PART]
    const float* p3;   // [NWB][PART]
    const float* p4;   // [NWB][PART4]
    float* grad;
    float* loss;
    float inv_count;
};

// deterministic sum of the per-wave partials into the parameter-vector layout
__global__ void lcf_reduce_kernel(const RedArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NPAR) return;
    if (p == NPAR) {
        float s = 0.0f;
        for (int w = 0; w < NWB; ++w) s += a.p4[(int64_t)w * PART4 + 66];
        *a.loss = s * a.inv_count;
        return;
    }
    const float* src;
    int stride, idx;
    if (p < OFF_B1) { src = a.p1; stride = PART1; idx = p; }
    else if (p < OFF_W2) { src = a.p1; stride = PART1; idx = 576 + (p - OFF_B1); }
    else if (p < OFF_B2) { src = a.p2; stride = PART; idx = p - OFF_W2; }
    else if (p < OFF_W3) { src = a.p2; stride = PART; idx = 9216 + (p - OFF_B2); }
    else if (p < OFF_B3) { src = a.p3; stride = PART; idx = p - OFF_W3; }
    else if (p < OFF_W4) { src = a.p3; stride = PART; idx = 9216 + (p - OFF_B3); }
    else { src = a.p4; stride = PART4; idx = p - OFF_W4; }
    float s = 0.0f;
    for (int w = 0; w < NWB; ++w) s += src[(int64_t)w * stride + idx];
    a.grad[p] = s;
}

// ---------------------------------------------------------------- optimiser, batches, fallback
__global__ void adam_kernel(float* w, uint16_t* wb, float* m, float* v, const float* g, int n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

__global__ void gather_kernel(const float2* src, int64_t nv, int T, const int64_t* idx, int64_t B, float2* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)T * B) return;
    const int t = (int)(i / B);
    const int64_t b = i - (int64_t)t * B;
    const int64_t gi = idx[b];
    const int64_t vol = gi / nv, vv = gi - vol * nv;
    dst[i] = src[(vol * T + t) * nv + vv];
}

__global__ void fb_partial_kernel(const float* pl, const float* ps, int64_t n, double* part) {
    __shared__ double s0[256], s1[256], s2[256];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float x = pl[i], y = ps[i];
        if (!isfinite(x)) a2 += 1.0;
        else {
            const double d = (double)x - (double)y;
            a0 += d * d;
        }
        a1 += (double)y * (double)y;
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s0[threadIdx.x] += s0[threadIdx.x + o];
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s0[0];
        part[3 * blockIdx.x + 1] = s1[0];
        part[3 * blockIdx.x + 2] = s2[0];
    }
}

__global__ void fb_decide_kernel(const double* part, int nblk, float tau_db, int* flag, float* d_db) {
    if (threadIdx.x != 0) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        a0 += part[3 * b];
        a1 += part[3 * b + 1];
        a2 += part[3 * b + 2];
    }
    const double d = a1 > 0.0 ? 10.0 * log10(fmax(a0, 1e-300) / a1) : 0.0;
    const int f = (a2 > 0.0) || !(a1 > 0.0) || !(d <= (double)tau_db);
    *flag = f;
    *d_db = a2 > 0.0 ? __builtin_nanf("") : (float)d;
}

__global__ void fb_select_kernel(const float* pl, const float* ps, int64_t n, const int* flag, float* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = *flag ? ps[i] : pl[i];
}

constexpr int FB_BLOCKS = 512;

size_t fwd_lds(int T) {   // the launch below takes the streamed kernel above 256 frames
    const int TP = 32 * ((T + 31) / 32) + 8;
    return (T > 256 ? 2 * (size_t)RING_ELEMS * 2 : (size_t)TP * RS * 2) + (size_t)(TP + 8) * 4 * 2;
}
size_t bwd_lds(int T) {
    const int TP = 32 * ((T + 31) / 32) + 8;
    return 68 * 4 + 2 * (size_t)T * 8 + 2 * (size_t)TP * CH * 2;
}
size_t wg_lds(int T, int layer) {
    const int TP = 32 * ((T + 31) / 32) + 8, T16 = (T + 15) / 16 * 16;
    return (size_t)T16 * CH * 2 + (size_t)TP * (layer == 1 ? 4 : CH) * 2;
}
size_t act_bytes(int64_t n, int T) { return round_up((size_t)n * act_stride(T) * 2, 256); }
size_t part_bytes() { return (size_t)NWB * (PART1 + 2 * PART + PART4) * 4; }

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t lcf_act_size(int64_t n_series, int32_t n_t) {
    if (n_series < 1 || n_t < 1) return 0;
    return act_bytes(n_series, n_t) + part_bytes();
}

extern "C" int lcf_forward(const float* w, const uint16_t* w_bf16, const float* x, int64_t n_series, int32_t n_t,
                           float eps, uint16_t* act, float* y, float* pd, void* stream) {
    FQ_REQUIRE(w && w_bf16 && x && aligned16(w_bf16) && aligned16(x), "null or misaligned pointer");
    FQ_REQUIRE(n_series >= 1 && n_t >= 1 && n_t <= FQ_MAX_NT, "bad sizes");
    FQ_REQUIRE(!act || aligned16(act), "misaligned act");
    FQ_REQUIRE(eps >= 0.0f, "eps must be >= 0");
    const size_t lds = fwd_lds(n_t);
    FQ_REQUIRE(lds <= 160 * 1024, "n_t too large");
    FwdArgs fa{w, w_bf16, reinterpret_cast<const float2*>(x), act, reinterpret_cast<float2*>(y), pd, n_series, n_t, eps};
    const unsigned grid = (unsigned)std::min<int64_t>(n_series, 8192);
    auto kern = n_t <= 256 ? (act ? lcf_fwd_kernel<4, true> : lcf_fwd_kernel<4, false>)
                           : (act ? lcf_fwd_kernel<8, true> : lcf_fwd_kernel<8, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, as_stream(stream), fa);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

extern "C" int lcf_backward(const float* w, const uint16_t* w_bf16, const float* x, const float* target,
                            int64_t n_series, int32_t n_t, float eps, uint16_t* act, float* grad, float* loss,
                            void* stream) {
    FQ_REQUIRE(w && w_bf16 && x && target && act && grad && loss, "null pointer");
    FQ_REQUIRE(aligned16(w_bf16) && aligned16(x) && aligned16(target) && aligned16(act), "misaligned pointer");
    FQ_REQUIRE(n_series >= 1 && n_t >= 1 && n_t <= FQ_MAX_NT, "bad sizes");
    hipStream_t s = as_stream(stream);
    char* base = reinterpret_cast<char*>(act) + act_bytes(n_series, n_t);
    float* p1 = reinterpret_cast<float*>(base);
    float* p2 = p1 + (size_t)NWB * PART1;
    float* p3 = p2 + (size_t)NWB * PART;
    float* p4 = p3 + (size_t)NWB * PART;
    const float inv_count = (float)(1.0 / ((double)n_series * 2.0 * n_t));
    BwdArgs ba{w, w_bf16, reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(target), act, p4,
               n_series, n_t, eps, inv_count};
    hipLaunchKernelGGL(lcf_bwd_series_kernel, dim3(NWB), dim3(64), bwd_lds(n_t), s, ba);
    FQ_LAUNCH_CHECK();
    WgArgs wa{act, p3, n_series, n_t, 3};
    hipLaunchKernelGGL(lcf_wgrad_kernel<3>, dim3(NWB), dim3(64), wg_lds(n_t, 3), s, wa);
    FQ_LAUNCH_CHECK();
    wa.part = p2;
    wa.layer = 2;
    hipLaunchKernelGGL(lcf_wgrad_kernel<2>, dim3(NWB), dim3(64), wg_lds(n_t, 2), s, wa);
    FQ_LAUNCH_CHECK();
    wa.part = p1;
    wa.layer = 1;
    hipLaunchKernelGGL(lcf_wgrad_kernel<1>, dim3(NWB), dim3(64), wg_lds(n_t, 1), s, wa);
    FQ_LAUNCH_CHECK();
    RedArgs ra{p1, p2, p3, p4, grad, loss, inv_count};
    hipLaunchKernelGGL(lcf_reduce_kernel, dim3((NPAR + 1 + 255) / 256), dim3(256), 0, s, ra);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

extern "C" int lcf_adam_step(float* w, uint16_t* w_bf16, float* m, float* v, const float* grad, int32_t n_param,
                             float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
    FQ_REQUIRE(w && w_bf16 && m && v && grad, "null pointer");
    FQ_REQUIRE(n_param >= 1 && step >= 1, "bad n_param / step");
    FQ_REQUIRE(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && lr >= 0, "bad Adam hyper-parameters");
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(adam_kernel, dim3((n_param + 255) / 256), dim3(256), 0, as_stream(stream), w, w_bf16, m, v,
                       grad, n_param, lr, beta1, beta2, eps, c1, c2);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

extern "C" int lcf_gather(const float* src, int64_t n_vox, int32_t n_t, int64_t n_vol, const int64_t* idx,
                          int64_t batch, float* dst, void* stream) {
    FQ_REQUIRE(src && idx && dst && aligned16(src) && aligned16(dst), "null or misaligned pointer");
    FQ_REQUIRE(n_vox >= 1 && n_t >= 1 && n_vol >= 1 && batch >= 1, "bad sizes");
    const int64_t total = (int64_t)n_t * batch;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, as_stream(stream),
                       reinterpret_cast<const float2*>(src), n_vox, n_t, idx, batch, reinterpret_cast<float2*>(dst));
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

extern "C" size_t fallback_workspace_size(int64_t n) {
    (void)n;
    return (size_t)FB_BLOCKS * 3 * sizeof(double);
}

extern "C" int lcf_fallback(const float* pd_l, const float* pd_s, int64_t n, float tau_db, void* ws, size_t ws_bytes,
                            float* out, int32_t* flag, float* d_db, void* stream) {
    FQ_REQUIRE(pd_l && pd_s && out && flag && d_db && ws, "null pointer");
    FQ_REQUIRE(n >= 1, "n must be >= 1");
    if (ws_bytes < fallback_workspace_size(n)) {
        set_error("workspace too small");
        return FQ_E_WORKSPACE;
    }
    hipStream_t s = as_stream(stream);
    double* part = reinterpret_cast<double*>(ws);
    hipLaunchKernelGGL(fb_partial_kernel, dim3(FB_BLOCKS), dim3(256), 0, s, pd_l, pd_s, n, part);
    FQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(fb_decide_kernel, dim3(1), dim3(64), 0, s, part, FB_BLOCKS, tau_db, flag, d_db);
    FQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(fb_select_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pd_l, pd_s, n, flag, out);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}
