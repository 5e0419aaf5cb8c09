// das_beamform: RF -> IQ demodulation and 3-D delay-and-sum with coherent compounding (gfx950).
//
// Stage 1, rf2iq: one workgroup per (frame block of 8, angle, element) stages the 8 RF
// traces in LDS and writes the baseband in a frame-blocked layout
//     bb[fblock][angle][element][sample][8 frames]   (complex64)
// so that one delay tap of one (angle, element) for all 8 frames of a block is a single
// 64-byte row.  b[n] = exp(-i w n) sum_k c_k rf[n-k] with precomputed complex taps
// c_k = 2 h_k exp(i w k), w = 2 pi fc/fs.
//
// Stage 2, DAS: one workgroup per (16x16x2 voxel tile, frame block).  Each thread owns a
// column of 2 voxels and keeps 2 x 8 complex accumulators.  The element loop stages, for
// every angle of the pass, the window of delay rows the tile can touch into LDS (the
// window is bounded from the tile's box: nearest/farthest point for the receive path,
// extreme corners for the transmit plane), then every thread forms its taps from LDS.
// Delays are split into an integer sample index and an FP32 fraction from FP64
// geometry; the phase exp(i 2 pi fc tau) is the product of a per-(voxel, angle) factor
// and a per-(voxel, element) factor, each taken from an FP64 cycle count, so no large
// argument ever reaches FP32 trigonometry.  The per-(voxel, element) work (FP64 receive
// distance, its phase) is shared by all angles and the per-(voxel, element, angle) work
// by the 8 frames of the block, as the paper does by building the delay operator once
// and applying it to every frame.
#include "fq_common.hpp"

namespace fq {
namespace {

constexpr int FB = 8;           // frames per block
constexpr int TILE_X = 16, TILE_Y = 16, VZ = 2;   // two voxels per thread: 167 VGPRs, 3 waves/SIMD
constexpr int DAS_THREADS = TILE_X * TILE_Y;
constexpr int ROW_F4 = 5;       // LDS row stride in float4 (4 used + 1 pad against bank conflicts)
constexpr int MAX_AT = 9;       // angles per DAS pass (compile-time unrolled)
constexpr int FIR_HALF = 16;
constexpr int IQ_THREADS = 256;
constexpr size_t DAS_LDS_BUDGET = 64 * 1024;

// --------------------------------------------------------------------------- rf2iq
struct IqArgs {
    const float* rf;       // [F][A][E][T]
    float2* bb;            // [nfb][A][E][T][FB]
    int F, A, E, T;
    int fb0;               // first global frame block of this launch
    double fc_fs;          // fc / fs
    float2 taps[2 * FIR_HALF + 1];
};

__global__ void __launch_bounds__(IQ_THREADS) rf2iq_kernel(const IqArgs a) {
    extern __shared__ float sh[];          // [FB][T + 2*FIR_HALF + 1]
    const int e = blockIdx.x, an = blockIdx.y, fbl = blockIdx.z;
    const int fb = a.fb0 + fbl;
    const int stride = a.T + 2 * FIR_HALF + 1;  // odd: frames fall in different banks
    for (int i = threadIdx.x; i < FB * stride; i += IQ_THREADS) {
        const int fl = i / stride, m = i - fl * stride - FIR_HALF;
        const int f = fb * FB + fl;
        float v = 0.0f;
        if (f < a.F && m >= 0 && m < a.T) v = a.rf[(((int64_t)f * a.A + an) * a.E + e) * a.T + m];
        sh[i] = v;
    }
    __syncthreads();
    float2* out = a.bb + (((int64_t)fbl * a.A + an) * a.E + e) * (int64_t)a.T * FB;
    for (int i = threadIdx.x; i < FB * a.T; i += IQ_THREADS) {
        const int n = i / FB, fl = i - n * FB;
        const float* row = sh + fl * stride + FIR_HALF + n;
        float re = 0.0f, im = 0.0f;
#pragma unroll
        for (int k = -FIR_HALF; k <= FIR_HALF; ++k) {
            const float v = row[-k];
            re = fmaf(a.taps[k + FIR_HALF].x, v, re);
            im = fmaf(a.taps[k + FIR_HALF].y, v, im);
        }
        const float2 rot = cis_cycles(-(double)n * a.fc_fs);
        out[i] = cmul(rot, make_float2(re, im));
    }
}

// --------------------------------------------------------------------------- DAS
struct DasArgs {
    const float4* bb;      // frame-blocked baseband, see header comment
    float2* iq;            // [F][Nv]
    int nx, ny, nz;
    int ntx, nty;          // tiles along x, y
    int64_t ntiles;        // tiles of the grid
    int64_t nwork;         // (tile, frame block) pairs of this launch
    double x0, y0, z0, dx, dy, dz;
    int nx_el;
    double pitch_x, pitch_y;
    double fs_c, fc_fs;    // fs/c, fc/fs
    int A, E, T, F;
    int a0, nang;          // angles of this pass
    int fb0;               // first global frame block of this launch
    int W;                 // LDS window rows per angle
    int accumulate;
    float inv_A;
    double ux[MAX_AT], uy[MAX_AT], uz[MAX_AT], t0s[MAX_AT];  // t0s = t0 * fs
    float dxz[MAX_AT];                                       // transmit delay per voxel step in z, samples
    float2 zeta[MAX_AT][VZ];                                 // exp(i 2 pi fc uz dz k / c)
};

template <int AT, int INTERP>
__global__ void __launch_bounds__(DAS_THREADS, 3) das_kernel(const DasArgs a) {
    constexpr int NT = INTERP ? 4 : 2;         // taps per delay
    constexpr int J0 = INTERP ? -1 : 0;        // first tap offset
    extern __shared__ float4 win[];            // [AT][W][ROW_F4]
    __shared__ int nlo_s[MAX_AT];

    // Workgroup id -> (tile, frame block), tiles fastest.  (Handing each XCD a contiguous
    // run of tiles cut the HBM traffic ~3x but ran 5.6% slower: the neighbouring tiles of one
    // XCD request the same delay rows at the same time.)
    const int64_t g = blockIdx.x;
    if (g >= a.nwork) return;
    const int tile = (int)(g % a.ntiles);
    const int txi = tile % a.ntx, tyi = (tile / a.ntx) % a.nty, tzi = tile / (a.ntx * a.nty);
    const int fbl = (int)(g / a.ntiles);
    const int fb = a.fb0 + fbl;
    const int lx = threadIdx.x % TILE_X, ly = threadIdx.x / TILE_X;
    const int ix = txi * TILE_X + lx, iy = tyi * TILE_Y + ly, iz0 = tzi * VZ;

    const double xv = a.x0 + ix * a.dx, yv = a.y0 + iy * a.dy, zv0 = a.z0 + iz0 * a.dz;
    // tile box (voxel centres, including voxels past the grid edge)
    const double bx0 = a.x0 + txi * TILE_X * a.dx, bx1 = bx0 + (TILE_X - 1) * a.dx;
    const double by0 = a.y0 + tyi * TILE_Y * a.dy, by1 = by0 + (TILE_Y - 1) * a.dy;
    const double bz0 = zv0, bz1 = zv0 + (VZ - 1) * a.dz;

    // per-angle transmit delay and phase of this thread's first voxel
    int ntx[AT];
    float ftx[AT];
    float2 ptx[AT];
#pragma unroll
    for (int j = 0; j < AT; ++j) {
        const double x = (a.ux[j] * xv + a.uy[j] * yv + a.uz[j] * zv0) * a.fs_c - a.t0s[j];
        const double fl = floor(x);
        ntx[j] = (int)fl;
        ftx[j] = (float)(x - fl);
        ptx[j] = cis_cycles(x * a.fc_fs);
    }

    float2 acc[VZ][FB];
#pragma unroll
    for (int k = 0; k < VZ; ++k)
#pragma unroll
        for (int q = 0; q < FB; ++q) acc[k][q] = make_float2(0.0f, 0.0f);

    const int ny_el = a.E / a.nx_el;
    const int64_t trace_rows = (int64_t)a.T;   // rows per (fb, angle, element) trace
    for (int e = 0; e < a.E; ++e) {
        const double pex = ((e % a.nx_el) - 0.5 * (a.nx_el - 1)) * a.pitch_x;
        const double pey = ((e / a.nx_el) - 0.5 * (ny_el - 1)) * a.pitch_y;
        __syncthreads();   // previous element's taps consumed
        if (threadIdx.x < AT) {
            const int j = threadIdx.x;
            // lowest delay over the tile box: transmit plane at its lowest corner,
            // receive distance at the box point nearest to the element
            const double tmin = (a.ux[j] * (a.ux[j] > 0 ? bx0 : bx1) + a.uy[j] * (a.uy[j] > 0 ? by0 : by1) +
                                 a.uz[j] * bz0) * a.fs_c - a.t0s[j];
            const double cx = fmin(fmax(pex, bx0), bx1) - pex, cy = fmin(fmax(pey, by0), by1) - pey;
            const double rmin = sqrt(cx * cx + cy * cy + bz0 * bz0) * a.fs_c;
            nlo_s[j] = (int)floor(tmin + rmin) - 2;
        }
        __syncthreads();
        // stage W rows per angle; rows outside [0, T) are zero (zero padding)
        const int per_ang = a.W * 4;
#pragma unroll
        for (int j = 0; j < AT; ++j) {
            const int64_t tr = ((int64_t)fbl * a.A + a.a0 + j) * a.E + e;
            const float4* src = a.bb + tr * trace_rows * 4;
            for (int rem = threadIdx.x; rem < per_ang; rem += DAS_THREADS) {
                const int r = rem >> 2, c4 = rem & 3;
                const int n = nlo_s[j] + r;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (n >= 0 && n < a.T) v = src[(int64_t)n * 4 + c4];
                win[(j * a.W + r) * ROW_F4 + c4] = v;
            }
        }
        __syncthreads();

        // receive geometry of the thread's voxels (FP64 distance, shared by all angles)
        const double ddx = xv - pex, ddy = yv - pey;
        const double dxy2 = ddx * ddx + ddy * ddy;
        int nrx[VZ];
        float frx[VZ];
        float2 prx[VZ];
#pragma unroll
        for (int k = 0; k < VZ; ++k) {
            const double z = zv0 + k * a.dz;
            const double rho = sqrt_nr(dxy2 + z * z);
            const double xr = rho * a.fs_c;
            const double fl = floor(xr);
            nrx[k] = (int)fl;
            frx[k] = (float)(xr - fl);
            prx[k] = cis_cycles(xr * a.fc_fs);
        }

#pragma unroll
        for (int j = 0; j < AT; ++j) {
            const int base = nlo_s[j];
#pragma unroll
            for (int k = 0; k < VZ; ++k) {
                const float s = ftx[j] + (float)k * a.dxz[j] + frx[k];
                const float sf = floorf(s);
                const float al = s - sf;
                int row = ntx[j] + nrx[k] + (int)sf - base + J0;
#ifdef FQ_DEBUG_WINDOW
                // debug builds: a tap outside the staged window poisons the voxel
                if (row < 0 || row > a.W - NT) acc[k][0].x = __builtin_nanf("");
#endif
                // The window bound (window_rows) covers every tap of the tile, so the clamp
                // never engages (checked on the host for the workload geometries and extreme
                // tilts); it keeps the LDS reads in bounds whatever the input.
                row = min(max(row, 0), a.W - NT);
                float2 P = cmul(ptx[j], prx[k]);
                if (k > 0) P = cmul(P, a.zeta[j][k]);
                float w[NT];
                if (INTERP == 0) {
                    w[0] = 1.0f - al;
                    w[1] = al;
                } else {
                    const float a2 = al * al, a3 = a2 * al;
                    w[0] = 0.5f * (-a3 + 2.0f * a2 - al);
                    w[1] = 0.5f * (3.0f * a3 - 5.0f * a2 + 2.0f);
                    w[2] = 0.5f * (-3.0f * a3 + 4.0f * a2 + al);
                    w[3] = 0.5f * (a3 - a2);
                }
                // taps combined with the real weights, then rotated: acc += P * sum_t w_t b_t
                const float nPy = -P.y;
                const float4* rp = win + (j * a.W + row) * ROW_F4;
#pragma unroll
                for (int q = 0; q < FB / 2; ++q) {
                    const float4 b0 = rp[q];
                    float4 B = make_float4(w[0] * b0.x, w[0] * b0.y, w[0] * b0.z, w[0] * b0.w);
#pragma unroll
                    for (int t = 1; t < NT; ++t) {
                        const float4 b = rp[t * ROW_F4 + q];
                        B.x = fmaf(w[t], b.x, B.x);
                        B.y = fmaf(w[t], b.y, B.y);
                        B.z = fmaf(w[t], b.z, B.z);
                        B.w = fmaf(w[t], b.w, B.w);
                    }
                    float2& c0 = acc[k][2 * q];
                    float2& c1 = acc[k][2 * q + 1];
                    c0.x = fmaf(P.x, B.x, c0.x);
                    c0.x = fmaf(nPy, B.y, c0.x);
                    c0.y = fmaf(P.x, B.y, c0.y);
                    c0.y = fmaf(P.y, B.x, c0.y);
                    c1.x = fmaf(P.x, B.z, c1.x);
                    c1.x = fmaf(nPy, B.w, c1.x);
                    c1.y = fmaf(P.x, B.w, c1.y);
                    c1.y = fmaf(P.y, B.z, c1.y);
                }
            }
        }
    }

    if (ix >= a.nx || iy >= a.ny) return;
    const int64_t nv = (int64_t)a.nx * a.ny * a.nz;
#pragma unroll
    for (int k = 0; k < VZ; ++k) {
        const int iz = iz0 + k;
        if (iz >= a.nz) break;
        const int64_t v = ix + (int64_t)a.nx * (iy + (int64_t)a.ny * iz);
#pragma unroll
        for (int q = 0; q < FB; ++q) {
            const int f = fb * FB + q;
            if (f >= a.F) break;
            float2* o = a.iq + (int64_t)f * nv + v;
            float2 r = make_float2(acc[k][q].x * a.inv_A, acc[k][q].y * a.inv_A);
            if (a.accumulate) {
                const float2 old = *o;
                r.x += old.x;
                r.y += old.y;
            }
            *o = r;
        }
    }
}

using DasFn = void (*)(const DasArgs);

template <int AT>
DasFn pick(int interp) {
    return interp ? das_kernel<AT, 1> : das_kernel<AT, 0>;
}

DasFn das_fn(int at, int interp) {
    switch (at) {
        case 1: return pick<1>(interp);
        case 2: return pick<2>(interp);
        case 3: return pick<3>(interp);
        case 4: return pick<4>(interp);
        case 5: return pick<5>(interp);
        case 6: return pick<6>(interp);
        case 7: return pick<7>(interp);
        case 8: return pick<8>(interp);
        default: return pick<9>(interp);
    }
}

// Low-pass taps: Hann(33)-windowed sinc with cutoff fc, unit DC gain; folded with the
// carrier as c_k = 2 h_k exp(i 2 pi fc k / fs).
void make_taps(double fc, double fs, float2* taps) {
    double h[2 * FIR_HALF + 1], sum = 0.0;
    for (int k = -FIR_HALF; k <= FIR_HALF; ++k) {
        const double w = 0.5 * (1.0 + std::cos(M_PI * k / (FIR_HALF + 1)));
        const double x = 2.0 * fc * k / fs;
        const double sn = k == 0 ? 1.0 : std::sin(M_PI * x) / (M_PI * x);
        h[k + FIR_HALF] = w * sn;
        sum += w * sn;
    }
    for (int k = -FIR_HALF; k <= FIR_HALF; ++k) {
        const double hk = 2.0 * h[k + FIR_HALF] / sum;
        const double ph = 2.0 * M_PI * fc * k / fs;
        taps[k + FIR_HALF] = make_float2((float)(hk * std::cos(ph)), (float)(hk * std::sin(ph)));
    }
}

// Upper bound on the delay-window rows a tile can touch for one (angle, element):
// receive-distance spread <= tile diameter, transmit spread <= |u|.extent, plus the
// interpolation taps and the flooring/rounding margins used by the kernel.
int window_rows(const fq_grid& g, const TxHost& th, double fs_c) {
    const double Lx = (TILE_X - 1) * g.dx, Ly = (TILE_Y - 1) * g.dy, Lz = (VZ - 1) * g.dz;
    const double diam = std::sqrt(Lx * Lx + Ly * Ly + Lz * Lz);
    double txr = 0.0;
    for (int j = 0; j < th.n; ++j)
        txr = std::max(txr, std::fabs(th.ux[j]) * Lx + std::fabs(th.uy[j]) * Ly + th.uz[j] * Lz);
    const int w = (int)std::floor((diam + txr) * fs_c) + 8;
    return (int)round_up((size_t)w, 8);
}

size_t block_bytes(int A, int E, int T) { return (size_t)A * E * T * FB * sizeof(float2); }

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" size_t das_workspace_size(const fq_probe* probe, const fq_tx* tx, int32_t n_frames, int32_t n_samples,
                                     int32_t minimum) {
    if (!probe || !tx || n_frames < 1 || n_samples < 1 || tx->n_angles < 1) return 0;
    const int nfb = (n_frames + FB - 1) / FB;
    const size_t b = block_bytes(tx->n_angles, probe->nx_el * probe->ny_el, n_samples);
    return minimum ? b : b * nfb;
}

extern "C" int das_window_rows(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid) {
    if (check_probe_tx(probe, tx) != FQ_OK) return -1;
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->dx > 0) || !(grid->dy > 0) ||
        !(grid->dz > 0)) {
        set_error("bad grid");
        return -1;
    }
    return window_rows(*grid, make_tx(*probe, *tx), probe->fs_hz / probe->c_mps);
}

namespace fq {
namespace {

struct DasPlan {
    IqArgs ia;
    DasArgs da;
    TxHost th;
    int A, E, T, nfb, at, W;
    size_t bblk, iq_lds, row_bytes;
    int64_t ntiles;
    double fs_c;
};

int das_prepare(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid, int32_t n_frames, int32_t n_samples,
                const float* rf, int32_t interp, void* ws, size_t ws_bytes, float* iq, DasPlan& P) {
    int st = check_probe_tx(probe, tx);
    if (st != FQ_OK) return st;
    FQ_REQUIRE(grid && grid->nx > 0 && grid->ny > 0 && grid->nz > 0 && grid->dx > 0 && grid->dy > 0 && grid->dz > 0,
               "bad grid");
    FQ_REQUIRE(grid->z0 > 0, "the voxel grid must lie in front of the array (z0 > 0)");
    FQ_REQUIRE(n_frames >= 1 && n_samples >= 2 && n_samples <= (1 << 20), "bad n_frames / n_samples");
    FQ_REQUIRE(interp == FQ_INTERP_LINEAR || interp == FQ_INTERP_HERMITE, "bad interp");
    FQ_REQUIRE(ws && aligned16(ws), "null or misaligned workspace");
    FQ_REQUIRE((!rf || aligned16(rf)) && (!iq || aligned16(iq)), "misaligned pointer");
    P.A = tx->n_angles;
    P.E = probe->nx_el * probe->ny_el;
    P.T = n_samples;
    P.bblk = block_bytes(P.A, P.E, P.T);
    if (ws_bytes < P.bblk) {
        set_error("workspace too small: %zu < %zu bytes", ws_bytes, P.bblk);
        return FQ_E_WORKSPACE;
    }
    P.th = make_tx(*probe, *tx);
    P.fs_c = probe->fs_hz / probe->c_mps;
    P.W = window_rows(*grid, P.th, P.fs_c);
    P.row_bytes = ROW_F4 * sizeof(float4);
    P.at = (int)std::min<size_t>(MAX_AT, DAS_LDS_BUDGET / (P.row_bytes * P.W));
    FQ_REQUIRE(P.at >= 1, "voxel spacing too coarse for the on-chip delay window (%d rows)", P.W);
    P.nfb = (n_frames + FB - 1) / FB;

    IqArgs& ia = P.ia;
    ia = IqArgs{};
    ia.rf = rf;
    ia.bb = reinterpret_cast<float2*>(ws);
    ia.F = n_frames;
    ia.A = P.A;
    ia.E = P.E;
    ia.T = P.T;
    ia.fc_fs = probe->fc_hz / probe->fs_hz;
    make_taps(probe->fc_hz, probe->fs_hz, ia.taps);
    P.iq_lds = sizeof(float) * FB * (size_t)(P.T + 2 * FIR_HALF + 1);
    FQ_REQUIRE(P.iq_lds <= 160 * 1024, "n_samples too large for on-chip demodulation");

    DasArgs& da = P.da;
    da = DasArgs{};
    da.bb = reinterpret_cast<const float4*>(ws);
    da.iq = reinterpret_cast<float2*>(iq);
    da.nx = grid->nx;
    da.ny = grid->ny;
    da.nz = grid->nz;
    da.ntx = (grid->nx + TILE_X - 1) / TILE_X;
    da.nty = (grid->ny + TILE_Y - 1) / TILE_Y;
    const int ntz = (grid->nz + VZ - 1) / VZ;
    da.x0 = grid->x0;
    da.y0 = grid->y0;
    da.z0 = grid->z0;
    da.dx = grid->dx;
    da.dy = grid->dy;
    da.dz = grid->dz;
    da.nx_el = probe->nx_el;
    da.pitch_x = probe->pitch_x;
    da.pitch_y = probe->pitch_y;
    da.fs_c = P.fs_c;
    da.fc_fs = probe->fc_hz / probe->fs_hz;
    da.A = P.A;
    da.E = P.E;
    da.T = P.T;
    da.F = n_frames;
    da.W = P.W;
    da.inv_A = 1.0f / (float)P.A;
    P.ntiles = (int64_t)da.ntx * da.nty * ntz;
    FQ_REQUIRE(P.ntiles < (1LL << 31), "grid too large");
    da.ntiles = P.ntiles;
    return FQ_OK;
}

int launch_demod(DasPlan& P, int fb0, int nb, hipStream_t s) {
    P.ia.fb0 = fb0;
    hipLaunchKernelGGL(rf2iq_kernel, dim3(P.E, P.A, nb), dim3(IQ_THREADS), P.iq_lds, s, P.ia);
    FQ_LAUNCH_CHECK();
    return FQ_OK;
}

int launch_das(DasPlan& P, int fb0, int nb, int interp, const fq_grid* grid, double fs_hz, hipStream_t s) {
    DasArgs& da = P.da;
    da.fb0 = fb0;
    da.nwork = P.ntiles * nb;
    FQ_REQUIRE(da.nwork * DAS_THREADS < (1LL << 32), "grid too large");
    for (int a0 = 0; a0 < P.A; a0 += P.at) {
        const int na = std::min(P.at, P.A - a0);
        da.a0 = a0;
        da.nang = na;
        da.accumulate = a0 > 0;
        for (int j = 0; j < na; ++j) {
            const int an = a0 + j;
            da.ux[j] = P.th.ux[an];
            da.uy[j] = P.th.uy[an];
            da.uz[j] = P.th.uz[an];
            da.t0s[j] = P.th.t0[an] * fs_hz;
            const double step = P.th.uz[an] * grid->dz * P.fs_c;     // samples per z step
            da.dxz[j] = (float)step;
            for (int k = 0; k < VZ; ++k) {
                const double cyc = k * step * da.fc_fs;
                const double fr = cyc - std::floor(cyc);
                da.zeta[j][k] = make_float2((float)std::cos(2 * M_PI * fr), (float)std::sin(2 * M_PI * fr));
            }
        }
        const size_t lds = P.row_bytes * (size_t)P.W * na;
        hipLaunchKernelGGL(das_fn(na, interp), dim3((unsigned)da.nwork), dim3(DAS_THREADS), lds, s, da);
        FQ_LAUNCH_CHECK();
    }
    return FQ_OK;
}

}  // namespace
}  // namespace fq

extern "C" int das_beamform(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid, int32_t n_frames,
                            int32_t n_samples, const float* rf, int32_t interp, void* ws, size_t ws_bytes,
                            float* iq, void* stream) {
    FQ_REQUIRE(rf && iq, "rf and iq must not be NULL");
    DasPlan P;
    int st = das_prepare(probe, tx, grid, n_frames, n_samples, rf, interp, ws, ws_bytes, iq, P);
    if (st != FQ_OK) return st;
    hipStream_t s = as_stream(stream);
    const int per_launch = (int)std::min<size_t>(P.nfb, ws_bytes / P.bblk);
    for (int fb0 = 0; fb0 < P.nfb; fb0 += per_launch) {
        const int nb = std::min(per_launch, P.nfb - fb0);
        if ((st = launch_demod(P, fb0, nb, s)) != FQ_OK) return st;
        if ((st = launch_das(P, fb0, nb, interp, grid, probe->fs_hz, s)) != FQ_OK) return st;
    }
    return FQ_OK;
}

extern "C" int das_demodulate(const fq_probe* probe, const fq_tx* tx, int32_t n_frames, int32_t n_samples,
                              const float* rf, void* ws, size_t ws_bytes, void* stream) {
    FQ_REQUIRE(rf, "rf must not be NULL");
    fq_grid g{1, 1, 1, 0.0, 0.0, 1.0, 1e-4, 1e-4, 1e-4};
    DasPlan P;
    int st = das_prepare(probe, tx, &g, n_frames, n_samples, rf, 0, ws, ws_bytes, nullptr, P);
    if (st != FQ_OK) return st;
    if (ws_bytes < P.bblk * P.nfb) {
        set_error("das_demodulate needs the full workspace (%zu bytes)", P.bblk * P.nfb);
        return FQ_E_WORKSPACE;
    }
    return launch_demod(P, 0, P.nfb, as_stream(stream));
}

extern "C" int das_delay_sum(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid, int32_t n_frames,
                             int32_t n_samples, int32_t interp, const void* ws, size_t ws_bytes, float* iq,
                             void* stream) {
    FQ_REQUIRE(iq, "iq must not be NULL");
    DasPlan P;
    int st = das_prepare(probe, tx, grid, n_frames, n_samples, nullptr, interp, const_cast<void*>(ws), ws_bytes, iq, P);
    if (st != FQ_OK) return st;
    if (ws_bytes < P.bblk * P.nfb) {
        set_error("das_delay_sum needs the full workspace (%zu bytes)", P.bblk * P.nfb);
        return FQ_E_WORKSPACE;
    }
    return launch_das(P, 0, P.nfb, interp, grid, probe->fs_hz, as_stream(stream));
}
