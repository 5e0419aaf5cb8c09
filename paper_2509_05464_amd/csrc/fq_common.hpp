// Shared host/device helpers of the gfx950 power-Doppler library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/fqpd.h"

namespace fq {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
int zero_async(void* p, size_t n_bytes, hipStream_t s);

// ------------------------------------------------------------------ spatial similarity
// Workspace bytes and launch of the SSM pass (ssm.hip); C == nullptr keeps the matrix in
// the workspace, k_out == nullptr skips the rank rule.
size_t ssm_bytes(int64_t n_vox, int n_t);
int launch_ssm(const float* iq, int64_t n_vox, int n_t, const double* vecs, int n_modes, char* ws, double* C,
               int* k_out, hipStream_t s);

#define FQ_REQUIRE(cond, ...)                         \
    do {                                              \
        if (!(cond)) {                                \
            ::fq::set_error(__VA_ARGS__);             \
            return FQ_E_INVALID;                      \
        }                                             \
    } while (0)

#define FQ_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::fq::set_error("%s failed: %s", #call, hipGetErrorString(e_));           \
            return FQ_E_HIP;                                                          \
        }                                                                             \
    } while (0)

#define FQ_LAUNCH_CHECK()                                                             \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) {                                                       \
            ::fq::set_error("kernel launch failed: %s", hipGetErrorString(e_));       \
            return FQ_E_HIP;                                                          \
        }                                                                             \
    } while (0)

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ geometry (host, FP64)
struct TxHost {
    int n;
    double ux[FQ_MAX_ANGLES], uy[FQ_MAX_ANGLES], uz[FQ_MAX_ANGLES];
    double t0[FQ_MAX_ANGLES];  // min over elements of u.p/c
};

// u_a and t0_a = min_e (u_a . p_e)/c.  u.p is linear in the element position, so its
// minimum over the regular array is reached at one of the four corner elements.
inline TxHost make_tx(const fq_probe& p, const fq_tx& t) {
    TxHost h{};
    h.n = t.n_angles;
    const double hx = 0.5 * (p.nx_el - 1) * p.pitch_x, hy = 0.5 * (p.ny_el - 1) * p.pitch_y;
    for (int a = 0; a < t.n_angles; ++a) {
        double sx = std::sin(t.tilt_rad[a][0]), sy = std::sin(t.tilt_rad[a][1]);
        h.ux[a] = sx;
        h.uy[a] = sy;
        h.uz[a] = std::sqrt(1.0 - sx * sx - sy * sy);
        h.t0[a] = (-std::fabs(sx) * hx - std::fabs(sy) * hy) / p.c_mps;
    }
    return h;
}

inline int check_probe_tx(const fq_probe* p, const fq_tx* t) {
    FQ_REQUIRE(p && t, "probe/tx must not be NULL");
    FQ_REQUIRE(p->nx_el > 0 && p->ny_el > 0 && p->nx_el * p->ny_el <= 65536, "bad element counts");
    FQ_REQUIRE(p->fs_hz > 0 && p->fc_hz > 0 && p->c_mps > 0 && p->fc_hz < 0.5 * p->fs_hz,
               "need fs > 2 fc > 0 and c > 0");
    FQ_REQUIRE(t->n_angles >= 1 && t->n_angles <= FQ_MAX_ANGLES, "n_angles must be 1..%d", FQ_MAX_ANGLES);
    for (int a = 0; a < t->n_angles; ++a) {
        double sx = std::sin(t->tilt_rad[a][0]), sy = std::sin(t->tilt_rad[a][1]);
        FQ_REQUIRE(sx * sx + sy * sy < 0.99, "transmit %d: tilt too large", a);
    }
    return FQ_OK;
}

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(i 2 pi frac) for the fractional part of a double-precision cycle count; the
// integer part is removed exactly in FP64 and the remainder, in turns, goes to the
// hardware sine and cosine (which take turns; absolute error ~1e-7).
__device__ __forceinline__ float2 cis_cycles(double cyc) {
    const float fr = (float)(cyc - floor(cyc));
    return make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
}

// sqrt(x) for x > 0 from the hardware 1/sqrt estimate and one FP64 Newton step
// (relative error ~1e-14).
__device__ __forceinline__ double sqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double r = x * y;
    return fma(fma(-r, r, x), 0.5 * y, r);
}

}  // namespace fq
