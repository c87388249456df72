// Internal helpers of libdmimo: error reporting, launch checks and the device
// functions that synthesise one channel term.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/dmimo.h"

namespace dmimo {

// ---------------------------------------------------------------------------
// host-side error state (thread-local)
// ---------------------------------------------------------------------------

void set_error(const char* fmt, ...);
void clear_error();

inline dmimo_status fail(dmimo_status st, const char* what) {
    set_error("%s", what);
    return st;
}

// checks the launch that was just made
dmimo_status check_launch(const char* kernel);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr double kSpeedOfLight = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// Constants of the free-space spherical-wave term for one carrier.
struct WaveConst {
    double inv_lam;    // 1 / lambda (FP64: phase in revolutions = d / lambda)
    double amp_c;      // lambda / (4 pi)
    double inv_dmin;   // 1 / d_min
    double a_los;      // sqrt(k/(1+k)) (1 for LoS)
    double a_nlos;     // sqrt(1/(1+k)) (0 for LoS)
};

dmimo_status make_wave_const(const dmimo_channel_params* p, WaveConst* out);

// Device copy of a point descriptor.
struct PointsDev {
    int32_t kind;
    int32_t nx, ny;
    double x0, y0, dx, dy, z;
    const double* xyz;
    int64_t n;   // points per deployment
};

dmimo_status make_points(const dmimo_points* p, PointsDev* out);

// ---------------------------------------------------------------------------
// device: point coordinates
// ---------------------------------------------------------------------------

__device__ __forceinline__ void point_xyz(const PointsDev& P, int64_t b, int64_t n,
                                          double& x, double& y, double& z) {
    if (P.kind == DMIMO_PTS_GRID) {
        const int32_t i = (int32_t)(n % P.nx);
        const int32_t j = (int32_t)(n / P.nx);
        x = P.x0 + ((double)i + 0.5) * P.dx;
        y = P.y0 + ((double)j + 0.5) * P.dy;
        z = P.z;
    } else {
        const double* q = P.xyz + (b * P.n + n) * 3;
        x = q[0];
        y = q[1];
        z = q[2];
    }
}

// ---------------------------------------------------------------------------
// device: one spherical-wave term
// ---------------------------------------------------------------------------
//
// Mixed mode (FP32 results): the squared distance, the distance and the phase
// in revolutions are FP64.  sqrt(d2) is an FP32 reciprocal-square-root seed
// refined by one Newton step in FP64: relative error about 1.5 * eps_seed^2,
// i.e. ~1e-13.  The fractional revolution frac(d / lambda) is exact in FP64.
// Rounded to FP32 it feeds the hardware sine/cosine, which take their
// argument in revolutions, so no FP32 range reduction is needed.  The
// amplitude lambda/(4 pi d) reuses the FP32 seed.
//
// Returns the phase-rotated unit phasor (c, -s) and the amplitude.

struct TermF32 {
    float amp;   // lambda / (4 pi max(d, d_min))
    float c;     // cos(2 pi frac(d/lambda))
    float s;     // sin(2 pi frac(d/lambda));  h = amp * (c - j s)
};

__device__ __forceinline__ TermF32 wave_term_f32(double dx, double dy, double dz,
                                                 double inv_lam, float amp_c,
                                                 float inv_dmin) {
    double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
    d2 = fmax(d2, 1e-24);
    const float rs = __builtin_amdgcn_rsqf((float)d2);
    const double y = (double)rs;
    const double s0 = d2 * y;
    const double e = fma(-s0, s0, d2);
    const double d = fma(e, 0.5 * y, s0);
    const double rev = d * inv_lam;
    const float fr = (float)(rev - floor(rev));
    TermF32 t;
    t.amp = amp_c * fminf(rs, inv_dmin);
    t.c = __builtin_amdgcn_cosf(fr);
    t.s = __builtin_amdgcn_sinf(fr);
    return t;
}

// FP64 mode: correctly rounded sqrt, FP64 sincospi of the exact fractional
// revolution, FP64 amplitude.
struct TermF64 {
    double amp;
    double c;
    double s;
};

__device__ __forceinline__ TermF64 wave_term_f64(double dx, double dy, double dz,
                                                 double inv_lam, double amp_c,
                                                 double inv_dmin) {
    const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double d = sqrt(d2);
    const double rev = d * inv_lam;
    const double fr = rev - floor(rev);
    TermF64 t;
    sincospi(2.0 * fr, &t.s, &t.c);
    t.amp = amp_c * fmin(1.0 / d, inv_dmin);
    return t;
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace dmimo
