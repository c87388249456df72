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

// FP64 mode.  Three pieces, all in FP64 VALU arithmetic:
//  - the distance: a hardware reciprocal-square-root seed, one Goldschmidt
//    step for sqrt(d2) and 1/(2 sqrt(d2)) together, then Markstein's two
//    residual corrections, which give the correctly rounded sqrt for the
//    normal-range d2 of any deployment (d2 is clamped to 1e-300: a point on an
//    antenna gets d = 1e-150 and phase 0 to the last bit);
//  - 1/d from the Goldschmidt estimate and one Newton step (within one ulp),
//    for the amplitude lambda / (4 pi max(d, d_min));
//  - sin and cos of 2 pi f for the exact fractional revolution f
//    (sincos_turn_f64).
struct TermF64 {
    double amp;
    double c;
    double s;
};

// a * b + c as the three-operand FP64 FMA.  With fma() the compiler picks the
// two-operand form, whose accumulator is overwritten, and copies each
// loop-invariant polynomial coefficient into it first: a 64-bit move per
// coefficient and term.  (Arithmetic only; no memory access.)
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// sin(2 pi f) and cos(2 pi f) for f in [-2^-50, 1].  The turn is cut into
// quarters: q = rint(4 f) and u = 4 f - q in [-1/2, 1/2] are exact, and
// x = u pi/2 in [-pi/4, pi/4] comes from pi/2 split into two doubles.  On that
// interval the Taylor series of sin through x^15 and of cos through x^16 leave
// truncation errors below 7e-17 and 3e-18 of the result; the coefficients are
// the exact 1/n! rounded once.  Quarter q rotates (sin x, cos x) by q right
// angles.  Error within 2 ulp (about 1.5e-16 absolute).  About 30 VALU
// instructions for both, against about 45 for the library's sincospi.
__device__ __forceinline__ void sincos_turn_f64(double f, double& s, double& c) {
    constexpr double kPio2Hi = 1.5707963267948966;       // pi/2 rounded to double
    constexpr double kPio2Lo = 6.123233995736766e-17;    // pi/2 - kPio2Hi
    const double f4 = 4.0 * f;
    const double q = rint(f4);
    const double u = f4 - q;
    const double x = fma(u, kPio2Hi, u * kPio2Lo);
    const double z = x * x;
    double ps = -1.0 / 1307674368000.0;                    // -1/15!
    ps = fma3(ps, z, 1.0 / 6227020800.0);
    ps = fma3(ps, z, -1.0 / 39916800.0);
    ps = fma3(ps, z, 1.0 / 362880.0);
    ps = fma3(ps, z, -1.0 / 5040.0);
    ps = fma3(ps, z, 1.0 / 120.0);
    ps = fma3(ps, z, -1.0 / 6.0);
    const double sx = fma(x * z, ps, x);
    double pc = 1.0 / 20922789888000.0;                     // 1/16!
    pc = fma3(pc, z, -1.0 / 87178291200.0);
    pc = fma3(pc, z, 1.0 / 479001600.0);
    pc = fma3(pc, z, -1.0 / 3628800.0);
    pc = fma3(pc, z, 1.0 / 40320.0);
    pc = fma3(pc, z, -1.0 / 720.0);
    pc = fma3(pc, z, 1.0 / 24.0);
    pc = fma3(pc, z, -0.5);
    const double cx = fma(z, pc, 1.0);
    const int iq = (int)q & 3;
    const bool odd = iq & 1;
    s = odd ? cx : sx;
    c = odd ? sx : cx;
    if (iq & 2) s = -s;
    if ((iq + 1) & 2) c = -c;
}

__device__ __forceinline__ TermF64 wave_term_f64(double dx, double dy, double dz,
                                                 double inv_lam, double amp_c,
                                                 double inv_dmin) {
    const double d2 = fmax(fma(dx, dx, fma(dy, dy, dz * dz)), 1e-300);
    const double y = __builtin_amdgcn_rsq(d2);
    double d = d2 * y;
    double h = 0.5 * y;
    const double r = fma(-h, d, 0.5);
    d = fma(d, r, d);
    h = fma(h, r, h);
    d = fma(fma(-d, d, d2), h, d);
    d = fma(fma(-d, d, d2), h, d);
    double inv = h + h;
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    const double rev = d * inv_lam;
    const double fr = rev - floor(rev);
    TermF64 t;
    sincos_turn_f64(fr, t.s, t.c);
    t.amp = amp_c * fmin(inv, inv_dmin);
    return t;
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace dmimo
