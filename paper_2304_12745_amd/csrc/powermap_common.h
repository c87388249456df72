// Pieces shared by the matrix-core power-map kernels.
#pragma once

#include <cmath>

#include "kernels.h"

namespace dmimo {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Device arguments of the FP32-output map kernels.
struct PmMapDev {
    PointsDev P;
    int M;
    int K;               // streams of the contraction
    int G;               // streams per output map: map g takes streams g G .. g G + G - 1
    double inv_lam;      // 1 / lambda: positions are converted to wavelengths
    float amp_rev;       // 1 / (4 pi): amplitude = amp_rev / d_rev
    float inv_dmin_rev;  // lambda / d_min
    int hexp;            // FP16 split maps: h is scaled by 2^hexp (see fp16_h_exponent)
    const double* ap;    // [M][3] metres
    const float2* W;     // [K][M]
    float sigma2;
    float* power;
    float* sinr;
    int32_t* best_k;
    float* per_stream;
};

// Map p of a batched launch: its weights and outputs.
__device__ __forceinline__ PmMapDev map_of(PmMapDev a, int64_t p) {
    const int64_t N = a.P.n;
    a.W += p * a.K * a.M;
    a.power += p * N;
    if (a.sinr) a.sinr += p * N;
    if (a.best_k) a.best_k += p * N;
    if (a.per_stream) a.per_stream += p * N * a.K;
    return a;
}

// Exponent e of the power-of-two scale 2^e that the FP16 split maps apply to
// h.  |h| <= (1 / (4 pi)) (lambda / d_min) by the near-field clamp, and e is
// the largest exponent <= 14 that keeps that bound times 2^e at or below
// 2^14 (FP16's largest finite value is 65504): 14 for the default d_min =
// lambda / (4 pi), less for a smaller d_min.
inline int fp16_h_exponent(float amp_rev, float inv_dmin_rev) {
    const double bound = (double)amp_rev * (double)inv_dmin_rev * (1.0 - 1e-6);
    int e = 14;
    if (bound > 1.0) e -= (int)std::ceil(std::log2(bound));
    return e;
}

inline PmMapDev make_map_dev(const PowermapArgs& a) {
    PmMapDev d;
    d.P = a.P;
    d.M = a.M;
    d.K = a.K;
    d.G = a.K;
    d.inv_lam = a.w.inv_lam;
    d.amp_rev = (float)(1.0 / (4.0 * kPi));
    d.inv_dmin_rev = (float)(a.w.inv_dmin / a.w.inv_lam);
    d.hexp = fp16_h_exponent(d.amp_rev, d.inv_dmin_rev);
    d.ap = a.ap;
    d.W = reinterpret_cast<const float2*>(a.W);
    d.sigma2 = (float)a.sigma2;
    d.power = reinterpret_cast<float*>(a.power);
    d.sinr = reinterpret_cast<float*>(a.sinr);
    d.best_k = a.best_k;
    d.per_stream = reinterpret_cast<float*>(a.per_stream);
    return d;
}

// Point n in wavelengths (FP64).
__device__ __forceinline__ void point_rev(const PmMapDev& a, int64_t n, double& x, double& y,
                                          double& z) {
    point_xyz(a.P, 0, n, x, y, z);
    x *= a.inv_lam;
    y *= a.inv_lam;
    z *= a.inv_lam;
}

// Grid points of a workgroup, wg_first + o for 0 <= o < npts (npts <= 2^20),
// by their offset from the workgroup's first point (i0, j0): one division per
// workgroup, and none per point when the workgroup lies within one grid row.
// Coordinates as point_rev, so the same bits.
struct WgGrid {
    int64_t first, last;   // wg_first, and its last point clamped to N - 1
    int64_t i0, j0;
    bool one_row;
};

__device__ __forceinline__ WgGrid wg_grid(const PmMapDev& a, int64_t wg_first, int npts) {
    WgGrid w;
    w.first = wg_first;
    w.last = min(wg_first + (int64_t)npts, a.P.n) - 1;
    w.j0 = wg_first / a.P.nx;
    w.i0 = wg_first - w.j0 * a.P.nx;
    w.one_row = w.i0 + (w.last - wg_first) < a.P.nx;
    return w;
}

// Point min(wg_first + o, N - 1) in wavelengths.
__device__ __forceinline__ void wg_point_rev(const PmMapDev& a, const WgGrid& w, int o, double& x,
                                             double& y, double& z) {
    const int64_t oc = min((int64_t)o, w.last - w.first);
    int64_t i, j;
    if (w.one_row) {
        i = w.i0 + oc;
        j = w.j0;
    } else {
        const uint32_t u = (uint32_t)(w.i0 + oc), nx = (uint32_t)a.P.nx;
        const uint32_t q = u / nx;
        i = u - q * nx;
        j = w.j0 + q;
    }
    x = (a.P.x0 + ((double)i + 0.5) * a.P.dx) * a.inv_lam;
    y = (a.P.y0 + ((double)j + 0.5) * a.P.dy) * a.inv_lam;
    z = a.P.z * a.inv_lam;
}

// One spherical-wave term with every length in wavelengths.
//   d2 = dx^2 + dy^2 + dz^2 (FP64).
//   d  = sqrt(d2): an FP32 rsq seed refined by one FP64 Newton step
//        (relative error ~1.5 eps_seed^2 ~ 1e-13).
//   fr = frac(d): exact in FP64, i.e. the phase 2 pi d / lambda reduced
//        to [0, 1) revolutions.
//   h  = amp * (cos 2 pi fr - j sin 2 pi fr), with amp = 1 / (4 pi max(d, d_min)).
// The hardware sin / cos take revolutions directly.  `scale` multiplies the
// amplitude (the FP16 split path uses it to place h in the FP16 range).
// GUARD = false when the caller knows d2 >= 1.001 d_min^2: the zero guard of
// the reciprocal square root and the near-field clamp then change no bit
// (rs stays below 1 / d_min by far more than the instruction's one-ulp error)
// and are left out.
template <bool GUARD = true>
__device__ __forceinline__ void wave_term_rev_d2(double d2, float amp_scaled, float inv_dmin_rev,
                                                 float& hr, float& hi) {
    const float rs = __builtin_amdgcn_rsqf(GUARD ? fmaxf((float)d2, 1e-30f) : (float)d2);
    const double y = (double)rs;
    const double s0 = d2 * y;
    const double e = fma(-s0, s0, d2);
    const double d = fma(e, 0.5 * y, s0);
    const float fr = (float)__builtin_amdgcn_fract(d);
    const float amp = amp_scaled * (GUARD ? fminf(rs, inv_dmin_rev) : rs);
    hr = amp * __builtin_amdgcn_cosf(fr);
    hi = -amp * __builtin_amdgcn_sinf(fr);
}

__device__ __forceinline__ void wave_term_rev(double dx, double dy, double dz, float amp_scaled,
                                              float inv_dmin_rev, float& hr, float& hi) {
    wave_term_rev_d2(fma(dx, dx, fma(dy, dy, dz * dz)), amp_scaled, inv_dmin_rev, hr, hi);
}

// Column layouts of the output tiles (see the kernels):
//   NT = 1 (K <= 8):  column j < 8 is Re z_j, column j >= 8 is Im z_{j-8}.
//   NT = 2, 4:        tile 2q holds Re z_{16q+j}, tile 2q+1 holds Im z_{16q+j}.
template <int NT>
__device__ __forceinline__ void column_stream(int nt, int j, int& k, int& part) {
    if (NT == 1) {
        k = j & 7;
        part = j >> 3;
    } else {
        k = 16 * (nt >> 1) + j;
        part = nt & 1;
    }
}

// B1 = [wr | wi] multiplies hr; B2 = [-wi | wr] multiplies hi.
__device__ __forceinline__ float b_value(float2 w, int part, bool second) {
    if (!second) return part == 0 ? w.x : w.y;
    return part == 0 ? -w.y : w.x;
}

// Floats per point in the epilogue buffer: every column of a tile (re^2 and
// im^2 separately for NT = 1, stream powers for NT >= 2), padded by one.
template <int NT>
constexpr int ep_stride() {
    return NT == 1 ? 20 : (NT == 2 ? 17 : 33);
}

// LDS bytes of the epilogue buffer of a workgroup of WAVES wavefronts.
template <int NT, int PT, int WAVES>
constexpr int ep_bytes() {
    return WAVES * 16 * PT * ep_stride<NT>() * 4;
}

// The outputs of one map at output index idx from the powers p[0 .. GS - 1]
// of its streams (GS unrolled; zero powers past the map's G streams change
// nothing): power, SINR of the strongest stream, its index, and the G
// per-stream powers at idx G.
template <int GS>
__device__ __forceinline__ void ep_group(const PmMapDev& a, const float* p, int64_t idx,
                                         int64_t ps_idx, int G) {
    float y = 0.0f, pb = -1.0f;
    int kb = 0;
#pragma unroll
    for (int k = 0; k < GS; ++k) {
        y += p[k];
        if (p[k] > pb) {
            pb = p[k];
            kb = k;
        }
    }
    a.power[idx] = y;
    if (a.sinr) {
        float intf = 0.0f;
#pragma unroll
        for (int k = 0; k < GS; ++k) intf += k != kb ? p[k] : 0.0f;
        a.sinr[idx] = pb / (intf + a.sigma2);
    }
    if (a.best_k) a.best_k[idx] = kb;
    if (a.per_stream) {
        float* ps = a.per_stream + ps_idx * G;
#pragma unroll
        for (int k = 0; k < GS; ++k)
            if (k < G) ps[k] = p[k];
    }
}

// Epilogue of all PT x NT accumulator tiles of a wave.
//
// The per-stream powers go through LDS.  Lane (grp, col) holds D[4 grp + r][col]
// of every tile, and writes column col of its four rows.  Then lane p < 16 PT
// reads back point p's K powers.  It forms the total power, the best stream
// (largest power, lowest index on ties) and the interference of the others,
// accumulating in ascending stream order.  `ep` is this wave's slice of the
// buffer.  The caller has made sure the LDS is no longer used for anything
// else, and every thread of the workgroup calls this function.
template <int NT, int PT>
__device__ __forceinline__ void map_epilogue(const PmMapDev& a, const f32x4 (&acc)[PT][NT],
                                             int64_t base, int lane, float* ep) {
    constexpr int KS = ep_stride<NT>();
    const int grp = lane >> 4;
    const int col = lane & 15;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float* row = ep + (16 * t + 4 * grp + r) * KS;
            if constexpr (NT == 1) {
                const float v = acc[t][0][r];
                row[col] = v * v;                       // re^2 (col < 8) or im^2 (col >= 8)
            } else {
                const float re0 = acc[t][0][r], im0 = acc[t][1][r];
                row[col] = re0 * re0 + im0 * im0;
                if constexpr (NT == 4) {
                    const float re1 = acc[t][2][r], im1 = acc[t][3][r];
                    row[16 + col] = re1 * re1 + im1 * im1;
                }
            }
        }
    }
    __syncthreads();   // every thread of the workgroup reaches the epilogue
    if (lane >= 16 * PT) return;
    const int64_t n = base + lane;
    if (n >= a.P.n) return;
    const float* row = ep + lane * KS;
    const int K = a.K;
    if constexpr (NT == 1) {
        // all 16 columns at once (rows are 16-byte aligned), streams unrolled
        float v[16];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float4 q = reinterpret_cast<const float4*>(row)[c];
            v[4 * c] = q.x;
            v[4 * c + 1] = q.y;
            v[4 * c + 2] = q.z;
            v[4 * c + 3] = q.w;
        }
        float p[8];
        float y = 0.0f, pb = -1.0f;
        int kb = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            p[k] = k < K ? v[k] + v[8 + k] : 0.0f;
            y += p[k];
            if (k < K && p[k] > pb) {
                pb = p[k];
                kb = k;
            }
        }
        a.power[n] = y;
        if (a.sinr) {
            float intf = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k != kb) intf += p[k];
            a.sinr[n] = pb * __builtin_amdgcn_rcpf(intf + a.sigma2);
        }
        if (a.best_k) a.best_k[n] = kb;
        if (a.per_stream) {
            float* ps = a.per_stream + n * K;
            for (int k = 0; k < K; ++k) ps[k] = v[k] + v[8 + k];
        }
        return;
    }
    // one output map per group of G streams (G = K: one map)
    const int G = a.G;
    const int64_t N = a.P.n;
    if (G == K || G == 8) {
        // one map, or maps of 8 streams: the row's 8 NT columns loaded at once
        // (columns past K hold zero powers, which change no sum, maximum or
        // index below)
        constexpr int S = 8 * NT;
        float p[S];
#pragma unroll
        for (int k = 0; k < S; ++k) p[k] = row[k];
        if (G == K) {
            ep_group<S>(a, p, n, n, K);
        } else {
#pragma unroll
            for (int o = 0; o < S / 8; ++o)
                if (8 * o < K) ep_group<8>(a, p + 8 * o, o * N + n, o * N + n, 8);
        }
        return;
    }
    for (int g0 = 0, o = 0; g0 < K; g0 += G, ++o) {
        const float* rg = row + g0;
        float y = 0.0f, pb = -1.0f;
        int kb = 0;
        for (int k = 0; k < G; ++k) {
            const float p = rg[k];
            y += p;
            if (p > pb) {
                pb = p;
                kb = k;
            }
        }
        a.power[o * N + n] = y;
        if (a.sinr) {
            float intf = 0.0f;
            for (int k = 0; k < G; ++k)
                if (k != kb) intf += rg[k];
            a.sinr[o * N + n] = pb / (intf + a.sigma2);
        }
        if (a.best_k) a.best_k[o * N + n] = kb;
        if (a.per_stream) {
            float* ps = a.per_stream + (o * N + n) * G;
            for (int k = 0; k < G; ++k) ps[k] = rg[k];
        }
    }
}

}  // namespace dmimo
