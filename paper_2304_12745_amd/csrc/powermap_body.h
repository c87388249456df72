// Per-workgroup bodies of the matrix-core power maps, shared by the map
// kernels (one launch per map) and the serving kernel (many queries per launch).
//
// Power maps with the K-stream contraction on the matrix cores.
//
// z[n][k] = sum_m h[n][m] w[k][m] is a complex (N x M) x (M x K) product.  In
// real arithmetic
//     [Re z | Im z] = hr * B1 + hi * B2,   B1 = [wr | wi],  B2 = [-wi | wr],
// and every 16-column output tile is accumulated by MFMAs whose A operand is
// the synthesised channel (16 points x k antennas) and whose B operand is a
// table of weights staged in LDS.  Lanes synthesise exactly the A elements
// they hold; h never leaves registers.
//
// FP32 mode: v_mfma_f32_16x16x4_f32 (A: lane 16k + i holds A[i][k]; B: lane
// 16k + j holds B[k][j]).  A lane synthesises one term per 16-point tile and
// 4-antenna step.
//
// Mixed modes: v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation.  Lane
// 16g + i holds A[i][8g .. 8g+7] and B[8g .. 8g+7][i], so a lane synthesises
// 8 consecutive antennas of one point per 32-antenna step.  Every FP32 value
// x is split as x = hi + lo, with hi = x rounded to 16 bits and lo = the
// remainder rounded to 16 bits.  Three products accumulate:
// A_hi B_hi + A_lo B_hi + A_hi B_lo.  The dropped A_lo B_lo term and the
// rounding of lo leave ~2^-21 (FP16) or ~2^-16 (BF16) relative error per
// term (split-precision products: Markidis et al. 2018, Ootomo and Yokota
// 2022).
//   FP16 keeps both halves in its normal range by scaling.  h is scaled by
//   2^hexp (14 for the default near-field clamp, where |h| <= 1; less for a
//   smaller d_min, so that |h| 2^hexp <= 2^14).  The weights of each
//   64-antenna chunk are scaled by a power of two that puts their largest
//   magnitude in [2^13, 2^14): one scale per chunk in map_x3_wg, one per
//   chunk and stream in map_x3w_wg.  The accumulator is rescaled by the exact
//   ratio when a scale changes, and by the inverse scales at the end.
//   BF16 has the FP32 exponent range and needs no scaling.
//
// Output tile D: lane 16g + j holds D[4g + r][j] in register r.  Column
// layouts are in powermap_common.h.
#pragma once

#include <type_traits>

#include "powermap_common.h"
#include "split16.h"

namespace dmimo {

constexpr int kChunk = 64;   // antennas per LDS stage

// ---------------------------------------------------------------------------
// FP32 VALU (K <= 2): one lane per point
// ---------------------------------------------------------------------------
//
// All lanes of a wavefront walk the antennas in the same order, so each
// antenna's position and its weights are wave-uniform: the compiler keeps
// them in scalar registers (scalar loads), and the VALU only synthesises h and
// runs the K complex MACs (4 or 8 FMA per term).  The reduction over antennas
// stays inside one lane in ascending m.

template <int KT>
__device__ __forceinline__ void map_valu_wg(const PmMapDev& a, int64_t wg_first) {
    const int64_t n = wg_first + threadIdx.x;
    const bool live = n < a.P.n;
    double px, py, pz;
    point_rev(a, live ? n : a.P.n - 1, px, py, pz);
    const int M = a.M;
    const float2* __restrict__ W = a.W;
    const double* __restrict__ ap = a.ap;
    float zr[KT], zi[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        zr[k] = 0.0f;
        zi[k] = 0.0f;
    }
    for (int m = 0; m < M; ++m) {
        float hr, hi;
        wave_term_rev(fma(-ap[3 * m + 0], a.inv_lam, px), fma(-ap[3 * m + 1], a.inv_lam, py),
                      fma(-ap[3 * m + 2], a.inv_lam, pz), a.amp_rev, a.inv_dmin_rev, hr, hi);
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const float2 w = W[(int64_t)k * M + m];
            zr[k] = fmaf(hr, w.x, fmaf(-hi, w.y, zr[k]));
            zi[k] = fmaf(hr, w.y, fmaf(hi, w.x, zi[k]));
        }
    }
    if (!live) return;
    float p[KT];
    float y = 0.0f, pb = -1.0f;
    int kb = 0;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        p[k] = zr[k] * zr[k] + zi[k] * zi[k];
        y += p[k];
        if (p[k] > pb) {
            pb = p[k];
            kb = k;
        }
    }
    a.power[n] = y;
    if (a.sinr) {
        float intf = 0.0f;
#pragma unroll
        for (int k = 0; k < KT; ++k)
            if (k != kb) intf += p[k];
        a.sinr[n] = pb / (intf + a.sigma2);
    }
    if (a.best_k) a.best_k[n] = kb;
    if (a.per_stream) {
#pragma unroll
        for (int k = 0; k < KT; ++k) a.per_stream[n * KT + k] = p[k];
    }
}

// ---------------------------------------------------------------------------
// FP32 MFMA
// ---------------------------------------------------------------------------

template <int NT, int PT, int WAVES>
constexpr int f32_lds_bytes() {
    constexpr int TB = kChunk * 3 * 8 + kChunk * (NT * 32 + 16) * 4;
    return TB > ep_bytes<NT, PT, WAVES>() ? TB : ep_bytes<NT, PT, WAVES>();
}

// One workgroup of the FP32 map: points wg_first .. wg_first + 16 PT WAVES - 1.
// smem: at least f32_lds_bytes<NT, PT, WAVES>() bytes, 16-byte aligned.
// The antenna steps of one LDS chunk: each step synthesises PT terms per lane
// (antenna 4 s + grp) and feeds them to the MFMAs.  ROW: slot 1 of s_ap holds
// fma(dy, dy, dz * dz) of the workgroup's grid row.
template <int NT, int PT, bool ROW, bool GUARD = true>
__device__ __forceinline__ void f32_steps(const PmMapDev& a, int steps, int grp, int col,
                                          const double* s_ap, const float* s_b, const double (&px)[PT],
                                          const double (&py)[PT], const double (&pz)[PT],
                                          f32x4 (&acc)[PT][NT]) {
    constexpr int BS = NT * 32 + 16;
    for (int s = 0; s < steps; ++s) {
        const int mm = 4 * s + grp;
        float hr[PT], hi[PT];
        if constexpr (ROW) {
            const double ax = s_ap[mm * 3 + 0];
            const double c = s_ap[mm * 3 + 1];
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                const double dx = px[t] - ax;
                wave_term_rev_d2<GUARD>(fma(dx, dx, c), 1.0f, a.inv_dmin_rev, hr[t], hi[t]);
            }
        } else {
            const double ax = s_ap[mm * 3 + 0];
            const double ay = s_ap[mm * 3 + 1];
            const double az = s_ap[mm * 3 + 2];
#pragma unroll
            for (int t = 0; t < PT; ++t)
                wave_term_rev(px[t] - ax, py[t] - ay, pz[t] - az, 1.0f, a.inv_dmin_rev, hr[t],
                              hi[t]);
        }
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const float b1 = s_b[mm * BS + q * 32 + col];
            const float b2 = s_b[mm * BS + q * 32 + 16 + col];
#pragma unroll
            for (int t = 0; t < PT; ++t)
                acc[t][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(hr[t], b1, acc[t][q], 0, 0, 0);
#pragma unroll
            for (int t = 0; t < PT; ++t)
                acc[t][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(hi[t], b2, acc[t][q], 0, 0, 0);
        }
    }
}

template <int NT, int PT, int WAVES>
__device__ __forceinline__ void map_f32_wg(const PmMapDev& a, int64_t wg_first, char* smem) {
    constexpr int NTH = 64 * WAVES;
    constexpr int BS = NT * 32 + 16;   // floats per antenna row (padded: disjoint banks per group)
    double* s_ap = reinterpret_cast<double*>(smem);
    float* s_b = reinterpret_cast<float*>(smem + kChunk * 3 * 8);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;
    const int grp = lane >> 4;
    const int64_t N = a.P.n;
    const int M = a.M;
    const int K = a.K;
    const int64_t base = wg_first + (int64_t)wave * (16 * PT);

    const bool grid = a.P.kind == DMIMO_PTS_GRID;
    const WgGrid wg = grid ? wg_grid(a, wg_first, 16 * PT * WAVES) : WgGrid{};
    double px[PT], py[PT], pz[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        if (grid) {
            wg_point_rev(a, wg, wave * (16 * PT) + 16 * t + col, px[t], py[t], pz[t]);
        } else {
            int64_t n = base + 16 * t + col;
            n = n < N ? n : N - 1;
            point_rev(a, n, px[t], py[t], pz[t]);
        }
    }

    f32x4 acc[PT][NT];
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};

    // When every point of the workgroup lies on one grid row, y and z are the
    // same for all of them, so fma(dy, dy, dz * dz) is formed once per antenna
    // (slot 1 of s_ap) and a term needs only dx: d2 = fma(dx, dx, C), the
    // same bits as the general path.  A chunk whose antennas all have
    // C >= 1.001 d_min^2 (every antenna off the row by more than d_min, as
    // for a map plane below ceiling access points) gives d2 >= C for every
    // term, so it runs without the zero guard and the near-field clamp (K <= 8,
    // where the synthesis bounds the kernel; wider kernels are MFMA-heavy and
    // keep one loop).
    // Padding slots take C = 1 (wavelengths squared, far above d_min^2) and
    // multiply zero weights.
    bool row = false;
    double ry = 0.0, rz = 0.0;
    const double dmin_rev = 1.0 / (double)a.inv_dmin_rev;
    const double far_c = 1.001 * dmin_rev * dmin_rev;
    if (grid) {
        row = wg.one_row;
        double rx;
        wg_point_rev(a, wg, 0, rx, ry, rz);
    }

    for (int m0 = 0; m0 < M; m0 += kChunk) {
        const int mc = min(kChunk, M - m0);
        __syncthreads();
        if (row) {
            for (int mm = tid; mm < kChunk; mm += NTH) {
                double ax = 0.0, c = 1.0;
                if (mm < mc) {
                    const double* q = a.ap + (int64_t)(m0 + mm) * 3;
                    ax = q[0] * a.inv_lam;
                    const double dy = ry - q[1] * a.inv_lam, dz = rz - q[2] * a.inv_lam;
                    c = fma(dy, dy, dz * dz);
                }
                s_ap[mm * 3 + 0] = ax;
                s_ap[mm * 3 + 1] = c;
            }
        } else {
            for (int e = tid; e < kChunk * 3; e += NTH) {
                const int mm = e / 3;
                s_ap[e] = mm < mc ? a.ap[(int64_t)(m0 + mm) * 3 + (e - 3 * mm)] * a.inv_lam : 0.0;
            }
        }
        for (int e = tid; e < kChunk * NT * 16; e += NTH) {
            const int mm = e / (NT * 16);
            const int r = e - mm * (NT * 16);
            const int q = r >> 4;
            const int j = r & 15;
            int k, part;
            column_stream<NT>(q, j, k, part);
            float2 w = make_float2(0.f, 0.f);
            if (k < K && mm < mc) {
                // the constant amplitude factor 1 / (4 pi) rides on W (the sums
                // are linear in it), so a term's amplitude is min(1/d, 1/d_min)
                w = a.W[(int64_t)k * M + m0 + mm];
                w = make_float2(a.amp_rev * w.x, a.amp_rev * w.y);
            }
            s_b[mm * BS + q * 32 + j] = b_value(w, part, false);
            s_b[mm * BS + q * 32 + 16 + j] = b_value(w, part, true);
        }
        __syncthreads();
        const int steps = (mc + 3) >> 2;
        if (NT == 1 && row && __all(s_ap[lane * 3 + 1] >= far_c))
            f32_steps<NT, PT, true, false>(a, steps, grp, col, s_ap, s_b, px, py, pz, acc);
        else if (row)
            f32_steps<NT, PT, true>(a, steps, grp, col, s_ap, s_b, px, py, pz, acc);
        else
            f32_steps<NT, PT, false>(a, steps, grp, col, s_ap, s_b, px, py, pz, acc);
    }
    __syncthreads();
    map_epilogue<NT, PT>(a, acc, base, lane,
                         reinterpret_cast<float*>(smem) + wave * 16 * PT * ep_stride<NT>());
}

// ---------------------------------------------------------------------------
// split-precision x3 (FP16 / BF16)
// ---------------------------------------------------------------------------


// LDS of the x3 map: the B tables of the two 32-antenna steps of a chunk,
// [step][tile][B1hi, B1lo, B2hi, B2lo][lane] x 16 B, and the antenna
// positions (wavelengths, SoA).  The epilogue reuses the same bytes.
template <int NT>
struct X3Tables {
    u32x4 b[2][NT][4][64];
    double x[kChunk], y[kChunk], z[kChunk];
};

template <int NT, int PT, int WAVES>
constexpr int x3_lds_bytes() {
    return (int)sizeof(X3Tables<NT>) > ep_bytes<NT, PT, WAVES>() ? (int)sizeof(X3Tables<NT>)
                                                                  : ep_bytes<NT, PT, WAVES>();
}

// One workgroup of the split-precision map: points wg_first .. + 16 PT WAVES - 1.
// smem: at least x3_lds_bytes<NT, PT, WAVES>() bytes; s_red: WAVES floats.
// The antenna steps of one chunk in the split-precision body: each lane
// synthesises 8 consecutive antennas of each of its PT points, splits them
// into hi / lo halves and runs the three products per tile.  ROW: table y
// holds fma(dy, dy, dz * dz) of the workgroup's grid row.
template <int NT, int PT, bool BF16, bool ROW>
__device__ __forceinline__ void x3_steps(const PmMapDev& a, const X3Tables<NT>& T, int steps, int grp,
                                         int lane, float amp_s, const double (&px)[PT],
                                         const double (&py)[PT], const double (&pz)[PT],
                                         f32x4 (&acc)[PT][NT]) {
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            u32x4 arh, arl, aih, ail;
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                const int mm = 32 * s + 8 * grp + i;
                float hr0, hi0, hr1, hi1;
                if constexpr (ROW) {
                    const double dx0 = px[t] - T.x[mm], dx1 = px[t] - T.x[mm + 1];
                    wave_term_rev_d2(fma(dx0, dx0, T.y[mm]), amp_s, a.inv_dmin_rev, hr0, hi0);
                    wave_term_rev_d2(fma(dx1, dx1, T.y[mm + 1]), amp_s, a.inv_dmin_rev, hr1, hi1);
                } else {
                    wave_term_rev(px[t] - T.x[mm], py[t] - T.y[mm], pz[t] - T.z[mm], amp_s,
                                  a.inv_dmin_rev, hr0, hi0);
                    wave_term_rev(px[t] - T.x[mm + 1], py[t] - T.y[mm + 1], pz[t] - T.z[mm + 1],
                                  amp_s, a.inv_dmin_rev, hr1, hi1);
                }
                float rr0, rr1, ri0, ri1;
                arh[i >> 1] = pack_hi<BF16>(hr0, hr1, rr0, rr1);
                aih[i >> 1] = pack_hi<BF16>(hi0, hi1, ri0, ri1);
                arl[i >> 1] = pack_lo<BF16>(rr0, rr1);
                ail[i >> 1] = pack_lo<BF16>(ri0, ri1);
            }
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const u32x4 b1h = T.b[s][q][0][lane], b1l = T.b[s][q][1][lane];
                const u32x4 b2h = T.b[s][q][2][lane], b2l = T.b[s][q][3][lane];
                f32x4 c = acc[t][q];
                c = mfma16<BF16>(arh, b1h, c);
                c = mfma16<BF16>(arl, b1h, c);
                c = mfma16<BF16>(arh, b1l, c);
                c = mfma16<BF16>(aih, b2h, c);
                c = mfma16<BF16>(ail, b2h, c);
                c = mfma16<BF16>(aih, b2l, c);
                acc[t][q] = c;
            }
        }
    }
}

// ROWS: allow the grid-row step loop (a second copy of the loop; the serving
// kernels, which hold more state, keep one copy and stay within 128 VGPRs).
template <int NT, int PT, bool BF16, int WAVES, bool ROWS = true>
__device__ __forceinline__ void map_x3_wg(const PmMapDev& a, int64_t wg_first, char* smem,
                                          float* s_red) {
    constexpr int NTH = 64 * WAVES;
    X3Tables<NT>& T = *reinterpret_cast<X3Tables<NT>*>(smem);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int grp = lane >> 4;
    const int64_t N = a.P.n;
    const int M = a.M;
    const int K = a.K;
    const int64_t base = wg_first + (int64_t)wave * (16 * PT);
    const int hexp = BF16 ? 0 : a.hexp;   // FP16 range placement of h
    const float amp_s = ldexpf(a.amp_rev, hexp);

    const bool grid = a.P.kind == DMIMO_PTS_GRID;
    const WgGrid wg = grid ? wg_grid(a, wg_first, 16 * PT * WAVES) : WgGrid{};
    double px[PT], py[PT], pz[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        if (grid) {
            wg_point_rev(a, wg, wave * (16 * PT) + 16 * t + (lane & 15), px[t], py[t], pz[t]);
        } else {
            int64_t n = base + 16 * t + (lane & 15);
            n = n < N ? n : N - 1;
            point_rev(a, n, px[t], py[t], pz[t]);
        }
    }

    // One accumulator per tile.  For FP16 it holds the sum so far in units of
    // the current chunk's weight scale, and is rescaled (exactly, by a power
    // of two) when the scale changes.
    f32x4 acc[PT][NT];
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    int wexp = 0;   // current chunk weight scale 2^wexp (FP16)

    // grid-row workgroups form (y - a_y)^2 + (z - a_z)^2 once per antenna, as
    // the FP32 body does (the same d2 bits).  Only for FP16 and NT >= 2: at
    // NT = 1 the second copy of the step loop would push the body past 128
    // VGPRs, and the BF16 body measured slower with it (hall map 7.50 vs
    // 7.03 ms, against 7.18 vs 7.65 ms for FP16).
    constexpr bool kRows = ROWS && NT >= 2 && !BF16;
    bool row = false;
    double ry = 0.0, rz = 0.0;
    if (kRows && grid) {
        row = wg.one_row;
        double rx;
        wg_point_rev(a, wg, 0, rx, ry, rz);
    }

    // table item of this thread: (step, tile, lane) = 8 antennas
    // 32 step + 8 (lane / 16) + i of column lane % 16 of the tile
    constexpr int kItems = 2 * NT * 64;
    for (int m0 = 0; m0 < M; m0 += kChunk) {
        const int mc = min(kChunk, M - m0);
        __syncthreads();
        constexpr int kPer = (kItems + NTH - 1) / NTH;
        float2 wv[kPer][8];
        float mx = 0.0f;
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int e = tid + NTH * it;
            const int s = e / (NT * 64);
            const int q = (e - s * NT * 64) >> 6;
            const int l = e & 63;
            int k, part;
            column_stream<NT>(q, l & 15, k, part);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int mm = 32 * s + 8 * (l >> 4) + i;
                float2 w = make_float2(0.f, 0.f);
                if (e < kItems && k < K && mm < mc) w = a.W[(int64_t)k * M + m0 + mm];
                wv[it][i] = w;
                mx = fmaxf(mx, fmaxf(fabsf(w.x), fabsf(w.y)));
            }
        }
        for (int e = tid; e < kChunk; e += NTH) {
            const bool live = e < mc;
            T.x[e] = live ? a.ap[(int64_t)(m0 + e) * 3 + 0] * a.inv_lam : 0.0;
            if (row) {         // slot y holds fma(dy, dy, dz * dz) of the workgroup's row
                double c = 0.0;
                if (live) {
                    const double dy = ry - a.ap[(int64_t)(m0 + e) * 3 + 1] * a.inv_lam;
                    const double dz = rz - a.ap[(int64_t)(m0 + e) * 3 + 2] * a.inv_lam;
                    c = fma(dy, dy, dz * dz);
                }
                T.y[e] = c;
            } else {
                T.y[e] = live ? a.ap[(int64_t)(m0 + e) * 3 + 1] * a.inv_lam : 0.0;
                T.z[e] = live ? a.ap[(int64_t)(m0 + e) * 3 + 2] * a.inv_lam : 0.0;
            }
        }
        float wscale = 1.0f;
        if constexpr (!BF16) {
            // chunk weight scale 2^(14 - e) with max |w| < 2^e
            for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_down(mx, off, 64));
            if (lane == 0) s_red[wave] = mx;
            __syncthreads();
            mx = s_red[0];
#pragma unroll
            for (int i = 1; i < WAVES; ++i) mx = fmaxf(mx, s_red[i]);
            const int ne = mx > 0.0f ? 14 - (ilogbf(mx) + 1) : wexp;
            if (m0 > 0 && ne != wexp) {
                const float f = ldexpf(1.0f, ne - wexp);
#pragma unroll
                for (int t = 0; t < PT; ++t)
#pragma unroll
                    for (int q = 0; q < NT; ++q) acc[t][q] *= f;
            }
            wexp = ne;
            wscale = ldexpf(1.0f, wexp);
        }
#pragma unroll
        for (int it = 0; it < kPer; ++it) {
            const int e = tid + NTH * it;
            if (e >= kItems) break;
            const int s = e / (NT * 64);
            const int q = (e - s * NT * 64) >> 6;
            const int l = e & 63;
            int k, part;
            column_stream<NT>(q, l & 15, k, part);
            u32x4 pk[4];
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
#pragma unroll
                for (int which = 0; which < 2; ++which) {
                    const float x0 = b_value(wv[it][i], part, which == 1) * wscale;
                    const float x1 = b_value(wv[it][i + 1], part, which == 1) * wscale;
                    float b0, b1, c0, c1;
                    const uint32_t h0 = to16<BF16>(x0, b0), h1 = to16<BF16>(x1, b1);
                    const uint32_t l0 = to16<BF16>(x0 - b0, c0), l1 = to16<BF16>(x1 - b1, c1);
                    pk[2 * which][i >> 1] = h0 | (h1 << 16);
                    pk[2 * which + 1][i >> 1] = l0 | (l1 << 16);
                }
            }
#pragma unroll
            for (int wh = 0; wh < 4; ++wh) T.b[s][q][wh][l] = pk[wh];
        }
        __syncthreads();
        const int steps = (mc + 31) >> 5;
        if (kRows && row)
            x3_steps<NT, PT, BF16, kRows>(a, T, steps, grp, lane, amp_s, px, py, pz, acc);
        else
            x3_steps<NT, PT, BF16, false>(a, T, steps, grp, lane, amp_s, px, py, pz, acc);
    }
    // undo the scales (exact powers of two)
    const float inv = BF16 ? 1.0f : ldexpf(1.0f, -wexp - hexp);
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[t][q] *= inv;
    __syncthreads();
    map_epilogue<NT, PT>(a, acc, base, lane,
                         reinterpret_cast<float*>(smem) + wave * 16 * PT * ep_stride<NT>());
}

// ---------------------------------------------------------------------------
// split-precision x3 for many streams (K > 8): several tiles per wave
// ---------------------------------------------------------------------------
//
// The same products as map_x3_wg, arranged for NT = 2 or 4 output tiles:
//  * a wave holds PT tiles of 16 points, so each split weight table in LDS
//    feeds PT tiles, and a workgroup stages one table per chunk for
//    16 PT WAVES points;
//  * the weights of the next chunk are loaded into registers while the
//    current chunk runs, and split into the other of two LDS buffers during
//    it;
//  * the two waves of a SIMD run half a step apart, so that the synthesis of
//    one overlaps the products of the other (four barriers per chunk);
//  * FP16 weights are scaled per chunk and stream: the eight threads that
//    stage one stream of a chunk are eight consecutive lanes, which find the
//    stream's largest magnitude among themselves (no cross-wave step);
//  * a grid-row workgroup whose chunk lies more than d_min below or beside the
//    row synthesises without the zero guard and the near-field clamp, which
//    change no bit there (as in the FP32 body).
// Accumulation order per output is fixed (chunks, then steps, then the six
// products in a fixed order), so a point's value does not depend on which
// workgroup or launch computes it.

// Slot of lane l's 16 bytes in a table row of step s.  The XOR spreads the
// eight lanes that a 16-byte LDS access serves together over eight distinct
// bank groups, both for the staging stores (lanes 16 g + k of one stream k,
// g = 0..3, in both steps) and for the operand loads (eight consecutive lanes).
__device__ __forceinline__ int x3w_slot(int l, int s) { return l ^ ((2 * (l >> 4) + s) & 7); }

template <int NT>
struct X3wBuf {
    u32x4 b[2][NT][4][64];                   // [step][tile][B1hi, B1lo, B2hi, B2lo][x3w_slot(lane)]
    double x[kChunk], y[kChunk], z[kChunk];  // antennas in wavelengths; grid row: y = C
    int32_t wexp[8 * NT];                    // FP16: scale exponent of each stream
    int32_t far;                             // grid row: C >= 1.001 d_min^2 for every antenna
    int32_t pad[3];
};

template <int NT, int PT, int WAVES>
constexpr int x3w_lds_bytes() {
    constexpr int T = 2 * (int)sizeof(X3wBuf<NT>);
    return T > ep_bytes<NT, PT, WAVES>() ? T : ep_bytes<NT, PT, WAVES>();
}

// Registers of one thread's share of the next chunk: the 8 weights of its
// staging item and, for threads 0..63, one antenna position.
struct X3wStage {
    float2 w[8];
    double ax, ay, az;
    int wexp;   // FP16: exponent of this thread's stream in the chunk staged last
    bool set;   // FP16: wexp has been chosen (the stream had a nonzero weight)
};

// Staging item of thread tid < 64 NT: stream k = tid / 8 and antennas
// 8 (tid % 8) .. 8 (tid % 8) + 7 of the chunk starting at m0.
template <int NT>
__device__ __forceinline__ void x3w_load(const PmMapDev& a, int m0, int tid, X3wStage& st) {
    const int M = a.M;
    const int mc = min(kChunk, M - m0);
    if (tid < 64 * NT) {
        const int k = tid >> 3;
        const int a8 = 8 * (tid & 7);
        const float2* src = a.W + (int64_t)k * M + m0 + a8;
        if (k < a.K && a8 + 8 <= mc) {
#pragma unroll
            for (int i = 0; i < 8; ++i) st.w[i] = src[i];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                st.w[i] = (k < a.K && a8 + i < mc) ? src[i] : make_float2(0.f, 0.f);
        }
    }
    if (tid < kChunk && tid < mc) {
        const double* q = a.ap + (int64_t)(m0 + tid) * 3;
        st.ax = q[0];
        st.ay = q[1];
        st.az = q[2];
    }
}

// Split the staged chunk into buffer T (every thread of the workgroup calls
// this).  Slots past the last antenna get zero weights and position x = 0,
// C = 1 (far from any row), or (0, 0, 0) off grid rows.
template <int NT, bool BF16>
__device__ __forceinline__ void x3w_write(const PmMapDev& a, X3wBuf<NT>& T, int m0, int tid,
                                          X3wStage& st, bool row, double ry, double rz,
                                          double far_c) {
    const int mc = min(kChunk, a.M - m0);
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mx = fmaxf(mx, fmaxf(fabsf(st.w[i].x), fabsf(st.w[i].y)));
    // the largest magnitude of the stream: its 8 items are lanes 8j .. 8j + 7
    // (DPP: swap neighbours, swap pairs, mirror within 8 lanes)
    mx = fmaxf(mx, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
                       __builtin_bit_cast(int, mx), 0xB1, 0xF, 0xF, false)));   // quad_perm [1,0,3,2]
    mx = fmaxf(mx, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
                       __builtin_bit_cast(int, mx), 0x4E, 0xF, 0xF, false)));   // quad_perm [2,3,0,1]
    mx = fmaxf(mx, __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
                       __builtin_bit_cast(int, mx), 0x141, 0xF, 0xF, false)));  // row_half_mirror
    if (tid < 64 * NT) {
        const int k = tid >> 3;
        const int g8 = tid & 7;
        // FP16: the first nonzero chunk of a stream gets the scale 2^(14 - e),
        // max |w| < 2^e, which puts its largest weight in [2^13, 2^14).  Later
        // chunks keep the scale while their scaled largest weight stays in
        // [2^4, 2^15) (FP16 normal, 11 bits for every weight within 2^-18 of
        // it), so the accumulators rarely need rescaling.  The scale is applied
        // by ldexp (exact, and no overflow of the factor itself).
        if (!BF16 && mx > 0.0f) {
            const int e = ilogbf(mx) + 1;
            if (!st.set || e + st.wexp > 15 || e + st.wexp < 5) {
                st.wexp = 14 - e;
                st.set = true;
            }
        }
        const int ex = BF16 ? 0 : st.wexp;
        u32x4 rh, rl, ih, il;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            float r0, r1, q0, q1;
            rh[i >> 1] = pack_hi<BF16>(ldexpf(st.w[i].x, ex), ldexpf(st.w[i + 1].x, ex), r0, r1);
            ih[i >> 1] = pack_hi<BF16>(ldexpf(st.w[i].y, ex), ldexpf(st.w[i + 1].y, ex), q0, q1);
            rl[i >> 1] = pack_lo<BF16>(r0, r1);
            il[i >> 1] = pack_lo<BF16>(q0, q1);
        }
        // hi(-x) = -hi(x) and lo(-x) = -lo(x) (both roundings are symmetric)
        const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        const int s = g8 >> 2;
        const int l = x3w_slot(16 * (g8 & 3) + (k & 15), s);
        const int qr = 2 * (k >> 4);
        // tile qr: Re z = hr wr - hi wi;  tile qr + 1: Im z = hr wi + hi wr
        T.b[s][qr][0][l] = rh;
        T.b[s][qr][1][l] = rl;
        T.b[s][qr][2][l] = ih ^ sgn;
        T.b[s][qr][3][l] = il ^ sgn;
        T.b[s][qr + 1][0][l] = ih;
        T.b[s][qr + 1][1][l] = il;
        T.b[s][qr + 1][2][l] = rh;
        T.b[s][qr + 1][3][l] = rl;
        if (g8 == 0) T.wexp[k] = st.wexp;
    }
    if (tid < kChunk) {
        const bool live = tid < mc;
        const double x = live ? st.ax * a.inv_lam : 0.0;
        T.x[tid] = x;
        if (row) {
            double c = 1.0;
            if (live) {
                const double dy = ry - st.ay * a.inv_lam, dz = rz - st.az * a.inv_lam;
                c = fma(dy, dy, dz * dz);
            }
            T.y[tid] = c;
            const bool all_far = __all(c >= far_c);   // wave 0: the 64 slots of the chunk
            if (tid == 0) T.far = all_far ? 1 : 0;
        } else {
            T.y[tid] = live ? st.ay * a.inv_lam : 0.0;
            T.z[tid] = live ? st.az * a.inv_lam : 0.0;
        }
    }
}

// The 8 terms of one point (antennas xs[i] of this lane's group) as the four
// split A operands.
template <bool BF16, bool ROW, bool GUARD>
__device__ __forceinline__ void x3w_synth(double px, double py, double pz, const double (&xs)[8],
                                          const double (&ys)[8], const double (&zs)[8], float amp_s,
                                          float inv_dmin_rev, u32x4& arh, u32x4& arl, u32x4& aih,
                                          u32x4& ail) {
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        float hr0, hi0, hr1, hi1;
        if constexpr (ROW) {
            const double dx0 = px - xs[i], dx1 = px - xs[i + 1];
            wave_term_rev_d2<GUARD>(fma(dx0, dx0, ys[i]), amp_s, inv_dmin_rev, hr0, hi0);
            wave_term_rev_d2<GUARD>(fma(dx1, dx1, ys[i + 1]), amp_s, inv_dmin_rev, hr1, hi1);
        } else {
            wave_term_rev(px - xs[i], py - ys[i], pz - zs[i], amp_s, inv_dmin_rev, hr0, hi0);
            wave_term_rev(px - xs[i + 1], py - ys[i + 1], pz - zs[i + 1], amp_s, inv_dmin_rev, hr1,
                          hi1);
        }
        float rr0, rr1, ri0, ri1;
        arh[i >> 1] = pack_hi<BF16>(hr0, hr1, rr0, rr1);
        aih[i >> 1] = pack_hi<BF16>(hi0, hi1, ri0, ri1);
        arl[i >> 1] = pack_lo<BF16>(rr0, rr1);
        ail[i >> 1] = pack_lo<BF16>(ri0, ri1);
    }
}

// Positions of this lane's 8 antennas in step s of the chunk.
template <int NT, bool ROW>
__device__ __forceinline__ void x3w_positions(const X3wBuf<NT>& T, int s, int grp, double (&xs)[8],
                                              double (&ys)[8], double (&zs)[8]) {
    const int m8 = 32 * s + 8 * grp;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        xs[i] = T.x[m8 + i];
        ys[i] = T.y[m8 + i];
        zs[i] = ROW ? 0.0 : T.z[m8 + i];
    }
}

// The terms of one step (32 antennas, positions xs, ys, zs of this lane's 8)
// for the PT tiles of a wave, as split A operands.
template <int PT, bool BF16, bool ROW, bool GUARD>
__device__ __forceinline__ void x3w_synth_step(const double (&xs)[8], const double (&ys)[8],
                                               const double (&zs)[8], float amp_s,
                                               float inv_dmin_rev, const double (&px)[PT],
                                               const double (&py)[PT], const double (&pz)[PT],
                                               u32x4 (&A)[PT][4]) {
#pragma unroll
    for (int t = 0; t < PT; ++t)
        x3w_synth<BF16, ROW, GUARD>(px[t], py[t], pz[t], xs, ys, zs, amp_s, inv_dmin_rev, A[t][0],
                                    A[t][1], A[t][2], A[t][3]);
}

// The products of step s for the PT tiles of a wave (slots past the last
// antenna carry zero weights); each B operand is loaded once for the PT tiles.
template <int NT, int PT, bool BF16>
__device__ __forceinline__ void x3w_mma_step(const X3wBuf<NT>& T, int s, int lane,
                                             const u32x4 (&A)[PT][4], f32x4 (&acc)[PT][NT]) {
    const int sl = x3w_slot(lane, s);
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const u32x4 b1h = T.b[s][q][0][sl], b1l = T.b[s][q][1][sl];
        const u32x4 b2h = T.b[s][q][2][sl], b2l = T.b[s][q][3][sl];
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            f32x4 c = acc[t][q];
            c = mfma16<BF16>(A[t][0], b1h, c);
            c = mfma16<BF16>(A[t][1], b1h, c);
            c = mfma16<BF16>(A[t][0], b1l, c);
            c = mfma16<BF16>(A[t][2], b2h, c);
            c = mfma16<BF16>(A[t][3], b2h, c);
            c = mfma16<BF16>(A[t][2], b2l, c);
            acc[t][q] = c;
        }
    }
}

// A workgroup barrier that the compiler schedules nothing across, so that the
// VALU phase and the matrix-core phase of a wave stay on their sides of it.
__device__ __forceinline__ void x3w_phase_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
}

// One workgroup: points wg_first .. wg_first + 16 PT WAVES - 1.  smem: at
// least x3w_lds_bytes<NT, PT, WAVES>() bytes, 16-byte aligned.
template <int NT, int PT, bool BF16, int WAVES>
__device__ __forceinline__ void map_x3w_wg(const PmMapDev& a, int64_t wg_first, char* smem) {
    static_assert(NT == 2 || NT == 4, "map_x3w_wg: 16 < K <= 32 or 8 < K <= 16");
    static_assert(64 * NT <= 64 * WAVES, "map_x3w_wg: one staging item per thread");
    X3wBuf<NT>* buf = reinterpret_cast<X3wBuf<NT>*>(smem);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int grp = lane >> 4;
    const int64_t N = a.P.n;
    const int M = a.M;
    const int64_t base = wg_first + (int64_t)wave * (16 * PT);
    const int hexp = BF16 ? 0 : a.hexp;
    const float amp_s = ldexpf(a.amp_rev, hexp);
    // the first chunk's weights and antenna positions, loaded before the
    // points are located so that their latency overlaps that arithmetic
    X3wStage st;
    st.wexp = 0;
    st.set = false;
    x3w_load<NT>(a, 0, tid, st);

    const bool grid = a.P.kind == DMIMO_PTS_GRID;
    const WgGrid wg = grid ? wg_grid(a, wg_first, 16 * PT * WAVES) : WgGrid{};
    double px[PT], py[PT], pz[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        if (grid) {
            wg_point_rev(a, wg, wave * (16 * PT) + 16 * t + (lane & 15), px[t], py[t], pz[t]);
        } else {
            int64_t n = base + 16 * t + (lane & 15);
            n = n < N ? n : N - 1;
            point_rev(a, n, px[t], py[t], pz[t]);
        }
    }
    const bool row = grid && wg.one_row;
    double ry = 0.0, rz = 0.0;
    if (row) {
        double rx;
        wg_point_rev(a, wg, 0, rx, ry, rz);
    }
    const double dmin_rev = 1.0 / (double)a.inv_dmin_rev;
    const double far_c = 1.001 * dmin_rev * dmin_rev;

    f32x4 acc[PT][NT];
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    int cur[NT / 2];   // FP16: exponent of this lane's column in each 16-stream block
#pragma unroll
    for (int b = 0; b < NT / 2; ++b) cur[b] = 0;

    const int nch = (M + kChunk - 1) / kChunk;
    // Waves w and w + 4 share a SIMD.  The second half of the workgroup runs
    // every step one phase behind the first: while one wave synthesises the
    // terms of a step on the VALU, the other runs the products of its last
    // step on the matrix cores, and a barrier ends each phase.  A products
    // phase also reads the antenna positions of the wave's next step, so that
    // its synthesis phase starts without waiting for LDS.  The weights of chunk
    // c + 1 are staged in the products phase of chunk c's first step: after the
    // last read of their buffer (chunk c - 1, ended by the barrier that opens
    // that phase for either half) and at least one barrier before the first
    // read of chunk c + 1 (the positions, in the products phase of chunk c's
    // second step).
    static_assert(WAVES == 8, "map_x3w_wg: two waves per SIMD");
    const bool late = wave >= 4;
    // the chunk loop, compiled once for grid-row workgroups and once for the
    // others (one copy of the accumulators per loop)
    auto run = [&](auto row_tag) {
        constexpr bool ROW = decltype(row_tag)::value;
        x3w_write<NT, BF16>(a, buf[0], 0, tid, st, ROW, ry, rz, far_c);
        if (nch > 1) x3w_load<NT>(a, kChunk, tid, st);
        __syncthreads();
        double xs[8], ys[8], zs[8];
        x3w_positions<NT, ROW>(buf[0], 0, grp, xs, ys, zs);
        bool guard = !ROW || !buf[0].far;
        if (late) x3w_phase_barrier();
        for (int c = 0; c < nch; ++c) {
            const X3wBuf<NT>& T = buf[c & 1];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                u32x4 A[PT][4];
                if (guard)
                    x3w_synth_step<PT, BF16, ROW, true>(xs, ys, zs, amp_s, a.inv_dmin_rev, px, py,
                                                        pz, A);
                else
                    x3w_synth_step<PT, BF16, ROW, false>(xs, ys, zs, amp_s, a.inv_dmin_rev, px, py,
                                                         pz, A);
                x3w_phase_barrier();
                if (!BF16 && s == 0) {
                    // the column's stream changed its scale: rescale its sums exactly
                    int ne[NT / 2];
                    bool moved = false;
#pragma unroll
                    for (int b = 0; b < NT / 2; ++b) {
                        ne[b] = T.wexp[16 * b + (lane & 15)];
                        moved = moved || (c > 0 && ne[b] != cur[b]);
                    }
                    if (__builtin_expect(__any(moved), 0)) {
#pragma unroll
                        for (int b = 0; b < NT / 2; ++b) {
                            const int d = c > 0 ? ne[b] - cur[b] : 0;
#pragma unroll
                            for (int t = 0; t < PT; ++t)
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    acc[t][2 * b][r] = ldexpf(acc[t][2 * b][r], d);
                                    acc[t][2 * b + 1][r] = ldexpf(acc[t][2 * b + 1][r], d);
                                }
                        }
                    }
#pragma unroll
                    for (int b = 0; b < NT / 2; ++b) cur[b] = ne[b];
                }
                // the positions of the next step
                if (s == 0) {
                    x3w_positions<NT, ROW>(T, 1, grp, xs, ys, zs);
                } else if (c + 1 < nch) {
                    const X3wBuf<NT>& Tn = buf[(c + 1) & 1];
                    x3w_positions<NT, ROW>(Tn, 0, grp, xs, ys, zs);
                    guard = !ROW || !Tn.far;
                }
                x3w_mma_step<NT, PT, BF16>(T, s, lane, A, acc);
                if (s == 0 && c + 1 < nch) {
                    // buffer (c + 1) & 1 was last read in chunk c - 1
                    x3w_write<NT, BF16>(a, buf[(c + 1) & 1], (c + 1) * kChunk, tid, st, ROW, ry, rz,
                                        far_c);
                    if (c + 2 < nch) x3w_load<NT>(a, (c + 2) * kChunk, tid, st);
                }
                x3w_phase_barrier();
            }
        }
        if (!late) x3w_phase_barrier();
    };
    if (row)
        run(std::true_type{});
    else
        run(std::false_type{});
    // undo the scales (exact powers of two)
    if constexpr (!BF16) {
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[t][q][r] = ldexpf(acc[t][q][r], -(cur[q >> 1] + hexp));
    }
    map_epilogue<NT, PT>(a, acc, base, lane,
                         reinterpret_cast<float*>(smem) + wave * 16 * PT * ep_stride<NT>());
}

}  // namespace dmimo
