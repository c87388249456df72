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
//   2^14 (|h| <= 1 always, by the near-field clamp).  The weights of each
//   64-antenna chunk are scaled by a power of two that puts their largest
//   magnitude in [2^13, 2^14).  The accumulator is rescaled by the exact
//   ratio when the chunk scale changes, and by the inverse scales at the end.
//   BF16 has the FP32 exponent range and needs no scaling.
//
// Output tile D: lane 16g + j holds D[4g + r][j] in register r.  Column
// layouts are in powermap_common.h.
#pragma once

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

constexpr float kHScale = 16384.0f;   // 2^14: FP16 range placement of h (|h| <= 1)

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
    const float hscale = BF16 ? 1.0f : kHScale;
    const float amp_s = a.amp_rev * hscale;

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
    const float inv = BF16 ? 1.0f : ldexpf(1.0f, -wexp) / kHScale;
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[t][q] *= inv;
    __syncthreads();
    map_epilogue<NT, PT>(a, acc, base, lane,
                         reinterpret_cast<float*>(smem) + wave * 16 * PT * ep_stride<NT>());
}

}  // namespace dmimo
