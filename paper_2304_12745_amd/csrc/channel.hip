// Channel synthesis: H[b][n][m] materialised in HBM (LoS or Rician).
//
// The kernel is bound by HBM writes: 8 B per term for complex64 (16 B for
// complex128), plus an 8 B NLoS read per term for Rician.  One wavefront walks
// one row (b, n) with its lanes over consecutive antennas, so every store is a
// contiguous 512 B (1 KiB for complex128) burst.  For M <= 64 a row takes
// pow2ceil(M) / 4 lanes (at least one), each with up to four antennas
// l + q lanes: four independent terms per lane, whose FP64 / transcendental
// chains overlap, and stores in whole 128 B segments.  The lane's antenna
// coordinates stay in registers while b does not change.  Waves grid-stride
// over the rows.  A lane keeps its row as (b, n), and on a grid as
// n = j nx + i, and advances them by the fixed stride with carries: the loop
// has no integer division, which would cost as much as the terms of a row.
// One deployment with wide rows and at least 4096 points (FP32 LoS, M even)
// takes channel_rows_kernel instead: a workgroup writes whole rows together
// with 16-byte stores of antenna pairs.
#include <type_traits>

#include "kernels.h"

namespace dmimo {

namespace {

struct ChannelArgs {
    WaveConst w;
    PointsDev P;
    const double* ap;    // [B][M][3]
    const float2* nlos;  // [B][N][M] or null
    void* H;
    int64_t B, N, M;
    int lpr_log2;        // log2(lanes per row)
    int64_t stride;      // rows per grid-stride step
    int64_t sb, sn;      // stride = sb N + sn
    int32_t si, sj;      // sn = sj nx + si (grid points)
    int lds_ap;          // rows wider than 64 antennas, B = 1: coordinates in LDS
};

// Antenna coordinates of a single deployment for the wide-row path, as
// planes x[M], y[M], z[M].
constexpr int kLdsApMax = 2048;

// One term; the NLoS draw is read and the term stored only where `valid`.
template <bool F64, bool RICIAN>
__device__ __forceinline__ void emit_term(const ChannelArgs& a, int64_t idx, bool valid, double dx,
                                          double dy, double dz) {
    if constexpr (F64) {
        const TermF64 t = wave_term_f64(dx, dy, dz, a.w.inv_lam, a.w.amp_c, a.w.inv_dmin);
        double hr = t.amp * t.c;
        double hi = -t.amp * t.s;
        if constexpr (RICIAN) {
            const float2 g = valid ? a.nlos[idx] : make_float2(0.0f, 0.0f);
            hr = t.amp * (a.w.a_los * t.c + a.w.a_nlos * (double)g.x);
            hi = t.amp * (-a.w.a_los * t.s + a.w.a_nlos * (double)g.y);
        }
        if (valid) reinterpret_cast<double2*>(a.H)[idx] = make_double2(hr, hi);
    } else {
        const TermF32 t = wave_term_f32(dx, dy, dz, a.w.inv_lam, (float)a.w.amp_c, (float)a.w.inv_dmin);
        float hr = t.amp * t.c;
        float hi = -t.amp * t.s;
        if constexpr (RICIAN) {
            const float2 g = valid ? a.nlos[idx] : make_float2(0.0f, 0.0f);
            hr = t.amp * fmaf((float)a.w.a_los, t.c, (float)a.w.a_nlos * g.x);
            hi = t.amp * fmaf(-(float)a.w.a_los, t.s, (float)a.w.a_nlos * g.y);
        }
        if (valid) reinterpret_cast<float2*>(a.H)[idx] = make_float2(hr, hi);
    }
}

// APL > 0: M <= APL * lanes per row, antennas l + q lpr (q < APL) per lane.
// APL = 0: lanes over the antennas of a row, 64 at a time.
template <bool F64, bool RICIAN, int APL>
__global__ __launch_bounds__(256) void channel_kernel(ChannelArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lpr = 1 << a.lpr_log2;
    const int rows_per_wave = 64 >> a.lpr_log2;
    const int sub = lane >> a.lpr_log2;
    const int l = lane & (lpr - 1);
    const int64_t rows = a.B * a.N;
    const bool grid = a.P.kind == DMIMO_PTS_GRID;
    extern __shared__ double s_ap[];
    if (APL == 0 && a.lds_ap) {
        for (int i = threadIdx.x; i < a.M; i += blockDim.x) {
            s_ap[i] = a.ap[3 * i + 0];
            s_ap[a.M + i] = a.ap[3 * i + 1];
            s_ap[2 * a.M + i] = a.ap[3 * i + 2];
        }
        __syncthreads();
    }

    int64_t r = wave * rows_per_wave + sub;
    if (r >= rows) return;
    int64_t b, n;
    int32_t gi = 0, gj = 0;
    if (rows <= 0xffffffffLL) {   // 32-bit division where it suffices
        const uint32_t ru = (uint32_t)r, nu = (uint32_t)a.N;
        const uint32_t bu = ru / nu;
        b = bu;
        n = ru - bu * nu;
        if (grid) {
            gj = (int32_t)((uint32_t)n / (uint32_t)a.P.nx);
            gi = (int32_t)(n - (int64_t)gj * a.P.nx);
        }
    } else {
        b = r / a.N;
        n = r - b * a.N;
        if (grid) {
            gj = (int32_t)(n / a.P.nx);
            gi = (int32_t)(n - (int64_t)gj * a.P.nx);
        }
    }
    constexpr int NA = APL > 0 ? APL : 1;
    int64_t bc = -1;
    double ax[NA], ay[NA], az[NA];
    for (; r < rows; r += a.stride) {
        double px, py, pz;
        if (grid) {
            px = a.P.x0 + ((double)gi + 0.5) * a.P.dx;
            py = a.P.y0 + ((double)gj + 0.5) * a.P.dy;
            pz = a.P.z;
        } else {
            const double* q = a.P.xyz + r * 3;
            px = q[0];
            py = q[1];
            pz = q[2];
        }
        const double* ap = a.ap + b * a.M * 3;
        if constexpr (APL > 0) {
            if (b != bc) {
#pragma unroll
                for (int q = 0; q < APL; ++q) {
                    // past M: a valid antenna's coordinates, never stored
                    const int64_t m = l + q * lpr < a.M ? l + q * lpr : a.M - 1;
                    ax[q] = ap[m * 3 + 0];
                    ay[q] = ap[m * 3 + 1];
                    az[q] = ap[m * 3 + 2];
                }
                bc = b;
            }
#pragma unroll
            for (int q = 0; q < APL; ++q) {
                const int64_t m = l + q * lpr;
                emit_term<F64, RICIAN>(a, r * a.M + m, m < a.M, px - ax[q], py - ay[q], pz - az[q]);
            }
        } else if (a.lds_ap) {
#pragma unroll 4
            for (int64_t m = l; m < a.M; m += lpr)
                emit_term<F64, RICIAN>(a, r * a.M + m, true, px - s_ap[m], py - s_ap[a.M + m],
                                       pz - s_ap[2 * a.M + m]);
        } else {
#pragma unroll 4
            for (int64_t m = l; m < a.M; m += lpr)
                emit_term<F64, RICIAN>(a, r * a.M + m, true, px - ap[m * 3 + 0], py - ap[m * 3 + 1],
                                       pz - ap[m * 3 + 2]);
        }
        n += a.sn;
        b += a.sb;
        if (n >= a.N) {
            n -= a.N;
            ++b;
        }
        if (grid) {
            gi += a.si;
            gj += a.sj;
            if (gi >= a.P.nx) {
                gi -= a.P.nx;
                ++gj;
            }
            if (gj >= a.P.ny) gj -= a.P.ny;
        }
    }
}

// Wide rows of one deployment (FP32 LoS, M even, 512 <= M <= 2048): a
// workgroup writes each of its kRowsPerWg consecutive rows together, two
// adjacent antennas per thread and one 16-byte store (4 KB per round of the
// 256 threads), the antenna coordinates in LDS.  Against one row per wave
// with 8-byte stores, the hall's 34.4 GB went from 66% to 71% of HBM peak
// (the same bits).
constexpr int kRowsPerWg = 16;

__global__ __launch_bounds__(256) void channel_rows_kernel(ChannelArgs a) {
    extern __shared__ double s_ap[];
    const int tid = threadIdx.x;
    for (int i = tid; i < a.M; i += 256) {
        s_ap[i] = a.ap[3 * i + 0];
        s_ap[a.M + i] = a.ap[3 * i + 1];
        s_ap[2 * a.M + i] = a.ap[3 * i + 2];
    }
    __syncthreads();
    const bool grid = a.P.kind == DMIMO_PTS_GRID;
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerWg;
    for (int i = 0; i < kRowsPerWg; ++i) {
        const int64_t r = r0 + i;
        if (r >= a.N) break;
        double px, py, pz;
        if (grid) {
            const int64_t gj = r / a.P.nx, gi = r - gj * a.P.nx;
            px = a.P.x0 + ((double)gi + 0.5) * a.P.dx;
            py = a.P.y0 + ((double)gj + 0.5) * a.P.dy;
            pz = a.P.z;
        } else {
            const double* q = a.P.xyz + r * 3;
            px = q[0];
            py = q[1];
            pz = q[2];
        }
        for (int64_t m = 2 * tid; m < a.M; m += 512) {
            const TermF32 t0 = wave_term_f32(px - s_ap[m], py - s_ap[a.M + m], pz - s_ap[2 * a.M + m],
                                             a.w.inv_lam, (float)a.w.amp_c, (float)a.w.inv_dmin);
            const TermF32 t1 = wave_term_f32(px - s_ap[m + 1], py - s_ap[a.M + m + 1],
                                             pz - s_ap[2 * a.M + m + 1], a.w.inv_lam, (float)a.w.amp_c,
                                             (float)a.w.inv_dmin);
            *reinterpret_cast<float4*>(reinterpret_cast<float2*>(a.H) + r * a.M + m) =
                make_float4(t0.amp * t0.c, -t0.amp * t0.s, t1.amp * t1.c, -t1.amp * t1.s);
        }
    }
}

}  // namespace

dmimo_status launch_channel(const WaveConst& w, const PointsDev& P, bool rician, int64_t B,
                            int64_t M, const double* ap, const void* nlos, bool f64, void* H,
                            hipStream_t s) {
    ChannelArgs a;
    a.w = w;
    a.P = P;
    a.ap = ap;
    a.nlos = reinterpret_cast<const float2*>(nlos);
    a.H = H;
    a.B = B;
    a.N = P.n;
    a.M = M;
    // rows of at most 64 antennas: pow2ceil(M) / 4 lanes per row (>= 1), up
    // to 4 antennas per lane; wider rows: 64 lanes, looping over antennas
    int lpr_log2 = 6, apl = 0;
    if (M <= 64) {
        int p2 = 1;
        while (p2 < M) p2 <<= 1;
        const int lpr = p2 >= 4 ? p2 / 4 : 1;
        lpr_log2 = 0;
        while ((1 << lpr_log2) < lpr) ++lpr_log2;
        apl = (int)((M + lpr - 1) / lpr) <= 2 ? 2 : 4;
    }
    a.lpr_log2 = lpr_log2;
    const int64_t rows = B * P.n;
    const int64_t rows_per_block = 4 * (64 >> lpr_log2);
    // workgroups per CU at most: 12 for the packed rows, 64 for wide rows
    const int64_t blocks = std::min<int64_t>(ceil_div(rows, rows_per_block), 256 * (apl ? 12 : 64));
    a.lds_ap = apl == 0 && B == 1 && M <= kLdsApMax;
    const size_t lds = a.lds_ap ? (size_t)(3 * M) * sizeof(double) : 0;
    a.stride = blocks * 4 * (64 >> lpr_log2);
    a.sb = a.stride / a.N;
    a.sn = a.stride - a.sb * a.N;
    a.si = a.sj = 0;
    if (P.kind == DMIMO_PTS_GRID) {
        a.sj = (int32_t)(a.sn / P.nx);
        a.si = (int32_t)(a.sn - (int64_t)a.sj * P.nx);
    }
    dim3 grid((unsigned)blocks), block(256);
    // (at least 256 workgroups of rows; fewer rows, e.g. a deployment's users,
    // keep one row per wave, which spreads them over more CUs)
    if (!f64 && !rician && apl == 0 && a.lds_ap && M % 2 == 0 && M >= 512 &&
        P.n >= 256 * kRowsPerWg && ceil_div(P.n, kRowsPerWg) <= 0x7fffffff) {
        channel_rows_kernel<<<dim3((unsigned)ceil_div(P.n, kRowsPerWg)), block, lds, s>>>(a);
        return check_launch("channel_rows_kernel");
    }
    auto go = [&](auto f64c, auto ricc) {
        constexpr bool F = decltype(f64c)::value, R = decltype(ricc)::value;
        if (apl == 0) channel_kernel<F, R, 0><<<grid, block, lds, s>>>(a);
        else if (apl == 2) channel_kernel<F, R, 2><<<grid, block, 0, s>>>(a);
        else channel_kernel<F, R, 4><<<grid, block, 0, s>>>(a);
    };
    using T = std::true_type;
    using Fl = std::false_type;
    if (f64) {
        if (rician) go(T{}, T{});
        else go(T{}, Fl{});
    } else {
        if (rician) go(Fl{}, T{});
        else go(Fl{}, Fl{});
    }
    return check_launch("channel_kernel");
}

}  // namespace dmimo
