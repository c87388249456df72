// Fused channel synthesis + coherent sums at N evaluation points.
//
// One lane owns one point.  All lanes of a wavefront walk the antennas in
// the same order, so each antenna's position (FP64 xyz) and its K weights
// w_km are wave-uniform.  The compiler keeps them in scalar registers (scalar
// loads through the constant cache), and the VALU only synthesises h[n][m]
// (FP64 distance and phase, FP32 amplitude and hardware sin/cos) and runs
// the K complex MACs.  No byte per term touches HBM: a point costs 12 B of
// coordinates at most (none on a grid) and 4-8 B of output per map.
//
// The reduction over antennas stays inside one lane in ascending m, so a
// point's result does not depend on how points are grouped into launches.
#include "kernels.h"
#include "powermap_body.h"
#include "powermap_mfma.h"

namespace dmimo {

namespace {

template <bool F64>
struct PmTypes;
template <>
struct PmTypes<false> {
    using R = float;
    using C = float2;
};
template <>
struct PmTypes<true> {
    using R = double;
    using C = double2;
};

struct PmDev {
    WaveConst w;
    PointsDev P;
    int M;
    int K;
    const double* __restrict__ ap;
    const void* __restrict__ W;
    double sigma2;
    void* power;
    void* sinr;
    int32_t* best_k;
    void* per_stream;
};

// Map p of a batched launch (grid row p): its weights and outputs.
template <bool F64>
__device__ __forceinline__ PmDev map_of(PmDev a, int64_t p) {
    using R = typename PmTypes<F64>::R;
    using C = typename PmTypes<F64>::C;
    const int64_t N = a.P.n;
    a.W = reinterpret_cast<const C*>(a.W) + p * a.K * a.M;
    a.power = reinterpret_cast<R*>(a.power) + p * N;
    if (a.sinr) a.sinr = reinterpret_cast<R*>(a.sinr) + p * N;
    if (a.best_k) a.best_k += p * N;
    if (a.per_stream) a.per_stream = reinterpret_cast<R*>(a.per_stream) + p * N * a.K;
    return a;
}

template <bool F64, typename R>
__device__ __forceinline__ void epilogue(const PmDev& a, int64_t n, const R* zr, const R* zi,
                                         int K) {
    using C = typename PmTypes<F64>::C;
    (void)sizeof(C);
    R y = 0, pb = -1;
    int best = 0;
    for (int k = 0; k < K; ++k) {
        const R p = zr[k] * zr[k] + zi[k] * zi[k];
        y += p;
        if (p > pb) {
            pb = p;
            best = k;
        }
    }
    reinterpret_cast<R*>(a.power)[n] = y;
    if (a.sinr) {
        R intf = 0;
        for (int k = 0; k < K; ++k)
            if (k != best) intf += zr[k] * zr[k] + zi[k] * zi[k];
        reinterpret_cast<R*>(a.sinr)[n] = pb / (intf + (R)a.sigma2);
    }
    if (a.best_k) a.best_k[n] = best;
    if (a.per_stream) {
        R* ps = reinterpret_cast<R*>(a.per_stream) + n * (int64_t)K;
        for (int k = 0; k < K; ++k) ps[k] = zr[k] * zr[k] + zi[k] * zi[k];
    }
}

// KT: accumulator count (compile time); K <= KT at run time.
template <int KT, bool F64>
__global__ __launch_bounds__(256) void powermap_valu_kernel(PmDev a0) {
    const PmDev a = map_of<F64>(a0, blockIdx.y);
    using R = typename PmTypes<F64>::R;
    using C = typename PmTypes<F64>::C;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = n < a.P.n;
    double px = 0, py = 0, pz = 0;
    if (live) point_xyz(a.P, 0, n, px, py, pz);
    const int K = a.K;
    const int M = a.M;
    const C* __restrict__ W = reinterpret_cast<const C*>(a.W);
    R zr[KT], zi[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        zr[k] = 0;
        zi[k] = 0;
    }
    const float amp_c = (float)a.w.amp_c;
    const float inv_dmin = (float)a.w.inv_dmin;
    for (int m = 0; m < M; ++m) {
        const double ax = a.ap[3 * m + 0];
        const double ay = a.ap[3 * m + 1];
        const double az = a.ap[3 * m + 2];
        R hr, hi;
        if constexpr (F64) {
            const TermF64 t = wave_term_f64(px - ax, py - ay, pz - az, a.w.inv_lam, a.w.amp_c,
                                            a.w.inv_dmin);
            hr = t.amp * t.c;
            hi = -t.amp * t.s;
        } else {
            const TermF32 t = wave_term_f32(px - ax, py - ay, pz - az, a.w.inv_lam, amp_c, inv_dmin);
            hr = t.amp * t.c;
            hi = -t.amp * t.s;
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (KT > 1 && k >= K) break;
            const C w = W[(int64_t)k * M + m];
            zr[k] = fma(hr, w.x, fma(-hi, w.y, zr[k]));
            zi[k] = fma(hr, w.y, fma(hi, w.x, zi[k]));
        }
    }
    if (live) epilogue<F64, R>(a, n, zr, zi, K);
}

template <int KT>
__global__ __launch_bounds__(256) void powermap_valu_f32_kernel(PmMapDev a) {
    map_valu_wg<KT>(map_of(a, blockIdx.y), (int64_t)blockIdx.x * 256);
}

template <bool F64>
dmimo_status launch_valu(const PmDev& d, int maps, hipStream_t s) {
    const int64_t blocks = ceil_div(d.P.n, 256);
    dim3 grid((unsigned)blocks, (unsigned)maps), block(256);
    const int K = d.K;
    if (K == 1) powermap_valu_kernel<1, F64><<<grid, block, 0, s>>>(d);
    else if (K <= 2) powermap_valu_kernel<2, F64><<<grid, block, 0, s>>>(d);
    else if (K <= 4) powermap_valu_kernel<4, F64><<<grid, block, 0, s>>>(d);
    else if (K <= 8) powermap_valu_kernel<8, F64><<<grid, block, 0, s>>>(d);
    else if (K <= 16) powermap_valu_kernel<16, F64><<<grid, block, 0, s>>>(d);
    else powermap_valu_kernel<32, F64><<<grid, block, 0, s>>>(d);
    return check_launch("powermap_valu_kernel");
}

}  // namespace

dmimo_status launch_powermap(const PowermapArgs& a, hipStream_t s) {
    PmDev d;
    d.w = a.w;
    d.P = a.P;
    d.M = a.M;
    d.K = a.K;
    d.ap = a.ap;
    d.W = a.W;
    d.sigma2 = a.sigma2;
    d.power = a.power;
    d.sinr = a.sinr;
    d.best_k = a.best_k;
    d.per_stream = a.per_stream;
    if (a.prec == DMIMO_F64) return launch_valu<true>(d, a.maps, s);
    if (a.prec == DMIMO_F32) {
        // one or two streams: four or eight FMA per term stay on the VALU
        if (a.K <= 2) {
            const PmMapDev m = make_map_dev(a);
            dim3 grid((unsigned)ceil_div(a.P.n, 256), (unsigned)a.maps), block(256);
            if (a.K == 1) powermap_valu_f32_kernel<1><<<grid, block, 0, s>>>(m);
            else powermap_valu_f32_kernel<2><<<grid, block, 0, s>>>(m);
            return check_launch("powermap_valu_f32_kernel");
        }
        return launch_powermap_f32_mfma(a, s);
    }
    return launch_powermap_mfma(a, s);
}

}  // namespace dmimo
