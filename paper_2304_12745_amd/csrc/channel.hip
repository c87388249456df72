// Channel synthesis: H[b][n][m] materialised in HBM (LoS or Rician).
//
// The kernel is bound by HBM writes: 8 B per term for complex64 (16 B for
// complex128), plus an 8 B NLoS read per term for Rician.  One wavefront walks
// one row (b, n) with its lanes over consecutive antennas, so every store is a
// contiguous 512 B (1 KiB for complex128) burst.  For M < 64 a wave packs
// 64 / pow2ceil(M) rows.  Waves grid-stride over the rows.
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
};

template <bool F64, bool RICIAN>
__global__ __launch_bounds__(256) void channel_kernel(ChannelArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int lpr = 1 << a.lpr_log2;
    const int rows_per_wave = 64 >> a.lpr_log2;
    const int sub = lane >> a.lpr_log2;
    const int l = lane & (lpr - 1);
    const int64_t rows = a.B * a.N;
    const float amp_c = (float)a.w.amp_c;
    const float inv_dmin = (float)a.w.inv_dmin;
    const float a_los = (float)a.w.a_los;
    const float a_nlos = (float)a.w.a_nlos;

    for (int64_t r0 = wave * rows_per_wave; r0 < rows; r0 += nwaves * rows_per_wave) {
        const int64_t r = r0 + sub;
        if (r >= rows) continue;
        const int64_t b = r / a.N;
        const int64_t n = r - b * a.N;
        double px, py, pz;
        point_xyz(a.P, b, n, px, py, pz);
        const double* ap = a.ap + b * a.M * 3;
        for (int64_t m = l; m < a.M; m += lpr) {
            const double dx = px - ap[m * 3 + 0];
            const double dy = py - ap[m * 3 + 1];
            const double dz = pz - ap[m * 3 + 2];
            const int64_t idx = r * a.M + m;
            if constexpr (F64) {
                const TermF64 t = wave_term_f64(dx, dy, dz, a.w.inv_lam, a.w.amp_c, a.w.inv_dmin);
                double hr = t.amp * t.c;
                double hi = -t.amp * t.s;
                if constexpr (RICIAN) {
                    const float2 g = a.nlos[idx];
                    hr = t.amp * (a.w.a_los * t.c + a.w.a_nlos * (double)g.x);
                    hi = t.amp * (-a.w.a_los * t.s + a.w.a_nlos * (double)g.y);
                }
                reinterpret_cast<double2*>(a.H)[idx] = make_double2(hr, hi);
            } else {
                const TermF32 t = wave_term_f32(dx, dy, dz, a.w.inv_lam, amp_c, inv_dmin);
                float hr = t.amp * t.c;
                float hi = -t.amp * t.s;
                if constexpr (RICIAN) {
                    const float2 g = a.nlos[idx];
                    hr = t.amp * fmaf(a_los, t.c, a_nlos * g.x);
                    hi = t.amp * fmaf(-a_los, t.s, a_nlos * g.y);
                }
                reinterpret_cast<float2*>(a.H)[idx] = make_float2(hr, hi);
            }
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
    int lpr_log2 = 6;
    while (lpr_log2 > 0 && (1 << (lpr_log2 - 1)) >= M) --lpr_log2;
    a.lpr_log2 = lpr_log2;
    const int64_t rows = B * P.n;
    const int64_t rows_per_block = 4 * (64 >> lpr_log2);
    const int64_t blocks = std::min<int64_t>(ceil_div(rows, rows_per_block), 256 * 64);
    dim3 grid((unsigned)blocks), block(256);
    if (f64) {
        if (rician) channel_kernel<true, true><<<grid, block, 0, s>>>(a);
        else channel_kernel<true, false><<<grid, block, 0, s>>>(a);
    } else {
        if (rician) channel_kernel<false, true><<<grid, block, 0, s>>>(a);
        else channel_kernel<false, false><<<grid, block, 0, s>>>(a);
    }
    return check_launch("channel_kernel");
}

}  // namespace dmimo
