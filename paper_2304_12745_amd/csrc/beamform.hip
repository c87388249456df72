// Precoders and their epilogues, one workgroup per deployment.
//
// ZF (eq. optim1 constraint H W^T = sigma D_gamma^{1/2}, or total-power
// scaling), after the Gram kernel has written G = H H^H to the workspace:
//   1. G -> FP64 in LDS, Cholesky G = L L^H (left-looking, one column per
//      step).  A pivot below tol * G_jj sets info = j+1.
//   2. L^-1 by forward substitution, one column per thread; tr(G^-1) = ||L^-1||_F^2.
//   3. G^-1 = L^-H L^-1 (FP64, K x K in LDS).
//   4. Column pass, one antenna per thread: x = G^-1 h_m, w_m = c * conj(x),
//      p_m = sum_k |w_km|^2 (of the stored W), and a partial sum of sqrt(p_m).
// MR / equal-gain MR: ||H||_F^2 by block reduction, then the column pass.
// Epilogue (all precoders): A = H W^T (FP64, one entry per thread, read back
// from the stored H and W), then SINR_k and the sum rate.
#include <cmath>

#include "kernels.h"

namespace dmimo {

namespace {

struct BfDev {
    int precoder;
    int K;
    int64_t M;
    const void* H;
    double gamma[DMIMO_K_MAX];
    double sigma2;
    double p_total;
    double pivot_tol;
    void* W;
    double* p_ant;
    double* l21;
    double* sinr;
    double* rsum;
    int32_t* info;
    const void* G;
};

template <typename T2>
__device__ __forceinline__ double2 ld2(const T2* p, int64_t i) {
    const T2 v = p[i];
    return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    // 256 threads = 4 waves
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    return t;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

template <typename T2, int KT>
__global__ __launch_bounds__(256) void beamform_kernel(BfDev a) {
    __shared__ double2 sL[KT][KT + 1];     // Cholesky factor, later A = H W^T
    __shared__ double2 sI[KT][KT + 1];     // L^-1
    __shared__ double2 sG[KT][KT + 1];     // G^-1
    __shared__ double red[8];
    __shared__ int s_fail;
    __shared__ double s_scale[KT];

    const int64_t b = blockIdx.x;
    const int K = a.K;
    const int64_t M = a.M;
    const int tid = threadIdx.x;
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + b * K * M;

    if (tid == 0) s_fail = 0;

    if (a.precoder == DMIMO_ZF) {
        const T2* Gb = reinterpret_cast<const T2*>(a.G) + b * K * K;
        for (int e = tid; e < K * K; e += blockDim.x) {
            const int i = e / K, j = e - (e / K) * K;
            sG[i][j] = ld2(Gb, e);   // G kept intact in sG for the pivot test
            sL[i][j] = make_double2(0.0, 0.0);
            sI[i][j] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        // 1. Cholesky, left-looking: column j uses columns < j.
        for (int j = 0; j < K; ++j) {
            if (tid == 0) {
                double d = sG[j][j].x;
                for (int p = 0; p < j; ++p) d -= sL[j][p].x * sL[j][p].x + sL[j][p].y * sL[j][p].y;
                if (!(d > a.pivot_tol * sG[j][j].x)) {
                    s_fail = j + 1;
                    d = 1.0;
                }
                sL[j][j] = make_double2(sqrt(d), 0.0);
            }
            __syncthreads();
            if (s_fail) break;
            const int i = j + 1 + tid;
            if (i < K) {
                double2 s = sG[i][j];
                for (int p = 0; p < j; ++p) {
                    const double2 t = cmulc(sL[i][p], sL[j][p]);
                    s.x -= t.x;
                    s.y -= t.y;
                }
                const double inv = 1.0 / sL[j][j].x;
                sL[i][j] = make_double2(s.x * inv, s.y * inv);
            }
            __syncthreads();
        }
        if (s_fail) {
            // zero outputs of this deployment
            for (int64_t e = tid; e < (int64_t)K * M; e += blockDim.x) {
                T2 z;
                z.x = 0;
                z.y = 0;
                Wb[e] = z;
            }
            if (a.p_ant)
                for (int64_t m = tid; m < M; m += blockDim.x) a.p_ant[b * M + m] = 0.0;
            if (a.sinr)
                for (int k = tid; k < K; k += blockDim.x) a.sinr[b * K + k] = 0.0;
            if (tid == 0) {
                if (a.l21) a.l21[b] = 0.0;
                if (a.rsum) a.rsum[b] = 0.0;
                if (a.info) a.info[b] = s_fail;
            }
            return;
        }
        // 2. L^-1: thread c solves L x = e_c (x_i = 0 for i < c).
        if (tid < K) {
            const int c = tid;
            for (int i = c; i < K; ++i) {
                double2 s = make_double2(i == c ? 1.0 : 0.0, 0.0);
                for (int p = c; p < i; ++p) {
                    const double2 t = cmul(sL[i][p], sI[p][c]);
                    s.x -= t.x;
                    s.y -= t.y;
                }
                const double inv = 1.0 / sL[i][i].x;
                sI[i][c] = make_double2(s.x * inv, s.y * inv);
            }
        }
        __syncthreads();
        double tr = 0.0;
        for (int e = tid; e < K * K; e += blockDim.x) {
            const double2 v = sI[e / K][e % K];
            tr += v.x * v.x + v.y * v.y;
        }
        tr = block_sum(tr, red);   // tr(G^-1) = ||L^-1||_F^2
        // 3. G^-1 = L^-H L^-1: (G^-1)_ij = sum_{p >= max(i,j)} conj(Li_pi) Li_pj
        for (int e = tid; e < K * K; e += blockDim.x) {
            const int i = e / K, j = e - (e / K) * K;
            double2 s = make_double2(0.0, 0.0);
            for (int p = (i > j ? i : j); p < K; ++p) {
                const double2 t = cconjmul(sI[p][i], sI[p][j]);
                s.x += t.x;
                s.y += t.y;
            }
            sG[i][j] = s;
        }
        if (tid < K) {
            s_scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total / tr)
                                           : sqrt(a.sigma2) * sqrt(a.gamma[tid]);
        }
        __syncthreads();
    } else {
        double f = 0.0;
        for (int64_t e = tid; e < (int64_t)K * M; e += blockDim.x) {
            const double2 h = ld2(Hb, e);
            f += h.x * h.x + h.y * h.y;
        }
        f = block_sum(f, red);
        if (tid < K) {
            if (a.precoder == DMIMO_MR)
                s_scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total) / sqrt(f) : 1.0;
            else
                s_scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total / ((double)K * (double)M)) : 1.0;
        }
        __syncthreads();
    }

    // 4. column pass
    double l21 = 0.0;
    for (int64_t m = tid; m < M; m += blockDim.x) {
        double2 hv[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k)
            hv[k] = k < K ? ld2(Hb, (int64_t)k * M + m) : make_double2(0.0, 0.0);
        double pm = 0.0;
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            if (k >= K) break;
            double2 w;
            if (a.precoder == DMIMO_ZF) {
                double2 x = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < KT; ++j) {
                    if (j >= K) break;
                    const double2 t = cmul(sG[k][j], hv[j]);
                    x.x += t.x;
                    x.y += t.y;
                }
                w = make_double2(s_scale[k] * x.x, -s_scale[k] * x.y);
            } else if (a.precoder == DMIMO_MR) {
                w = make_double2(s_scale[k] * hv[k].x, -s_scale[k] * hv[k].y);
            } else {
                const double mag = sqrt(hv[k].x * hv[k].x + hv[k].y * hv[k].y);
                w = mag > 0.0 ? make_double2(s_scale[k] * hv[k].x / mag, -s_scale[k] * hv[k].y / mag)
                              : make_double2(s_scale[k], 0.0);
            }
            T2 ws;
            ws.x = w.x;
            ws.y = w.y;
            Wb[(int64_t)k * M + m] = ws;
            const double wr = (double)ws.x, wi = (double)ws.y;
            pm += wr * wr + wi * wi;
        }
        if (a.p_ant) a.p_ant[b * M + m] = pm;
        l21 += sqrt(pm);
    }
    l21 = block_sum(l21, red);
    if (tid == 0) {
        if (a.l21) a.l21[b] = l21;
        if (a.info) a.info[b] = 0;
    }
    if (!a.sinr && !a.rsum) return;

    // make this block's W stores visible to its own later loads
    __threadfence_block();
    __syncthreads();
    // 5. A = H W^T, one entry (k, j) per thread
    for (int e = tid; e < K * K; e += blockDim.x) {
        const int k = e / K, j = e - (e / K) * K;
        double2 s = make_double2(0.0, 0.0);
        for (int64_t m = 0; m < M; ++m) {
            const double2 t = cmul(ld2(Hb, (int64_t)k * M + m), ld2((const T2*)Wb, (int64_t)j * M + m));
            s.x += t.x;
            s.y += t.y;
        }
        sL[k][j] = s;
    }
    __syncthreads();
    double rate = 0.0;
    if (tid < K) {
        const int k = tid;
        double sig = 0.0, intf = 0.0;
        for (int j = 0; j < K; ++j) {
            const double p = sL[k][j].x * sL[k][j].x + sL[k][j].y * sL[k][j].y;
            if (j == k) sig = p;
            else intf += p;
        }
        const double snr = sig / (intf + a.sigma2);
        if (a.sinr) a.sinr[b * K + k] = snr;
        rate = log2(1.0 + snr);
    }
    rate = block_sum(rate, red);
    if (tid == 0 && a.rsum) a.rsum[b] = rate;
}

template <typename T2>
dmimo_status launch_typed(const BfDev& d, int64_t B, hipStream_t s) {
    dim3 grid((unsigned)B), block(256);
    if (d.K <= 8) beamform_kernel<T2, 8><<<grid, block, 0, s>>>(d);
    else if (d.K <= 16) beamform_kernel<T2, 16><<<grid, block, 0, s>>>(d);
    else beamform_kernel<T2, 32><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_kernel");
}

}  // namespace

dmimo_status launch_beamform(const BeamformArgs& a, hipStream_t s) {
    if (a.B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "beamform: B too large");
    BfDev d;
    d.precoder = a.precoder;
    d.K = a.K;
    d.M = a.M;
    d.H = a.H;
    for (int k = 0; k < DMIMO_K_MAX; ++k) d.gamma[k] = a.gamma[k];
    d.sigma2 = a.sigma2;
    d.p_total = a.p_total;
    // pivot tolerance relative to G_jj, matched to the Gram's precision
    d.pivot_tol = a.prec == DMIMO_F64 ? 1e-12 : (a.prec == DMIMO_MIX_BF16X3 ? 1e-4 : 1e-6);
    d.W = a.W;
    d.p_ant = a.p_ant;
    d.l21 = a.l21;
    d.sinr = a.sinr;
    d.rsum = a.rsum;
    d.info = a.info;
    d.G = a.ws;
    if (a.precoder == DMIMO_ZF) {
        dmimo_status st = launch_gram(a.B, a.K, a.M, a.H, a.prec, a.ws, s);
        if (st) return st;
    }
    if (a.prec == DMIMO_F64) return launch_typed<double2>(d, a.B, s);
    return launch_typed<float2>(d, a.B, s);
}

}  // namespace dmimo
