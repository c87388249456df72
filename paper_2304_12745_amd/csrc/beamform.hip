// Precoders and their epilogues, one 256-thread workgroup per deployment.
// Deployments of at most 8 users and 256 antennas (128 in FP64) take the
// one-pass kernel further down; the general kernel follows.
//
// ZF (eq. optim1 constraint H W^T = sigma D_gamma^{1/2}, or total-power
// scaling) runs after the Gram kernel has written G = H H^H to the workspace:
//   1. G -> FP64 in LDS, inverted in place by Gauss-Jordan elimination
//      without pivoting (G is Hermitian positive definite), every thread
//      updating its entries in each of the K steps.  The pivot of step j is
//      the diagonal entry of the Schur complement, L_jj^2 of the Cholesky
//      factor; one below tol * G_jj sets info = j+1.  tr(G^-1) is the sum of
//      the inverse's diagonal.
// MR / equal-gain MR: ||H||_F^2 by block reduction.
// Then, for every tile of 64 antennas:
//   4. H tile -> LDS.  Four threads per antenna form x = G^-1 h_m (ZF) or the
//      MR weights, write w_m = c conj(x) to HBM and to LDS, and reduce
//      p_m = sum_k |w_km|^2 of the stored W.
//   5. The K x K gains A = H W^T accumulate in FP64 from the two LDS tiles.
//      Four adjacent threads share an entry, each taking every fourth antenna,
//      and combine their partial sums after the last tile.
// Epilogue: SINR_k from A, sum rate, sum_m sqrt(p_m).
// Every read of H and W after the first comes from LDS, so a deployment reads
// H once and writes W once.
#include <cmath>

#include "kernels.h"

namespace dmimo {

namespace {

constexpr int kCols = 64;   // antennas per tile
constexpr int kThreads = 256;

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
__device__ __forceinline__ double2 to_d2(T2 v) {
    return make_double2((double)v.x, (double)v.y);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) t += red[i];
    return t;
}

__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

template <typename T2, int KT>
struct BfShared {
    double2 ginv[KT][KT + 1];                 // G, then G^-1 (ZF)
    union {
        struct {
            T2 h[KT][kCols + 1];              // H tile
            T2 w[KT][kCols + 1];              // W tile (stored precision)
        } t;
        double2 A[KT][KT + 1];                // gains, after the tiles
    } u;
    double red[kThreads / 64];
    double scale[KT];
    double d0[KT];                            // diagonal of G
};

template <typename T2, int KT>
__global__ __launch_bounds__(kThreads) void beamform_kernel(BfDev a) {
    __shared__ BfShared<T2, KT> S;

    const int64_t b = blockIdx.x;
    const int K = a.K;
    const int64_t M = a.M;
    const int tid = threadIdx.x;
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + b * K * M;

    if (a.precoder == DMIMO_ZF) {
        const T2* Gb = reinterpret_cast<const T2*>(a.G) + b * K * K;
        for (int e = tid; e < K * K; e += kThreads) {
            const int i = e / K, j = e - (e / K) * K;
            const double2 g = to_d2(Gb[e]);
            S.ginv[i][j] = g;
            if (i == j) S.d0[i] = g.x;   // G_jj for the pivot test
        }
        __syncthreads();
        // 1. G^-1 by Gauss-Jordan elimination without pivoting, in place; all
        //    threads read step p's pivot row and column, then write their
        //    entries.  The pivot of step p is the Schur complement's diagonal
        //    entry (L_pp^2 of the Cholesky factor).
        constexpr int QG = (KT * KT + kThreads - 1) / kThreads;
        int fail = 0;
        for (int p = 0; p < K; ++p) {
            const double piv = S.ginv[p][p].x;
            if (!(piv > a.pivot_tol * S.d0[p])) {
                fail = p + 1;
                break;
            }
            const double inv = 1.0 / piv;
            double2 nv[QG];
#pragma unroll
            for (int q = 0; q < QG; ++q) {
                const int e = tid + kThreads * q;
                if (e < K * K) {
                    const int i = e / K, j = e - (e / K) * K;
                    const double2 gpj = S.ginv[p][j], gip = S.ginv[i][p];
                    const double2 r = j == p ? make_double2(inv, 0.0) : make_double2(gpj.x * inv, gpj.y * inv);
                    if (i == p) {
                        nv[q] = r;
                    } else {
                        const double2 g = j == p ? make_double2(0.0, 0.0) : S.ginv[i][j];
                        nv[q] = make_double2(fma(-gip.x, r.x, fma(gip.y, r.y, g.x)),
                                             fma(-gip.x, r.y, fma(-gip.y, r.x, g.y)));
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QG; ++q) {
                const int e = tid + kThreads * q;
                if (e < K * K) S.ginv[e / K][e - (e / K) * K] = nv[q];
            }
            __syncthreads();
        }
        if (fail) {
            for (int64_t e = tid; e < (int64_t)K * M; e += kThreads) {
                T2 z;
                z.x = 0;
                z.y = 0;
                Wb[e] = z;
            }
            if (a.p_ant)
                for (int64_t m = tid; m < M; m += kThreads) a.p_ant[b * M + m] = 0.0;
            if (a.sinr)
                for (int k = tid; k < K; k += kThreads) a.sinr[b * K + k] = 0.0;
            if (tid == 0) {
                if (a.l21) a.l21[b] = 0.0;
                if (a.rsum) a.rsum[b] = 0.0;
                if (a.info) a.info[b] = fail;
            }
            return;
        }
        double tr = 0.0;   // tr(G^-1)
        for (int k = 0; k < K; ++k) tr += S.ginv[k][k].x;
        if (tid < K)
            S.scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total / tr) : sqrt(a.sigma2) * sqrt(a.gamma[tid]);
        __syncthreads();
    } else {
        double f = 0.0;
        for (int64_t e = tid; e < (int64_t)K * M; e += kThreads) {
            const double2 h = to_d2(Hb[e]);
            f += h.x * h.x + h.y * h.y;
        }
        f = block_sum(f, S.red);
        if (tid < K) {
            if (a.precoder == DMIMO_MR)
                S.scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total) / sqrt(f) : 1.0;
            else
                S.scale[tid] = a.p_total > 0.0 ? sqrt(a.p_total / ((double)K * (double)M)) : 1.0;
        }
        __syncthreads();
    }

    // 4-5. tiles of kCols antennas
    // column pass: thread -> (column c = tid / 4, row group g = tid % 4, rows g, g+4, ...)
    const int cc = tid >> 2;
    const int rg = tid & 3;
    // gains: the K x K matrix in 8 x 8 blocks of BS x BS entries; block tid / 4,
    // antennas c = tid % 4 (mod 4).  A block reuses each h and w value it reads
    // BS times.
    constexpr int BS = KT / 8;
    const int k0 = BS * (cc >> 3), j0 = BS * (cc & 7);
    double2 acc[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) acc[u][v] = make_double2(0.0, 0.0);
    double l21 = 0.0;
    const bool want_gain = a.sinr || a.rsum;

    for (int64_t m0 = 0; m0 < M; m0 += kCols) {
        const int mc = (int)(M - m0 < kCols ? M - m0 : kCols);
        __syncthreads();
        for (int e = tid; e < K * kCols; e += kThreads) {
            const int k = e / kCols, c = e - k * kCols;
            if (c < mc) S.u.t.h[k][c] = Hb[(int64_t)k * M + m0 + c];
        }
        __syncthreads();
        if (cc < mc) {
            const int64_t m = m0 + cc;
            double pm = 0.0;
            // ZF: x_k = sum_j G^-1[k][j] h_j for this thread's users k = rg + 4 t,
            // each h_j read once
            constexpr int KU = KT / 4;
            double2 x[KU];
            if (a.precoder == DMIMO_ZF) {
#pragma unroll
                for (int t = 0; t < KU; ++t) x[t] = make_double2(0.0, 0.0);
                for (int j = 0; j < K; ++j) {
                    const double2 hj = to_d2(S.u.t.h[j][cc]);
#pragma unroll
                    for (int t = 0; t < KU; ++t) cfma(x[t], S.ginv[rg + 4 * t][j], hj);
                }
            }
#pragma unroll
            for (int t = 0; t < KU; ++t) {
                const int k = rg + 4 * t;
                if (k >= K) break;
                double2 w;
                if (a.precoder == DMIMO_ZF) {
                    w = make_double2(S.scale[k] * x[t].x, -S.scale[k] * x[t].y);
                } else {
                    const double2 h = to_d2(S.u.t.h[k][cc]);
                    if (a.precoder == DMIMO_MR) {
                        w = make_double2(S.scale[k] * h.x, -S.scale[k] * h.y);
                    } else {
                        const double mag = sqrt(h.x * h.x + h.y * h.y);
                        w = mag > 0.0 ? make_double2(S.scale[k] * h.x / mag, -S.scale[k] * h.y / mag)
                                      : make_double2(S.scale[k], 0.0);
                    }
                }
                T2 ws;
                ws.x = w.x;
                ws.y = w.y;
                Wb[(int64_t)k * M + m] = ws;
                S.u.t.w[k][cc] = ws;
                pm += (double)ws.x * (double)ws.x + (double)ws.y * (double)ws.y;
            }
            // the four threads of a column are adjacent lanes
            pm += __shfl_xor(pm, 1, 64);
            pm += __shfl_xor(pm, 2, 64);
            if (rg == 0) {
                if (a.p_ant) a.p_ant[b * M + m] = pm;
                l21 += sqrt(pm);
            }
        }
        if (!want_gain) continue;
        __syncthreads();
        if (k0 < K && j0 < K)
            for (int c = rg; c < mc; c += 4) {
                double2 hk[BS], wj[BS];
#pragma unroll
                for (int u = 0; u < BS; ++u) {
                    hk[u] = k0 + u < K ? to_d2(S.u.t.h[k0 + u][c]) : make_double2(0.0, 0.0);
                    wj[u] = j0 + u < K ? to_d2(S.u.t.w[j0 + u][c]) : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < BS; ++u)
#pragma unroll
                    for (int v = 0; v < BS; ++v) cfma(acc[u][v], hk[u], wj[v]);
            }
    }
    l21 = block_sum(l21, S.red);
    if (tid == 0) {
        if (a.l21) a.l21[b] = l21;
        if (a.info) a.info[b] = 0;
    }
    if (!want_gain) return;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) {
            double2 t = acc[u][v];
            t.x += __shfl_xor(t.x, 1, 64);
            t.y += __shfl_xor(t.y, 1, 64);
            t.x += __shfl_xor(t.x, 2, 64);
            t.y += __shfl_xor(t.y, 2, 64);
            if (rg == 0 && k0 + u < K && j0 + v < K) S.u.A[k0 + u][j0 + v] = t;
        }
    __syncthreads();
    double rate = 0.0;
    if (tid < K) {
        const int k = tid;
        double sig = 0.0, intf = 0.0;
        for (int j = 0; j < K; ++j) {
            const double2 v = S.u.A[k][j];
            const double p = v.x * v.x + v.y * v.y;
            if (j == k) sig = p;
            else intf += p;
        }
        const double snr = sig / (intf + a.sigma2);
        if (a.sinr) a.sinr[b * K + k] = snr;
        rate = log2(1.0 + snr);
    }
    rate = block_sum(rate, S.red);
    if (tid == 0 && a.rsum) a.rsum[b] = rate;
}

// Deployments of at most 8 users and kSmallMaxM antennas (kSmallMaxM / 2 in
// FP64) in one pass, H and W resident in LDS, five barriers (three for MR):
//   1. H -> LDS; per-wave partials of ||H||_F^2 (MR).
//   2. ZF: G = H H^H in FP64 from the stored H, four threads per entry (no
//      Gram launch; the call's precision does not apply to this G).
//   3. ZF: wave 0 inverts G by Gauss-Jordan elimination without pivoting, one
//      lane per entry of G padded to 8 x 8 with the identity.  For a
//      Hermitian positive definite G the pivot of step p is the diagonal entry
//      of the Schur complement left after p steps, which is L_pp^2 of the
//      Cholesky factor: the pivot test is the general kernel's.
//      tr(G^-1) is the sum of the inverse's diagonal.
//   4. W and p_m as in the general kernel.
//   5. Gains A = H W^T in FP64 from the two LDS arrays; SINR, sum rate and
//      ||W||_{2,1} in wave 0.
constexpr int kSmallK = 8;
constexpr int kSmallMaxM = 256;

template <typename T2, int MT>
struct BfSmallShared {
    T2 h[kSmallK][MT + 1];
    T2 w[kSmallK][MT + 1];
    double2 g[kSmallK][kSmallK + 1];   // G, then G^-1
    double2 A[kSmallK][kSmallK + 1];   // gains
    double red[kThreads / 64];         // ||H||_F^2 per wave
    double red2[kThreads / 64];        // ||W||_{2,1} per wave
    double scale[kSmallK];
    int fail;
};

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double lane_value(double v, int l) {   // l uniform over the wave
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

template <typename T2, int MT>
__global__ __launch_bounds__(kThreads) void beamform_small_kernel(BfDev a) {
    __shared__ BfSmallShared<T2, MT> S;

    const int64_t b = blockIdx.x;
    const int K = a.K;
    const int M = (int)a.M;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + b * K * M;
    const bool zf = a.precoder == DMIMO_ZF;
    // antenna (tid / 4 within a tile of 64) and user phase (tid % 4) in step 4;
    // entry (tid / 4 = 8 i + j) and antenna phase (tid % 4) in steps 2 and 5
    const int cc = tid >> 2, rg = tid & 3;
    const int ei = cc >> 3, ej = cc & 7;

    // 1.
    double f = 0.0;
    for (int e = tid; e < K * M; e += kThreads) {
        const int k = e / M, c = e - k * M;
        const T2 v = Hb[e];
        S.h[k][c] = v;
        f += (double)v.x * v.x + (double)v.y * v.y;
    }
    f = wave_sum(f);
    if (lane == 0) S.red[wv] = f;
    __syncthreads();

    double mr_scale = 1.0;
    if (zf) {
        // 2.
        double2 s = make_double2(0.0, 0.0);
        if (ei < K && ej < K)
            for (int c = rg; c < M; c += 4) {
                const double2 x = to_d2(S.h[ei][c]), y = to_d2(S.h[ej][c]);
                s.x = fma(x.x, y.x, fma(x.y, y.y, s.x));
                s.y = fma(x.y, y.x, fma(-x.x, y.y, s.y));
            }
        s.x += __shfl_xor(s.x, 1, 64);
        s.y += __shfl_xor(s.y, 1, 64);
        s.x += __shfl_xor(s.x, 2, 64);
        s.y += __shfl_xor(s.y, 2, 64);
        if (rg == 0 && ei < K && ej < K) S.g[ei][ej] = ei == ej ? make_double2(s.x, 0.0) : s;
        __syncthreads();
        // 3.
        if (wv == 0) {
            const int i = lane >> 3, j = lane & 7;
            double2 g = (i < K && j < K) ? S.g[i][j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
            const double g0 = g.x;
            int fail = 0;
            for (int p = 0; p < K; ++p) {
                const double piv = lane_value(g.x, 9 * p);
                if (!(piv > a.pivot_tol * lane_value(g0, 9 * p))) {
                    fail = p + 1;
                    break;
                }
                const double inv = 1.0 / piv;
                const double2 gpj = make_double2(__shfl(g.x, 8 * p + j, 64), __shfl(g.y, 8 * p + j, 64));
                const double2 gip = make_double2(__shfl(g.x, 8 * i + p, 64), __shfl(g.y, 8 * i + p, 64));
                // row p of the reduced system; the slot of column p takes the
                // inverse's column p
                const double2 r = j == p ? make_double2(inv, 0.0) : make_double2(gpj.x * inv, gpj.y * inv);
                if (i == p) {
                    g = r;
                } else {
                    const double2 base = j == p ? make_double2(0.0, 0.0) : g;
                    g = make_double2(fma(-gip.x, r.x, fma(gip.y, r.y, base.x)),
                                     fma(-gip.x, r.y, fma(-gip.y, r.x, base.y)));
                }
            }
            const double tr = wave_sum(i == j && i < K ? g.x : 0.0);
            if (i < K && j < K) S.g[i][j] = g;
            if (lane < K)
                S.scale[lane] = a.p_total > 0.0 ? sqrt(a.p_total / tr) : sqrt(a.sigma2) * sqrt(a.gamma[lane]);
            if (lane == 0) S.fail = fail;
        }
        __syncthreads();
        if (S.fail) {
            for (int e = tid; e < K * M; e += kThreads) {
                T2 z;
                z.x = 0;
                z.y = 0;
                Wb[e] = z;
            }
            if (a.p_ant)
                for (int m = tid; m < M; m += kThreads) a.p_ant[b * M + m] = 0.0;
            if (a.sinr && tid < K) a.sinr[b * K + tid] = 0.0;
            if (tid == 0) {
                if (a.l21) a.l21[b] = 0.0;
                if (a.rsum) a.rsum[b] = 0.0;
                if (a.info) a.info[b] = S.fail;
            }
            return;
        }
    } else if (a.precoder == DMIMO_MR) {
        const double fs = S.red[0] + S.red[1] + S.red[2] + S.red[3];
        mr_scale = a.p_total > 0.0 ? sqrt(a.p_total) / sqrt(fs) : 1.0;
    } else {
        mr_scale = a.p_total > 0.0 ? sqrt(a.p_total / ((double)K * (double)M)) : 1.0;
    }

    // 4.
    double l21 = 0.0;
    for (int m0 = 0; m0 < M; m0 += 64) {
        const int c = m0 + cc;
        if (c >= M) break;
        double pm = 0.0;
        for (int k = rg; k < K; k += 4) {
            double2 w;
            if (zf) {
                double2 x = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < kSmallK; ++j) {
                    if (j >= K) break;
                    cfma(x, S.g[k][j], to_d2(S.h[j][c]));
                }
                w = make_double2(S.scale[k] * x.x, -S.scale[k] * x.y);
            } else {
                const double2 h = to_d2(S.h[k][c]);
                if (a.precoder == DMIMO_MR) {
                    w = make_double2(mr_scale * h.x, -mr_scale * h.y);
                } else {
                    const double mag = sqrt(h.x * h.x + h.y * h.y);
                    w = mag > 0.0 ? make_double2(mr_scale * h.x / mag, -mr_scale * h.y / mag)
                                  : make_double2(mr_scale, 0.0);
                }
            }
            T2 ws;
            ws.x = w.x;
            ws.y = w.y;
            Wb[(int64_t)k * M + c] = ws;
            S.w[k][c] = ws;
            pm += (double)ws.x * (double)ws.x + (double)ws.y * (double)ws.y;
        }
        // the four threads of an antenna are adjacent lanes
        pm += __shfl_xor(pm, 1, 64);
        pm += __shfl_xor(pm, 2, 64);
        if (rg == 0) {
            if (a.p_ant) a.p_ant[b * M + c] = pm;
            l21 += sqrt(pm);
        }
    }
    l21 = wave_sum(l21);
    if (lane == 0) S.red2[wv] = l21;
    __syncthreads();

    // 5.
    const bool want_gain = a.sinr || a.rsum;
    if (want_gain) {
        double2 s = make_double2(0.0, 0.0);
        if (ei < K && ej < K)
            for (int c = rg; c < M; c += 4) cfma(s, to_d2(S.h[ei][c]), to_d2(S.w[ej][c]));
        s.x += __shfl_xor(s.x, 1, 64);
        s.y += __shfl_xor(s.y, 1, 64);
        s.x += __shfl_xor(s.x, 2, 64);
        s.y += __shfl_xor(s.y, 2, 64);
        if (rg == 0 && ei < K && ej < K) S.A[ei][ej] = s;
        __syncthreads();
    }
    if (wv != 0) return;
    double rate = 0.0;
    if (want_gain && lane < K) {
        double sig = 0.0, intf = 0.0;
        for (int j = 0; j < K; ++j) {
            const double2 v = S.A[lane][j];
            const double p = v.x * v.x + v.y * v.y;
            if (j == lane) sig = p;
            else intf += p;
        }
        const double snr = sig / (intf + a.sigma2);
        if (a.sinr) a.sinr[b * K + lane] = snr;
        rate = log2(1.0 + snr);
    }
    rate = wave_sum(rate);
    if (lane == 0) {
        if (a.rsum) a.rsum[b] = rate;
        if (a.l21) a.l21[b] = S.red2[0] + S.red2[1] + S.red2[2] + S.red2[3];
        if (a.info) a.info[b] = 0;
    }
}

template <typename T2>
dmimo_status launch_typed(const BfDev& d, int64_t B, hipStream_t s) {
    dim3 grid((unsigned)B), block(kThreads);
    if (d.K <= 8) beamform_kernel<T2, 8><<<grid, block, 0, s>>>(d);
    else if (d.K <= 16) beamform_kernel<T2, 16><<<grid, block, 0, s>>>(d);
    else beamform_kernel<T2, 32><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_kernel");
}

// The one-pass kernel's antenna limit: LDS holds H and W, 8 x (MT + 1) each.
int64_t small_max_m(int prec) { return prec == DMIMO_F64 ? kSmallMaxM / 2 : kSmallMaxM; }

template <typename T2, int MT_WIDE>
dmimo_status launch_small(const BfDev& d, int64_t B, hipStream_t s) {
    dim3 grid((unsigned)B), block(kThreads);
    if (d.M <= 64) beamform_small_kernel<T2, 64><<<grid, block, 0, s>>>(d);
    else beamform_small_kernel<T2, MT_WIDE><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_small_kernel");
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
    if (a.K <= kSmallK && a.M <= small_max_m(a.prec)) {
        // G is formed in FP64 in the kernel, so the FP64 Gram's tolerance
        // applies to FP64 input and the FP32 one to every other mode
        d.pivot_tol = a.prec == DMIMO_F64 ? 1e-12 : 1e-6;
        if (a.prec == DMIMO_F64) return launch_small<double2, kSmallMaxM / 2>(d, a.B, s);
        return launch_small<float2, kSmallMaxM>(d, a.B, s);
    }
    if (a.precoder == DMIMO_ZF) {
        dmimo_status st = launch_gram(a.B, a.K, a.M, a.H, a.prec, a.ws, s);
        if (st) return st;
    }
    if (a.prec == DMIMO_F64) return launch_typed<double2>(d, a.B, s);
    return launch_typed<float2>(d, a.B, s);
}

}  // namespace dmimo
