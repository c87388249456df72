// Precoders and their epilogues, one 256-thread workgroup per deployment.
// Deployments of at most 8 users and 256 antennas (128 in FP64) take the
// one-pass kernel further down (several precoders of the same channels in one
// launch, precoder p on grid row p; it can also synthesise the users' LoS
// channels itself and write them out); calls of at most 64 deployments with
// M > 448 take the wide path, which spreads each deployment over workgroups
// of 64 antennas; the general kernel follows.
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

constexpr int kMultiMax = 8;   // precoders per multi-precoder call

struct BfDev {
    int precoder;
    int precs[kMultiMax];   // one-pass kernel: precoder of grid row p
    int64_t B;
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
    // one-pass kernel only: the users' channels synthesised in the kernel
    // (user_xyz != NULL) from [B][K][3] users and [B][M][3] antennas, and
    // written to H_out by grid row 0
    const double* user_xyz;
    const double* ap_xyz;
    double inv_lam, amp_c, inv_dmin;
    void* H_out;
};

// One LoS term of the channel synthesis, with the channel kernel's arithmetic
// (the same bits): h = amp (cos - j sin) of the FP32 or FP64 term.
template <typename T2>
__device__ __forceinline__ T2 synth_term(const BfDev& a, double dx, double dy, double dz);
template <>
__device__ __forceinline__ float2 synth_term<float2>(const BfDev& a, double dx, double dy, double dz) {
    const TermF32 t = wave_term_f32(dx, dy, dz, a.inv_lam, (float)a.amp_c, (float)a.inv_dmin);
    return make_float2(t.amp * t.c, -t.amp * t.s);
}
template <>
__device__ __forceinline__ double2 synth_term<double2>(const BfDev& a, double dx, double dy, double dz) {
    const TermF64 t = wave_term_f64(dx, dy, dz, a.inv_lam, a.amp_c, a.inv_dmin);
    return make_double2(t.amp * t.c, -t.amp * t.s);
}

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

// Gauss-Jordan elimination without pivoting of the K x K matrix in g (LDS),
// in place, by all threads of the workgroup: each step reads its pivot row
// and column, then every thread writes its entries.  The pivot of step p is
// the diagonal entry of the Schur complement (L_pp^2 of the Cholesky factor);
// one not above tol * d0[p] stops the elimination.  Returns 0, or p + 1 for
// the failed step (the same value in every thread).
template <int KT>
__device__ int gj_invert(double2 (*g)[KT + 1], const double* d0, int K, double tol) {
    constexpr int QG = (KT * KT + kThreads - 1) / kThreads;
    const int tid = threadIdx.x;
    for (int p = 0; p < K; ++p) {
        const double piv = g[p][p].x;
        if (!(piv > tol * d0[p])) return p + 1;
        const double inv = 1.0 / piv;
        double2 nv[QG];
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            const int e = tid + kThreads * q;
            if (e < K * K) {
                const int i = e / K, j = e - (e / K) * K;
                const double2 gpj = g[p][j], gip = g[i][p];
                const double2 r = j == p ? make_double2(inv, 0.0) : make_double2(gpj.x * inv, gpj.y * inv);
                if (i == p) {
                    nv[q] = r;
                } else {
                    const double2 x = j == p ? make_double2(0.0, 0.0) : g[i][j];
                    nv[q] = make_double2(fma(-gip.x, r.x, fma(gip.y, r.y, x.x)),
                                         fma(-gip.x, r.y, fma(-gip.y, r.x, x.y)));
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            const int e = tid + kThreads * q;
            if (e < K * K) g[e / K][e - (e / K) * K] = nv[q];
        }
        __syncthreads();
    }
    return 0;
}

// Loads G[b] (as written by the Gram) into g and its diagonal into d0.
template <typename T2, int KT>
__device__ void load_gram(const BfDev& a, int64_t b, double2 (*g)[KT + 1], double* d0) {
    const int K = a.K;
    const T2* Gb = reinterpret_cast<const T2*>(a.G) + b * K * K;
    for (int e = threadIdx.x; e < K * K; e += kThreads) {
        const int i = e / K, j = e - (e / K) * K;
        const double2 v = to_d2(Gb[e]);
        g[i][j] = v;
        if (i == j) d0[i] = v.x;
    }
}

template <int KT>
__device__ __forceinline__ double zf_scale(const BfDev& a, double tr, int k) {
    return a.p_total > 0.0 ? sqrt(a.p_total / tr) : sqrt(a.sigma2) * sqrt(a.gamma[k]);
}

// Thread roles of one 64-antenna tile (256 threads):
//   column pass: antenna cc = tid / 4, users rg, rg + 4, ... (rg = tid % 4);
//   gains: the K x K matrix in 8 x 8 blocks of BS x BS entries, block tid / 4,
//   antennas c = rg (mod 4); a block reuses each h and w value it reads BS times.
template <int KT>
struct TileRoles {
    static constexpr int BS = KT / 8;
    int cc, rg, k0, j0;
    __device__ TileRoles() {
        cc = threadIdx.x >> 2;
        rg = threadIdx.x & 3;
        k0 = BS * (cc >> 3);
        j0 = BS * (cc & 7);
    }
};

// Stages H[b][:, m0 .. m0 + mc) into h (LDS) with 256 threads: a thread's
// KT/4 loads are all issued before its LDS stores.
template <typename T2>
struct Scalar;
template <>
struct Scalar<float2> {
    using type = float;
};
template <>
struct Scalar<double2> {
    using type = double;
};

// (The staged values are kept as scalar arrays, which stay in registers; an
// array of vector-type unions can end up in scratch.)
template <typename T2, int KT>
__device__ __forceinline__ void stage_tile(const T2* Hb, int K, int64_t M, int64_t m0, int mc,
                                           T2 (*h)[kCols + 1]) {
    using S = typename Scalar<T2>::type;
    constexpr int IT = KT * kCols / kThreads;
    S vx[IT], vy[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + kThreads * it;
        const int k = e / kCols, c = e - k * kCols;
        if (k < K && c < mc) {
            const T2 t = Hb[(int64_t)k * M + m0 + c];
            vx[it] = t.x;
            vy[it] = t.y;
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + kThreads * it;
        const int k = e / kCols, c = e - k * kCols;
        if (k < K && c < mc) {
            T2 t;
            t.x = vx[it];
            t.y = vy[it];
            h[k][c] = t;
        }
    }
}

// One tile, with H[b][:, m0 .. m0 + mc) already in h (LDS): forms and stores
// W and p_m (scale[k] per user; ZF: W = scale conj(G^-1 h)), adds sqrt(p_m) to
// l21 and, if want_gain, the tile's share of A = H W^T to acc.
template <typename T2, int KT>
__device__ void bf_tile(const BfDev& a, int64_t b, int64_t m0, int mc, const TileRoles<KT>& R,
                        const double2 (*ginv)[KT + 1], const double* scale, const T2 (*h)[kCols + 1],
                        T2 (*w)[kCols + 1], bool want_gain,
                        double2 (&acc)[TileRoles<KT>::BS][TileRoles<KT>::BS], double& l21) {
    constexpr int BS = TileRoles<KT>::BS;
    const int K = a.K;
    const int64_t M = a.M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + b * K * M;
    const int cc = R.cc, rg = R.rg;
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
                const double2 hj = to_d2(h[j][cc]);
#pragma unroll
                for (int t = 0; t < KU; ++t) cfma(x[t], ginv[rg + 4 * t][j], hj);
            }
        }
#pragma unroll
        for (int t = 0; t < KU; ++t) {
            const int k = rg + 4 * t;
            if (k >= K) break;
            double2 wv;
            if (a.precoder == DMIMO_ZF) {
                wv = make_double2(scale[k] * x[t].x, -scale[k] * x[t].y);
            } else {
                const double2 hk = to_d2(h[k][cc]);
                if (a.precoder == DMIMO_MR) {
                    wv = make_double2(scale[k] * hk.x, -scale[k] * hk.y);
                } else {
                    const double mag = sqrt(hk.x * hk.x + hk.y * hk.y);
                    wv = mag > 0.0 ? make_double2(scale[k] * hk.x / mag, -scale[k] * hk.y / mag)
                                   : make_double2(scale[k], 0.0);
                }
            }
            T2 ws;
            ws.x = wv.x;
            ws.y = wv.y;
            Wb[(int64_t)k * M + m] = ws;
            w[k][cc] = ws;
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
    if (!want_gain) return;
    __syncthreads();
    const int k0 = R.k0, j0 = R.j0;
    if (k0 < K && j0 < K)
        for (int c = rg; c < mc; c += 4) {
            double2 hk[BS], wj[BS];
#pragma unroll
            for (int u = 0; u < BS; ++u) {
                hk[u] = k0 + u < K ? to_d2(h[k0 + u][c]) : make_double2(0.0, 0.0);
                wj[u] = j0 + u < K ? to_d2(w[j0 + u][c]) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < BS; ++u)
#pragma unroll
                for (int v = 0; v < BS; ++v) cfma(acc[u][v], hk[u], wj[v]);
        }
}

// Sum of a block's partial gains over its four antenna phases (adjacent lanes).
template <int BS>
__device__ __forceinline__ double2 phase_sum(double2 t) {
    t.x += __shfl_xor(t.x, 1, 64);
    t.y += __shfl_xor(t.y, 1, 64);
    t.x += __shfl_xor(t.x, 2, 64);
    t.y += __shfl_xor(t.y, 2, 64);
    return t;
}

// SINR_k of the gains A (LDS) and the sum rate, by the first wave.
template <int KT>
__device__ void gains_epilogue(const BfDev& a, int64_t b, const double2 (*A)[KT + 1], double* red) {
    const int K = a.K;
    double rate = 0.0;
    const int tid = threadIdx.x;
    if (tid < K) {
        double sig = 0.0, intf = 0.0;
        for (int j = 0; j < K; ++j) {
            const double2 v = A[tid][j];
            const double p = v.x * v.x + v.y * v.y;
            if (j == tid) sig = p;
            else intf += p;
        }
        const double snr = sig / (intf + a.sigma2);
        if (a.sinr) a.sinr[b * K + tid] = snr;
        rate = log2(1.0 + snr);
    }
    rate = block_sum(rate, red);
    if (tid == 0 && a.rsum) a.rsum[b] = rate;
}

// Outputs of a deployment whose ZF pivot p failed: W, p_m, SINR, ||W||_{2,1}
// and the sum rate zero, info = p.  The W and p_m zeros cover the antennas
// [m_lo, m_hi); the rest is written by thread block `owner` only.
template <typename T2>
__device__ void zf_failed(const BfDev& a, int64_t b, int fail, int64_t m_lo, int64_t m_hi, bool owner) {
    const int K = a.K, tid = threadIdx.x;
    const int64_t M = a.M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + b * K * M;
    for (int64_t e = tid; e < (int64_t)K * (m_hi - m_lo); e += kThreads) {
        const int64_t k = e / (m_hi - m_lo), m = m_lo + (e - k * (m_hi - m_lo));
        T2 z;
        z.x = 0;
        z.y = 0;
        Wb[k * M + m] = z;
    }
    if (a.p_ant)
        for (int64_t m = m_lo + tid; m < m_hi; m += kThreads) a.p_ant[b * M + m] = 0.0;
    if (!owner) return;
    if (a.sinr)
        for (int k = tid; k < K; k += kThreads) a.sinr[b * K + k] = 0.0;
    if (tid == 0) {
        if (a.l21) a.l21[b] = 0.0;
        if (a.rsum) a.rsum[b] = 0.0;
        if (a.info) a.info[b] = fail;
    }
}

template <typename T2, int KT>
__global__ __launch_bounds__(kThreads) void beamform_kernel(BfDev a) {
    __shared__ BfShared<T2, KT> S;
    constexpr int BS = TileRoles<KT>::BS;

    const int64_t b = blockIdx.x;
    const int K = a.K;
    const int64_t M = a.M;
    const int tid = threadIdx.x;
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;

    if (a.precoder == DMIMO_ZF) {
        load_gram<T2, KT>(a, b, S.ginv, S.d0);
        __syncthreads();
        // 1. G^-1 in place
        const int fail = gj_invert<KT>(S.ginv, S.d0, K, a.pivot_tol);
        if (fail) {
            zf_failed<T2>(a, b, fail, 0, M, true);
            return;
        }
        double tr = 0.0;   // tr(G^-1)
        for (int k = 0; k < K; ++k) tr += S.ginv[k][k].x;
        if (tid < K) S.scale[tid] = zf_scale<KT>(a, tr, tid);
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

    // 2-3. tiles of kCols antennas
    const TileRoles<KT> R;
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
        stage_tile<T2, KT>(Hb, K, M, m0, mc, S.u.t.h);
        __syncthreads();
        bf_tile<T2, KT>(a, b, m0, mc, R, S.ginv, S.scale, S.u.t.h, S.u.t.w, want_gain, acc, l21);
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
            const double2 t = phase_sum<BS>(acc[u][v]);
            if (R.rg == 0 && R.k0 + u < K && R.j0 + v < K) S.u.A[R.k0 + u][R.j0 + v] = t;
        }
    __syncthreads();
    gains_epilogue<KT>(a, b, S.u.A, S.red);
}

// ---------------------------------------------------------------------------
// Few deployments with many antennas (B <= kWideMaxB, at least kWideMinTiles
// tiles of 64 antennas), every step spread over the tiles:
//   bfw_gram_kernel   ZF, per (tile, deployment): the tile's share of G, FP64;
//   bfw_prep_kernel   ZF, per deployment: G = the shares summed in tile order
//                     (FP64 in every mode), inverted by Gauss-Jordan;
//   bfw_norm_kernel   MR with p_total > 0, per (tile, deployment): the tile's
//                     share of ||H||_F^2;
//   bfw_tile_kernel   per (tile, deployment): the scale (MR: from the norm
//                     shares in tile order, the same bits in every tile), W,
//                     p_m and the tile's share of the gains A = H W^T;
//   bfw_final_kernel  per deployment: the shares summed in tile order, SINR,
//                     sum rate, ||W||_{2,1}.
// Workspace: ZF first holds the Gram slot, G^-1 [B][K][K] and scale [B][K]
// (FP64) and the failed pivot [B]; then, for every precoder, tile shares
// [B][T][K][K] (FP64; ZF: first of G, then of the gains) and sqrt(p_m) sums
// [B][T]; MR and equal-gain MR end with the ||H||_F^2 shares [B][T].
// ---------------------------------------------------------------------------
constexpr int64_t kWideMaxB = 64;
constexpr int64_t kWideMinTiles = 8;

struct BfWide {
    double2* ginv;
    double* scale;
    int32_t* fail;
    double2* gpart;
    double* lpart;
    double* npart;
    int64_t T;
};

// The tile's share of ||H||_F^2: each thread's staged values in a fixed order,
// then the block sum.
template <typename T2, int KT>
__global__ __launch_bounds__(kThreads) void bfw_norm_kernel(BfDev a, BfWide wd) {
    __shared__ double red[kThreads / 64];
    using S = typename Scalar<T2>::type;
    constexpr int IT = KT * kCols / kThreads;
    const int64_t t = blockIdx.x, b = blockIdx.y;
    const int K = a.K;
    const int64_t M = a.M, m0 = t * kCols;
    const int mc = (int)(M - m0 < kCols ? M - m0 : kCols);
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    S vx[IT], vy[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + kThreads * it;
        const int k = e / kCols, c = e - k * kCols;
        vx[it] = 0;
        vy[it] = 0;
        if (k < K && c < mc) {
            const T2 v = Hb[(int64_t)k * M + m0 + c];
            vx[it] = v.x;
            vy[it] = v.y;
        }
    }
    double f = 0.0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const double x = vx[it], y = vy[it];
        f += x * x + y * y;
    }
    f = block_sum(f, red);
    if (threadIdx.x == 0) wd.npart[b * wd.T + t] = f;
}

// The tile's share of G = H H^H, FP64 sums, in the gain-share slot of the
// workspace (consumed by bfw_prep_kernel before the tiles overwrite it).
template <typename T2, int KT>
__global__ __launch_bounds__(kThreads) void bfw_gram_kernel(BfDev a, BfWide wd) {
    __shared__ T2 h[KT][kCols + 1];
    constexpr int BS = TileRoles<KT>::BS;
    const int64_t t = blockIdx.x, b = blockIdx.y;
    const int K = a.K, tid = threadIdx.x;
    const int64_t M = a.M, m0 = t * kCols;
    const int mc = (int)(M - m0 < kCols ? M - m0 : kCols);
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    stage_tile<T2, KT>(Hb, K, M, m0, mc, h);
    __syncthreads();
    const TileRoles<KT> R;
    double2 acc[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) acc[u][v] = make_double2(0.0, 0.0);
    if (R.k0 < K && R.j0 < K)
        for (int c = R.rg; c < mc; c += 4) {
            double2 hk[BS], hj[BS];
#pragma unroll
            for (int u = 0; u < BS; ++u) {
                hk[u] = R.k0 + u < K ? to_d2(h[R.k0 + u][c]) : make_double2(0.0, 0.0);
                hj[u] = R.j0 + u < K ? to_d2(h[R.j0 + u][c]) : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < BS; ++u)
#pragma unroll
                for (int v = 0; v < BS; ++v) {   // h_k conj(h_j)
                    acc[u][v].x = fma(hk[u].x, hj[v].x, fma(hk[u].y, hj[v].y, acc[u][v].x));
                    acc[u][v].y = fma(hk[u].y, hj[v].x, fma(-hk[u].x, hj[v].y, acc[u][v].y));
                }
        }
    double2* gp = wd.gpart + (b * wd.T + t) * K * K;
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) {
            const double2 sum = phase_sum<BS>(acc[u][v]);
            if (R.rg == 0 && R.k0 + u < K && R.j0 + v < K) gp[(R.k0 + u) * K + R.j0 + v] = sum;
        }
}

// G of deployment b from the tiles' shares (tile order; the diagonal's
// imaginary part set to zero), inverted in place; G^-1, the scale and the
// failed pivot to the workspace.
template <int KT>
__global__ __launch_bounds__(kThreads) void bfw_prep_kernel(BfDev a, BfWide wd) {
    __shared__ double2 g[KT][KT + 1];
    __shared__ double d0[KT];
    const int64_t b = blockIdx.x;
    const int K = a.K, tid = threadIdx.x;
    for (int e = tid; e < K * K; e += kThreads) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int64_t t = 0; t < wd.T; ++t) {   // loads issued together, sums in tile order
            const double2 v = wd.gpart[(b * wd.T + t) * K * K + e];
            s.x += v.x;
            s.y += v.y;
        }
        const int i = e / K, j = e - (e / K) * K;
        if (i == j) {
            s.y = 0.0;
            d0[i] = s.x;
        }
        g[i][j] = s;
    }
    __syncthreads();
    const int fail = gj_invert<KT>(g, d0, K, a.pivot_tol);
    for (int e = tid; e < K * K; e += kThreads) wd.ginv[b * K * K + e] = g[e / K][e - (e / K) * K];
    double tr = 0.0;
    for (int k = 0; k < K; ++k) tr += g[k][k].x;
    if (tid < K) wd.scale[b * K + tid] = fail ? 0.0 : zf_scale<KT>(a, tr, tid);
    if (tid == 0) wd.fail[b] = fail;
}

template <typename T2, int KT>
__global__ __launch_bounds__(kThreads) void bfw_tile_kernel(BfDev a, BfWide wd) {
    __shared__ double2 ginv[KT][KT + 1];
    __shared__ T2 h[KT][kCols + 1];
    __shared__ T2 w[KT][kCols + 1];
    __shared__ double scale[KT];
    __shared__ double red[kThreads / 64];
    constexpr int BS = TileRoles<KT>::BS;
    const int64_t t = blockIdx.x, b = blockIdx.y;
    const int K = a.K, tid = threadIdx.x;
    const int64_t M = a.M, m0 = t * kCols;
    const int mc = (int)(M - m0 < kCols ? M - m0 : kCols);
    const bool zf = a.precoder == DMIMO_ZF;
    const int fail = zf ? wd.fail[b] : 0;
    if (fail) {
        zf_failed<T2>(a, b, fail, m0, m0 + mc, false);
        return;
    }
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    if (zf) {
        for (int e = tid; e < K * K; e += kThreads) ginv[e / K][e - (e / K) * K] = wd.ginv[b * K * K + e];
        if (tid < K) scale[tid] = wd.scale[b * K + tid];
    } else if (a.precoder == DMIMO_MR && a.p_total > 0.0) {
        // ||H||_F^2 from the tiles' shares: a fixed order, so every tile of
        // the deployment gets the same scale
        double f = 0.0;
        for (int64_t i = tid; i < wd.T; i += kThreads) f += wd.npart[b * wd.T + i];
        f = block_sum(f, red);
        if (tid < K) scale[tid] = sqrt(a.p_total) / sqrt(f);
    } else if (tid < K) {
        scale[tid] = a.precoder == DMIMO_MR_PHASE && a.p_total > 0.0
                         ? sqrt(a.p_total / ((double)K * (double)M))
                         : 1.0;
    }
    stage_tile<T2, KT>(Hb, K, M, m0, mc, h);
    __syncthreads();
    const TileRoles<KT> R;
    double2 acc[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) acc[u][v] = make_double2(0.0, 0.0);
    double l21 = 0.0;
    const bool want_gain = a.sinr || a.rsum;
    bf_tile<T2, KT>(a, b, m0, mc, R, ginv, scale, h, w, want_gain, acc, l21);
    l21 = block_sum(l21, red);
    if (tid == 0) wd.lpart[b * wd.T + t] = l21;
    if (!want_gain) return;
    double2* gp = wd.gpart + (b * wd.T + t) * K * K;
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) {
            const double2 s = phase_sum<BS>(acc[u][v]);
            if (R.rg == 0 && R.k0 + u < K && R.j0 + v < K) gp[(R.k0 + u) * K + R.j0 + v] = s;
        }
}

template <int KT>
__global__ __launch_bounds__(kThreads) void bfw_final_kernel(BfDev a, BfWide wd) {
    __shared__ double2 A[KT][KT + 1];
    __shared__ double red[kThreads / 64];
    const int64_t b = blockIdx.x;
    const int K = a.K, tid = threadIdx.x;
    const int fail = a.precoder == DMIMO_ZF ? wd.fail[b] : 0;
    if (fail) {
        if (a.sinr)
            for (int k = tid; k < K; k += kThreads) a.sinr[b * K + k] = 0.0;
        if (tid == 0) {
            if (a.l21) a.l21[b] = 0.0;
            if (a.rsum) a.rsum[b] = 0.0;
            if (a.info) a.info[b] = fail;
        }
        return;
    }
    const bool want_gain = a.sinr || a.rsum;
    if (want_gain) {
        for (int e = tid; e < K * K; e += kThreads) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll 8
            for (int64_t t = 0; t < wd.T; ++t) {   // loads issued together, sums in tile order
                const double2 v = wd.gpart[(b * wd.T + t) * K * K + e];
                s.x += v.x;
                s.y += v.y;
            }
            A[e / K][e - (e / K) * K] = s;
        }
        __syncthreads();
        gains_epilogue<KT>(a, b, A, red);
    }
    if (tid == 0) {
        double l = 0.0;
        for (int64_t t = 0; t < wd.T; ++t) l += wd.lpart[b * wd.T + t];
        if (a.l21) a.l21[b] = l;
        if (a.info) a.info[b] = 0;
    }
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
    // grid row `row`: precoder precs[row] and its outputs, [P][B][...]
    const int64_t row = blockIdx.y;
    const int precoder = a.precs[row];
    double* const p_ant = a.p_ant ? a.p_ant + row * a.B * M : nullptr;
    double* const l21_out = a.l21 ? a.l21 + row * a.B : nullptr;
    double* const sinr = a.sinr ? a.sinr + row * a.B * K : nullptr;
    double* const rsum = a.rsum ? a.rsum + row * a.B : nullptr;
    int32_t* const info = a.info ? a.info + row * a.B : nullptr;
    const T2* Hb = reinterpret_cast<const T2*>(a.H) + b * K * M;
    T2* Wb = reinterpret_cast<T2*>(a.W) + (row * a.B + b) * K * M;
    const bool zf = precoder == DMIMO_ZF;
    // antenna (tid / 4 within a tile of 64) and user phase (tid % 4) in step 4;
    // entry (tid / 4 = 8 i + j) and antenna phase (tid % 4) in steps 2 and 5
    const int cc = tid >> 2, rg = tid & 3;
    const int ei = cc >> 3, ej = cc & 7;

    // 1.
    double f = 0.0;
    if (a.user_xyz) {
        // the users' channels of this deployment, synthesised here
        const double* ub = a.user_xyz + b * K * 3;
        const double* apb = a.ap_xyz + b * M * 3;
        T2* Ho = reinterpret_cast<T2*>(a.H_out) + b * K * M;
        for (int e = tid; e < K * M; e += kThreads) {
            const int k = e / M, c = e - k * M;
            const T2 v = synth_term<T2>(a, ub[3 * k + 0] - apb[3 * c + 0], ub[3 * k + 1] - apb[3 * c + 1],
                                        ub[3 * k + 2] - apb[3 * c + 2]);
            S.h[k][c] = v;
            if (row == 0) Ho[e] = v;
            f += (double)v.x * v.x + (double)v.y * v.y;
        }
    } else {
        for (int e = tid; e < K * M; e += kThreads) {
            const int k = e / M, c = e - k * M;
            const T2 v = Hb[e];
            S.h[k][c] = v;
            f += (double)v.x * v.x + (double)v.y * v.y;
        }
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
            if (p_ant)
                for (int m = tid; m < M; m += kThreads) p_ant[b * M + m] = 0.0;
            if (sinr && tid < K) sinr[b * K + tid] = 0.0;
            if (tid == 0) {
                if (l21_out) l21_out[b] = 0.0;
                if (rsum) rsum[b] = 0.0;
                if (info) info[b] = S.fail;
            }
            return;
        }
    } else if (precoder == DMIMO_MR) {
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
                if (precoder == DMIMO_MR) {
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
            if (p_ant) p_ant[b * M + c] = pm;
            l21 += sqrt(pm);
        }
    }
    l21 = wave_sum(l21);
    if (lane == 0) S.red2[wv] = l21;
    __syncthreads();

    // 5.
    const bool want_gain = sinr || rsum;
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
        if (sinr) sinr[b * K + lane] = snr;
        rate = log2(1.0 + snr);
    }
    rate = wave_sum(rate);
    if (lane == 0) {
        if (rsum) rsum[b] = rate;
        if (l21_out) l21_out[b] = S.red2[0] + S.red2[1] + S.red2[2] + S.red2[3];
        if (info) info[b] = 0;
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

size_t ws_align(size_t n) { return (n + 255) & ~(size_t)255; }

bool wide_shape(int64_t B, int64_t M) {
    return B <= kWideMaxB && (M + kCols - 1) / kCols >= kWideMinTiles;
}

// Byte offsets of the wide path's workspace (layout above bfw_norm_kernel);
// MR and equal-gain MR share one layout.
struct WideLayout {
    size_t ginv = 0, scale = 0, fail = 0, gpart = 0, lpart = 0, npart = 0, total = 0;
};

WideLayout wide_layout(int precoder, int64_t B, int K, int64_t M, int prec) {
    const int64_t T = (M + kCols - 1) / kCols;
    WideLayout L;
    size_t n = 0;
    if (precoder == DMIMO_ZF) {
        n = ws_align((size_t)B * K * K * (prec == DMIMO_F64 ? 16 : 8));   // Gram slot
        L.ginv = n;
        n += ws_align((size_t)B * K * K * sizeof(double2));
        L.scale = n;
        n += ws_align((size_t)B * K * sizeof(double));
        L.fail = n;
        n += ws_align((size_t)B * sizeof(int32_t));
    }
    L.gpart = n;
    n += ws_align((size_t)B * T * K * K * sizeof(double2));
    L.lpart = n;
    n += ws_align((size_t)B * T * sizeof(double));
    if (precoder != DMIMO_ZF) {
        L.npart = n;
        n += ws_align((size_t)B * T * sizeof(double));
    }
    L.total = n;
    return L;
}

template <typename T2, int KT>
void launch_wide_kt(const BfDev& d, const BfWide& wd, int64_t B, hipStream_t s) {
    const dim3 tiles((unsigned)wd.T, (unsigned)B), one((unsigned)B), block(kThreads);
    if (d.precoder == DMIMO_ZF) {
        bfw_gram_kernel<T2, KT><<<tiles, block, 0, s>>>(d, wd);
        bfw_prep_kernel<KT><<<one, block, 0, s>>>(d, wd);
    } else if (d.precoder == DMIMO_MR && d.p_total > 0.0) {
        bfw_norm_kernel<T2, KT><<<tiles, block, 0, s>>>(d, wd);
    }
    bfw_tile_kernel<T2, KT><<<tiles, block, 0, s>>>(d, wd);
    bfw_final_kernel<KT><<<one, block, 0, s>>>(d, wd);
}

template <typename T2>
dmimo_status launch_wide(const BfDev& d, int64_t B, int prec, hipStream_t s) {
    const int K = d.K;
    const WideLayout L = wide_layout(d.precoder == DMIMO_ZF ? DMIMO_ZF : DMIMO_MR, B, K, d.M, prec);
    char* p = static_cast<char*>(const_cast<void*>(d.G));
    BfWide wd;
    wd.T = (d.M + kCols - 1) / kCols;
    wd.ginv = d.precoder == DMIMO_ZF ? reinterpret_cast<double2*>(p + L.ginv) : nullptr;
    wd.scale = d.precoder == DMIMO_ZF ? reinterpret_cast<double*>(p + L.scale) : nullptr;
    wd.fail = d.precoder == DMIMO_ZF ? reinterpret_cast<int32_t*>(p + L.fail) : nullptr;
    wd.gpart = reinterpret_cast<double2*>(p + L.gpart);
    wd.lpart = reinterpret_cast<double*>(p + L.lpart);
    wd.npart = d.precoder == DMIMO_ZF ? nullptr : reinterpret_cast<double*>(p + L.npart);
    if (K <= 8) launch_wide_kt<T2, 8>(d, wd, B, s);
    else if (K <= 16) launch_wide_kt<T2, 16>(d, wd, B, s);
    else launch_wide_kt<T2, 32>(d, wd, B, s);
    return check_launch("beamform (wide path)");
}

// The one-pass kernel's antenna limit: LDS holds H and W, 8 x (MT + 1) each.
int64_t small_max_m(int prec) { return prec == DMIMO_F64 ? kSmallMaxM / 2 : kSmallMaxM; }

// Shapes past the one-pass kernel that the batched kernel takes from H (MR or
// ZF, 8 < K <= 16, M <= 256, FP32 or MIX): one persistent launch, the Gram on
// the matrix cores and G^-1 in FP64, no workspace (launch_beamform_batched_h,
// batched.hip).
bool batched_h_shape(int precoder, int K, int64_t M, int prec) {
    return (precoder == DMIMO_ZF || precoder == DMIMO_MR) && prec != DMIMO_F64 && K > kSmallK &&
           K <= 16 && M <= 256;
}

template <typename T2, int MT_WIDE>
dmimo_status launch_small(const BfDev& d, int64_t B, int P, hipStream_t s) {
    dim3 grid((unsigned)B, (unsigned)P), block(kThreads);
    if (d.M <= 64) beamform_small_kernel<T2, 64><<<grid, block, 0, s>>>(d);
    else beamform_small_kernel<T2, MT_WIDE><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_small_kernel");
}

}  // namespace

// batched.hip: dmimo_beamform_batched's kernel with the channel given (a.H,
// [B][K][M] complex64), K <= 16, M <= 256, FP32 or MIX; no workspace.
dmimo_status launch_beamform_batched_h(const BeamformArgs& a, hipStream_t s);

size_t beamform_workspace_bytes(int precoder, int64_t B, int K, int64_t M, int prec) {
    const int layout = precoder == DMIMO_ZF ? DMIMO_ZF : DMIMO_MR;
    if (batched_h_shape(precoder, K, M, prec)) return 0;
    if (!wide_shape(B, M) || (K <= kSmallK && M <= small_max_m(prec)))
        return layout == DMIMO_ZF ? ws_align((size_t)B * K * K * (prec == DMIMO_F64 ? 16 : 8)) : 0;
    return wide_layout(layout, B, K, M, prec).total;
}

dmimo_status launch_beamform(const BeamformArgs& a, hipStream_t s) {
    if (a.B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "beamform: B too large");
    BfDev d;
    d.precoder = a.precoder;
    for (int i = 0; i < kMultiMax; ++i) d.precs[i] = a.precoder;
    d.B = a.B;
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
    d.user_xyz = nullptr;
    d.ap_xyz = nullptr;
    d.inv_lam = d.amp_c = d.inv_dmin = 0.0;
    d.H_out = nullptr;
    if (a.K <= kSmallK && a.M <= small_max_m(a.prec)) {
        // G is formed in FP64 in the kernel, so the FP64 Gram's tolerance
        // applies to FP64 input and the FP32 one to every other mode
        d.pivot_tol = a.prec == DMIMO_F64 ? 1e-12 : 1e-6;
        if (a.prec == DMIMO_F64) return launch_small<double2, kSmallMaxM / 2>(d, a.B, 1, s);
        return launch_small<float2, kSmallMaxM>(d, a.B, 1, s);
    }
    if (batched_h_shape(a.precoder, a.K, a.M, a.prec)) return launch_beamform_batched_h(a, s);
    if (wide_shape(a.B, a.M)) {
        // ZF: G from FP64 tile sums, so the FP64 Gram's tolerance for FP64
        // input and the FP32 one otherwise
        d.pivot_tol = a.prec == DMIMO_F64 ? 1e-12 : 1e-6;
        if (a.prec == DMIMO_F64) return launch_wide<double2>(d, a.B, a.prec, s);
        return launch_wide<float2>(d, a.B, a.prec, s);
    }
    if (a.precoder == DMIMO_ZF) {
        dmimo_status st = launch_gram(a.B, a.K, a.M, a.H, a.prec, a.ws, s);
        if (st) return st;
    }
    if (a.prec == DMIMO_F64) return launch_typed<double2>(d, a.B, s);
    return launch_typed<float2>(d, a.B, s);
}

size_t beamform_multi_workspace_bytes(int P, const int* precoders, int64_t B, int K, int64_t M,
                                      int prec) {
    size_t n = 0;
    for (int i = 0; i < P; ++i) n += ws_align(beamform_workspace_bytes(precoders[i], B, K, M, prec));
    return n;
}

namespace {

dmimo_status multi_impl(const BeamformArgs& a, int P, const int* precoders, const WaveConst* w,
                        const double* ap_xyz, const double* user_xyz, hipStream_t s) {
    if (P < 1 || P > kMultiMax) return fail(DMIMO_E_SHAPE, "beamform: 1 <= P <= 8 precoders");
    if (a.B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "beamform: B too large");
    const bool synth = user_xyz != nullptr;
    if (a.K <= kSmallK && a.M <= small_max_m(a.prec)) {
        // every precoder on the one-pass kernel: precoder p on grid row p
        BfDev d;
        d.precoder = precoders[0];
        for (int i = 0; i < kMultiMax; ++i) d.precs[i] = precoders[i < P ? i : 0];
        d.B = a.B;
        d.K = a.K;
        d.M = a.M;
        d.H = a.H;
        for (int k = 0; k < DMIMO_K_MAX; ++k) d.gamma[k] = a.gamma[k];
        d.sigma2 = a.sigma2;
        d.p_total = a.p_total;
        d.pivot_tol = a.prec == DMIMO_F64 ? 1e-12 : 1e-6;
        d.W = a.W;
        d.p_ant = a.p_ant;
        d.l21 = a.l21;
        d.sinr = a.sinr;
        d.rsum = a.rsum;
        d.info = a.info;
        d.G = a.ws;
        d.user_xyz = user_xyz;
        d.ap_xyz = ap_xyz;
        d.inv_lam = synth ? w->inv_lam : 0.0;
        d.amp_c = synth ? w->amp_c : 0.0;
        d.inv_dmin = synth ? w->inv_dmin : 0.0;
        d.H_out = synth ? const_cast<void*>(a.H) : nullptr;
        if (a.prec == DMIMO_F64) return launch_small<double2, kSmallMaxM / 2>(d, a.B, P, s);
        return launch_small<float2, kSmallMaxM>(d, a.B, P, s);
    }
    if (synth) {
        // the channel kernel first, then the precoders from H
        PointsDev up;
        up.kind = DMIMO_PTS_LIST;
        up.nx = up.ny = 0;
        up.x0 = up.y0 = up.dx = up.dy = up.z = 0.0;
        up.xyz = user_xyz;
        up.n = a.K;
        const dmimo_status st = launch_channel(*w, up, false, a.B, a.M, ap_xyz, nullptr,
                                               a.prec == DMIMO_F64, const_cast<void*>(a.H), s);
        if (st) return st;
    }
    // otherwise one call per precoder, in order, each with its workspace slice
    const size_t esz = a.prec == DMIMO_F64 ? 16 : 8;
    char* ws = static_cast<char*>(a.ws);
    for (int i = 0; i < P; ++i) {
        BeamformArgs one = a;
        one.precoder = precoders[i];
        const int64_t r = i;
        one.W = static_cast<char*>(a.W) + r * a.B * a.K * a.M * esz;
        one.p_ant = a.p_ant ? a.p_ant + r * a.B * a.M : nullptr;
        one.l21 = a.l21 ? a.l21 + r * a.B : nullptr;
        one.sinr = a.sinr ? a.sinr + r * a.B * a.K : nullptr;
        one.rsum = a.rsum ? a.rsum + r * a.B : nullptr;
        one.info = a.info ? a.info + r * a.B : nullptr;
        one.ws = ws;
        const dmimo_status st = launch_beamform(one, s);
        if (st) return st;
        ws += ws_align(beamform_workspace_bytes(precoders[i], a.B, a.K, a.M, a.prec));
    }
    return DMIMO_OK;
}

}  // namespace

dmimo_status launch_beamform_multi(const BeamformArgs& a, int P, const int* precoders,
                                   hipStream_t s) {
    return multi_impl(a, P, precoders, nullptr, nullptr, nullptr, s);
}

dmimo_status launch_beamform_users(const BeamformArgs& a, int P, const int* precoders,
                                   const WaveConst& w, const double* ap_xyz, const double* user_xyz,
                                   hipStream_t s) {
    return multi_impl(a, P, precoders, &w, ap_xyz, user_xyz, s);
}

}  // namespace dmimo
