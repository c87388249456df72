// Proximal gradient descent on the PA-consumption Lagrangian (Sec. IV, eq.
// proxgd) and its deep-unfolded form (Sec. V, eq. unfoldednet), batched over
// channels.
//
// Layer i, with sigma = sqrt(sigma2) and d_k = sigma sqrt(gamma_k):
//   A = W H^T                                  (K x K)
//   V = W - eta_i (A - D) H^*                  (the complex gradient step)
//   w_m = (1 - lambda_i eta_i / max(||v_m||, lambda_i eta_i)) v_m    (every antenna m)
// Work per layer: 2 K^2 M complex MACs = 16 K^2 M real flops.
//
// K <= 8 (pgd_mfma_kernel): both products run on v_mfma_f32_16x16x4_f32 in
// the real embedding of the complex matrices, which fills the 16 x 16 tile
// exactly for K = 8 and wastes nothing:
//   step 1  D1 = [Wr; Wi] [Hr; Hi]^T        16 x 16, summed over the antennas:
//           Ar = D1[a][b] - D1[8+a][8+b],  Ai = D1[a][8+b] + D1[8+a][b];
//   step 2  [Gr; Gi] = [[Ar~, Ai], [Ai, -Ar~]] [Hr; Hi]   with Ar~ = Ar - D,
//           i.e. G = (A - D) H^*, 16 x 16 per block of 16 antennas.
// One wave owns 64 antennas; a channel with M antennas takes ceil(M / 64)
// waves of one workgroup, whose step-1 partial sums meet in LDS (one barrier
// per layer, double-buffered).  H stays in registers in both operand layouts
// for all layers; W lives in registers in the step-2 output layout and goes
// through LDS once per layer to reach the step-1 operand layout.
//
// 8 < K <= 16 (pgd_kernel): FP32 VALU, one 256-thread workgroup per channel,
// H and W in LDS.
#include <cmath>

#include "kernels.h"
#include "pgd_mfma.h"
#include "split16.h"

namespace dmimo {

namespace {

constexpr int kPgdThreads = 256;
constexpr int kPgdMaxM = 256;

struct PgdDev {
    int K;
    int M;
    int layers;
    const float2* H;
    const float2* W0;
    float2* W;
    const double* lambdas;
    const double* etas;
    float d[16];          // sigma sqrt(gamma_k); sqrt(gamma_k) in the normalised mode
    double sigma2;        // noise power of sinr / rsum (1 in the normalised mode)
    double* l21;
    double* rsum;
    // normalised mode (the PA-aware precoder on any deployment): per channel
    // {1/s, 1/L} of Hn = H / s; steps are eta_i / L; W = (sigma / s) Wn on output
    const double* pa;     // [B][2] or NULL
    double sigma;         // sqrt of the deployment's noise power
    double* p_ant;        // [B][M] or NULL: per-antenna power of the output W
    double* sinr;         // [B][K] or NULL
};

// Per-channel factors of the normalised mode.
struct PgdScale {
    float hs;             // H -> Hn
    double es;            // eta_i -> eta_i / L
    double ws;            // Wn -> W
};

__device__ __forceinline__ PgdScale pgd_scale(const PgdDev& a, int64_t b) {
    PgdScale c{1.0f, 1.0, 1.0};
    if (a.pa) {
        c.hs = (float)a.pa[2 * b];
        c.es = a.pa[2 * b + 1];
        c.ws = a.sigma * a.pa[2 * b];
    }
    return c;
}

// Normalisation of the PA-aware precoder, one workgroup of NT threads per
// channel: s^2 = mean |h|^2, G = H H^H in FP64, and the largest eigenvalue of
// G.  H passes through LDS in chunks of 64 antennas; each Gram entry sums its
// antennas in order.  The eigenvalue comes from repeated squaring,
// S <- S^2 / tr(S^2) from S = G / tr G, twelve times (S ~ G^4096 / tr, a
// projector onto the top eigenspace unless the top two eigenvalues agree to
// ~1e-3 relative, when any vector of their span gives a Rayleigh quotient
// within that of lambda_max), then the Rayleigh quotient of G at the
// largest-norm column of S.  Writes {1/s, s^2 / lambda_max(G)} =
// {1/s, 1/lambda_max(Hn Hn^H)}; an all-zero channel gets {0, 0}, which makes
// its output W = 0.
constexpr int kPrepChunk = 64;

template <int KM>
struct PrepShared {
    double Gr[KM][KM + 1], Gi[KM][KM + 1];            // G
    double Sr[KM][KM + 1], Si[KM][KM + 1];            // S
    union {
        struct {
            double r[KM][KM + 1], i[KM][KM + 1];      // S^2
        } t;
        float2 h[KM][kPrepChunk + 1];                 // chunk of H
    } u;
    double colnorm[KM];
    double red[16];
};

template <int NT>
__device__ __forceinline__ double prep_block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (NT == 64) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    return t;
}

template <int KM, int NT>
__global__ __launch_bounds__(NT) void pa_prepare_kernel(const float2* H, int K, int M, double* pa) {
    constexpr int QE = (KM * KM + NT - 1) / NT;   // Gram entries per thread
    __shared__ PrepShared<KM> S;
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    const float2* Hb = H + b * K * M;
    double p = 0.0;
    double2 acc[QE];
#pragma unroll
    for (int q = 0; q < QE; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int m0 = 0; m0 < M; m0 += kPrepChunk) {
        const int mc = M - m0 < kPrepChunk ? M - m0 : kPrepChunk;
        __syncthreads();
        {   // a thread's loads all issued before its LDS stores
            constexpr int IT = KM * kPrepChunk / NT;
            float2 hv[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + NT * it;
                const int k = e / kPrepChunk, c = e - k * kPrepChunk;
                if (k < K && c < mc) hv[it] = Hb[(int64_t)k * M + m0 + c];
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + NT * it;
                const int k = e / kPrepChunk, c = e - k * kPrepChunk;
                if (k < K && c < mc) {
                    S.u.h[k][c] = hv[it];
                    p += (double)hv[it].x * hv[it].x + (double)hv[it].y * hv[it].y;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QE; ++q) {
            const int e = tid + NT * q;
            if (e < K * K) {
                const int k = e / K, j = e - k * K;
                double gr = acc[q].x, gi = acc[q].y;
                for (int c = 0; c < mc; ++c) {
                    const float2 hk = S.u.h[k][c], hj = S.u.h[j][c];
                    gr += (double)hk.x * hj.x + (double)hk.y * hj.y;
                    gi += (double)hk.y * hj.x - (double)hk.x * hj.y;
                }
                acc[q] = make_double2(gr, gi);
            }
        }
    }
    p = prep_block_sum<NT>(p, S.red);
    // S = G / tr G  (tr G = sum |h|^2 = p)
    const double inv_tr = p > 0.0 ? 1.0 / p : 0.0;
#pragma unroll
    for (int q = 0; q < QE; ++q) {
        const int e = tid + NT * q;
        if (e < K * K) {
            const int k = e / K, j = e - k * K;
            S.Gr[k][j] = acc[q].x;
            S.Gi[k][j] = acc[q].y;
            S.Sr[k][j] = acc[q].x * inv_tr;
            S.Si[k][j] = acc[q].y * inv_tr;
        }
    }
    __syncthreads();
    for (int it = 0; it < 12; ++it) {
        double dpart = 0.0;                        // this thread's share of tr(S^2)
        for (int e = tid; e < K * K; e += NT) {
            const int k = e / K, j = e - k * K;
            double tr = 0.0, ti = 0.0;
            for (int l = 0; l < K; ++l) {
                tr += S.Sr[k][l] * S.Sr[l][j] - S.Si[k][l] * S.Si[l][j];
                ti += S.Sr[k][l] * S.Si[l][j] + S.Si[k][l] * S.Sr[l][j];
            }
            S.u.t.r[k][j] = tr;
            S.u.t.i[k][j] = ti;
            if (k == j) dpart += tr;
        }
        dpart = prep_block_sum<NT>(dpart, S.red);
        const double inv = dpart > 0.0 ? 1.0 / dpart : 0.0;
        __syncthreads();
        for (int e = tid; e < K * K; e += NT) {
            const int k = e / K, j = e - k * K;
            S.Sr[k][j] = S.u.t.r[k][j] * inv;
            S.Si[k][j] = S.u.t.i[k][j] * inv;
        }
        __syncthreads();
    }
    if (tid < K) {
        double c = 0.0;
        for (int k = 0; k < K; ++k) c += S.Sr[k][tid] * S.Sr[k][tid] + S.Si[k][tid] * S.Si[k][tid];
        S.colnorm[tid] = c;
    }
    __syncthreads();
    if (tid >= 64) return;   // K <= 64: the rest runs in wave 0
    int jb = 0;
    for (int j = 1; j < K; ++j)
        if (S.colnorm[j] > S.colnorm[jb]) jb = j;
    // Rayleigh quotient of G at v = S[:, jb]: lane k holds v_k and (G v)_k
    double num = 0.0, den = 0.0;
    if (tid < K) {
        double yr = 0.0, yi = 0.0;
        for (int j = 0; j < K; ++j) {
            yr += S.Gr[tid][j] * S.Sr[j][jb] - S.Gi[tid][j] * S.Si[j][jb];
            yi += S.Gr[tid][j] * S.Si[j][jb] + S.Gi[tid][j] * S.Sr[j][jb];
        }
        num = S.Sr[tid][jb] * yr + S.Si[tid][jb] * yi;
        den = S.Sr[tid][jb] * S.Sr[tid][jb] + S.Si[tid][jb] * S.Si[tid][jb];
    }
    for (int off = 32; off > 0; off >>= 1) {
        num += __shfl_xor(num, off, 64);
        den += __shfl_xor(den, off, 64);
    }
    if (tid == 0) {
        const double lam = den > 0.0 ? num / den : 0.0;
        const double s2 = p / ((double)K * M);
        const bool ok = s2 > 0.0 && lam > 0.0;
        pa[2 * b] = ok ? 1.0 / sqrt(s2) : 0.0;
        pa[2 * b + 1] = ok ? s2 / lam : 0.0;
    }
}

__device__ __forceinline__ void cfmaf(float2& acc, float2 a, float2 b) {   // acc += a b
    acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}
__device__ __forceinline__ void cfmaf_conj(float2& acc, float2 a, float2 b) {   // acc += a conj(b)
    acc.x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x));
    acc.y = fmaf(a.y, b.x, fmaf(-a.x, b.y, acc.y));
}

template <int KT>
__global__ __launch_bounds__(kPgdThreads) void pgd_kernel(PgdDev a) {
    __shared__ float2 sH[KT][kPgdMaxM + 1];
    __shared__ float2 sW[KT][kPgdMaxM + 1];
    __shared__ float2 sA[KT][KT + 1];
    __shared__ double sP[KT][KT + 1];
    __shared__ double red[kPgdThreads / 64];

    const int64_t b = blockIdx.x;
    const int K = a.K, M = a.M;
    const int tid = threadIdx.x;
    const float2* Hb = a.H + b * K * M;
    const PgdScale cs = pgd_scale(a, b);

    for (int e = tid; e < K * M; e += kPgdThreads) {
        const int k = e / M, m = e - k * M;
        const float2 h = make_float2(cs.hs * Hb[e].x, cs.hs * Hb[e].y);
        sH[k][m] = h;
        sW[k][m] = a.W0 ? a.W0[b * K * M + e] : make_float2(h.x, -h.y);   // W(0) = H^*
    }
    __syncthreads();

    // A entries: e = tid / S for S = threads per entry
    constexpr int S = kPgdThreads / (KT * KT) >= 4 ? 4 : kPgdThreads / (KT * KT);
    const int ae = tid / S, as = tid % S;
    const int ak = ae / KT, aj = ae % KT;
    // step / prox: column c = tid / 4 of each pass, rows r, r + 4, ...
    const int cc = tid >> 2, rg = tid & 3;

    for (int layer = 0; layer < a.layers; ++layer) {
        const float eta = (float)(a.etas[layer] * cs.es);
        const float thr = (float)(a.lambdas[layer] * a.etas[layer] * cs.es);
        // A = W H^T
        float2 acc = make_float2(0.f, 0.f);
        if (ae < KT * KT && ak < K && aj < K)
            for (int m = as; m < M; m += S) cfmaf(acc, sW[ak][m], sH[aj][m]);
        if (S >= 2) {
            acc.x += __shfl_xor(acc.x, 1, 64);
            acc.y += __shfl_xor(acc.y, 1, 64);
        }
        if (S >= 4) {
            acc.x += __shfl_xor(acc.x, 2, 64);
            acc.y += __shfl_xor(acc.y, 2, 64);
        }
        if (as == 0 && ae < KT * KT) sA[ak][aj] = acc;
        __syncthreads();
        // V = W - eta (A H^* - D H^*), then the column prox
        for (int m0 = 0; m0 < M; m0 += kPgdThreads / 4) {
            const int m = m0 + cc;
            float2 v[(KT + 3) / 4];
            float n2 = 0.0f;
#pragma unroll
            for (int r = 0; r < (KT + 3) / 4; ++r) {
                const int k = rg + 4 * r;
                v[r] = make_float2(0.f, 0.f);
                if (k < K && m < M) {
                    float2 g = make_float2(0.f, 0.f);
                    for (int j = 0; j < K; ++j) cfmaf_conj(g, sA[k][j], sH[j][m]);
                    const float2 h = sH[k][m];
                    g.x -= a.d[k] * h.x;
                    g.y += a.d[k] * h.y;           // - d_k conj(h)
                    const float2 w = sW[k][m];
                    v[r] = make_float2(fmaf(-eta, g.x, w.x), fmaf(-eta, g.y, w.y));
                    n2 = fmaf(v[r].x, v[r].x, fmaf(v[r].y, v[r].y, n2));
                }
            }
            n2 += __shfl_xor(n2, 1, 64);
            n2 += __shfl_xor(n2, 2, 64);
            const float nrm = sqrtf(n2);
            const float sc = thr > 0.0f ? 1.0f - thr / fmaxf(nrm, thr) : 1.0f;
#pragma unroll
            for (int r = 0; r < (KT + 3) / 4; ++r) {
                const int k = rg + 4 * r;
                if (k < K && m < M) sW[k][m] = make_float2(sc * v[r].x, sc * v[r].y);
            }
        }
        __syncthreads();
    }

    // outputs: W, p_m, ||W||_{2,1}, SINR_k, sum rate (SINR from the normalised
    // gains with unit noise in the normalised mode, which is the same SINR)
    float2* Wb = a.W + b * K * M;
    const float wsf = (float)cs.ws;
    for (int e = tid; e < K * M; e += kPgdThreads) {
        const float2 w = sW[e / M][e % M];
        Wb[e] = make_float2(wsf * w.x, wsf * w.y);
    }
    if (a.l21 || a.p_ant) {
        double s = 0.0;
        for (int m = tid; m < M; m += kPgdThreads) {
            double p = 0.0;
            for (int k = 0; k < K; ++k) p += (double)sW[k][m].x * sW[k][m].x + (double)sW[k][m].y * sW[k][m].y;
            if (a.p_ant) a.p_ant[b * M + m] = cs.ws * cs.ws * p;
            s += sqrt(p);
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0 && a.l21) a.l21[b] = cs.ws * (red[0] + red[1] + red[2] + red[3]);
        __syncthreads();
    }
    if (a.rsum || a.sinr) {
        // gains A = H W^T in FP64, one entry per thread
        double2 g = make_double2(0.0, 0.0);
        const int k = tid / KT, j = tid % KT;
        if (tid < KT * KT && k < K && j < K)
            for (int m = 0; m < M; ++m) {
                const float2 h = sH[k][m], w = sW[j][m];
                g.x += (double)h.x * w.x - (double)h.y * w.y;
                g.y += (double)h.x * w.y + (double)h.y * w.x;
            }
        __syncthreads();
        if (tid < KT * KT && k < K && j < K) sP[k][j] = g.x * g.x + g.y * g.y;
        __syncthreads();
        if (tid == 0) {
            double r = 0.0;
            for (int kk = 0; kk < K; ++kk) {
                double sig = 0.0, intf = 0.0;
                for (int jj = 0; jj < K; ++jj) (jj == kk ? sig : intf) += sP[kk][jj];
                const double sn = sig / (intf + a.sigma2);
                if (a.sinr) a.sinr[b * K + kk] = sn;
                r += log2(1.0 + sn);
            }
            if (a.rsum) a.rsum[b] = r;
        }
    }
}


// Outputs of a PGD workgroup from the planar W in sX (normalised mode:
// scaled back): W, p_m, ||W||_{2,1}, and from the last D1 partials (parity
// ph) the SINR_k and the sum rate.  Every thread of the block calls it after
// a barrier that follows the last partials.
template <int NW>
__device__ __forceinline__ void pgd_outputs(const PgdDev& a, int64_t b, int tid, int lane, int wave,
                                            const float* sX, int stride, float* sD, int ph,
                                            const PgdScale& cs) {
    const int K = a.K, M = a.M;
    const bool gains = a.rsum || a.sinr;
    // outputs from the planar W (scaled back in the normalised mode)
    float2* Wb = a.W + b * K * M;
    const float wsf = (float)cs.ws;
    for (int e = tid; e < K * M; e += blockDim.x) {
        const int k = e / M, m = e - k * M;
        Wb[e] = make_float2(wsf * sX[k * stride + m], wsf * sX[(8 + k) * stride + m]);
    }
    // scratch for the reductions: the partial buffer of the other parity
    double* red = reinterpret_cast<double*>(sD + (ph ^ 1) * NW * kPartFloats);
    if (a.l21 || a.p_ant) {
        double s = 0.0;
        for (int m = tid; m < M; m += blockDim.x) {
            double p = 0.0;
            for (int k = 0; k < K; ++k) {
                const double x = sX[k * stride + m], y = sX[(8 + k) * stride + m];
                p += x * x + y * y;
            }
            if (a.p_ant) a.p_ant[b * M + m] = cs.ws * cs.ws * p;
            s += sqrt(p);
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[64 + wave] = s;
    }
    if (gains && wave == 0) {
        // gains G = H W^T = A^T with A = W H^T from the last MFMA pass:
        // lane 8 k + j holds |G_kj|^2 = |A_jk|^2
        const int k = lane >> 3, j = lane & 7;
        red[lane] = (k < K && j < K) ? (double)gain_sq<NW>(sD + ph * NW * kPartFloats, j, k) : 0.0;
    }
    __syncthreads();
    if (tid == 0 && a.l21) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += red[64 + w];
        a.l21[b] = cs.ws * t;
    }
    if (gains && wave == 0) {
        // user k = lane < K: SINR_k and log2(1 + SINR_k), then a sum over the 8 lanes
        double r = 0.0;
        if (lane < K) {
            double sig = 0.0, intf = 0.0;
            for (int jj = 0; jj < K; ++jj) (jj == lane ? sig : intf) += red[lane * 8 + jj];
            const double sn = sig / (intf + a.sigma2);
            if (a.sinr) a.sinr[b * K + lane] = sn;
            r = log2(1.0 + sn);
        }
        for (int off = 4; off > 0; off >>= 1) r += __shfl_xor(r, off, 64);
        if (lane == 0 && a.rsum) a.rsum[b] = r;
    }
}

template <int AW, int NW>
__global__ __launch_bounds__(64 * NW) void pgd_mfma_kernel(PgdDev a) {
    constexpr int NQ = AW / 16;                // 16-antenna blocks per wave
    extern __shared__ float smem[];
    const int stride = pl_stride(AW * NW);
    float* sX = smem;                          // [16][stride]   H, then W
    float* sD = smem + 16 * stride;            // [2][NW][16][17] D1 partials

    const PgdLane<AW> L;
    const int64_t b = blockIdx.x;
    const int K = a.K, M = a.M;
    const float2* Hb = a.H + b * K * M;
    const PgdScale cs = pgd_scale(a, b);

    load_planar<AW / 8>(sX, stride, AW * NW, Hb, K, M, false, cs.hs);
    __syncthreads();
    float HA[AW / 4], HB[NQ][4];
    read_op_a(sX, stride, L, HA);
    read_op_b2(sX, stride, L, HB);
    __syncthreads();
    if (a.W0) load_planar<AW / 8>(sX, stride, AW * NW, a.W0 + b * K * M, K, M, false, 1.0f);
    else load_planar<AW / 8>(sX, stride, AW * NW, Hb, K, M, true, cs.hs);         // W(0) = H^*
    __syncthreads();
    float WD[NQ][4], WA[AW / 4];
    read_out_d(sX, stride, L, WD);
    read_op_a(sX, stride, L, WA);
    const float dg = a.d[L.lo & 7];

    int ph = 0;
    for (int layer = 0; layer < a.layers; ++layer) {
        const float eta = (float)(a.etas[layer] * cs.es);
        const float thr = (float)(a.lambdas[layer] * a.etas[layer] * cs.es);
        put_partial(sD + (ph * NW + L.wave) * kPartFloats, L, d1_partial<AW>(WA, HA));
        __syncthreads();
        float E[4];                            // (A - D), embedded
        embed_operand<NW>(sD + ph * NW * kPartFloats, L, dg, E);
        ph ^= 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const f32x4 g = apply_block(E, HB, q);
            float v[4];
            float n2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = fmaf(-eta, g[r], WD[q][r]);
                n2 = fmaf(v[r], v[r], n2);
            }
            const float sc = prox_scale(col_norm(column_sum(n2)), thr);
#pragma unroll
            for (int r = 0; r < 4; ++r) WD[q][r] = sc * v[r];
        }
        write_out_d(sX, stride, L, WD);
        wave_lds_sync();
        read_op_a(sX, stride, L, WA);
    }
    const bool gains = a.rsum || a.sinr;
    if (gains) put_partial(sD + (ph * NW + L.wave) * kPartFloats, L, d1_partial<AW>(WA, HA));
    __syncthreads();
    pgd_outputs<NW>(a, b, L.tid, L.lane, L.wave, sX, stride, sD, ph, cs);
}

// ---------------------------------------------------------------------------
// BF16x3: the same layer with both products on the BF16 matrix cores, each
// FP32 operand split as hi + lo (BF16) and the three products hi*hi + lo*hi +
// hi*lo accumulated in FP32 (relative error near 2^-17 per product).  Unlike
// the FP32 MFMA, the BF16 MFMA overlaps the VALU work of the other waves.
//   step 1  v_mfma_f32_16x16x32_bf16: 32 antennas per product; lane (hi, lo)
//           holds row lo at antennas c0 + 32 t + 8 hi + j (t < 2, j < 8);
//   step 2  v_mfma_f32_16x16x16_bf16: lane (hi, lo) holds E[lo][4 hi + j]
//           and H16[4 hi + j][c0 + 16 q + lo] (j < 4).
// 64 antennas per wave.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void read_op_a32(const float* sX, int stride, const PgdLane<64>& L,
                                            float (&XA)[16]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        // 32-byte aligned: stride and c0 + 32 t + 8 hi are multiples of 4 floats
        const float4* src = reinterpret_cast<const float4*>(sX + L.lo * stride + L.c0 + 32 * t + 8 * L.hi);
        const float4 u = src[0], v = src[1];
        XA[8 * t + 0] = u.x; XA[8 * t + 1] = u.y; XA[8 * t + 2] = u.z; XA[8 * t + 3] = u.w;
        XA[8 * t + 4] = v.x; XA[8 * t + 5] = v.y; XA[8 * t + 6] = v.z; XA[8 * t + 7] = v.w;
    }
}

__device__ __forceinline__ void split_x8(const float* x, u32x4& hi, u32x4& lo) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float r0, r1;
        hi[i] = pack_hi<true>(x[2 * i], x[2 * i + 1], r0, r1);
        lo[i] = pack_lo<true>(r0, r1);
    }
}

__device__ __forceinline__ void split_x4(const float* x, u32x2& hi, u32x2& lo) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        float r0, r1;
        hi[i] = pack_hi<true>(x[2 * i], x[2 * i + 1], r0, r1);
        lo[i] = pack_lo<true>(r0, r1);
    }
}

// This wave's share of D1 = X16 H16^T over its 64 antennas, x3.
__device__ __forceinline__ f32x4 d1_partial_x3(const float (&XA)[16], const u32x4 (&Hh)[2],
                                               const u32x4 (&Hl)[2]) {
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        u32x4 xh, xl;
        split_x8(XA + 8 * t, xh, xl);
        d = mfma16<true>(xh, Hh[t], d);
        d = mfma16<true>(xl, Hh[t], d);
        d = mfma16<true>(xh, Hl[t], d);
    }
    return d;
}

// Entry E[i][l] of [[Br, Bi], [Bi, -Br]], B = (X H^T) - diag(dg), from the NW
// partials of D1 (summed in wave order).
template <int NW>
__device__ __forceinline__ float embed_entry(const float* parts, int i, int l, float dg) {
    const int ia = i & 7, lb = l & 7;
    const bool itop = i < 8;
    const bool same = itop == (l < 8);
    const int a1 = ia * 17 + (same ? lb : 8 + lb);
    const int a2 = (8 + ia) * 17 + (same ? 8 + lb : lb);
    float x = 0.0f, y = 0.0f;
#pragma unroll
    for (int p = 0; p < NW; ++p) {
        x += parts[p * kPartFloats + a1];
        y += parts[p * kPartFloats + a2];
    }
    float v = same ? x - y : x + y;
    if (same && ia == lb) v -= dg;
    return (same && !itop) ? -v : v;
}

template <int NW>
__global__ __launch_bounds__(64 * NW) void pgd_x3_kernel(PgdDev a) {
    extern __shared__ float smem[];
    const int stride = pl_stride(64 * NW);
    float* sX = smem;                          // [16][stride]   H, then W
    float* sD = smem + 16 * stride;            // [2][NW][16][17] D1 partials

    const PgdLane<64> L;
    const int64_t b = blockIdx.x;
    const int K = a.K, M = a.M;
    const float2* Hb = a.H + b * K * M;
    const PgdScale cs = pgd_scale(a, b);

    load_planar<8>(sX, stride, 64 * NW, Hb, K, M, false, cs.hs);
    __syncthreads();
    u32x4 HAh[2], HAl[2];
    {
        float h[16];
        read_op_a32(sX, stride, L, h);
        split_x8(h, HAh[0], HAl[0]);
        split_x8(h + 8, HAh[1], HAl[1]);
    }
    u32x2 HBh[4], HBl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = sX[(4 * L.hi + j) * stride + L.c0 + 16 * q + L.lo];
        split_x4(h, HBh[q], HBl[q]);
    }
    __syncthreads();
    if (a.W0) load_planar<8>(sX, stride, 64 * NW, a.W0 + b * K * M, K, M, false, 1.0f);
    else load_planar<8>(sX, stride, 64 * NW, Hb, K, M, true, cs.hs);         // W(0) = H^*
    __syncthreads();
    float WD[4][4], WA[16];
    read_out_d<64>(sX, stride, L, WD);
    read_op_a32(sX, stride, L, WA);
    const float dg = a.d[L.lo & 7];

    int ph = 0;
    for (int layer = 0; layer < a.layers; ++layer) {
        const float eta = (float)(a.etas[layer] * cs.es);
        const float thr = (float)(a.lambdas[layer] * a.etas[layer] * cs.es);
        put_partial(sD + (ph * NW + L.wave) * kPartFloats, L, d1_partial_x3(WA, HAh, HAl));
        __syncthreads();
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) e[j] = embed_entry<NW>(sD + ph * NW * kPartFloats, L.lo, 4 * L.hi + j, dg);
        ph ^= 1;
        u32x2 Eh, El;
        split_x4(e, Eh, El);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f32x4 g = {0.f, 0.f, 0.f, 0.f};
            g = mfma16k16_bf16(Eh, HBh[q], g);
            g = mfma16k16_bf16(El, HBh[q], g);
            g = mfma16k16_bf16(Eh, HBl[q], g);
            float v[4];
            float n2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = fmaf(-eta, g[r], WD[q][r]);
                n2 = fmaf(v[r], v[r], n2);
            }
            const float sc = prox_scale(col_norm(column_sum(n2)), thr);
#pragma unroll
            for (int r = 0; r < 4; ++r) WD[q][r] = sc * v[r];
        }
        write_out_d(sX, stride, L, WD);
        wave_lds_sync();
        read_op_a32(sX, stride, L, WA);
    }
    const bool gains = a.rsum || a.sinr;
    if (gains) put_partial(sD + (ph * NW + L.wave) * kPartFloats, L, d1_partial_x3(WA, HAh, HAl));
    __syncthreads();
    pgd_outputs<NW>(a, b, L.tid, L.lane, L.wave, sX, stride, sD, ph, cs);
}

}  // namespace

namespace {

PgdDev make_pgd_dev(int K, int M, const void* H, const double* gamma, double sigma2, int layers,
                    const double* lambdas, const double* etas, const void* W0, void* W, double* l21,
                    double* rsum) {
    PgdDev d;
    d.K = K;
    d.M = M;
    d.layers = layers;
    d.H = reinterpret_cast<const float2*>(H);
    d.W0 = reinterpret_cast<const float2*>(W0);
    d.W = reinterpret_cast<float2*>(W);
    d.lambdas = lambdas;
    d.etas = etas;
    const double sigma = std::sqrt(sigma2);
    for (int k = 0; k < 16; ++k) d.d[k] = k < K ? (float)(sigma * std::sqrt(gamma ? gamma[k] : 1.0)) : 0.0f;
    d.sigma2 = sigma2;
    d.l21 = l21;
    d.rsum = rsum;
    d.pa = nullptr;
    d.sigma = sigma;
    d.p_ant = nullptr;
    d.sinr = nullptr;
    return d;
}

template <int AW>
void launch_mfma(const PgdDev& d, dim3 grid, int nw, hipStream_t s) {
    const size_t lds = pgd_mfma_lds_bytes(AW, nw);
    switch (nw) {
        case 1: pgd_mfma_kernel<AW, 1><<<grid, dim3(64), lds, s>>>(d); break;
        case 2: pgd_mfma_kernel<AW, 2><<<grid, dim3(128), lds, s>>>(d); break;
        case 3: pgd_mfma_kernel<AW, 3><<<grid, dim3(192), lds, s>>>(d); break;
        default: pgd_mfma_kernel<AW, 4><<<grid, dim3(256), lds, s>>>(d); break;
    }
}

dmimo_status run_pgd(const PgdDev& d, int64_t B, int prec, hipStream_t s) {
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "pgd: B too large");
    const dim3 grid((unsigned)B);
    if (prec == DMIMO_MIX_BF16X3) {            // K <= 8 (validated by the caller)
        const int nw = (d.M + 63) / 64;
        const size_t lds = pgd_mfma_lds_bytes(64, nw);
        switch (nw) {
            case 1: pgd_x3_kernel<1><<<grid, dim3(64), lds, s>>>(d); break;
            case 2: pgd_x3_kernel<2><<<grid, dim3(128), lds, s>>>(d); break;
            case 3: pgd_x3_kernel<3><<<grid, dim3(192), lds, s>>>(d); break;
            default: pgd_x3_kernel<4><<<grid, dim3(256), lds, s>>>(d); break;
        }
        return check_launch("pgd_x3_kernel");
    }
    if (d.K <= 8) {
        const int aw = pgd_antennas_per_wave(B, d.M);
        const int nw = (d.M + aw - 1) / aw;
        if (aw == 16) launch_mfma<16>(d, grid, nw, s);
        else if (aw == 32) launch_mfma<32>(d, grid, nw, s);
        else launch_mfma<64>(d, grid, nw, s);
        return check_launch("pgd_mfma_kernel");
    }
    pgd_kernel<16><<<grid, dim3(kPgdThreads), 0, s>>>(d);
    return check_launch("pgd_kernel");
}

}  // namespace

dmimo_status launch_pgd(int64_t B, int K, int M, const void* H, const double* gamma, double sigma2,
                        int layers, const double* lambdas, const double* etas, const void* W0,
                        void* W, double* l21, double* rsum, int prec, hipStream_t s) {
    const PgdDev d = make_pgd_dev(K, M, H, gamma, sigma2, layers, lambdas, etas, W0, W, l21, rsum);
    return run_pgd(d, B, prec, s);
}

dmimo_status launch_pa_precoder(int64_t B, int K, int M, const void* H, const double* gamma,
                                double sigma2, int layers, const double* lambdas,
                                const double* eta_rel, void* W, double* p_ant, double* l21,
                                double* sinr, double* rsum, void* ws, int prec, hipStream_t s) {
    // the normalised problem has unit noise: d_k = sqrt(gamma_k), SINR with noise 1
    PgdDev d = make_pgd_dev(K, M, H, gamma, 1.0, layers, lambdas, eta_rel, nullptr, W, l21, rsum);
    d.pa = static_cast<const double*>(ws);
    d.sigma = std::sqrt(sigma2);
    d.p_ant = p_ant;
    d.sinr = sinr;
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "pa_precoder: B too large");
    dmimo_status st = launch_pa_prepare(B, K, M, H, static_cast<double*>(ws), s);
    if (st) return st;
    return run_pgd(d, B, prec, s);
}

dmimo_status launch_pa_prepare(int64_t B, int K, int M, const void* H, double* pa, hipStream_t s) {
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "pa_precoder: B too large");
    const float2* h = reinterpret_cast<const float2*>(H);
    if (K <= 16) pa_prepare_kernel<16, 64><<<dim3((unsigned)B), dim3(64), 0, s>>>(h, K, M, pa);
    else pa_prepare_kernel<32, 256><<<dim3((unsigned)B), dim3(256), 0, s>>>(h, K, M, pa);
    return check_launch("pa_prepare_kernel");
}

}  // namespace dmimo
