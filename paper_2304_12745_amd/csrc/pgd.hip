// Proximal gradient descent on the PA-consumption Lagrangian (Sec. IV, eq.
// proxgd) and its deep-unfolded form (Sec. V, eq. unfoldednet), batched over
// channels: one workgroup per channel, H and W resident in LDS for all layers.
//
// Layer i, with sigma = sqrt(sigma2) and d_k = sigma sqrt(gamma_k):
//   A = W H^T                                  (K x K)
//   V = W - eta_i (A H^* - D H^*)             (the complex gradient step)
//   w_m = (1 - lambda_i eta_i / max(||v_m||, lambda_i eta_i)) v_m    (every antenna m)
// Work per layer: 2 K^2 M complex MACs.  A takes four threads per entry
// (each every fourth antenna, combined by two lane shuffles).  The step and
// the prox take four adjacent threads per antenna column (rows k = r, r+4,
// ...), whose shuffles give the column norm.  FP32 arithmetic; lambda_i and
// eta_i come from device arrays (uniform scalar loads).
#include <cmath>

#include "kernels.h"

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
    float d[16];          // sigma sqrt(gamma_k)
    double sigma2;
    double* l21;
    double* rsum;
};

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

    for (int e = tid; e < K * M; e += kPgdThreads) {
        const int k = e / M, m = e - k * M;
        const float2 h = Hb[e];
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
        const float eta = (float)a.etas[layer];
        const float thr = (float)(a.lambdas[layer] * a.etas[layer]);
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

    // outputs: W, ||W||_{2,1}, sum rate
    float2* Wb = a.W + b * K * M;
    for (int e = tid; e < K * M; e += kPgdThreads) Wb[e] = sW[e / M][e % M];
    if (a.l21) {
        double s = 0.0;
        for (int m = tid; m < M; m += kPgdThreads) {
            double p = 0.0;
            for (int k = 0; k < K; ++k) p += (double)sW[k][m].x * sW[k][m].x + (double)sW[k][m].y * sW[k][m].y;
            s += sqrt(p);
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) a.l21[b] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
    if (a.rsum) {
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
                r += log2(1.0 + sig / (intf + a.sigma2));
            }
            a.rsum[b] = r;
        }
    }
}

}  // namespace

dmimo_status launch_pgd(int64_t B, int K, int M, const void* H, const double* gamma, double sigma2,
                        int layers, const double* lambdas, const double* etas, const void* W0,
                        void* W, double* l21, double* rsum, hipStream_t s) {
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
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "pgd: B too large");
    dim3 grid((unsigned)B), block(kPgdThreads);
    if (K <= 8) pgd_kernel<8><<<grid, block, 0, s>>>(d);
    else pgd_kernel<16><<<grid, block, 0, s>>>(d);
    return check_launch("pgd_kernel");
}

}  // namespace dmimo
