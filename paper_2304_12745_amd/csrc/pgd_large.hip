// The PA-aware precoder for deployments too large for one workgroup: up to
// 32 users and 4096 antennas (e.g. a 32 x 32 ceiling grid serving 32 users).
// Same problem and normalisation as the one-workgroup path (eq. optim1 by the
// PGD layers of Sec. IV on Hn = H / s with unit noise, W = (sigma / s) Wn).
//
// Real embedding with 64 rows: X64 = [Xr; Xi] (rows 0..31 real parts, 32..63
// imaginary parts, zero beyond K), H64 likewise.  Per layer, with A = W H^T:
//   D1 = X64 H64^T (64 x 64):  Ar = D1[a][b] - D1[32+a][32+b],
//                              Ai = D1[a][32+b] + D1[32+a][b];
//   E  = [[Ar - D, Ai], [Ai, -(Ar - D)]];   E H64 = [Re((A - D) H^*); Im(...)].
// The antennas are cut into slabs of 64; one four-wave workgroup owns a slab
// of one deployment, wave w the 16-row tile w of both products.  Each layer
// is two launches:
//   lg_reduce_kernel  sums the slabs' D1 partials (fixed slab order) into E,
//                     one entry per thread;
//   lg_layer_kernel   per slab: G = E H64 (64 MFMA 16x16x4 per wave),
//                     V = W - eta G, the column prox (column norms combined
//                     across the waves in LDS), W back to memory, and the
//                     slab's D1 partial of the new W (64 MFMA per wave) for
//                     the next layer.
// lg_init_kernel writes W(0) = Hn^* and its partials; lg_final_kernel maps W
// back and forms p_m, ||W||_{2,1}, SINR_k and the sum rate.
#include <cmath>

#include "kernels.h"
#include "pgd_mfma.h"

namespace dmimo {

namespace {

constexpr int kLgMaxK = 32;
constexpr int kLgMaxM = 4096;
constexpr int kLgSlab = 64;
constexpr int kLgRows = 64;
constexpr int kLgStride = kLgSlab + 4;     // planar LDS row stride (floats)
constexpr int kLgPart = kLgRows * kLgRows;   // floats of one D1 partial / of E

struct LgDev {
    int K, M, S, layers;
    const float2* H;
    float2* W;
    const double* lambdas;   // [layers]
    const double* eta_rel;   // [layers], steps in units of 1 / L
    const double* pa;        // [B][2] {1/s, 1/L}
    float d[kLgMaxK];        // sqrt(gamma_k) (unit noise)
    double sigma;            // back-mapping W = sigma / s Wn
    float* part;             // [2][B][S][64][64]
    float* E;                // [B][64][64]
    double* p_ant;           // [B][M] or NULL
    double* l21;             // [B] or NULL
    double* sinr;            // [B][K] or NULL
    double* rsum;            // [B] or NULL
    int64_t B;
};

__device__ __forceinline__ float* part_ptr(const LgDev& a, int parity, int64_t b, int slab) {
    return a.part + (((int64_t)parity * a.B + b) * a.S + slab) * kLgPart;
}

// Planar image of rows of X (K x M complex64) at the slab's antennas, scaled
// and optionally conjugated: sX[R][c], R < 32 real parts, R >= 32 imaginary.
// 256 threads; the loop is unrolled so that all of a thread's loads are in
// flight together.
constexpr int kLgThreads = 256;
__device__ __forceinline__ void lg_load_slab(float* sX, const float2* X, int K, int M, int c0,
                                             float scale, bool conj) {
    float2 x[kLgMaxK * kLgSlab / kLgThreads];
#pragma unroll
    for (int it = 0; it < kLgMaxK * kLgSlab / kLgThreads; ++it) {
        const int e = threadIdx.x + kLgThreads * it;
        const int k = e / kLgSlab, c = e - k * kLgSlab;
        x[it] = (k < K && c0 + c < M) ? X[(int64_t)k * M + c0 + c] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < kLgMaxK * kLgSlab / kLgThreads; ++it) {
        const int e = threadIdx.x + kLgThreads * it;
        const int k = e / kLgSlab, c = e - k * kLgSlab;
        sX[k * kLgStride + c] = scale * x[it].x;
        sX[(kLgMaxK + k) * kLgStride + c] = conj ? -(scale * x[it].y) : scale * x[it].y;
    }
}

// Row tile r of the slab's D1 partial: X64 (planar sX) times H64^T (planar
// sH); lane (hi, lo) ends with D1[16 r + 4 hi + v][16 r' + lo] in acc[r'][v].
__device__ __forceinline__ void lg_partial(const float* sX, const float* sH, int r, int lo, int hi,
                                           f32x4 (&acc)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int c = 0; c < 16; ++c) {
        const float xa = sX[(16 * r + lo) * kLgStride + 16 * hi + c];
        float ha[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) ha[q] = sH[(16 * q + lo) * kLgStride + 16 * hi + c];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa, ha[q], acc[q], 0, 0, 0);
    }
}

__device__ __forceinline__ void lg_store_partial(float* dst, int r, int lo, int hi, const f32x4 (&acc)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(16 * r + 4 * hi + v) * kLgRows + 16 * q + lo] = acc[q][v];
}

// W(0) = Hn^* and its D1 partials (parity 0).
__global__ __launch_bounds__(256) void lg_init_kernel(LgDev a) {
    __shared__ __attribute__((aligned(16))) float sH[kLgRows * kLgStride];
    __shared__ __attribute__((aligned(16))) float sW[kLgRows * kLgStride];
    const int64_t b = blockIdx.y;
    const int slab = blockIdx.x, c0 = kLgSlab * slab;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lo = lane & 15, hi = lane >> 4;
    const float hs = (float)a.pa[2 * b];
    const float2* Hb = a.H + b * a.K * a.M;
    lg_load_slab(sH, Hb, a.K, a.M, c0, hs, false);
    lg_load_slab(sW, Hb, a.K, a.M, c0, hs, true);
    __syncthreads();
    float2* Wb = a.W + b * a.K * a.M;
    for (int e = tid; e < a.K * kLgSlab; e += 256) {
        const int k = e / kLgSlab, c = e - k * kLgSlab;
        if (c0 + c < a.M)
            Wb[(int64_t)k * a.M + c0 + c] = make_float2(sW[k * kLgStride + c], sW[(kLgMaxK + k) * kLgStride + c]);
    }
    f32x4 acc[4];
    lg_partial(sW, sH, wave, lo, hi, acc);
    lg_store_partial(part_ptr(a, 0, b, slab), wave, lo, hi, acc);
}

// E of one deployment from the S partials of parity `par`: one entry per
// thread, workgroup (64 entries, deployment b).
__global__ __launch_bounds__(64) void lg_reduce_kernel(LgDev a, int par) {
    const int64_t b = blockIdx.y;
    const int e = blockIdx.x * 64 + threadIdx.x;           // < 4096
    const int R = e / kLgRows, C = e % kLgRows;
    const float* p0 = part_ptr(a, par, b, 0);
    const int ra = R & 31, cb = C & 31;
    const bool top = R < 32, same = top == (C < 32);
    // Ar[ra][cb] = D1[ra][cb] - D1[32+ra][32+cb];  Ai = D1[ra][32+cb] + D1[32+ra][cb]
    const int i1 = ra * kLgRows + (same ? cb : 32 + cb);
    const int i2 = (32 + ra) * kLgRows + (same ? 32 + cb : cb);
    float x = 0.f, y = 0.f;
#pragma unroll 8
    for (int sl = 0; sl < a.S; ++sl) {   // loads issued together, sums in slab order
        x += p0[(int64_t)sl * kLgPart + i1];
        y += p0[(int64_t)sl * kLgPart + i2];
    }
    float v = same ? x - y : x + y;
    if (same && ra == cb && ra < a.K) v -= a.d[ra];
    a.E[b * kLgPart + e] = (same && !top) ? -v : v;
}

// One layer on one slab, then the slab's D1 partial of the new W (parity
// `par ^ 1`).  Wave w: rows 16 w .. 16 w + 15 of G, V, W and of the partial.
__global__ __launch_bounds__(256) void lg_layer_kernel(LgDev a, int layer, int par) {
    __shared__ __attribute__((aligned(16))) float sH[kLgRows * kLgStride];
    __shared__ __attribute__((aligned(16))) float sW[kLgRows * kLgStride];
    __shared__ __attribute__((aligned(16))) float sE[kLgRows * kLgStride];
    __shared__ float sN[4][kLgSlab];                   // per-wave column sums of |v|^2
    const int64_t b = blockIdx.y;
    const int slab = blockIdx.x, c0 = kLgSlab * slab;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lo = lane & 15, hi = lane >> 4;
    const float hs = (float)a.pa[2 * b];
    const double es = a.pa[2 * b + 1];
    const float eta = (float)(a.eta_rel[layer] * es);
    const float thr = (float)(a.lambdas[layer] * a.eta_rel[layer] * es);
    const float2* Hb = a.H + b * a.K * a.M;
    float2* Wb = a.W + b * a.K * a.M;
    lg_load_slab(sH, Hb, a.K, a.M, c0, hs, false);
    lg_load_slab(sW, Wb, a.K, a.M, c0, 1.0f, false);
    {
        const float4* Eb = reinterpret_cast<const float4*>(a.E + b * kLgPart);
#pragma unroll
        for (int e = tid; e < kLgPart / 4; e += 256) {
            const int row = e >> 4, c4 = e & 15;
            *reinterpret_cast<float4*>(sE + row * kLgStride + 4 * c4) = Eb[e];
        }
    }
    __syncthreads();

    // G row tile w = E[16 w .. 16 w + 15][:] H64, antenna blocks q, 16 k-steps
    f32x4 g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) g[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int s = 0; s < 16; ++s) {
        const float ev = sE[(16 * w + lo) * kLgStride + 4 * s + hi];
        float hb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) hb[q] = sH[(4 * s + hi) * kLgStride + 16 * q + lo];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev, hb[q], g[q], 0, 0, 0);
    }
    // V = W - eta G on rows 16 w + 4 hi + v; this wave's share of each column's |v|^2
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float n2 = 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float x = fmaf(-eta, g[q][v], sW[(16 * w + 4 * hi + v) * kLgStride + 16 * q + lo]);
            g[q][v] = x;
            n2 = fmaf(x, x, n2);
        }
        n2 = column_sum(n2);
        if (hi == 0) sN[w][16 * q + lo] = n2;
    }
    __syncthreads();                       // all V formed and all W read; column sums in sN
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 16 * q + lo;
        const float n2 = (sN[0][c] + sN[1][c]) + (sN[2][c] + sN[3][c]);
        const float sc = prox_scale(col_norm(n2), thr);
#pragma unroll
        for (int v = 0; v < 4; ++v) sW[(16 * w + 4 * hi + v) * kLgStride + c] = sc * g[q][v];
    }
    __syncthreads();
    for (int e = tid; e < a.K * kLgSlab; e += 256) {
        const int k = e / kLgSlab, c = e - k * kLgSlab;
        if (c0 + c < a.M)
            Wb[(int64_t)k * a.M + c0 + c] = make_float2(sW[k * kLgStride + c], sW[(kLgMaxK + k) * kLgStride + c]);
    }
    f32x4 acc[4];
    lg_partial(sW, sH, w, lo, hi, acc);
    lg_store_partial(part_ptr(a, par ^ 1, b, slab), w, lo, hi, acc);
}

// Per deployment: SINR_k and the sum rate from the last partials (gains of
// the normalised problem with unit noise, the same SINR), then W = (sigma/s) Wn,
// p_m and ||W||_{2,1}.
__global__ __launch_bounds__(256) void lg_final_kernel(LgDev a, int par) {
    __shared__ double gain[kLgMaxK][kLgMaxK + 1];
    __shared__ double red[4];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    const int K = a.K, M = a.M;
    const float* p0 = part_ptr(a, par, b, 0);
    // |G_kj|^2 with G = Hn Wn^T = A^T, A = Wn Hn^T: entry (k, j) = |A_jk|^2
    for (int e = tid; e < K * K; e += 256) {
        const int k = e / K, j = e - k * K;
        float re = 0.f, im = 0.f;
#pragma unroll 8
        for (int sl = 0; sl < a.S; ++sl) {
            const float* q = p0 + (int64_t)sl * kLgPart;
            re += q[j * kLgRows + k] - q[(32 + j) * kLgRows + 32 + k];
            im += q[j * kLgRows + 32 + k] + q[(32 + j) * kLgRows + k];
        }
        gain[k][j] = (double)re * re + (double)im * im;
    }
    __syncthreads();
    if (tid < 64) {
        double r = 0.0;
        if (tid < K) {
            double sig = 0.0, intf = 0.0;
            for (int j = 0; j < K; ++j) (j == tid ? sig : intf) += gain[tid][j];
            const double sn = sig / (intf + 1.0);
            if (a.sinr) a.sinr[b * K + tid] = sn;
            r = log2(1.0 + sn);
        }
        for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off, 64);
        if (tid == 0 && a.rsum) a.rsum[b] = r;
    }
    const double ws = a.sigma * a.pa[2 * b];
    const float wsf = (float)ws;
    float2* Wb = a.W + b * K * M;
    double l = 0.0;
    for (int m = tid; m < M; m += 256) {
        double p = 0.0;
        float2 wv[kLgMaxK];   // all K loads of the antenna issued together
#pragma unroll
        for (int k = 0; k < kLgMaxK; ++k)
            if (k < K) wv[k] = Wb[(int64_t)k * M + m];
#pragma unroll
        for (int k = 0; k < kLgMaxK; ++k) {
            if (k < K) {
                const float2 w = wv[k];
                p += (double)w.x * w.x + (double)w.y * w.y;
                Wb[(int64_t)k * M + m] = make_float2(wsf * w.x, wsf * w.y);
            }
        }
        if (a.p_ant) a.p_ant[b * M + m] = ws * ws * p;
        l += sqrt(p);
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = l;
    __syncthreads();
    if (tid == 0 && a.l21) a.l21[b] = ws * (red[0] + red[1] + red[2] + red[3]);
}

}  // namespace

size_t pa_large_workspace_bytes(int64_t B, int K, int M) {
    (void)K;
    const int64_t S = (M + kLgSlab - 1) / kLgSlab;
    return sizeof(float) * (size_t)(2 * B * S + B) * kLgPart;
}

// ws: [B][2] normalisation factors (aligned to 256 B), then the partials and E.
dmimo_status launch_pa_large(int64_t B, int K, int M, const void* H, const double* gamma,
                             double sigma2, int layers, const double* lambdas, const double* eta_rel,
                             void* W, double* p_ant, double* l21, double* sinr, double* rsum,
                             void* ws, size_t pa_bytes, hipStream_t s) {
    if (K > kLgMaxK || M > kLgMaxM) return fail(DMIMO_E_SHAPE, "pa_precoder: K <= 32 and M <= 4096");
    if (B > 0xffff) return fail(DMIMO_E_SHAPE, "pa_precoder: at most 65535 deployments per call on this path");
    LgDev a;
    a.K = K;
    a.M = M;
    a.S = (M + kLgSlab - 1) / kLgSlab;
    a.layers = layers;
    a.H = reinterpret_cast<const float2*>(H);
    a.W = reinterpret_cast<float2*>(W);
    a.lambdas = lambdas;
    a.eta_rel = eta_rel;
    a.pa = static_cast<const double*>(ws);
    for (int k = 0; k < kLgMaxK; ++k) a.d[k] = k < K ? (float)std::sqrt(gamma ? gamma[k] : 1.0) : 0.0f;
    a.sigma = std::sqrt(sigma2);
    a.part = reinterpret_cast<float*>(static_cast<char*>(ws) + pa_bytes);
    a.E = a.part + 2 * B * a.S * kLgPart;
    a.p_ant = p_ant;
    a.l21 = l21;
    a.sinr = sinr;
    a.rsum = rsum;
    a.B = B;
    dmimo_status st = launch_pa_prepare(B, K, M, H, static_cast<double*>(ws), s);
    if (st) return st;
    const dim3 slabs((unsigned)a.S, (unsigned)B), entries(kLgPart / 64, (unsigned)B);
    lg_init_kernel<<<slabs, 256, 0, s>>>(a);
    int par = 0;
    for (int i = 0; i < layers; ++i) {
        lg_reduce_kernel<<<entries, 64, 0, s>>>(a, par);
        lg_layer_kernel<<<slabs, 256, 0, s>>>(a, i, par);
        par ^= 1;
    }
    lg_final_kernel<<<dim3((unsigned)B), 256, 0, s>>>(a, par);
    return check_launch("pa_precoder (slab path)");
}

}  // namespace dmimo
