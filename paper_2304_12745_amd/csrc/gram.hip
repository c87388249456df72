// K x K Gram G = H H^H per deployment (VALU paths: FP64 and FP32).
//
// One workgroup per deployment.  H[b] is streamed through LDS in tiles of
// 64 antennas.  Each thread owns entries (k, j) with j >= k of the upper
// triangle and accumulates sum_m h_km conj(h_jm).  It writes that entry and
// its conjugate mirror, so G is exactly Hermitian, with a zero imaginary
// diagonal.  Work is 4 K^2 M real FMA per deployment for 8 K M bytes read:
// HBM-bound for every K <= 32.
#include "kernels.h"
#include "gram_mfma.h"

namespace dmimo {

namespace {

constexpr int kTile = 64;

template <typename T2, typename R>
__global__ __launch_bounds__(256) void gram_valu_kernel(const T2* __restrict__ H,
                                                        T2* __restrict__ G, int K,
                                                        int64_t M) {
    __shared__ R sre[DMIMO_K_MAX][kTile + 1];
    __shared__ R sim[DMIMO_K_MAX][kTile + 1];
    const int64_t b = blockIdx.x;
    const T2* Hb = H + b * K * M;
    const int tid = threadIdx.x;
    const int nent = K * K;
    // each thread owns up to 4 entries (K <= 32 -> K^2 <= 1024 = 4 * 256)
    R accr[4] = {0, 0, 0, 0};
    R acci[4] = {0, 0, 0, 0};
    for (int64_t m0 = 0; m0 < M; m0 += kTile) {
        const int mc = (int)std::min<int64_t>(kTile, M - m0);
        __syncthreads();
        for (int e = tid; e < K * kTile; e += blockDim.x) {
            const int k = e / kTile;
            const int mm = e - k * kTile;
            if (mm < mc) {
                const T2 h = Hb[(int64_t)k * M + m0 + mm];
                sre[k][mm] = (R)h.x;
                sim[k][mm] = (R)h.y;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            if (e >= nent) break;
            const int k = e / K;
            const int j = e - k * K;
            if (j < k) continue;
            R ar = accr[q], ai = acci[q];
            for (int mm = 0; mm < mc; ++mm) {
                const R kr = sre[k][mm], ki = sim[k][mm];
                const R jr = sre[j][mm], ji = sim[j][mm];
                ar = fma(kr, jr, fma(ki, ji, ar));
                ai = fma(ki, jr, fma(-kr, ji, ai));
            }
            accr[q] = ar;
            acci[q] = ai;
        }
    }
    T2* Gb = G + b * K * K;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + q * 256;
        if (e >= nent) break;
        const int k = e / K;
        const int j = e - k * K;
        if (j < k) continue;
        T2 v;
        v.x = accr[q];
        v.y = (j == k) ? (R)0 : acci[q];
        Gb[(int64_t)k * K + j] = v;
        if (j != k) {
            T2 c;
            c.x = v.x;
            c.y = -v.y;
            Gb[(int64_t)j * K + k] = c;
        }
    }
}

}  // namespace

dmimo_status launch_gram(int64_t B, int K, int64_t M, const void* H, int prec, void* G,
                         hipStream_t s) {
    dim3 grid((unsigned)B), block(256);
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "gram: B too large");
    switch (prec) {
        case DMIMO_F64:
            gram_valu_kernel<double2, double><<<grid, block, 0, s>>>(
                reinterpret_cast<const double2*>(H), reinterpret_cast<double2*>(G), K, M);
            return check_launch("gram_valu_kernel<f64>");
        case DMIMO_F32:
            gram_valu_kernel<float2, float><<<grid, block, 0, s>>>(
                reinterpret_cast<const float2*>(H), reinterpret_cast<float2*>(G), K, M);
            return check_launch("gram_valu_kernel<f32>");
        default:
            return launch_gram_mfma(B, K, M, reinterpret_cast<const float2*>(H),
                                    prec == DMIMO_MIX_BF16X3, reinterpret_cast<float2*>(G), s);
    }
}

}  // namespace dmimo
