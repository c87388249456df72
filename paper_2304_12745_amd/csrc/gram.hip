// K x K Gram G = H H^H per deployment (VALU paths: FP64 and FP32).
//
// One workgroup per deployment.  H[b] is streamed through LDS in tiles of
// 64 antennas.  G is cut into 8 x 8 blocks of KT/8 x KT/8 entries (KT = 8,
// 16 or 32 >= K); the four adjacent threads of a block take every fourth
// antenna, so each h value a thread reads feeds KT/8 complex products, and
// combine their sums at the end.  Only blocks on or above the diagonal are
// formed; each entry (k, j), j >= k, is written with its conjugate mirror, so
// G is exactly Hermitian with a zero imaginary diagonal.  Work is 4 K^2 M
// real FMA per deployment for 8 K M bytes read.
#include "kernels.h"
#include "gram_mfma.h"

namespace dmimo {

namespace {

constexpr int kTile = 64;

template <typename T2, typename R, int KT>
__global__ __launch_bounds__(256) void gram_valu_kernel(const T2* __restrict__ H,
                                                        T2* __restrict__ G, int K,
                                                        int64_t M) {
    constexpr int BS = KT / 8;
    // row stride with stride * BS = 4 (mod 32): the 8 block columns x 4
    // antenna phases of a wave's reads fall in distinct 4-byte banks
    constexpr int LS = kTile + 4 / BS;
    __shared__ R sre[KT][LS];
    __shared__ R sim[KT][LS];
    const int64_t b = blockIdx.x;
    const T2* Hb = H + b * K * M;
    const int tid = threadIdx.x;
    const int blk = tid >> 2, ph = tid & 3;
    const int k0 = BS * (blk >> 3), j0 = BS * (blk & 7);
    const bool active = j0 >= k0 && k0 < K && j0 < K;
    R ar[BS][BS], ai[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) ar[u][v] = ai[u][v] = (R)0;
    for (int64_t m0 = 0; m0 < M; m0 += kTile) {
        const int mc = (int)std::min<int64_t>(kTile, M - m0);
        __syncthreads();
        {   // 256 threads; a thread's loads all issued before its LDS stores
            constexpr int IT = KT * kTile / 256;
            T2 hv[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + 256 * it;
                const int k = e / kTile, mm = e - k * kTile;
                if (k < K && mm < mc) hv[it] = Hb[(int64_t)k * M + m0 + mm];
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + 256 * it;
                const int k = e / kTile, mm = e - k * kTile;
                if (k < K && mm < mc) {
                    sre[k][mm] = (R)hv[it].x;
                    sim[k][mm] = (R)hv[it].y;
                }
            }
        }
        __syncthreads();
        if (active)
            for (int mm = ph; mm < mc; mm += 4) {
                R kr[BS], ki[BS], jr[BS], ji[BS];
#pragma unroll
                for (int u = 0; u < BS; ++u) {
                    // rows past K are never written out; read a valid row instead
                    const int k = k0 + u < K ? k0 + u : k0;
                    const int j = j0 + u < K ? j0 + u : j0;
                    kr[u] = sre[k][mm];
                    ki[u] = sim[k][mm];
                    jr[u] = sre[j][mm];
                    ji[u] = sim[j][mm];
                }
#pragma unroll
                for (int u = 0; u < BS; ++u)
#pragma unroll
                    for (int v = 0; v < BS; ++v) {
                        ar[u][v] = fma(kr[u], jr[v], fma(ki[u], ji[v], ar[u][v]));
                        ai[u][v] = fma(ki[u], jr[v], fma(-kr[u], ji[v], ai[u][v]));
                    }
            }
    }
    T2* Gb = G + b * K * K;
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v) {
            R xr = ar[u][v], xi = ai[u][v];
            xr += __shfl_xor(xr, 1, 64);
            xi += __shfl_xor(xi, 1, 64);
            xr += __shfl_xor(xr, 2, 64);
            xi += __shfl_xor(xi, 2, 64);
            const int k = k0 + u, j = j0 + v;
            if (ph != 0 || !active || k >= K || j >= K || j < k) continue;
            T2 g;
            g.x = xr;
            g.y = (j == k) ? (R)0 : xi;
            Gb[(int64_t)k * K + j] = g;
            if (j != k) {
                T2 c;
                c.x = g.x;
                c.y = -g.y;
                Gb[(int64_t)j * K + k] = c;
            }
        }
}

template <typename T2, typename R>
void launch_valu(dim3 grid, dim3 block, const T2* H, T2* G, int K, int64_t M, hipStream_t s) {
    if (K <= 8) gram_valu_kernel<T2, R, 8><<<grid, block, 0, s>>>(H, G, K, M);
    else if (K <= 16) gram_valu_kernel<T2, R, 16><<<grid, block, 0, s>>>(H, G, K, M);
    else gram_valu_kernel<T2, R, 32><<<grid, block, 0, s>>>(H, G, K, M);
}

}  // namespace

// batched.hip: FP32 and MIX at K <= 16, M <= 256 on the matrix cores,
// persistent workgroups (G complex64).
dmimo_status launch_gram_batched(int64_t B, int K, int64_t M, const void* H, int prec, void* G,
                                 hipStream_t s);

// Where that kernel measured faster than the one-wave MIX kernel and the VALU
// FP32 kernel (16 384 deployments): MIX with K M > 512 (K = 16, M = 256:
// 0.113 against 0.326 ms FP16x3), FP32 with K > 12 and M > 128 (K = 16,
// M = 256: 0.119 against 0.184 ms; at K <= 8 the VALU kernel's K^2 work is
// the smaller, and at M <= 64 one wave of four has antennas).
bool gram_batched_shape(int K, int64_t M, int prec) {
    if (prec == DMIMO_F64 || K > 16 || M > 256) return false;
    return prec == DMIMO_F32 ? K > 12 && M > 128 : (int64_t)K * M > 512;
}

dmimo_status launch_gram(int64_t B, int K, int64_t M, const void* H, int prec, void* G,
                         hipStream_t s) {
    dim3 grid((unsigned)B), block(256);
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "gram: B too large");
    if (gram_batched_shape(K, M, prec)) return launch_gram_batched(B, K, M, H, prec, G, s);
    switch (prec) {
        case DMIMO_F64:
            launch_valu<double2, double>(grid, block, reinterpret_cast<const double2*>(H),
                                         reinterpret_cast<double2*>(G), K, M, s);
            return check_launch("gram_valu_kernel<f64>");
        case DMIMO_F32:
            launch_valu<float2, float>(grid, block, reinterpret_cast<const float2*>(H),
                                       reinterpret_cast<float2*>(G), K, M, s);
            return check_launch("gram_valu_kernel<f32>");
        default:
            return launch_gram_mfma(B, K, M, reinterpret_cast<const float2*>(H),
                                    prec == DMIMO_MIX_BF16X3, reinterpret_cast<float2*>(G), s);
    }
}

}  // namespace dmimo
