// K x K Gram G = H H^H on the matrix cores: FP16 or BF16 hi/lo x3 products,
// FP32 accumulation (split-precision products: Markidis et al. 2018, Ootomo
// and Yokota 2022).
//
// Real form: with Hr, Hi the real and imaginary parts of H (K x M),
//     Re G = [Hr | Hi] [Hr | Hi]^T,   Im G = [Hi | -Hr] [Hr | Hi]^T,
// a pair of real products over the 2M-long stacked axis.  v_mfma_f32_16x16x32
// consumes 32 stacked values = 16 antennas per step.  Lane 16g + i holds
// A[i][8g .. 8g+7] and B[8g .. 8g+7][i].  The stacked axis of a step is
// ordered (Hr of antennas 0-7, Hi of 0-7, Hr of 8-15, Hi of 8-15), so lane
// (g, i) needs 8 consecutive antennas of user i.  It loads those 8 complex
// values once and builds from them:
//   * its A element of [Hr | Hi],
//   * its A element of [Hi | -Hr],
//   * its B element: B = [Hr | Hi]^T, whose column i equals row i of A.  For a
//     diagonal 16 x 16 tile the B registers ARE the A registers.
// K <= 16 uses one tile pair.  K <= 32 uses the three distinct tile pairs of
// the 2 x 2 block Hermitian matrix.  Every value x is split into
// hi = rn16(x), lo = rn16(x - hi), and three products accumulate:
// A_hi B_hi + A_lo B_hi + A_hi B_lo.
//
// FP16 scaling: each deployment's H is scaled by a power of two that puts
// max |h| in [2^13, 2^14), so hi and lo stay in the FP16 normal range.  G is
// scaled back exactly.  BF16 needs no scaling.
//
// One wavefront per deployment, four deployments per workgroup.  The kernel
// reads H once from HBM (plus one cached pass for the FP16 scale); the
// upper triangle is written and mirrored, so G is exactly Hermitian.
#include "gram_mfma.h"

namespace dmimo {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool BF16>
__device__ __forceinline__ uint32_t rn16(float x, float& back) {
    if constexpr (BF16) {
        const __bf16 h = (__bf16)x;
        back = (float)h;
        return __builtin_bit_cast(uint16_t, h);
    } else {
        const _Float16 h = (_Float16)x;
        back = (float)h;
        return __builtin_bit_cast(uint16_t, h);
    }
}

template <bool BF16>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
    if constexpr (BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// hi / lo 16-bit packs of 8 FP32 values
template <bool BF16>
__device__ __forceinline__ void split8(const float (&x)[8], u32x4& hi, u32x4& lo) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float b0, b1, c0, c1;
        const uint32_t h0 = rn16<BF16>(x[2 * i], b0), h1 = rn16<BF16>(x[2 * i + 1], b1);
        const uint32_t l0 = rn16<BF16>(x[2 * i] - b0, c0), l1 = rn16<BF16>(x[2 * i + 1] - b1, c1);
        hi[i] = h0 | (h1 << 16);
        lo[i] = l0 | (l1 << 16);
    }
}

// RB = number of 16-user row blocks (1: K <= 16, 2: K <= 32)
template <int RB, bool BF16>
__global__ __launch_bounds__(256) void gram_x3_kernel(const float2* __restrict__ H,
                                                      float2* __restrict__ G, int64_t B, int K,
                                                      int64_t M) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;   // whole wavefront exits together
    const int i = lane & 15;
    const int g = lane >> 4;
    const int half = g >> 1;     // antennas 0-7 or 8-15 of the step
    const bool imag = g & 1;     // this lane's stacked slot: Hr (even g) or Hi (odd g)
    const float2* Hb = H + b * K * M;

    // FP16: deployment scale 2^s with max |h| 2^s in [2^13, 2^14)
    float scale = 1.0f;
    if constexpr (!BF16) {
        float mx = 0.0f;
        for (int64_t e = lane; e < (int64_t)K * M; e += 64) {
            const float2 h = Hb[e];
            mx = fmaxf(mx, fmaxf(fabsf(h.x), fabsf(h.y)));
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (mx > 0.0f) scale = ldexpf(1.0f, 14 - (ilogbf(mx) + 1));
    }

    f32x4 accr[RB * (RB + 1) / 2], acci[RB * (RB + 1) / 2];
#pragma unroll
    for (int t = 0; t < RB * (RB + 1) / 2; ++t) {
        accr[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        acci[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    for (int64_t m0 = 0; m0 < M; m0 += 16) {
        u32x4 ar_h[RB], ar_l[RB], ai_h[RB], ai_l[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int k = 16 * rb + i;
            float xr[8], xi[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t m = m0 + 8 * half + q;
                float2 h = make_float2(0.f, 0.f);
                if (k < K && m < M) h = Hb[(int64_t)k * M + m];
                // [Hr | Hi] slot and [Hi | -Hr] slot of this lane
                xr[q] = (imag ? h.y : h.x) * scale;
                xi[q] = (imag ? -h.x : h.y) * scale;
            }
            split8<BF16>(xr, ar_h[rb], ar_l[rb]);
            split8<BF16>(xi, ai_h[rb], ai_l[rb]);
        }
        // tile (r, c), r <= c: rows of block r against columns of block c
        int t = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
            for (int c = r; c < RB; ++c, ++t) {
                f32x4 gr = accr[t], gi = acci[t];
                gr = mfma16<BF16>(ar_h[r], ar_h[c], gr);
                gr = mfma16<BF16>(ar_l[r], ar_h[c], gr);
                gr = mfma16<BF16>(ar_h[r], ar_l[c], gr);
                gi = mfma16<BF16>(ai_h[r], ar_h[c], gi);
                gi = mfma16<BF16>(ai_l[r], ar_h[c], gi);
                gi = mfma16<BF16>(ai_h[r], ar_l[c], gi);
                accr[t] = gr;
                acci[t] = gi;
            }
        }
    }

    // lane (g, j) holds tile entry (4 g + r, j); write the upper triangle and
    // mirror it
    const float inv = 1.0f / (scale * scale);   // exact: a power of two
    float2* Gb = G + b * K * K;
    int t = 0;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
        for (int c = r; c < RB; ++c, ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * r + 4 * g + q;
                const int j = 16 * c + i;
                if (k >= K || j >= K || j < k) continue;
                const float re = accr[t][q] * inv;
                const float im = k == j ? 0.0f : acci[t][q] * inv;
                Gb[(int64_t)k * K + j] = make_float2(re, im);
                if (j != k) Gb[(int64_t)j * K + k] = make_float2(re, -im);
            }
        }
    }
}

}  // namespace

dmimo_status launch_gram_mfma(int64_t B, int K, int64_t M, const float2* H, bool bf16, float2* G,
                              hipStream_t s) {
    const int64_t blocks = ceil_div(B, 4);
    if (blocks > 0x7fffffff) return fail(DMIMO_E_SHAPE, "gram: B too large");
    dim3 grid((unsigned)blocks), block(256);
    if (K <= 16) {
        if (bf16) gram_x3_kernel<1, true><<<grid, block, 0, s>>>(H, G, B, K, M);
        else gram_x3_kernel<1, false><<<grid, block, 0, s>>>(H, G, B, K, M);
    } else {
        if (bf16) gram_x3_kernel<2, true><<<grid, block, 0, s>>>(H, G, B, K, M);
        else gram_x3_kernel<2, false><<<grid, block, 0, s>>>(H, G, B, K, M);
    }
    return check_launch("gram_x3_kernel");
}

}  // namespace dmimo
