// Register layouts and building blocks shared by the PGD / unfolded-PGD
// kernels that run the layer's two complex products on
// v_mfma_f32_16x16x4_f32 (K <= 8 users).
//
// Real embedding.  A K x M complex matrix X is held as 16 real rows
// X16 = [Xr; Xi] (rows K..7 and 8+K..15 are zero).  Then, with H16 = [Hr; Hi]:
//   D1 = X16 H16^T (16 x 16)  gives A = X H^T as
//        Ar = D1[a][b] - D1[8+a][8+b],  Ai = D1[a][8+b] + D1[8+a][b];
//   with E = [[Br, Bi], [Bi, -Br]] for a K x K complex B,
//        E H16 = [Re(B H^*); Im(B H^*)]   (16 x M).
// Both are exact 16 x 16 MFMA tiles at K = 8.
//
// One wave owns AW antennas c0 .. c0+AW-1 (AW = 16, 32 or 64; fewer antennas
// per wave give shorter MFMA chains and more waves when channels are few).
// Lane (hi, lo) = (lane >> 4, lane & 15).
//   operand layout  "A":  AW/4 floats, row lo at antennas c0 + (AW/4) hi + c;
//                         serves as both operands of D1 (the antenna order
//                         inside a sum is free).
//   operand layout  "B2": [q][s], row 4 s + hi at antenna c0 + 16 q + lo
//                         (B operand of E H16, block q < AW/16 of 16 antennas, k-step s).
//   output layout   "D":  [q][r], row 4 hi + r at antenna c0 + 16 q + lo
//                         (the MFMA result layout of E H16).
//   E operand:            [s], E[lo][4 s + hi].
// MFMA 16x16x4 f32: A[i][k] in lane 16 k + i, B[k][j] in lane 16 k + j,
// D[i][j] in lane 16 (i / 4) + j, register i % 4.
#pragma once

#include "dmimo_internal.h"

namespace dmimo {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPgdMfmaMaxWaves = 4;     // waves per channel
constexpr int kPartFloats = 16 * 17;    // one wave's D1 partial, padded rows

// Planar LDS image: row p * 8 + k holds part p (0 re, 1 im) of row k.  Row
// stride AW nw + 4 floats (AW nw is a multiple of 16) puts the four 16-lane
// groups of a wave on distinct banks and keeps rows 16-byte aligned.
__host__ __device__ __forceinline__ int pl_stride(int ncol) { return ncol + 4; }

template <int AW>
struct PgdLane {
    int tid, wave, lane, lo, hi, c0;
    __device__ PgdLane() {
        tid = threadIdx.x;
        wave = tid >> 6;
        lane = tid & 63;
        lo = lane & 15;
        hi = lane >> 4;
        c0 = AW * wave;
    }
};

// scale * X (K x M, complex64, row-major) into the planar image, zero padded
// to 8 x ncol, optionally conjugated.  All threads of the block take part.
// IT = 8 ncol / blockDim.x iterations per thread, a compile-time count so
// that all of a thread's loads are issued before its LDS stores.
template <int IT>
__device__ __forceinline__ void load_planar(float* sX, int stride, int ncol, const float2* X, int K,
                                            int M, bool conj, float scale = 1.0f) {
    float vx[IT], vy[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + blockDim.x * it;
        const int k = e / ncol, m = e - k * ncol;
        float2 x = make_float2(0.f, 0.f);
        if (e < 8 * ncol && k < K && m < M) x = X[k * M + m];
        vx[it] = x.x;
        vy[it] = x.y;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + blockDim.x * it;
        const int k = e / ncol, m = e - k * ncol;
        if (e < 8 * ncol) {
            sX[k * stride + m] = scale * vx[it];
            sX[(8 + k) * stride + m] = conj ? -(scale * vy[it]) : scale * vy[it];
        }
    }
}

template <int AW>
__device__ __forceinline__ void read_op_a(const float* sX, int stride, const PgdLane<AW>& L,
                                          float (&XA)[AW / 4]) {
    // 16-byte aligned: stride and c0 + (AW/4) hi are multiples of 4 floats
    const float4* src = reinterpret_cast<const float4*>(sX + L.lo * stride + L.c0 + (AW / 4) * L.hi);
#pragma unroll
    for (int t = 0; t < AW / 16; ++t) {
        const float4 v = src[t];
        XA[4 * t] = v.x;
        XA[4 * t + 1] = v.y;
        XA[4 * t + 2] = v.z;
        XA[4 * t + 3] = v.w;
    }
}

template <int AW>
__device__ __forceinline__ void read_op_b2(const float* sX, int stride, const PgdLane<AW>& L,
                                           float (&XB)[AW / 16][4]) {
#pragma unroll
    for (int q = 0; q < AW / 16; ++q)
#pragma unroll
        for (int s = 0; s < 4; ++s) XB[q][s] = sX[(4 * s + L.hi) * stride + L.c0 + 16 * q + L.lo];
}

template <int AW>
__device__ __forceinline__ void read_out_d(const float* sX, int stride, const PgdLane<AW>& L,
                                           float (&XD)[AW / 16][4]) {
#pragma unroll
    for (int q = 0; q < AW / 16; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) XD[q][r] = sX[(4 * L.hi + r) * stride + L.c0 + 16 * q + L.lo];
}

template <int AW>
__device__ __forceinline__ void write_out_d(float* sX, int stride, const PgdLane<AW>& L,
                                            const float (&XD)[AW / 16][4]) {
#pragma unroll
    for (int q = 0; q < AW / 16; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sX[(4 * L.hi + r) * stride + L.c0 + 16 * q + L.lo] = XD[q][r];
}

// Orders this wave's LDS writes before its later LDS reads of other lanes' data.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// This wave's share of D1 = X16 H16^T over its AW antennas.
template <int AW>
__device__ __forceinline__ f32x4 d1_partial(const float (&XA)[AW / 4], const float (&HA)[AW / 4]) {
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < AW / 4; ++c) d = __builtin_amdgcn_mfma_f32_16x16x4f32(XA[c], HA[c], d, 0, 0, 0);
    return d;
}

template <int AW>
__device__ __forceinline__ void put_partial(float* part, const PgdLane<AW>& L, f32x4 d) {
#pragma unroll
    for (int r = 0; r < 4; ++r) part[(4 * L.hi + r) * 17 + L.lo] = d[r];
}

// E operand of B = (X H^T) - diag(dg) from the NW partials of D1 (each
// entry summed over the partials in wave order); dg is this lane's diagonal
// entry d[lo & 7], zero for no shift.  Column l = 4 s + hi lies in the top
// half exactly for s < 2, so the block of every entry is known per s.
template <int NW, int AW>
__device__ __forceinline__ void embed_operand(const float* parts, const PgdLane<AW>& L, float dg,
                                              float (&E)[4]) {
    const int ia = L.lo & 7;
    const bool itop = L.lo < 8;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int lb = (4 * s + L.hi) & 7;
        const bool same = (s < 2) == itop;          // +-(Br)[ia][lb], else Bi[ia][lb]
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
        E[s] = (same && !itop) ? -v : v;
    }
}

// |A_jk|^2 of A = X H^T (j = row, k = column, both < 8) from the NW partials.
template <int NW>
__device__ __forceinline__ float gain_sq(const float* parts, int j, int k) {
    float re = 0.0f, im = 0.0f;
#pragma unroll
    for (int p = 0; p < NW; ++p) {
        const float* q = parts + p * kPartFloats;
        re += q[j * 17 + k] - q[(8 + j) * 17 + 8 + k];
        im += q[j * 17 + 8 + k] + q[(8 + j) * 17 + k];
    }
    return re * re + im * im;
}

// Block q of E H16 = [Re(B H^*); Im(B H^*)] in the output layout.
template <int NQ>
__device__ __forceinline__ f32x4 apply_block(const float (&E)[4], const float (&HB)[NQ][4], int q) {
    f32x4 g = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) g = __builtin_amdgcn_mfma_f32_16x16x4f32(E[s], HB[q][s], g, 0, 0, 0);
    return g;
}

// Sum over the four lanes of an antenna column (hi = 0..3), with the gfx950
// row swaps: after permlane16_swap / permlane32_swap of x with itself the
// two results of a lane are x of the lane and x of its partner in the other
// row (16 apart) / half (32 apart).  Every lane of a column gets the same
// bits: (x0 + x1) + (x2 + x3), each pair added in the same order.
__device__ __forceinline__ float column_sum(float x) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// Column norm and prox scale 1 - thr / max(n, thr), with the hardware square
// root and reciprocal (about 1 ulp each).  The branch on n > thr keeps a
// switched-off column exactly zero (thr * rcp(thr) need not round to 1);
// at thr = 0 the prox is the identity.
__device__ __forceinline__ float col_norm(float n2) { return __builtin_amdgcn_sqrtf(n2); }
__device__ __forceinline__ float prox_scale(float nrm, float thr) {
    if (!(thr > 0.0f)) return 1.0f;
    return nrm > thr ? 1.0f - thr * __builtin_amdgcn_rcpf(nrm) : 0.0f;
}

inline size_t pgd_mfma_lds_bytes(int aw, int nw) {
    return sizeof(float) * (16 * (size_t)pl_stride(aw * nw) + 2 * (size_t)nw * kPartFloats);
}

// Antennas per wave: 64 when the launch has at least one wave per SIMD at
// 64 (1024 waves); else the smallest of 16 / 32 / 64 that still covers M
// with at most 4 waves.  Measured at K = 8, M = 64: 16 antennas per wave win
// at 64 channels (training batches), 64 win at 1024 channels (7.2 vs 5.2 ms
// for 5000 iterations), where the cross-wave sums cost more than the extra
// waves bring.
inline int pgd_antennas_per_wave(int64_t channels, int M) {
    const int64_t waves64 = channels * ((M + 63) / 64);
    if (waves64 >= 1024) return 64;
    if (M <= 64) return 16;
    if (M <= 128) return 32;
    return 64;
}

}  // namespace dmimo
