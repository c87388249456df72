// Split-precision building blocks: an FP32 value x as hi + lo with hi, lo
// in FP16 or BF16, and the three products hi*hi + lo*hi + hi*lo on the
// FP16/BF16 matrix cores with FP32 accumulation (the published split-precision
// method: Markidis et al. 2018; Ootomo and Yokota 2022).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dmimo {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool BF16>
__device__ __forceinline__ uint32_t pack_hi(float x0, float x1, float& r0, float& r1) {
    // hi parts of x0, x1 packed in one register; r0, r1 = the FP32 remainders
    if constexpr (BF16) {
        const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
        const uint32_t b0 = __builtin_bit_cast(uint16_t, h0), b1 = __builtin_bit_cast(uint16_t, h1);
        r0 = x0 - __uint_as_float(b0 << 16);
        r1 = x1 - __uint_as_float(b1 << 16);
        return b0 | (b1 << 16);
    } else {
        const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x0, x1));
        // x - hi, exact, by one mixed-precision FMA each that reads its FP16
        // half in place (instead of a conversion back to FP32 and a subtraction)
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r0) : "v"(h), "v"(x0));
        asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r1) : "v"(h), "v"(x1));
        return h;
    }
}

template <bool BF16>
__device__ __forceinline__ uint32_t pack_lo(float r0, float r1) {
    if constexpr (BF16) {
        const __bf16 h0 = (__bf16)r0, h1 = (__bf16)r1;
        return (uint32_t)__builtin_bit_cast(uint16_t, h0) |
               ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    } else {
        return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(r0, r1));
    }
}

// round-to-nearest 16-bit value of x (table entries)
template <bool BF16>
__device__ __forceinline__ uint16_t to16(float x, float& back) {
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

// v_mfma_f32_16x16x16_bf16: A[i][4g..4g+3] in lane 16 g + i, B[4g..4g+3][j]
// in lane 16 g + j, four BF16 values in two registers.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16k16_bf16(u32x2 a, u32x2 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                     __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}

}  // namespace dmimo
