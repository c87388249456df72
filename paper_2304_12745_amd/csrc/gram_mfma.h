// Split-precision MFMA Gram (FP16 or BF16 hi/lo x3, FP32 accumulation).
#pragma once
#include "dmimo_internal.h"

namespace dmimo {
dmimo_status launch_gram_mfma(int64_t B, int K, int64_t M, const float2* H, bool bf16, float2* G,
                              hipStream_t s);
}
