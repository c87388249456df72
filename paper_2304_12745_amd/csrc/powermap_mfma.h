// Power map with the K-stream contraction on MFMA.
#pragma once
#include "kernels.h"

namespace dmimo {
// FP32 mode, K >= 3: contraction on FP32 MFMA.
dmimo_status launch_powermap_f32_mfma(const PowermapArgs& a, hipStream_t s);
// Mixed modes (FP16 / BF16 hi-lo x3 MFMA).
dmimo_status launch_powermap_mfma(const PowermapArgs& a, hipStream_t s);
}
