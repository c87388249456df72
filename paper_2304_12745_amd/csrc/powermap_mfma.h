// Power map with the K-stream contraction on MFMA.
#pragma once
#include "kernels.h"

namespace dmimo {
dmimo_status launch_powermap_mfma(const PowermapArgs& a, hipStream_t s);
}
