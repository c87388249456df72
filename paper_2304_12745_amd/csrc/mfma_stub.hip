#include "gram_mfma.h"
#include "powermap_mfma.h"

namespace dmimo {
dmimo_status launch_gram_mfma(int64_t, int, int64_t, const float2*, bool, float2*, hipStream_t) {
    return fail(DMIMO_E_UNSUPPORTED, "gram: mixed precision not built yet");
}
}
