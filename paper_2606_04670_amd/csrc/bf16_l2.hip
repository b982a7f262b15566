// BF16-MFMA l2 bound path (placeholder until the kernel lands).
#include "host_common.hpp"

namespace lip {

lip_status run_bounds_bf16(const MetricInfo &, const float *, const float *, int64_t, float,
                           const float *, const float *, int64_t, float *, float *, float *,
                           int32_t *, int32_t *, void *, size_t, hipStream_t)
{
    return LIP_E_UNSUPPORTED;
}

size_t bf16_extra_bytes(int64_t, int64_t, int) { return 0; }

}  // namespace lip
