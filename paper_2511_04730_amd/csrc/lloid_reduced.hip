// Reduced-precision variants of the correlation and mixing contractions.
#include <hip/hip_runtime.h>

#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

hipError_t launch_corr_reduced(const LaunchCtx &, int, const CorrItem *, int32_t) { return hipErrorNotSupported; }

hipError_t launch_mix_reduced(const LaunchCtx &, int, const MixItem *, int32_t, const MixBank *, const MixSlice *,
                              const float *, float *, PartialPeak *, int32_t, int32_t, int32_t, int32_t, int32_t) {
    return hipErrorNotSupported;
}

hipError_t launch_convert_reduced(hipStream_t, const double *, int32_t, int32_t, int32_t, const double *, int, int,
                                  void *, void *, int32_t, float *) {
    return hipErrorNotSupported;
}

}  // namespace lloid
