// Work table and launches of the xi^2 statistic (Sec. II.D.2), shared by the
// host plan (lloid_plan.hip) and its kernel (lloid_xi2.hip).  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lloid.h"

namespace lloid {

// One entry per template, banks in order.
struct XiTemplate {
    int64_t series_off;      // float offset of detector 0's series of this template
    int64_t det_stride;      // floats between detectors (M F 2)
    int64_t peak_off;        // entry of detector 0's trigger (and its xi^2 output)
    int64_t acf_off;         // float offset of the template's R(t), t = -delta..delta, (re, im)
    int32_t A, M;            // autocorrelation length (odd); templates of the bank
};

// xi^2 at the triggers of one stride
hipError_t launch_xi2(hipStream_t, const XiTemplate *tab, int32_t n_tmpl, int32_t n_det, int32_t F,
                      const float *prev, const float *cur, const float *next, const lloid_peak *peaks,
                      const float *acf, float *out);
// float64 -> float32 copy of the autocorrelations
hipError_t launch_convert_f64_f32(hipStream_t, const double *src, int64_t n, float *dst);

}  // namespace lloid
