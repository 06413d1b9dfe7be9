// Work tables and launches of the overlapping trigger windows, coincidence
// and clustering (Sec. II.D.3-4), shared by the host plan (lloid_plan.hip)
// and its kernels (lloid_coinc.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lloid.h"

namespace lloid {

constexpr int kCoincMaxDet = 8;   // detectors a coincidence call supports

// one entry per template, banks in order
struct TrigTemplate {
    int64_t series_off;      // float offset of detector 0's series of this template
    int64_t det_stride;      // floats between detectors (M F 2)
    int64_t peak_off;        // entry of detector 0's trigger
    int32_t M, pad_;         // templates of the bank
};

// one entry per bank
struct CoincBank {
    int64_t peak_off;        // first trigger entry of the bank
    int32_t M, pad_;
};

// coincidence windows in samples, w[a][d] for detectors a, d
struct CoincWindows {
    int32_t w[kCoincMaxDet][kCoincMaxDet];
};

// window triggers: the stride's trigger merged with the last `overlap`
// samples of the previous stride's series (prev may be null)
hipError_t launch_window_triggers(hipStream_t, const TrigTemplate *tab, int32_t n_tmpl, int32_t n_det, int32_t F,
                                  const float *prev, const lloid_peak *peaks, int32_t overlap, float threshold,
                                  lloid_peak *triggers);
// per bank: the coincident event with the largest network SNR
hipError_t launch_coinc(hipStream_t, const CoincBank *banks, int32_t n_banks, int32_t n_det, const CoincWindows &w,
                        const lloid_peak *triggers, lloid_event *events);

}  // namespace lloid
