// Constants and per-push state of the whitener kernels (lloid_whiten.hip).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lloid {

constexpr int kWhitenMaxDet = 32;        // detectors per whitener (one gap-mask bit each)
constexpr int kWhitenMaxMed = 15;        // longest median
constexpr float kEulerGammaExp = 1.7810724179901979f;   // e^gamma: chi^2_2 arithmetic over geometric mean

// per push: which detectors skip their block, and the blocks each has seen
// (including this push's)
struct WhitenDetState {
    uint32_t gap_mask;
    int32_t n_avg;
    int32_t blocks[kWhitenMaxDet];
};

hipError_t launch_whiten_block(hipStream_t, const float *in, int64_t in_ld, const float *prev_in, float *prev_out,
                               const float *hann, int32_t N, int32_t Z, int32_t H, uint32_t gap_mask, int32_t n_det,
                               void *blk);
// N-point transform of n_det rows, ping-ponging between a and b; *result
// is the buffer holding the transform (twiddles of an N_table-point table)
hipError_t launch_fft(hipStream_t, void *a, void *b, int32_t N, int32_t N_table, int32_t inverse, const void *tw,
                      int32_t n_det, void **result);
hipError_t launch_whiten_psd(hipStream_t, const void *X, int32_t N, int32_t K, int32_t n_out, float inv_w2,
                             float *ring, int32_t n_med, float *log_geo, const WhitenDetState &s, const float *beta,
                             float d_factor, void *Y, int32_t n_det);
hipError_t launch_whiten_ola(hipStream_t, const void *y, const float *tukey, int32_t n_out, int32_t h_out,
                             uint32_t gap_mask, const float *acc_in, float *acc_out, float *out, int64_t out_ld,
                             int32_t n_det);
hipError_t launch_whiten_exp(hipStream_t, const float *lg, int64_t n, float *psd);

}  // namespace lloid
