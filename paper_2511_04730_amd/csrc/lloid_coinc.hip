// Overlapping trigger windows, coincidence across detectors and clustering
// per sub-bank (Sec. II.D.3-4).
//
// Window k covers top-rate samples [kF - O, (k+1)F): the stride's trigger
// (from the peak kernel) merged with the maximum of |z| over the last O
// samples of the previous stride's series, the earlier sample winning ties.
// One wave per template scans those O contiguous complex samples of every
// detector (template-major series: 512 contiguous bytes per load).
//
// Coincidence is per template: each detector whose window trigger reaches
// the threshold anchors a candidate holding every other such detector
// within the pair's window (in samples, inclusive); a candidate holding two
// or more detectors is an event, its network SNR^2 the sum of the held
// SNR^2 in detector order.  A template keeps its best candidate (first
// anchor on ties); each sub-bank keeps its best template (lowest on ties).
// One work group per bank; the decision quantities are summed in FP32
// without contraction, in a fixed order, so the result is reproducible
// bit for bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lloid_coinc.h"
#include "lloid_device.h"

namespace lloid {
namespace {

constexpr int kTrigWaves = 4;    // templates per work group
constexpr int kCoincThreads = 256;

__device__ __forceinline__ void max_first(float &p2, int &idx, float &re, float &im, int o) {
    const float q2 = __shfl_xor(p2, o, 64);
    const int qi = __shfl_xor(idx, o, 64);
    const float qr = __shfl_xor(re, o, 64);
    const float qm = __shfl_xor(im, o, 64);
    if (better(q2, qi, p2, idx)) {
        p2 = q2;
        idx = qi;
        re = qr;
        im = qm;
    }
}

__global__ __launch_bounds__(64 * kTrigWaves) void window_trigger_kernel(
    const TrigTemplate *__restrict__ tab, int32_t n_tmpl, int32_t n_det, int32_t F, const float *__restrict__ prev,
    const lloid_peak *__restrict__ peaks, int32_t overlap, float threshold, lloid_peak *__restrict__ triggers) {
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kTrigWaves + (threadIdx.x >> 6));
    if (i >= n_tmpl) return;
    const TrigTemplate e = tab[i];
    for (int det = 0; det < n_det; ++det) {
        const int64_t pk = e.peak_off + (int64_t)det * e.M;
        const lloid_peak cur = peaks[pk];
        if (!prev || overlap == 0) {              // first (shortened) window: the stride itself
            if (lane == 0) triggers[pk] = cur;
            continue;
        }
        // the overlap's samples: index -overlap .. -1 relative to the stride
        const float *z = prev + e.series_off + (int64_t)det * e.det_stride;
        float p2 = -1.f, re = 0.f, im = 0.f;
        int idx = 0x7fffffff;
        for (int c = lane; c < overlap; c += 64) {
            const int t = F - overlap + c;
            const float2 v = *reinterpret_cast<const float2 *>(z + 2 * (int64_t)t);
            const float q2 = v.x * v.x + v.y * v.y;
            if (better(q2, c - overlap, p2, idx)) {
                p2 = q2;
                idx = c - overlap;
                re = v.x;
                im = v.y;
            }
        }
        for (int o = 32; o >= 1; o >>= 1) max_first(p2, idx, re, im, o);
        if (lane == 0) {
            const float c2 = cur.re * cur.re + cur.im * cur.im;
            // the overlap precedes the stride: it wins ties
            if (p2 >= c2) {
                const float snr = sqrtf(p2);
                triggers[pk] = lloid_peak{snr, idx, re, im, snr >= threshold ? 1 : 0};
            } else {
                triggers[pk] = cur;
            }
        }
    }
}

#pragma clang fp contract(off)
__global__ __launch_bounds__(kCoincThreads) void coinc_kernel(const CoincBank *__restrict__ banks, int32_t n_det,
                                                             CoincWindows w, const lloid_peak *__restrict__ trig,
                                                             lloid_event *__restrict__ events) {
    __shared__ float s_s2[kCoincThreads / 64];
    __shared__ int s_m[kCoincThreads / 64];
    __shared__ uint32_t s_mask[kCoincThreads / 64];
    const CoincBank b = banks[blockIdx.x];
    float best2 = 0.f;                       // events have s2 >= 2 threshold^2 > 0
    int best_m = 0x7fffffff;
    uint32_t best_mask = 0;
    for (int m = threadIdx.x; m < b.M; m += kCoincThreads) {
        float snr[kCoincMaxDet];
        int idx[kCoincMaxDet];
        bool up[kCoincMaxDet];
#pragma unroll
        for (int d = 0; d < kCoincMaxDet; ++d) {
            up[d] = false;
            snr[d] = 0.f;
            idx[d] = 0;
            if (d < n_det) {
                const lloid_peak p = trig[b.peak_off + (int64_t)d * b.M + m];
                snr[d] = p.snr;
                idx[d] = p.index;
                up[d] = p.above != 0;
            }
        }
        float t2 = 0.f;
        uint32_t tmask = 0;
#pragma unroll
        for (int a = 0; a < kCoincMaxDet; ++a) {
            if (!up[a]) continue;
            float s2 = 0.f;
            uint32_t mask = 0;
            int held = 0;
#pragma unroll
            for (int d = 0; d < kCoincMaxDet; ++d) {
                const int dt = idx[d] - idx[a];
                if (up[d] && (d == a || (dt <= w.w[a][d] && -dt <= w.w[a][d]))) {
                    s2 = s2 + snr[d] * snr[d];
                    mask |= 1u << d;
                    ++held;
                }
            }
            if (held >= 2 && s2 > t2) {
                t2 = s2;
                tmask = mask;
            }
        }
        if (tmask && t2 > best2) {           // m increases: the lowest template keeps ties
            best2 = t2;
            best_m = m;
            best_mask = tmask;
        }
    }
    // work-group maximum, lowest template on ties
    for (int o = 32; o >= 1; o >>= 1) {
        const float q2 = __shfl_xor(best2, o, 64);
        const int qm = __shfl_xor(best_m, o, 64);
        const uint32_t qk = __shfl_xor(best_mask, o, 64);
        if (q2 > best2 || (q2 == best2 && qm < best_m)) {
            best2 = q2;
            best_m = qm;
            best_mask = qk;
        }
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_s2[wv] = best2;
        s_m[wv] = best_m;
        s_mask[wv] = best_mask;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kCoincThreads / 64; ++k) {
            if (s_s2[k] > best2 || (s_s2[k] == best2 && s_m[k] < best_m)) {
                best2 = s_s2[k];
                best_m = s_m[k];
                best_mask = s_mask[k];
            }
        }
        lloid_event ev;
        if (best_mask) {
            ev.network_snr = sqrtf(best2);
            ev.template_index = best_m;
            ev.det_mask = best_mask;
            ev.n_det = __builtin_popcount(best_mask);
        } else {
            ev.network_snr = 0.f;
            ev.template_index = -1;
            ev.det_mask = 0;
            ev.n_det = 0;
        }
        events[blockIdx.x] = ev;
    }
}
#pragma clang fp contract(on)

}  // namespace

hipError_t launch_window_triggers(hipStream_t st, const TrigTemplate *tab, int32_t n_tmpl, int32_t n_det, int32_t F,
                                  const float *prev, const lloid_peak *peaks, int32_t overlap, float threshold,
                                  lloid_peak *triggers) {
    if (n_tmpl <= 0) return hipSuccess;
    const int blocks = (n_tmpl + kTrigWaves - 1) / kTrigWaves;
    hipLaunchKernelGGL(window_trigger_kernel, dim3(blocks), dim3(64 * kTrigWaves), 0, st, tab, n_tmpl, n_det, F, prev,
                       peaks, overlap, threshold, triggers);
    return hipGetLastError();
}

hipError_t launch_coinc(hipStream_t st, const CoincBank *banks, int32_t n_banks, int32_t n_det, const CoincWindows &w,
                        const lloid_peak *triggers, lloid_event *events) {
    if (n_banks <= 0) return hipSuccess;
    hipLaunchKernelGGL(coinc_kernel, dim3(n_banks), dim3(kCoincThreads), 0, st, banks, n_det, w, triggers, events);
    return hipGetLastError();
}

}  // namespace lloid
