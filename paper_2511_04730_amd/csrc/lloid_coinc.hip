// Overlapping trigger windows, coincidence across detectors and clustering
// per sub-bank (Sec. II.D.3-4).
//
// Window k covers top-rate samples [kF - O, (k+1)F): the stride's trigger
// (from the peak kernel) merged with the maximum of |z| over the last O
// samples of the previous stride's series, the earlier sample winning ties.
// One wave per template scans those O contiguous complex samples of up to
// four detectors at once (template-major series: 512 contiguous bytes per
// load).
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

typedef float f32x2 __attribute__((ext_vector_type(2)));
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

// Detectors d0 .. d0 + ND - 1 of every template: the overlap loads of all
// of them for four 64-sample chunks are issued before the first is used
// (lanes past the overlap re-read its last sample and are masked out of the
// maximum; the running maximum is updated with selects, not branches, so
// no branch holds a load's wait inside its iteration).
template <int ND>
__global__ __launch_bounds__(64 * kTrigWaves) void window_trigger_kernel(
    const TrigTemplate *__restrict__ tab, int32_t n_tmpl, int32_t d0, int32_t F, const float *__restrict__ prev,
    const lloid_peak *__restrict__ peaks, int32_t overlap, float threshold, lloid_peak *__restrict__ triggers) {
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kTrigWaves + (threadIdx.x >> 6));
    if (i >= n_tmpl) return;
    const TrigTemplate e = tab[i];
    if (!prev || overlap == 0) {                  // first (shortened) window: the stride itself
        if (lane < ND) {
            const int64_t pk = e.peak_off + (int64_t)(d0 + lane) * e.M;
            triggers[pk] = peaks[pk];
        }
        return;
    }
    // lane j < ND reads detector j's stride trigger now, so that its load
    // overlaps the overlap's loads
    const int64_t pk = e.peak_off + (int64_t)(d0 + (lane < ND ? lane : 0)) * e.M;
    const lloid_peak cur = peaks[pk];
    float p2[ND], re[ND], im[ND];
    int idx[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        p2[j] = -1.f;
        re[j] = im[j] = 0.f;
        idx[j] = 0x7fffffff;
    }
    // the overlap's samples: index -overlap .. -1 relative to the stride
    // groups of four 64-sample chunks, every load in flight at once (chunks
    // past the overlap re-read its last sample, masked)
    for (int c0 = 0; c0 < overlap; c0 += 4 * 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = c0 + u * 64 + lane;
            const bool in = k < overlap;
            const int t = F - overlap + (in ? k : overlap - 1);
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                const float *z = prev + e.series_off + (int64_t)(d0 + j) * e.det_stride;
                const f32x2 v = ld_global<f32x2>(z + 2 * (int64_t)t);
                const float q2 = in ? v.x * v.x + v.y * v.y : -2.f;   // below the initial -1: never taken
                const bool take = (q2 > p2[j]) | ((q2 == p2[j]) & (k - overlap < idx[j]));
                p2[j] = take ? q2 : p2[j];
                idx[j] = take ? k - overlap : idx[j];
                re[j] = take ? v.x : re[j];
                im[j] = take ? v.y : im[j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        for (int o = 32; o >= 1; o >>= 1) max_first(p2[j], idx[j], re[j], im[j], o);
    }
    if (lane < ND) {
        // lane j finishes detector j (the values are wave-uniform after the reduction)
        float bp2 = p2[0], bre = re[0], bim = im[0];
        int bidx = idx[0];
#pragma unroll
        for (int j = 1; j < ND; ++j) {
            if (lane == j) {
                bp2 = p2[j];
                bre = re[j];
                bim = im[j];
                bidx = idx[j];
            }
        }
        const float c2 = cur.re * cur.re + cur.im * cur.im;
        if (bp2 >= c2) {                          // the overlap precedes the stride: it wins ties
            const float snr = sqrtf(bp2);
            triggers[pk] = lloid_peak{snr, bidx, bre, bim, snr >= threshold ? 1 : 0};
        } else {
            triggers[pk] = cur;
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
    const dim3 grid((n_tmpl + kTrigWaves - 1) / kTrigWaves), block(64 * kTrigWaves);
    for (int d0 = 0; d0 < n_det; d0 += 4) {
        switch (n_det - d0 < 4 ? n_det - d0 : 4) {
            case 1: hipLaunchKernelGGL(window_trigger_kernel<1>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, peaks, overlap, threshold, triggers); break;
            case 2: hipLaunchKernelGGL(window_trigger_kernel<2>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, peaks, overlap, threshold, triggers); break;
            case 3: hipLaunchKernelGGL(window_trigger_kernel<3>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, peaks, overlap, threshold, triggers); break;
            default: hipLaunchKernelGGL(window_trigger_kernel<4>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, peaks, overlap, threshold, triggers); break;
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_coinc(hipStream_t st, const CoincBank *banks, int32_t n_banks, int32_t n_det, const CoincWindows &w,
                        const lloid_peak *triggers, lloid_event *events) {
    if (n_banks <= 0) return hipSuccess;
    hipLaunchKernelGGL(coinc_kernel, dim3(n_banks), dim3(kCoincThreads), 0, st, banks, n_det, w, triggers, events);
    return hipGetLastError();
}

}  // namespace lloid
