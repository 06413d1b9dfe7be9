// Signal-consistency statistic xi^2 at the triggers (Sec. II.D.2):
//
//   xi^2 = sum_t |z(t_p + t) - z(t_p) R(t)|^2 / sum_t (2 - 2 |R(t)|^2),
//   t = -delta..delta, delta = (A - 1) / 2,
//
// z the complex SNR series of one template and detector, t_p its trigger
// index in the stride, R the template's autocorrelation (R(0) = 1).  The
// sums run over top-rate samples; samples in a neighbouring stride that is
// not given are left out of both.
//
// The series are template-major ([n_det][M][F] complex per bank), so one
// template's window is contiguous: one wave per template, lanes over the
// window's samples (64 consecutive complex values = 512 contiguous bytes per
// load), up to four detectors per launch so that each autocorrelation value
// is loaded once for all of them.
// The work is HBM-bound: A complex samples per trigger plus A per template.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_xi2.h"

namespace lloid {
namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kXiWaves = 4;   // templates per work group
constexpr int kXiDets = 4;    // detectors per launch over a template's window

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Detectors d0 .. d0 + ND - 1 of every template: each autocorrelation value
// is loaded once for all ND of them.  The loop body is branch-free (every
// load has a valid address; samples of a missing neighbour stride are read
// from the current one and weighted by zero), so the compiler can keep
// several iterations' loads in flight.
template <int ND>
__global__ __launch_bounds__(64 * kXiWaves) void xi2_kernel(const XiTemplate *__restrict__ tab, int32_t n_tmpl,
                                                           int32_t d0, int32_t F, const float *prev,
                                                           const float *cur, const float *next,
                                                           const lloid_peak *__restrict__ peaks,
                                                           const float *__restrict__ acf, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kXiWaves + (threadIdx.x >> 6));
    if (i >= n_tmpl) return;
    const XiTemplate e = tab[i];
    const int A = e.A, delta = (A - 1) >> 1;
    const f32x2 *R = reinterpret_cast<const f32x2 *>(acf + e.acf_off);
    // byte offsets of the neighbouring strides' series from the current one
    // (0 when absent: such samples are read from the current stride, unused)
    const bool hp = prev != nullptr, hn = next != nullptr;
    const int64_t dprev = hp ? (int64_t)((intptr_t)prev - (intptr_t)cur) : 0;
    const int64_t dnext = hn ? (int64_t)((intptr_t)next - (intptr_t)cur) : 0;
    int tp[ND];
    bool ok[ND];
    const char *zrow[ND];
    f32x2 z0[ND];
    float num[ND], den[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const int64_t row = e.series_off + (int64_t)(d0 + j) * e.det_stride;   // float offset of z[0]
        const int t = __builtin_amdgcn_readfirstlane(peaks[e.peak_off + (int64_t)(d0 + j) * e.M].index);
        // a trigger of this stride, or of its window's overlap into the previous one
        ok[j] = (t >= 0 && t < F) || (hp && t >= -F && t < 0);
        tp[j] = ok[j] ? t : 0;
        zrow[j] = reinterpret_cast<const char *>(cur + row);
        z0[j] = tp[j] < 0 ? ld_global<f32x2>(prev + row + 2 * (int64_t)(tp[j] + F))
                          : ld_global<f32x2>(cur + row + 2 * (int64_t)tp[j]);
        num[j] = den[j] = 0.f;
    }
    // a uniform trip count (lanes past the window re-read its last sample and
    // add nothing), so that no branch separates the iterations' loads
    const int n_chunks = (A + 63) >> 6;
#pragma unroll 4
    for (int c = 0; c < n_chunks; ++c) {
        const bool in = c * 64 + lane < A;
        const int t = in ? c * 64 + lane : A - 1;
        const f32x2 r = ld_global<f32x2>(R + t);
        const float w = 2.f - 2.f * (r.x * r.x + r.y * r.y);
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const int s = tp[j] - delta + t;  // in [-2F, 2F) since delta <= F and tp >= -F
            const bool lo2 = s < -F;          // before the previous stride: never available
            const bool lo = s < 0, hi = s >= F;
            const int sl = lo2 ? 0 : (lo ? s + F : (hi ? s - F : s));
            const int64_t off = (int64_t)sl * 8 + (lo ? dprev : (hi ? dnext : 0));
            const f32x2 z = ld_global<f32x2>(zrow[j] + off);
            // 1 or 0 as a factor, not a select: a select would let the
            // compiler move the load under a branch (one wait per sample)
            const float use = (in && !lo2 && (!lo || hp) && (!hi || hn)) ? 1.f : 0.f;
            const float dre = z.x - (z0[j].x * r.x - z0[j].y * r.y);
            const float dim = z.y - (z0[j].x * r.y + z0[j].y * r.x);
            num[j] += use * (dre * dre + dim * dim);
            den[j] += use * w;
        }
    }
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        const float a = wave_sum(num[j]), b = wave_sum(den[j]);
        if (lane == 0) out[e.peak_off + (int64_t)(d0 + j) * e.M] = ok[j] ? a / b : __builtin_nanf("");
    }
}

__global__ void convert_f64_f32(const double *__restrict__ src, int64_t n, float *__restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = (float)src[k];
}

}  // namespace

hipError_t launch_xi2(hipStream_t st, const XiTemplate *tab, int32_t n_tmpl, int32_t n_det, int32_t F,
                      const float *prev, const float *cur, const float *next, const lloid_peak *peaks,
                      const float *acf, float *out) {
    if (n_tmpl <= 0) return hipSuccess;
    const int blocks = (n_tmpl + kXiWaves - 1) / kXiWaves;
    const dim3 grid(blocks), block(64 * kXiWaves);
    for (int d0 = 0; d0 < n_det; d0 += kXiDets) {
        switch (std::min(kXiDets, n_det - d0)) {
            case 1: hipLaunchKernelGGL(xi2_kernel<1>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, cur, next, peaks, acf, out); break;
            case 2: hipLaunchKernelGGL(xi2_kernel<2>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, cur, next, peaks, acf, out); break;
            case 3: hipLaunchKernelGGL(xi2_kernel<3>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, cur, next, peaks, acf, out); break;
            default: hipLaunchKernelGGL(xi2_kernel<4>, grid, block, 0, st, tab, n_tmpl, d0, F, prev, cur, next, peaks, acf, out); break;
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_convert_f64_f32(hipStream_t st, const double *src, int64_t n, float *dst) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(convert_f64_f32, dim3((unsigned)blocks), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}

}  // namespace lloid
