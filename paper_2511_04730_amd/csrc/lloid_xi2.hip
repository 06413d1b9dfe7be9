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
// load), detectors in turn (the autocorrelation row is re-read from L1/L2).
// The work is HBM-bound: A complex samples per trigger plus A per template.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_xi2.h"

namespace lloid {
namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kXiWaves = 4;   // templates per work group

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64 * kXiWaves) void xi2_kernel(const XiTemplate *__restrict__ tab, int32_t n_tmpl,
                                                           int32_t n_det, int32_t F, const float *prev,
                                                           const float *cur, const float *next,
                                                           const lloid_peak *__restrict__ peaks,
                                                           const float *__restrict__ acf, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kXiWaves + (threadIdx.x >> 6));
    if (i >= n_tmpl) return;
    const XiTemplate e = tab[i];
    const int A = e.A, delta = (A - 1) >> 1;
    const f32x2 *R = reinterpret_cast<const f32x2 *>(acf + e.acf_off);
    for (int det = 0; det < n_det; ++det) {
        const int64_t row = e.series_off + (int64_t)det * e.det_stride;   // float offset of z[0]
        const int64_t pk = e.peak_off + (int64_t)det * e.M;
        const int tp = __builtin_amdgcn_readfirstlane(peaks[pk].index);
        if (tp < 0 || tp >= F) {              // not a trigger of this stride
            if (lane == 0) out[pk] = __builtin_nanf("");
            continue;
        }
        const f32x2 z0 = ld_global<f32x2>(cur + row + 2 * (int64_t)tp);
        float num = 0.f, den = 0.f;
#pragma unroll 4
        for (int t = lane; t < A; t += 64) {
            const int s = tp - delta + t;     // in [-F, 2F) since delta <= F
            const float *src = s < 0 ? prev : (s >= F ? next : cur);
            const int sl = s < 0 ? s + F : (s >= F ? s - F : s);
            if (src) {
                const f32x2 r = ld_global<f32x2>(R + t);
                const f32x2 z = ld_global<f32x2>(src + row + 2 * (int64_t)sl);
                const float dre = z.x - (z0.x * r.x - z0.y * r.y);
                const float dim = z.y - (z0.x * r.y + z0.y * r.x);
                num += dre * dre + dim * dim;
                den += 2.f - 2.f * (r.x * r.x + r.y * r.y);
            }
        }
        num = wave_sum(num);
        den = wave_sum(den);
        if (lane == 0) out[pk] = num / den;
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
    hipLaunchKernelGGL(xi2_kernel, dim3(blocks), dim3(64 * kXiWaves), 0, st, tab, n_tmpl, n_det, F, prev, cur, next,
                       peaks, acf, out);
    return hipGetLastError();
}

hipError_t launch_convert_f64_f32(hipStream_t st, const double *src, int64_t n, float *dst) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(convert_f64_f32, dim3((unsigned)blocks), dim3(256), 0, st, src, n, dst);
    return hipGetLastError();
}

}  // namespace lloid
