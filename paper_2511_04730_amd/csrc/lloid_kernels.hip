// Device kernels of the LLOID filtering core for gfx950 (CDNA4).
//
// One stride runs six kernels, all over precomputed work tables:
//   ingest    strain stride -> top-rate history ring (gaps become zeros)
//   down      decimation to every slice rate, Eq. (sinc) kernel, zero phase
//   corr      per-slice basis correlation, a Hankel(strain) x basis
//             contraction on MFMA with LDS-staged tiles, split over taps
//             (lloid_corr.hip)
//   reduce    fixed-order sum of the tap splits into the basis-output ring
//   mix       mixing-matrix contraction on MFMA fused with the polyphase
//             upsample-and-add chain (lowest rate first), the SNR series
//             write and per-tile peak candidates (lloid_mix.hip)
//   peaks     fixed-order reduction of the candidates, one trigger per
//             template (Sec. II.D.1)
// Every output element has exactly one owner and every sum has a fixed
// order, so repeated runs are bit-identical.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {


// ------------------------------------------------------------------ ingest
__global__ void ingest_kernel(const float *__restrict__ strain, int64_t src_det_stride, uint32_t gap_mask,
                              float *__restrict__ xring, int64_t det_stride, int32_t cap, int32_t F,
                              const int64_t *__restrict__ stride_ctr) {
    const int det = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F) return;
    const int64_t k = *stride_ctr;
    const float v = ((gap_mask >> det) & 1u) ? 0.0f : strain[(int64_t)det * src_det_stride + i];
    const int64_t pos = posmod(k * F + i, cap);
    float *r = xring + det * det_stride;
    r[pos] = v;
    r[pos + cap] = v;
}

hipError_t launch_ingest(const LaunchCtx &ctx, const float *strain, int64_t src_det_stride, uint32_t gap_mask,
                         float *xring, int64_t ring_det_stride, int32_t cap, int32_t F, int32_t n_det) {
    dim3 grid((F + 255) / 256, n_det);
    hipLaunchKernelGGL(ingest_kernel, grid, dim3(256), 0, ctx.stream, strain, src_det_stride, gap_mask, xring,
                       ring_det_stride, cap, F, ctx.stride_ctr);
    return hipGetLastError();
}

// -------------------------------------------------------------- decimation
// d_D[m] = sum_{t=0}^{2c} g[t] x[D m + t - c] for the chunk of outputs
// m = k f - n_down + m0 + i, i < chunk (these are the f outputs of stride k
// that the strain received so far fully determines).  The strain segment is
// staged in LDS with one pad word per 32 so that lanes reading with stride D
// fall in distinct banks.
__device__ __forceinline__ int lds_pad(int a) { return a + (a >> 5); }

__global__ __launch_bounds__(256) void down_kernel(const DownItem *__restrict__ items,
                                                   const int64_t *__restrict__ stride_ctr) {
    extern __shared__ float sm[];
    const DownItem it = items[blockIdx.x];
    const int64_t k = *stride_ctr;
    const int ntap = 2 * it.c + 1;
    float *taps = sm;
    float *xs = sm + ntap;
    const int64_t m_first = k * it.f - it.n_down + it.m0;
    const int64_t x_first = m_first * it.D - it.c;
    const int seg = (it.chunk - 1) * it.D + ntap;
    const int64_t base = posmod(x_first, it.capx);
    for (int t = threadIdx.x; t < ntap; t += blockDim.x) taps[t] = it.taps[t];
    for (int t = threadIdx.x; t < seg; t += blockDim.x) xs[lds_pad(t)] = it.xring[base + t];
    __syncthreads();
    // T = blockDim / chunk threads share an output (T = 4 for 64 outputs),
    // thread part p < T summing the taps p, p + T, ...; the parts are added
    // in order, so the result does not depend on scheduling
    const int T = blockDim.x / it.chunk;
    const int o = threadIdx.x % it.chunk, part = threadIdx.x / it.chunk;
    float acc = 0.0f;
    const int b = o * it.D;
    if (T == 1) {
        for (int t = 0; t < ntap; ++t) acc = fmaf(taps[t], xs[lds_pad(b + t)], acc);
    } else if (part < T) {
        for (int t = part; t < ntap; t += T) acc = fmaf(taps[t], xs[lds_pad(b + t)], acc);
    }
    float *red = xs + lds_pad(seg);   // blockDim floats past the staged segment
    if (T > 1) {
        __syncthreads();
        red[threadIdx.x] = acc;
        __syncthreads();
        if (part == 0)
            for (int q = 1; q < T; ++q) acc += red[q * it.chunk + o];
    }
    if (part == 0) {
        const int64_t pos = posmod(m_first + o, it.capd);
        it.dring[pos] = acc;
        it.dring[pos + it.capd] = acc;
    }
}

hipError_t launch_down(const LaunchCtx &ctx, const DownItem *items, int32_t n_items, int32_t max_lds_floats) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(down_kernel, dim3(n_items), dim3(256), (size_t)max_lds_floats * sizeof(float), ctx.stream,
                       items, ctx.stride_ctr);
    return hipGetLastError();
}

// Sum the split partials of 64 new columns x 32 basis rows in a fixed
// order (split 0 first), transpose through LDS and append them to the
// basis-output ring (16-byte groups of consecutive outputs per sample,
// outputs L .. Lpad-1 zero).  16-bit forms store y as hi = T(y) and
// lo = T(y - hi) in two planes.
template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceItem *__restrict__ items,
                                                     const int64_t *__restrict__ stride_ctr) {
    __shared__ float sm[32][65];
    const ReduceItem it = items[blockIdx.x];
    const int64_t k = *stride_ctr;
    const int ncols = min(64, it.f - it.c0);
    const int64_t plane = (int64_t)it.Lpad * it.f;
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
        const int l = e >> 6, c = e & 63;
        float s = 0.0f;
        if (c < ncols && it.l0 + l < it.L) {
            const float *p = it.part + (int64_t)(it.l0 + l) * it.f + it.c0 + c;
            for (int sp = 0; sp < it.nsplit; ++sp) s += p[sp * plane];
        }
        sm[l][c] = s;
    }
    __syncthreads();
    const int64_t q0 = k * it.f + it.la + it.c0;
    const int64_t mask = it.capY - 1;
    constexpr int V = sizeof(T) == 4 ? 4 : 8;   // outputs per thread and row: 16 bytes
    const int nrow = min(32, it.Lpad - it.l0);
    const int groups = nrow / V;
    // consecutive threads write consecutive positions of one 16-byte group
    for (int e = threadIdx.x; e < ncols * groups; e += 256) {
        const int c = e % ncols, l = (e / ncols) * V;
        const int64_t pos = (q0 + c) & mask;
        const int64_t o = ring_index<V>(pos, it.l0 + l, it.capY);
        const int64_t om = ring_index<V>(pos + it.capY, it.l0 + l, it.capY);
        if constexpr (sizeof(T) == 4) {
            const float4 v = make_float4(sm[l][c], sm[l + 1][c], sm[l + 2][c], sm[l + 3][c]);
            float *ring = static_cast<float *>(it.yring);
            *reinterpret_cast<float4 *>(ring + o) = v;
            *reinterpret_cast<float4 *>(ring + om) = v;
        } else {
            typedef T T8 __attribute__((ext_vector_type(8)));
            T8 h, lo;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float y = sm[l + i][c];
                h[i] = (T)y;
                lo[i] = (T)(y - (float)h[i]);
            }
            T *hi_plane = static_cast<T *>(it.yring);
            T *lo_plane = hi_plane + 2LL * it.capY * it.Lpad;
            *reinterpret_cast<T8 *>(hi_plane + o) = h;
            *reinterpret_cast<T8 *>(hi_plane + om) = h;
            *reinterpret_cast<T8 *>(lo_plane + o) = lo;
            *reinterpret_cast<T8 *>(lo_plane + om) = lo;
        }
    }
}

hipError_t launch_reduce(const LaunchCtx &ctx, int precision, const ReduceItem *items, int32_t n_items) {
    if (n_items == 0) return hipSuccess;
    switch (precision) {
        case LLOID_FP32:
            hipLaunchKernelGGL(reduce_kernel<float>, dim3(n_items), dim3(256), 0, ctx.stream, items, ctx.stride_ctr);
            break;
        case LLOID_BF16X3:
        case LLOID_FP8_BF16:
            hipLaunchKernelGGL(reduce_kernel<__bf16>, dim3(n_items), dim3(256), 0, ctx.stream, items,
                               ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL(reduce_kernel<_Float16>, dim3(n_items), dim3(256), 0, ctx.stream, items,
                               ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
__global__ void ring_gather_kernel(const void *__restrict__ ring, int32_t Lpad, int32_t cap, int64_t a, int32_t len,
                                   int32_t rows, float *__restrict__ dst, int64_t dst_ld, int64_t dst_off) {
    const int r = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows || c >= len) return;
    const int64_t p = posmod(a, cap) + c;   // mirror ring: p < 2 cap
    float v;
    const int64_t o = ring_index<16 / sizeof(T)>(p, r, cap);
    if constexpr (sizeof(T) == 4) {
        v = static_cast<const float *>(ring)[o];
    } else {
        const T *hi = static_cast<const T *>(ring);
        v = (float)hi[o] + (float)hi[2LL * cap * Lpad + o];
    }
    dst[r * dst_ld + dst_off + c] = v;
}

hipError_t launch_ring_gather(hipStream_t st, int precision, const void *ring, int32_t Lpad, int32_t cap, int64_t a,
                              int32_t len, int32_t rows, float *dst, int64_t dst_ld, int64_t dst_off) {
    if (len <= 0 || rows <= 0) return hipSuccess;
    const dim3 grid((len + 255) / 256, rows);
    switch (precision) {
        case LLOID_FP32:
            hipLaunchKernelGGL(ring_gather_kernel<float>, grid, dim3(256), 0, st, ring, Lpad, cap, a, len, rows, dst,
                               dst_ld, dst_off);
            break;
        case LLOID_BF16X3:
        case LLOID_FP8_BF16:
            hipLaunchKernelGGL(ring_gather_kernel<__bf16>, grid, dim3(256), 0, st, ring, Lpad, cap, a, len, rows, dst,
                               dst_ld, dst_off);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL(ring_gather_kernel<_Float16>, grid, dim3(256), 0, st, ring, Lpad, cap, a, len, rows,
                               dst, dst_ld, dst_off);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t configure_down_lds(size_t down_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(down_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)down_bytes);
}

// ----------------------------------------------------------------- peaks
__global__ __launch_bounds__(256) void peaks_kernel(const PeakItem *__restrict__ items,
                                                    const PartialPeak *__restrict__ partials,
                                                    lloid_peak *__restrict__ peaks, float threshold,
                                                    int64_t *__restrict__ stride_ctr) {
    const PeakItem it = items[blockIdx.x];
    for (int i = threadIdx.x; i < it.M; i += blockDim.x) {
        const PartialPeak *p = partials + it.part_off + (int64_t)i * it.n_ttiles;
        PartialPeak b = p[0];
        for (int t = 1; t < it.n_ttiles; ++t) {
            const PartialPeak o = p[t];
            if (better(o.p2, o.idx, b.p2, b.idx)) b = o;
        }
        const float snr = sqrtf(b.p2);
        peaks[it.peak_off + i] = lloid_peak{snr, b.idx, b.re, b.im, snr >= threshold ? 1 : 0};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && stride_ctr) {
        // every kernel of this stride has read the counter; advance it
        stride_ctr[0] += 1;
    }
}

hipError_t launch_peaks(const LaunchCtx &ctx, const PeakItem *items, int32_t n_items, const PartialPeak *partials,
                        lloid_peak *peaks, float threshold, int64_t *stride_ctr_advance) {
    hipLaunchKernelGGL(peaks_kernel, dim3(n_items > 0 ? n_items : 1), dim3(256), 0, ctx.stream, items, partials,
                       peaks, threshold, stride_ctr_advance);
    return hipGetLastError();
}

// --------------------------------------------------- plan-time conversion
// Per real row r: inv[r] = 1 / sqrt(sum_s sum_l W^s[r,l]^2) in FP64 (or 1).
// One wave per row: the lanes stride over the row's basis coefficients of
// every slice (consecutive lanes read consecutive doubles), then a fixed
// butterfly sums the 64 partial sums.
__global__ void normalize_kernel(const double *const *__restrict__ W64, const int32_t *__restrict__ Ls,
                                 int32_t n_slices, int32_t rows, int32_t normalize, double *__restrict__ inv) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;   // wave-uniform
    double s = 0.0;
    for (int i = 0; i < n_slices; ++i) {
        const double *w = W64[i] + (int64_t)r * Ls[i];
        for (int l = lane; l < Ls[i]; l += 64) s = fma(w[l], w[l], s);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) inv[r] = (normalize && s > 0.0) ? 1.0 / sqrt(s) : 1.0;
}

hipError_t launch_normalize(hipStream_t st, const double *const *W64, const int32_t *Ls, int32_t n_slices,
                            int32_t rows, int32_t normalize, double *inv_norm) {
    hipLaunchKernelGGL(normalize_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, W64, Ls, n_slices, rows,
                       normalize, inv_norm);
    return hipGetLastError();
}

// v = src * row_scale -> hi = T(v) (round to nearest even), lo = T(v - hi)
// with the residual formed in FP64 (lo is skipped when dst_lo is NULL).
// The destination is row-major [rows][dst_ld] or, for frag != 0, the mixing
// kernel's fragment order over a [rows_pad][dst_ld] matrix (the caller's
// buffer holds the padding, zero-filled).
template <typename T>
__global__ void convert_split_kernel(const double *__restrict__ src, int32_t rows, int32_t cols, int32_t src_ld,
                                     const double *__restrict__ row_scale, T *__restrict__ hi, T *__restrict__ lo,
                                     int32_t dst_ld, int32_t frag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const double v = src[(int64_t)r * src_ld + c] * (row_scale ? row_scale[r] : 1.0);
    const int64_t o = frag ? frag_index<8>(r, c, dst_ld) : (int64_t)r * dst_ld + c;
    const T h = (T)(float)v;
    hi[o] = h;
    if (lo) lo[o] = (T)(float)(v - (double)(float)h);
}

hipError_t launch_convert_reduced(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                                  const double *row_scale, int precision, int role, void *dst_hi, void *dst_lo,
                                  int32_t dst_ld, float *row_scale_out) {
    (void)row_scale_out;
    const int32_t frag = role == ROLE_MIXING;
    const int64_t n = (int64_t)rows * cols;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (precision == LLOID_BF16X3 || precision == LLOID_FP8_BF16) {
        hipLaunchKernelGGL(convert_split_kernel<__bf16>, grid, dim3(256), 0, st, src, rows, cols, src_ld, row_scale,
                           static_cast<__bf16 *>(dst_hi), static_cast<__bf16 *>(dst_lo), dst_ld, frag);
    } else if (precision == LLOID_FP16) {
        hipLaunchKernelGGL(convert_split_kernel<_Float16>, grid, dim3(256), 0, st, src, rows, cols, src_ld,
                           row_scale, static_cast<_Float16 *>(dst_hi), static_cast<_Float16 *>(dst_lo), dst_ld, frag);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

__global__ void convert_f32_kernel(const double *__restrict__ src, int32_t rows, int32_t cols, int32_t src_ld,
                                   const double *__restrict__ row_scale, float *__restrict__ dst, int32_t dst_ld,
                                   int32_t frag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const double v = src[(int64_t)r * src_ld + c] * (row_scale ? row_scale[r] : 1.0);
    dst[frag ? frag_index<4>(r, c, dst_ld) : (int64_t)r * dst_ld + c] = (float)v;
}

hipError_t launch_convert_rows(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                               const double *row_scale, int precision, int role, float *dst32, void *dst_hi,
                               void *dst_lo, int32_t dst_ld, float *row_scale_out) {
    const int64_t n = (int64_t)rows * cols;
    if (n == 0) return hipSuccess;
    if (dst32) {
        hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, rows,
                           cols, src_ld, row_scale, dst32, dst_ld, (int32_t)(role == ROLE_MIXING));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (dst_hi)
        return launch_convert_reduced(st, src, rows, cols, src_ld, row_scale, precision, role, dst_hi, dst_lo,
                                      dst_ld, row_scale_out);
    return hipSuccess;
}

}  // namespace lloid
