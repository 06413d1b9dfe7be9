// Kernels of the gradient of the SNR-reconstruction loss and of the FP64
// re-orthonormalisation of refined bases.
//
//   L = sum_{r,t} (rho[r,t] - target[r,t])^2,  R = rho - target
//   dL/dW^s = 2 G^s Y^s^T,   dL/dY^s = 2 W^s^T G^s,
//   dL/dU^s[l,n] = sum_q dL/dY^s[l,q] d^s[q - delay - (N-1) + n]
// with G^s the residual taken down to the slice's rate by the transposed
// upsampling stages.  The transposed zero-phase polyphase stage is a
// decimating correlation with the same sub-kernels:
//   G_{j+1}[m] = sum_{q=m-N_up}^{m+N_up} sum_{ph<p} G_j[p q + ph] z_ph[q + N_up - m]
// (phase 0: weight 1 at q = m, the copy case of Eq. (upsample)).
#include <hip/hip_runtime.h>

#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

// ---------------------------------------------------------------- capture
// dst[r * dst_ld + dst_off + c] = ring[r * ring_ld + ((a + c) mod cap)], c < len
__global__ void copy_window_kernel(const float *__restrict__ ring, int64_t ring_ld, int32_t cap, int64_t a,
                                   int32_t len, int32_t rows, float *__restrict__ dst, int64_t dst_ld,
                                   int64_t dst_off) {
    const int r = blockIdx.y;
    if (r >= rows) return;
    int64_t p = a % cap;
    if (p < 0) p += cap;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < len; c += gridDim.x * blockDim.x)
        dst[r * dst_ld + dst_off + c] = ring[r * ring_ld + p + c];   // mirror ring: p + c < 2 cap
}

hipError_t launch_copy_window(hipStream_t st, const float *ring, int64_t ring_ld, int32_t cap, int64_t a,
                              int32_t len, int32_t rows, float *dst, int64_t dst_ld, int64_t dst_off) {
    if (len <= 0 || rows <= 0) return hipSuccess;
    dim3 grid((unsigned)std::min<int64_t>((len + 255) / 256, 64), rows);
    hipLaunchKernelGGL(copy_window_kernel, grid, dim3(256), 0, st, ring, ring_ld, cap, a, len, rows, dst, dst_ld,
                       dst_off);
    return hipGetLastError();
}

// R[(2i + c) * ld + t0 + t] = series[((det M + i) F + t) 2 + c] - target[same], and
// per-block partial sums of R^2 (FP64) into loss_part[blockIdx]
__global__ __launch_bounds__(256) void residual_kernel(const float *__restrict__ series,
                                                       const float *__restrict__ target, int32_t M, int32_t F,
                                                       float *__restrict__ R, int64_t ld, int64_t t0,
                                                       double *__restrict__ loss_part) {
    __shared__ double red[256];
    const int64_t n = (int64_t)M * F;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / F, t = e % F;
        const float2 s = reinterpret_cast<const float2 *>(series)[e];
        const float2 g = reinterpret_cast<const float2 *>(target)[e];
        const float re = s.x - g.x, im = s.y - g.y;
        R[(2 * i) * ld + t0 + t] = re;
        R[(2 * i + 1) * ld + t0 + t] = im;
        acc += (double)re * re + (double)im * im;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

hipError_t launch_residual(hipStream_t st, const float *series, const float *target, int32_t M, int32_t F, float *R,
                           int64_t ld, int64_t t0, double *loss_part, int32_t blocks) {
    hipLaunchKernelGGL(residual_kernel, dim3(blocks), dim3(256), 0, st, series, target, M, F, R, ld, t0, loss_part);
    return hipGetLastError();
}

__global__ void sum_f64_kernel(const double *__restrict__ part, int32_t n, double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_sum_f64(hipStream_t st, const double *part, int32_t n, double *out) {
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, st, part, n, out);
    return hipGetLastError();
}

// ------------------------------------------------- transposed upsampling
// g: [rows][ng] at level indices g_lo + i; out: [rows][na] at a_lo + m
__global__ void upsample_adjoint_kernel(const float *__restrict__ g, int64_t g_ld, int64_t g_lo, int64_t ng,
                                        float *__restrict__ out, int64_t o_ld, int64_t a_lo, int64_t na, int32_t p,
                                        int32_t nup, const float *__restrict__ taps) {
    const int r = blockIdx.y;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < na; m += (int64_t)gridDim.x * blockDim.x) {
        const int64_t am = a_lo + m;
        float acc = 0.0f;
        for (int64_t q = am - nup; q <= am + nup; ++q) {
            const int t = (int)(q + nup - am);
            for (int ph = 0; ph < p; ++ph) {
                const int64_t i = p * q + ph - g_lo;
                if (i < 0 || i >= ng) continue;
                const float w = ph == 0 ? (t == nup ? 1.0f : 0.0f) : taps[ph * kUpTaps + t];
                acc = fmaf(g[r * g_ld + i], w, acc);
            }
        }
        out[r * o_ld + m] = acc;
    }
}

hipError_t launch_upsample_adjoint(hipStream_t st, const float *g, int64_t g_ld, int64_t g_lo, int64_t ng,
                                   float *out, int64_t o_ld, int64_t a_lo, int64_t na, int32_t rows, int32_t p,
                                   int32_t nup, const float *taps) {
    dim3 grid((unsigned)std::min<int64_t>((na + 255) / 256, 1024), rows);
    hipLaunchKernelGGL(upsample_adjoint_kernel, grid, dim3(256), 0, st, g, g_ld, g_lo, ng, out, o_ld, a_lo, na, p,
                       nup, taps);
    return hipGetLastError();
}

// ------------------------------------------------------- strided GEMM
// part[split][m][n] = sum_{k in split} A(m,k) B(k,n),
// A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn]; 64 x 64 tiles, four
// waves of 16 columns x 64 rows on v_mfma_f32_16x16x4_f32, 32-deep K stages
// in LDS.  Out-of-range rows/columns/K read as zero.
constexpr int kGT = 64, kGK = 32;
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float *__restrict__ A, int64_t sam, int64_t sak,
                                                       const float *__restrict__ B, int64_t sbk, int64_t sbn,
                                                       int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                                       float *__restrict__ part) {
    __shared__ float As[kGT][kGK + 2];
    __shared__ float Bs[kGK][kGT + 2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
    const int64_t k_begin = (int64_t)blockIdx.z * ksplit;
    const int64_t k_end = std::min<int64_t>(K, k_begin + ksplit);
    floatx4 acc[4] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f},
                      floatx4{0.f, 0.f, 0.f, 0.f}};
    const bool a_kfast = sak == 1, b_nfast = sbn == 1;
    for (int64_t kk = k_begin; kk < k_end; kk += kGK) {
        __syncthreads();
        for (int e = tid; e < kGT * kGK; e += 256) {
            int mm, k;
            if (a_kfast) { mm = e / kGK; k = e % kGK; } else { k = e / kGT; mm = e % kGT; }
            const int64_t gm = m0 + mm, gk = kk + k;
            As[mm][k] = (gm < M && gk < k_end) ? A[gm * sam + gk * sak] : 0.0f;
            int nn, k2;
            if (b_nfast) { k2 = e / kGT; nn = e % kGT; } else { nn = e / kGK; k2 = e % kGK; }
            const int64_t gn = n0 + nn, gk2 = kk + k2;
            Bs[k2][nn] = (gn < N && gk2 < k_end) ? B[gk2 * sbk + gn * sbn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            const float b = Bs[ks + lk][wave * 16 + li];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma_16x16x4_f32(As[mb * 16 + li][ks + lk], b, acc[mb]);
        }
    }
    const int64_t n = n0 + wave * 16 + li;
    if (n < N) {
        float *o = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + mb * 16 + lk * 4 + v;
                if (m < M) o[m * N + n] = acc[mb][v];
            }
    }
}

hipError_t launch_gemm_f32(hipStream_t st, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                           int64_t sbn, int64_t M, int64_t N, int64_t K, int64_t ksplit, float *part) {
    const int64_t ns = (K + ksplit - 1) / ksplit;
    dim3 grid((unsigned)((M + kGT - 1) / kGT), (unsigned)((N + kGT - 1) / kGT), (unsigned)ns);
    hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, part);
    return hipGetLastError();
}

// dst[r * d_ld + c] (=|+=) alpha * sum_s part[s][r][c]   (fixed order)
__global__ void sum_parts_kernel(const float *__restrict__ part, int32_t nsplit, int64_t plane, int32_t cols,
                                 int64_t p_ld, float *__restrict__ dst, int64_t d_ld, float alpha, int32_t accumulate) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int i = 0; i < nsplit; ++i) s += part[i * plane + r * p_ld + c];
        float *o = dst + r * d_ld + c;
        *o = accumulate ? *o + alpha * s : alpha * s;
    }
}

hipError_t launch_sum_parts(hipStream_t st, const float *part, int32_t nsplit, int64_t plane, int32_t rows,
                            int32_t cols, int64_t p_ld, float *dst, int64_t d_ld, float alpha, int32_t accumulate) {
    dim3 grid((unsigned)std::min<int64_t>((cols + 255) / 256, 1024), rows);
    hipLaunchKernelGGL(sum_parts_kernel, grid, dim3(256), 0, st, part, nsplit, plane, cols, p_ld, dst, d_ld, alpha,
                       accumulate);
    return hipGetLastError();
}

}  // namespace lloid

// ------------------------------------------- FP8 basis values (refinement)
// The values the FP8 form's correlation uses for a basis row, as float64:
// one block per row, e = floor(log2(448 / max|u|)), e4m3 (round to nearest
// even, from float32) of u 2^e, times 2^-e.  Quantisation-aware refinement
// evaluates the loss at these values and applies the gradient to the
// unrounded rows.
namespace {

__global__ __launch_bounds__(256) void quantize_fp8_rows_kernel(const double *__restrict__ src, int32_t cols,
                                                                double *__restrict__ dst) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const double *u = src + (int64_t)r * cols;
    double mx = 0.0;
    for (int c = threadIdx.x; c < cols; c += 256) mx = fmax(mx, fabs(u[c]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const int e = red[0] > 0.0 ? (int)floor(log2(448.0 / red[0])) : 0;
    const double s = ldexp(1.0, e);
    for (int c = threadIdx.x; c < cols; c += 256) {
        const uint32_t b = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32((float)(u[c] * s), 0.0f, 0, false) & 0xffu;
        dst[(int64_t)r * cols + c] = ldexp((double)__builtin_amdgcn_cvt_f32_fp8((int)b, 0), -e);
    }
}

}  // namespace

extern "C" lloid_status lloid_quantize_fp8_rows(const double *U, int32_t rows, int32_t cols, double *Uq,
                                                void *stream) {
    if (!U || !Uq || rows < 1 || cols < 1) return LLOID_E_ARG;
    hipLaunchKernelGGL(quantize_fp8_rows_kernel, dim3(rows), dim3(256), 0, static_cast<hipStream_t>(stream), U, cols,
                       Uq);
    return hipGetLastError() == hipSuccess ? LLOID_OK : LLOID_E_HIP;
}
