// Device kernels of the LLOID filtering core for gfx950 (CDNA4).
//
// One stride runs six kernels, all over precomputed work tables:
//   ingest    strain stride -> top-rate history ring (gaps become zeros)
//   down      decimation to every slice rate, Eq. (sinc) kernel, zero phase
//   corr      per-slice basis correlation, a Hankel(strain) x basis
//             contraction on MFMA with LDS-staged tiles, split over taps
//   reduce    fixed-order sum of the tap splits into the basis-output ring
//   mix       mixing-matrix contraction on MFMA fused with the polyphase
//             upsample-and-add chain (lowest rate first), the SNR series
//             write and per-tile peak candidates
//   peaks     fixed-order reduction of the candidates, one trigger per
//             template (Sec. II.D.1)
// Every output element has exactly one owner and every sum has a fixed
// order, so repeated runs are bit-identical.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

__device__ __forceinline__ int64_t posmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// ------------------------------------------------------------------ ingest
__global__ void ingest_kernel(const float *__restrict__ strain, uint32_t gap_mask, float *__restrict__ xring,
                              int64_t det_stride, int32_t cap, int32_t F, const int64_t *__restrict__ stride_ctr) {
    const int det = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F) return;
    const int64_t k = *stride_ctr;
    const float v = ((gap_mask >> det) & 1u) ? 0.0f : strain[(int64_t)det * F + i];
    const int64_t pos = posmod(k * F + i, cap);
    float *r = xring + det * det_stride;
    r[pos] = v;
    r[pos + cap] = v;
}

hipError_t launch_ingest(const LaunchCtx &ctx, const float *strain, uint32_t gap_mask, float *xring,
                         int64_t ring_det_stride, int32_t cap, int32_t F, int32_t n_det) {
    dim3 grid((F + 255) / 256, n_det);
    hipLaunchKernelGGL(ingest_kernel, grid, dim3(256), 0, ctx.stream, strain, gap_mask, xring, ring_det_stride,
                       cap, F, ctx.stride_ctr);
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
    const int i = threadIdx.x;
    if (i < it.chunk) {
        float acc = 0.0f;
        const int b = i * it.D;
        for (int t = 0; t < ntap; ++t) acc = fmaf(taps[t], xs[lds_pad(b + t)], acc);
        const int64_t pos = posmod(m_first + i, it.capd);
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

// ------------------------------------------------------- basis correlation
// Y[l][c] = sum_n U[l][n] d[k f + off + c + n]: A = U (rows l, K = taps),
// B = Hankel window of the stream (K = taps, N = columns), on
// v_mfma_f32_16x16x4_f32.  The work group owns all Lpad rows and 64 columns
// (one 16-column block per wave); taps advance in chunks of kCorrTK staged
// in LDS: the basis tile row-major with row stride kCorrTK + 2 (the 16 rows x
// 2 taps a half-wave reads fall in distinct banks) and the strain segment
// kCorrTQ + kCorrTK long, from which every lane reads its Hankel entry.
constexpr int kUS = kCorrTK + 2;

template <int MBMAX>
__global__ __launch_bounds__(256) void corr_f32_kernel(const CorrItem *__restrict__ items,
                                                       const int64_t *__restrict__ stride_ctr) {
    __shared__ float Us[MBMAX * 16 * kUS];
    __shared__ float ds[kCorrTQ + kCorrTK];
    const CorrItem it = items[blockIdx.x];
    const int64_t kstr = *stride_ctr;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int rows = it.mb * 16;

    floatx4 acc[MBMAX];
#pragma unroll
    for (int m = 0; m < MBMAX; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int64_t dbase = kstr * it.f + it.off + it.col0 + it.k0;
    for (int kk = 0; kk < it.klen; kk += kCorrTK) {
        __syncthreads();
        // basis tile: rows x kCorrTK taps, float2 per thread-step
        for (int e = tid; e < rows * (kCorrTK / 2); e += 256) {
            const int r = e / (kCorrTK / 2), t2 = e % (kCorrTK / 2);
            const float2 v = *reinterpret_cast<const float2 *>(it.U + (int64_t)r * it.Npad + it.k0 + kk + 2 * t2);
            Us[r * kUS + 2 * t2] = v.x;
            Us[r * kUS + 2 * t2 + 1] = v.y;
        }
        const int64_t p0 = posmod(dbase + kk, it.cap);
        for (int e = tid; e < kCorrTQ + kCorrTK; e += 256) ds[e] = it.ring[p0 + e];
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kCorrTK; ks += 4) {
            const float b = ds[wave * 16 + li + ks + lk];
#pragma unroll
            for (int m = 0; m < MBMAX; ++m) {
                if (m < it.mb) {
                    const float a = Us[(m * 16 + li) * kUS + ks + lk];
                    acc[m] = mfma_16x16x4_f32(a, b, acc[m]);
                }
            }
        }
    }
    const int c = wave * 16 + li;
    if (c < it.ncols) {
#pragma unroll
        for (int m = 0; m < MBMAX; ++m) {
            if (m < it.mb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = m * 16 + lk * 4 + v;
                    it.part[(int64_t)r * it.f + it.col0 + c] = acc[m][v];
                }
            }
        }
    }
}

hipError_t launch_corr_reduced(const LaunchCtx &ctx, int precision, const CorrItem *items, int32_t n_items);

hipError_t launch_corr(const LaunchCtx &ctx, int precision, const CorrItem *items, int32_t n_items) {
    if (n_items == 0) return hipSuccess;
    if (precision != LLOID_FP32) return launch_corr_reduced(ctx, precision, items, n_items);
    hipLaunchKernelGGL(corr_f32_kernel<kMaxBasis / 16>, dim3(n_items), dim3(256), 0, ctx.stream, items, ctx.stride_ctr);
    return hipGetLastError();
}

// ------------------------------------------------------ split-K reduction
__global__ __launch_bounds__(256) void reduce_kernel(const ReduceItem *__restrict__ items,
                                                     const int64_t *__restrict__ stride_ctr) {
    const ReduceItem it = items[blockIdx.x];
    const int l = blockIdx.y;
    if (l >= it.L) return;
    const int64_t k = *stride_ctr;
    const int64_t q0 = k * it.f + it.la;
    const int64_t plane = (int64_t)it.Lpad * it.f;
    float *row = it.yring + (int64_t)l * 2 * it.capY;
    for (int c = threadIdx.x; c < it.f; c += blockDim.x) {
        float s = 0.0f;
        const float *p = it.part + (int64_t)l * it.f + c;
        for (int sp = 0; sp < it.nsplit; ++sp) s += p[sp * plane];
        const int64_t pos = posmod(q0 + c, it.capY);
        row[pos] = s;
        row[pos + it.capY] = s;
    }
}

hipError_t launch_reduce(const LaunchCtx &ctx, const ReduceItem *items, int32_t n_items, int32_t max_rows) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(n_items, max_rows), dim3(256), 0, ctx.stream, items, ctx.stride_ctr);
    return hipGetLastError();
}

// ------------------------------------------- mixing + upsample-and-add chain
// One work group = 32 real rows (16 templates) x kMixTN top-rate samples of
// one bank and detector.  Levels run lowest rate first; level j covers the
// local window [lo_j + t0/P_j, +n_j): the tile plus the polyphase halo its
// upper level reads.  Per level:
//   acc = H_up(level j+1)  (Eq. (upsample), zero-phase: phase-0 samples are
//                            copied, others take 2 N_up + 1 taps)
//       + sum over slices at rate j of W~^s (rows) x y^s (window)   [MFMA]
// Level j >= 1 is kept in LDS for the next level; level 0 goes to the SNR
// series (interleaved re, im) and to per-lane running peaks.  The W~ rows of
// all slices of a level are staged together in LDS with row stride
// SW = 2 mod 32 so the 16 rows x 2 taps of a half-wave hit distinct banks;
// level buffers use row stride S = 8 mod 32.
struct PeakCand {
    float p2;
    int idx;
    float re, im;
};

__device__ __forceinline__ bool better(float p2, int idx, float bp2, int bidx) {
    return p2 > bp2 || (p2 == bp2 && idx < bidx);
}

__device__ __forceinline__ float upsample_at(const float *__restrict__ prev_row, int i, int lo_prev, int logp,
                                             const float *__restrict__ taps, int ntap, int nup) {
    const int q = i >> logp;
    const int ph = i & ((1 << logp) - 1);
    if (ph == 0) return prev_row[q - lo_prev];
    const float *z = taps + ph * kUpTaps;
    const float *src = prev_row + (q + nup - lo_prev);
    float s = 0.0f;
    for (int t = 0; t < ntap; ++t) s = fmaf(src[-t], z[t], s);
    return s;
}

template <typename Op>
__global__ __launch_bounds__(256) void mix_kernel(const MixItem *__restrict__ items, const MixBank *__restrict__ banks,
                                                  const MixSlice *__restrict__ slices,
                                                  const float *__restrict__ uptaps, float *__restrict__ series,
                                                  PartialPeak *__restrict__ partials, int32_t F, int32_t n_det,
                                                  int32_t S, int32_t SW, int32_t nup,
                                                  const int64_t *__restrict__ stride_ctr) {
    extern __shared__ float sm[];
    constexpr int TM = kMixTM;
    float *bufA = sm;
    float *bufB = sm + TM * S;
    float *Ws = sm + 2 * TM * S;
    __shared__ PeakCand wbest[4][TM / 2];

    const MixItem it = items[blockIdx.x];
    const MixBank &B = banks[it.bank];
    const int64_t k = *stride_ctr;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int ntap = 2 * nup + 1;

    float *prev = bufA, *cur = bufB;
    int lo_prev = 0;
    PeakCand best[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) best[t] = PeakCand{-1.0f, 0x7fffffff, 0.f, 0.f};

    for (int j = B.nlev - 1; j >= 0; --j) {
        const int lo = B.lo[j] + it.t0 / B.P[j];
        const int n = B.n[j];
        const int64_t abs0 = k * (int64_t)B.rate[j] + lo;
        __syncthreads();   // previous level complete; Ws free
        // stage the W~ rows of every slice at this level
        int lsum = 0;
        for (int s = B.slice_begin[j]; s < B.slice_begin[j + 1]; ++s) {
            const MixSlice &ms = slices[s];
            Op::stage_w(ms, it.r0, Ws, SW, lsum, tid);
            lsum += ms.Lpad;
        }
        __syncthreads();
        const bool has_up = (j < B.nlev - 1);
        const int logp = has_up ? __ffs(B.p[j + 1]) - 1 : 0;
        const float *taps = has_up ? uptaps + (B.p[j + 1] - 1) * kUpTaps : nullptr;
        const int nb = (n + 15) >> 4;
        for (int cb = wave; cb < nb; cb += 4) {
            const int c = cb * 16 + li;
            const bool valid = c < n;
            floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
            int lb = 0;
            for (int s = B.slice_begin[j]; s < B.slice_begin[j + 1]; ++s) {
                const MixSlice &ms = slices[s];
                const float *Y = ms.Y + (int64_t)it.det * ms.ydet;
                const int64_t pos0 = posmod(abs0, ms.capY) + c;
                Op::contract(Y, ms, pos0, valid, Ws, SW, lb, li, lg, acc);
                lb += ms.Lpad;
            }
            if (!valid) continue;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = m * 16 + lg * 4 + v;
                    float val = acc[m][v];
                    if (has_up) val += upsample_at(prev + r * S, lo + c, lo_prev, logp, taps, ntap, nup);
                    acc[m][v] = val;
                    if (j > 0) cur[r * S + c] = val;
                }
            }
            if (j == 0) {
                const int t = it.t0 + c;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float re = acc[m][2 * h], im = acc[m][2 * h + 1];
                        const int tl = m * 8 + lg * 2 + h;   // template within the tile
                        const int tmpl = it.r0 / 2 + tl;
                        if (series && tmpl < B.M) {
                            float2 *o = reinterpret_cast<float2 *>(series + B.series_off) +
                                        ((int64_t)it.det * B.M + tmpl) * F + t;
                            *o = make_float2(re, im);
                        }
                        const float p2 = re * re + im * im;
                        if (better(p2, t, best[m * 2 + h].p2, best[m * 2 + h].idx))
                            best[m * 2 + h] = PeakCand{p2, t, re, im};
                    }
                }
            }
        }
        float *tmp = prev;
        prev = cur;
        cur = tmp;
        lo_prev = lo;
    }
    // peak candidates: reduce over the 16 lanes of a row group, then waves
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        PeakCand b = best[q];
        for (int off = 1; off < 16; off <<= 1) {
            PeakCand o;
            o.p2 = __shfl_xor(b.p2, off, 64);
            o.idx = __shfl_xor(b.idx, off, 64);
            o.re = __shfl_xor(b.re, off, 64);
            o.im = __shfl_xor(b.im, off, 64);
            if (better(o.p2, o.idx, b.p2, b.idx)) b = o;
        }
        if (li == 0) wbest[wave][(q >> 1) * 8 + lg * 2 + (q & 1)] = b;
    }
    __syncthreads();
    if (tid < TM / 2) {
        PeakCand b = wbest[0][tid];
        for (int w = 1; w < 4; ++w) {
            const PeakCand o = wbest[w][tid];
            if (better(o.p2, o.idx, b.p2, b.idx)) b = o;
        }
        const int tmpl = it.r0 / 2 + tid;
        if (tmpl < B.M) {
            const int64_t pi = B.part_off + ((int64_t)it.det * B.M + tmpl) * B.n_ttiles + it.t0 / kMixTN;
            partials[pi] = PartialPeak{b.p2, b.idx, b.re, b.im};
        }
    }
}

struct MixF32 {
    static __device__ __forceinline__ void stage_w(const MixSlice &ms, int r0, float *Ws, int SW, int lbase, int tid) {
        const int Lp = ms.Lpad;
        for (int e = tid; e < kMixTM * Lp; e += 256) {
            const int r = e / Lp, l = e % Lp;
            Ws[r * SW + lbase + l] = ms.W[(int64_t)(r0 + r) * Lp + l];
        }
    }
    static __device__ __forceinline__ void contract(const float *Y, const MixSlice &ms, int64_t pos0, bool valid,
                                                    const float *Ws, int SW, int lb, int li, int lg,
                                                    floatx4 (&acc)[2]) {
        const int64_t rs = 2 * (int64_t)ms.capY;
        for (int l = 0; l < ms.Lpad; l += 4) {
            const float b = valid ? Y[(int64_t)(l + lg) * rs + pos0] : 0.0f;
            const float a0 = Ws[li * SW + lb + l + lg];
            const float a1 = Ws[(16 + li) * SW + lb + l + lg];
            acc[0] = mfma_16x16x4_f32(a0, b, acc[0]);
            acc[1] = mfma_16x16x4_f32(a1, b, acc[1]);
        }
    }
};

hipError_t launch_mix_reduced(const LaunchCtx &ctx, int precision, const MixItem *items, int32_t n_items,
                              const MixBank *banks, const MixSlice *slices, const float *uptaps, float *series,
                              PartialPeak *partials, int32_t F, int32_t n_det, int32_t S, int32_t SW, int32_t nup);

hipError_t launch_mix(const LaunchCtx &ctx, int precision, const MixItem *items, int32_t n_items,
                      const MixBank *banks, const MixSlice *slices, const float *uptaps, float *series,
                      PartialPeak *partials, int32_t F, int32_t n_det, int32_t S, int32_t SW, int32_t nup) {
    if (n_items == 0) return hipSuccess;
    if (precision != LLOID_FP32)
        return launch_mix_reduced(ctx, precision, items, n_items, banks, slices, uptaps, series, partials, F,
                                  n_det, S, SW, nup);
    const size_t lds = (size_t)(2 * kMixTM * S + kMixTM * SW) * sizeof(float);
    hipLaunchKernelGGL(mix_kernel<MixF32>, dim3(n_items), dim3(256), lds, ctx.stream, items, banks, slices, uptaps,
                       series, partials, F, n_det, S, SW, nup, ctx.stride_ctr);
    return hipGetLastError();
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
__global__ void normalize_kernel(const double *const *__restrict__ W64, const int32_t *__restrict__ Ls,
                                 int32_t n_slices, int32_t rows, int32_t normalize, double *__restrict__ inv) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double s = 0.0;
    for (int i = 0; i < n_slices; ++i) {
        const double *w = W64[i] + (int64_t)r * Ls[i];
        for (int l = 0; l < Ls[i]; ++l) s = fma(w[l], w[l], s);
    }
    inv[r] = (normalize && s > 0.0) ? 1.0 / sqrt(s) : 1.0;
}

hipError_t launch_normalize(hipStream_t st, const double *const *W64, const int32_t *Ls, int32_t n_slices,
                            int32_t rows, int32_t normalize, double *inv_norm) {
    hipLaunchKernelGGL(normalize_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, W64, Ls, n_slices, rows,
                       normalize, inv_norm);
    return hipGetLastError();
}

hipError_t launch_convert_reduced(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                                  const double *row_scale, int precision, int role, void *dst_hi, void *dst_lo,
                                  int32_t dst_ld, float *row_scale_out);

__global__ void convert_f32_kernel(const double *__restrict__ src, int32_t rows, int32_t cols, int32_t src_ld,
                                   const double *__restrict__ row_scale, float *__restrict__ dst, int32_t dst_ld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const double v = src[(int64_t)r * src_ld + c] * (row_scale ? row_scale[r] : 1.0);
    dst[(int64_t)r * dst_ld + c] = (float)v;
}

hipError_t launch_convert_rows(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                               const double *row_scale, int precision, int role, float *dst32, void *dst_hi,
                               void *dst_lo, int32_t dst_ld, float *row_scale_out) {
    const int64_t n = (int64_t)rows * cols;
    if (n == 0) return hipSuccess;
    if (dst32) {
        hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, rows,
                           cols, src_ld, row_scale, dst32, dst_ld);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (dst_hi)
        return launch_convert_reduced(st, src, rows, cols, src_ld, row_scale, precision, role, dst_hi, dst_lo,
                                      dst_ld, row_scale_out);
    return hipSuccess;
}

}  // namespace lloid
