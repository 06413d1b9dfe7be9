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
constexpr int kTKF = 32;             // taps per LDS stage
constexpr int kUS = kTKF + 2;

template <int MBMAX>
__global__ __launch_bounds__(256) void corr_f32_kernel(const CorrItem *__restrict__ items,
                                                       const int64_t *__restrict__ stride_ctr) {
    // double-buffered: the next stage's tiles are loaded into registers while
    // the current stage's MFMAs run from LDS
    __shared__ float Us[2][MBMAX * 16 * kUS];
    __shared__ float ds[2][kCorrTQ + kTKF];
    constexpr int PER = (MBMAX * 16 * (kTKF / 2) + 255) / 256;
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
    float2 ureg[PER];
    float dreg = 0.0f;
    auto gload = [&](int kk) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            if (e < rows * (kTKF / 2)) {
                const int r = e / (kTKF / 2), t2 = e % (kTKF / 2);
                ureg[i] = *reinterpret_cast<const float2 *>(it.U + (int64_t)r * it.Npad + it.k0 + kk + 2 * t2);
            }
        }
        const int64_t p0 = posmod(dbase + kk, it.cap);
        if (tid < kCorrTQ + kTKF) dreg = it.ring[p0 + tid];
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            if (e < rows * (kTKF / 2)) {
                const int r = e / (kTKF / 2), t2 = e % (kTKF / 2);
                Us[buf][r * kUS + 2 * t2] = ureg[i].x;
                Us[buf][r * kUS + 2 * t2 + 1] = ureg[i].y;
            }
        }
        if (tid < kCorrTQ + kTKF) ds[buf][tid] = dreg;
    };
    const int nchunks = it.klen / kTKF;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) gload((c + 1) * kTKF);
#pragma unroll
        for (int ks = 0; ks < kTKF; ks += 4) {
            const float b = ds[buf][wave * 16 + li + ks + lk];
#pragma unroll
            for (int m = 0; m < MBMAX; ++m) {
                if (m < it.mb) {
                    const float a = Us[buf][(m * 16 + li) * kUS + ks + lk];
                    acc[m] = mfma_16x16x4_f32(a, b, acc[m]);
                }
            }
        }
        if (c + 1 < nchunks) lstore(buf ^ 1);
        __syncthreads();
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

// 16-bit correlation on v_mfma_f32_16x16x32_{bf16,f16}: eight consecutive
// taps per lane and K-group.  The basis tile is staged row-major with row
// stride 72 elements (144 B = 16 mod 128, 16-B fragment reads of a half-wave
// in distinct banks).  A Hankel fragment d[q + n .. q + n + 7] starts at an
// arbitrary element, so the strain segment is staged as 8 copies shifted by
// 0..7 elements: the fragment is read from copy (q + n) mod 8 at an aligned
// offset.  The strain is split on the fly, d = d_hi + d_lo.
//   SPLIT_U (bf16x3): U_hi d_lo + U_lo d_hi + U_hi d_hi
//   otherwise (fp16): U d_lo + U d_hi
template <typename T, typename T8, bool SPLIT_U>
__global__ __launch_bounds__(256) void corr16_kernel(const CorrItem *__restrict__ items,
                                                     const int64_t *__restrict__ stride_ctr) {
    constexpr int TK = 64;
    constexpr int US = TK + 8;
    constexpr int MBMAX = kMaxBasis / 16;
    constexpr int DL = kCorrTQ + TK + 8;
    __shared__ __attribute__((aligned(16))) T Uh[MBMAX * 16 * US];
    __shared__ __attribute__((aligned(16))) T Ul[SPLIT_U ? MBMAX * 16 * US : 8];
    __shared__ __attribute__((aligned(16))) T Dh[8 * DL];
    __shared__ __attribute__((aligned(16))) T Dl[8 * DL];
    const CorrItem it = items[blockIdx.x];
    const int64_t kstr = *stride_ctr;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int rows = it.mb * 16;
    const T *gh = static_cast<const T *>(it.Uhi);
    const T *gl = static_cast<const T *>(it.Ulo);

    floatx4 acc[MBMAX];
#pragma unroll
    for (int m = 0; m < MBMAX; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int64_t dbase = kstr * it.f + it.off + it.col0 + it.k0;
    for (int kk = 0; kk < it.klen; kk += TK) {
        __syncthreads();
        for (int e = tid; e < rows * (TK / 8); e += 256) {
            const int r = e / (TK / 8), c8 = e % (TK / 8);
            const int64_t g = (int64_t)r * it.Npad + it.k0 + kk + 8 * c8;
            *reinterpret_cast<uint4 *>(&Uh[r * US + 8 * c8]) = *reinterpret_cast<const uint4 *>(gh + g);
            if (SPLIT_U)
                *reinterpret_cast<uint4 *>(&Ul[r * US + 8 * c8]) = *reinterpret_cast<const uint4 *>(gl + g);
        }
        const int64_t p0 = posmod(dbase + kk, it.cap);
        for (int e = tid; e < kCorrTQ + TK; e += 256) {
            const float v = it.ring[p0 + e];
            const T h = (T)v;
            const T l = (T)(v - (float)h);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int i = e - s;
                if (i >= 0 && i < DL) {
                    Dh[s * DL + i] = h;
                    Dl[s * DL + i] = l;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 32) {
            const int idx = wave * 16 + li + ks + 8 * lk;
            const int sft = idx & 7;
            const T8 bh = *reinterpret_cast<const T8 *>(&Dh[sft * DL + idx - sft]);
            const T8 bl = *reinterpret_cast<const T8 *>(&Dl[sft * DL + idx - sft]);
#pragma unroll
            for (int m = 0; m < MBMAX; ++m) {
                if (m < it.mb) {
                    const int off = (m * 16 + li) * US + ks + 8 * lk;
                    const T8 ah = *reinterpret_cast<const T8 *>(&Uh[off]);
                    acc[m] = mfma16(ah, bl, acc[m]);
                    if (SPLIT_U) acc[m] = mfma16(*reinterpret_cast<const T8 *>(&Ul[off]), bh, acc[m]);
                    acc[m] = mfma16(ah, bh, acc[m]);
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

hipError_t launch_corr_reduced(const LaunchCtx &ctx, int precision, const CorrItem *items, int32_t n_items) {
    switch (precision) {
        case LLOID_BF16X3:
            hipLaunchKernelGGL((corr16_kernel<__bf16, bf16x8, true>), dim3(n_items), dim3(256), 0, ctx.stream, items,
                               ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL((corr16_kernel<_Float16, halfx8, false>), dim3(n_items), dim3(256), 0, ctx.stream,
                               items, ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

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
// all slices of a level are staged together in LDS (row stride SW chosen so
// a half-wave's fragment reads hit distinct banks); level buffers use row
// stride S = 2 mod 32.
//
// The polyphase upsample is a banded contraction into the same MFMA
// accumulator: for the 16 output columns of a block starting at level index
// i0, with q0 = floor(i0/p) and lane column c (i = i0 + c, q = floor(i/p),
// ph = i mod p, off = q - q0),
//   H_up(prev)[r][c] = sum_k prev[r][q0 - N_up + k] Ker[k][c],
//   Ker[k][c] = z_ph[off + 2 N_up - k]  for off <= k <= off + 2 N_up, else 0,
// and for phase 0 Ker is the unit vector at k = off + N_up (the copy case of
// Eq. (upsample)).  off <= 7 and 2 N_up <= 16, so a 24- (FP32) or 32-wide
// (16-bit) window of prev holds every tap.
struct PeakCand {
    float p2;
    int idx;
    float re, im;
};

__device__ __forceinline__ bool better(float p2, int idx, float bp2, int bidx) {
    return p2 > bp2 || (p2 == bp2 && idx < bidx);
}

__device__ __forceinline__ float ker_value(int k, int off, int ph, int nup, const float *__restrict__ taps) {
    if (ph == 0) return k == off + nup ? 1.0f : 0.0f;
    const int t = off + 2 * nup - k;
    return (t >= 0 && t <= 2 * nup) ? taps[ph * kUpTaps + t] : 0.0f;
}

struct UpArgs {
    const float *prev;       // level j+1 buffer, row stride S
    int S, n_prev, m0;       // m0: buffer index of the window start
    int off, ph, nup;
    const float *taps;       // sub-kernels of this stage, [p][kUpTaps]
    bool valid;
};

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
        const int n_prev = has_up ? B.n[j + 1] : 0;
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
            if (has_up) {
                const int i0 = lo + cb * 16;
                const int q0 = i0 >> logp;   // arithmetic shift: floor for negative indices
                const int i = i0 + li;
                UpArgs ua{prev, S, n_prev, q0 - nup - lo_prev, (i >> logp) - q0, i & ((1 << logp) - 1), nup,
                          taps, valid};
                Op::upsample(ua, li, lg, acc);
            }
            if (!valid) continue;
            if (j > 0) {
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v) cur[(m * 16 + lg * 4 + v) * S + c] = acc[m][v];
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
    // All basis-output loads of the column block are issued before the first
    // MFMA, so their latency is paid once per block, not once per k-step.
    static __device__ __forceinline__ void contract(const float *Y, const MixSlice &ms, int64_t pos0, bool valid,
                                                    const float *Ws, int SW, int lb, int li, int lg,
                                                    floatx4 (&acc)[2]) {
        constexpr int KS = kMaxBasis / 4;
        const int64_t rs = 2 * (int64_t)ms.capY;
        const int nks = ms.Lpad >> 2;
        float bv[KS];
#pragma unroll
        for (int t = 0; t < KS; ++t) bv[t] = (valid && t < nks) ? Y[(int64_t)(4 * t + lg) * rs + pos0] : 0.0f;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            if (t < nks) {
                const float a0 = Ws[li * SW + lb + 4 * t + lg];
                const float a1 = Ws[(16 + li) * SW + lb + 4 * t + lg];
                acc[0] = mfma_16x16x4_f32(a0, bv[t], acc[0]);
                acc[1] = mfma_16x16x4_f32(a1, bv[t], acc[1]);
            }
        }
    }
    // 24-wide window, six K-steps of 4
    static __device__ __forceinline__ void upsample(const UpArgs &u, int li, int lg, floatx4 (&acc)[2]) {
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int kk = 4 * t + lg;
            const float b = u.valid ? ker_value(kk, u.off, u.ph, u.nup, u.taps) : 0.0f;
            const int idx = min(u.m0 + kk, u.n_prev - 1);
            const float a0 = u.prev[li * u.S + idx];
            const float a1 = u.prev[(16 + li) * u.S + idx];
            acc[0] = mfma_16x16x4_f32(a0, b, acc[0]);
            acc[1] = mfma_16x16x4_f32(a1, b, acc[1]);
        }
    }
};

// 16-bit mixing on v_mfma_f32_16x16x32_{bf16,f16}.  The W~ rows are staged in
// LDS as T (hi part, then lo part at offset 32 SW), row stride SW = 8 mod 64
// elements so each 16-B fragment read of a half-wave hits distinct banks.  The
// basis outputs are FP32 in the ring and are split on the fly:
// y = y_hi + y_lo, y_hi = T(y), y_lo = T(y - y_hi).
//   SPLIT_W (bf16x3): W_hi y_lo + W_lo y_hi + W_hi y_hi
//   otherwise (fp16): W y_lo + W y_hi
template <typename T, typename T8, bool SPLIT_W>
struct Mix16 {
    static __device__ __forceinline__ T8 mfma_in(const T *p) { return *reinterpret_cast<const T8 *>(p); }
    static __device__ __forceinline__ void stage_w(const MixSlice &ms, int r0, float *Wsf, int SW, int lbase,
                                                   int tid) {
        T *wh = reinterpret_cast<T *>(Wsf);
        T *wl = wh + kMixTM * SW;
        const int Lp = ms.Lpad;
        const T *gh = static_cast<const T *>(ms.Whi);
        const T *gl = static_cast<const T *>(ms.Wlo);
        for (int e = tid; e < kMixTM * Lp; e += 256) {
            const int r = e / Lp, l = e % Lp;
            wh[r * SW + lbase + l] = gh[(int64_t)(r0 + r) * Lp + l];
            if (SPLIT_W) wl[r * SW + lbase + l] = gl[(int64_t)(r0 + r) * Lp + l];
        }
    }
    static __device__ __forceinline__ void contract(const float *Y, const MixSlice &ms, int64_t pos0, bool valid,
                                                    const float *Wsf, int SW, int lb, int li, int lg,
                                                    floatx4 (&acc)[2]) {
        constexpr int KS = kMaxBasis / 32;
        const T *wh = reinterpret_cast<const T *>(Wsf);
        const T *wl = wh + kMixTM * SW;
        const int64_t rs = 2 * (int64_t)ms.capY;
        const int nks = ms.Lpad >> 5;
        float yv[KS][8];
#pragma unroll
        for (int t = 0; t < KS; ++t)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                yv[t][j] = (valid && t < nks) ? Y[(int64_t)(32 * t + 8 * lg + j) * rs + pos0] : 0.0f;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            if (t < nks) {
                T8 bh, bl;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const T h = (T)yv[t][j];
                    bh[j] = h;
                    bl[j] = (T)(yv[t][j] - (float)h);
                }
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int off = (m * 16 + li) * SW + lb + 32 * t + 8 * lg;
                    const T8 ah = mfma_in(wh + off);
                    acc[m] = mfma16(ah, bl, acc[m]);
                    if (SPLIT_W) acc[m] = mfma16(mfma_in(wl + off), bh, acc[m]);
                    acc[m] = mfma16(ah, bh, acc[m]);
                }
            }
        }
    }
    // 32-wide window, one K-step; both operands split (three products), so
    // the interpolation keeps ~16 (bf16) or ~22 (fp16) significant bits
    static __device__ __forceinline__ void upsample(const UpArgs &u, int li, int lg, floatx4 (&acc)[2]) {
        T8 kh, kl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float kv = u.valid ? ker_value(8 * lg + j, u.off, u.ph, u.nup, u.taps) : 0.0f;
            const T h = (T)kv;
            kh[j] = h;
            kl[j] = (T)(kv - (float)h);
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            T8 ph, pl;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int idx = min(u.m0 + 8 * lg + j, u.n_prev - 1);
                const float pv = u.prev[(m * 16 + li) * u.S + idx];
                const T h = (T)pv;
                ph[j] = h;
                pl[j] = (T)(pv - (float)h);
            }
            acc[m] = mfma16(ph, kl, acc[m]);
            acc[m] = mfma16(pl, kh, acc[m]);
            acc[m] = mfma16(ph, kh, acc[m]);
        }
    }
};

// Raise the dynamic-LDS limit of the kernels whose tiles depend on the plan
// (gfx950 has 160 KB of LDS per work group).
hipError_t configure_lds(int precision, size_t mix_bytes, size_t down_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(down_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)down_bytes);
    if (e != hipSuccess) return e;
    const void *mix = nullptr;
    switch (precision) {
        case LLOID_FP32: mix = reinterpret_cast<const void *>(mix_kernel<MixF32>); break;
        case LLOID_BF16X3: mix = reinterpret_cast<const void *>(mix_kernel<Mix16<__bf16, bf16x8, true>>); break;
        case LLOID_FP16: mix = reinterpret_cast<const void *>(mix_kernel<Mix16<_Float16, halfx8, false>>); break;
        default: return hipErrorNotSupported;
    }
    return hipFuncSetAttribute(mix, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mix_bytes);
}

hipError_t launch_mix(const LaunchCtx &ctx, int precision, const MixItem *items, int32_t n_items,
                      const MixBank *banks, const MixSlice *slices, const float *uptaps, float *series,
                      PartialPeak *partials, int32_t F, int32_t n_det, int32_t S, int32_t SW, int32_t nup) {
    if (n_items == 0) return hipSuccess;
    const size_t lds = (size_t)(2 * kMixTM * S + kMixTM * SW) * sizeof(float);
    switch (precision) {
        case LLOID_FP32:
            hipLaunchKernelGGL(mix_kernel<MixF32>, dim3(n_items), dim3(256), lds, ctx.stream, items, banks, slices,
                               uptaps, series, partials, F, n_det, S, SW, nup, ctx.stride_ctr);
            break;
        case LLOID_BF16X3:
            hipLaunchKernelGGL((mix_kernel<Mix16<__bf16, bf16x8, true>>), dim3(n_items), dim3(256), lds, ctx.stream,
                               items, banks, slices, uptaps, series, partials, F, n_det, S, SW, nup, ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL((mix_kernel<Mix16<_Float16, halfx8, false>>), dim3(n_items), dim3(256), lds,
                               ctx.stream, items, banks, slices, uptaps, series, partials, F, n_det, S, SW, nup,
                               ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
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

// v = src * row_scale -> hi = T(v) (round to nearest even), lo = T(v - hi)
// with the residual formed in FP64 (lo is skipped when dst_lo is NULL).
template <typename T>
__global__ void convert_split_kernel(const double *__restrict__ src, int32_t rows, int32_t cols, int32_t src_ld,
                                     const double *__restrict__ row_scale, T *__restrict__ hi, T *__restrict__ lo,
                                     int32_t dst_ld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    const double v = src[(int64_t)r * src_ld + c] * (row_scale ? row_scale[r] : 1.0);
    const T h = (T)(float)v;
    hi[(int64_t)r * dst_ld + c] = h;
    if (lo) lo[(int64_t)r * dst_ld + c] = (T)(float)(v - (double)(float)h);
}

hipError_t launch_convert_reduced(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                                  const double *row_scale, int precision, int role, void *dst_hi, void *dst_lo,
                                  int32_t dst_ld, float *row_scale_out) {
    (void)role;
    (void)row_scale_out;
    const int64_t n = (int64_t)rows * cols;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (precision == LLOID_BF16X3) {
        hipLaunchKernelGGL(convert_split_kernel<__bf16>, grid, dim3(256), 0, st, src, rows, cols, src_ld, row_scale,
                           static_cast<__bf16 *>(dst_hi), static_cast<__bf16 *>(dst_lo), dst_ld);
    } else if (precision == LLOID_FP16) {
        hipLaunchKernelGGL(convert_split_kernel<_Float16>, grid, dim3(256), 0, st, src, rows, cols, src_ld,
                           row_scale, static_cast<_Float16 *>(dst_hi), static_cast<_Float16 *>(dst_lo), dst_ld);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

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
