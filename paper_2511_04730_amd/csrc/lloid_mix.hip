// Mixing-matrix contraction fused with the polyphase upsample-and-add chain,
// the SNR series write and per-tile trigger candidates (Sec. II.C.2
// "Filtering and reconstruction", "Upsampling SNR segments", "Combining SNR
// segments"; the recursion of the pre-synchronisation equation, Sec. II.C.3).
//
// One work group = kMixTM = 64 real rows (32 templates) x kMixTN = 256
// top-rate samples of one bank and detector.  Levels run lowest rate first;
// level j covers the local window [lo_j + t0/P_j, +n_j): the tile plus the
// halo its upper level reads.  Per level:
//   acc = sum over slices at rate j of W~^s (rows) x y^s (window)   [MFMA]
//       + H_up(level j+1)                                           [MFMA]
// Level j >= 1 is kept in LDS for the next level; level 0 goes to the SNR
// series (interleaved re, im) and to the running trigger candidates.
//
// Both operands of the mixing contraction come straight from memory into
// MFMA registers, with no LDS staging and no barrier: W~ rows are row-major
// [rows][Lpad] and the basis-output rings are time-major [position][Lpad]
// (one row per sample), so the K elements a lane supplies (8 consecutive
// basis rows for the 16-bit forms, 4 for FP32) are one 16-byte load on
// either side.  The 16-bit rings already hold y as hi + lo, split once when
// the reduction appends them.  Each wave owns the column blocks
// cb = wave, wave + 4, ... of the window and all four 16-row blocks, so
// every y fragment it loads feeds four row blocks.
//
// The polyphase upsample is a banded contraction into the same accumulator:
// for the 16 output columns of a block starting at level index i0, with
// q0 = floor(i0/p) and lane column c (i = i0 + c, q = floor(i/p),
// ph = i mod p, off = q - q0),
//   H_up(prev)[r][c] = sum_k prev[r][q0 - N_up + k] Ker[k][c],
//   Ker[k][c] = z_ph[off + 2 N_up - k]  for off <= k <= off + 2 N_up, else 0,
// and for phase 0 Ker is the unit vector at k = off + N_up (the copy case of
// Eq. (upsample)).  off <= 7 and 2 N_up <= 16, so a 24- (FP32) or 32-wide
// (16-bit) window of prev holds every tap.  One LDS buffer holds a level:
// level j's accumulators stay in registers until every wave has read level
// j+1, then overwrite it.
#include <hip/hip_runtime.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

constexpr int kRB = kMixTM / 16;   // 16-row blocks per work group
constexpr int kCB = 4;             // column blocks per wave (4 waves x 4 x 16 = kMixTN)

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
};

// ------------------------------------------------------------------ FP32
// 16 basis rows per step as four 16x16x4 MFMAs; lane group g supplies basis
// rows l0 + 4g .. l0 + 4g + 3, one per MFMA, on both sides.
struct MixF32 {
    static constexpr int K = 16;
    struct A {
        float4 w[kRB];
    };
    struct B {
        float4 y;
    };
    static __device__ __forceinline__ void load_a(A &a, const MixSlice &ms, int r0, int l0, int li, int lg) {
#pragma unroll
        for (int m = 0; m < kRB; ++m)
            a.w[m] = *reinterpret_cast<const float4 *>(ms.W + (int64_t)(r0 + 16 * m + li) * ms.Lpad + l0 + 4 * lg);
    }
    static __device__ __forceinline__ void load_b(B &b, const void *ring, const MixSlice &ms, int p, int l0,
                                                  int lg) {
        b.y = *reinterpret_cast<const float4 *>(static_cast<const float *>(ring) + (int64_t)p * ms.Lpad + l0 +
                                                 4 * lg);
    }
    static __device__ __forceinline__ void mma(floatx4 (&acc)[kRB], const A &a, const B &b) {
#pragma unroll
        for (int m = 0; m < kRB; ++m) {
            acc[m] = mfma_16x16x4_f32(a.w[m].x, b.y.x, acc[m]);
            acc[m] = mfma_16x16x4_f32(a.w[m].y, b.y.y, acc[m]);
            acc[m] = mfma_16x16x4_f32(a.w[m].z, b.y.z, acc[m]);
            acc[m] = mfma_16x16x4_f32(a.w[m].w, b.y.w, acc[m]);
        }
    }
    // 24-wide window, six K-steps of 4
    static __device__ __forceinline__ void upsample(const UpArgs &u, int li, int lg, floatx4 (&acc)[kRB]) {
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int kk = 4 * t + lg;
            const float b = ker_value(kk, u.off, u.ph, u.nup, u.taps);
            const int idx = min(u.m0 + kk, u.n_prev - 1);
#pragma unroll
            for (int m = 0; m < kRB; ++m) acc[m] = mfma_16x16x4_f32(u.prev[(16 * m + li) * u.S + idx], b, acc[m]);
        }
    }
};

// ---------------------------------------------------------------- 16-bit
// v_mfma_f32_16x16x32_{bf16,f16}: 32 basis rows per step.
//   SPLIT_W (bf16x3): W_hi y_lo + W_lo y_hi + W_hi y_hi
//   otherwise (fp16): W y_lo + W y_hi
template <typename T, typename T8, bool SPLIT_W>
struct Mix16 {
    static constexpr int K = 32;
    struct A {
        T8 h[kRB];
        T8 l[SPLIT_W ? kRB : 1];
    };
    struct B {
        T8 h, l;
    };
    static __device__ __forceinline__ void load_a(A &a, const MixSlice &ms, int r0, int l0, int li, int lg) {
#pragma unroll
        for (int m = 0; m < kRB; ++m) {
            const int64_t o = (int64_t)(r0 + 16 * m + li) * ms.Lpad + l0 + 8 * lg;
            a.h[m] = *reinterpret_cast<const T8 *>(static_cast<const T *>(ms.Whi) + o);
            if constexpr (SPLIT_W) a.l[m] = *reinterpret_cast<const T8 *>(static_cast<const T *>(ms.Wlo) + o);
        }
    }
    static __device__ __forceinline__ void load_b(B &b, const void *ring, const MixSlice &ms, int p, int l0,
                                                  int lg) {
        const T *hi = static_cast<const T *>(ring);
        const int64_t o = (int64_t)p * ms.Lpad + l0 + 8 * lg;
        b.h = *reinterpret_cast<const T8 *>(hi + o);
        b.l = *reinterpret_cast<const T8 *>(hi + 2LL * ms.capY * ms.Lpad + o);
    }
    static __device__ __forceinline__ void mma(floatx4 (&acc)[kRB], const A &a, const B &b) {
#pragma unroll
        for (int m = 0; m < kRB; ++m) {
            acc[m] = mfma16(a.h[m], b.l, acc[m]);
            if constexpr (SPLIT_W) acc[m] = mfma16(a.l[m], b.h, acc[m]);
            acc[m] = mfma16(a.h[m], b.h, acc[m]);
        }
    }
    // 32-wide window, one K-step; both operands split (three products), so
    // the interpolation keeps ~16 (bf16) or ~22 (fp16) significant bits
    static __device__ __forceinline__ void upsample(const UpArgs &u, int li, int lg, floatx4 (&acc)[kRB]) {
        T8 kh, kl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float kv = ker_value(8 * lg + j, u.off, u.ph, u.nup, u.taps);
            const T h = (T)kv;
            kh[j] = h;
            kl[j] = (T)(kv - (float)h);
        }
#pragma unroll
        for (int m = 0; m < kRB; ++m) {
            T8 ph, pl;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int idx = min(u.m0 + 8 * lg + j, u.n_prev - 1);
                const float pv = u.prev[(16 * m + li) * u.S + idx];
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

// ------------------------------------------------------------------ kernel
template <typename Op>
__global__ __launch_bounds__(256) void mix_kernel(const MixItem *__restrict__ items, const MixBank *__restrict__ banks,
                                                  const MixSlice *__restrict__ slices,
                                                  const float *__restrict__ uptaps, float *__restrict__ series,
                                                  PartialPeak *__restrict__ partials, int32_t F, int32_t S,
                                                  int32_t nup, int32_t n_items, int32_t group,
                                                  const int64_t *__restrict__ stride_ctr) {
    extern __shared__ float lvl[];   // [kMixTM][S]: one level of the chain
    __shared__ PeakCand wbest[4][kMixTM / 2];
    const int item = xcd_item(group);
    if (item >= n_items) return;
    const MixItem it = items[item];
    const MixBank &B = banks[it.bank];
    // ring positions are taken modulo capY, a power of two dividing 2^32
    const uint32_t kstr = (uint32_t)*stride_ctr;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;

    PeakCand best[2 * kRB];
#pragma unroll
    for (int t = 0; t < 2 * kRB; ++t) best[t] = PeakCand{-1.0f, 0x7fffffff, 0.f, 0.f};

    int lo_prev = 0;
    for (int j = B.nlev - 1; j >= 0; --j) {
        const int lo = B.lo[j] + (it.t0 >> B.shP[j]);
        const int n = B.n[j];
        const int nb = (n + 15) >> 4;
        floatx4 acc[kCB][kRB];
#pragma unroll
        for (int i = 0; i < kCB; ++i)
#pragma unroll
            for (int m = 0; m < kRB; ++m) acc[i][m] = floatx4{0.f, 0.f, 0.f, 0.f};

        for (int s = B.slice_begin[j]; s < B.slice_begin[j + 1]; ++s) {
            const MixSlice &ms = slices[s];
            const uint32_t pos0 = (kstr * (uint32_t)B.rate[j] + (uint32_t)lo) & (uint32_t)(ms.capY - 1);
            const void *ring = static_cast<const char *>(ms.Y) + (int64_t)it.det * ms.ydet * 4;
            // columns past the window read its last sample (finite, never
            // stored); the window (n <= capY, checked at plan time) is
            // contiguous in the mirror ring, the mask only guards the address
            int pc[kCB];
#pragma unroll
            for (int i = 0; i < kCB; ++i)
                pc[i] = (int)((pos0 + (uint32_t)min((wave + 4 * i) * 16 + li, n - 1)) & (uint32_t)(2 * ms.capY - 1));
            for (int l0 = 0; l0 < ms.Lpad; l0 += Op::K) {
                typename Op::A a;
                typename Op::B b[kCB];
                Op::load_a(a, ms, it.r0, l0, li, lg);
#pragma unroll
                for (int i = 0; i < kCB; ++i)
                    if (wave + 4 * i < nb) Op::load_b(b[i], ring, ms, pc[i], l0, lg);
#pragma unroll
                for (int i = 0; i < kCB; ++i)
                    if (wave + 4 * i < nb) Op::mma(acc[i], a, b[i]);
            }
        }
        if (j < B.nlev - 1) {
            const int logp = B.shp[j + 1];
            const float *taps = uptaps + (B.p[j + 1] - 1) * kUpTaps;
            const int n_prev = B.n[j + 1];
#pragma unroll
            for (int i = 0; i < kCB; ++i) {
                const int cb = wave + 4 * i;
                if (cb >= nb) continue;   // wave-uniform
                const int i0 = lo + cb * 16;
                const int q0 = i0 >> logp;   // arithmetic shift: floor for negative indices
                const int ii = i0 + li;
                const UpArgs ua{lvl, S, n_prev, q0 - nup - lo_prev, (ii >> logp) - q0, ii & ((1 << logp) - 1), nup,
                                taps};
                Op::upsample(ua, li, lg, acc[i]);
            }
        }
        __syncthreads();   // every wave is done reading level j+1
#pragma unroll
        for (int i = 0; i < kCB; ++i) {
            const int cb = wave + 4 * i;
            if (cb >= nb) continue;
            const int c = cb * 16 + li;
            if (c >= n) continue;
            if (j > 0) {
#pragma unroll
                for (int m = 0; m < kRB; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v) lvl[(16 * m + 4 * lg + v) * S + c] = acc[i][m][v];
            } else {
                const int t = it.t0 + c;
#pragma unroll
                for (int m = 0; m < kRB; ++m) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float re = acc[i][m][2 * h], im = acc[i][m][2 * h + 1];
                        const int tmpl = it.r0 / 2 + 8 * m + 2 * lg + h;
                        if (series && tmpl < B.M) {
                            float2 *o = reinterpret_cast<float2 *>(series + B.series_off) +
                                        ((int64_t)it.det * B.M + tmpl) * F + t;
                            *o = make_float2(re, im);
                        }
                        const float p2 = re * re + im * im;
                        if (better(p2, t, best[2 * m + h].p2, best[2 * m + h].idx))
                            best[2 * m + h] = PeakCand{p2, t, re, im};
                    }
                }
            }
        }
        __syncthreads();   // level j complete before it is read as prev
        lo_prev = lo;
    }
    // trigger candidates: reduce over the 16 lanes of a row group, then waves
#pragma unroll
    for (int q = 0; q < 2 * kRB; ++q) {
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
    if (tid < kMixTM / 2) {
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

size_t mix_lds(int precision, int S) {
    if (precision < LLOID_FP32 || precision > LLOID_FP8_BF16) return 0;
    return (size_t)kMixTM * S * sizeof(float);
}

hipError_t configure_down_lds(size_t down_bytes);

// Raise the dynamic-LDS limit of the kernels whose tiles depend on the plan
// (gfx950 has 160 KB of LDS per work group).
hipError_t configure_lds(int precision, size_t mix_bytes, size_t down_bytes) {
    hipError_t e = configure_down_lds(down_bytes);
    if (e != hipSuccess) return e;
    const void *mix = nullptr;
    switch (precision) {
        case LLOID_FP32: mix = reinterpret_cast<const void *>(mix_kernel<MixF32>); break;
        case LLOID_BF16X3:
        case LLOID_FP8_BF16: mix = reinterpret_cast<const void *>(mix_kernel<Mix16<__bf16, bf16x8, true>>); break;
        case LLOID_FP16: mix = reinterpret_cast<const void *>(mix_kernel<Mix16<_Float16, halfx8, false>>); break;
        default: return hipErrorNotSupported;
    }
    return hipFuncSetAttribute(mix, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mix_bytes);
}

hipError_t launch_mix(const LaunchCtx &ctx, int precision, const MixItem *items, int32_t n_items,
                      const MixBank *banks, const MixSlice *slices, const float *uptaps, float *series,
                      PartialPeak *partials, int32_t F, int32_t n_det, int32_t S, int32_t SW, int32_t nup,
                      int32_t group) {
    (void)n_det;
    (void)SW;
    if (n_items == 0) return hipSuccess;
    const size_t lds = mix_lds(precision, S);
    const dim3 grid(xcd_grid(n_items, group));
    switch (precision) {
        case LLOID_FP32:
            hipLaunchKernelGGL(mix_kernel<MixF32>, grid, dim3(256), lds, ctx.stream, items, banks, slices, uptaps,
                               series, partials, F, S, nup, n_items, group, ctx.stride_ctr);
            break;
        case LLOID_BF16X3:
        case LLOID_FP8_BF16:
            hipLaunchKernelGGL((mix_kernel<Mix16<__bf16, bf16x8, true>>), grid, dim3(256), lds, ctx.stream, items,
                               banks, slices, uptaps, series, partials, F, S, nup, n_items, group, ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL((mix_kernel<Mix16<_Float16, halfx8, false>>), grid, dim3(256), lds, ctx.stream,
                               items, banks, slices, uptaps, series, partials, F, S, nup, n_items, group,
                               ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace lloid
