// Mixing-matrix contraction fused with the polyphase upsample-and-add chain,
// the SNR series write and per-tile trigger candidates (Sec. II.C.2
// "Filtering and reconstruction", "Upsampling SNR segments", "Combining SNR
// segments"; the recursion of the pre-synchronisation equation, Sec. II.C.3).
//
// One work group = 32 real rows (16 templates) x kMixTN top-rate samples of
// one bank and detector.  Levels run lowest rate first; level j covers the
// local window [lo_j + t0/P_j, +n_j): the tile plus the halo its upper level
// reads.  Per level:
//   acc = sum over slices at rate j of W~^s (rows) x y^s (window)   [MFMA]
//       + H_up(level j+1)                                           [MFMA]
// Level j >= 1 is kept in LDS for the next level; level 0 goes to the SNR
// series (interleaved re, im) and to the running trigger candidates.
//
// The basis rows of a level stream through LDS in chunks of CH rows: the
// chunk's basis-output window (CH x n_j) and W~ block (32 x CH) are loaded
// with coalesced reads into registers while the previous chunk's MFMAs run
// (the first chunk of the next level is fetched during this level's
// upsampling and epilogue), then stored to LDS after a barrier.  Each wave
// accumulates its own column blocks (cb = wave, wave+4, ...) over all
// chunks of the level.
//
// The polyphase upsample is a banded contraction into the same accumulator:
// for the 16 output columns of a block starting at level index i0, with
// q0 = floor(i0/p) and lane column c (i = i0 + c, q = floor(i/p),
// ph = i mod p, off = q - q0),
//   H_up(prev)[r][c] = sum_k prev[r][q0 - N_up + k] Ker[k][c],
//   Ker[k][c] = z_ph[off + 2 N_up - k]  for off <= k <= off + 2 N_up, else 0,
// and for phase 0 Ker is the unit vector at k = off + N_up (the copy case of
// Eq. (upsample)).  off <= 7 and 2 N_up <= 16, so a 24- (FP32) or 32-wide
// (16-bit) window of prev holds every tap.
#include <hip/hip_runtime.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

constexpr int kSY = kMixTN + 16;   // chunk row stride (floats): 16 mod 32

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

// ------------------------------------------------------------------ FP32
struct MixF32 {
    static constexpr int CH = 16;
    static constexpr int WCS = CH + 2;            // W chunk row stride: 2 mod 32 words
    static constexpr int WC_FLOATS = kMixTM * WCS;
    struct Regs {
        float y[CH];
        float2 w;
    };
    static __device__ __forceinline__ void load(Regs &g, const MixSlice &ms, const float *Y, int64_t pos0, int n,
                                                int r0, int l0, int tid) {
        const int64_t rs = 2LL * ms.capY;
#pragma unroll
        for (int i = 0; i < CH; ++i) g.y[i] = tid < n ? Y[(int64_t)(l0 + i) * rs + pos0 + tid] : 0.0f;
        const int e = 2 * tid, r = e / CH, kk = e % CH;   // 32 rows x 16 = 512 values
        g.w = *reinterpret_cast<const float2 *>(ms.W + (int64_t)(r0 + r) * ms.Lpad + l0 + kk);
    }
    static __device__ __forceinline__ void store(const Regs &g, float *Ys, float *Wc, int tid) {
#pragma unroll
        for (int i = 0; i < CH; ++i) Ys[i * kSY + tid] = g.y[i];
        const int e = 2 * tid, r = e / CH, kk = e % CH;
        Wc[r * WCS + kk] = g.w.x;
        Wc[r * WCS + kk + 1] = g.w.y;
    }
    static __device__ __forceinline__ void mma(const float *Ys, const float *Wc, int cb, int li, int lg,
                                               floatx4 (&acc)[2]) {
#pragma unroll
        for (int t = 0; t < CH / 4; ++t) {
            const float b = Ys[(4 * t + lg) * kSY + cb * 16 + li];
            acc[0] = mfma_16x16x4_f32(Wc[li * WCS + 4 * t + lg], b, acc[0]);
            acc[1] = mfma_16x16x4_f32(Wc[(16 + li) * WCS + 4 * t + lg], b, acc[1]);
        }
    }
    // 24-wide window, six K-steps of 4
    static __device__ __forceinline__ void upsample(const UpArgs &u, int li, int lg, floatx4 (&acc)[2]) {
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int kk = 4 * t + lg;
            const float b = u.valid ? ker_value(kk, u.off, u.ph, u.nup, u.taps) : 0.0f;
            const int idx = min(u.m0 + kk, u.n_prev - 1);
            acc[0] = mfma_16x16x4_f32(u.prev[li * u.S + idx], b, acc[0]);
            acc[1] = mfma_16x16x4_f32(u.prev[(16 + li) * u.S + idx], b, acc[1]);
        }
    }
};

// ---------------------------------------------------------------- 16-bit
// v_mfma_f32_16x16x32_{bf16,f16}; W~ hi (and lo) staged as T, row stride 40
// elements (80 B: the 16-B fragment reads of a half-wave hit distinct banks);
// basis outputs staged as FP32 and split on the fly, y = T(y) + T(y - T(y)).
//   SPLIT_W (bf16x3): W_hi y_lo + W_lo y_hi + W_hi y_hi
//   otherwise (fp16): W y_lo + W y_hi
template <typename T, typename T8, bool SPLIT_W>
struct Mix16 {
    static constexpr int CH = 32;
    static constexpr int WCS = CH + 8;
    static constexpr int WC_FLOATS = kMixTM * WCS;   // hi + lo parts of 2-byte T
    struct Regs {
        float y[CH];
        uint2 wh, wl;
    };
    static __device__ __forceinline__ void load(Regs &g, const MixSlice &ms, const float *Y, int64_t pos0, int n,
                                                int r0, int l0, int tid) {
        const int64_t rs = 2LL * ms.capY;
#pragma unroll
        for (int i = 0; i < CH; ++i) g.y[i] = tid < n ? Y[(int64_t)(l0 + i) * rs + pos0 + tid] : 0.0f;
        const int e = 4 * tid, r = e / CH, kk = e % CH;   // 32 rows x 32 = 1024 values per part
        const int64_t o = (int64_t)(r0 + r) * ms.Lpad + l0 + kk;
        g.wh = *reinterpret_cast<const uint2 *>(static_cast<const T *>(ms.Whi) + o);
        if (SPLIT_W) g.wl = *reinterpret_cast<const uint2 *>(static_cast<const T *>(ms.Wlo) + o);
    }
    static __device__ __forceinline__ void store(const Regs &g, float *Ys, float *Wcf, int tid) {
#pragma unroll
        for (int i = 0; i < CH; ++i) Ys[i * kSY + tid] = g.y[i];
        T *wh = reinterpret_cast<T *>(Wcf);
        T *wl = wh + kMixTM * WCS;
        const int e = 4 * tid, r = e / CH, kk = e % CH;
        *reinterpret_cast<uint2 *>(wh + r * WCS + kk) = g.wh;
        if (SPLIT_W) *reinterpret_cast<uint2 *>(wl + r * WCS + kk) = g.wl;
    }
    static __device__ __forceinline__ void mma(const float *Ys, const float *Wcf, int cb, int li, int lg,
                                               floatx4 (&acc)[2]) {
        const T *wh = reinterpret_cast<const T *>(Wcf);
        const T *wl = wh + kMixTM * WCS;
        T8 bh, bl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float y = Ys[(8 * lg + j) * kSY + cb * 16 + li];
            const T h = (T)y;
            bh[j] = h;
            bl[j] = (T)(y - (float)h);
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int off = (m * 16 + li) * WCS + 8 * lg;
            const T8 ah = *reinterpret_cast<const T8 *>(wh + off);
            acc[m] = mfma16(ah, bl, acc[m]);
            if (SPLIT_W) acc[m] = mfma16(*reinterpret_cast<const T8 *>(wl + off), bh, acc[m]);
            acc[m] = mfma16(ah, bh, acc[m]);
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

// ------------------------------------------------------------------ kernel
template <typename Op>
__global__ __launch_bounds__(256) void mix_kernel(const MixItem *__restrict__ items, const MixBank *__restrict__ banks,
                                                  const MixSlice *__restrict__ slices,
                                                  const float *__restrict__ uptaps, float *__restrict__ series,
                                                  PartialPeak *__restrict__ partials, int32_t F, int32_t S,
                                                  int32_t nup, int32_t n_items, int32_t group,
                                                  const int64_t *__restrict__ stride_ctr) {
    extern __shared__ float sm[];
    constexpr int TM = kMixTM;
    float *bufA = sm;
    float *bufB = sm + TM * S;
    float *Ys = sm + 2 * TM * S;
    float *Wc = Ys + Op::CH * kSY;
    __shared__ PeakCand wbest[4][TM / 2];

    const int item = xcd_item(group);
    if (item >= n_items) return;
    const MixItem it = items[item];
    const MixBank &B = banks[it.bank];
    const int64_t kstr = *stride_ctr;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;

    // chunk cursor: level cj, slice cs, first basis row cl; cj < 0 at the end
    int cj = B.nlev - 1, cs = B.slice_begin[B.nlev - 1], cl = 0;
    auto settle = [&]() {
        while (cj >= 0) {
            if (cs < B.slice_begin[cj + 1]) {
                if (cl < slices[cs].Lpad) return;
                ++cs;
                cl = 0;
                continue;
            }
            --cj;
            if (cj >= 0) {
                cs = B.slice_begin[cj];
                cl = 0;
            }
        }
    };
    typename Op::Regs g;
    auto fetch = [&]() {
        const MixSlice &ms = slices[cs];
        const int lo = B.lo[cj] + it.t0 / B.P[cj];
        const int64_t pos0 = posmod(kstr * (int64_t)B.rate[cj] + lo, ms.capY);
        Op::load(g, ms, ms.Y + (int64_t)it.det * ms.ydet, pos0, B.n[cj], it.r0, cl, tid);
    };
    settle();
    if (cj >= 0) fetch();

    float *prev = bufA, *cur = bufB;
    int lo_prev = 0;
    PeakCand best[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) best[t] = PeakCand{-1.0f, 0x7fffffff, 0.f, 0.f};

    for (int j = B.nlev - 1; j >= 0; --j) {
        const int lo = B.lo[j] + it.t0 / B.P[j];
        const int n = B.n[j];
        const int nb = (n + 15) >> 4;
        floatx4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        while (cj == j) {
            __syncthreads();   // the previous chunk's LDS reads are done
            Op::store(g, Ys, Wc, tid);
            __syncthreads();
            cl += Op::CH;
            settle();
            if (cj >= 0) fetch();   // next chunk (possibly of a lower level) in flight during the MFMAs
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int cb = wave + 4 * i;
                if (cb < nb) Op::mma(Ys, Wc, cb, li, lg, acc[i]);
            }
        }
        const bool has_up = (j < B.nlev - 1);
        const int logp = has_up ? __ffs(B.p[j + 1]) - 1 : 0;
        const float *taps = has_up ? uptaps + (B.p[j + 1] - 1) * kUpTaps : nullptr;
        const int n_prev = has_up ? B.n[j + 1] : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cb = wave + 4 * i;
            if (cb >= nb) continue;   // wave-uniform
            const int c = cb * 16 + li;
            const bool valid = c < n;
            if (has_up) {
                const int i0 = lo + cb * 16;
                const int q0 = i0 >> logp;   // arithmetic shift: floor for negative indices
                const int ii = i0 + li;
                UpArgs ua{prev, S, n_prev, q0 - nup - lo_prev, (ii >> logp) - q0, ii & ((1 << logp) - 1), nup,
                          taps, valid};
                Op::upsample(ua, li, lg, acc[i]);
            }
            if (!valid) continue;
            if (j > 0) {
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int v = 0; v < 4; ++v) cur[(m * 16 + lg * 4 + v) * S + c] = acc[i][m][v];
            } else {
                const int t = it.t0 + c;
#pragma unroll
                for (int m = 0; m < 2; ++m) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float re = acc[i][m][2 * h], im = acc[i][m][2 * h + 1];
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
        __syncthreads();   // level j complete before it is read as prev
        float *tmp = prev;
        prev = cur;
        cur = tmp;
        lo_prev = lo;
    }
    // trigger candidates: reduce over the 16 lanes of a row group, then waves
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

template <typename Op>
static size_t mix_lds_bytes(int S) {
    return (size_t)(2 * kMixTM * S + Op::CH * kSY + Op::WC_FLOATS) * sizeof(float);
}

size_t mix_lds(int precision, int S) {
    switch (precision) {
        case LLOID_FP32: return mix_lds_bytes<MixF32>(S);
        case LLOID_BF16X3:
        case LLOID_FP8_BF16: return mix_lds_bytes<Mix16<__bf16, bf16x8, true>>(S);
        case LLOID_FP16: return mix_lds_bytes<Mix16<_Float16, halfx8, false>>(S);
        default: return 0;
    }
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
            hipLaunchKernelGGL(mix_kernel<MixF32>, grid, dim3(256), lds, ctx.stream, items, banks, slices,
                               uptaps, series, partials, F, S, nup, n_items, group, ctx.stride_ctr);
            break;
        case LLOID_BF16X3:
        case LLOID_FP8_BF16:
            hipLaunchKernelGGL((mix_kernel<Mix16<__bf16, bf16x8, true>>), grid, dim3(256), lds, ctx.stream,
                               items, banks, slices, uptaps, series, partials, F, S, nup, n_items, group, ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL((mix_kernel<Mix16<_Float16, halfx8, false>>), grid, dim3(256), lds,
                               ctx.stream, items, banks, slices, uptaps, series, partials, F, S, nup,
                               n_items, group, ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace lloid
