// Mixing-matrix contraction fused with the polyphase upsample-and-add chain,
// the SNR series write and per-tile trigger candidates (Sec. II.C.2
// "Filtering and reconstruction", "Upsampling SNR segments", "Combining SNR
// segments"; the recursion of the pre-synchronisation equation, Sec. II.C.3).
//
// One work group = kMixTM = 128 real rows (64 templates) x kMixTN = 256
// top-rate samples of one bank and detector.  Levels run lowest rate first;
// level j covers the local window [lo_j + t0/P_j, +n_j): the tile plus the
// halo its upper level reads.  Per level:
//   acc = H_up(level j+1)                                           [MFMA]
//       + sum over slices at rate j of W~^s (rows) x y^s (window)   [MFMA]
// Level j >= 1 is kept in LDS for the next level; level 0 goes to the SNR
// series (interleaved re, im) and to the running trigger candidates.
//
// The contraction runs over chunks of K basis rows (32 for the 16-bit
// forms, 16 for FP32).  In the 16-bit forms the work group copies, per
// chunk, the y window of all its columns from the ring into an LDS stage
// with asynchronous buffer-to-LDS loads (two stages, in the level buffer,
// which is free while a level contracts), and every wave loads its W~
// fragments into registers, both one chunk ahead of the MFMAs.  The FP32
// form, whose four MFMAs per loaded K group already cover the loads, takes
// both operands straight from memory into registers.  The K elements a lane
// supplies (8 consecutive basis rows for the 16-bit forms, 4 for FP32) are
// one 16-byte access on either side, and both operands are stored so that
// the 16 lanes of a K group read 256 contiguous bytes: W~ in 16-row
// fragment order, the basis-output rings (and the stages) grouped by 16
// bytes of outputs with consecutive positions adjacent (layouts in
// MixSlice).  The 16-bit rings already hold y as hi + lo, split once when
// they are written.  The four waves split the tile 2 x 2: a wave owns the
// four 16-row blocks of one half of the rows and the column blocks cb = wc,
// wc + 2, ... of the window, so every y fragment it reads feeds four row
// blocks and every W~ fragment up to eight column blocks.
//
// The polyphase upsample is a banded contraction into the same accumulator:
// for the 16 output columns of a block starting at level index i0, with
// q0 = floor(i0/p) and lane column c (i = i0 + c, q = floor(i/p),
// ph = i mod p, off = q - q0),
//   H_up(prev)[r][c] = sum_k prev[r][q0 - N_up + k] Ker[k][c],
//   Ker[k][c] = z_ph[off + 2 N_up - k]  for off <= k <= off + 2 N_up, else 0,
// and for phase 0 Ker is the unit vector at k = off + N_up (the copy case of
// Eq. (upsample)).  off <= 7 and 2 N_up <= 16, so a 24- (FP32) or 32-wide
// (16-bit) window of prev holds every tap.  One LDS buffer holds a level
// (FP32, or hi and lo planes split once when the level is written, so that
// the 16-bit fragments are aligned vector reads).  In the 16-bit forms a
// level first adds the upsampled level j+1 into its accumulators, then
// (after a barrier) uses the buffer for its y stages, and finally
// overwrites it with level j; the FP32 form contracts first and upsamples
// after.
#include <hip/hip_runtime.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

typedef float f32x2 __attribute__((ext_vector_type(2)));

// The four waves tile the work group's kMixTM x kMixTN block as kWR x kWC:
// wave (wr, wc) owns rows wr kMixTM/kWR .. + kMixTM/kWR (kRB 16-row
// blocks) and the column blocks cb = wc, wc + kWC, ... (kCB of them).
constexpr int kWR = 2, kWC = 2;
constexpr int kRB = kMixTM / (16 * kWR);
constexpr int kCB = kMixTN / (16 * kWC);
constexpr int kCBH = kCB / 2;      // column blocks per operand load (direct-load form)

__device__ __forceinline__ float ker_value(int k, int off, int ph, int nup, const float *__restrict__ taps) {
    if (ph == 0) return k == off + nup ? 1.0f : 0.0f;
    const int t = off + 2 * nup - k;
    return (t >= 0 && t <= 2 * nup) ? taps[ph * kUpTaps + t] : 0.0f;
}

// b = the better of b and the candidate of the lane that DPP control CTRL
// selects (a permutation within each row of 16 lanes; VALU only)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ void reduce_dpp(PeakCand &b) {
    PeakCand o;
    o.p2 = __int_as_float(dpp_i<CTRL>(__float_as_int(b.p2)));
    o.idx = dpp_i<CTRL>(b.idx);
    o.re = __int_as_float(dpp_i<CTRL>(__float_as_int(b.re)));
    o.im = __int_as_float(dpp_i<CTRL>(__float_as_int(b.im)));
    if (better(o.p2, o.idx, b.p2, b.idx)) b = o;
}

// Polyphase position of lane column c of a block at level index i0 (the
// block's first output): q0 = floor(i0/p), off = floor(i/p) - q0, ph = i mod p.
// For p <= 16 a block start is a multiple of 16 past the level's window
// start lo, so off and ph depend on lo + c only and the kernel fragment of
// a lane is the same for every block of the level; the block's window of
// the lower level then starts at m0 = (16 / p) cb.
struct UpPos {
    int off, ph;
};
__device__ __forceinline__ UpPos up_pos(int i0, int c, int logp) {
    const int q0 = i0 >> logp;   // arithmetic shift: floor for negative indices
    const int ii = i0 + c;
    return UpPos{(ii >> logp) - q0, ii & ((1 << logp) - 1)};
}

// Per slice, a wave addresses W~ and its basis-output ring through buffer
// resources: per-lane byte offsets (row of W~, ring position of each of its
// column blocks, plus the lane group's K offset) are fixed for the slice and
// the step over basis rows is a scalar offset.
//
// ------------------------------------------------------------------ FP32
// 16 basis rows per step as four 16x16x4 MFMAs; lane group g supplies basis
// rows l0 + 4g .. l0 + 4g + 3, one per MFMA, on both sides.
struct MixF32 {
    static constexpr int K = 16;
    // FP32: the four MFMAs per loaded K group already cover the operand
    // loads; the direct-load contraction is faster than staging here
    static constexpr bool STAGED = false;
    struct Src {
        __amdgpu_buffer_rsrc_t w, y;
        int ys;                  // ring bytes per basis row step
        int va[kRB], vb[kCB];
    };
    struct FragA {
        float4 a[kRB];
    };
    struct FragB {
        float4 b[kCBH];
    };
    static __device__ __forceinline__ void init(Src &s, const MixSlice &ms, const void *ring, int r0, const int (&p)[kCB],
                                                int li, int lg) {
        // r0: first row of this wave (a multiple of 16)
        s.w = buffer_rsrc(ms.W, (uint32_t)ms.rows_pad * ms.Lpad * 4);
        s.y = buffer_rsrc(ring, (uint32_t)(2 * ms.capY) * ms.Lpad * 4);
        s.ys = 8 * ms.capY;
#pragma unroll
        for (int m = 0; m < kRB; ++m) s.va[m] = (((r0 >> 4) + m) * (ms.Lpad / 4) + lg) * 256 + 16 * li;
#pragma unroll
        for (int i = 0; i < kCB; ++i) s.vb[i] = (lg * 2 * ms.capY + p[i]) * 16;
    }
    static __device__ __forceinline__ void load_a(FragA &f, const Src &s, int l0) {
#pragma unroll
        for (int m = 0; m < kRB; ++m) f.a[m] = buffer_load16<float4>(s.w, s.va[m], l0 * 64);
    }
    static __device__ __forceinline__ void load_b(FragB &f, const Src &s, int l0, int i0) {
#pragma unroll
        for (int i = 0; i < kCBH; ++i) f.b[i] = buffer_load16<float4>(s.y, s.vb[i0 + i], l0 * s.ys);
    }
    static __device__ __forceinline__ void mma(floatx4 (&acc)[kCB][kRB], const FragA &a, const FragB &f, int i0,
                                               int ncb) {
#pragma unroll
        for (int i = 0; i < kCBH; ++i) {
            if (i0 + i >= ncb) continue;
#pragma unroll
            for (int m = 0; m < kRB; ++m) {
                acc[i0 + i][m] = mfma_16x16x4_f32(a.a[m].x, f.b[i].x, acc[i0 + i][m]);
                acc[i0 + i][m] = mfma_16x16x4_f32(a.a[m].y, f.b[i].y, acc[i0 + i][m]);
                acc[i0 + i][m] = mfma_16x16x4_f32(a.a[m].z, f.b[i].z, acc[i0 + i][m]);
                acc[i0 + i][m] = mfma_16x16x4_f32(a.a[m].w, f.b[i].w, acc[i0 + i][m]);
            }
        }
    }
    // level buffer: float [kMixTM][kMixS]
    static constexpr int LVL_BYTES = kMixTM * kMixS * 4;
    static __device__ __forceinline__ void lvl_store(void *lvl, int row, int col, float v) {
        static_cast<float *>(lvl)[row * kMixS + col] = v;
    }
    // 24-wide window, six K-steps of 4; lane group g holds Ker[4t + g][c]
    struct KerF {
        float b[6];
    };
    static __device__ __forceinline__ KerF ker(UpPos u, int nup, const float *taps, int lg) {
        KerF k;
#pragma unroll
        for (int t = 0; t < 6; ++t) k.b[t] = ker_value(4 * t + lg, u.off, u.ph, nup, taps);
        return k;
    }
    template <bool P2, int RB>
    static __device__ __forceinline__ void upsample(const void *lvl, int rw, int m0, int n_prev, const KerF &k,
                                                    int li, int lg, floatx4 (&acc)[RB]) {
        static_assert(RB == kRB, "the FP32 form keeps the 2 x 2 wave layout");
        const float *prev = static_cast<const float *>(lvl) + rw * kMixS;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int idx = min(m0 + 4 * t + lg, n_prev - 1);
#pragma unroll
            for (int m = 0; m < kRB; ++m) acc[m] = mfma_16x16x4_f32(prev[(16 * m + li) * kMixS + idx], k.b[t], acc[m]);
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
    static constexpr bool STAGED = true;   // y through LDS stages, W~ in registers ahead of the MFMAs
    static constexpr int PLANES = 2;       // ring planes: hi, lo
    static constexpr int RING_G = 8;       // ring outputs per 16-byte group
    template <int RB>
    static constexpr int a_loads = RB * (SPLIT_W ? 2 : 1);   // W~ loads per wave and chunk
    struct ASrc {
        __amdgpu_buffer_rsrc_t wh, wl;
        int va0;       // per lane: row block 0 of this wave, lane group's K offset
        int mstride;   // bytes from one 16-row block to the next (wave-uniform)
    };
    // W~ fragments of RB 16-row blocks
    template <int RB>
    struct FragA {
        T8 h[RB], l[SPLIT_W ? RB : 1];
    };
    struct FragB {
        T8 h, l;
    };
    static __device__ __forceinline__ void init_a(ASrc &s, const MixSlice &ms, int r0, int li, int lg) {
        const uint32_t wbytes = (uint32_t)ms.rows_pad * ms.Lpad * 2;
        s.wh = buffer_rsrc(ms.Whi, wbytes);
        if constexpr (SPLIT_W) s.wl = buffer_rsrc(ms.Wlo, wbytes);
        s.mstride = (ms.Lpad / 8) * 256;
        s.va0 = ((r0 >> 4) * (ms.Lpad / 8) + lg) * 256 + 16 * li;
    }
    template <int RB>
    static __device__ __forceinline__ void load_a(FragA<RB> &f, const ASrc &s, int l0) {
#pragma unroll
        for (int m = 0; m < RB; ++m) {
            f.h[m] = buffer_load16<T8>(s.wh, s.va0, l0 * 32 + m * s.mstride);
            if constexpr (SPLIT_W) f.l[m] = buffer_load16<T8>(s.wl, s.va0, l0 * 32 + m * s.mstride);
        }
    }
    // column block cb of an LDS stage [PLANES][4 groups][ncs][16 bytes]
    static __device__ __forceinline__ void read_b(FragB &f, const char *stage, int ncs, int cb, int li, int lg) {
        const char *p = stage + (lg * ncs + cb * 16 + li) * 16;
        f.h = *reinterpret_cast<const T8 *>(p);
        f.l = *reinterpret_cast<const T8 *>(p + 4 * ncs * 16);
    }
    template <int RB>
    static __device__ __forceinline__ void mma(floatx4 (&acc)[RB], const FragA<RB> &a, const FragB &f) {
#pragma unroll
        for (int m = 0; m < RB; ++m) {
            acc[m] = mfma16(a.h[m], f.l, acc[m]);
            if constexpr (SPLIT_W) acc[m] = mfma16(a.l[m], f.h, acc[m]);
            acc[m] = mfma16(a.h[m], f.h, acc[m]);
        }
    }
    // level buffer: T hi [kMixTM][SB] then T lo [kMixTM][SB], written once
    // per level as hi = T(v), lo = T(v - hi).  SB = 152: 304-byte rows keep
    // 16-byte fragments aligned, and the widest read (a level-1 window of
    // 145 plus the 8 columns an idle lane group re-reads) fits.
    static constexpr int SB = 152;
    static constexpr int LVL_BYTES = 2 * kMixTM * SB * 2;
    static __device__ __forceinline__ void lvl_store(void *lvl, int row, int col, float v) {
        T *hi = static_cast<T *>(lvl);
        const T h = (T)v;
        hi[row * SB + col] = h;
        hi[kMixTM * SB + row * SB + col] = (T)(v - (float)h);
    }
    // 32-wide window, one K-step; both operands split (three products), so
    // the interpolation keeps ~16 (bf16) or ~22 (fp16) significant bits.
    // Ker[k][c] is zero for k >= 24 (off <= 7), so lane group 3 re-reads
    // group 2's window (finite values) instead of columns past the row.
    struct KerF {
        T8 h, l;
    };
    static __device__ __forceinline__ KerF ker(UpPos u, int nup, const float *taps, int lg) {
        KerF k;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float kv = ker_value(8 * lg + j, u.off, u.ph, nup, taps);
            const T h = (T)kv;
            k.h[j] = h;
            k.l[j] = (T)(kv - (float)h);
        }
        return k;
    }
    // p = 2: m0 = 8 cb, so every window read is 16-byte aligned
    template <bool P2, int RB>
    static __device__ __forceinline__ void upsample(const void *lvl, int rw, int m0, int n_prev, const KerF &k,
                                                    int li, int lg, floatx4 (&acc)[RB]) {
        static_assert(P2, "16-bit fragment reads need p = 2");
        (void)n_prev;
        const T *hi = static_cast<const T *>(lvl);
        const int e = m0 + 8 * min(lg, 2);
#pragma unroll
        for (int m = 0; m < RB; ++m) {
            const T *ph = hi + (rw + 16 * m + li) * SB + e;
            const T8 ah = *reinterpret_cast<const T8 *>(ph);
            const T8 al = *reinterpret_cast<const T8 *>(ph + kMixTM * SB);
            acc[m] = mfma16(ah, k.l, acc[m]);
            acc[m] = mfma16(al, k.h, acc[m]);
            acc[m] = mfma16(ah, k.h, acc[m]);
        }
    }
    // any other ratio: a 24-wide window in six FP32 16x16x4 steps (as the
    // FP32 form), each level value read as hi + lo; lane group g holds
    // Ker[4t + g][c]
    struct KerF32 {
        float b[6];
    };
    static __device__ __forceinline__ KerF32 ker32(UpPos u, int nup, const float *taps, int lg) {
        KerF32 k;
#pragma unroll
        for (int t = 0; t < 6; ++t) k.b[t] = ker_value(4 * t + lg, u.off, u.ph, nup, taps);
        return k;
    }
    template <int RB>
    static __device__ __forceinline__ void upsample32(const void *lvl, int rw, int m0, int n_prev, const KerF32 &k,
                                                      int li, int lg, floatx4 (&acc)[RB]) {
        const T *hi = static_cast<const T *>(lvl);
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int idx = min(m0 + 4 * t + lg, n_prev - 1);
#pragma unroll
            for (int m = 0; m < RB; ++m) {
                const int o = (rw + 16 * m + li) * SB + idx;
                acc[m] = mfma_16x16x4_f32((float)hi[o] + (float)hi[kMixTM * SB + o], k.b[t], acc[m]);
            }
        }
    }
};

// Per slice of the staged (16-bit) contraction: the basis-output ring's
// buffer resource and per-lane offsets of the y copies, and W~'s operand source.
template <typename Op>
struct StageSrc {
    __amdgpu_buffer_rsrc_t ry;
    int plane;   // bytes per ring plane
    int cap16;   // bytes per K group of the ring
    int vbase;   // per lane: first copy; copy cq < nq - 1 adds 1024 cq
    int vlast;   // per lane: the last copy (clamped to the window)
    int Lpad;
    typename Op::ASrc as;
};

// ------------------------------------------------------------------ kernel
template <int V>
struct IntC {
    static constexpr int value = V;
};
// The lower levels' windows are at most kMixS columns: at most kCBL column
// blocks, which one wave of the lower levels' 4 x 1 layout holds for its two
// row blocks in 80 accumulator registers (instead of 128), so that a third
// pipeline stage fits (below).
constexpr int kCBL = (kMixS + 15) / 16;
// three lower-level stages (both planes, four K groups, the staged columns
// rounded up to 64) fit the level buffer
constexpr int kLowStageBytes = 2 * 4 * (((kMixS + 15) / 16 * 16 + 63) / 64) * 1024;
static_assert(3 * kLowStageBytes <= Mix16<__bf16, bf16x8, true>::LVL_BYTES, "three lower-level stages");
// two private stages per wave (both planes, four K groups, 64 columns)
static_assert(4 * 2 * 2 * 4 * 1024 <= Mix16<__bf16, bf16x8, true>::LVL_BYTES, "private lower-level stages");

// s_waitcnt vmcnt(N) (gfx9 encoding: low four bits and bits 15:14; the LDS
// and export counters left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

template <typename Op>
__global__ __launch_bounds__(256, 2) void mix_kernel(const MixItem *__restrict__ items, const MixBank *__restrict__ banks,
                                                  const MixSlice *__restrict__ slices,
                                                  const float *__restrict__ uptaps, float *__restrict__ series,
                                                  PartialPeak *__restrict__ partials, int32_t F, int32_t S,
                                                  int32_t nup, int32_t n_items, int32_t group,
                                                  const int64_t *__restrict__ stride_ctr) {
    extern __shared__ __attribute__((aligned(16))) char lds[];   // one level of the chain, then the bank's taps
    void *lvl = lds;
    __shared__ PeakCand wbest[4][8 * kRB];
    const int item = xcd_item(group);
    if (item >= n_items) return;
    const MixItem it = items[item];
    const MixBank &B = banks[it.bank];
    // ring positions are taken modulo capY, a power of two dividing 2^32
    const uint32_t kstr = (uint32_t)*stride_ctr;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar branches below
    const int wr = wave / kWC, wc = wave % kWC;
    const int rw = wr * (kMixTM / kWR);   // first row of this wave within the tile
    const int li = lane & 15, lg = lane >> 4;
    // the polyphase sub-kernels of every stage of the bank, read by the
    // upsampling (first used after the lowest level's barriers)
    float *tp = reinterpret_cast<float *>(lds + Op::LVL_BYTES);
    for (int j = 1; j < B.nlev; ++j) {
        const float *src = uptaps + (B.p[j] - 1) * kUpTaps;
        for (int e = tid; e < B.p[j] * kUpTaps; e += 256) tp[B.up_off[j] + e] = src[e];
    }
    // the upsampling reads a few columns past a level's window (weighted by
    // zero taps): the buffer starts as zeros and only ever holds finite values
    for (int e = tid; e < Op::LVL_BYTES / 16; e += 256) reinterpret_cast<uint4 *>(lds)[e] = uint4{0, 0, 0, 0};

    int lo_prev = 0;

    // acc += H_up(level j + 1), read from the LDS level buffer (levels below
    // the lowest); acc has NC column blocks cb = wc + kWC i.  Ratio p = 2 (the
    // usual octave step) takes aligned window reads and one kernel fragment
    // for every block of the level (block starts are multiples of 16 past the
    // window start); any other ratio takes element reads (hi + lo) into
    // FP32 products and the fragment of each block.  The FP32 form reads
    // elements at every ratio and shares the fragment for p <= 16.
    // A wave layout: first row ry of the wave's RB 16-row blocks (RB from
    // acc's type) and its column blocks cb = cb0 + cst i, i < NC.
    //
    // acc += H_up(level j + 1), read from the LDS level buffer (levels below
    // the lowest)
    auto upsample_level = [&](int j, int lo, int nb, auto &acc, int ry, int cb0, int cst) {
        constexpr int NC = sizeof(acc) / sizeof(acc[0]);
        constexpr int RB = sizeof(acc[0]) / sizeof(floatx4);
        if (j < B.nlev - 1) {
            const int logp = B.shp[j + 1];
            const float *taps = tp + B.up_off[j + 1];
            const int n_prev = B.n[j + 1];
            if constexpr (!Op::STAGED) {
                // FP32: one loop, the shared fragment for p <= 16
                const typename Op::KerF k0 = Op::ker(up_pos(lo, li, logp), nup, taps, lg);
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    const int cb = cb0 + cst * i;
                    if (cb >= nb) continue;   // wave-uniform
                    const int i0 = lo + cb * 16;
                    const int m0 = (i0 >> logp) - nup - lo_prev;
                    if (logp <= 4) {
                        Op::template upsample<false, RB>(lvl, ry, m0, n_prev, k0, li, lg, acc[i]);
                    } else {
                        const typename Op::KerF kb = Op::ker(up_pos(i0, li, logp), nup, taps, lg);
                        Op::template upsample<false, RB>(lvl, ry, m0, n_prev, kb, li, lg, acc[i]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else if (logp == 1) {
                const typename Op::KerF k0 = Op::ker(up_pos(lo, li, 1), nup, taps, lg);
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    const int cb = cb0 + cst * i;
                    if (cb >= nb) continue;   // wave-uniform
                    const int m0 = ((lo + cb * 16) >> 1) - nup - lo_prev;
                    Op::template upsample<true, RB>(lvl, ry, m0, n_prev, k0, li, lg, acc[i]);
                    __builtin_amdgcn_sched_barrier(0);   // keep one block's LDS reads in flight at a time
                }
            } else {
                // a rolled loop over the blocks (this path is rare: one copy
                // of its element reads instead of one per block); each block's
                // tile goes to its accumulators, still zero at this point, so
                // the sum is exact
                const int ncb = min(NC, max(0, (nb - cb0 + cst - 1) / cst));
#pragma unroll 1
                for (int i = 0; i < ncb; ++i) {
                    const int i0 = lo + (cb0 + cst * i) * 16;
                    const int m0 = (i0 >> logp) - nup - lo_prev;
                    const auto kb = Op::ker32(up_pos(i0, li, logp), nup, taps, lg);
                    floatx4 t[RB];
#pragma unroll
                    for (int m = 0; m < RB; ++m) t[m] = floatx4{0.f, 0.f, 0.f, 0.f};
                    Op::template upsample32<RB>(lvl, ry, m0, n_prev, kb, li, lg, t);
#pragma unroll
                    for (int q = 0; q < NC; ++q)
                        if (q == i)   // wave-uniform
#pragma unroll
                            for (int m = 0; m < RB; ++m) acc[q][m] += t[m];
                }
            }
        }
    };

    // level j >= 1: acc goes to the LDS level buffer for the next level up
    auto write_level = [&](int n, int nb, const auto &acc, int ry, int cb0, int cst) {
        constexpr int NC = sizeof(acc) / sizeof(acc[0]);
        constexpr int RB = sizeof(acc[0]) / sizeof(floatx4);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int cb = cb0 + cst * i;
            if (cb >= nb) continue;
            const int c = cb * 16 + li;
            if (c >= n) continue;
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) Op::lvl_store(lvl, ry + 16 * m + 4 * lg + v, c, acc[i][m][v]);
        }
    };

    // level 0: SNR series and trigger candidates.  Lane (li, lg) holds
    // templates t8 + 8 m + h, t8 = (r0 + rw)/2 + 2 lg, at the samples
    // t0 + cb 16 + li; one template's candidate is live at a time.
    auto epilogue = [&](int n, int nb, const auto &acc) {
        constexpr int NC = sizeof(acc) / sizeof(acc[0]);
        const int t8 = (it.r0 + rw) / 2 + 2 * lg;
        float2 *orow = series ? reinterpret_cast<float2 *>(series + B.series_off) +
                                    ((int64_t)it.det * B.M + t8) * F + it.t0 + li
                              : nullptr;
#pragma unroll
        for (int m = 0; m < kRB; ++m) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bool live = t8 + 8 * m + h < B.M;
                PeakCand b{-1.0f, 0x7fffffff, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    const int cb = wc + kWC * i;
                    if (cb >= nb) continue;
                    const int c = cb * 16 + li;
                    if (c >= n) continue;
                    const float re = acc[i][m][2 * h], im = acc[i][m][2 * h + 1];
                    // streamed past the caches: the series is never re-read by this
                    // launch and would otherwise evict W~ and the basis outputs
                    if (orow && live)
                        __builtin_nontemporal_store(f32x2{re, im},
                                                    reinterpret_cast<f32x2 *>(orow + (int64_t)(8 * m + h) * F + cb * 16));
                    const float p2 = re * re + im * im;
                    if (better(p2, it.t0 + c, b.p2, b.idx)) b = PeakCand{p2, it.t0 + c, re, im};
                }
                // reduce over the 16 lanes of the row group: pairs, quads,
                // half rows, rows (the order is total, so any butterfly gives
                // the same candidate)
                reduce_dpp<0xB1>(b);    // quad_perm 1, 0, 3, 2
                reduce_dpp<0x4E>(b);    // quad_perm 2, 3, 0, 1
                reduce_dpp<0x141>(b);   // row_half_mirror
                reduce_dpp<0x140>(b);   // row_mirror
                if (li == 0) wbest[wave][8 * m + 2 * lg + h] = b;
            }
        }
    };

    if constexpr (Op::STAGED) {
        // One level of the 16-bit forms: upsampled level j + 1 into the
        // accumulators, then the contraction over the chunks (slice s, basis
        // rows l0 .. l0 + K) of level j.  Each chunk's y window (ncs columns,
        // every group of the K rows, both planes) is copied by the work group
        // from the ring into one of DEPTH LDS stages (in the level buffer,
        // free while a level contracts) with asynchronous buffer-to-LDS loads,
        // and each wave's W~ fragments are loaded into one of DEPTH register
        // sets, DEPTH - 1 chunks ahead of the MFMAs: per chunk one wait (for
        // that chunk's loads only) and one barrier, then the loads of chunk
        // c + DEPTH - 1 go out (into the stage and registers chunk c - 1 used)
        // before chunk c's MFMAs.  The top level runs two stages (a 256-column
        // stage is 32 KB) and the 2 x 2 wave layout (each W~ fragment feeds up
        // to eight column blocks).  The lower levels, whose windows stage at
        // most 192 columns (24 KB), run three stages, so that their short
        // chunks overlap two chunks' load latency instead of one, and a 4 x 1
        // layout: wave w owns rows 32 w .. 32 w + 31 (two row blocks) and every
        // column block of the window, so each W~ fragment is loaded by one wave
        // only (in the 2 x 2 layout the two waves of a row half load the same
        // fragments, which at these few column blocks per chunk costs more
        // than the second read of each y fragment from LDS).  A lower level
        // whose window fits one 64-column copy (the rates an eighth of the
        // top rate and below) gives every wave two stages of its own, into
        // which it copies all four K groups itself: its chunks then wait for
        // their own loads only, with no barrier (four times the copies of
        // the small window, from the L2).
        auto staged_level = [&](int j, auto ncb_c, auto depth_c, auto top_c, auto priv_c) {
            constexpr int NC = decltype(ncb_c)::value;
            constexpr int DEPTH = decltype(depth_c)::value;
            constexpr bool TOP = decltype(top_c)::value;   // level 0
            // windows of at most 64 columns: every wave copies all four K
            // groups into DEPTH stages of its own, so a chunk needs its own
            // loads only (a wait, no barrier)
            constexpr bool PRIV = decltype(priv_c)::value;
            static_assert(!PRIV || (NC * 16 <= 64 && !TOP), "private stages: one 64-column copy");
            constexpr int RB = TOP ? kRB : kMixTM / 64;    // 16-row blocks per wave
            const int ry = TOP ? rw : 32 * wave;           // first row of this wave
            const int cb0 = TOP ? wc : 0, cst = TOP ? kWC : 1;
            const int lo = B.lo[j] + (it.t0 >> B.shP[j]);
            const int n = B.n[j];
            const int nb = (n + 15) >> 4;
            floatx4 acc[NC][RB];
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int m = 0; m < RB; ++m) acc[i][m] = floatx4{0.f, 0.f, 0.f, 0.f};
            // this wave's column blocks cb = cb0 + cst i, i < ncb
            const int ncb = min(NC, max(0, (nb - cb0 + cst - 1) / cst));
            upsample_level(j, lo, nb, acc, ry, cb0, cst);
            __syncthreads();   // every wave is done reading level j+1: the buffer now stages y
            {
                const int sb = B.slice_begin[j], se = B.slice_begin[j + 1];
                const int ncs = min(kMixTN, (nb * 16 + 63) & ~63);   // staged columns
                const int nq = ncs >> 6;                             // 64-column copies per plane and group
                const int stage_bytes = Op::PLANES * 4 * nq * 1024;  // DEPTH stages fit LVL_BYTES
                const int wbase = PRIV ? wave * DEPTH * stage_bytes : 0;   // this wave's stages (PRIV)
                const uint32_t rate = (uint32_t)B.rate[j];
                // Per slice (set up once when the issue cursor reaches it): the
                // ring's buffer resource and, per lane, the byte offset of each
                // of its (up to four) 64-column copies.  Wave w copies K group
                // w of every plane; the step over basis rows is the scalar
                // offset alone.
                using YCtx = StageSrc<Op>;
                auto prepare = [&](int sl, YCtx &c) {
                    const MixSlice &ms = slices[sl];
                    const uint32_t cap2 = 2u * (uint32_t)ms.capY;
                    const uint32_t pos0 = (kstr * rate + (uint32_t)lo) & (uint32_t)(ms.capY - 1);
                    const char *ring = static_cast<const char *>(ms.Y) + (int64_t)it.det * ms.ydet * 4;
                    const uint32_t plane = cap2 * (uint32_t)ms.Lpad * (16 / Op::RING_G);
                    c.plane = (int)plane;
                    c.ry = buffer_rsrc(ring, plane * Op::PLANES);
                    c.cap16 = (int)cap2 * 16;
                    // columns past the window re-read its last sample (finite,
                    // never stored): every copy stays inside the window, which is
                    // contiguous in the mirror ring (n <= capY, checked at plan time).
                    // Only the last copy can reach past it (n > ncs - 64).
                    const uint32_t g0 = (uint32_t)wave * cap2 + pos0;
                    c.vbase = (int)((g0 + (uint32_t)lane) * 16u);
                    c.vlast = (int)((g0 + (uint32_t)min((nq - 1) * 64 + lane, n - 1)) * 16u);
                    c.Lpad = ms.Lpad;
                    Op::init_a(c.as, ms, it.r0 + ry, li, lg);
                };
                // per wave and chunk: nq copies per plane, then the W~ loads
                auto issue = [&](const YCtx &c, int l0, int so, typename Op::template FragA<RB> &fa) {
                    // the builtin's operands are plain locals: taken straight from
                    // the struct, the host pass drops the kernel's instantiation
                    const int soff = (l0 / Op::RING_G) * c.cap16;
                    __amdgpu_buffer_rsrc_t ry = c.ry;
                    const int vb = c.vbase, vl = c.vlast, pln = c.plane, c16 = c.cap16;
                    typedef __attribute__((address_space(3))) void *lds_ptr;
                    if constexpr (PRIV) {
                        // one copy (nq = 1) per plane and K group g, from the
                        // group's ring rows (g cap16 bytes past group 0)
                        const int vl0 = vl - wave * c16;
#pragma unroll
                        for (int pl = 0; pl < Op::PLANES; ++pl)
#pragma unroll
                            for (int g = 0; g < 4; ++g)
                                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                    ry, (lds_ptr)(lds + wbase + so + (pl * 4 + g) * ncs * 16), 16, vl0,
                                    soff + pl * pln + g * c16, 0, 0);
                        Op::load_a(fa, c.as, l0);
                        return;
                    }
#pragma unroll
                    for (int pl = 0; pl < Op::PLANES; ++pl) {
                        char *dst = lds + so + (pl * 4 + wave) * ncs * 16;
                        const int sp = soff + pl * pln;
                        // copies 0 .. nq - 2 (wave-uniform count), then the last.  The
                        // immediate offset moves both the global and the LDS address.
                        if (nq > 1) __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)dst, 16, vb, sp, 0, 0);
                        if (nq > 2) __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)dst, 16, vb, sp, 1024, 0);
                        if (nq > 3) __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)dst, 16, vb, sp, 2048, 0);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)(dst + (nq - 1) * 1024), 16, vl, sp, 0, 0);
                    }
                    Op::load_a(fa, c.as, l0);
                };
                // wait until the chunk about to be used has landed, with
                // `ahead` later chunks (0 or 1) still in flight: loads return
                // in issue order, so the count allows exactly their loads
                auto wait_chunk = [&](int ahead) {
                    if (ahead == 0) wait_vmcnt<0>();
                    else if (PRIV) wait_vmcnt<2 * 4 + Op::template a_loads<RB>>();
                    else if (nq == 1) wait_vmcnt<2 * 1 + Op::template a_loads<RB>>();
                    else if (nq == 2) wait_vmcnt<2 * 2 + Op::template a_loads<RB>>();
                    else if (nq == 3) wait_vmcnt<2 * 3 + Op::template a_loads<RB>>();
                    else wait_vmcnt<2 * 4 + Op::template a_loads<RB>>();
                };
                if (sb < se) {
                    YCtx yc;   // the slice of the issue cursor
                    int is = sb, il = 0, issued = 0;
                    bool more = true;   // the cursor is at a chunk not yet issued
                    prepare(sb, yc);
                    auto advance = [&]() {
                        il += Op::K;
                        if (il >= yc.Lpad) {
                            ++is;
                            il = 0;
                            more = is < se;
                            if (more) prepare(is, yc);
                        }
                    };
                    typename Op::template FragA<RB> fa[DEPTH];
#pragma unroll
                    for (int p = 0; p < DEPTH - 1; ++p) {
                        if (more) {
                            issue(yc, il, p * stage_bytes, fa[p]);
                            ++issued;
                            advance();
                        }
                    }
                    // chunk c uses stage and register set u = c mod DEPTH; false
                    // once every chunk is consumed (wave-uniform)
                    int c = 0;
                    auto step = [&](auto u_c) -> bool {
                        constexpr int u = decltype(u_c)::value;
                        if (c >= issued) return false;
                        wait_chunk(issued - c - 1);
                        if constexpr (!PRIV) __syncthreads();   // ... for every wave; stage (c - 1) mod DEPTH is free
                        if (more) {
                            constexpr int q = (u + DEPTH - 1) % DEPTH;
                            issue(yc, il, q * stage_bytes, fa[q]);
                            ++issued;
                            advance();
                        }
                        const char *st = lds + wbase + u * stage_bytes;
#pragma unroll
                        for (int i = 0; i < NC; ++i) {
                            if (i >= ncb) break;   // wave-uniform
                            typename Op::FragB b;
                            Op::read_b(b, st, ncs, cb0 + cst * i, li, lg);
                            Op::mma(acc[i], fa[u], b);
                        }
                        ++c;
                        return true;
                    };
                    for (;;) {
                        if (!step(IntC<0>{})) break;
                        if (!step(IntC<1>{})) break;
                        if constexpr (DEPTH > 2)
                            if (!step(IntC<2>{})) break;
                    }
                }
            }
            __syncthreads();   // every wave is done reading the stages
            if constexpr (!TOP) {
                write_level(n, nb, acc, ry, cb0, cst);
                __syncthreads();   // level j complete before it is read as prev
                lo_prev = lo;
            } else {
                epilogue(n, nb, acc);
            }
        };
        for (int j = B.nlev - 1; j >= 1; --j) {   // 4 x 1
            if (B.n[j] <= 64)
                staged_level(j, IntC<4>{}, IntC<2>{}, IntC<0>{}, IntC<1>{});
            else
                staged_level(j, IntC<kCBL>{}, IntC<3>{}, IntC<0>{}, IntC<0>{});
        }
        staged_level(0, IntC<kCB>{}, IntC<2>{}, IntC<1>{}, IntC<0>{});
    } else {
        for (int j = B.nlev - 1; j >= 0; --j) {
            const int lo = B.lo[j] + (it.t0 >> B.shP[j]);
            const int n = B.n[j];
            const int nb = (n + 15) >> 4;
            floatx4 acc[kCB][kRB];
#pragma unroll
            for (int i = 0; i < kCB; ++i)
#pragma unroll
                for (int m = 0; m < kRB; ++m) acc[i][m] = floatx4{0.f, 0.f, 0.f, 0.f};
            // this wave's column blocks cb = wc + kWC i, i < ncb
            const int ncb = min(kCB, max(0, (nb - wc + kWC - 1) / kWC));
            // direct-load contraction: both operands straight into registers
            for (int s = B.slice_begin[j]; s < B.slice_begin[j + 1]; ++s) {
                const MixSlice &ms = slices[s];
                const uint32_t pos0 = (kstr * (uint32_t)B.rate[j] + (uint32_t)lo) & (uint32_t)(ms.capY - 1);
                const void *ring = static_cast<const char *>(ms.Y) + (int64_t)it.det * ms.ydet * 4;
                // columns past the window read its last sample (finite, never
                // stored); the window (n <= capY, checked at plan time) is
                // contiguous in the mirror ring, and the buffer range guards the rest
                int pc[kCB];
#pragma unroll
                for (int i = 0; i < kCB; ++i) pc[i] = (int)pos0 + min((wc + kWC * i) * 16 + li, n - 1);
                typename Op::Src src;
                Op::init(src, ms, ring, it.r0 + rw, pc, li, lg);
                // loads are unconditional: idle column blocks re-read the
                // window's last sample (L1 hits)
                for (int l0 = 0; l0 < ms.Lpad; l0 += Op::K) {
                    typename Op::FragA a;
                    typename Op::FragB b;
                    Op::load_a(a, src, l0);
                    Op::load_b(b, src, l0, 0);
                    Op::mma(acc, a, b, 0, ncb);
                    if (ncb > kCBH) {
                        Op::load_b(b, src, l0, kCBH);
                        Op::mma(acc, a, b, kCBH, ncb);
                    }
                }
            }
            upsample_level(j, lo, nb, acc, rw, wc, kWC);
            __syncthreads();   // every wave is done reading level j+1
            if (j > 0) {
                write_level(n, nb, acc, rw, wc, kWC);
                __syncthreads();   // level j complete before it is read as prev
                lo_prev = lo;
            } else {
                epilogue(n, nb, acc);
            }
        }
    }
    __syncthreads();
    // the kWC waves of a row group hold candidates of the same templates
    if (tid < kMixTM / 2) {
        const int g = tid / (8 * kRB), tl = tid % (8 * kRB);
        PeakCand b = wbest[g * kWC][tl];
        for (int w = 1; w < kWC; ++w) {
            const PeakCand o = wbest[g * kWC + w][tl];
            if (better(o.p2, o.idx, b.p2, b.idx)) b = o;
        }
        const int tmpl = it.r0 / 2 + tid;
        if (tmpl < B.M) {
            const int64_t pi = B.part_off + ((int64_t)it.det * B.M + tmpl) * B.n_ttiles + it.t0 / kMixTN;
            partials[pi] = PartialPeak{b.p2, b.idx, b.re, b.im};
        }
    }
}

size_t mix_lds(int precision, int S, int TP) {
    if (S != kMixS) return 0;
    switch (precision) {
        case LLOID_FP32: return (size_t)MixF32::LVL_BYTES + (size_t)TP * sizeof(float);
        case LLOID_BF16X3:
        case LLOID_FP8_BF16: return (size_t)Mix16<__bf16, bf16x8, true>::LVL_BYTES + (size_t)TP * sizeof(float);
        case LLOID_FP16: return (size_t)Mix16<_Float16, halfx8, false>::LVL_BYTES + (size_t)TP * sizeof(float);
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
                      PartialPeak *partials, int32_t F, int32_t n_det, int32_t S, int32_t TP, int32_t nup,
                      int32_t group) {
    (void)n_det;
    if (n_items == 0) return hipSuccess;
    const size_t lds = mix_lds(precision, S, TP);
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
