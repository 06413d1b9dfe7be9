// Per-slice basis correlation (Sec. II.C.2 "Filtering and reconstruction",
// with the integer read offsets of the pre-synchronisation equation,
// Sec. II.C.3):
//   Y[l][c] = sum_n U[l][n] d[k f + off + c + n]
// as a dense contraction on MFMA: A = U (rows l, K = taps), B = the Hankel
// window of the stream at the slice rate (K = taps, N = output columns).
//
// A work item is one slice and detector, up to kCorrMB x 16 = 64 basis
// rows, up to kCorrTQ = 512 output columns and one split of the taps.  Its
// four waves own the 16-column blocks cb = wave, wave + 4, ... of the item,
// so every basis fragment a wave reads from LDS feeds up to eight column
// blocks (and every strain fragment up to kCorrMB row blocks); the wide
// item spreads each stage's basis tile and barriers over many columns.  Taps advance in
// stages through two LDS buffers: while the current stage's MFMAs run from
// one, the next stage (fetched into registers during the previous stage) is
// stored into the other and the stage after it is fetched.
//
// Forms (the Op structs):
//   F32   v_mfma_f32_16x16x4_f32, one tap per lane and K group;
//   16-bit v_mfma_f32_16x16x32_{bf16,f16}, eight consecutive taps per lane:
//         a Hankel fragment d[q + n .. q + n + 7] starts at any element, so
//         the strain segment is staged as 8 copies shifted by 0..7 and read
//         from copy (q + n) mod 8 at an aligned offset; the strain is split
//         on the fly, d = d_hi + d_lo;
//           SPLIT_U (bf16x3): U_hi d_lo + U_lo d_hi + U_hi d_hi
//           otherwise (fp16): U d_lo + U d_hi
//   FP8   v_mfma_f32_16x16x128_f8f6f4 on e4m3 operands (OCP e4m3 on gfx950,
//         128 taps per instruction): the basis rows
//         hold e4m3(u_l 2^e_l) with one power-of-two scale per basis vector
//         (largest |u| near the e4m3 maximum 448), the strain is scaled by
//         kFp8StrainScale and split into two e4m3 parts; outputs are
//         rescaled by uscale[l] = 2^-e_l / kFp8StrainScale.
// The partial sums of a split go to part[l * f + c]; the reduction adds the
// splits in a fixed order.  A slice with one split writes its outputs
// straight into the basis-output ring instead (four consecutive basis
// outputs of a sample per lane, inside one 16-byte group; hi and lo planes
// for the 16-bit forms).  The prefetch registers use plain vector types:
// HIP's uint4 / float4 are union-based structs that the compiler does not
// promote to registers, which put them in scratch memory.
#include <hip/hip_runtime.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

constexpr int kCB = kCorrTQ / 64;   // column blocks per wave (four waves); the FP8 form: kCorrTQ8 / 64

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr float kFp8StrainScale = 8.0f;

__device__ __forceinline__ uint32_t fp8_byte(float v) {
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xffu;
}
__device__ __forceinline__ float fp8_value(uint32_t b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }

// strain samples of a stage: TQ + TK (+ 8 for the shifted copies)
template <int TK, int TQ = kCorrTQ>
struct StrainRegs {
    static constexpr int N = TQ + TK;
    static constexpr int PER = (N + 255) / 256;
    float v[PER];
    // samples past the item's columns + the stage's taps are never used:
    // zeros, unread (taps < TK when a stage reaches past the item's end)
    __device__ __forceinline__ void load(const CorrItem &it, int64_t p0, int tid, int taps = TK) {
        const int lim = min(N, it.ncols + taps);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            v[i] = e < lim ? ld_global<float>(it.ring + p0 + e) : 0.0f;   // mirror ring: p0 + e < 2 cap
        }
    }
};

// ------------------------------------------------------------------ FP32
struct CorrF32 {
    static constexpr int CB = kCB;
    static constexpr int TK = 32;
    static constexpr int US = TK + 2;   // 16 rows x 2 taps of a half-wave in distinct banks
    struct Smem {
        float U[kCorrMB * 16 * US];
        float d[kCorrTQ + TK];
    };
    static constexpr int PER = kCorrMB * 16 * (TK / 4) / 256;
    struct Regs {
        f32x4 u[PER];   // plain vector type: promoted to registers (HIP's float4 is not)
        StrainRegs<TK> d;
    };
    static __device__ __forceinline__ void gload(Regs &g, const CorrItem &it, int64_t p0, int kk, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 4), c4 = e % (TK / 4);
            if (r < it.mb * 16)
                g.u[i] = ld_global<f32x4>(it.U + (int64_t)(it.r0 + r) * it.Npad + it.k0 + kk + 4 * c4);
        }
        g.d.load(it, p0, tid);
    }
    static __device__ __forceinline__ void lstore(const Regs &g, Smem &s, const CorrItem &it, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 4), c4 = e % (TK / 4);
            if (r < it.mb * 16) {
                float *u = &s.U[r * US + 4 * c4];
                u[0] = g.u[i].x;
                u[1] = g.u[i].y;
                u[2] = g.u[i].z;
                u[3] = g.u[i].w;
            }
        }
#pragma unroll
        for (int i = 0; i < StrainRegs<TK>::PER; ++i) {
            const int e = tid + 256 * i;
            if (e < StrainRegs<TK>::N) s.d[e] = g.d.v[i];
        }
    }
    static __device__ __forceinline__ void compute(const Smem &s, floatx4 (&acc)[kCorrMB][CB], int mb, int ncb,
                                                   int wave, int li, int lg) {
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            float b[kCB];
#pragma unroll
            for (int i = 0; i < kCB; ++i) b[i] = s.d[(wave + 4 * i) * 16 + li + ks + lg];
#pragma unroll
            for (int m = 0; m < kCorrMB; ++m) {
                if (m >= mb) continue;
                const float a = s.U[(m * 16 + li) * US + ks + lg];
#pragma unroll
                for (int i = 0; i < kCB; ++i)
                    if (i < ncb) acc[m][i] = mfma_16x16x4_f32(a, b[i], acc[m][i]);
            }
        }
    }
    static __device__ __forceinline__ float scale(const CorrItem &, int) { return 1.0f; }
    using RingT = float;
};

// ---------------------------------------------------------------- 16-bit
template <typename T, typename T8, bool SPLIT_U>
struct Corr16 {
    static constexpr int CB = kCB;
    static constexpr int TK = 64;
    static constexpr int US = TK + 8;   // 144 B rows: 16-B fragment reads of a half-wave in distinct banks
    static constexpr int DL = kCorrTQ + TK + 8;
    struct Smem {
        T Uh[kCorrMB * 16 * US];
        T Ul[SPLIT_U ? kCorrMB * 16 * US : 8];
        T Dh[8 * DL];
        T Dl[8 * DL];
    };
    static constexpr int PER = kCorrMB * 16 * (TK / 8) / 256;
    // strain of a stage by sample pairs: pair p = tid + 256 i holds d[2p],
    // d[2p + 1] and the next sample d[2p + 2]
    static constexpr int NS = kCorrTQ + TK, NP = NS / 2, PPER = (NP + 255) / 256;
    struct Regs {
        u32x4 uh[PER], ul[SPLIT_U ? PER : 1];   // plain vector type: promoted to registers (HIP's uint4 is not)
        float d[PPER][3];
    };
    static __device__ __forceinline__ void gload(Regs &g, const CorrItem &it, int64_t p0, int kk, int tid) {
        const T *gh = static_cast<const T *>(it.Uhi);
        const T *gl = static_cast<const T *>(it.Ulo);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 8), c8 = e % (TK / 8);
            if (r < it.mb * 16) {
                const int64_t o = (int64_t)(it.r0 + r) * it.Npad + it.k0 + kk + 8 * c8;
                g.uh[i] = ld_global<u32x4>(gh + o);
                if constexpr (SPLIT_U) g.ul[i] = ld_global<u32x4>(gl + o);
            }
        }
        // samples past the item's columns + the stage's taps are never used: zeros
        const int lim = min(NS, it.ncols + TK);
#pragma unroll
        for (int i = 0; i < PPER; ++i) {
            const int e0 = 2 * (tid + 256 * i);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                g.d[i][q] = e0 + q < lim ? ld_global<float>(it.ring + p0 + e0 + q) : 0.0f;   // mirror ring
        }
    }
    static __device__ __forceinline__ void lstore(const Regs &g, Smem &s, const CorrItem &it, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 8), c8 = e % (TK / 8);
            if (r < it.mb * 16) {
                *reinterpret_cast<u32x4 *>(&s.Uh[r * US + 8 * c8]) = g.uh[i];
                if constexpr (SPLIT_U) *reinterpret_cast<u32x4 *>(&s.Ul[r * US + 8 * c8]) = g.ul[i];
            }
        }
        // copy sft holds d[i + sft] at position i.  Pair p writes whole
        // words: word p - s (positions 2p - 2s, + 1) of copy 2s is d[2p],
        // d[2p + 1] and of copy 2s + 1 is d[2p + 1], d[2p + 2]; consecutive
        // lanes write consecutive words (distinct banks)
        typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int k = 0; k < PPER; ++k) {
            const int p = tid + 256 * k;
            if (p >= NP) continue;
            T h[3], l[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                h[q] = (T)g.d[k][q];
                l[q] = (T)(g.d[k][q] - (float)h[q]);
            }
            const uint32_t he = __builtin_bit_cast(uint32_t, T2{h[0], h[1]});
            const uint32_t le = __builtin_bit_cast(uint32_t, T2{l[0], l[1]});
            const uint32_t ho = __builtin_bit_cast(uint32_t, T2{h[1], h[2]});
            const uint32_t lo = __builtin_bit_cast(uint32_t, T2{l[1], l[2]});
#pragma unroll
            for (int sh = 0; sh < 4; ++sh) {
                const int w = p - sh;
                if (w < 0) continue;
                *reinterpret_cast<uint32_t *>(&s.Dh[2 * sh * DL + 2 * w]) = he;
                *reinterpret_cast<uint32_t *>(&s.Dl[2 * sh * DL + 2 * w]) = le;
                *reinterpret_cast<uint32_t *>(&s.Dh[(2 * sh + 1) * DL + 2 * w]) = ho;
                *reinterpret_cast<uint32_t *>(&s.Dl[(2 * sh + 1) * DL + 2 * w]) = lo;
            }
        }
    }
    static __device__ __forceinline__ void compute(const Smem &s, floatx4 (&acc)[kCorrMB][CB], int mb, int ncb,
                                                   int wave, int li, int lg) {
#pragma unroll
        for (int ks = 0; ks < TK; ks += 32) {
            T8 bh[kCB], bl[kCB];
#pragma unroll
            for (int i = 0; i < kCB; ++i) {
                const int idx = (wave + 4 * i) * 16 + li + ks + 8 * lg;
                const int sft = idx & 7;
                bh[i] = *reinterpret_cast<const T8 *>(&s.Dh[sft * DL + idx - sft]);
                bl[i] = *reinterpret_cast<const T8 *>(&s.Dl[sft * DL + idx - sft]);
            }
#pragma unroll
            for (int m = 0; m < kCorrMB; ++m) {
                if (m >= mb) continue;
                const int off = (m * 16 + li) * US + ks + 8 * lg;
                const T8 ah = *reinterpret_cast<const T8 *>(&s.Uh[off]);
                T8 al;
                if constexpr (SPLIT_U) al = *reinterpret_cast<const T8 *>(&s.Ul[off]);
#pragma unroll
                for (int i = 0; i < kCB; ++i) {
                    if (i >= ncb) continue;
                    acc[m][i] = mfma16(ah, bl[i], acc[m][i]);
                    if constexpr (SPLIT_U) acc[m][i] = mfma16(al, bh[i], acc[m][i]);
                    acc[m][i] = mfma16(ah, bh[i], acc[m][i]);
                }
            }
        }
    }
    static __device__ __forceinline__ float scale(const CorrItem &, int) { return 1.0f; }
    using RingT = T;
};

// ------------------------------------------------------------------ FP8
// v_mfma_f32_16x16x128_f8f6f4 with both operands e4m3 (no block scales):
// 128 taps per MFMA, lane group g supplying taps 32 g .. 32 g + 31 of its row
// (A) or column (B) as 32 bytes.  A stage is 128 taps; its tap range past
// the item's end (a split of 64 x odd taps) reads as zero on both sides.
struct Corr8 {
    static constexpr int CB = kCorrTQ8 / 64;   // 256 columns per item: the accumulators of 128-tap fragments fit
    static constexpr int TK = 128;
    static constexpr int US = TK + 16;   // bytes per basis row (16-byte aligned rows)
    static constexpr int DL = kCorrTQ8 + TK + 8;
    struct Smem {
        uint8_t U[kCorrMB * 16 * US];
        uint8_t Dh[8 * DL];
        uint8_t Dl[8 * DL];
    };
    static constexpr int PER = kCorrMB * 16 * (TK / 8) / 256;
    struct Regs {
        u32x2 u[PER];
        StrainRegs<TK, kCorrTQ8> d;
    };
    static __device__ __forceinline__ void gload(Regs &g, const CorrItem &it, int64_t p0, int kk, int tid) {
        const uint8_t *gu = static_cast<const uint8_t *>(it.Uhi);
        const int kmax = it.klen - kk;   // taps of this stage inside the item
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 8), c8 = e % (TK / 8);
            g.u[i] = u32x2{0u, 0u};
            if (r < it.mb * 16 && 8 * c8 < kmax)
                g.u[i] = ld_global<u32x2>(gu + (int64_t)(it.r0 + r) * it.Npad + it.k0 + kk + 8 * c8);
        }
        g.d.load(it, p0, tid, min(TK, kmax));
    }
    static __device__ __forceinline__ void lstore(const Regs &g, Smem &s, const CorrItem &it, int tid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (TK / 8), c8 = e % (TK / 8);
            if (r < it.mb * 16) *reinterpret_cast<u32x2 *>(&s.U[r * US + 8 * c8]) = g.u[i];
        }
        // one byte per sample and copy
#pragma unroll
        for (int k = 0; k < StrainRegs<TK, kCorrTQ8>::PER; ++k) {
            const int e = tid + 256 * k;
            if (e >= StrainRegs<TK, kCorrTQ8>::N) continue;
            // saturate at the e4m3 maximum (whitened samples beyond 56 sigma)
            const float v = fminf(fmaxf(g.d.v[k] * kFp8StrainScale, -448.0f), 448.0f);
            const uint32_t h = fp8_byte(v);
            const uint32_t l = fp8_byte(v - fp8_value(h));
#pragma unroll
            for (int sft = 0; sft < 8; ++sft) {
                const int i = e - sft;
                if (i >= 0) {
                    s.Dh[sft * DL + i] = (uint8_t)h;
                    s.Dl[sft * DL + i] = (uint8_t)l;
                }
            }
        }
    }
    // 32 bytes of a shifted strain copy starting at element idx (8-byte aligned reads)
    static __device__ __forceinline__ i32x8 hankel32(const uint8_t *D, int idx) {
        const int sft = idx & 7;
        typedef int i32x2 __attribute__((ext_vector_type(2)));
        const i32x2 *p = reinterpret_cast<const i32x2 *>(&D[sft * DL + idx - sft]);
        const i32x2 a = p[0], b = p[1], c = p[2], d = p[3];
        return i32x8{a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
    }
    static __device__ __forceinline__ void compute(const Smem &s, floatx4 (&acc)[kCorrMB][CB], int mb, int ncb,
                                                   int wave, int li, int lg) {
        i32x8 a[kCorrMB];
#pragma unroll
        for (int m = 0; m < kCorrMB; ++m) {
            if (m >= mb) continue;
            a[m] = *reinterpret_cast<const i32x8 *>(&s.U[(m * 16 + li) * US + 32 * lg]);   // 16-byte aligned
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            if (i >= ncb) continue;
            const int idx = (wave + 4 * i) * 16 + li + 32 * lg;
            const i32x8 bh = hankel32(s.Dh, idx), bl = hankel32(s.Dl, idx);
#pragma unroll
            for (int m = 0; m < kCorrMB; ++m) {
                if (m >= mb) continue;
                acc[m][i] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[m], bl, acc[m][i], 0, 0, 0, 0, 0, 0);
                acc[m][i] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[m], bh, acc[m][i], 0, 0, 0, 0, 0, 0);
            }
        }
    }
    static __device__ __forceinline__ float scale(const CorrItem &it, int row) { return ld_global<float>(it.uscale + it.r0 + row); }
    using RingT = __bf16;   // the FP8 form mixes in BF16x3
};

// Four consecutive basis outputs row .. row + 3 (row a multiple of 4, so
// inside one 16-byte group) of one sample into the basis-output ring at
// position pos and its mirror pos + capY: FP32, or hi and lo planes.
template <typename T>
__device__ __forceinline__ void ring_store4(void *ring, int64_t pos, int row, int Lpad, int capY, float4 v) {
    const int64_t o = ring_index<16 / sizeof(T)>(pos, row, capY), om = ring_index<16 / sizeof(T)>(pos + capY, row, capY);
    if constexpr (sizeof(T) == 4) {
        float *r = static_cast<float *>(ring);
        *reinterpret_cast<float4 *>(r + o) = v;
        *reinterpret_cast<float4 *>(r + om) = v;
    } else {
        typedef T T4 __attribute__((ext_vector_type(4)));
        const float x[4] = {v.x, v.y, v.z, v.w};
        T4 h, l;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h[i] = (T)x[i];
            l[i] = (T)(x[i] - (float)h[i]);
        }
        T *hi = static_cast<T *>(ring);
        T *lo = hi + 2LL * capY * Lpad;
        *reinterpret_cast<T4 *>(hi + o) = h;
        *reinterpret_cast<T4 *>(hi + om) = h;
        *reinterpret_cast<T4 *>(lo + o) = l;
        *reinterpret_cast<T4 *>(lo + om) = l;
    }
}

// ------------------------------------------------------------------ kernel
template <typename Op>
__global__ __launch_bounds__(256, 2) void corr_kernel(const CorrItem *__restrict__ items, int32_t n_items,
                                                      int32_t group, const int64_t *__restrict__ stride_ctr) {
    __shared__ __attribute__((aligned(16))) typename Op::Smem sm[2];
    const int item = xcd_item(group);
    if (item >= n_items) return;
    const CorrItem it = items[item];
    const int64_t kstr = *stride_ctr;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    // this wave's column blocks cb = wave + 4 i, i < ncb
    constexpr int CB = Op::CB;
    const int ncb = min(CB, max(0, (((it.ncols + 15) >> 4) - wave + 3) >> 2));

    floatx4 acc[kCorrMB][CB];
#pragma unroll
    for (int m = 0; m < kCorrMB; ++m)
#pragma unroll
        for (int i = 0; i < CB; ++i) acc[m][i] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int64_t dbase = kstr * it.f + it.off + it.col0 + it.k0;
    // Two LDS stage buffers: stage k is computed from buffer k mod 2 while
    // stage k + 1 is stored into the other one and stage k + 2 is fetched
    // into registers, one barrier per stage.
    typename Op::Regs g;
    Op::gload(g, it, posmod(dbase, it.cap), 0, tid);
    Op::lstore(g, sm[0], it, tid);
    if (Op::TK < it.klen) Op::gload(g, it, posmod(dbase + Op::TK, it.cap), Op::TK, tid);
    int buf = 0;
    for (int kk = 0; kk < it.klen; kk += Op::TK) {
        __syncthreads();   // stage kk is in sm[buf]; every wave is done reading sm[buf ^ 1]
        if (kk + Op::TK < it.klen) {
            Op::lstore(g, sm[buf ^ 1], it, tid);
            if (kk + 2 * Op::TK < it.klen)
                Op::gload(g, it, posmod(dbase + kk + 2 * Op::TK, it.cap), kk + 2 * Op::TK, tid);
        }
        // the stage's matrix products at raised wave priority, so that the
        // scheduler favours the waves feeding the matrix cores over those
        // still storing or loading a stage (1 % on the batched workload)
        __builtin_amdgcn_s_setprio(1);
        Op::compute(sm[buf], acc, it.mb, ncb, wave, li, lg);
        __builtin_amdgcn_s_setprio(0);
        buf ^= 1;
    }
    const int64_t q0 = kstr * it.f + it.la + it.col0;
#pragma unroll
    for (int i = 0; i < CB; ++i) {
        if (i >= ncb) continue;
        const int c = (wave + 4 * i) * 16 + li;
        if (c >= it.ncols) continue;
#pragma unroll
        for (int m = 0; m < kCorrMB; ++m) {
            if (m >= it.mb) continue;
            const int r = m * 16 + lg * 4;   // this lane's 4 consecutive rows
            const float4 v = make_float4(acc[m][i][0] * Op::scale(it, r), acc[m][i][1] * Op::scale(it, r + 1),
                                         acc[m][i][2] * Op::scale(it, r + 2), acc[m][i][3] * Op::scale(it, r + 3));
            if (it.yring) {
                ring_store4<typename Op::RingT>(it.yring, (q0 + c) & (it.capY - 1), it.r0 + r, it.Lpad, it.capY, v);
            } else {
                float *p = it.part + (int64_t)(it.r0 + r) * it.f + it.col0 + c;
                p[0] = v.x;
                p[it.f] = v.y;
                p[2 * it.f] = v.z;
                p[3 * it.f] = v.w;
            }
        }
    }
}

// Basis rows to e4m3 with a power-of-two scale per row: one block per row,
// e = floor(log2(448 / max|u|)); dst = e4m3(u 2^e); scale[r] = 2^-e / kFp8StrainScale.
__global__ __launch_bounds__(256) void convert_fp8_rows_kernel(const double *__restrict__ src, int32_t cols,
                                                               int32_t src_ld, uint8_t *__restrict__ dst,
                                                               int32_t dst_ld, float *__restrict__ scale) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    double mx = 0.0;
    for (int c = threadIdx.x; c < cols; c += 256) mx = fmax(mx, fabs(src[(int64_t)r * src_ld + c]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const int e = red[0] > 0.0 ? (int)floor(log2(448.0 / red[0])) : 0;
    const double s = ldexp(1.0, e);
    for (int c = threadIdx.x; c < cols; c += 256)
        dst[(int64_t)r * dst_ld + c] = (uint8_t)fp8_byte((float)(src[(int64_t)r * src_ld + c] * s));
    if (threadIdx.x == 0) scale[r] = (float)(ldexp(1.0, -e) / kFp8StrainScale);
}

hipError_t launch_convert_fp8_rows(hipStream_t st, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                                   uint8_t *dst, int32_t dst_ld, float *scale) {
    hipLaunchKernelGGL(convert_fp8_rows_kernel, dim3(rows), dim3(256), 0, st, src, cols, src_ld, dst, dst_ld, scale);
    return hipGetLastError();
}

hipError_t launch_corr(const LaunchCtx &ctx, int precision, const CorrItem *items, int32_t n_items, int32_t group) {
    if (n_items == 0) return hipSuccess;
    const dim3 grid(xcd_grid(n_items, group));
    switch (precision) {
        case LLOID_FP32:
            hipLaunchKernelGGL(corr_kernel<CorrF32>, grid, dim3(256), 0, ctx.stream, items, n_items, group,
                               ctx.stride_ctr);
            break;
        case LLOID_FP8_BF16:
            hipLaunchKernelGGL(corr_kernel<Corr8>, grid, dim3(256), 0, ctx.stream, items, n_items, group,
                               ctx.stride_ctr);
            break;
        case LLOID_BF16X3:
            hipLaunchKernelGGL((corr_kernel<Corr16<__bf16, bf16x8, true>>), grid, dim3(256), 0, ctx.stream, items,
                               n_items, group, ctx.stride_ctr);
            break;
        case LLOID_FP16:
            hipLaunchKernelGGL((corr_kernel<Corr16<_Float16, halfx8, false>>), grid, dim3(256), 0, ctx.stream, items,
                               n_items, group, ctx.stride_ctr);
            break;
        default:
            return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace lloid
