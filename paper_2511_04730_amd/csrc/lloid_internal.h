// Internal layout shared by the host plan (lloid_plan.hip) and the device
// kernels (lloid_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lloid.h"

namespace lloid {

// ---------------------------------------------------------------- constants
constexpr int kMaxLevels = 12;        // distinct rates per bank (top included)
constexpr int kMaxBasis = 160;        // L^s limit, and per bank and rate (ABI)
constexpr int kCorrTQ = 512;          // correlation item: output columns (128 per wave)
constexpr int kCorrTQ8 = 256;         // ... in the FP8 form (64 per wave)
constexpr int kCorrMB = 4;            // correlation item: 16-row blocks of basis vectors
constexpr int kCorrTK = 64;           // tap padding of the basis rows
constexpr int kCorrSplitK = 512;      // taps per correlation work item
constexpr int kMixTM = 128;           // mixing tile: real rows (64 templates)
constexpr int kMixTN = 256;           // mixing tile: top-rate samples
constexpr int kUpTaps = 17;           // 2 N_up + 1 taps per polyphase branch
// mixing level-buffer row stride (floats): at least the widest window of a
// lower level, kMixTN / 2 + 2 N_up + 1 <= 145, and 18 mod 32 (the
// upsampling's 16 rows x 2 columns per half-wave fall in distinct banks)
constexpr int kMixS = 146;
constexpr int kMaxLdsBytes = 96 * 1024;   // dynamic LDS per work group we allow (160 KB on gfx950)
constexpr int kXcds = 8;              // accelerator complex dies of the MI355X

// grid length for xcd_item(): whole rounds of kXcds groups
inline int xcd_grid(int n_items, int group) {
    if (group <= 0) return n_items;
    const int round = kXcds * group;
    return (n_items + round - 1) / round * round;
}

// -------------------------------------------------------------- work items
// Basis correlation (Sec. II.C.2 "Filtering and reconstruction"):
//   y_l[q] = sum_n u_l[n] d[q + n + off],  off = -delay - (N-1)
// for the f new columns q = k f + la + c, c in [col0, col0+ncols), basis
// rows l in [r0, r0 + 16 mb), taps n in [k0, k0+klen).  The partial result
// goes to part[l * f + c].
struct CorrItem {
    const float *U;          // [Lpad][Npad] fp32 (FP32 mode)
    const void *Uhi;         // reduced-precision basis, [Lpad][Npad]
    const void *Ulo;         // low part (BF16X3) or nullptr
    const float *ring;       // stream at the slice rate for this detector (mirror ring)
    float *part;             // partial [Lpad][f] for this split
    const float *uscale;     // FP8: per-row scale or nullptr
    int64_t off;             // la - delay - (N - 1)  (index = k f + off + c + n)
    int32_t Npad, Lpad, cap, f;
    int32_t col0, ncols, k0, klen;
    int32_t mb;              // 16-row blocks of this item (<= kCorrMB)
    int32_t r0;              // first basis row of this item
    // one tap split: the outputs go straight to the basis-output ring (see
    // MixSlice; new columns q = k f + la + c) instead of a partial plane
    void *yring;             // ring of this detector, or nullptr
    int32_t capY, la;
};

// Deterministic split-K reduction of 64 new columns x 32 basis rows
// [l0, l0 + 32) of one slice and detector into its basis-output ring
// (see MixSlice for the layout).
struct ReduceItem {
    const float *part;       // [nsplit][Lpad][f]
    void *yring;             // ring of this detector
    int32_t nsplit, L, Lpad, f, capY, la, c0, l0;
};

// Decimation (Eq. (sinc) kernel, zero phase): d_D[m] = sum_t g[t] x[D m + t - c]
// for m in [k f - n_down + m0, ... + chunk).
struct DownItem {
    const float *xring;      // top-rate mirror ring of this detector
    float *dring;            // output mirror ring at rate F/D
    const float *taps;       // 2c+1 taps
    int32_t D, c, f, m0, chunk, capx, capd, n_down;
};

// Mixing + upsample-and-add (Sec. II.C.2 "Upsampling", "Combining", Sec. II.C.3).
// Basis-output ring of a slice and detector: a mirror ring of 2 capY
// positions (capY a power of two; position q at q mod capY and
// q mod capY + capY) holding the Lpad basis outputs of each sample, in
// 16-byte groups of G = 16 / sizeof(T) consecutive outputs: group g of every
// position comes before group g + 1, i.e. element (pos, l) of a plane is at
//   ((l / G) 2 capY + pos) G + l mod G
// so the 16-byte MFMA fragments of 16 consecutive positions are 256
// contiguous bytes.
//   FP32 form:    one float plane (G = 4)
//   16-bit forms: T hi plane, then T lo plane, y = hi + lo (G = 8)
// Either way 4 bytes per element; ydet counts 4-byte elements.
// The mixing rows are stored in fragment order: 16 x G tiles of the
// [rows_pad][Lpad] matrix, tile (r / 16, l / G) at ((r / 16) (Lpad / G) +
// l / G) 16 G, row-major inside, so that one K group of a 16-row fragment
// is 256 contiguous bytes.
struct MixSlice {
    const float *W;          // fp32 normalised mixing rows (fragment order)
    const void *Whi;         // reduced precision
    const void *Wlo;
    const void *Y;           // basis-output ring of detector 0
    int64_t ydet;            // 4-byte elements between detectors' rings
    int32_t L, Lpad, capY, level;
    int32_t rows_pad;        // rows of W (a multiple of kMixTM)
    int32_t pad_;
};

struct MixBank {
    int32_t M;               // complex templates
    int32_t nlev;            // levels 0..nlev-1 (0 = top rate)
    int32_t rate[kMaxLevels];
    int32_t P[kMaxLevels];       // decimation of the level w.r.t. the top rate
    int32_t shP[kMaxLevels];     // log2 P
    int32_t p[kMaxLevels];       // p[j] = rate[j-1] / rate[j] (j >= 1)
    int32_t shp[kMaxLevels];     // log2 p
    int32_t lo[kMaxLevels];      // window start of tile t0 = 0, local index
    int32_t n[kMaxLevels];       // window length
    int32_t up_off[kMaxLevels];  // offset of stage j's sub-kernels in the bank's LDS tap copy
    int32_t slice_begin[kMaxLevels + 1];  // MixSlice range per level
    int64_t series_off;          // float offset of the bank's series block
    int64_t peak_off;            // entry offset of the bank's peak block
    int64_t part_off;            // offset of the bank's partial peaks
    int32_t n_ttiles;
    int32_t pad_;
};

struct MixItem {
    int32_t bank, det, r0, t0;
};

struct PartialPeak {
    float p2;                // max |z|^2
    int32_t idx;             // in-stride index
    float re, im;
};

struct PeakItem {
    int64_t part_off;        // first partial of this bank/detector
    int64_t peak_off;        // first output entry
    int32_t M, n_ttiles;
};

// ---------------------------------------------------------------- launches
struct LaunchCtx {
    hipStream_t stream;
    const int64_t *stride_ctr;   // device stride counter
};

hipError_t launch_ingest(const LaunchCtx &, const float *strain, int64_t src_det_stride, uint32_t gap_mask,
                         float *xring, int64_t ring_det_stride, int32_t cap, int32_t F, int32_t n_det);
hipError_t launch_down(const LaunchCtx &, const DownItem *items, int32_t n_items, int32_t max_lds_floats);
hipError_t launch_corr(const LaunchCtx &, int precision, const CorrItem *items, int32_t n_items, int32_t group);
hipError_t launch_reduce(const LaunchCtx &, int precision, const ReduceItem *items, int32_t n_items);
hipError_t launch_mix(const LaunchCtx &, int precision, const MixItem *items, int32_t n_items,
                      const MixBank *banks, const MixSlice *slices, const float *uptaps,
                      float *series, PartialPeak *partials, int32_t F, int32_t n_det,
                      int32_t S, int32_t TP, int32_t nup, int32_t group);
hipError_t launch_peaks(const LaunchCtx &, const PeakItem *items, int32_t n_items,
                        const PartialPeak *partials, lloid_peak *peaks, float threshold,
                        int64_t *stride_ctr_advance);
hipError_t configure_lds(int precision, size_t mix_bytes, size_t down_bytes);
size_t mix_lds(int precision, int S, int TP);   // dynamic LDS bytes of the mix kernel
inline size_t mix_lds_bytes(int precision, int S, int TP) { return mix_lds(precision, S, TP); }
// FP8 e4m3 rows with one power-of-two scale per row (basis role of LLOID_FP8_BF16)
hipError_t launch_convert_fp8_rows(hipStream_t, const double *src, int32_t rows, int32_t cols, int32_t src_ld,
                                   uint8_t *dst, int32_t dst_ld, float *scale);

// rows [0, rows) of a basis-output ring, positions a .. a+len-1,
// as float rows dst[r * dst_ld + dst_off + c]
hipError_t launch_ring_gather(hipStream_t, int precision, const void *ring, int32_t Lpad, int32_t cap, int64_t a,
                              int32_t len, int32_t rows, float *dst, int64_t dst_ld, int64_t dst_off);

// gradient and re-orthonormalisation (lloid_grad.hip)
// the gradient's capture of one stride: item rows are copied from their
// mirror rings (basis outputs in 4-output groups, or plain streams)
struct CaptureItem {
    const float *src;
    int64_t src_ld;   // plain ring: floats per row
    int64_t base, step;
    float *dst;
    int64_t dst_ld, dst_lo;
    int32_t cap, grouped, len, row0;
};
hipError_t launch_capture(hipStream_t, const CaptureItem *items, const int32_t *row_item, int32_t rows,
                          int32_t max_len, int64_t k);
hipError_t launch_residual(hipStream_t, const float *series, const float *target, int32_t M, int32_t F,
                           float *R, int64_t ld, int64_t t0, double *loss_part, int32_t blocks);
hipError_t launch_sum_f64(hipStream_t, const double *part, int32_t n, double *out);
hipError_t launch_upsample_adjoint(hipStream_t, const float *g, int64_t g_ld, int64_t g_lo, int64_t ng,
                                   float *out, int64_t o_ld, int64_t a_lo, int64_t na, int32_t rows,
                                   int32_t p, int32_t nup, const float *taps);
hipError_t launch_gemm_abt(hipStream_t, const float *A, int64_t lda, const float *B, int64_t ldb, int32_t M,
                           int32_t N, int64_t K, int64_t ksplit, float *part);
hipError_t launch_gemm_atb(hipStream_t, const float *W, int32_t ldw, const float *G, int64_t ldg, int32_t K,
                           int64_t n_out, float alpha, float *out, int64_t ldo);
hipError_t launch_sum_parts(hipStream_t, const float *part, int32_t nsplit, int64_t plane, int32_t rows,
                            int32_t cols, int64_t p_ld, float *dst, int64_t d_ld, float alpha,
                            int32_t accumulate);
hipError_t launch_cholesky_qr2(hipStream_t, double *U, int32_t L, int32_t N, double *W, int32_t rows,
                               double *G, double *Cinv, int32_t *info);
hipError_t launch_clear_info(hipStream_t, int32_t *info, int32_t n);
hipError_t launch_normalize(hipStream_t, const double *const *W64, const int32_t *Ls,
                            int32_t n_slices, int32_t rows, int32_t normalize, double *inv_norm);
hipError_t launch_convert_rows(hipStream_t, const double *src, int32_t rows, int32_t cols,
                               int32_t src_ld, const double *row_scale, int precision, int role,
                               float *dst32, void *dst_hi, void *dst_lo, int32_t dst_ld,
                               float *row_scale_out);

// destination layouts of launch_convert_rows: row-major [rows][dst_ld], or
// the mixing kernel's fragment order (see MixSlice)
enum { ROLE_ROWS = 0, ROLE_MIXING = 1 };

}  // namespace lloid
