/*
 * lloid.h -- C ABI of the MI355X LLOID filtering core.
 *
 * LLOID (Low-Latency Online Inspiral Detection) filters whitened strain with
 * a template bank compressed by time slicing and SVD (Sec. II.C of the SGNL
 * paper, arXiv:2511.04730).  Per 1-s stride and detector the library
 *   1. decimates the strain to every slice rate with the sinc-windowed-sinc
 *      kernel of Eq. (sinc)                                  (Sec. II.C.2),
 *   2. correlates each slice's orthonormal basis filters u^s_l with the
 *      stream at its rate, reading it at the pre-synchronised offset of the
 *      recursion equation of Sec. II.C.3,
 *   3. reconstructs every template's SNR at that rate with the mixing
 *      matrix sigma^s_l nu^s_il                              (Sec. II.C.2),
 *   4. upsamples with the polyphase form of Eq. (upsample) and adds, lowest
 *      rate first, up to the top rate                        (Sec. II.C.2-3),
 *   5. reports per template the maximum |complex SNR| in the stride, its
 *      index, its value and whether it reaches the threshold (Sec. II.D.1).
 * The SNR for stride k covers top-rate samples [kF, (k+1)F): no latency is
 * added, as long as every slice's delay covers the resampling look-ahead
 * (Sec. II.C.2 "Combining SNR segments").
 *
 * Conventions
 *   - Signatures use only C types; device buffers are plain pointers to
 *     device memory; streams are hipStream_t passed as void*.
 *   - Every call returns an lloid_status.  Argument and shape errors are
 *     detected on the host before anything is enqueued.  A HIP launch or
 *     copy error is returned as LLOID_E_HIP; an asynchronous device error is
 *     reported by the next call that synchronises.
 *   - No call throws or aborts.  A plan must not be used by two host
 *     threads at once; distinct plans are independent.
 *   - Rows 2i and 2i+1 of a mixing matrix are the cosine (real) and sine
 *     (imaginary) filters of template i; complex SNR z_i = rho_2i + i rho_2i+1.
 */
#ifndef LLOID_H
#define LLOID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LLOID_OK = 0,
    LLOID_E_ARG = -1,         /* NULL pointer, out-of-range enum or count       */
    LLOID_E_SHAPE = -2,       /* inconsistent sizes (rates, taps, basis counts) */
    LLOID_E_LATENCY = -3,     /* a slice delay shorter than its look-ahead      */
    LLOID_E_NOMEM = -4,       /* device or host allocation failed               */
    LLOID_E_HIP = -5,         /* a HIP runtime call failed                      */
    LLOID_E_STATE = -6,       /* call not valid in the plan's current state     */
    LLOID_E_UNSUPPORTED = -7  /* valid request the library does not implement  */
} lloid_status;

/* Arithmetic of the correlation and mixing contractions (accumulation is
 * always FP32).  FP32: FP32 operands.  BF16X3: both operands of both
 * contractions split into bf16 hi + lo parts, three products (hi*hi + hi*lo +
 * lo*hi).  FP16: fp16 basis and mixing, strain and basis outputs split into
 * fp16 hi + lo.  FP8_BF16: fp8 e4m3 correlation with a power-of-two scale
 * per basis vector and per stride, bf16x3 mixing. */
typedef enum {
    LLOID_FP32 = 0,
    LLOID_BF16X3 = 1,
    LLOID_FP16 = 2,
    LLOID_FP8_BF16 = 3
} lloid_precision;

/* One time slice of one bank (Sec. II.C.1).
 *   rate_hz  f^s, the top rate divided by a power of two D, 1 <= D <= 64
 *   delay    t^s * f^s: time before merger of the slice's latest tap, in
 *            samples at f^s
 *   n_taps   N^s; n_basis L^s with 1 <= L^s <= 160 (and at most 160 basis
 *            vectors per bank and rate, each count rounded up to 16)
 *   basis    host, row-major [L^s][N^s], float64: u^s_l[n], taps in
 *            chronological order (column N^s-1 is closest to merger)
 *   mixing   host, row-major [2M][L^s], float64: sigma^s_l nu^s_il        */
typedef struct {
    int32_t rate_hz;
    int64_t delay;
    int32_t n_taps;
    int32_t n_basis;
    const double *basis;
    const double *mixing;
} lloid_slice;

typedef struct {
    int32_t n_templates;       /* M complex templates (2M real filters) */
    int32_t n_slices;
    const lloid_slice *slices;
} lloid_bank;

typedef struct {
    int32_t sample_rate_hz;    /* F, the top rate; one stride = F samples        */
    int32_t n_detectors;       /* 1..32                                          */
    int32_t n_down;            /* decimator half-length at the target rate (32)  */
    int32_t n_up;              /* interpolator half-length, input samples (8)    */
    int32_t precision;         /* lloid_precision                                */
    int32_t normalize;         /* 1: scale each real row to unit reconstructed
                                  norm sum_s sum_l W^s[r,l]^2 = 1, in FP64       */
    float snr_threshold;       /* trigger threshold on |z| (4.0)                 */
} lloid_config;

/* Trigger of one template in one stride (Sec. II.D.1): the maximum |z| over
 * the stride, the lowest in-stride index attaining it, z there, and
 * above = (snr >= threshold). 20 bytes. */
typedef struct {
    float snr;
    int32_t index;
    float re;
    float im;
    int32_t above;
} lloid_peak;

typedef struct lloid_plan lloid_plan;

/* Build a plan: validates every bank, groups slices by rate, derives the
 * pre-synchronised read offsets, copies the banks to the device (the caller
 * may free its arrays on return), normalises the mixing rows in FP64 on the
 * device and converts them to the chosen precision, and allocates the
 * per-detector history buffers.  The plan starts at stride 0 with zero
 * history.  `stream` (hipStream_t or NULL) orders the set-up work; the call
 * synchronises it before returning.
 * Errors: LLOID_E_ARG, LLOID_E_SHAPE (a rate that is not the top rate over
 * a power of two, a top rate that is not a multiple of 256, a negative
 * delay, no taps or basis vectors), LLOID_E_LATENCY (a slice needs strain
 * from the future of the stride), LLOID_E_UNSUPPORTED (a decimation factor
 * above 64, more than 160 basis vectors per bank and rate, more than 12
 * rates per bank, or upsampling taps beyond the mixing kernel's LDS),
 * LLOID_E_NOMEM, LLOID_E_HIP. */
lloid_status lloid_plan_create(const lloid_config *config, const lloid_bank *banks,
                               int32_t n_banks, void *stream, lloid_plan **out);

void lloid_plan_destroy(lloid_plan *plan);

/* Sizes and offsets of a plan's outputs (see lloid_push_stride). */
typedef enum {
    LLOID_Q_N_BANKS = 0,
    LLOID_Q_TOTAL_TEMPLATES = 1,     /* sum of M_b                                */
    LLOID_Q_SERIES_FLOATS = 2,       /* floats of one stride's SNR output         */
    LLOID_Q_N_PEAKS = 3,             /* lloid_peak entries per stride             */
    LLOID_Q_BANK_SERIES_OFFSET = 4,  /* index = bank: float offset of its block   */
    LLOID_Q_BANK_PEAK_OFFSET = 5,    /* index = bank: entry offset of its block   */
    LLOID_Q_BANK_TEMPLATES = 6,      /* index = bank: M_b                         */
    LLOID_Q_STRIDE = 7,              /* strides pushed so far                     */
    LLOID_Q_N_SLICES = 8,            /* slices over all banks                     */
    LLOID_Q_SLICE_LOOKAHEAD = 9,     /* index = global slice: look-ahead samples  */
    LLOID_Q_FLOPS_PER_STRIDE = 10,   /* algorithmic flops of one stride           */
    LLOID_Q_DEVICE_BYTES = 11,       /* device memory the plan holds              */
    LLOID_Q_OPTION = 12              /* index = lloid_option: its current value   */
} lloid_query;

lloid_status lloid_plan_query(const lloid_plan *plan, int32_t what, int32_t index, int64_t *value);

/* Filter the next stride.
 *   strain_dev  device, [n_det][F] float32: whitened strain of this stride
 *   gap_mask    bit d set: detector d's stride is a gap and is taken as zeros
 *   snr_dev     device or NULL.  If not NULL, receives for every bank b the
 *               block [n_det][M_b][F][2] float32 at LLOID_Q_BANK_SERIES_OFFSET:
 *               interleaved (re, im) of z_i at top-rate samples kF..kF+F-1
 *   peaks_dev   device, receives for every bank b the block [n_det][M_b] of
 *               lloid_peak at LLOID_Q_BANK_PEAK_OFFSET
 * All buffers are caller-owned and must stay valid until the work enqueued
 * on `stream` completes.  Strides must be pushed in order.
 * Errors: LLOID_E_ARG (NULL strain or peaks), LLOID_E_HIP. */
lloid_status lloid_push_stride(lloid_plan *plan, const float *strain_dev, uint32_t gap_mask,
                               float *snr_dev, lloid_peak *peaks_dev, void *stream);

/* Zero all history and restart at stride 0. */
lloid_status lloid_reset(lloid_plan *plan, void *stream);

/* Streaming state (all history buffers and the stride counter) as an opaque
 * blob: size in bytes, save to a host buffer, load from one saved by a plan
 * created with the same banks and config.  Save and load synchronise
 * `stream`.  Errors: LLOID_E_ARG, LLOID_E_STATE (blob from another plan
 * layout), LLOID_E_HIP. */
lloid_status lloid_state_size(const lloid_plan *plan, size_t *bytes);
lloid_status lloid_state_save(lloid_plan *plan, void *host_dst, size_t bytes, void *stream);
lloid_status lloid_state_load(lloid_plan *plan, const void *host_src, size_t bytes, void *stream);

/* Internal streams, for stage-by-stage checks.  Copies samples [m_lo, m_hi)
 * (absolute indices at the stream's rate) of detector `det` into the host
 * buffer `dst` (float32, m_hi - m_lo values per row):
 *   LLOID_INSPECT_DOWNSAMPLED  index = decimation factor D (1 = input
 *                              strain); one row
 *   LLOID_INSPECT_BASIS_OUT    index = global slice (banks in order, slices
 *                              in order); L^s rows of y^s_l
 * Only samples still held in the history are available
 * (LLOID_E_STATE otherwise).  Synchronises `stream`. */
typedef enum { LLOID_INSPECT_DOWNSAMPLED = 0, LLOID_INSPECT_BASIS_OUT = 1 } lloid_inspect_what;
lloid_status lloid_inspect(lloid_plan *plan, int32_t what, int32_t index, int32_t det,
                           int64_t m_lo, int64_t m_hi, float *dst, void *stream);

/* Gradient of the SNR-reconstruction loss, for refining compressed banks
 * (an extension; the paper builds banks by SVD only, Sec. II.C.1):
 *   L = sum over detectors, banks, real rows r and top-rate samples
 *       t in [0, n_strides F) of (rho[r,t] - target[r,t])^2
 * where rho is the plan's own output for the strain segment, filtered from
 * zero history.  The plan's streaming state (history and stride count) is
 * saved to host memory before and restored before the call returns, on
 * success and on error, so a live plan keeps its history and the next
 * lloid_push_stride continues where it left off.  rho is linear in every
 * W^s and every U^s:
 *   dL/dW^s = 2 G^s Y^s^T,  dL/dU^s[l,n] = 2 sum_q (W^s^T G^s)[l,q] d^s[q - delay - (N-1) + n],
 * with Y^s the basis outputs, d^s the decimated strain and G^s the residual
 * taken down to the slice's rate by the transposed upsampling stages.
 *   strain_dev  device [n_det][n_strides F] float32
 *   target_dev  device [n_strides][series floats] float32: per stride the
 *               layout lloid_push_stride writes (e.g. the output of a plan
 *               holding the uncompressed slices)
 *   loss_out    host, receives L
 *   dW_dev      device float32: for every slice in bank order, its
 *               [2M_b][L_s] block, packed back to back
 *   dU_dev      device float32: for every slice, its [L_s][N_s] block
 * The gradient is with respect to the mixing rows the plan uses (create the
 * plan with normalize = 0 to differentiate the given W).  Each call
 * allocates, and frees before returning, a device workspace of about twice
 * the segment's series size (LLOID_E_NOMEM if it does not fit).  FP32 plans
 * only (LLOID_E_UNSUPPORTED otherwise).  Synchronises `stream`. */
lloid_status lloid_grad(lloid_plan *plan, const float *strain_dev, int32_t n_strides, const float *target_dev,
                        double *loss_out, float *dW_dev, float *dU_dev, void *stream);

/* Replace one slice's basis and mixing matrix (global slice index, banks in
 * order) with device float64 arrays U [L][N] and W [2M][L]; they are
 * converted to the plan's precision.  Plans created with normalize = 1 return
 * LLOID_E_STATE (the row norms couple all slices of a bank). */
lloid_status lloid_set_slice(lloid_plan *plan, int32_t slice, const double *U_dev, const double *W_dev,
                             void *stream);

/* Re-orthonormalise refined bases in float64 on the device (CholeskyQR2):
 * two passes of G = U U^T = C C^T (Cholesky), U <- C^-1 U, W <- W C, so
 * that U has orthonormal rows and W U is unchanged.  U_dev [L][N], W_dev
 * [rows][L], device float64, updated in place; 1 <= L <= 160.
 * LLOID_E_STATE if a Gram matrix is not positive definite.  Synchronises. */
lloid_status lloid_orthonormalize(double *U_dev, int32_t L, int32_t N, double *W_dev, int32_t rows, void *stream);

/* The same re-orthonormalisation for callers that cannot allocate device
 * memory (code under HIP graph capture, tight refinement loops, harnesses
 * that forbid hipMalloc): no hipMalloc, hipFree or allocating library call,
 * and no synchronisation; it only enqueues on `stream`.  Its Gram matrix,
 * Cholesky factor and its inverse live in a static device array of the library
 * (409 856 bytes per GPU, held until the process ends), which every call on
 * that GPU shares: calls that overlap on one GPU race and must be ordered
 * by the caller (one stream, or events).  Results are those of
 * lloid_orthonormalize (same kernels).
 *   U_dev, W_dev, L, N, rows  as lloid_orthonormalize; 1 <= L <= 160
 *   info_dev  device int32[2] or NULL: per CholeskyQR pass 0, or the first
 *             column + 1 whose pivot was not positive (the role of
 *             lloid_orthonormalize's LLOID_E_STATE); cleared by the call
 * Errors: LLOID_E_ARG (NULL U or W, L < 1, N < L, rows < 1),
 * LLOID_E_UNSUPPORTED (L > 160: the Gram matrix would not fit the static
 * array), LLOID_E_HIP. */
lloid_status lloid_orthonormalize_noalloc(double *U_dev, int32_t L, int32_t N, double *W_dev, int32_t rows,
                                          int32_t *info_dev, void *stream);

/* Plan options (lloid_set_option; current values via lloid_plan_query with
 * LLOID_Q_OPTION).  The three tiling options change only how the work is cut
 * into work groups, never what is computed; results stay deterministic for a
 * given setting, but the correlation split changes the FP32 summation order.
 * Setting one of them synchronises the device and drops a captured graph.
 *   LLOID_OPT_CORR_SPLIT  taps per correlation work item (multiple of 64,
 *                    64..65536; default chosen at plan time: the longest
 *                    power of two from 8192 down to 512 that still yields
 *                    2048 items).  The partial planes are reallocated.
 *   LLOID_OPT_CORR_COLS   output columns per correlation work item (a
 *                    multiple of 64 up to 512; default 512, or 64 when
 *                    512-column items at a 512-tap split would number fewer
 *                    than 2048).
 *   LLOID_OPT_CORR_GROUP  consecutive correlation items kept on one XCD
 *                    (0..64; 0 = dispatch order; default 16).
 *   LLOID_OPT_MIX_GROUP   consecutive mixing items kept on one XCD
 *                    (0..256; 0 = dispatch order; default 32).
 *   LLOID_OPT_MIX_TBLOCK  time tiles per block of the mixing item order
 *                    (1..64; default 1): per bank and detector the items
 *                    run in blocks of this many 256-sample time tiles, row
 *                    tiles inner within a block, so that the items an XCD
 *                    runs together share W~ rows and basis-output windows.
 *   LLOID_OPT_GRAPH  1: lloid_push_stride copies the strain into a
 *                    plan-owned staging buffer on the call's stream and then
 *                    replays one captured HIP graph of the stride's kernels
 *                    (one graph launch per stride; the stride index lives in
 *                    device memory, so the same graph serves every stride).
 *                    The graph is captured on first use and again whenever
 *                    the output pointers or the gap mask change.
 *                    0 (default): the kernels are launched one by one.
 *                    While profiling is enabled, kernels are launched one by
 *                    one regardless.
 * Errors: LLOID_E_ARG (unknown option or value), LLOID_E_HIP, LLOID_E_NOMEM
 * (reallocating the partial planes failed; the plan must then be destroyed). */
typedef enum {
    LLOID_OPT_GRAPH = 0,
    LLOID_OPT_CORR_SPLIT = 1,
    LLOID_OPT_CORR_GROUP = 2,
    LLOID_OPT_MIX_GROUP = 3,
    LLOID_OPT_CORR_COLS = 4,
    LLOID_OPT_MIX_TBLOCK = 5
} lloid_option;
lloid_status lloid_set_option(lloid_plan *plan, int32_t option, int64_t value);

/* Signal-consistency statistic xi^2 at the triggers (Sec. II.D.2):
 *   xi^2 = sum_t |z(t_p + t) - z(t_p) R(t)|^2 / sum_t (2 - 2 |R(t)|^2),
 *   t = -delta..delta (top-rate samples), delta = (A - 1) / 2,
 * for the complex SNR z of one template and detector around its trigger
 * index t_p, with R the template's complex autocorrelation, normalised to
 * R(0) = 1 and oriented so that E[z(t) conj z(0)] = 2 R(t) in white noise:
 * R(t) = sum_j h[j] conj h[j - t] / sum_j |h[j]|^2 for the complex filter
 * h = h_cos + i h_sin indexed by time before merger.
 *
 * lloid_set_autocorrelation stores the autocorrelations, stacked across the
 * plan's banks (Sec. II.D.2).
 *   acf_dev   device, float64: for every bank b in order, its block
 *             [M_b][A_b][2] of (re, im) R_i(t), t = -delta_b..delta_b
 *   acf_len   host [n_banks]: A_b, odd, 3 <= A_b <= 2 F + 1
 * They are converted to float32 in plan-owned memory (replacing earlier
 * ones); the caller may free acf_dev on return.  Synchronises `stream`.
 * Errors: LLOID_E_ARG, LLOID_E_SHAPE (an even, too short or too long A_b),
 * LLOID_E_NOMEM, LLOID_E_HIP.
 *
 * lloid_xi2 computes xi^2 at every trigger of stride k (trigger window =
 * the stride; the threshold flag is left to the caller).
 *   prev_dev, cur_dev, next_dev  device series of strides k - 1, k, k + 1
 *             as lloid_push_stride writes them (cur_dev required).  prev or
 *             next may be NULL (first or last stride of the data): samples
 *             there are left out of both sums.  With next_dev given, call
 *             after stride k + 1 has been filtered (delta samples of latency).
 *   peaks_dev device, the triggers of stride k: those of lloid_push_stride
 *             (index in [0, F)) or the window triggers of lloid_coincidence
 *             (index in [-F, F), negative inside the previous stride, which
 *             prev_dev must then hold)
 *   xi2_dev   device float32 [LLOID_Q_N_PEAKS], entry for entry with the
 *             triggers; NaN where a trigger index lies outside [0, F), or
 *             outside [-F, F) when prev_dev is given.
 * Errors: LLOID_E_ARG (NULL cur, peaks or output), LLOID_E_STATE (no
 * autocorrelations stored), LLOID_E_HIP. */
lloid_status lloid_set_autocorrelation(lloid_plan *plan, const double *acf_dev, const int32_t *acf_len,
                                       void *stream);
lloid_status lloid_xi2(lloid_plan *plan, const float *prev_dev, const float *cur_dev, const float *next_dev,
                       const lloid_peak *peaks_dev, float *xi2_dev, void *stream);

/* Overlapping trigger windows, coincidence and clustering (Sec. II.D.3-4).
 *
 * Window k covers top-rate samples [kF - overlap, (k+1)F): its trigger per
 * template and detector is the maximum |z| over the last `overlap` samples
 * of stride k - 1 and the whole of stride k (the earlier sample on ties);
 * the first window (prev_dev NULL) is stride k alone.  Coincidence is per
 * template: every detector whose window trigger reaches the plan's
 * threshold anchors a candidate that holds it and each other such detector
 * whose trigger lies within window[anchor][other] samples (inclusive); a
 * candidate holding two or more detectors is an event with network SNR
 * sqrt(sum of the held SNR^2).  A template keeps its best candidate (the
 * lowest anchor on ties) and each sub-bank keeps its best template (the
 * lowest on ties): at most one event per bank and window.  Network SNR^2
 * is summed in detector order in FP32.
 *   prev_dev     device, series of stride k - 1 as lloid_push_stride writes
 *                it, or NULL (first window)
 *   peaks_dev    device, the triggers of stride k (lloid_push_stride)
 *   overlap      samples, 0 <= overlap <= F: the largest light travel time
 *                between the detectors plus the coincidence buffer
 *   window       host [n_det][n_det] int32, samples >= 0: per detector pair
 *                the light travel time plus the buffer (diagonal unused)
 *   triggers_dev device, receives the window triggers [LLOID_Q_N_PEAKS]
 *                (lloid_peak; index relative to the start of stride k,
 *                negative inside the overlap)
 *   events_dev   device, receives one lloid_event per bank
 * Errors: LLOID_E_ARG (NULL peaks, window or outputs), LLOID_E_SHAPE
 * (overlap outside [0, F], a negative window), LLOID_E_UNSUPPORTED (more
 * than 8 detectors), LLOID_E_NOMEM, LLOID_E_HIP. */
typedef struct {
    float network_snr;        /* 0 when the bank has no event             */
    int32_t template_index;   /* template within the bank, -1: no event   */
    uint32_t det_mask;        /* bit d: detector d's trigger is held      */
    int32_t n_det;            /* detectors held (0: no event)             */
} lloid_event;
lloid_status lloid_coincidence(lloid_plan *plan, const float *prev_dev, const lloid_peak *peaks_dev, int32_t overlap,
                               const int32_t *window, lloid_peak *triggers_dev, lloid_event *events_dev,
                               void *stream);

/* PSD estimation and whitening with frequency-domain downsampling
 * (Sec. II.B.2), upstream of the filter; one whitener serves n_detectors
 * streams.  Each push takes H = N/2 - Z new samples per detector at the
 * input rate and returns H/D whitened samples at the output rate:
 *   - the last 2H inputs times the periodic Hann window sin^2(pi m / 2H)
 *     (which sums to one at hop H), zero-padded by Z on each side, go
 *     through an N-point FFT; only the first N/(2D) + 1 bins are kept
 *     (downsampling by D in the frequency domain);
 *   - per bin the instantaneous PSD |X|^2 / sum(hann^2) joins the last
 *     n_med estimates; the median of the most recent c of them (c the
 *     largest odd count available) over beta_c, the median-to-geometric-mean
 *     ratio of chi^2_2 bins, updates a running average of the log over
 *     min(blocks seen, n_avg) blocks; PSD = geometric mean x e^gamma,
 *     including the current block;
 *   - X / sqrt(D PSD) goes through the N/D-point inverse FFT (real DC and
 *     Nyquist bins), is tapered by a Tukey window that is one over the
 *     segment and a raised cosine over each Z/D-sample pad, and is
 *     overlap-added; the first H/D accumulated samples are the output.
 * Push i = 1, 2, ... returns the whitened input times [iH - 2H - Z,
 * iH - H - Z): a latency of N/2 input samples.  White noise comes out with
 * unit variance at every D.
 * A detector whose gap_mask bit is set adds no block and no PSD estimate
 * for that push (its input is taken as zeros for later blocks); its
 * accumulator keeps draining.
 *   config       n_detectors 1..32; block N a power of two, 64..2^20; pad Z
 *                with 0 <= 4Z <= N; decimation D a power of two dividing Z
 *                and H with N/D >= 16; n_med odd, 1..15; n_avg >= 1
 *   in_dev       device [n_det][H] float32
 *   out_dev      device [n_det][H/D] float32
 *   psd_dev      device [n_det][N/(2D) + 1] float32: the current PSD
 *                (per-sample variance units)
 * Errors: LLOID_E_ARG, LLOID_E_SHAPE, LLOID_E_NOMEM, LLOID_E_HIP.  Create
 * synchronises `stream`; push and psd only enqueue on it. */
typedef struct lloid_whitener lloid_whitener;
typedef struct {
    int32_t n_detectors;
    int32_t block;
    int32_t pad;
    int32_t decimation;
    int32_t n_med;
    int32_t n_avg;
} lloid_whiten_config;
lloid_status lloid_whitener_create(const lloid_whiten_config *config, void *stream, lloid_whitener **whitener);
void lloid_whitener_destroy(lloid_whitener *whitener);
lloid_status lloid_whitener_push(lloid_whitener *whitener, const float *in_dev, uint32_t gap_mask, float *out_dev,
                                 void *stream);
lloid_status lloid_whitener_psd(lloid_whitener *whitener, float *psd_dev, void *stream);

/* SVD bank construction (Sec. II.C.1) for one time slice: the rank-L
 * truncation of the slice's template matrix H (device float64 [rows][N],
 * rows = 2M real templates in the slice's samples) as basis rows U and
 * mixing rows W with W U = H P_L, P_L the projector on the top-L right
 * singular subspace (the best rank-L approximation, as the truncated SVD
 * gives; the basis is an orthonormal basis of that subspace, not
 * necessarily the singular vectors themselves).  Subspace iteration
 * U <- orth((H^T H) U), CholeskyQR2 after each product, `iters` times;
 * the error shrinks by (sigma_{L+1} / sigma_L)^2 per iteration.
 *   U_dev  device float64 [L][N]: in, the starting rows (for instance
 *          seeded Gaussian); out, the orthonormal basis
 *   W_dev  device float64 [rows][L]: out, H U^T
 * 1 <= L <= min(160, rows, N) and rows N < 2^28 (H under 2 GiB: the
 * products address it with 32-bit byte offsets).  Synchronises `stream`.
 * Errors: LLOID_E_ARG, LLOID_E_NOMEM, LLOID_E_STATE (the iterated rows
 * became linearly dependent: a start without components in the subspace,
 * or a rank of H below L), LLOID_E_HIP. */
lloid_status lloid_svd_basis(const double *H_dev, int32_t rows, int32_t N, int32_t L, int32_t iters, double *U_dev,
                             double *W_dev, void *stream);

/* FP8 basis values for quantisation-aware refinement (extension): writes
 * to Uq_dev the values the FP8_BF16 form correlates with for the rows of
 * U_dev (device float64 [rows][cols], row-major; Uq_dev the same shape,
 * may not alias): per row a power-of-two scale 2^e with e =
 * floor(log2(448 / max|u|)), e4m3 (OCP, round to nearest even) of the
 * float32-rounded u 2^e, times 2^-e.  A refinement that evaluates the loss
 * of an FP32 plan at these values and applies the gradient to U (straight
 * through the rounding) optimises the bank for the FP8 form.  Enqueues on
 * `stream`.  Errors: LLOID_E_ARG, LLOID_E_HIP. */
lloid_status lloid_quantize_fp8_rows(const double *U_dev, int32_t rows, int32_t cols, double *Uq_dev, void *stream);

/* Per-kernel timing of lloid_push_stride with HIP events recorded on the
 * call's stream around each of the stride's kernels:
 *   0 ingest, 1 decimation, 2 basis correlation, 3 split reduction,
 *   4 mixing + upsample-and-add + series + peak candidates, 5 triggers,
 *   6 xi^2 for lloid_xi2, 7 window triggers and 8 coincidence for
 *   lloid_coincidence.
 * lloid_profile_enable(plan, 1) starts a new accumulation (0 stops it);
 * lloid_profile_read synchronises the recorded events and returns the
 * summed duration (ms) and the number of launches of one kernel since the
 * accumulation started.  Errors: LLOID_E_ARG, LLOID_E_HIP. */
typedef enum {
    LLOID_K_INGEST = 0, LLOID_K_DOWN = 1, LLOID_K_CORR = 2,
    LLOID_K_REDUCE = 3, LLOID_K_MIX = 4, LLOID_K_PEAKS = 5, LLOID_K_XI2 = 6,
    LLOID_K_TRIGGERS = 7, LLOID_K_COINC = 8, LLOID_K_COUNT = 9
} lloid_kernel_id;
lloid_status lloid_profile_enable(lloid_plan *plan, int32_t enable);
lloid_status lloid_profile_read(lloid_plan *plan, int32_t kernel, double *total_ms, int64_t *launches);

const char *lloid_status_string(lloid_status status);

#ifdef __cplusplus
}
#endif

#endif /* LLOID_H */
