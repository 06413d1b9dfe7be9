// Host side of the LLOID C ABI: plan construction, work tables, stride launches.
//
// Plan construction validates every bank, groups each bank's slices by rate
// into a chain of levels (top rate first; Sec. II.C.1 slices, Sec. II.C.3
// "Multidimensional filtering" groups by rate), derives the integer
// look-ahead of every level from the polyphase index ranges (the cumulative
// upsampling half-lengths of the pre-synchronisation equation, Sec. II.C.3),
// checks that every slice delay covers it plus the decimator half-length,
// sizes the history rings, builds the work tables of the six per-stride
// kernels, and moves the bank to the device (FP64 normalisation there).
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "lloid_coinc.h"
#include "lloid_internal.h"
#include "lloid_xi2.h"

using namespace lloid;

#define HIP_OK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return LLOID_E_HIP;      \
    } while (0)

namespace {

constexpr uint64_t kStateMagic = 0x4c4c4f4944535433ull;   // "LLOIDST3": grouped basis-output rings

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
int64_t floordiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Eq. (sinc): g[k] = sinc((k-c)/f) sinc((k-c)/c), k = 0..2c.
double sinc_pi(double x) { return x == 0.0 ? 1.0 : std::sin(M_PI * x) / (M_PI * x); }
std::vector<double> sinc_windowed_sinc(int f, int c) {
    std::vector<double> g(2 * c + 1);
    for (int k = 0; k <= 2 * c; ++k) {
        const double u = k - c;
        g[k] = sinc_pi(u / f) * sinc_pi(u / c);
    }
    return g;
}

struct Ring {
    float *base = nullptr;   // n_det rings of 2*cap floats
    int32_t cap = 0;
    int64_t det_stride = 0;
    int64_t need = 0;        // required span (samples)
};

struct PSlice {
    int bank, rate, D, level, N, L, Npad, Lpad, la, nsplit, capY;
    int64_t delay;
    float *U32 = nullptr;
    float *W32 = nullptr;    // FP32 mixing rows, row-major (gradient)
    float *Wf32 = nullptr;   // the same in the mixing kernel's fragment order
    void *Uhi = nullptr, *Ulo = nullptr, *Whi = nullptr, *Wlo = nullptr;
    float *uscale = nullptr;
    float *yring = nullptr;  // n_det rings of Lpad x 2 capY (layout in MixSlice)
    int64_t ydet = 0;
    float *part = nullptr;   // n_det x [nsplit][Lpad][f]
    int64_t part_det = 0;
};

struct PBank {
    int M, nlev, rows_pad;
    std::vector<int> rates, la;
    std::vector<int> slices;   // plan slice ids, sorted by level
    int64_t series_off, peak_off, part_off;
};

}  // namespace

struct lloid_plan {
    lloid_config cfg{};
    int F = 0, n_det = 0, nup = 8, ndown = 32, precision = 0;
    int64_t stride = 0;
    std::vector<PSlice> slices;
    std::vector<PBank> banks;
    std::map<int, Ring> rings;     // by decimation factor D (1 = strain)
    std::vector<void *> allocs;
    size_t device_bytes = 0;

    CorrItem *d_corr = nullptr;
    int n_corr = 0;
    ReduceItem *d_reduce = nullptr;
    int n_reduce = 0, reduce_rows = 0;
    DownItem *d_down = nullptr;
    int n_downitems = 0, down_lds = 0;
    MixItem *d_mix = nullptr;
    int n_mix = 0;
    MixBank *d_mbanks = nullptr;
    MixSlice *d_mslices = nullptr;
    int mixS = 0, mixTP = 0;   // mix level-buffer row stride, upsampling taps in LDS
    PeakItem *d_peakitems = nullptr;
    int n_peakitems = 0;
    PartialPeak *d_partials = nullptr;
    float *d_uptaps = nullptr;
    int64_t *d_stride = nullptr;
    int64_t series_floats = 0, n_peaks = 0, total_templates = 0;

    // xi^2: per-template table and float32 autocorrelations (lloid_set_autocorrelation)
    XiTemplate *d_xitab = nullptr;
    float *d_acf = nullptr;
    int32_t n_xi = 0;
    size_t xi_bytes = 0;

    // coincidence: per-template and per-bank tables (built on first use)
    TrigTemplate *d_trigtab = nullptr;
    CoincBank *d_coincbanks = nullptr;

    // graph mode (LLOID_OPT_GRAPH)
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    float *d_instage = nullptr;   // [n_det][F] strain staging read by the graph
    float *g_snr = nullptr;
    lloid_peak *g_peaks = nullptr;
    uint32_t g_gap = 0;
    double flops = 0.0;
    int ksplit = kCorrSplitK;      // taps per correlation work item
    int corr_cols = kCorrTQ;       // output columns per correlation work item
    int corr_group = 16;           // consecutive correlation items per XCD
    int mix_group = 32;            // consecutive mixing items per XCD
    int mix_tblock = 1;            // time tiles per block of the mixing item order
    std::vector<MixItem> h_mix;    // mixing items in bank, detector, time tile, row tile order

    // per-kernel event timing (lloid_profile_*)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kernel;
    double prof_ms[LLOID_K_COUNT] = {0};
    int64_t prof_n[LLOID_K_COUNT] = {0};

    template <typename T>
    lloid_status alloc(T **p, size_t count, bool zero = true) {
        void *q = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return LLOID_E_NOMEM;
        }
        allocs.push_back(q);
        device_bytes += bytes;
        if (zero && hipMemset(q, 0, bytes) != hipSuccess) return LLOID_E_HIP;
        *p = static_cast<T *>(q);
        return LLOID_OK;
    }
    // free a plan-time staging buffer early
    void release(void *p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) {
            (void)hipFree(p);
            allocs.erase(it);
        }
    }
    ~lloid_plan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
    // events bracketing one kernel launch when profiling
    hipError_t mark(int kernel, hipStream_t st, bool begin) {
        if (!profiling) return hipSuccess;
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev_pool.push_back(e);
        }
        if (begin) ev_kernel.push_back(kernel);
        return hipEventRecord(ev_pool[ev_used++], st);
    }
};

#define ST_OK(expr)                              \
    do {                                         \
        lloid_status s_ = (expr);                \
        if (s_ != LLOID_OK) return s_;           \
    } while (0)

namespace {

template <typename T>
lloid_status upload(lloid_plan *P, T **dst, const std::vector<T> &v, hipStream_t st) {
    ST_OK(P->alloc(dst, v.size(), false));
    if (!v.empty()) HIP_OK(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return LLOID_OK;
}

// Correlation work items and their split-K reduction for the current tiling:
// one item per (slice, detector, tap split, column tile, 128-row block),
// largest first.  Slices with one split write the basis-output ring
// directly; the others get partial planes (reallocated to match) and
// reduction items.
lloid_status build_corr_tables(lloid_plan *P, hipStream_t st) {
    const int ND = P->n_det;
    P->release(P->d_corr);
    P->release(P->d_reduce);
    P->d_corr = nullptr;
    P->d_reduce = nullptr;
    std::vector<CorrItem> items;
    std::vector<ReduceItem> red;
    P->reduce_rows = 0;
    for (auto &s : P->slices) {
        const Ring &r = P->rings[s.D];
        const int f = s.rate;
        s.nsplit = (s.Npad + P->ksplit - 1) / P->ksplit;
        P->release(s.part);
        s.part = nullptr;
        s.part_det = (int64_t)s.nsplit * s.Lpad * f;
        if (s.nsplit > 1) ST_OK(P->alloc(&s.part, (size_t)ND * s.part_det, false));
        for (int det = 0; det < ND; ++det) {
            for (int sp = 0; sp < s.nsplit; ++sp) {
                const int k0 = sp * P->ksplit;
                const int klen = std::min(P->ksplit, s.Npad - k0);
                const int cols = P->precision == LLOID_FP8_BF16 ? std::min(P->corr_cols, kCorrTQ8) : P->corr_cols;
                for (int c0 = 0; c0 < f; c0 += cols)
                for (int r0 = 0; r0 < s.Lpad; r0 += kCorrMB * 16) {
                    CorrItem it{};
                    it.U = s.U32;
                    it.Uhi = s.Uhi;
                    it.Ulo = s.Ulo;
                    it.ring = r.base + det * r.det_stride;
                    it.part = s.part ? s.part + det * s.part_det + (int64_t)sp * s.Lpad * f : nullptr;
                    it.uscale = s.uscale;
                    it.off = (int64_t)s.la - s.delay - (s.N - 1);
                    it.Npad = s.Npad;
                    it.Lpad = s.Lpad;
                    it.cap = r.cap;
                    it.f = f;
                    it.col0 = c0;
                    it.ncols = std::min(cols, f - c0);
                    it.k0 = k0;
                    it.klen = klen;
                    it.mb = std::min(kCorrMB, (s.Lpad - r0) / 16);
                    it.r0 = r0;
                    if (s.nsplit == 1) {   // no reduction: straight to the ring
                        it.yring = s.yring + det * s.ydet;
                        it.capY = s.capY;
                        it.la = s.la;
                    }
                    items.push_back(it);
                }
            }
            if (s.nsplit == 1) continue;
            for (int c0 = 0; c0 < f; c0 += 64)
                for (int l0 = 0; l0 < s.Lpad; l0 += 32)
                    red.push_back(ReduceItem{s.part + det * s.part_det, s.yring + det * s.ydet, s.nsplit, s.L,
                                             s.Lpad, f, s.capY, s.la, c0, l0});
            P->reduce_rows = std::max(P->reduce_rows, s.L);
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const CorrItem &a, const CorrItem &b) {
        return (int64_t)a.klen * a.mb * a.ncols > (int64_t)b.klen * b.mb * b.ncols;
    });
    P->n_corr = (int)items.size();
    P->n_reduce = (int)red.size();
    ST_OK(upload(P, &P->d_corr, items, st));
    ST_OK(upload(P, &P->d_reduce, red, st));
    HIP_OK(hipStreamSynchronize(st));
    return LLOID_OK;
}

lloid_status validate(const lloid_config *c, const lloid_bank *banks, int32_t n_banks) {
    if (!c || !banks || n_banks < 1) return LLOID_E_ARG;
    if (c->sample_rate_hz <= 0 || c->sample_rate_hz % kMixTN) return LLOID_E_SHAPE;
    if (c->n_detectors < 1 || c->n_detectors > 32) return LLOID_E_ARG;
    if (c->n_down < 1 || c->n_down > 64 || c->n_up < 1 || c->n_up > 8) return LLOID_E_ARG;
    if (c->precision < LLOID_FP32 || c->precision > LLOID_FP8_BF16) return LLOID_E_ARG;
    if (!std::isfinite(c->snr_threshold)) return LLOID_E_ARG;
    for (int b = 0; b < n_banks; ++b) {
        const lloid_bank &B = banks[b];
        if (B.n_templates < 1 || B.n_slices < 1 || !B.slices) return LLOID_E_ARG;
        for (int s = 0; s < B.n_slices; ++s) {
            const lloid_slice &S = B.slices[s];
            if (!S.basis || !S.mixing) return LLOID_E_ARG;
            if (S.rate_hz <= 0 || c->sample_rate_hz % S.rate_hz) return LLOID_E_SHAPE;
            const int D = c->sample_rate_hz / S.rate_hz;
            if (!is_pow2(D)) return LLOID_E_SHAPE;
            if (D > 64) return LLOID_E_UNSUPPORTED;
            if (S.n_taps < 1 || S.n_basis < 1 || S.delay < 0) return LLOID_E_SHAPE;
            if (S.n_basis > kMaxBasis) return LLOID_E_UNSUPPORTED;
        }
    }
    return LLOID_OK;
}

}  // namespace

// ---------------------------------------------- no-allocation scratch
// Device memory of lloid_orthonormalize_noalloc: the Gram matrix / Cholesky
// factor and its inverse (at most kNoAllocMaxBasis^2 doubles each) followed
// by the two breakdown flags used when the caller passes no flag buffer.  One copy per
// GPU, held until the process ends; every call on a GPU shares it, so calls
// that overlap on one GPU race.  Host code must use the address from
// hipGetSymbolAddress (per device), never the array's name.
namespace {
constexpr int kNoAllocMaxBasis = kMaxBasis;
constexpr int64_t kScratchGramDoubles = (int64_t)kNoAllocMaxBasis * kNoAllocMaxBasis;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[2 * kScratchGramDoubles + 32];

namespace {
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
hipError_t scratch_address(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

namespace {
// The mixing items of one bank and detector in blocks of `tblock` time
// tiles: row tiles inner within a block, so that a group of consecutive
// items (dealt to one XCD) covers a few row tiles x a few time tiles and
// shares both the W~ rows and the basis-output windows in that XCD's L2.
// The input is in bank, detector, time tile, row tile order.
std::vector<MixItem> mix_item_order(const std::vector<MixItem> &items, int tblock) {
    if (tblock <= 1) return items;
    std::vector<MixItem> out(items);
    std::stable_sort(out.begin(), out.end(), [&](const MixItem &a, const MixItem &b) {
        if (a.bank != b.bank) return a.bank < b.bank;
        if (a.det != b.det) return a.det < b.det;
        const int ba = a.t0 / (tblock * kMixTN), bb = b.t0 / (tblock * kMixTN);
        if (ba != bb) return ba < bb;
        if (a.r0 != b.r0) return a.r0 < b.r0;
        return a.t0 < b.t0;
    });
    return out;
}
}  // namespace

extern "C" {

const char *lloid_status_string(lloid_status s) {
    switch (s) {
        case LLOID_OK: return "ok";
        case LLOID_E_ARG: return "invalid argument";
        case LLOID_E_SHAPE: return "inconsistent shapes or rates";
        case LLOID_E_LATENCY: return "slice delay shorter than its resampling look-ahead";
        case LLOID_E_NOMEM: return "out of device or host memory";
        case LLOID_E_HIP: return "HIP runtime error";
        case LLOID_E_STATE: return "invalid plan state for this call";
        case LLOID_E_UNSUPPORTED: return "valid request the library does not implement";
    }
    return "unknown status";
}

lloid_status lloid_plan_create(const lloid_config *config, const lloid_bank *banks, int32_t n_banks, void *stream,
                               lloid_plan **out) {
    if (!out) return LLOID_E_ARG;
    *out = nullptr;
    ST_OK(validate(config, banks, n_banks));
    hipStream_t st = static_cast<hipStream_t>(stream);

    lloid_plan *P = new (std::nothrow) lloid_plan();
    if (!P) return LLOID_E_NOMEM;
    struct Guard {
        lloid_plan *p;
        ~Guard() { delete p; }
    } guard{P};

    P->cfg = *config;
    P->F = config->sample_rate_hz;
    P->n_det = config->n_detectors;
    P->nup = config->n_up;
    P->ndown = config->n_down;
    P->precision = config->precision;
    const int F = P->F, ND = P->n_det, nup = P->nup, ndown = P->ndown;

    // ---------------------------------------------------------- chains
    int64_t series_off = 0, peak_off = 0, part_off = 0;
    const int n_ttiles = F / kMixTN;
    for (int b = 0; b < n_banks; ++b) {
        const lloid_bank &B = banks[b];
        PBank pb;
        pb.M = B.n_templates;
        pb.rows_pad = (int)round_up(2 * (int64_t)B.n_templates, kMixTM);
        std::vector<int> rates{F};
        for (int s = 0; s < B.n_slices; ++s) rates.push_back(B.slices[s].rate_hz);
        std::sort(rates.begin(), rates.end(), std::greater<int>());
        rates.erase(std::unique(rates.begin(), rates.end()), rates.end());
        if ((int)rates.size() > kMaxLevels) return LLOID_E_UNSUPPORTED;
        pb.rates = rates;
        pb.nlev = (int)rates.size();
        // look-ahead per level: window of stride 0 is [-la_j, f_j + la_j)
        pb.la.assign(pb.nlev, 0);
        int64_t hi = F;
        for (int j = 1; j < pb.nlev; ++j) {
            const int p = rates[j - 1] / rates[j];
            hi = floordiv(hi - 1, p) + nup + 1;
            pb.la[j] = (int)(hi - rates[j]);
        }
        std::vector<int> lsum(pb.nlev, 0);
        for (int s = 0; s < B.n_slices; ++s) {
            const lloid_slice &S = B.slices[s];
            PSlice ps{};
            ps.bank = b;
            ps.rate = S.rate_hz;
            ps.D = F / S.rate_hz;
            ps.level = (int)(std::find(rates.begin(), rates.end(), S.rate_hz) - rates.begin());
            ps.N = S.n_taps;
            ps.L = S.n_basis;
            ps.Npad = (int)round_up(S.n_taps, kCorrTK);
            // 16-bit MFMA takes 32 basis vectors per step in the mixing
            ps.Lpad = (int)round_up(S.n_basis, P->precision == LLOID_FP32 ? 16 : 32);
            ps.la = pb.la[ps.level];
            ps.delay = S.delay;
            ps.nsplit = (int)((ps.Npad + kCorrSplitK - 1) / kCorrSplitK);
            const int f = S.rate_hz;
            // power of two: the mixing takes ring positions with a mask
            ps.capY = 1;
            while (ps.capY < f + 2 * ps.la + 16) ps.capY *= 2;
            // pre-synchronisation: the newest sample the slice reads must be
            // available at the end of the stride
            const int64_t need = ps.la + (ps.D > 1 ? ndown : 0);
            if (S.delay < need) return LLOID_E_LATENCY;
            lsum[ps.level] += ps.Lpad;
            if (lsum[ps.level] > kMaxBasis) return LLOID_E_UNSUPPORTED;
            pb.slices.push_back((int)P->slices.size());
            P->slices.push_back(ps);
        }
        std::stable_sort(pb.slices.begin(), pb.slices.end(),
                         [&](int a, int c) { return P->slices[a].level < P->slices[c].level; });
        pb.series_off = series_off;
        pb.peak_off = peak_off;
        pb.part_off = part_off;
        series_off += (int64_t)ND * pb.M * F * 2;
        peak_off += (int64_t)ND * pb.M;
        part_off += (int64_t)ND * pb.M * n_ttiles;
        P->banks.push_back(pb);
        P->total_templates += pb.M;
    }
    P->series_floats = series_off;

    // Correlation tiling: 512-column items and the longest tap split of
    // 8192..512 that still gives at least 2048 work items (8 per CU); longer
    // splits write fewer partial planes for the reduction to read back.
    // Banks too small for that get 64-column items.
    {
        auto count = [&](int cols, int split) {
            int64_t items = 0;
            for (auto &s : P->slices)
                items += (int64_t)ND * ((s.rate + cols - 1) / cols) * ((s.Npad + split - 1) / split) *
                         ((s.Lpad + kCorrMB * 16 - 1) / (kCorrMB * 16));
            return items;
        };
        P->corr_cols = count(kCorrTQ, kCorrSplitK) >= 2048 ? kCorrTQ : 64;
        P->ksplit = kCorrSplitK;
        for (int cand = 8192; cand >= kCorrSplitK; cand /= 2) {
            if (count(P->corr_cols, cand) >= 2048) {
                P->ksplit = cand;
                break;
            }
        }
    }
    P->n_peaks = peak_off;

    // ---------------------------------------------------------- rings
    int Dmax = 1;
    for (auto &s : P->slices) Dmax = std::max(Dmax, s.D);
    P->rings[1].need = F + 2LL * Dmax * ndown + 1;
    for (auto &s : P->slices) {
        Ring &r = P->rings[s.D];
        const int f = s.rate;
        const int64_t span = (s.D > 1) ? (int64_t)f - ndown + s.delay + s.N - 1 - s.la : (int64_t)F + s.delay + s.N - 1;
        r.need = std::max(r.need, std::max<int64_t>(span, f));
    }
    for (auto &kv : P->rings) {
        Ring &r = kv.second;
        if (r.need + 64 > INT32_MAX / 2) return LLOID_E_UNSUPPORTED;
        r.cap = (int32_t)round_up(r.need + 64, 64);
        r.det_stride = 2LL * r.cap;
        ST_OK(P->alloc(&r.base, (size_t)ND * r.det_stride));
    }

    // ---------------------------------------------------------- device bank
    // FP64 staging, normalisation (per bank, over all its slices), conversion
    {
        std::vector<double *> w64(P->slices.size(), nullptr);
        size_t max_u = 0;
        for (auto &s : P->slices) max_u = std::max(max_u, (size_t)s.L * s.N);
        double *u64 = nullptr;
        ST_OK(P->alloc(&u64, max_u, false));
        for (int b = 0; b < n_banks; ++b) {
            const lloid_bank &B = banks[b];
            PBank &pb = P->banks[b];
            const int rows = 2 * pb.M;
            std::vector<int32_t> Ls;
            std::vector<const double *> wp;
            int sidx0 = -1;
            for (int s = 0; s < B.n_slices; ++s) {
                const int id = (int)(std::find_if(P->slices.begin(), P->slices.end(),
                                                  [&](const PSlice &x) { return x.bank == b; }) -
                                     P->slices.begin()) + s;
                if (sidx0 < 0) sidx0 = id;
                PSlice &ps = P->slices[id];
                ST_OK(P->alloc(&w64[id], (size_t)rows * ps.L, false));
                HIP_OK(hipMemcpyAsync(w64[id], B.slices[s].mixing, sizeof(double) * rows * ps.L,
                                      hipMemcpyHostToDevice, st));
                Ls.push_back(ps.L);
                wp.push_back(w64[id]);
            }
            const double **d_wp = nullptr;
            int32_t *d_Ls = nullptr;
            double *inv = nullptr;
            ST_OK(upload(P, &d_wp, wp, st));
            ST_OK(upload(P, &d_Ls, Ls, st));
            ST_OK(P->alloc(&inv, rows, false));
            HIP_OK(launch_normalize(st, d_wp, d_Ls, (int32_t)Ls.size(), rows, P->cfg.normalize, inv));
            for (int s = 0; s < B.n_slices; ++s) {
                const int id = sidx0 + s;
                PSlice &ps = P->slices[id];
                // mixing rows [rows_pad][Lpad], basis [Lpad][Npad], zero padded
                HIP_OK(hipMemcpyAsync(u64, B.slices[s].basis, sizeof(double) * ps.L * ps.N, hipMemcpyHostToDevice,
                                      st));
                if (P->precision == LLOID_FP32) {
                    ST_OK(P->alloc(&ps.W32, (size_t)pb.rows_pad * ps.Lpad));
                    ST_OK(P->alloc(&ps.Wf32, (size_t)pb.rows_pad * ps.Lpad));
                    HIP_OK(launch_convert_rows(st, w64[id], rows, ps.L, ps.L, inv, LLOID_FP32, ROLE_ROWS, ps.W32,
                                               nullptr, nullptr, ps.Lpad, nullptr));
                    HIP_OK(launch_convert_rows(st, w64[id], rows, ps.L, ps.L, inv, LLOID_FP32, ROLE_MIXING, ps.Wf32,
                                               nullptr, nullptr, ps.Lpad, nullptr));
                    ST_OK(P->alloc(&ps.U32, (size_t)ps.Lpad * ps.Npad));
                    HIP_OK(launch_convert_rows(st, u64, ps.L, ps.N, ps.N, nullptr, LLOID_FP32, ROLE_ROWS, ps.U32,
                                               nullptr, nullptr, ps.Npad, nullptr));
                } else {
                    // 16-bit parts: hi and lo of W (bf16x3) or W alone (fp16);
                    // hi and lo of U (bf16x3) or U alone (fp16)
                    const bool split = P->precision != LLOID_FP16;   // bf16x3 mixing for BF16X3 and FP8_BF16
                    uint16_t *wh = nullptr, *wl = nullptr, *uh = nullptr, *ul = nullptr;
                    ST_OK(P->alloc(&wh, (size_t)pb.rows_pad * ps.Lpad));
                    if (split) ST_OK(P->alloc(&wl, (size_t)pb.rows_pad * ps.Lpad));
                    HIP_OK(launch_convert_rows(st, w64[id], rows, ps.L, ps.L, inv, P->precision, ROLE_MIXING, nullptr,
                                               wh, wl, ps.Lpad, nullptr));
                    if (P->precision == LLOID_FP8_BF16) {
                        // e4m3 basis, one power-of-two scale per basis vector
                        uint8_t *u8 = nullptr;
                        ST_OK(P->alloc(&u8, (size_t)ps.Lpad * ps.Npad));
                        ST_OK(P->alloc(&ps.uscale, (size_t)ps.Lpad));
                        HIP_OK(launch_convert_fp8_rows(st, u64, ps.L, ps.N, ps.N, u8, ps.Npad, ps.uscale));
                        uh = reinterpret_cast<uint16_t *>(u8);
                    } else {
                        ST_OK(P->alloc(&uh, (size_t)ps.Lpad * ps.Npad));
                        if (P->precision == LLOID_BF16X3) ST_OK(P->alloc(&ul, (size_t)ps.Lpad * ps.Npad));
                        HIP_OK(launch_convert_rows(st, u64, ps.L, ps.N, ps.N, nullptr, P->precision, ROLE_ROWS,
                                                   nullptr, uh, ul, ps.Npad, nullptr));
                    }
                    ps.Whi = wh;
                    ps.Wlo = wl;
                    ps.Uhi = uh;
                    ps.Ulo = ul;
                }
                HIP_OK(hipStreamSynchronize(st));   // u64 staging is reused
            }
            for (int s = 0; s < B.n_slices; ++s) P->release(w64[sidx0 + s]);
            P->release(d_wp);
            P->release(d_Ls);
            P->release(inv);
        }
        HIP_OK(hipStreamSynchronize(st));
        P->release(u64);
    }

    // ---------------------------------------------------------- per-slice buffers
    for (auto &s : P->slices) {
        s.ydet = (int64_t)s.Lpad * 2 * s.capY;
        ST_OK(P->alloc(&s.yring, (size_t)ND * s.ydet));
    }

    // ---------------------------------------------------------- resampler taps
    {
        std::vector<float> up((size_t)(256 - 1 + 256) * kUpTaps, 0.0f);
        for (int p = 2; p <= 256; p *= 2) {
            const int c = p * nup;
            const std::vector<double> g = sinc_windowed_sinc(p, c);
            float *z = up.data() + (size_t)(p - 1) * kUpTaps;
            for (int ph = 0; ph < p; ++ph)
                for (int t = 0; t <= 2 * nup; ++t) {
                    const int idx = t * p + ph;
                    z[ph * kUpTaps + t] = idx <= 2 * c ? (float)g[idx] : 0.0f;
                }
        }
        ST_OK(upload(P, &P->d_uptaps, up, st));
    }
    std::map<int, float *> dtaps;
    for (auto &kv : P->rings) {
        const int D = kv.first;
        if (D == 1) continue;
        const int c = D * ndown;
        std::vector<double> g = sinc_windowed_sinc(D, c);
        double sum = 0.0;
        for (double v : g) sum += v;
        std::vector<float> gf(g.size());
        for (size_t i = 0; i < g.size(); ++i) gf[i] = (float)(std::sqrt((double)D) * g[i] / sum);
        float *d = nullptr;
        ST_OK(upload(P, &d, gf, st));
        dtaps[D] = d;
    }

    // ---------------------------------------------------------- work tables
    {
        std::vector<DownItem> items;
        int lds = 0;
        const Ring &xr = P->rings[1];
        for (auto &kv : P->rings) {
            const int D = kv.first;
            if (D == 1) continue;
            const Ring &dr = kv.second;
            const int f = F / D;
            const int chunk = std::min(256, f);
            const int c = D * ndown;
            const int seg = (chunk - 1) * D + 2 * c + 1;
            lds = std::max(lds, 2 * c + 1 + seg + (seg >> 5) + 1 + 256);   // + the partial sums
            for (int det = 0; det < ND; ++det)
                for (int m0 = 0; m0 < f; m0 += chunk)
                    items.push_back(DownItem{xr.base + det * xr.det_stride, dr.base + det * dr.det_stride, dtaps[D],
                                             D, c, f, m0, std::min(chunk, f - m0), xr.cap, dr.cap, ndown});
        }
        if (lds * 4 > kMaxLdsBytes) return LLOID_E_UNSUPPORTED;
        P->down_lds = lds;
        P->n_downitems = (int)items.size();
        ST_OK(upload(P, &P->d_down, items, st));
    }
    ST_OK(build_corr_tables(P, st));
    for (auto &s : P->slices)   // algorithmic flops: correlation and mixing contractions
        P->flops += (double)ND * (2.0 * s.L * s.N * s.rate + 2.0 * 2.0 * P->banks[s.bank].M * s.L * s.rate);
    {
        std::vector<MixBank> mb;
        std::vector<MixSlice> ms;
        std::vector<MixItem> items;
        std::vector<PeakItem> pk;
        int S = 0, TP = 0;
        for (int b = 0; b < n_banks; ++b) {
            PBank &pb = P->banks[b];
            MixBank m{};
            m.M = pb.M;
            m.nlev = pb.nlev;
            int64_t lo = 0, hi = kMixTN;
            int tp = 0;   // floats of this bank's upsampling sub-kernels
            for (int j = 0; j < pb.nlev; ++j) {
                m.rate[j] = pb.rates[j];
                m.P[j] = F / pb.rates[j];
                m.shP[j] = ilog2(m.P[j]);
                if (j > 0) {
                    const int p = pb.rates[j - 1] / pb.rates[j];
                    m.p[j] = p;
                    m.shp[j] = ilog2(p);
                    m.up_off[j] = tp;
                    tp += p * kUpTaps;
                    lo = floordiv(lo, p) - nup;
                    hi = floordiv(hi - 1, p) + nup + 1;
                    S = std::max<int>(S, (int)(hi - lo));
                    if (p > 256) return LLOID_E_UNSUPPORTED;
                }
                m.lo[j] = (int)lo;
                m.n[j] = (int)(hi - lo);
            }
            int cursor = (int)ms.size();
            for (int j = 0; j <= pb.nlev; ++j) m.slice_begin[j] = cursor;
            for (int j = 0; j < pb.nlev; ++j) {
                m.slice_begin[j] = (int)ms.size();
                for (int id : pb.slices) {
                    PSlice &s = P->slices[id];
                    if (s.level != j) continue;
                    if (m.n[j] > s.capY) return LLOID_E_UNSUPPORTED;   // a tile's window must fit the ring
                    ms.push_back(MixSlice{s.Wf32, s.Whi, s.Wlo, s.yring, s.ydet, s.L, s.Lpad, s.capY, s.level, pb.rows_pad, 0});
                }
            }
            m.slice_begin[pb.nlev] = (int)ms.size();
            TP = std::max(TP, tp);
            m.series_off = pb.series_off;
            m.peak_off = pb.peak_off;
            m.part_off = pb.part_off;
            m.n_ttiles = n_ttiles;
            mb.push_back(m);
            // row tiles innermost: the work groups that run together on one
            // XCD read the same basis-output window from its L2
            for (int det = 0; det < ND; ++det) {
                for (int t0 = 0; t0 < F; t0 += kMixTN)
                    for (int r0 = 0; r0 < pb.rows_pad; r0 += kMixTM) items.push_back(MixItem{b, det, r0, t0});
                pk.push_back(PeakItem{pb.part_off + (int64_t)det * pb.M * n_ttiles, pb.peak_off + (int64_t)det * pb.M,
                                      pb.M, n_ttiles});
            }
            // upsampling flops: non-phase-0 outputs x 2 (2 N_up + 1)
            for (int j = 1; j < pb.nlev; ++j)
                P->flops += (double)ND * 2.0 * pb.M * (pb.rates[j - 1] - pb.rates[j]) * 2.0 * (2 * nup + 1);
        }
        for (auto &kv : P->rings)
            if (kv.first > 1) P->flops += (double)ND * (F / kv.first) * 2.0 * (2 * kv.first * ndown + 1);
        // level-buffer row stride: >= the widest lower-level window, 2 or 18
        // mod 32 words (the upsample's 16 rows x 2 columns per half-wave hit
        // distinct banks); every window must fit one 256-thread row load
        if (S > kMixTN) return LLOID_E_UNSUPPORTED;
        if (S > kMixS) return LLOID_E_UNSUPPORTED;
        P->mixS = kMixS;
        P->mixTP = TP;
        const size_t mix_lds = mix_lds_bytes(P->precision, P->mixS, P->mixTP);
        if (mix_lds == 0 || mix_lds > (size_t)kMaxLdsBytes) return LLOID_E_UNSUPPORTED;
        HIP_OK(configure_lds(P->precision, mix_lds, (size_t)P->down_lds * 4));
        P->n_mix = (int)items.size();
        P->n_peakitems = (int)pk.size();
        ST_OK(upload(P, &P->d_mbanks, mb, st));
        ST_OK(upload(P, &P->d_mslices, ms, st));
        P->h_mix = items;
        ST_OK(upload(P, &P->d_mix, mix_item_order(items, 1), st));
        ST_OK(upload(P, &P->d_peakitems, pk, st));
        ST_OK(P->alloc(&P->d_partials, (size_t)std::max<int64_t>(part_off, 1)));
    }
    ST_OK(P->alloc(&P->d_stride, 1));
    ST_OK(P->alloc(&P->d_instage, (size_t)ND * F));
    HIP_OK(hipStreamSynchronize(st));
    guard.p = nullptr;
    *out = P;
    return LLOID_OK;
}

void lloid_plan_destroy(lloid_plan *plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    delete plan;
}

lloid_status lloid_plan_query(const lloid_plan *P, int32_t what, int32_t index, int64_t *value) {
    if (!P || !value) return LLOID_E_ARG;
    const int nb = (int)P->banks.size();
    switch (what) {
        case LLOID_Q_N_BANKS: *value = nb; return LLOID_OK;
        case LLOID_Q_TOTAL_TEMPLATES: *value = P->total_templates; return LLOID_OK;
        case LLOID_Q_SERIES_FLOATS: *value = P->series_floats; return LLOID_OK;
        case LLOID_Q_N_PEAKS: *value = P->n_peaks; return LLOID_OK;
        case LLOID_Q_STRIDE: *value = P->stride; return LLOID_OK;
        case LLOID_Q_N_SLICES: *value = (int64_t)P->slices.size(); return LLOID_OK;
        case LLOID_Q_FLOPS_PER_STRIDE: *value = (int64_t)P->flops; return LLOID_OK;
        case LLOID_Q_DEVICE_BYTES: *value = (int64_t)P->device_bytes; return LLOID_OK;
        default: break;
    }
    if (what == LLOID_Q_OPTION) {
        switch (index) {
            case LLOID_OPT_GRAPH: *value = P->use_graph ? 1 : 0; return LLOID_OK;
            case LLOID_OPT_CORR_SPLIT: *value = P->ksplit; return LLOID_OK;
            case LLOID_OPT_CORR_GROUP: *value = P->corr_group; return LLOID_OK;
            case LLOID_OPT_MIX_GROUP: *value = P->mix_group; return LLOID_OK;
            case LLOID_OPT_MIX_TBLOCK: *value = P->mix_tblock; return LLOID_OK;
            case LLOID_OPT_CORR_COLS: *value = P->corr_cols; return LLOID_OK;
            default: return LLOID_E_ARG;
        }
    }
    if (what == LLOID_Q_SLICE_LOOKAHEAD) {
        if (index < 0 || index >= (int)P->slices.size()) return LLOID_E_ARG;
        *value = P->slices[index].la;
        return LLOID_OK;
    }
    if (index < 0 || index >= nb) return LLOID_E_ARG;
    switch (what) {
        case LLOID_Q_BANK_SERIES_OFFSET: *value = P->banks[index].series_off; return LLOID_OK;
        case LLOID_Q_BANK_PEAK_OFFSET: *value = P->banks[index].peak_off; return LLOID_OK;
        case LLOID_Q_BANK_TEMPLATES: *value = P->banks[index].M; return LLOID_OK;
        default: return LLOID_E_ARG;
    }
}

static lloid_status enqueue_stride(lloid_plan *P, hipStream_t st, const float *strain, uint32_t gap_mask,
                                   float *snr, lloid_peak *peaks, int64_t src_det_stride = 0);

lloid_status lloid_push_stride(lloid_plan *P, const float *strain, uint32_t gap_mask, float *snr, lloid_peak *peaks,
                               void *stream) {
    if (!P || !strain || !peaks) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!P->use_graph || P->profiling) {
        ST_OK(enqueue_stride(P, st, strain, gap_mask, snr, peaks));
        P->stride += 1;
        return LLOID_OK;
    }
    if (!P->gexec || P->g_snr != snr || P->g_peaks != peaks || P->g_gap != gap_mask) {
        if (P->gexec) HIP_OK(hipGraphExecDestroy(P->gexec));
        if (P->graph) HIP_OK(hipGraphDestroy(P->graph));
        P->gexec = nullptr;
        P->graph = nullptr;
        HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
        const lloid_status s = enqueue_stride(P, P->cap_stream, P->d_instage, gap_mask, snr, peaks);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
        if (s != LLOID_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return LLOID_E_HIP;
        P->graph = g;
        HIP_OK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
        P->g_snr = snr;
        P->g_peaks = peaks;
        P->g_gap = gap_mask;
    }
    HIP_OK(hipMemcpyAsync(P->d_instage, strain, sizeof(float) * P->n_det * P->F, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipGraphLaunch(P->gexec, st));
    P->stride += 1;
    return LLOID_OK;
}

lloid_status lloid_set_option(lloid_plan *P, int32_t option, int64_t value) {
    if (!P) return LLOID_E_ARG;
    if (option == LLOID_OPT_GRAPH) {
        if (value != 0 && value != 1) return LLOID_E_ARG;
        if (value && !P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        P->use_graph = value != 0;
        return LLOID_OK;
    }
    switch (option) {
        case LLOID_OPT_CORR_SPLIT:
            if (value < kCorrTK || value > 65536 || value % kCorrTK) return LLOID_E_ARG;
            break;
        case LLOID_OPT_CORR_GROUP:
            if (value < 0 || value > 64) return LLOID_E_ARG;
            break;
        case LLOID_OPT_CORR_COLS:
            if (value < 64 || value > kCorrTQ || value % 64) return LLOID_E_ARG;
            break;
        case LLOID_OPT_MIX_GROUP:
            if (value < 0 || value > 256) return LLOID_E_ARG;
            break;
        case LLOID_OPT_MIX_TBLOCK:
            if (value < 1 || value > 64) return LLOID_E_ARG;
            break;
        default:
            return LLOID_E_ARG;
    }
    // the captured graph holds the old work tables and launch shapes
    HIP_OK(hipDeviceSynchronize());
    if (P->gexec) HIP_OK(hipGraphExecDestroy(P->gexec));
    if (P->graph) HIP_OK(hipGraphDestroy(P->graph));
    P->gexec = nullptr;
    P->graph = nullptr;
    if (option == LLOID_OPT_CORR_SPLIT) {
        if (P->ksplit == (int)value) return LLOID_OK;
        P->ksplit = (int)value;
        return build_corr_tables(P, nullptr);
    }
    if (option == LLOID_OPT_CORR_COLS) {
        if (P->corr_cols == (int)value) return LLOID_OK;
        P->corr_cols = (int)value;
        return build_corr_tables(P, nullptr);
    }
    if (option == LLOID_OPT_CORR_GROUP) P->corr_group = (int)value;
    if (option == LLOID_OPT_MIX_GROUP) P->mix_group = (int)value;
    if (option == LLOID_OPT_MIX_TBLOCK && P->mix_tblock != (int)value) {
        P->mix_tblock = (int)value;
        const std::vector<MixItem> order = mix_item_order(P->h_mix, P->mix_tblock);
        HIP_OK(hipMemcpy(P->d_mix, order.data(), sizeof(MixItem) * order.size(), hipMemcpyHostToDevice));
    }
    return LLOID_OK;
}

static lloid_status enqueue_stride(lloid_plan *P, hipStream_t st, const float *strain, uint32_t gap_mask,
                                   float *snr, lloid_peak *peaks, int64_t src_det_stride) {
    LaunchCtx ctx{st, P->d_stride};
    const Ring &xr = P->rings[1];
    HIP_OK(P->mark(LLOID_K_INGEST, st, true));
    HIP_OK(launch_ingest(ctx, strain, src_det_stride ? src_det_stride : P->F, gap_mask, xr.base, xr.det_stride,
                         xr.cap, P->F, P->n_det));
    HIP_OK(P->mark(LLOID_K_INGEST, st, false));
    HIP_OK(P->mark(LLOID_K_DOWN, st, true));
    HIP_OK(launch_down(ctx, P->d_down, P->n_downitems, P->down_lds));
    HIP_OK(P->mark(LLOID_K_DOWN, st, false));
    HIP_OK(P->mark(LLOID_K_CORR, st, true));
    HIP_OK(launch_corr(ctx, P->precision, P->d_corr, P->n_corr, P->corr_group));
    HIP_OK(P->mark(LLOID_K_CORR, st, false));
    HIP_OK(P->mark(LLOID_K_REDUCE, st, true));
    HIP_OK(launch_reduce(ctx, P->precision, P->d_reduce, P->n_reduce));
    HIP_OK(P->mark(LLOID_K_REDUCE, st, false));
    HIP_OK(P->mark(LLOID_K_MIX, st, true));
    HIP_OK(launch_mix(ctx, P->precision, P->d_mix, P->n_mix, P->d_mbanks, P->d_mslices, P->d_uptaps, snr,
                      P->d_partials, P->F, P->n_det, P->mixS, P->mixTP, P->nup, P->mix_group));
    HIP_OK(P->mark(LLOID_K_MIX, st, false));
    HIP_OK(P->mark(LLOID_K_PEAKS, st, true));
    HIP_OK(launch_peaks(ctx, P->d_peakitems, P->n_peakitems, P->d_partials, peaks, P->cfg.snr_threshold,
                        P->d_stride));
    HIP_OK(P->mark(LLOID_K_PEAKS, st, false));
    return LLOID_OK;
}

static lloid_status profile_collect(lloid_plan *P) {
    if (P->ev_used == 0) return LLOID_OK;
    HIP_OK(hipEventSynchronize(P->ev_pool[P->ev_used - 1]));
    for (size_t i = 0; i < P->ev_kernel.size(); ++i) {
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, P->ev_pool[2 * i], P->ev_pool[2 * i + 1]));
        P->prof_ms[P->ev_kernel[i]] += ms;
        P->prof_n[P->ev_kernel[i]] += 1;
    }
    P->ev_used = 0;
    P->ev_kernel.clear();
    return LLOID_OK;
}

lloid_status lloid_profile_enable(lloid_plan *P, int32_t enable) {
    if (!P) return LLOID_E_ARG;
    ST_OK(profile_collect(P));
    for (int k = 0; k < LLOID_K_COUNT; ++k) {
        P->prof_ms[k] = 0.0;
        P->prof_n[k] = 0;
    }
    P->profiling = enable != 0;
    return LLOID_OK;
}

lloid_status lloid_profile_read(lloid_plan *P, int32_t kernel, double *total_ms, int64_t *launches) {
    if (!P || !total_ms || !launches || kernel < 0 || kernel >= LLOID_K_COUNT) return LLOID_E_ARG;
    ST_OK(profile_collect(P));
    *total_ms = P->prof_ms[kernel];
    *launches = P->prof_n[kernel];
    return LLOID_OK;
}

lloid_status lloid_reset(lloid_plan *P, void *stream) {
    if (!P) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (auto &kv : P->rings)
        HIP_OK(hipMemsetAsync(kv.second.base, 0, sizeof(float) * P->n_det * kv.second.det_stride, st));
    for (auto &s : P->slices) HIP_OK(hipMemsetAsync(s.yring, 0, sizeof(float) * P->n_det * s.ydet, st));
    HIP_OK(hipMemsetAsync(P->d_stride, 0, sizeof(int64_t), st));
    HIP_OK(hipStreamSynchronize(st));
    P->stride = 0;
    return LLOID_OK;
}

static size_t state_bytes(const lloid_plan *P) {
    size_t n = 4 * sizeof(uint64_t);
    for (auto &kv : P->rings) n += sizeof(float) * P->n_det * kv.second.det_stride;
    for (auto &s : P->slices) n += sizeof(float) * P->n_det * s.ydet;
    return n;
}

static uint64_t layout_tag(const lloid_plan *P) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix(P->F);
    mix(P->n_det);
    for (auto &kv : P->rings) {
        mix(kv.first);
        mix(kv.second.cap);
    }
    for (auto &s : P->slices) {
        mix(s.Lpad);
        mix(s.capY);
        mix(s.rate);
    }
    return h;
}

lloid_status lloid_state_size(const lloid_plan *P, size_t *bytes) {
    if (!P || !bytes) return LLOID_E_ARG;
    *bytes = state_bytes(P);
    return LLOID_OK;
}

lloid_status lloid_state_save(lloid_plan *P, void *dst, size_t bytes, void *stream) {
    if (!P || !dst || bytes < state_bytes(P)) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint64_t *h = static_cast<uint64_t *>(dst);
    h[0] = kStateMagic;
    h[1] = layout_tag(P);
    h[2] = (uint64_t)P->stride;
    h[3] = 0;
    char *c = static_cast<char *>(dst) + 4 * sizeof(uint64_t);
    for (auto &kv : P->rings) {
        const size_t n = sizeof(float) * P->n_det * kv.second.det_stride;
        HIP_OK(hipMemcpyAsync(c, kv.second.base, n, hipMemcpyDeviceToHost, st));
        c += n;
    }
    for (auto &s : P->slices) {
        const size_t n = sizeof(float) * P->n_det * s.ydet;
        HIP_OK(hipMemcpyAsync(c, s.yring, n, hipMemcpyDeviceToHost, st));
        c += n;
    }
    HIP_OK(hipStreamSynchronize(st));
    return LLOID_OK;
}

lloid_status lloid_state_load(lloid_plan *P, const void *src, size_t bytes, void *stream) {
    if (!P || !src || bytes < state_bytes(P)) return LLOID_E_ARG;
    const uint64_t *h = static_cast<const uint64_t *>(src);
    if (h[0] != kStateMagic || h[1] != layout_tag(P)) return LLOID_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *c = static_cast<const char *>(src) + 4 * sizeof(uint64_t);
    for (auto &kv : P->rings) {
        const size_t n = sizeof(float) * P->n_det * kv.second.det_stride;
        HIP_OK(hipMemcpyAsync(kv.second.base, c, n, hipMemcpyHostToDevice, st));
        c += n;
    }
    for (auto &s : P->slices) {
        const size_t n = sizeof(float) * P->n_det * s.ydet;
        HIP_OK(hipMemcpyAsync(s.yring, c, n, hipMemcpyHostToDevice, st));
        c += n;
    }
    const int64_t k = (int64_t)h[2];
    HIP_OK(hipMemcpyAsync(P->d_stride, &k, sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    P->stride = k;
    return LLOID_OK;
}

lloid_status lloid_inspect(lloid_plan *P, int32_t what, int32_t index, int32_t det, int64_t m_lo, int64_t m_hi,
                           float *dst, void *stream) {
    if (!P || !dst || det < 0 || det >= P->n_det || m_hi < m_lo) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OK(hipStreamSynchronize(st));
    const int64_t len = m_hi - m_lo;
    if (what == LLOID_INSPECT_DOWNSAMPLED) {
        auto itr = P->rings.find(index);
        if (itr == P->rings.end()) return LLOID_E_ARG;
        const Ring &r = itr->second;
        const int f = P->F / index;
        const int64_t newest = index == 1 ? P->stride * P->F - 1 : P->stride * f - P->ndown - 1;
        if (m_hi - 1 > newest || m_lo <= newest - r.cap || len > r.cap) return LLOID_E_STATE;
        const int64_t pos = ((m_lo % r.cap) + r.cap) % r.cap;
        HIP_OK(hipMemcpy(dst, r.base + det * r.det_stride + pos, sizeof(float) * len, hipMemcpyDeviceToHost));
        return LLOID_OK;
    }
    if (what == LLOID_INSPECT_BASIS_OUT) {
        if (index < 0 || index >= (int)P->slices.size()) return LLOID_E_ARG;
        const PSlice &s = P->slices[index];
        const int64_t newest = P->stride * s.rate + s.la - 1;
        if (m_hi - 1 > newest || m_lo <= newest - s.capY || len > s.capY) return LLOID_E_STATE;
        float *tmp = nullptr;
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMalloc(&tmp, sizeof(float) * (size_t)s.L * len));
        hipError_t e = launch_ring_gather(nullptr, P->precision, s.yring + det * s.ydet, s.Lpad, s.capY, m_lo,
                                          (int32_t)len, s.L, tmp, len, 0);
        if (e == hipSuccess) e = hipMemcpy(dst, tmp, sizeof(float) * (size_t)s.L * len, hipMemcpyDeviceToHost);
        (void)hipFree(tmp);
        HIP_OK(e);
        return LLOID_OK;
    }
    return LLOID_E_ARG;
}

// ------------------------------------------------------------------ gradient
// Forward over the segment with the stride kernels, capturing each stride's
// new basis-output columns and decimated samples and the residual; then per
// bank and detector the transposed upsampling chain and, per slice, the
// three contractions of dL/dW, dL/dY and dL/dU (the last one on the
// correlation kernel: a Hankel window of the decimated strain again).
namespace {
constexpr int64_t kGradSplitU = 8192;    // K split of dU (K = time)
// zero tail of the gradient's linear strain segments: the correlation reads
// up to kCorrTQ + 64 samples past a window start
constexpr int64_t kSegPad = kCorrTQ + 64;
constexpr int kLossBlocks = 1024;   // residual work groups (loss partials) per stride, bank and detector

// K split of dW = 2 G Y^T (K = time at the slice's rate): 128 splits of
// the top rate's 64 s segment, at least 512 samples each
int64_t dw_split(int64_t k) { return std::max<int64_t>(512, round_up((k + 127) / 128, 256)); }

int64_t seg_lo(const PBank &b, int j, int nup) {
    int64_t lo = 0;
    for (int i = 1; i <= j; ++i) lo = floordiv(lo, b.rates[i - 1] / b.rates[i]) - nup;
    return lo;
}
int64_t seg_hi(const PBank &b, int j, int nup, int64_t top) {
    int64_t hi = top;
    for (int i = 1; i <= j; ++i) hi = floordiv(hi - 1, b.rates[i - 1] / b.rates[i]) + nup + 1;
    return hi;
}
}  // namespace

lloid_status lloid_grad(lloid_plan *P, const float *strain, int32_t T, const float *target, double *loss_out,
                        float *dW, float *dU, void *stream) {
    if (!P || !strain || !target || !loss_out || !dW || !dU || T < 1) return LLOID_E_ARG;
    if (P->precision != LLOID_FP32) return LLOID_E_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int F = P->F, ND = P->n_det, nup = P->nup;
    const int64_t TF = (int64_t)T * F;
    std::vector<void *> tmp;   // per-call buffers, freed on return
    struct Free {
        lloid_plan *P;
        std::vector<void *> *v;
        ~Free() {
            (void)hipDeviceSynchronize();
            for (void *p : *v) P->release(p);
        }
    } guard{P, &tmp};
    auto get = [&](auto **p, size_t n, bool zero) -> lloid_status {
        ST_OK(P->alloc(p, n, zero));
        tmp.push_back(*p);
        return LLOID_OK;
    };
    // the caller's streaming state (history and stride counter) is saved to
    // host memory and restored on every return, so a live plan can be
    // differentiated without losing its history
    std::vector<uint64_t> saved((state_bytes(P) + sizeof(uint64_t) - 1) / sizeof(uint64_t));
    ST_OK(lloid_state_save(P, saved.data(), saved.size() * sizeof(uint64_t), stream));
    struct Restore {
        lloid_plan *P;
        std::vector<uint64_t> *blob;
        void *stream;
        bool graph;
        ~Restore() {
            (void)hipDeviceSynchronize();
            (void)lloid_state_load(P, blob->data(), blob->size() * sizeof(uint64_t), stream);
            P->use_graph = graph;
        }
    } restore{P, &saved, stream, P->use_graph};
    ST_OK(lloid_reset(P, stream));
    const bool graph = P->use_graph;
    P->use_graph = false;

    // ---- workspace
    float *series = nullptr;
    lloid_peak *peaks = nullptr;
    ST_OK(get(&series, (size_t)P->series_floats, false));
    ST_OK(get(&peaks, (size_t)P->n_peaks, false));
    const int nbd = (int)P->banks.size() * ND;
    double *loss_part = nullptr, *loss_d = nullptr;
    ST_OK(get(&loss_part, (size_t)T * nbd * kLossBlocks, true));
    ST_OK(get(&loss_d, 1, true));
    int64_t *zero = nullptr;
    ST_OK(get(&zero, 1, true));
    // residual rows [2 M][RLD], zero past TF (the products read whole 32-sample chunks)
    const int64_t RLD = round_up(TF, 64);
    std::vector<float *> R(nbd, nullptr);
    for (size_t b = 0; b < P->banks.size(); ++b)
        for (int d = 0; d < ND; ++d) ST_OK(get(&R[b * ND + d], (size_t)2 * P->banks[b].M * RLD, true));
    const int ns = (int)P->slices.size();
    std::vector<float *> yseg(ns, nullptr);
    std::vector<int64_t> qld(ns), slo(ns), sq(ns);
    std::map<int, int64_t> dlo;
    for (int i = 0; i < ns; ++i) {
        const PSlice &s = P->slices[i];
        const PBank &b = P->banks[s.bank];
        slo[i] = seg_lo(b, s.level, nup);
        sq[i] = seg_hi(b, s.level, nup, TF) - slo[i];
        qld[i] = round_up(sq[i], 64);
        ST_OK(get(&yseg[i], (size_t)ND * s.Lpad * qld[i], true));
        const int64_t need = slo[i] - s.delay - (s.N - 1);
        dlo[s.D] = std::min(dlo.count(s.D) ? dlo[s.D] : 0, need);
    }
    std::map<int, float *> dseg;
    std::map<int, int64_t> dlen;
    for (auto &kv : dlo) {
        const int D = kv.first;
        dlen[D] = TF / D - kv.second + 256;
        ST_OK(get(&dseg[D], (size_t)ND * (dlen[D] + kSegPad), true));
    }

    // ---- capture table: per stride, every slice's basis outputs (its L rows,
    // `rate` new positions at k rate + la) and every decimated stream (F / D
    // new samples) into the linear segments, one launch
    std::vector<CaptureItem> cap;
    std::vector<int32_t> caprow;
    int32_t cap_len = 0;
    auto add_item = [&](CaptureItem it, int rows) {
        it.row0 = (int32_t)caprow.size();
        for (int r = 0; r < rows; ++r) caprow.push_back((int32_t)cap.size());
        cap_len = std::max(cap_len, it.len);
        cap.push_back(it);
    };
    for (int i = 0; i < ns; ++i) {
        const PSlice &s = P->slices[i];
        for (int d = 0; d < ND; ++d)
            add_item(CaptureItem{s.yring + d * s.ydet, 0, s.la, s.rate, yseg[i] + (int64_t)d * s.Lpad * qld[i], qld[i],
                                 slo[i], s.capY, 1, s.rate, 0},
                     s.L);
    }
    for (auto &kv : dseg) {
        const int D = kv.first;
        const Ring &r = P->rings[D];
        const int f = F / D;
        for (int d = 0; d < ND; ++d)
            add_item(CaptureItem{r.base + d * r.det_stride, 0, D == 1 ? 0 : -(int64_t)P->ndown, D == 1 ? F : f,
                                 kv.second + d * (dlen[D] + kSegPad), 0, dlo[D], r.cap, 0, f, 0},
                     1);
    }
    const int32_t cap_rows = (int32_t)caprow.size();
    CaptureItem *d_cap = nullptr;
    int32_t *d_caprow = nullptr;
    ST_OK(get(&d_cap, cap.size(), false));
    ST_OK(get(&d_caprow, std::max<size_t>(caprow.size(), 1), false));
    HIP_OK(hipMemcpyAsync(d_cap, cap.data(), sizeof(CaptureItem) * cap.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(d_caprow, caprow.data(), sizeof(int32_t) * caprow.size(), hipMemcpyHostToDevice, st));

    // ---- forward with capture
    for (int k = 0; k < T; ++k) {
        ST_OK(enqueue_stride(P, st, strain + (int64_t)k * F, 0, series, peaks, TF));
        for (size_t b = 0; b < P->banks.size(); ++b) {
            const PBank &pb = P->banks[b];
            for (int d = 0; d < ND; ++d) {
                const int64_t so = pb.series_off + (int64_t)d * pb.M * F * 2;
                HIP_OK(launch_residual(st, series + so, target + (int64_t)k * P->series_floats + so, pb.M, F,
                                       R[b * ND + d], RLD, (int64_t)k * F,
                                       loss_part + ((int64_t)k * nbd + b * ND + d) * kLossBlocks, kLossBlocks));
            }
        }
        HIP_OK(launch_capture(st, d_cap, d_caprow, cap_rows, cap_len, k));
    }
    P->stride = T;
    P->use_graph = graph;
    HIP_OK(launch_sum_f64(st, loss_part, T * nbd * kLossBlocks, loss_d));

    // ---- transposed chain and contractions
    int64_t gmax = 0, pmax = 0, dymax = 0;
    for (int i = 0; i < ns; ++i) {
        const PSlice &s = P->slices[i];
        const int64_t rows = 2LL * P->banks[s.bank].M;
        pmax = std::max(pmax, ((sq[i] + dw_split(sq[i]) - 1) / dw_split(sq[i])) * rows * s.L);
        pmax = std::max(pmax, (qld[i] / kGradSplitU + 1) * s.Lpad * s.N);
        dymax = std::max(dymax, (int64_t)s.Lpad * qld[i]);
    }
    for (auto &pb : P->banks)
        for (int j = 1; j < pb.nlev; ++j)
            gmax = std::max<int64_t>(gmax, 2LL * pb.M * round_up(seg_hi(pb, j, nup, TF) - seg_lo(pb, j, nup), 64));
    float *part = nullptr, *dy = nullptr, *g1 = nullptr, *g2 = nullptr;
    ST_OK(get(&part, (size_t)pmax, false));
    ST_OK(get(&dy, (size_t)dymax, false));
    ST_OK(get(&g1, (size_t)std::max<int64_t>(gmax, 1), false));
    ST_OK(get(&g2, (size_t)std::max<int64_t>(gmax, 1), false));
    CorrItem *d_items = nullptr;
    int64_t max_items = 1;
    for (int i = 0; i < ns; ++i)
        max_items = std::max(max_items, ((P->slices[i].N + kCorrTQ - 1) / kCorrTQ) * (qld[i] / kGradSplitU + 1) *
                                            ((P->slices[i].Lpad + kCorrMB * 16 - 1) / (kCorrMB * 16)));
    ST_OK(get(&d_items, (size_t)max_items, false));

    std::vector<int64_t> offW(ns), offU(ns);
    int64_t ow = 0, ou = 0;
    for (int i = 0; i < ns; ++i) {
        offW[i] = ow;
        offU[i] = ou;
        ow += 2LL * P->banks[P->slices[i].bank].M * P->slices[i].L;
        ou += (int64_t)P->slices[i].L * P->slices[i].N;
    }
    for (size_t b = 0; b < P->banks.size(); ++b) {
        const PBank &pb = P->banks[b];
        const int64_t rows = 2LL * pb.M;
        for (int d = 0; d < ND; ++d) {
            const float *G = R[b * ND + d];
            int64_t glo = 0, gn = TF, gld = RLD;   // G: [rows][gld], level indices glo .. glo + gn - 1
            float *bufs[2] = {g1, g2};
            for (int j = 0; j < pb.nlev; ++j) {
                if (j > 0) {
                    const int p = pb.rates[j - 1] / pb.rates[j];
                    const int64_t lo = seg_lo(pb, j, nup), n = seg_hi(pb, j, nup, TF) - lo;
                    float *out = bufs[j & 1];
                    const int64_t nld = round_up(n, 64);
                    HIP_OK(launch_upsample_adjoint(st, G, gld, glo, gn, out, nld, lo, n, (int32_t)rows, p, nup,
                                                   P->d_uptaps + (p - 1) * kUpTaps));
                    G = out;
                    glo = lo;
                    gn = n;
                    gld = nld;
                }
                for (int i : pb.slices) {
                    const PSlice &s = P->slices[i];
                    if (s.level != j) continue;
                    const float *Y = yseg[i] + (int64_t)d * s.Lpad * qld[i];
                    // dW = 2 G Y^T  (Y rows zero past L and columns zero past gn, like G's)
                    const int64_t ks = dw_split(gn), nw = (gn + ks - 1) / ks;
                    HIP_OK(launch_gemm_abt(st, G, gld, Y, qld[i], (int32_t)rows, s.L, gn, ks, part));
                    HIP_OK(launch_sum_parts(st, part, (int32_t)nw, rows * s.L, (int32_t)rows, s.L, s.L,
                                            dW + offW[i], s.L, 2.0f, d > 0));
                    // dY = 2 W^T G  into [Lpad][qld] (qld == gld), every element written
                    HIP_OK(launch_gemm_atb(st, s.W32, s.Lpad, G, gld, (int32_t)rows, qld[i], 2.0f, dy, qld[i]));
                    // dU[l][n] = sum_q dY[l][q] d[q + lo - delay - (N-1) + n]
                    std::vector<CorrItem> items;
                    const int64_t nsu = (qld[i] + kGradSplitU - 1) / kGradSplitU;
                    for (int64_t sp = 0; sp < nsu; ++sp)
                        for (int c0 = 0; c0 < s.N; c0 += kCorrTQ)
                        for (int r0 = 0; r0 < s.Lpad; r0 += kCorrMB * 16) {
                            CorrItem it{};
                            it.U = dy;
                            it.ring = dseg[s.D] + d * (dlen[s.D] + kSegPad);
                            it.part = part + sp * s.Lpad * s.N;
                            it.off = glo - s.delay - (s.N - 1) - dlo[s.D];
                            it.Npad = (int32_t)qld[i];
                            it.Lpad = s.Lpad;
                            it.cap = (int32_t)dlen[s.D];
                            it.f = s.N;
                            it.col0 = c0;
                            it.ncols = std::min(kCorrTQ, s.N - c0);
                            it.k0 = (int32_t)(sp * kGradSplitU);
                            it.klen = (int32_t)std::min<int64_t>(kGradSplitU, qld[i] - sp * kGradSplitU);
                            it.mb = std::min(kCorrMB, (s.Lpad - r0) / 16);
                            it.r0 = r0;
                            items.push_back(it);
                        }
                    HIP_OK(hipMemcpyAsync(d_items, items.data(), sizeof(CorrItem) * items.size(),
                                          hipMemcpyHostToDevice, st));
                    LaunchCtx ctx{st, zero};
                    HIP_OK(launch_corr(ctx, LLOID_FP32, d_items, (int32_t)items.size(), 0));
                    HIP_OK(launch_sum_parts(st, part, (int32_t)nsu, (int64_t)s.Lpad * s.N, s.L, s.N, s.N,
                                            dU + offU[i], s.N, 1.0f, d > 0));
                    HIP_OK(hipStreamSynchronize(st));   // items buffer reused
                }
            }
        }
    }
    HIP_OK(hipMemcpyAsync(loss_out, loss_d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return LLOID_OK;
}

lloid_status lloid_set_slice(lloid_plan *P, int32_t slice, const double *U, const double *W, void *stream) {
    if (!P || !U || !W || slice < 0 || slice >= (int)P->slices.size()) return LLOID_E_ARG;
    if (P->cfg.normalize) return LLOID_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    PSlice &s = P->slices[slice];
    const int rows = 2 * P->banks[s.bank].M;
    if (P->precision == LLOID_FP32) {
        HIP_OK(launch_convert_rows(st, W, rows, s.L, s.L, nullptr, LLOID_FP32, ROLE_ROWS, s.W32, nullptr, nullptr,
                                   s.Lpad, nullptr));
        HIP_OK(launch_convert_rows(st, W, rows, s.L, s.L, nullptr, LLOID_FP32, ROLE_MIXING, s.Wf32, nullptr, nullptr,
                                   s.Lpad, nullptr));
        HIP_OK(launch_convert_rows(st, U, s.L, s.N, s.N, nullptr, LLOID_FP32, ROLE_ROWS, s.U32, nullptr, nullptr,
                                   s.Npad, nullptr));
    } else {
        HIP_OK(launch_convert_rows(st, W, rows, s.L, s.L, nullptr, P->precision, ROLE_MIXING, nullptr, s.Whi, s.Wlo,
                                   s.Lpad, nullptr));
        if (P->precision == LLOID_FP8_BF16) {
            // e4m3 basis with its per-vector scales, as at plan creation
            HIP_OK(launch_convert_fp8_rows(st, U, s.L, s.N, s.N, static_cast<uint8_t *>(s.Uhi), s.Npad, s.uscale));
        } else {
            HIP_OK(launch_convert_rows(st, U, s.L, s.N, s.N, nullptr, P->precision, ROLE_ROWS, nullptr, s.Uhi, s.Ulo,
                                       s.Npad, nullptr));
        }
    }
    HIP_OK(hipStreamSynchronize(st));
    return LLOID_OK;
}

lloid_status lloid_set_autocorrelation(lloid_plan *P, const double *acf, const int32_t *acf_len, void *stream) {
    if (!P || !acf || !acf_len) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<XiTemplate> tab;
    tab.reserve((size_t)P->total_templates);
    int64_t floats = 0;
    for (size_t b = 0; b < P->banks.size(); ++b) {
        const int A = acf_len[b];
        if (A < 3 || A % 2 == 0 || A > 2 * P->F + 1) return LLOID_E_SHAPE;
        const PBank &pb = P->banks[b];
        for (int m = 0; m < pb.M; ++m) {
            XiTemplate e{};
            e.series_off = pb.series_off + (int64_t)m * P->F * 2;
            e.det_stride = (int64_t)pb.M * P->F * 2;
            e.peak_off = pb.peak_off + m;
            e.acf_off = floats;
            e.A = A;
            e.M = pb.M;
            tab.push_back(e);
            floats += 2 * (int64_t)A;
        }
    }
    // drop earlier autocorrelations (hipFree waits for work that uses them)
    P->release(P->d_acf);
    P->release(P->d_xitab);
    P->device_bytes -= P->xi_bytes;
    P->d_acf = nullptr;
    P->d_xitab = nullptr;
    P->n_xi = 0;
    const size_t before = P->device_bytes;
    float *acf32 = nullptr;
    XiTemplate *xtab = nullptr;
    ST_OK(P->alloc(&acf32, (size_t)floats, false));
    ST_OK(upload(P, &xtab, tab, st));
    HIP_OK(launch_convert_f64_f32(st, acf, floats, acf32));
    HIP_OK(hipStreamSynchronize(st));
    P->xi_bytes = P->device_bytes - before;
    P->d_acf = acf32;
    P->d_xitab = xtab;
    P->n_xi = (int32_t)tab.size();
    return LLOID_OK;
}

lloid_status lloid_xi2(lloid_plan *P, const float *prev, const float *cur, const float *next, const lloid_peak *peaks,
                       float *out, void *stream) {
    if (!P || !cur || !peaks || !out) return LLOID_E_ARG;
    if (!P->d_xitab) return LLOID_E_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OK(P->mark(LLOID_K_XI2, st, true));
    HIP_OK(launch_xi2(st, P->d_xitab, P->n_xi, P->n_det, P->F, prev, cur, next, peaks, P->d_acf, out));
    HIP_OK(P->mark(LLOID_K_XI2, st, false));
    return LLOID_OK;
}

lloid_status lloid_coincidence(lloid_plan *P, const float *prev, const lloid_peak *peaks, int32_t overlap,
                               const int32_t *window, lloid_peak *triggers, lloid_event *events, void *stream) {
    if (!P || !peaks || !window || !triggers || !events) return LLOID_E_ARG;
    if (P->n_det > kCoincMaxDet) return LLOID_E_UNSUPPORTED;
    if (overlap < 0 || overlap > P->F) return LLOID_E_SHAPE;
    CoincWindows w{};
    for (int a = 0; a < P->n_det; ++a)
        for (int d = 0; d < P->n_det; ++d) {
            if (window[a * P->n_det + d] < 0) return LLOID_E_SHAPE;
            w.w[a][d] = window[a * P->n_det + d];
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!P->d_trigtab) {
        std::vector<TrigTemplate> tab;
        std::vector<CoincBank> cb;
        tab.reserve((size_t)P->total_templates);
        for (const PBank &pb : P->banks) {
            for (int m = 0; m < pb.M; ++m) {
                TrigTemplate e{};
                e.series_off = pb.series_off + (int64_t)m * P->F * 2;
                e.det_stride = (int64_t)pb.M * P->F * 2;
                e.peak_off = pb.peak_off + m;
                e.M = pb.M;
                tab.push_back(e);
            }
            CoincBank c{};
            c.peak_off = pb.peak_off;
            c.M = pb.M;
            cb.push_back(c);
        }
        TrigTemplate *t = nullptr;
        CoincBank *c = nullptr;
        ST_OK(upload(P, &t, tab, st));
        ST_OK(upload(P, &c, cb, st));
        HIP_OK(hipStreamSynchronize(st));
        P->d_trigtab = t;
        P->d_coincbanks = c;
    }
    HIP_OK(P->mark(LLOID_K_TRIGGERS, st, true));
    HIP_OK(launch_window_triggers(st, P->d_trigtab, (int32_t)P->total_templates, P->n_det, P->F, prev, peaks, overlap,
                                  P->cfg.snr_threshold, triggers));
    HIP_OK(P->mark(LLOID_K_TRIGGERS, st, false));
    HIP_OK(P->mark(LLOID_K_COINC, st, true));
    HIP_OK(launch_coinc(st, P->d_coincbanks, (int32_t)P->banks.size(), P->n_det, w, triggers, events));
    HIP_OK(P->mark(LLOID_K_COINC, st, false));
    return LLOID_OK;
}

lloid_status lloid_orthonormalize(double *U, int32_t L, int32_t N, double *W, int32_t rows, void *stream) {
    if (!U || !W || L < 1 || L > kMaxBasis || N < L || rows < 1) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *G = nullptr;
    int32_t *info = nullptr;
    if (hipMalloc(&G, sizeof(double) * 2 * L * L) != hipSuccess) return LLOID_E_NOMEM;   // G, then C^-1
    if (hipMalloc(&info, sizeof(int32_t) * 2) != hipSuccess) {
        (void)hipFree(G);
        return LLOID_E_NOMEM;
    }
    int32_t h[2] = {0, 0};
    hipError_t e = launch_clear_info(st, info, 2);
    if (e == hipSuccess) e = launch_cholesky_qr2(st, U, L, N, W, rows, G, G + L * L, info);
    if (e == hipSuccess) e = hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(G);
    (void)hipFree(info);
    if (e != hipSuccess) return LLOID_E_HIP;
    return (h[0] || h[1]) ? LLOID_E_STATE : LLOID_OK;
}

lloid_status lloid_orthonormalize_noalloc(double *U, int32_t L, int32_t N, double *W, int32_t rows,
                                          int32_t *info_dev, void *stream) {
    if (!U || !W || L < 1 || N < L || rows < 1) return LLOID_E_ARG;
    if (L > kNoAllocMaxBasis) return LLOID_E_UNSUPPORTED;   // the Gram matrix would not fit the scratch array
    double *base = nullptr;
    if (scratch_address(&base) != hipSuccess) return LLOID_E_HIP;
    double *G = base, *Cinv = base + kScratchGramDoubles;
    int32_t *info = info_dev ? info_dev : reinterpret_cast<int32_t *>(base + 2 * kScratchGramDoubles);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_clear_info(st, info, 2);
    if (e == hipSuccess) e = launch_cholesky_qr2(st, U, L, N, W, rows, G, Cinv, info);
    return e == hipSuccess ? LLOID_OK : LLOID_E_HIP;
}

}  // extern "C"
