// PSD estimation and whitening with frequency-domain downsampling
// (Sec. II.B.2), one stream per detector, all detectors in each launch.
//
// Per push of H = N/2 - Z new samples: the last 2H inputs times a periodic
// Hann window, zero-padded by Z on each side, go through an N-point FFT; the
// first N/(2D) + 1 bins are kept (downsampling by D in the frequency
// domain); each bin's instantaneous PSD |X|^2 / sum(hann^2) enters a ring of
// the last n_med estimates, whose median (of the c most recent, c odd),
// divided by the chi^2_2 median-to-geometric-mean factor, updates a running
// log geometric mean; PSD = geometric mean x e^gamma.  The bins divided by
// sqrt(D PSD) go through an N/D-point inverse FFT, are tapered by a Tukey
// window and overlap-added; the first H/D samples of the accumulator are
// the output.
//
// The FFTs are radix-4 Stockham passes through global memory (self-sorting,
// one launch per pass, one 4-point butterfly per thread; one radix-2 pass
// first when log2 N is odd): the transforms are small (at most a few
// hundred KB per detector) and bound by launch latency, not bandwidth.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/lloid.h"
#include "lloid_whiten.h"

namespace lloid {
namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Windowed, zero-padded block: n in [0, N); the segment is the previous H
// inputs followed by the new H.  prev_out receives the new H inputs (zeros
// for a gap) for the next push.
__global__ void whiten_block_kernel(const float *__restrict__ in, int64_t in_ld, const float *__restrict__ prev_in,
                                    float *__restrict__ prev_out, const float *__restrict__ hann, int32_t N,
                                    int32_t Z, int32_t H, uint32_t gap_mask, f32x2 *__restrict__ blk) {
    const int det = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool gap = (gap_mask >> det) & 1u;
    const int m = n - Z;
    float v = 0.f;
    if (m >= 0 && m < 2 * H) {
        const float x = m < H ? prev_in[(int64_t)det * H + m] : (gap ? 0.f : in[det * in_ld + (m - H)]);
        v = hann[m] * x;
    }
    blk[(int64_t)det * N + n] = f32x2{v, 0.f};
    if (n < H) prev_out[(int64_t)det * H + n] = gap ? 0.f : in[det * in_ld + n];
}

// One radix-2 Stockham pass of an N-point transform with butterfly half-size
// m: reads j and j + N/2, writes 2m floor(j/m) + (j mod m) and that + m.
// Twiddle exp(sign 2 pi i k / 2m) = table[k * twstep] (conjugated for the
// inverse), table[q] = exp(-2 pi i q / N_table).
__global__ void fft_pass_kernel(const f32x2 *__restrict__ src, f32x2 *__restrict__ dst, int32_t N, int32_t m,
                                int32_t twstep, int32_t inverse, const f32x2 *__restrict__ tw) {
    const int det = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N / 2) return;
    const f32x2 *x = src + (int64_t)det * N;
    f32x2 *y = dst + (int64_t)det * N;
    const int k = j & (m - 1);
    const f32x2 a = x[j], b = x[j + N / 2];
    f32x2 w = tw[(int64_t)k * twstep];
    if (inverse) w.y = -w.y;
    const f32x2 wb = f32x2{w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x};
    const int o = ((j - k) << 1) + k;
    y[o] = a + wb;
    y[o + m] = a - wb;
}

// One radix-4 Stockham pass with sub-transform size m: reads j + q N/4
// (q = 0..3), twiddles exp(sign 2 pi i q k / 4m), a 4-point DFT, writes
// 4m floor(j/m) + (j mod m) + q m.
__global__ void fft_pass4_kernel(const f32x2 *__restrict__ src, f32x2 *__restrict__ dst, int32_t N, int32_t m,
                                 int32_t twstep, int32_t inverse, const f32x2 *__restrict__ tw) {
    const int det = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int Q = N / 4;
    if (j >= Q) return;
    const f32x2 *x = src + (int64_t)det * N;
    f32x2 *y = dst + (int64_t)det * N;
    const int k = j & (m - 1);
    f32x2 a[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x2 v = x[j + q * Q];
        if (q == 0) {
            a[0] = v;
        } else {
            f32x2 w = tw[(int64_t)q * k * twstep];
            if (inverse) w.y = -w.y;
            a[q] = f32x2{w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x};
        }
    }
    const f32x2 b0 = a[0] + a[2], b1 = a[0] - a[2], b2 = a[1] + a[3], d = a[1] - a[3];
    // (a1 - a3) times -i (forward) or +i (inverse)
    const f32x2 b3 = inverse ? f32x2{-d.y, d.x} : f32x2{d.y, -d.x};
    const int o = 4 * (j - k) + k;
    y[o] = b0 + b2;
    y[o + m] = b1 + b3;
    y[o + 2 * m] = b0 - b2;
    y[o + 3 * m] = b1 - b3;
}

// Per bin k < K = N_out/2 + 1: instantaneous PSD into the ring, running
// estimate, whitened bin into the inverse transform's input (Hermitian
// extension; real DC and Nyquist bins).
__global__ void whiten_psd_kernel(const f32x2 *__restrict__ X, int32_t N, int32_t K, int32_t n_out,
                                  float inv_w2, float *__restrict__ ring, int32_t n_med, float *__restrict__ log_geo,
                                  WhitenDetState st, const float *__restrict__ beta, float d_factor,
                                  f32x2 *__restrict__ Y) {
    const int det = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K || ((st.gap_mask >> det) & 1u)) return;
    const f32x2 x = X[(int64_t)det * N + k];
    const float p = (x.x * x.x + x.y * x.y) * inv_w2;
    const int blocks = st.blocks[det];                   // including this one
    float *r = ring + (int64_t)det * n_med * K;
    r[(int64_t)((blocks - 1) % n_med) * K + k] = p;
    int c = blocks < n_med ? blocks : n_med;
    c -= 1 - (c & 1);                                    // largest odd count
    float v[kWhitenMaxMed];
    for (int i = 0; i < c; ++i) v[i] = (i == 0) ? p : r[(int64_t)((blocks - 1 - i + n_med) % n_med) * K + k];
    for (int i = 1; i < c; ++i) {                        // insertion sort, c <= 15
        const float t = v[i];
        int q = i - 1;
        while (q >= 0 && v[q] > t) {
            v[q + 1] = v[q];
            --q;
        }
        v[q + 1] = t;
    }
    const float med = v[c / 2];
    float *lg = log_geo + (int64_t)det * K + k;
    const int cnt = blocks < st.n_avg ? blocks : st.n_avg;
    const float g = *lg + (logf(med / beta[c]) - *lg) / (float)cnt;
    *lg = g;
    const float psd = expf(g) * kEulerGammaExp;
    const float s = 1.f / sqrtf(d_factor * psd);
    f32x2 yk = f32x2{x.x * s, x.y * s};
    f32x2 *y = Y + (int64_t)det * n_out;
    if (k == 0 || k == K - 1) yk.y = 0.f;
    y[k] = yk;
    if (k > 0 && k < K - 1) y[n_out - k] = f32x2{yk.x, -yk.y};
}

// Tukey-windowed overlap-add of the inverse transform (scaled by 1/N_out),
// output of the first H_out samples, accumulator shifted into acc_out.
__global__ void whiten_ola_kernel(const f32x2 *__restrict__ y, const float *__restrict__ tukey, int32_t n_out,
                                  int32_t h_out, uint32_t gap_mask, const float *__restrict__ acc_in,
                                  float *__restrict__ acc_out, float *__restrict__ out, int64_t out_ld) {
    const int det = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_out) return;
    const bool gap = (gap_mask >> det) & 1u;
    float v = acc_in[(int64_t)det * n_out + n];
    if (!gap) v += tukey[n] * y[(int64_t)det * n_out + n].x * (1.f / (float)n_out);
    if (n < h_out) {
        out[det * out_ld + n] = v;
        acc_out[(int64_t)det * n_out + n_out - h_out + n] = 0.f;
    } else {
        acc_out[(int64_t)det * n_out + n - h_out] = v;
    }
}

// PSD = exp(log geometric mean) x e^gamma
__global__ void whiten_exp_kernel(const float *__restrict__ lg, int64_t n, float *__restrict__ psd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) psd[i] = expf(lg[i]) * kEulerGammaExp;
}

}  // namespace

hipError_t launch_whiten_exp(hipStream_t st, const float *lg, int64_t n, float *psd) {
    hipLaunchKernelGGL(whiten_exp_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lg, n, psd);
    return hipGetLastError();
}

hipError_t launch_whiten_block(hipStream_t st, const float *in, int64_t in_ld, const float *prev_in, float *prev_out,
                               const float *hann, int32_t N, int32_t Z, int32_t H, uint32_t gap_mask, int32_t n_det,
                               void *blk) {
    hipLaunchKernelGGL(whiten_block_kernel, dim3((N + 255) / 256, n_det), dim3(256), 0, st, in, in_ld, prev_in,
                       prev_out, hann, N, Z, H, gap_mask, static_cast<f32x2 *>(blk));
    return hipGetLastError();
}

hipError_t launch_fft(hipStream_t st, void *a, void *b, int32_t N, int32_t N_table, int32_t inverse, const void *tw,
                      int32_t n_det, void **result) {
    f32x2 *src = static_cast<f32x2 *>(a), *dst = static_cast<f32x2 *>(b);
    int log2n = 0;
    while ((1 << log2n) < N) ++log2n;
    int m = 1;
    if (log2n & 1) {                     // one radix-2 pass, then radix-4
        hipLaunchKernelGGL(fft_pass_kernel, dim3((N / 2 + 255) / 256, n_det), dim3(256), 0, st, src, dst, N, 1,
                           N_table / 2, inverse, static_cast<const f32x2 *>(tw));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        f32x2 *t = src;
        src = dst;
        dst = t;
        m = 2;
    }
    for (; m < N; m <<= 2) {
        hipLaunchKernelGGL(fft_pass4_kernel, dim3((N / 4 + 255) / 256, n_det), dim3(256), 0, st, src, dst, N, m,
                           N_table / (4 * m), inverse, static_cast<const f32x2 *>(tw));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        f32x2 *t = src;
        src = dst;
        dst = t;
    }
    *result = src;
    return hipSuccess;
}

hipError_t launch_whiten_psd(hipStream_t st, const void *X, int32_t N, int32_t K, int32_t n_out, float inv_w2,
                             float *ring, int32_t n_med, float *log_geo, const WhitenDetState &s, const float *beta,
                             float d_factor, void *Y, int32_t n_det) {
    hipLaunchKernelGGL(whiten_psd_kernel, dim3((K + 255) / 256, n_det), dim3(256), 0, st,
                       static_cast<const f32x2 *>(X), N, K, n_out, inv_w2, ring, n_med, log_geo, s, beta, d_factor,
                       static_cast<f32x2 *>(Y));
    return hipGetLastError();
}

hipError_t launch_whiten_ola(hipStream_t st, const void *y, const float *tukey, int32_t n_out, int32_t h_out,
                             uint32_t gap_mask, const float *acc_in, float *acc_out, float *out, int64_t out_ld,
                             int32_t n_det) {
    hipLaunchKernelGGL(whiten_ola_kernel, dim3((n_out + 255) / 256, n_det), dim3(256), 0, st,
                       static_cast<const f32x2 *>(y), tukey, n_out, h_out, gap_mask, acc_in, acc_out, out, out_ld);
    return hipGetLastError();
}

}  // namespace lloid

// ------------------------------------------------------------------ host
using namespace lloid;

namespace {

// beta_c = exp(E[log median of c unit exponentials] + gamma) for odd c: the
// median is order statistic k = (c+1)/2, density C (1 - e^-x)^(k-1)
// e^-(c-k+1)x, C = c! / ((k-1)! (c-k)!).  With x = e^s the integrand of
// E[log x] is smooth and decays on both sides; the trapezoid rule on
// s in [-60, 6] (step 2^-10) converges to double precision.
double median_bias(int c) {
    const int k = (c + 1) / 2;
    double C = 1.0;                      // c! / ((k-1)! (c-k)!)
    for (int i = 1; i <= c; ++i) C *= i;
    for (int i = 1; i <= k - 1; ++i) C /= i;
    for (int i = 1; i <= c - k; ++i) C /= i;
    const double h = 1.0 / 1024.0;
    double sum = 0.0;
    for (double s = -60.0; s <= 6.0; s += h) {
        const double x = std::exp(s);
        sum += s * C * std::pow(-std::expm1(-x), k - 1) * std::exp(-(c - k + 1) * x) * x;
    }
    const double gamma = 0.57721566490153286061;
    return std::exp(sum * h + gamma);
}

}  // namespace

struct lloid_whitener {
    lloid_whiten_config cfg{};
    int H = 0, n_out = 0, h_out = 0, K = 0;
    float inv_w2 = 0.f;
    std::vector<void *> allocs;
    float *hann = nullptr, *tukey = nullptr, *beta = nullptr, *ring = nullptr, *log_geo = nullptr;
    float *prev[2] = {nullptr, nullptr}, *acc[2] = {nullptr, nullptr};
    void *tw = nullptr, *blk[2] = {nullptr, nullptr}, *ybuf[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t blocks[kWhitenMaxDet] = {0};

    template <typename T>
    bool alloc(T **p, size_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        allocs.push_back(q);
        *p = static_cast<T *>(q);
        return true;
    }
    ~lloid_whitener() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

extern "C" {

lloid_status lloid_whitener_create(const lloid_whiten_config *c, void *stream, lloid_whitener **out) {
    if (!c || !out) return LLOID_E_ARG;
    *out = nullptr;
    const int N = c->block, Z = c->pad, D = c->decimation, ND = c->n_detectors;
    if (ND < 1 || ND > kWhitenMaxDet || c->n_med < 1 || c->n_med > kWhitenMaxMed || c->n_med % 2 == 0 ||
        c->n_avg < 1)
        return LLOID_E_ARG;
    if (N < 64 || N > (1 << 20) || (N & (N - 1)) || D < 1 || (D & (D - 1)) || Z < 0 || 4 * Z > N ||
        Z % D || (N / 2 - Z) % D || N / D < 16)
        return LLOID_E_SHAPE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    lloid_whitener *w = new (std::nothrow) lloid_whitener();
    if (!w) return LLOID_E_NOMEM;
    w->cfg = *c;
    w->H = N / 2 - Z;
    w->n_out = N / D;
    w->h_out = w->H / D;
    w->K = w->n_out / 2 + 1;
    const int H = w->H, n_out = w->n_out, zo = Z / D;
    std::vector<float> hann(2 * H), tukey(n_out, 1.f), beta(kWhitenMaxMed + 1, 1.f), tw(2 * (size_t)N);
    const double pi = 3.14159265358979323846;
    double w2 = 0.0;
    for (int m = 0; m < 2 * H; ++m) {
        const double v = std::sin(pi * m / (2.0 * H));
        hann[m] = (float)(v * v);
        w2 += (v * v) * (v * v);
    }
    w->inv_w2 = (float)(1.0 / w2);
    for (int n = 0; n < zo; ++n) {
        const float r = (float)(0.5 * (1.0 - std::cos(pi * n / zo)));
        tukey[n] = r;
        tukey[n_out - 1 - n] = r;
    }
    for (int cc = 1; cc <= c->n_med; cc += 2) beta[cc] = (float)median_bias(cc);
    for (int q = 0; q < N; ++q) {         // the full circle: radix-4 passes index up to 3N/4
        tw[2 * q] = (float)std::cos(-2.0 * pi * q / N);
        tw[2 * q + 1] = (float)std::sin(-2.0 * pi * q / N);
    }
    bool ok = w->alloc(&w->hann, 2 * H) && w->alloc(&w->tukey, n_out) && w->alloc(&w->beta, kWhitenMaxMed + 1);
    ok = ok && w->alloc(reinterpret_cast<float **>(&w->tw), 2 * (size_t)N);
    for (int i = 0; i < 2 && ok; ++i) {
        ok = w->alloc(&w->prev[i], (size_t)ND * H) && w->alloc(&w->acc[i], (size_t)ND * n_out) &&
             w->alloc(reinterpret_cast<float **>(&w->blk[i]), (size_t)ND * N * 2) &&
             w->alloc(reinterpret_cast<float **>(&w->ybuf[i]), (size_t)ND * n_out * 2);
    }
    ok = ok && w->alloc(&w->ring, (size_t)ND * c->n_med * w->K) && w->alloc(&w->log_geo, (size_t)ND * w->K);
    if (!ok) {
        delete w;
        return LLOID_E_NOMEM;
    }
    hipError_t e = hipMemcpyAsync(w->hann, hann.data(), hann.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(w->tukey, tukey.data(), tukey.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(w->beta, beta.data(), beta.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(w->tw, tw.data(), tw.size() * 4, hipMemcpyHostToDevice, st);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMemsetAsync(w->prev[i], 0, sizeof(float) * ND * H, st);
        if (e == hipSuccess) e = hipMemsetAsync(w->acc[i], 0, sizeof(float) * ND * n_out, st);
    }
    if (e == hipSuccess) e = hipMemsetAsync(w->log_geo, 0, sizeof(float) * ND * w->K, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete w;
        return LLOID_E_HIP;
    }
    *out = w;
    return LLOID_OK;
}

void lloid_whitener_destroy(lloid_whitener *w) {
    if (!w) return;
    (void)hipDeviceSynchronize();
    delete w;
}

lloid_status lloid_whitener_push(lloid_whitener *w, const float *in, uint32_t gap_mask, float *out, void *stream) {
    if (!w || !in || !out) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int ND = w->cfg.n_detectors, N = w->cfg.block;
    WhitenDetState s{};
    s.gap_mask = gap_mask;
    s.n_avg = w->cfg.n_avg;
    for (int d = 0; d < ND; ++d) {
        if (!((gap_mask >> d) & 1u)) w->blocks[d] += 1;
        s.blocks[d] = w->blocks[d];
    }
    const int c = w->cur;
    hipError_t e = launch_whiten_block(st, in, w->H, w->prev[c], w->prev[1 - c], w->hann, N, w->cfg.pad, w->H,
                                       gap_mask, ND, w->blk[0]);
    void *X = nullptr, *y = nullptr;
    if (e == hipSuccess) e = launch_fft(st, w->blk[0], w->blk[1], N, N, 0, w->tw, ND, &X);
    if (e == hipSuccess)
        e = launch_whiten_psd(st, X, N, w->K, w->n_out, w->inv_w2, w->ring, w->cfg.n_med, w->log_geo, s, w->beta,
                              (float)w->cfg.decimation, w->ybuf[0], ND);
    if (e == hipSuccess) e = launch_fft(st, w->ybuf[0], w->ybuf[1], w->n_out, N, 1, w->tw, ND, &y);
    if (e == hipSuccess)
        e = launch_whiten_ola(st, y, w->tukey, w->n_out, w->h_out, gap_mask, w->acc[c], w->acc[1 - c], out, w->h_out,
                              ND);
    if (e != hipSuccess) return LLOID_E_HIP;
    w->cur = 1 - c;
    return LLOID_OK;
}

lloid_status lloid_whitener_psd(lloid_whitener *w, float *psd, void *stream) {
    if (!w || !psd) return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = (int64_t)w->cfg.n_detectors * w->K;
    if (launch_whiten_exp(st, w->log_geo, n, psd) != hipSuccess) return LLOID_E_HIP;
    return LLOID_OK;
}

}  // extern "C"
