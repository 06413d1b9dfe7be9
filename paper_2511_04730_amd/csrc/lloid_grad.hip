// Kernels of the gradient of the SNR-reconstruction loss and of the FP64
// re-orthonormalisation of refined bases.
//
//   L = sum_{r,t} (rho[r,t] - target[r,t])^2,  R = rho - target
//   dL/dW^s = 2 G^s Y^s^T,   dL/dY^s = 2 W^s^T G^s,
//   dL/dU^s[l,n] = sum_q dL/dY^s[l,q] d^s[q - delay - (N-1) + n]
// with G^s the residual taken down to the slice's rate by the transposed
// upsampling stages.  The transposed zero-phase polyphase stage is a
// decimating correlation with the same sub-kernels:
//   G_{j+1}[m] = sum_{q=m-N_up}^{m+N_up} sum_{ph<p} G_j[p q + ph] z_ph[q + N_up - m]
// (phase 0: weight 1 at q = m, the copy case of Eq. (upsample)).
#include <hip/hip_runtime.h>

#include "lloid_device.h"
#include "lloid_internal.h"
#include "lloid_mfma.h"

namespace lloid {

// ---------------------------------------------------------------- capture
// One stride's capture, every ring in one launch: work group (x, g) copies
// row r = g - row0 of item row_item[g], positions a .. a + len - 1 with
// a = base + k step (stride k), from the item's mirror ring (a basis-output
// ring in 4-output groups, or a plain stream ring) to its dst row r at
// columns a - dst_lo onwards.
__global__ __launch_bounds__(256) void capture_kernel(const CaptureItem *__restrict__ items,
                                                      const int32_t *__restrict__ row_item, int64_t k) {
    const CaptureItem it = items[row_item[blockIdx.y]];
    const int r = (int)blockIdx.y - it.row0;
    const int64_t a = it.base + k * it.step;
    const int64_t p0 = posmod(a, it.cap);
    float *d = it.dst + r * it.dst_ld + (a - it.dst_lo);
    for (int c = blockIdx.x * 256 + threadIdx.x; c < it.len; c += gridDim.x * 256) {
        const int64_t p = p0 + c;   // mirror ring: p < 2 cap
        d[c] = it.grouped ? it.src[ring_index<4>(p, r, it.cap)] : it.src[r * it.src_ld + p];
    }
}

hipError_t launch_capture(hipStream_t st, const CaptureItem *items, const int32_t *row_item, int32_t rows,
                          int32_t max_len, int64_t k) {
    if (rows <= 0 || max_len <= 0) return hipSuccess;
    dim3 grid((unsigned)std::min(16, (max_len + 255) / 256), (unsigned)rows);
    hipLaunchKernelGGL(capture_kernel, grid, dim3(256), 0, st, items, row_item, k);
    return hipGetLastError();
}

// R[(2i + c) * ld + t0 + t] = series[((det M + i) F + t) 2 + c] - target[same], and
// per-block partial sums of R^2 (FP64) into loss_part[blockIdx].  Block b
// takes the templates [b M / blocks, (b + 1) M / blocks), whole rows of F
// samples each (no index division per element; a block with no template
// writes a zero partial).
__global__ __launch_bounds__(256) void residual_kernel(const float *__restrict__ series,
                                                       const float *__restrict__ target, int32_t M, int32_t F,
                                                       float *__restrict__ R, int64_t ld, int64_t t0,
                                                       double *__restrict__ loss_part) {
    __shared__ double red[256];
    const int i0 = (int)((int64_t)blockIdx.x * M / gridDim.x), i1 = (int)((int64_t)(blockIdx.x + 1) * M / gridDim.x);
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        const float2 *s = reinterpret_cast<const float2 *>(series) + (int64_t)i * F;
        const float2 *g = reinterpret_cast<const float2 *>(target) + (int64_t)i * F;
        float *rr = R + (2 * (int64_t)i) * ld + t0;
        for (int t = threadIdx.x; t < F; t += 256) {
            const float2 a = s[t], b = g[t];
            const float re = a.x - b.x, im = a.y - b.y;
            rr[t] = re;
            rr[ld + t] = im;
            acc += (double)re * re + (double)im * im;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

hipError_t launch_residual(hipStream_t st, const float *series, const float *target, int32_t M, int32_t F, float *R,
                           int64_t ld, int64_t t0, double *loss_part, int32_t blocks) {
    hipLaunchKernelGGL(residual_kernel, dim3(blocks), dim3(256), 0, st, series, target, M, F, R, ld, t0, loss_part);
    return hipGetLastError();
}

__global__ void sum_f64_kernel(const double *__restrict__ part, int32_t n, double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_sum_f64(hipStream_t st, const double *part, int32_t n, double *out) {
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, st, part, n, out);
    return hipGetLastError();
}

// ------------------------------------------------- transposed upsampling
// g: [rows][g_ld] holding level indices g_lo .. g_lo + ng - 1; out:
// [rows][o_ld] at a_lo + m for m < na, zeros in the padding na .. o_ld - 1.
// out[m] = sum over t (0 .. 2 nup) and phase ph (0 .. p - 1) of
// g[p (a_lo + m - nup + t) + ph - g_lo] w(t, ph), w the polyphase taps (phase
// 0: the unit tap at t = nup).  A work group takes 256 consecutive outputs of
// one row: the window of g they read (256 p + 2 nup p + p values) is staged
// in LDS with coalesced loads (zero outside [0, ng)).
constexpr int kAdjMaxP = 8;   // LDS window for p up to 8; larger p reads g directly
__global__ __launch_bounds__(256) void upsample_adjoint_kernel(const float *__restrict__ g, int64_t g_ld, int64_t g_lo,
                                                               int64_t ng, float *__restrict__ out, int64_t o_ld,
                                                               int64_t a_lo, int64_t na, int32_t p, int32_t nup,
                                                               const float *__restrict__ taps) {
    __shared__ float win[256 * kAdjMaxP + 2 * 8 * kAdjMaxP + kAdjMaxP];
    const int r = blockIdx.y;
    const float *grow = g + r * g_ld;
    const int64_t m0 = (int64_t)blockIdx.x * 256;
    const int64_t m = m0 + threadIdx.x;
    const int T = 2 * nup + 1;
    if (p <= kAdjMaxP && nup <= 8) {
        // window: g indices i0 .. i0 + wn - 1, i0 = p (a_lo + m0 - nup) - g_lo
        const int64_t i0 = (int64_t)p * (a_lo + m0 - nup) - g_lo;
        const int wn = 256 * p + 2 * nup * p + p;
        for (int e = threadIdx.x; e < wn; e += 256) {
            const int64_t i = i0 + e;
            win[e] = (i >= 0 && i < ng) ? grow[i] : 0.0f;
        }
        __syncthreads();
        if (m >= na) {
            if (m < o_ld) out[r * o_ld + m] = 0.0f;   // row padding read by the products
            return;
        }
        const float *wbase = win + p * threadIdx.x;   // g at q = a_lo + m - nup + t: wbase[p t + ph]
        float acc = wbase[p * nup];                   // phase 0, the unit tap
        for (int t = 0; t < T; ++t)
            for (int ph = 1; ph < p; ++ph) acc = fmaf(wbase[p * t + ph], taps[ph * kUpTaps + t], acc);
        out[r * o_ld + m] = acc;
        return;
    }
    if (m >= na) {
        if (m < o_ld) out[r * o_ld + m] = 0.0f;
        return;
    }
    const int64_t am = a_lo + m;
    float acc = 0.0f;
    for (int64_t q = am - nup; q <= am + nup; ++q) {
        const int t = (int)(q + nup - am);
        for (int ph = 0; ph < p; ++ph) {
            const int64_t i = p * q + ph - g_lo;
            if (i < 0 || i >= ng) continue;
            const float w = ph == 0 ? (t == nup ? 1.0f : 0.0f) : taps[ph * kUpTaps + t];
            acc = fmaf(grow[i], w, acc);
        }
    }
    out[r * o_ld + m] = acc;
}

// The same for p = 2 or 4 and N_up = 8: a work group takes 1024 outputs of
// one row, and its window of g is stored de-interleaved, one LDS plane per
// phase (plane ph, entry j: g at p (a_lo + m0 - N_up + j) + ph), so that a
// thread's four consecutive outputs read each plane as float4 (a 20-entry
// run per phase) and the 17 taps of a phase are registers.  Plane strides
// of 1056 (p = 2) and 1040 (p = 4) words keep the de-interleaving stores on
// distinct banks.
template <int P, int NUP>
__global__ __launch_bounds__(256) void upsample_adjoint_planes_kernel(const float *__restrict__ g, int64_t g_ld,
                                                                      int64_t g_lo, int64_t ng,
                                                                      float *__restrict__ out, int64_t o_ld,
                                                                      int64_t a_lo, int64_t na,
                                                                      const float *__restrict__ taps) {
    constexpr int TPB = 1024, T = 2 * NUP + 1, NQ = TPB + 2 * NUP, PS = P == 2 ? 1056 : 1040;
    static_assert(PS >= NQ && NUP % 4 == 0 && T + 3 <= 20, "plane layout");
    __shared__ __align__(16) float pl[P][PS];
    const int r = blockIdx.y;
    const int64_t m0 = (int64_t)blockIdx.x * TPB;
    const int64_t i0 = (int64_t)P * (a_lo + m0 - NUP) - g_lo;   // g index of plane 0, entry 0
    const float *gw = g + r * g_ld + i0;
    const int64_t elo = -i0, ehi = ng - i0;                     // valid window entries: [elo, ehi)
    for (int e = threadIdx.x; e < P * NQ; e += 256) pl[e % P][e / P] = (e >= elo && e < ehi) ? gw[e] : 0.0f;
    __syncthreads();
    const int o = 4 * threadIdx.x;
    const int64_t m = m0 + o;
    if (m >= o_ld) return;
    floatx4 acc = *reinterpret_cast<const floatx4 *>(&pl[0][o + NUP]);   // phase 0: the unit tap
#pragma unroll
    for (int ph = 1; ph < P; ++ph) {
        float v[20];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const floatx4 x = *reinterpret_cast<const floatx4 *>(&pl[ph][o + 4 * q]);
#pragma unroll
            for (int u = 0; u < 4; ++u) v[4 * q + u] = x[u];
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float w = taps[ph * kUpTaps + t];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = fmaf(v[u + t], w, acc[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (m + u >= na) acc[u] = 0.0f;   // row padding read by the products
    *reinterpret_cast<floatx4 *>(out + r * o_ld + m) = acc;
}

hipError_t launch_upsample_adjoint(hipStream_t st, const float *g, int64_t g_ld, int64_t g_lo, int64_t ng,
                                   float *out, int64_t o_ld, int64_t a_lo, int64_t na, int32_t rows, int32_t p,
                                   int32_t nup, const float *taps) {
    if (na <= 0 || rows <= 0) return hipSuccess;
    if (o_ld < na) return hipErrorInvalidValue;
    if ((p == 2 || p == 4) && nup == 8 && o_ld % 4 == 0) {
        dim3 grid((unsigned)((o_ld + 1023) / 1024), rows);
        if (p == 2)
            hipLaunchKernelGGL((upsample_adjoint_planes_kernel<2, 8>), grid, dim3(256), 0, st, g, g_ld, g_lo, ng, out,
                               o_ld, a_lo, na, taps);
        else
            hipLaunchKernelGGL((upsample_adjoint_planes_kernel<4, 8>), grid, dim3(256), 0, st, g, g_ld, g_lo, ng, out,
                               o_ld, a_lo, na, taps);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((o_ld + 255) / 256), rows);
    hipLaunchKernelGGL(upsample_adjoint_kernel, grid, dim3(256), 0, st, g, g_ld, g_lo, ng, out, o_ld, a_lo, na, p,
                       nup, taps);
    return hipGetLastError();
}

// --------------------------------------------------- dW = 2 G Y^T (partials)
// part[z][m][n] = sum over k in [z ksplit, (z + 1) ksplit) of A[m][k] B[n][k]:
// A [M][lda] (the residual G at one rate) and B [N][ldb] (the captured
// basis outputs Y), both contiguous in k and zero from the valid length K
// to the next multiple of 32 (their row padding).  One wave takes 32 rows
// (two 16-row blocks) and NB column blocks (the group blockIdx.z of 16 NB
// columns; B rows past N are clamped and their outputs dropped); each lane loads 8 consecutive
// k of its row as two float4, so the MFMA step s sums k = 8 lk + s over the
// four lane groups lk (the same order for A and B).  The next 32-deep chunk
// is in flight while the current one is multiplied; no LDS and no barrier.
template <int NB>
__global__ __launch_bounds__(256) void gemm_abt_kernel(const float *__restrict__ A, int64_t lda,
                                                       const float *__restrict__ B, int64_t ldb, int32_t M,
                                                       int32_t N, int64_t K, int64_t ksplit,
                                                       float *__restrict__ part) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int m0 = ((int)blockIdx.x * 4 + wave) * 32;
    if (m0 >= M) return;   // whole waves only: the kernel has no barrier
    const int64_t kb = (int64_t)blockIdx.y * ksplit;
    const int nch = (int)((std::min<int64_t>(K, kb + ksplit) - kb + 31) / 32);
    const float *pa[2], *pb[NB];
#pragma unroll
    for (int r = 0; r < 2; ++r) pa[r] = A + (int64_t)std::min(m0 + 16 * r + li, M - 1) * lda + kb + 8 * lk;
#pragma unroll
    for (int c = 0; c < NB; ++c)
        pb[c] = B + (int64_t)std::min((int)blockIdx.z * 16 * NB + 16 * c + li, N - 1) * ldb + kb + 8 * lk;
    struct Chunk {
        floatx4 a[2][2], b[NB][2];
    };
    auto load = [&](Chunk &x, int ch) {
        const int64_t o = (int64_t)ch * 32;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 2; ++r) x.a[r][h] = *reinterpret_cast<const floatx4 *>(pa[r] + o + 4 * h);
#pragma unroll
            for (int c = 0; c < NB; ++c) x.b[c][h] = *reinterpret_cast<const floatx4 *>(pb[c] + o + 4 * h);
        }
    };
    floatx4 acc[2][NB];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto mul = [&](const Chunk &x) {
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    acc[r][c] = mfma_16x16x4_f32(x.a[r][s >> 2][s & 3], x.b[c][s >> 2][s & 3], acc[r][c]);
    };
    Chunk x0, x1;
    load(x0, 0);
    int ch = 0;
    for (; ch + 2 <= nch; ch += 2) {
        load(x1, ch + 1);
        mul(x0);
        if (ch + 2 < nch) load(x0, ch + 2);
        mul(x1);
    }
    if (ch < nch) mul(x0);
    float *o = part + (int64_t)blockIdx.y * M * N;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int n = (int)blockIdx.z * 16 * NB + 16 * c + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + 16 * r + 4 * lk + v;
                if (m < M && n < N) o[(int64_t)m * N + n] = acc[r][c][v];
            }
        }
}

hipError_t launch_gemm_abt(hipStream_t st, const float *A, int64_t lda, const float *B, int64_t ldb, int32_t M,
                           int32_t N, int64_t K, int64_t ksplit, float *part) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (ksplit % 32 || lda % 4 || ldb % 4) return hipErrorInvalidValue;
    const int nb = std::min(4, (N + 15) / 16);
    dim3 grid((unsigned)((M + 127) / 128), (unsigned)((K + ksplit - 1) / ksplit), (unsigned)((N + 16 * nb - 1) / (16 * nb)));
    switch (nb) {
    case 1: hipLaunchKernelGGL(gemm_abt_kernel<1>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, ksplit, part); break;
    case 2: hipLaunchKernelGGL(gemm_abt_kernel<2>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, ksplit, part); break;
    case 3: hipLaunchKernelGGL(gemm_abt_kernel<3>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, ksplit, part); break;
    default: hipLaunchKernelGGL(gemm_abt_kernel<4>, grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, ksplit, part);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ dY = 2 W^T G
// out[l][n] = alpha sum_k W[k][l] G[k][n] for l < ldw and n < n_out: W
// [K][ldw] (the FP32 mixing rows, zero past the valid basis count; ldw a
// multiple of 16), G [K][ldg] (zero from its valid length to ldg, a multiple
// of 4).  A work group takes 128 columns and the row group blockIdx.y of
// 16 NBR rows; 32-deep chunks of G (32 x 128) and of W go through two LDS
// buffers with one barrier per chunk, the next chunk's global loads in
// flight during the current chunk's MFMAs.  Wave w owns columns
// 32 w .. 32 w + 31 of the tile and every row block.  LDS row strides of
// 144 and 80 words put the four k rows of a fragment read in four different
// 16-bank groups.
template <int NBR>
__global__ __launch_bounds__(256) void gemm_atb_kernel(const float *__restrict__ W, int32_t ldw,
                                                       const float *__restrict__ G, int64_t ldg, int32_t K,
                                                       int64_t n_out, float alpha, float *__restrict__ out,
                                                       int64_t ldo) {
    constexpr int LDW = 16 * NBR, GS = 144, WS = NBR <= 4 ? 80 : 144;
    constexpr int WF = 8 * LDW;                // float4 of a 32-row W chunk
    constexpr int WJ = (WF + 255) / 256;       // of them per thread
    __shared__ __align__(16) float Gs[2][32][GS];
    __shared__ __align__(16) float Ws[2][32][WS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int64_t n0 = (int64_t)blockIdx.x * 128;
    const int gr = tid >> 5, gc = tid & 31;   // G chunk: rows gr + 8 j, float4 column gc
    const bool g_ok = n0 / 4 + gc < ldg / 4;
    const float *gp = G + n0 + 4 * gc;
    const int l0 = (int)blockIdx.y * LDW;      // first row of the group (a column of W)
    floatx4 g[4], w[WJ];
    const floatx4 z4{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int kk) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kk + gr + 8 * j;
            g[j] = (g_ok && k < K) ? *reinterpret_cast<const floatx4 *>(gp + (int64_t)k * ldg) : z4;
        }
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
            const int f = tid + 256 * j, k = kk + f / (LDW / 4), c = l0 + 4 * (f % (LDW / 4));
            w[j] = (f < WF && k < K && c < ldw) ? *reinterpret_cast<const floatx4 *>(W + (int64_t)k * ldw + c) : z4;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < 4; ++j) *reinterpret_cast<floatx4 *>(&Gs[buf][gr + 8 * j][4 * gc]) = g[j];
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
            const int f = tid + 256 * j;
            if (f < WF) *reinterpret_cast<floatx4 *>(&Ws[buf][f / (LDW / 4)][4 * (f % (LDW / 4))]) = w[j];
        }
    };
    floatx4 acc[NBR][2];
#pragma unroll
    for (int r = 0; r < NBR; ++r) acc[r][0] = acc[r][1] = z4;
    const int nch = (K + 31) / 32;
    load(0);
    store(0);
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(32 * (ch + 1));
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int k = 4 * s + lk;
            const float b0 = Gs[buf][k][32 * wave + li], b1 = Gs[buf][k][32 * wave + 16 + li];
#pragma unroll
            for (int r = 0; r < NBR; ++r) {
                const float a = Ws[buf][k][16 * r + li];
                acc[r][0] = mfma_16x16x4_f32(a, b0, acc[r][0]);
                acc[r][1] = mfma_16x16x4_f32(a, b1, acc[r][1]);
            }
        }
        if (ch + 1 < nch) store(buf ^ 1);
    }
#pragma unroll
    for (int r = 0; r < NBR; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int64_t n = n0 + 32 * wave + 16 * c + li;
            if (n >= n_out) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int l = l0 + 16 * r + 4 * lk + v;
                if (l < ldw) out[(int64_t)l * ldo + n] = alpha * acc[r][c][v];
            }
        }
}

hipError_t launch_gemm_atb(hipStream_t st, const float *W, int32_t ldw, const float *G, int64_t ldg, int32_t K,
                           int64_t n_out, float alpha, float *out, int64_t ldo) {
    if (K <= 0 || n_out <= 0) return hipSuccess;
    if (ldw <= 0 || ldw % 16 || ldg % 4) return hipErrorInvalidValue;
    const int nbr = std::min(8, ldw / 16);
    dim3 grid((unsigned)((n_out + 127) / 128), (unsigned)((ldw + 16 * nbr - 1) / (16 * nbr)));
#define LLOID_ATB(R)                                                                                                   \
    case R:                                                                                                            \
        hipLaunchKernelGGL(gemm_atb_kernel<R>, grid, dim3(256), 0, st, W, ldw, G, ldg, K, n_out, alpha, out, ldo);    \
        break;
    switch (nbr) {
        LLOID_ATB(1)
        LLOID_ATB(2)
        LLOID_ATB(3)
        LLOID_ATB(4)
        LLOID_ATB(5)
        LLOID_ATB(6)
        LLOID_ATB(7)
        LLOID_ATB(8)
    }
#undef LLOID_ATB
    return hipGetLastError();
}

// dst[r * d_ld + c] (=|+=) alpha * sum_s part[s][r][c]   (fixed order)
__global__ void sum_parts_kernel(const float *__restrict__ part, int32_t nsplit, int64_t plane, int32_t cols,
                                 int64_t p_ld, float *__restrict__ dst, int64_t d_ld, float alpha, int32_t accumulate) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int i = 0; i < nsplit; ++i) s += part[i * plane + r * p_ld + c];
        float *o = dst + r * d_ld + c;
        *o = accumulate ? *o + alpha * s : alpha * s;
    }
}

hipError_t launch_sum_parts(hipStream_t st, const float *part, int32_t nsplit, int64_t plane, int32_t rows,
                            int32_t cols, int64_t p_ld, float *dst, int64_t d_ld, float alpha, int32_t accumulate) {
    dim3 grid((unsigned)std::min<int64_t>((cols + 255) / 256, 1024), rows);
    hipLaunchKernelGGL(sum_parts_kernel, grid, dim3(256), 0, st, part, nsplit, plane, cols, p_ld, dst, d_ld, alpha,
                       accumulate);
    return hipGetLastError();
}

}  // namespace lloid

// ------------------------------------------- FP8 basis values (refinement)
// The values the FP8 form's correlation uses for a basis row, as float64:
// one block per row, e = floor(log2(448 / max|u|)), e4m3 (round to nearest
// even, from float32) of u 2^e, times 2^-e.  Quantisation-aware refinement
// evaluates the loss at these values and applies the gradient to the
// unrounded rows.
namespace {

__global__ __launch_bounds__(256) void quantize_fp8_rows_kernel(const double *__restrict__ src, int32_t cols,
                                                                double *__restrict__ dst) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const double *u = src + (int64_t)r * cols;
    double mx = 0.0;
    for (int c = threadIdx.x; c < cols; c += 256) mx = fmax(mx, fabs(u[c]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const int e = red[0] > 0.0 ? (int)floor(log2(448.0 / red[0])) : 0;
    const double s = ldexp(1.0, e);
    for (int c = threadIdx.x; c < cols; c += 256) {
        const uint32_t b = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32((float)(u[c] * s), 0.0f, 0, false) & 0xffu;
        dst[(int64_t)r * cols + c] = ldexp((double)__builtin_amdgcn_cvt_f32_fp8((int)b, 0), -e);
    }
}

}  // namespace

extern "C" lloid_status lloid_quantize_fp8_rows(const double *U, int32_t rows, int32_t cols, double *Uq,
                                                void *stream) {
    if (!U || !Uq || rows < 1 || cols < 1) return LLOID_E_ARG;
    hipLaunchKernelGGL(quantize_fp8_rows_kernel, dim3(rows), dim3(256), 0, static_cast<hipStream_t>(stream), U, cols,
                       Uq);
    return hipGetLastError() == hipSuccess ? LLOID_OK : LLOID_E_HIP;
}
