// FP64 dense linear algebra on the matrix cores (v_mfma_f64_16x16x4_f64):
// the CholeskyQR2 re-orthonormalisation of refined bases and the SVD bank
// construction of Sec. II.C.1 (rank-L truncation of a slice's template
// matrix by subspace iteration).
//
// A 16x16x4 FP64 MFMA takes one double of A (row lane mod 16, K index
// lane / 16) and one of B (column lane mod 16, same K index) per lane and
// accumulates a 16x16 tile held as four doubles per lane: double v of lane
// l is row l / 16 + 4 v, column l mod 16 (checked on the device: unlike the
// FP32 16x16 tiles, whose lane holds four consecutive rows).  Only the pairing of A's and B's K
// index matters for a contraction, so a lane may walk its own K range in any
// order as long as both operands follow it.
//
// CholeskyQR2 (two passes of G = U U^T = C C^T, U <- C^-1 U, W <- W C):
//   gram_f64_kernel      G = U U^T, one 16x16 tile per work group, the four
//                        waves splitting K and summing in a fixed order
//   chol_inv_kernel      lower factor C and its inverse (one work group,
//                        right-looking; in LDS for L <= 100)
//   left_apply_kernel    U <- C^-1 U in place, 64 columns of U per work
//                        group staged in LDS
//   right_apply_kernel   W <- W C in place, 64 rows of W per work group
// Subspace iteration:
//   gemm_f64_kernel      general strided product split over K into partial
//                        planes, summed in a fixed order (sum_parts_kernel)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lloid_device.h"
#include "lloid_internal.h"

namespace lloid {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// --------------------------------------------------------------- GEMM
// part[z][m][n] = sum over k in [z ksplit, (z + 1) ksplit) of A(m,k) B(k,n),
// A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn].  64 x 64 tile per work
// group, 32-deep K stages in LDS, the next stage's operands loaded into
// registers while the MFMAs run on the current one; wave w owns the tile's
// columns 16 w .. + 15 for NMB 16-row blocks (NMB < 4 when the whole product
// has fewer rows: a 40-row product runs three).  Both operands are read
// through buffer resources: an element outside the matrix or the work
// group's K range takes an offset past the resource and reads as zero, with
// no branch.  LDS strides: 36 doubles per A row and 80 per B row, so that a
// wave's 64 fragment reads spread over all banks (two passes, the minimum
// for 8-byte reads).
constexpr int kDT = 64, kDK = 32;
constexpr int kDPer = kDT * kDK / 256;   // elements of each operand a thread stages per K stage
constexpr int kAS = kDK + 4, kBS = kDT + 16;
constexpr int kOutOfRange = 0x7FFFFFF0;  // an offset past every resource (matrices < 2 GiB)
__device__ __forceinline__ double buffer_load_f64(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <int NMB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ A, int64_t sam, int64_t sak,
                                                       const double *__restrict__ B, int64_t sbk, int64_t sbn,
                                                       int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                                       double *__restrict__ part) {
    __shared__ double As[kDT * kAS];
    __shared__ double Bs[kDK * kBS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * kDT, n0 = (int64_t)blockIdx.y * kDT;
    const int64_t k_begin = (int64_t)blockIdx.z * ksplit;
    const int64_t k_end = k_begin + ksplit < K ? k_begin + ksplit : K;
    const __amdgpu_buffer_rsrc_t rA = buffer_rsrc(A, (uint32_t)(((M - 1) * sam + (K - 1) * sak + 1) * 8));
    const __amdgpu_buffer_rsrc_t rB = buffer_rsrc(B, (uint32_t)(((K - 1) * sbk + (N - 1) * sbn + 1) * 8));
    // the (row, k) and (k, column) each thread stages: the fast index of the
    // source runs over consecutive threads
    int am[kDPer], ak[kDPer], bn[kDPer], bk[kDPer];
#pragma unroll
    for (int i = 0; i < kDPer; ++i) {
        const int e = tid + 256 * i;
        am[i] = sak == 1 ? e / kDK : e % kDT;
        ak[i] = sak == 1 ? e % kDK : e / kDT;
        bn[i] = sbn == 1 ? e % kDT : e / kDK;
        bk[i] = sbn == 1 ? e / kDT : e % kDK;
    }
    double ra[kDPer], rb[kDPer];
    auto fetch = [&](int64_t kk) {
#pragma unroll
        for (int i = 0; i < kDPer; ++i) {
            const int64_t gm = m0 + am[i], gk = kk + ak[i];
            ra[i] = buffer_load_f64(rA, (gm < M && gk < k_end) ? (int)((gm * sam + gk * sak) * 8) : kOutOfRange);
            const int64_t gn = n0 + bn[i], gk2 = kk + bk[i];
            rb[i] = buffer_load_f64(rB, (gn < N && gk2 < k_end) ? (int)((gk2 * sbk + gn * sbn) * 8) : kOutOfRange);
        }
    };
    f64x4 acc[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) acc[mb] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (k_begin < k_end) fetch(k_begin);
    for (int64_t kk = k_begin; kk < k_end; kk += kDK) {
        __syncthreads();   // the previous stage has been read
#pragma unroll
        for (int i = 0; i < kDPer; ++i) {
            As[am[i] * kAS + ak[i]] = ra[i];
            Bs[bk[i] * kBS + bn[i]] = rb[i];
        }
        __syncthreads();
        if (kk + kDK < k_end) fetch(kk + kDK);
#pragma unroll
        for (int ks = 0; ks < kDK; ks += 4) {
            const double b = Bs[(ks + lg) * kBS + wave * 16 + li];
            double a[NMB];
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) a[mb] = As[(mb * 16 + li) * kAS + ks + lg];
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) acc[mb] = mfma_f64(a[mb], b, acc[mb]);
        }
    }
    const int64_t n = n0 + wave * 16 + li;
    if (n < N) {
        double *o = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + mb * 16 + lg + 4 * v;
                if (m < M) o[m * N + n] = acc[mb][v];
            }
    }
}

// out[i] = sum_s part[s plane + i], s = 0, 1, ... in order (four planes'
// loads in flight at a time)
__global__ __launch_bounds__(256) void sum_parts_kernel(const double *__restrict__ part, int32_t nsplit, int64_t plane,
                                                        double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= plane) return;
    double s = 0.0;
    int p = 0;
    for (; p + 4 <= nsplit; p += 4) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = part[(p + u) * plane + i];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u];
    }
    for (; p < nsplit; ++p) s += part[p * plane + i];
    out[i] = s;
}

// C (M x N, row-major) = A(m,k) B(k,n) over K, with nsplit K splits
// (part holds nsplit x M x N doubles; nsplit = 1 writes C directly)
hipError_t launch_gemm_f64(hipStream_t st, const double *A, int64_t sam, int64_t sak, const double *B, int64_t sbk,
                           int64_t sbn, int64_t M, int64_t N, int64_t K, int32_t nsplit, double *part, double *C) {
    int64_t ksplit = (K + nsplit - 1) / nsplit;
    ksplit = (ksplit + kDK - 1) / kDK * kDK;
    const int64_t ns = (K + ksplit - 1) / ksplit;
    dim3 grid((unsigned)((M + kDT - 1) / kDT), (unsigned)((N + kDT - 1) / kDT), (unsigned)ns);
    double *dst = ns == 1 ? C : part;
    const int nmb = M >= kDT ? 4 : (int)((M + 15) / 16);
    switch (nmb) {
        case 1:
            hipLaunchKernelGGL(gemm_f64_kernel<1>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, dst);
            break;
        case 2:
            hipLaunchKernelGGL(gemm_f64_kernel<2>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, dst);
            break;
        case 3:
            hipLaunchKernelGGL(gemm_f64_kernel<3>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, dst);
            break;
        default:
            hipLaunchKernelGGL(gemm_f64_kernel<4>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, dst);
            break;
    }
    if (ns > 1)
        hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, st, part, (int32_t)ns,
                           M * N, C);
    return hipGetLastError();
}

// ------------------------------------------------------------ Gram
// Partial Gram matrices of U [L][N] over kz ranges of taps: work group
// (bi, bj, z), bi >= bj, computes the 16x16 tile of sum over k in range z of
// U[r][k] U[c][k] for rows 16 bi .. and columns 16 bj .. and its mirror, into
// G + z L^2.  Wave w takes K blocks of 16 taps w, w + 4, ... of the range
// (four per trip); lane (li, lg) supplies taps 4 lg .. 4 lg + 3 of a block,
// one per MFMA, for row 16 bi + li (A) and row 16 bj + li (B).  The four
// waves' tiles are summed in wave order; the factor kernel sums the kz
// partial matrices in order.
__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ U, int32_t L, int32_t N,
                                                       int32_t krange, double *__restrict__ G) {
    __shared__ double red[4][64 * 4];
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bj > bi) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int ra = bi * 16 + li, rb = bj * 16 + li;
    const double *ua = U + (int64_t)(ra < L ? ra : 0) * N;
    const double *ub = U + (int64_t)(rb < L ? rb : 0) * N;
    const bool va = ra < L, vb = rb < L;
    const int kb = blockIdx.z * krange, ke = min(N, kb + krange);
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    // four blocks per trip: all 32 loads of a lane are in flight before its MFMAs
    for (int k0 = kb + wave * 16; k0 < ke; k0 += 256) {
        double a[16], b[16];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 64 * u + 4 * lg;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = k + s < ke;
                a[4 * u + s] = (va && in) ? ua[k + s] : 0.0;
                b[4 * u + s] = (vb && in) ? ub[k + s] : 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) acc = mfma_f64(a[t], b[t], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][lane * 4 + v] = acc[v];
    __syncthreads();
    if (wave == 0) {
        double *g = G + (int64_t)blockIdx.z * L * L;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double s = ((red[0][lane * 4 + v] + red[1][lane * 4 + v]) + red[2][lane * 4 + v]) + red[3][lane * 4 + v];
            const int r = bi * 16 + lg + 4 * v, c = bj * 16 + li;
            if (r < L && c < L) {
                g[r * L + c] = s;
                g[c * L + r] = s;
            }
        }
    }
}

// ------------------------------------------------------- Cholesky, inverse
// One work group sums the kz partial Gram matrices (in order) into the L x L
// SPD matrix G, factors G = C C^T (C lower) and inverts C, both right-looking
// in one sweep with one barrier per column.  Step j reads the pivot d =
// G_j[j][j] of the current Schur complement and column j of it, unscaled:
//   Cholesky: G[i][k] -= G[i][j] G[k][j] / d          for j < k <= i,
//   inverse (forward elimination of C X = I, X = I at the start):
//             X[i][c] -= (G[i][j] / d) X[j][c]         for i > j, c <= j,
// which equal the textbook updates with C[i][j] = G[i][j] / sqrt(d) and
// X[j] / sqrt(d); those two scalings of column j of G and row j of X are
// done in step j + 1 (nothing reads or writes them there) or after the
// sweep.  Every thread reads the pivot itself.  A pivot that is not
// positive is replaced by 1 (so the passes run on) and, if info[0] is still
// 0, recorded there as its column + 1; info is never reset here, so a
// breakdown stays reported until the caller clears it (launch_clear_info).
// LDS holds both matrices for L <= kCholLds (dynamic LDS); above that they
// are updated in place in global memory.  On return G holds C (upper
// triangle zero) and Cinv its inverse.
constexpr int kCholLds = 100;   // 2 x 100^2 doubles = 160000 bytes of LDS
constexpr int kGramSplit = 8;   // most partial Gram products the SVD construction sums
template <bool LDS>
__global__ __launch_bounds__(256) void chol_inv_kernel(const double *Gp, int32_t kz, double *G,
                                                       int32_t L, double *__restrict__ Cinv, int32_t *info) {
    extern __shared__ double sm[];
    double *a = LDS ? sm : G;
    double *x = LDS ? sm + L * L : Cinv;
    const int tid = threadIdx.x, ti = tid >> 4, tk = tid & 15;
    const int64_t LL = (int64_t)L * L;
    if (LDS) {
        // thread t sums elements t + 256 q over the partial planes in plane
        // order, every element of a plane loaded before the adds
        constexpr int Q = (kCholLds * kCholLds + 255) / 256;
        double v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = 0.0;
        for (int z = 0; z < kz; ++z) {
            double t[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) t[q] = tid + 256 * q < LL ? Gp[z * LL + tid + 256 * q] : 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] += t[q];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = tid + 256 * q;
            if (e < LL) {
                a[e] = v[q];
                x[e] = (e / L == e % L) ? 1.0 : 0.0;
            }
        }
    } else {
        for (int e = tid; e < L * L; e += 256) {
            double s = Gp[e];
            for (int z = 1; z < kz; ++z) s += Gp[z * LL + e];
            a[e] = s;
            x[e] = (e / L == e % L) ? 1.0 : 0.0;
        }
    }
    double rp = 1.0;   // 1 / sqrt(pivot) of the previous step
    for (int j = 0; j < L; ++j) {
        __syncthreads();   // step j - 1's updates are visible
        double d = a[j * L + j];
        if (!(d > 0.0)) {
            if (tid == 0 && info[0] == 0) info[0] = j + 1;
            d = 1.0;
        }
        const double rd = 1.0 / d;
        if (j > 0) {   // deferred scalings of step j - 1
            const int p = j - 1;
            for (int i = p + 1 + tid; i < L; i += 256) a[i * L + p] *= rp;
            if (tid == 0) a[p * L + p] = 1.0 / rp;
            for (int c = tid; c <= p; c += 256) x[p * L + c] *= rp;
        }
        // thread (ti, tk) of a 16 x 16 grid: rows i = j + 1 + ti + 16 m
        for (int i = j + 1 + ti; i < L; i += 16) {
            const double f = a[i * L + j] * rd;
            for (int k = j + 1 + tk; k <= i; k += 16) a[i * L + k] -= f * a[k * L + j];
            for (int c = tk; c <= j; c += 16) x[i * L + c] -= f * x[j * L + c];
        }
        rp = 1.0 / sqrt(d);
    }
    __syncthreads();
    {
        const int p = L - 1;
        if (tid == 0) a[p * L + p] = 1.0 / rp;
        for (int c = tid; c <= p; c += 256) x[p * L + c] *= rp;
    }
    __syncthreads();
    for (int e = tid; e < L * L; e += 256) {
        const bool upper = e % L > e / L;
        G[e] = upper ? 0.0 : a[e];
        if (LDS) Cinv[e] = x[e];
    }
}

// The same sweep for L <= 64 with the matrices in registers: wave w holds
// rows i = w + 4 r (r < 16) of G and of X, lane k their column k.  The steps
// are unrolled, so that the register of row j (wave j mod 4, r = j / 4) is
// fixed at compile time.  Step j publishes column j of G (lane j of every
// wave) and row j of X (wave j mod 4) through LDS, double-buffered by the
// parity of j so that one barrier per step suffices; then each wave updates
// only its rows i > j (a wave-uniform branch per row), the lanes selecting
// the columns the update touches.  Column j of G is final after step j and
// row i of X after step i; the scalings by 1 / sqrt(pivot) are applied when
// the results are written, from the pivots kept in LDS.
constexpr int kCholReg = 64;
__global__ __launch_bounds__(256) void chol_inv_reg_kernel(const double *Gp, int32_t kz, double *G, int32_t L,
                                                           double *__restrict__ Cinv, int32_t *info) {
    __shared__ double col[2][kCholReg], xrow[2][kCholReg], piv[kCholReg], rps[kCholReg];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t LL = (int64_t)L * L;
    double a[16], x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        a[r] = 0.0;
        x[r] = lane == w + 4 * r ? 1.0 : 0.0;
    }
    // partial Gram matrices summed in plane order, two planes' rows in flight together
    for (int z = 0; z < kz; z += 2) {
        double t[2][16];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = w + 4 * r;
                t[u][r] = (i < L && lane < L && z + u < kz) ? Gp[(z + u) * LL + i * L + lane] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r) a[r] += t[u][r];
    }
#pragma unroll
    for (int j = 0; j < kCholReg; ++j) {
        if (j < L) {   // uniform
            const int b = j & 1;
            if (lane == j) {
#pragma unroll
                for (int r = 0; r < 16; ++r) col[b][w + 4 * r] = a[r];
            }
            if (w == (j & 3)) xrow[b][lane] = x[j >> 2];
            __syncthreads();
            double d = col[b][j];
            if (!(d > 0.0)) {
                if (tid == 0 && info[0] == 0) info[0] = j + 1;
                d = 1.0;
            }
            // 1 / d: hardware reciprocal and two Newton steps (full double precision)
            double rd = __builtin_amdgcn_rcp(d);
            rd = fma(rd, fma(-d, rd, 1.0), rd);
            rd = fma(rd, fma(-d, rd, 1.0), rd);
            const double cj = col[b][lane], xr = xrow[b][lane];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = w + 4 * r;
                if (i > j && i < L) {   // uniform
                    const double f = col[b][i] * rd;
                    a[r] = (lane > j && lane <= i) ? fma(-f, cj, a[r]) : a[r];
                    x[r] = lane <= j ? fma(-f, xr, x[r]) : x[r];
                }
            }
            if (tid == 0) piv[j] = d;
        }
    }
    __syncthreads();
    if (tid < L) rps[tid] = 1.0 / sqrt(piv[tid]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = w + 4 * r;
        if (i < L && lane < L) {
            G[i * L + lane] = lane < i ? a[r] * rps[lane] : (lane == i ? 1.0 / rps[i] : 0.0);
            Cinv[i * L + lane] = lane <= i ? x[r] * rps[i] : 0.0;
        }
    }
}

// --------------------------------------------------- triangular applies
// U <- Cinv U in place for U [L][N], Cinv lower triangular: work group t
// stages columns 64 t .. 64 t + 63 of U (Lp = L rounded up to 16 rows) in
// LDS; wave w computes their 16-column block w for every 16-row block, K
// running over the block's lower-triangular range only.
constexpr int kApplyCols = 64;
__global__ __launch_bounds__(256) void left_apply_kernel(const double *__restrict__ Cinv, int32_t L,
                                                         double *__restrict__ U, int32_t N) {
    extern __shared__ double tile[];   // [Lp][kApplyCols + 1]
    constexpr int TS = kApplyCols + 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int Lp = (L + 15) & ~15, n0 = blockIdx.x * kApplyCols;
    for (int e = tid; e < Lp * kApplyCols; e += 256) {
        const int r = e / kApplyCols, c = e % kApplyCols;
        tile[r * TS + c] = (r < L && n0 + c < N) ? U[(int64_t)r * N + n0 + c] : 0.0;
    }
    __syncthreads();
    f64x4 acc[kMaxBasis / 16];
#pragma unroll
    for (int mb = 0; mb < kMaxBasis / 16; ++mb) acc[mb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int mb = 0; mb < kMaxBasis / 16; ++mb) {
        if (mb * 16 >= Lp) break;
        const int r = mb * 16 + li;
        const double *crow = Cinv + (int64_t)(r < L ? r : 0) * L;
        for (int k0 = 0; k0 < (mb + 1) * 16; k0 += 4) {   // Cinv[r][k] = 0 for k > r
            const int k = k0 + lg;
            const double a = (r < L && k < L) ? crow[k] : 0.0;
            acc[mb] = mfma_f64(a, tile[k * TS + wave * 16 + li], acc[mb]);
        }
    }
    const int c = n0 + wave * 16 + li;
    if (c < N) {
#pragma unroll
        for (int mb = 0; mb < kMaxBasis / 16; ++mb) {
            if (mb * 16 >= Lp) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = mb * 16 + lg + 4 * v;
                if (r < L) U[(int64_t)r * N + c] = acc[mb][v];
            }
        }
    }
}

// W <- W C in place for W [rows][L], C lower triangular: work group t stages
// rows 64 t .. 64 t + 63 of W in LDS; wave w computes their 16-row block w for
// every 16-column block cb, K = l running over cb 16 .. L only.
constexpr int kApplyRows = 64;
__global__ __launch_bounds__(256) void right_apply_kernel(double *__restrict__ W, int32_t rows, int32_t L,
                                                          const double *__restrict__ C) {
    extern __shared__ double tile[];   // [kApplyRows][Lp + 1]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int Lp = (L + 15) & ~15, TS = Lp + 1, r0 = blockIdx.x * kApplyRows;
    for (int e = tid; e < kApplyRows * Lp; e += 256) {
        const int r = e / Lp, c = e % Lp;
        tile[r * TS + c] = (r0 + r < rows && c < L) ? W[(int64_t)(r0 + r) * L + c] : 0.0;
    }
    __syncthreads();
    f64x4 acc[kMaxBasis / 16];
#pragma unroll
    for (int cb = 0; cb < kMaxBasis / 16; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double *arow = tile + (wave * 16 + li) * TS;
#pragma unroll
    for (int cb = 0; cb < kMaxBasis / 16; ++cb) {
        if (cb * 16 >= Lp) break;
        const int c = cb * 16 + li;
        for (int k0 = cb * 16; k0 < Lp; k0 += 4) {   // C[k][c] = 0 for k < c
            const int k = k0 + lg;
            const double b = (k < L && c < L) ? C[k * L + c] : 0.0;
            acc[cb] = mfma_f64(arow[k], b, acc[cb]);
        }
    }
#pragma unroll
    for (int cb = 0; cb < kMaxBasis / 16; ++cb) {
        if (cb * 16 >= Lp) break;
        const int c = cb * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + wave * 16 + lg + 4 * v;
            if (r < rows && c < L) W[(int64_t)r * L + c] = acc[cb][v];
        }
    }
}

__global__ void clear_info_kernel(int32_t *info, int32_t n) {
    if ((int)threadIdx.x < n) info[threadIdx.x] = 0;
}

// A kernel rather than a memset, so that the clear can sit in a captured graph.
hipError_t launch_clear_info(hipStream_t st, int32_t *info, int32_t n) {
    hipLaunchKernelGGL(clear_info_kernel, dim3(1), dim3(64), 0, st, info, n);
    return hipGetLastError();
}

static size_t chol_lds(int L) { return sizeof(double) * 2 * (size_t)L * L; }
static size_t left_apply_lds(int L) { return sizeof(double) * (size_t)((L + 15) & ~15) * (kApplyCols + 1); }
static size_t right_apply_lds(int L) { return sizeof(double) * (size_t)kApplyRows * (((L + 15) & ~15) + 1); }

// The applies stage up to 160 rows (or columns) of doubles and the factor
// kernel two 100 x 100 matrices: raise their dynamic-LDS limit once per
// process.
static hipError_t configure_apply_lds() {
    static hipError_t done = [] {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(left_apply_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)left_apply_lds(kMaxBasis));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(right_apply_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)right_apply_lds(kMaxBasis));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(chol_inv_kernel<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)chol_lds(kCholLds));
        return e;
    }();
    return done;
}

// `passes` CholeskyQR passes (1 or 2) on U [L][N] (and W [rows][L] unless
// rows == 0); G and Cinv hold L x L doubles each; info[pass] receives the
// first failing column + 1 of that pass's factorisation if it is still 0
// (cleared by the caller).  With Gpart (kz_max x L x L doubles) the Gram
// matrix is summed from up to kz_max partial products over ranges of at least
// 64 taps (enough work groups to cover the chip for small L); without it, from
// one.
static hipError_t cholesky_qr(hipStream_t st, double *U, int32_t L, int32_t N, double *W, int32_t rows, double *G,
                              double *Cinv, double *Gpart, int32_t kz_max, int32_t *info, int passes) {
    hipError_t e = configure_apply_lds();
    if (e != hipSuccess) return e;
    const int lb = (L + 15) / 16;
    int32_t kz = 1;
    if (Gpart) {
        const int tiles = lb * (lb + 1) / 2;
        kz = std::max(1, std::min({kz_max, 256 / tiles, (N + 63) / 64}));
    }
    const int32_t krange = (N + kz - 1) / kz;
    kz = (N + krange - 1) / krange;
    double *gp = kz > 1 ? Gpart : G;
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(gram_f64_kernel, dim3(lb, lb, kz), dim3(256), 0, st, U, L, N, krange, gp);
        if (L <= kCholReg)
            hipLaunchKernelGGL(chol_inv_reg_kernel, dim3(1), dim3(256), 0, st, gp, kz, G, L, Cinv, info + pass);
        else if (L <= kCholLds)
            hipLaunchKernelGGL(chol_inv_kernel<true>, dim3(1), dim3(256), chol_lds(L), st, gp, kz, G, L, Cinv,
                               info + pass);
        else
            hipLaunchKernelGGL(chol_inv_kernel<false>, dim3(1), dim3(256), 0, st, gp, kz, G, L, Cinv, info + pass);
        hipLaunchKernelGGL(left_apply_kernel, dim3((unsigned)((N + kApplyCols - 1) / kApplyCols)), dim3(256),
                           left_apply_lds(L), st, Cinv, L, U, N);
        if (rows > 0)   // rows == 0: orthonormalise U alone
            hipLaunchKernelGGL(right_apply_kernel, dim3((unsigned)((rows + kApplyRows - 1) / kApplyRows)), dim3(256),
                               right_apply_lds(L), st, W, rows, L, G);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_cholesky_qr2(hipStream_t st, double *U, int32_t L, int32_t N, double *W, int32_t rows, double *G,
                               double *Cinv, int32_t *info) {
    return cholesky_qr(st, U, L, N, W, rows, G, Cinv, nullptr, 1, info, 2);
}

}  // namespace lloid

// ------------------------------------------------ SVD bank construction
// The rank-L truncation of a slice's template matrix H (rows x N, float64)
// by subspace iteration, each half step orthonormalised:
//   P = orth(U H^T)   (L x rows: the row space of H U^T, transposed),
//   U = orth(P H)     (L x N),
// so every CholeskyQR factors a matrix of condition at most sigma_1 / sigma_L
// (orthonormalising only after the full H^T H product would square that and
// break the Cholesky factorisation for steep spectra).  U's rows converge to
// an orthonormal basis of the top-L right singular subspace (error ratio
// (sigma_{L+1} / sigma_L)^2 per iteration, when sigma_L > sigma_{L+1}; without
// a gap the captured energy still converges to the optimum), and W = H U^T,
// so that W U = H P_L, the best rank-L approximation.  One CholeskyQR pass
// per half step; two on the start and on the final basis.  Both products run
// on the FP64 GEMM split over K.
extern "C" lloid_status lloid_svd_basis(const double *H, int32_t rows, int32_t N, int32_t L, int32_t iters, double *U,
                                        double *W, void *stream) {
    using namespace lloid;
    if (!H || !U || !W || rows < 1 || N < 1 || L < 1 || L > kMaxBasis || L > rows || L > N || iters < 1 ||
        (int64_t)rows * N >= ((int64_t)1 << 28))
        return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // K splits: enough work groups for the chip on the two products
    const int32_t split_p = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, 256 / ((rows + 63) / 64)));
    const int32_t split_u = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, 256 / ((N + 63) / 64)));
    const int32_t split_w = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, 256 / ((rows + 63) / 64)));
    const int64_t part_n = std::max<int64_t>(std::max<int64_t>((int64_t)split_p * L * rows, (int64_t)split_u * L * N),
                                             (int64_t)split_w * rows * L);
    // partial Gram planes: up to kGramSplit, fewer for large L
    const int32_t kz_max = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kGramSplit, 65536 / ((int64_t)L * L)));
    double *P = nullptr, *G = nullptr, *Ci = nullptr, *part = nullptr, *Gp = nullptr;
    int32_t *info = nullptr;
    lloid_status status = LLOID_OK;
    if (hipMalloc(&P, sizeof(double) * rows * L) != hipSuccess || hipMalloc(&G, sizeof(double) * L * L) != hipSuccess ||
        hipMalloc(&Ci, sizeof(double) * L * L) != hipSuccess || hipMalloc(&info, sizeof(int32_t) * 2) != hipSuccess ||
        hipMalloc(&part, sizeof(double) * part_n) != hipSuccess ||
        hipMalloc(&Gp, sizeof(double) * kz_max * L * L) != hipSuccess)
        status = LLOID_E_NOMEM;
    hipError_t e = hipSuccess;
    if (status == LLOID_OK) {
        // cleared once: a breakdown in any pass stays latched until the end
        e = launch_clear_info(st, info, 2);
        if (e == hipSuccess) e = cholesky_qr(st, U, L, N, nullptr, 0, G, Ci, Gp, kz_max, info, 2);   // orthonormal start
        for (int it = 0; it < iters && e == hipSuccess; ++it) {
            // P = U H^T  (L x rows, K = N taps), then orthonormal rows
            e = launch_gemm_f64(st, U, N, 1, H, 1, N, L, rows, N, split_p, part, P);
            if (e == hipSuccess) e = cholesky_qr(st, P, L, rows, nullptr, 0, G, Ci, Gp, kz_max, info, 1);
            // U = P H  (L x N, K = rows), then orthonormal rows
            if (e == hipSuccess) e = launch_gemm_f64(st, P, rows, 1, H, N, 1, L, N, rows, split_u, part, U);
            if (e == hipSuccess)
                e = cholesky_qr(st, U, L, N, nullptr, 0, G, Ci, Gp, kz_max, info, it == iters - 1 ? 2 : 1);
        }
        if (e == hipSuccess) e = launch_gemm_f64(st, H, N, 1, U, 1, N, rows, L, N, split_w, part, W);   // W = H U^T
        int32_t h[2] = {0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) status = LLOID_E_HIP;
        else if (h[0] || h[1]) status = LLOID_E_STATE;
    }
    (void)hipFree(P);
    (void)hipFree(G);
    (void)hipFree(Ci);
    (void)hipFree(info);
    (void)hipFree(part);
    (void)hipFree(Gp);
    return status;
}
