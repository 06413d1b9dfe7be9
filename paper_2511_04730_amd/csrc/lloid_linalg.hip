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

#include "lloid_internal.h"

namespace lloid {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// --------------------------------------------------------------- GEMM
// part[z][m][n] = sum over k in [z ksplit, (z + 1) ksplit) of A(m,k) B(k,n),
// A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn].  64 x 64 tile per work
// group, 16-deep K stages in LDS; wave w owns the tile's columns 16 w .. + 15
// for all four 16-row blocks.  Out-of-range rows, columns and K read as zero.
constexpr int kDT = 64, kDK = 16;
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ A, int64_t sam, int64_t sak,
                                                       const double *__restrict__ B, int64_t sbk, int64_t sbn,
                                                       int64_t M, int64_t N, int64_t K, int64_t ksplit,
                                                       double *__restrict__ part) {
    __shared__ double As[kDT][kDK + 1];
    __shared__ double Bs[kDK][kDT + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * kDT, n0 = (int64_t)blockIdx.y * kDT;
    const int64_t k_begin = (int64_t)blockIdx.z * ksplit;
    const int64_t k_end = k_begin + ksplit < K ? k_begin + ksplit : K;
    f64x4 acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = f64x4{0.0, 0.0, 0.0, 0.0};
    const bool a_kfast = sak == 1, b_nfast = sbn == 1;
    for (int64_t kk = k_begin; kk < k_end; kk += kDK) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kDT * kDK / 256; ++i) {
            const int e = tid + 256 * i;
            int mm, k;
            if (a_kfast) {
                mm = e / kDK;
                k = e % kDK;
            } else {
                k = e / kDT;
                mm = e % kDT;
            }
            const int64_t gm = m0 + mm, gk = kk + k;
            As[mm][k] = (gm < M && gk < k_end) ? A[gm * sam + gk * sak] : 0.0;
            int nn, k2;
            if (b_nfast) {
                k2 = e / kDT;
                nn = e % kDT;
            } else {
                nn = e / kDK;
                k2 = e % kDK;
            }
            const int64_t gn = n0 + nn, gk2 = kk + k2;
            Bs[k2][nn] = (gn < N && gk2 < k_end) ? B[gk2 * sbk + gn * sbn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kDK; ks += 4) {
            const double b = Bs[ks + lg][wave * 16 + li];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma_f64(As[mb * 16 + li][ks + lg], b, acc[mb]);
        }
    }
    const int64_t n = n0 + wave * 16 + li;
    if (n < N) {
        double *o = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + mb * 16 + lg + 4 * v;
                if (m < M) o[m * N + n] = acc[mb][v];
            }
    }
}

// out[i] = sum_s part[s plane + i], s = 0, 1, ... in order
__global__ __launch_bounds__(256) void sum_parts_kernel(const double *__restrict__ part, int32_t nsplit, int64_t plane,
                                                        double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= plane) return;
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += part[p * plane + i];
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
    hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, ksplit, dst);
    if (ns > 1)
        hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, st, part, (int32_t)ns,
                           M * N, C);
    return hipGetLastError();
}

// ------------------------------------------------------------ Gram
// G = U U^T for U [L][N]: work group (bi, bj), bi >= bj, computes the 16x16
// tile G[16 bi ..][16 bj ..] and its mirror.  Wave w takes K blocks of 16
// taps w, w + 4, ... (four per trip); lane (li, lg) supplies taps
// 4 lg .. 4 lg + 3 of a block, one per MFMA, for row 16 bi + li (A) and row
// 16 bj + li (B).  The four waves' tiles are summed in wave order.
__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ U, int32_t L, int32_t N,
                                                       double *__restrict__ G) {
    __shared__ double red[4][64 * 4];
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bj > bi) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
    const int ra = bi * 16 + li, rb = bj * 16 + li;
    const double *ua = U + (int64_t)(ra < L ? ra : 0) * N;
    const double *ub = U + (int64_t)(rb < L ? rb : 0) * N;
    const bool va = ra < L, vb = rb < L;
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    // four blocks per trip: all 32 loads of a lane are in flight before its MFMAs
    for (int k0 = wave * 16; k0 < N; k0 += 256) {
        double a[16], b[16];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 64 * u + 4 * lg;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = k + s < N;
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
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double s = ((red[0][lane * 4 + v] + red[1][lane * 4 + v]) + red[2][lane * 4 + v]) + red[3][lane * 4 + v];
            const int r = bi * 16 + lg + 4 * v, c = bj * 16 + li;
            if (r < L && c < L) {
                G[r * L + c] = s;
                G[c * L + r] = s;
            }
        }
    }
}

// ------------------------------------------------------- Cholesky, inverse
// One work group factors the L x L SPD matrix G = C C^T (C lower) and
// inverts C, both right-looking so that every step is one parallel update
// between two barriers:
//   Cholesky, column j: pivot sqrt(G[j][j]), column j below it divided by
//   the pivot, trailing lower triangle G[i][k] -= G[i][j] G[k][j];
//   inverse (forward elimination of C X = I, X = I at the start), row j:
//   X[j][c] /= C[j][j] for c <= j, then X[i][c] -= C[i][j] X[j][c] for
//   i > j, c <= j.
// A pivot that is not positive is replaced by 1 (so the passes run on) and,
// if info[0] is still 0, recorded there as its column + 1; info is never
// reset here, so a breakdown stays reported until the caller clears it
// (launch_clear_info).  LDS holds both matrices for L <= kCholLds (dynamic
// LDS); above that they are updated in place in global memory.  On return
// G holds C (upper triangle zero) and Cinv its inverse.
constexpr int kCholLds = 100;   // 2 x 100^2 doubles = 160000 bytes of LDS
template <bool LDS>
__global__ __launch_bounds__(256) void chol_inv_kernel(double *__restrict__ G, int32_t L,
                                                       double *__restrict__ Cinv, int32_t *info) {
    extern __shared__ double sm[];
    __shared__ double piv;
    double *a = LDS ? sm : G;
    double *x = LDS ? sm + L * L : Cinv;
    const int tid = threadIdx.x;
    for (int e = tid; e < L * L; e += 256) {
        if (LDS) a[e] = G[e];
        x[e] = (e / L == e % L) ? 1.0 : 0.0;
    }
    for (int j = 0; j < L; ++j) {
        __syncthreads();
        if (tid == 0) {
            double d = a[j * L + j];
            if (!(d > 0.0)) {
                if (info[0] == 0) info[0] = j + 1;
                d = 1.0;
            }
            piv = sqrt(d);
            a[j * L + j] = piv;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < L; i += 256) a[i * L + j] /= piv;
        __syncthreads();
        // thread (ti, tk) of a 16 x 16 grid updates rows i = j + 1 + ti + 16 m,
        // columns k = j + 1 + tk + 16 n, k <= i
        for (int i = j + 1 + (tid >> 4); i < L; i += 16) {
            const double aij = a[i * L + j];
            for (int k = j + 1 + (tid & 15); k <= i; k += 16) a[i * L + k] -= aij * a[k * L + j];
        }
    }
    for (int j = 0; j < L; ++j) {
        __syncthreads();
        const double cjj = a[j * L + j];
        for (int c = tid; c <= j; c += 256) x[j * L + c] /= cjj;
        __syncthreads();
        for (int i = j + 1 + (tid >> 4); i < L; i += 16) {
            const double aij = a[i * L + j];
            for (int c = tid & 15; c <= j; c += 16) x[i * L + c] -= aij * x[j * L + c];
        }
    }
    __syncthreads();
    for (int e = tid; e < L * L; e += 256) {
        const bool upper = e % L > e / L;
        G[e] = upper ? 0.0 : a[e];
        if (LDS) Cinv[e] = x[e];
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
// (cleared by the caller).
hipError_t launch_cholesky_qr(hipStream_t st, double *U, int32_t L, int32_t N, double *W, int32_t rows, double *G,
                              double *Cinv, int32_t *info, int passes) {
    hipError_t e = configure_apply_lds();
    if (e != hipSuccess) return e;
    const unsigned lb = (unsigned)((L + 15) / 16);
    for (int pass = 0; pass < passes; ++pass) {
        hipLaunchKernelGGL(gram_f64_kernel, dim3(lb, lb), dim3(256), 0, st, U, L, N, G);
        if (L <= kCholLds)
            hipLaunchKernelGGL(chol_inv_kernel<true>, dim3(1), dim3(256), chol_lds(L), st, G, L, Cinv, info + pass);
        else
            hipLaunchKernelGGL(chol_inv_kernel<false>, dim3(1), dim3(256), 0, st, G, L, Cinv, info + pass);
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
    return launch_cholesky_qr(st, U, L, N, W, rows, G, Cinv, info, 2);
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
    if (!H || !U || !W || rows < 1 || N < 1 || L < 1 || L > kMaxBasis || L > rows || L > N || iters < 1)
        return LLOID_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // K splits: enough work groups for the chip on the two products
    const int32_t split_p = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, 256 / ((rows + 63) / 64)));
    const int32_t split_u = (int32_t)std::max<int64_t>(1, std::min<int64_t>(32, 256 / ((N + 63) / 64)));
    const int32_t split_w = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, 256 / ((rows + 63) / 64)));
    const int64_t part_n = std::max<int64_t>(std::max<int64_t>((int64_t)split_p * L * rows, (int64_t)split_u * L * N),
                                             (int64_t)split_w * rows * L);
    double *P = nullptr, *G = nullptr, *Ci = nullptr, *part = nullptr;
    int32_t *info = nullptr;
    lloid_status status = LLOID_OK;
    if (hipMalloc(&P, sizeof(double) * rows * L) != hipSuccess || hipMalloc(&G, sizeof(double) * L * L) != hipSuccess ||
        hipMalloc(&Ci, sizeof(double) * L * L) != hipSuccess || hipMalloc(&info, sizeof(int32_t) * 2) != hipSuccess ||
        hipMalloc(&part, sizeof(double) * part_n) != hipSuccess)
        status = LLOID_E_NOMEM;
    hipError_t e = hipSuccess;
    if (status == LLOID_OK) {
        // cleared once: a breakdown in any pass stays latched until the end
        e = launch_clear_info(st, info, 2);
        if (e == hipSuccess) e = launch_cholesky_qr(st, U, L, N, nullptr, 0, G, Ci, info, 2);   // orthonormal start
        for (int it = 0; it < iters && e == hipSuccess; ++it) {
            // P = U H^T  (L x rows, K = N taps), then orthonormal rows
            e = launch_gemm_f64(st, U, N, 1, H, 1, N, L, rows, N, split_p, part, P);
            if (e == hipSuccess) e = launch_cholesky_qr(st, P, L, rows, nullptr, 0, G, Ci, info, 1);
            // U = P H  (L x N, K = rows), then orthonormal rows
            if (e == hipSuccess) e = launch_gemm_f64(st, P, rows, 1, H, N, 1, L, N, rows, split_u, part, U);
            if (e == hipSuccess) e = launch_cholesky_qr(st, U, L, N, nullptr, 0, G, Ci, info, it == iters - 1 ? 2 : 1);
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
    return status;
}
