// dense.hip -- the dense force solve of Sec. 3.2: the Schur complement C is
// factored once (C = L L^T, FP64) and its inverse factor W = L^{-1} kept, so
// that every later solve is f = W^T (W b), two triangular matrix-vector
// products that stream W from HBM.
//
// Factorisation: recursive on halves, so that all but the 64 x 64 diagonal
// leaves is matrix multiplication on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  For A = [A11 .; A21 A22] with L11 = chol(A11),
// W11 = L11^{-1}:
//   L21 = A21 W11^T,   A22 <- A22 - L21 L21^T,   L22 = chol(A22),
//   W21 = -W22 (L21 W11).
// Each leaf is factored and inverted by one workgroup in LDS.
// Matrices are row-major doubles with a leading dimension; only the lower
// triangle of A is read.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace lgfib {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kLeaf = 64;   // leaf order of the recursive factorisation
constexpr int kKT = 16;     // K slice staged in LDS per GEMM step

// C = alpha op(A) op(B) + beta C with op(A)(m, k) = A[m lda + k] and
// op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n].  Tile (32 FM)^2 per
// workgroup of four waves, each wave (16 FM)^2 as FM x FM blocks of 16 x 16.
// lower != 0 skips tiles that lie strictly above the diagonal m = n.
template <int FM, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                  long lda, const double *__restrict__ Bm, long ldb, double beta,
                                                  double *__restrict__ C, long ldc, int lower) {
    constexpr int T = 32 * FM;              // tile edge
    constexpr int PER = T * kKT / 256;      // staged values per thread and operand
    __shared__ double As[T][kKT + 1];       // [m][k]
    __shared__ double Bs[T][kKT + 1];       // [n][k]
    const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
    if (lower && n0 > m0 + T - 1) return;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = (wave / 2) * 16 * FM, wn = (wave % 2) * 16 * FM;
    f64x4 acc[FM][FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FM; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    double ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            {
                const int mm = e / kKT, kk = e % kKT, m = m0 + mm, k = k0 + kk;
                ra[q] = (m < M && k < K) ? A[(long)m * lda + k] : 0.0;
            }
            if (TB) {
                const int nn = e / kKT, kk = e % kKT, n = n0 + nn, k = k0 + kk;
                rb[q] = (n < N && k < K) ? Bm[(long)n * ldb + k] : 0.0;
            } else {
                const int kk = e / T, nn = e % T, n = n0 + nn, k = k0 + kk;
                rb[q] = (n < N && k < K) ? Bm[(long)k * ldb + n] : 0.0;
            }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            As[e / kKT][e % kKT] = ra[q];
            if (TB)
                Bs[e / kKT][e % kKT] = rb[q];
            else
                Bs[e % T][e / T] = rb[q];
        }
    };
    fetch(0);
    stage();
    __syncthreads();
    // operand layout of v_mfma_f64_16x16x4f64: lane l holds A[row l%16][k l/16]
    // and B[k l/16][col l%16]; the result D[row l/16 + 4q][col l%16] in acc[q]
    // (rows interleaved, unlike the 16x16x16 BF16 form)
    const int r = lane % 16, kq = lane / 16;
    for (int k0 = 0; k0 < K; k0 += kKT) {
        const bool more = k0 + kKT < K;
        if (more) fetch(k0 + kKT);
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 4) {
            double a[FM], b[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[wm + 16 * i + r][ks + kq];
#pragma unroll
            for (int j = 0; j < FM; ++j) b[j] = Bs[wn + 16 * j + r][ks + kq];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (more) {
            stage();
            __syncthreads();
        }
    }
    const int c = lane % 16, rq = lane / 16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + rq + 4 * q, n = n0 + wn + 16 * j + c;
                if (m < M && n < N) {
                    double v = alpha * acc[i][j][q];
                    if (beta != 0.0) v += beta * C[(long)m * ldc + n];
                    C[(long)m * ldc + n] = v;
                }
            }
}

int gemm_f64(int M, int N, int K, double alpha, const double *A, long lda, const double *B, long ldb, bool tb,
             double beta, double *C, long ldc, bool lower, hipStream_t st) {
    if (M <= 0 || N <= 0) return LGFIB_OK;
    const bool big = (long)M * N >= 512l * 512;
    const int T = big ? 128 : 64;
    const dim3 grid((N + T - 1) / T, (M + T - 1) / T);
    const int lw = lower ? 1 : 0;
    if (big) {
        if (tb)
            hipLaunchKernelGGL((k_gemm_f64<4, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                               ldc, lw);
        else
            hipLaunchKernelGGL((k_gemm_f64<4, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                               ldc, lw);
    } else {
        if (tb)
            hipLaunchKernelGGL((k_gemm_f64<2, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                               ldc, lw);
        else
            hipLaunchKernelGGL((k_gemm_f64<2, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                               ldc, lw);
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// value of v in lane `lane` (uniform; lane is a compile-time constant here)
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Leaf: Cholesky factor and its inverse of an n x n block (n <= 64) by one
// wavefront, entirely in registers: lane i keeps row i of the block (rows
// n..63 padded with the identity, whose factor is the identity).  Step k,
// right-looking: pivot and column entries are read from their owner lanes,
// every lane scales its column-k entry and updates the rest of its row.
// Then lane j builds column j of W = L^{-1} by forward substitution,
// W[j][j] = 1 / L[j][j], W[q][j] = -(sum_{k<q} L[q][k] W[k][j]) / L[q][q],
// reading row q of L from lane q.  A pivot that is not positive sets *bad;
// the factor then holds NaN.
__global__ __launch_bounds__(kLeaf) void k_chol_leaf(double *__restrict__ A, long lda, double *__restrict__ W, long ldw,
                                                     int n, int *__restrict__ bad) {
    const int i = threadIdx.x;
    double r[kLeaf];
#pragma unroll
    for (int j = 0; j < kLeaf; ++j) r[j] = i < n ? (j <= i ? A[(long)i * lda + j] : 0.0) : (j == i ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < kLeaf; ++k) {
        const double d = lane_value(r[k], k);
        if (!(d > 0.0) && i == 0) *bad = 1;
        const double piv = d > 0.0 ? sqrt(d) : NAN, inv = 1.0 / piv;
        r[k] = i > k ? r[k] * inv : (i == k ? piv : r[k]);
        const double lik = r[k];
#pragma unroll
        for (int j = k + 1; j < kLeaf; ++j) r[j] -= lik * lane_value(r[k], j);
    }
    // column j = i of the inverse
    const int j = i;
    double w[kLeaf];
#pragma unroll
    for (int q = 0; q < kLeaf; ++q) w[q] = 0.0;
#pragma unroll
    for (int q = 0; q < kLeaf; ++q) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < q; ++k) s += lane_value(r[k], q) * w[k];
        const double dq = 1.0 / lane_value(r[q], q);
        w[q] = q > j ? -s * dq : (q == j ? dq : 0.0);
    }
    if (i < n) {
#pragma unroll
        for (int q = 0; q < kLeaf; ++q) {
            if (q < n) {
                if (q <= i) A[(long)i * lda + q] = r[q];   // row i of L
                W[(long)q * ldw + j] = w[q];               // column j of W
            }
        }
    }
}

__global__ void k_copy2d(const double *__restrict__ src, long lds, double *__restrict__ dst, long ldd, int rows,
                         int cols) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)rows * cols) return;
    const int i = (int)(t / cols), j = (int)(t % cols);
    dst[(long)i * ldd + j] = src[(long)i * lds + j];
}

__global__ void k_zero2d(double *__restrict__ dst, long ldd, int rows, int cols) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)rows * cols) return;
    dst[(long)(t / cols) * ldd + t % cols] = 0.0;
}

static inline unsigned nblk256(long n) { return (unsigned)((n + 255) / 256); }

// factor the n x n block at A (lower) into L (in place) and W = L^{-1};
// S: workspace of at least (n/2 + 64) * (n/2 + 64) doubles
static int chol_rec(lgfib_ctx *ctx, int n, double *A, long lda, double *W, long ldw, double *S, int *bad,
                    hipStream_t st) {
    int rc;
    if (n <= kLeaf) {
        ProfScope ps(ctx, "k_chol_leaf", st);
        hipLaunchKernelGGL(k_chol_leaf, dim3(1), dim3(kLeaf), 0, st, A, lda, W, ldw, n, bad);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    const int n1 = kLeaf * ((n + 2 * kLeaf - 1) / (2 * kLeaf)), n2 = n - n1;
    double *A21 = A + (long)n1 * lda, *A22 = A21 + n1, *W21 = W + (long)n1 * ldw, *W22 = W21 + n1;
    if ((rc = chol_rec(ctx, n1, A, lda, W, ldw, S, bad, st))) return rc;
    {
        ProfScope ps(ctx, "k_gemm_f64", st);
        // S = L21 = A21 W11^T, copied over A21
        if ((rc = gemm_f64(n2, n1, n1, 1.0, A21, lda, W, ldw, true, 0.0, S, n1, false, st))) return rc;
        hipLaunchKernelGGL(k_copy2d, dim3(nblk256((long)n2 * n1)), dim3(256), 0, st, S, (long)n1, A21, lda, n2, n1);
        LGF_HIP(hipGetLastError());
        // A22 -= L21 L21^T (tiles on and below the diagonal)
        if ((rc = gemm_f64(n2, n2, n1, -1.0, A21, lda, A21, lda, true, 1.0, A22, lda, true, st))) return rc;
    }
    if ((rc = chol_rec(ctx, n2, A22, lda, W22, ldw, S, bad, st))) return rc;
    {
        ProfScope ps(ctx, "k_gemm_f64", st);
        // W21 = -W22 (L21 W11)
        if ((rc = gemm_f64(n2, n1, n1, 1.0, A21, lda, W, ldw, false, 0.0, S, n1, false, st))) return rc;
        if ((rc = gemm_f64(n2, n1, n2, -1.0, W22, ldw, S, n1, false, 0.0, W21, ldw, false, st))) return rc;
    }
    return LGFIB_OK;
}

int chol_factor_f64(lgfib_ctx *ctx, int n, double *A, long lda, double *W, long ldw, hipStream_t st) {
    if (n == 0) return LGFIB_OK;
    int rc;
    const size_t h = (size_t)n / 2 + kLeaf;
    if ((rc = ctx->dense_ws.reserve(h * h * sizeof(double))) || (rc = ctx->dense_flag.reserve(sizeof(int))))
        return rc;
    LGF_HIP(hipMemsetAsync(ctx->dense_flag.p, 0, sizeof(int), st));
    // the strict upper blocks of W are never written by the recursion
    hipLaunchKernelGGL(k_zero2d, dim3(nblk256((long)n * n)), dim3(256), 0, st, W, ldw, n, n);
    LGF_HIP(hipGetLastError());
    if ((rc = chol_rec(ctx, n, A, lda, W, ldw, ctx->dense_ws.as<double>(), ctx->dense_flag.as<int>(), st))) return rc;
    int bad = 0;
    LGF_HIP(hipMemcpyAsync(&bad, ctx->dense_flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    LGF_HIP(hipStreamSynchronize(st));
    if (bad) return fail(LGFIB_ENOTSPD, "Cholesky factorisation: the matrix is not positive definite");
    return LGFIB_OK;
}

// y = W b, W lower triangular: one wavefront per row, j <= i
__global__ __launch_bounds__(256) void k_trmv_rows(const double *__restrict__ W, long ldw, const double *__restrict__ b,
                                                   double *__restrict__ y, int n) {
    const int row = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (row >= n) return;
    const double *w = W + (long)row * ldw;
    double s = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;   // four loads in flight per lane
    int j = lane;
    for (; j + 192 <= row; j += 256) {
        s += w[j] * b[j];
        s1 += w[j + 64] * b[j + 64];
        s2 += w[j + 128] * b[j + 128];
        s3 += w[j + 192] * b[j + 192];
    }
    for (; j <= row; j += 64) s += w[j] * b[j];
    s += (s1 + s2) + s3;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[row] = s;
}

constexpr int kColChunks = 32;   // row chunks of the transposed product

// part[r][j] = sum over rows i of chunk r with i >= j of W[i][j] y[i]
__global__ __launch_bounds__(256) void k_trmv_cols(const double *__restrict__ W, long ldw, const double *__restrict__ y,
                                                   double *__restrict__ part, int n, int rows_per) {
    const int j = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
    const int j0 = blockIdx.x * 256;
    const int i0 = max(r * rows_per, j0), i1 = min((r + 1) * rows_per, n);
    double s = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (j < n) {
        const double *wc = W + j;
        int i = i0;
        for (; i + 3 < i1; i += 4) {   // entries above the diagonal are not part of W
            const double w0 = wc[(long)i * ldw], w1 = wc[(long)(i + 1) * ldw], w2 = wc[(long)(i + 2) * ldw],
                         w3 = wc[(long)(i + 3) * ldw];
            s += (i >= j ? w0 : 0.0) * y[i];
            s1 += (i + 1 >= j ? w1 : 0.0) * y[i + 1];
            s2 += (i + 2 >= j ? w2 : 0.0) * y[i + 2];
            s3 += (i + 3 >= j ? w3 : 0.0) * y[i + 3];
        }
        for (; i < i1; ++i) s += (i >= j ? wc[(long)i * ldw] : 0.0) * y[i];
        part[(long)r * n + j] = s + ((s1 + s2) + s3);
    }
}

__global__ void k_sum_parts(const double *__restrict__ part, double *__restrict__ x, int n, int nparts) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int r = 0; r < nparts; ++r) s += part[(long)r * n + j];
    x[j] = s;
}

int chol_solve_f64(lgfib_ctx *ctx, int n, const double *W, long ldw, const double *b, double *x, hipStream_t st) {
    if (n == 0) return LGFIB_OK;
    int rc;
    if ((rc = ctx->dense_solve_ws.reserve((size_t)(kColChunks + 1) * n * sizeof(double)))) return rc;
    double *y = ctx->dense_solve_ws.as<double>(), *part = y + n;
    {
        ProfScope ps(ctx, "k_trmv_rows", st);
        hipLaunchKernelGGL(k_trmv_rows, dim3((n + 3) / 4), dim3(256), 0, st, W, ldw, b, y, n);
        LGF_HIP(hipGetLastError());
    }
    {
        ProfScope ps(ctx, "k_trmv_cols", st);
        const int rows_per = (n + kColChunks - 1) / kColChunks;
        hipLaunchKernelGGL(k_trmv_cols, dim3((n + 255) / 256, kColChunks), dim3(256), 0, st, W, ldw, y, part, n,
                           rows_per);
        LGF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sum_parts, dim3((n + 255) / 256), dim3(256), 0, st, part, x, n, kColChunks);
        LGF_HIP(hipGetLastError());
    }
    return LGFIB_OK;
}

}  // namespace lgfib

using namespace lgfib;

static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

extern "C" int ib_chol_factor(lgfib_ctx *ctx, int n, double *A, int lda, double *W, int ldw, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "ib_chol_factor: null context");
    if (n < 0 || lda < std::max(n, 1) || ldw < std::max(n, 1))
        return fail(LGFIB_EINVAL, "ib_chol_factor: need n >= 0 and leading dimensions >= n");
    if (n > 0 && (!A || !W)) return fail(LGFIB_EINVAL, "ib_chol_factor: null matrix");
    if (n > 0 && overlaps(A, ((size_t)(n - 1) * lda + n) * 8, W, ((size_t)(n - 1) * ldw + n) * 8))
        return fail(LGFIB_EINVAL, "ib_chol_factor: A and W overlap");
    LGF_HIP(hipSetDevice(ctx->device));
    return chol_factor_f64(ctx, n, A, lda, W, ldw, (hipStream_t)stream);
}

extern "C" int ib_chol_solve(lgfib_ctx *ctx, int n, const double *W, int ldw, const double *b, double *x,
                             lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "ib_chol_solve: null context");
    if (n < 0 || ldw < std::max(n, 1)) return fail(LGFIB_EINVAL, "ib_chol_solve: need n >= 0 and ldw >= n");
    if (n > 0 && (!W || !b || !x)) return fail(LGFIB_EINVAL, "ib_chol_solve: null pointer");
    LGF_HIP(hipSetDevice(ctx->device));
    return chol_solve_f64(ctx, n, W, ldw, b, x, (hipStream_t)stream);
}
