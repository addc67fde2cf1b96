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
constexpr int kKT = 32;     // K slice staged in LDS per GEMM step (16 and 64 measured slower)

// C = alpha op(A) op(B) + beta C with op(A)(m, k) = A[m lda + k] and
// op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n].  Tile (32 FM)^2 per
// workgroup of four waves, each wave (16 FM)^2 as FM x FM blocks of 16 x 16.
// lower != 0 skips tiles that lie strictly above the diagonal m = n.  tri
// names an operand that is lower triangular (zero above its diagonal), whose
// zero part a tile then skips along k: kTriBtLower, op(B)(k, n) = B[n][k]
// with k <= n; kTriBLower, op(B)(k, n) = B[k][n] with k >= n; kTriALower,
// op(A)(m, k) = A[m][k] with k <= m.  The skipped entries must be zero.
template <int FM, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                  long lda, const double *__restrict__ Bm, long ldb, double beta,
                                                  double *__restrict__ C, long ldc, int lower, int tri) {
    constexpr int T = 32 * FM;              // tile edge
    constexpr int PER = T * kKT / 256;      // staged values per thread and operand
    // two LDS buffers: slice s + 1 is staged while slice s is multiplied
    __shared__ double As[2][T][kKT + 1];    // [m][k]
    __shared__ double Bs[2][T][kKT + 1];    // [n][k]
    const int m0 = blockIdx.y * T, n0 = blockIdx.x * T;
    if (lower && n0 > m0 + T - 1) return;
    // k range of the tile (tile edges are multiples of kKT)
    const int kb = tri == kTriBLower ? min(n0, K) : 0;
    const int ke = tri == kTriBtLower ? min(n0 + T, K) : (tri == kTriALower ? min(m0 + T, K) : K);
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = (wave / 2) * 16 * FM, wn = (wave % 2) * 16 * FM;
    f64x4 acc[FM][FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FM; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    double ra[PER], rb[PER];
    // slice k0 .. k0 + kKT - 1 into registers.  Loads are clamped into the
    // matrices, so they need no branch: rows of A past M and columns of B
    // past N only reach outputs that are not stored, and entries at k >= ke
    // are zeroed in A alone, which removes their products.
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            {
                const int mm = e / kKT, kk = e % kKT, m = m0 + mm, k = k0 + kk;
                const double v = A[(long)min(m, M - 1) * lda + min(k, ke - 1)];
                ra[q] = k < ke ? v : 0.0;
            }
            if (TB) {
                const int nn = e / kKT, kk = e % kKT, n = n0 + nn, k = k0 + kk;
                rb[q] = Bm[(long)min(n, N - 1) * ldb + min(k, ke - 1)];
            } else {
                const int kk = e / T, nn = e % T, n = n0 + nn, k = k0 + kk;
                rb[q] = Bm[(long)min(k, ke - 1) * ldb + min(n, N - 1)];
            }
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + 256 * q;
            As[buf][e / kKT][e % kKT] = ra[q];
            if (TB)
                Bs[buf][e / kKT][e % kKT] = rb[q];
            else
                Bs[buf][e % T][e / T] = rb[q];
        }
    };
    fetch(kb);
    stage(0);
    __syncthreads();
    // operand layout of v_mfma_f64_16x16x4f64: lane l holds A[row l%16][k l/16]
    // and B[k l/16][col l%16]; the result D[row l/16 + 4q][col l%16] in acc[q]
    // (rows interleaved, unlike the 16x16x16 BF16 form)
    const int r = lane % 16, kq = lane / 16;
    const int nslice = (ke - kb + kKT - 1) / kKT;
    for (int s = 0; s < nslice; ++s) {
        const int buf = s & 1;
        fetch(kb + (s + 1) * kKT);   // zeros after the last slice
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 4) {
            double a[FM], b[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[buf][wm + 16 * i + r][ks + kq];
#pragma unroll
            for (int j = 0; j < FM; ++j) b[j] = Bs[buf][wn + 16 * j + r][ks + kq];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        stage(buf ^ 1);
        __syncthreads();
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
             double beta, double *C, long ldc, bool lower, int tri, hipStream_t st) {
    if (M <= 0 || N <= 0) return LGFIB_OK;
    if (K <= 0) return fail(LGFIB_EINVAL, "gemm_f64: empty inner dimension");
    // 64-edge tiles for every product: the 128-edge form (FM = 4) measured
    // slower even on the 3300-edge products of the top split (fewer
    // workgroups in flight)
    constexpr int T = 64;
    const dim3 grid((N + T - 1) / T, (M + T - 1) / T);
    const int lw = lower ? 1 : 0;
    if (tb)
        hipLaunchKernelGGL((k_gemm_f64<2, true>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                           ldc, lw, tri);
    else
        hipLaunchKernelGGL((k_gemm_f64<2, false>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                           ldc, lw, tri);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// 1 / sqrt(d) to double precision: the hardware estimate and two Newton
// steps y <- y + y (1 - d y^2) / 2 (NaN for d < 0, infinity for d = 0)
__device__ __forceinline__ double rsqrt_f64(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(0.5 * y, fma(-d, y * y, 1.0), y);
    return y;
}

// Leaf: Cholesky factor L and its inverse W = L^{-1} of an n x n block
// (n <= kLeaf) by one workgroup of 256 threads (rows n..kLeaf-1 padded with
// the identity, whose factor is the identity).  Thread t works on row
// i = t / 4 and the columns j = t mod 4 (mod 4).
// Factor, right-looking, four columns per outer step: in registers,
// r[m] = a[i][4 (c + m) + t mod 4] for the current column group c (the
// array shifts down by one after each group, so that its indices stay
// constants).  Step k reads column k (final, not yet scaled) from LDS, where
// it is published with zeros in rows <= k and its pivot d_k = a[k][k] in a
// slot of its own; every thread then subtracts a[i][k] a[j][k] / d_k from all
// of its entries, which leaves rows <= k and columns <= k as they are, and
// scales its column-k entry, L[k][k] = sqrt(d_k), L[i][k] = a[i][k] / L[k][k].
// The holders of column k + 1 update it first and publish it into the other
// of two buffers, so a step needs one barrier.  Entries above the diagonal
// are garbage (finite) and never stored.
// Inverse, from L W = I row by row: row k of W (the residual, not yet
// divided by L[k][k]) is published; its holders divide their copy by L[k][k]
// and the rows q > k subtract L[q][k] / L[k][k] times it.  The entries of W
// above the diagonal stay exactly zero, so every step can run over all of
// them.  A pivot that is not positive sets *bad; the factor then holds NaN.
// On return, ls holds W (row stride kLeaf + 1; the padding rows and columns
// n..kLeaf-1 hold the identity).
constexpr int kLeafThreads = 256;
constexpr int kLeafPer = kLeaf * kLeaf / kLeafThreads;   // entries of a row part
constexpr int kLP = kLeaf + 1;                           // row stride of the LDS tiles
struct LeafLds {
    double ls[kLeaf * kLP];     // the factor, then W (staging of the outputs)
    double vec[2][2 * kLeaf];   // column k of the factor / row k of W (upper half: slack)
    double piv_in[2];           // d_k
    double rdiag[kLeaf];        // 1 / L[k][k]
};
__device__ __forceinline__ void leaf_run(double *__restrict__ A, long lda, double *__restrict__ W, long ldw, int n,
                                         int *__restrict__ bad, LeafLds &sm) {
    constexpr int L = kLeaf, LP = kLP, PER = kLeafPer;
    static_assert(PER * 4 == L && L * 4 == kLeafThreads, "four threads per row");
    double *ls = sm.ls;
    double(*vec)[2 * L] = sm.vec;
    double *piv_in = sm.piv_in;
    double *rdiag = sm.rdiag;
    const int t = threadIdx.x, ri = t >> 2, part = t & 3;
    double r[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int j = 4 * m + part;
        r[m] = ri < n ? (j <= ri ? A[(long)ri * lda + j] : 0.0) : (j == ri ? 1.0 : 0.0);
    }
    for (int e = t; e < 2 * L; e += kLeafThreads) vec[0][e] = vec[1][e] = 0.0;
    __syncthreads();
    if (part == 0) {
        vec[0][ri] = ri > 0 ? r[0] : 0.0;
        if (ri == 0) piv_in[0] = r[0];
    }
#pragma unroll 1
    for (int c = 0; c < PER; ++c) {
#pragma unroll
        for (int pk = 0; pk < 4; ++pk) {
            const int k = 4 * c + pk;
            const double *col = vec[pk & 1];
            const double *colj = col + 4 * c + part;   // colj[4 m] = a[4 (c + m) + part][k]
            __syncthreads();
            const double d = piv_in[pk & 1], cri = col[ri];
            double cj[PER];
#pragma unroll
            for (int m = 0; m < PER; ++m) cj[m] = colj[4 * m];
            const double ip = rsqrt_f64(d), piv = d * ip, invd = ip * ip;
            const double lik = cri * invd;
            const int m1 = (pk + 1) / 4, p1 = (pk + 1) % 4;   // column k + 1
            r[m1] = fma(-lik, cj[m1], r[m1]);
            if (part == p1 && k + 1 < L) {
                vec[(pk + 1) & 1][ri] = ri > k + 1 ? r[m1] : 0.0;
                if (ri == k + 1) piv_in[(pk + 1) & 1] = r[m1];
            }
#pragma unroll
            for (int m = 0; m < PER; ++m)
                if (m != m1) r[m] = fma(-lik, cj[m], r[m]);
            r[0] = part == pk ? (ri == k ? piv : r[0] * ip) : r[0];
            if (t == 0) {
                rdiag[k] = ip;
                if (!(d > 0.0)) *bad = 1;
            }
        }
        const int j = 4 * c + part;
        ls[ri * LP + j] = j <= ri ? r[0] : 0.0;
#pragma unroll
        for (int m = 0; m + 1 < PER; ++m) r[m] = r[m + 1];
        r[PER - 1] = 0.0;
    }
    __syncthreads();
    for (int e = t; e < L * L; e += kLeafThreads) {   // rows of L, coalesced
        const int i = e / L, j = e % L;
        if (i < n && j <= i) A[(long)i * lda + j] = ls[i * LP + j];
    }
    double w[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) w[m] = 4 * m + part == ri ? 1.0 : 0.0;
    if (ri == 0) {
#pragma unroll
        for (int m = 0; m < PER; ++m) vec[0][4 * m + part] = w[m];
    }
    double lq = ls[ri * LP] * rdiag[0];   // L[i][k] / L[k][k] for k = 0
#pragma unroll 2
    for (int k = 0; k < L; ++k) {
        const double *row = vec[k & 1];
        const double ik = rdiag[k];
        const double lq_next = k + 1 < L ? ls[ri * LP + k + 1] * rdiag[k + 1] : 0.0;
        __syncthreads();
        if (ri == k) {
#pragma unroll
            for (int m = 0; m < PER; ++m) w[m] *= ik;
        } else if (ri > k) {
#pragma unroll
            for (int m = 0; m < PER; ++m) w[m] -= lq * row[4 * m + part];
            if (ri == k + 1) {
#pragma unroll
                for (int m = 0; m < PER; ++m) vec[(k + 1) & 1][4 * m + part] = w[m];
            }
        }
        lq = lq_next;
    }
    __syncthreads();   // every read of the factor in ls is done
#pragma unroll
    for (int m = 0; m < PER; ++m) ls[ri * LP + 4 * m + part] = w[m];
    __syncthreads();
    for (int e = t; e < L * L; e += kLeafThreads) {   // W, zeros above the diagonal
        const int i = e / L, j = e % L;
        if (i < n && j < n) W[(long)i * ldw + j] = j <= i ? ls[i * LP + j] : 0.0;
    }
}

__global__ __launch_bounds__(kLeafThreads) void k_chol_leaf(double *__restrict__ A, long lda, double *__restrict__ W,
                                                            long ldw, int n, int *__restrict__ bad) {
    __shared__ LeafLds sm;
    leaf_run(A, lda, W, ldw, n, bad, sm);
}

// C = X Y^T for 64 x 64 tiles in LDS (row stride kLP): C[i][j] = sum_k
// X(i, k) Y[j][k], with X(i, k) = X[i][k], or X[k][i] when XT.  Wave w of
// four takes the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 FP64 MFMA blocks;
// out(i, j, v) receives each result.
template <bool XT, class Out>
__device__ __forceinline__ void mm64(const double *__restrict__ X, const double *__restrict__ Y, Out out) {
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
    const int r = lane % 16, kq = lane / 16;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < kLeaf; k0 += 4) {
        const int k = k0 + kq;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = XT ? X[k * kLP + wm + 16 * i + r] : X[(wm + 16 * i + r) * kLP + k];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Y[(wn + 16 * j + r) * kLP + k];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // result D[row l/16 + 4q][col l%16] in acc[q]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) out(wm + 16 * i + kq + 4 * q, wn + 16 * j + r, acc[i][j][q]);
}

// One node of the recursion with n1 = kLeaf, n2 = n - kLeaf <= kLeaf, in one
// workgroup: the leaf of A11, L21 = A21 W11^T, A22 -= L21 L21^T, the leaf of
// A22, then W21 = -W22 (L21 W11), formed as -W22 (W11^T L21^T)^T.  The same
// steps as the recursion below a node of this size, without its launches.
__global__ __launch_bounds__(kLeafThreads) void k_chol_node(double *__restrict__ A, long lda, double *__restrict__ W,
                                                            long ldw, int n, int *__restrict__ bad) {
    constexpr int L = kLeaf, LP = kLP;
    __shared__ LeafLds sm;
    __shared__ double Wb[L * LP];   // W11
    __shared__ double Xb[L * LP];   // A21, then L21
    __shared__ double Tb[L * LP];   // S^T = (L21 W11)^T
    const int t = threadIdx.x, n2 = n - L;
    double *A21 = A + (long)L * lda, *A22 = A21 + L, *W21 = W + (long)L * ldw, *W22 = W21 + L;
    leaf_run(A, lda, W, ldw, L, bad, sm);
    for (int e = t; e < L * L; e += kLeafThreads) {
        const int i = e / L, j = e % L;
        Wb[i * LP + j] = sm.ls[i * LP + j];
        Xb[i * LP + j] = i < n2 ? A21[(long)i * lda + j] : 0.0;
    }
    __syncthreads();
    // L21 = A21 W11^T, kept in registers until every wave has read A21
    double l21[16];
    int li[16], lj[16], nl = 0;
    mm64<false>(Xb, Wb, [&](int i, int j, double v) {
        li[nl] = i;
        lj[nl] = j;
        l21[nl++] = v;
    });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        Xb[li[q] * LP + lj[q]] = l21[q];
        if (li[q] < n2) A21[(long)li[q] * lda + lj[q]] = l21[q];
    }
    __syncthreads();
    // A22 -= L21 L21^T on and below the diagonal
    mm64<false>(Xb, Xb, [&](int i, int j, double v) {
        if (i < n2 && j <= i) A22[(long)i * lda + j] -= v;
    });
    __syncthreads();
    leaf_run(A22, lda, W22, ldw, n2, bad, sm);
    // S^T = W11^T L21^T
    mm64<true>(Wb, Xb, [&](int i, int j, double v) { Tb[i * LP + j] = v; });
    __syncthreads();
    // W21 = -W22 S
    mm64<false>(sm.ls, Tb, [&](int i, int j, double v) {
        if (i < n2) W21[(long)i * ldw + j] = -v;
    });
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
        hipLaunchKernelGGL(k_chol_leaf, dim3(1), dim3(kLeafThreads), 0, st, A, lda, W, ldw, n, bad);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    if (n <= 2 * kLeaf) {
        ProfScope ps(ctx, "k_chol_node", st);
        hipLaunchKernelGGL(k_chol_node, dim3(1), dim3(kLeafThreads), 0, st, A, lda, W, ldw, n, bad);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    const int n1 = kLeaf * ((n + 2 * kLeaf - 1) / (2 * kLeaf)), n2 = n - n1;
    double *A21 = A + (long)n1 * lda, *A22 = A21 + n1, *W21 = W + (long)n1 * ldw, *W22 = W21 + n1;
    if ((rc = chol_rec(ctx, n1, A, lda, W, ldw, S, bad, st))) return rc;
    {
        ProfScope ps(ctx, "k_gemm_f64", st);
        // S = L21 = A21 W11^T, copied over A21
        if ((rc = gemm_f64(n2, n1, n1, 1.0, A21, lda, W, ldw, true, 0.0, S, n1, false, kTriBtLower, st)))
            return rc;
        hipLaunchKernelGGL(k_copy2d, dim3(nblk256((long)n2 * n1)), dim3(256), 0, st, S, (long)n1, A21, lda, n2, n1);
        LGF_HIP(hipGetLastError());
        // A22 -= L21 L21^T (tiles on and below the diagonal)
        if ((rc = gemm_f64(n2, n2, n1, -1.0, A21, lda, A21, lda, true, 1.0, A22, lda, true, kTriNone, st)))
            return rc;
    }
    if ((rc = chol_rec(ctx, n2, A22, lda, W22, ldw, S, bad, st))) return rc;
    {
        ProfScope ps(ctx, "k_gemm_f64", st);
        // W21 = -W22 (L21 W11)
        if ((rc = gemm_f64(n2, n1, n1, 1.0, A21, lda, W, ldw, false, 0.0, S, n1, false, kTriBLower, st)))
            return rc;
        if ((rc = gemm_f64(n2, n1, n2, -1.0, W22, ldw, S, n1, false, 0.0, W21, ldw, false, kTriALower, st)))
            return rc;
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
    // unrolled twice so that eight loads per lane are in flight (the
    // accumulation order is that of the plain loop)
#pragma unroll 2
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
        // (unrolling this loop twice measured slower: 0.065 -> 0.069 ms for
        // the three solve kernels at 6600 unknowns)
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

// the partial sums added in chunk order; a compile-time count lets every
// load be issued before the first add
__global__ void k_sum_parts(const double *__restrict__ part, double *__restrict__ x, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double v[kColChunks];
#pragma unroll
    for (int r = 0; r < kColChunks; ++r) v[r] = part[(long)r * n + j];
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kColChunks; ++r) s += v[r];
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
        hipLaunchKernelGGL(k_sum_parts, dim3((n + 255) / 256), dim3(256), 0, st, part, x, n);
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
