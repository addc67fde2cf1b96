// multilevel.hip -- multilevel interpolation evaluator of the lattice
// convolution u = dx^2 G * f (Sec. 2.2, Eq. dpoisson_conv), FP64.
//
// The paper evaluates these convolutions with a kernel-independent,
// interpolation-based multipole method on the block grid and gives no steps;
// the method here is a block tree with p^3 lattice nodes per cluster:
//
//   P2M   per source block: node charges M_a = sum_cells S_a(x) f(x), S_a the
//         tensor Lagrange basis of the block's nodes;
//   M2M   per parent cluster: M_a = sum over children and their nodes of the
//         parent's basis at the child node times the child's charge;
//   M2L   per pair of clusters (target c, source s) on a level's interaction
//         list: Phi_b(c) += sum_a G(y_b - x_a) M_a(s); the pairs are grouped
//         by the displacement D = c - s, and each group is a GEMM of its
//         p^3 x p^3 node matrix with the gathered charges on the matrix
//         cores, tiles of 128 pairs added atomically into Phi (one target
//         receives several displacements);
//   L2L   per target cluster below the top: Phi(c) = parent's Phi
//         interpolated at c's nodes (a plain store that precedes M2L);
//   leaf  per target block: L2P (Phi interpolated at the cells) plus the exact
//         sum over the neighbouring source blocks.  For B = 8 that sum runs on
//         the matrix cores, one 512 x 512 matrix per neighbour displacement
//         (k_ml_pairs_mfma below); for B = 4 in the leaf kernel, the kernel's
//         2B x 2B x 2B corner held in LDS, one thread owning one x-row of B
//         target cells (B^2 FMAs per 3B/2 loads).
//
// Interaction lists: at the top level every non-neighbour pair; below it the
// children of the parent's neighbours (and the parent) that are not
// neighbours.  Every block pair is counted once, at the finest level where
// the two are apart, or in the leaf sum if they are neighbours.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "conv_common.h"
#include "internal.h"

namespace lgfib {
namespace {

constexpr int kTopSpan = 4;   // top level: at most this many clusters per axis
constexpr int kNearTile = 128;   // pairs (and output columns) per MFMA tile
constexpr int kNearKT = 32;      // contraction terms staged in LDS per step

struct CKey {
    int32_t x, y, z;
    bool operator==(const CKey &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct CKeyHash {
    size_t operator()(const CKey &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int32_t v : {k.x, k.y, k.z}) {
            h ^= (uint32_t)v;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};
using CMap = std::unordered_map<CKey, int, CKeyHash>;

inline CKey parent_of(const CKey &c) { return {c.x >> 1, c.y >> 1, c.z >> 1}; }   // floor(c / 2)
inline int octant_of(const CKey &c) { return (c.x & 1) | ((c.y & 1) << 1) | ((c.z & 1) << 2); }
inline bool adjacent(const CKey &a, const CKey &b) {
    return std::abs(a.x - b.x) <= 1 && std::abs(a.y - b.y) <= 1 && std::abs(a.z - b.z) <= 1;
}

// rounded Chebyshev nodes of a cluster side of L cells (empty if two coincide)
std::vector<int> cluster_nodes(int L, int p) {
    std::vector<int> t(p);
    for (int j = 0; j < p; ++j)
        t[j] = (int)std::floor((L - 1) / 2.0 * (1.0 - std::cos(M_PI * (2 * j + 1) / (2.0 * p))) + 0.5);
    for (int j = 1; j < p; ++j)
        if (t[j] <= t[j - 1]) return {};
    return t;
}

double lagrange(const std::vector<int> &t, int j, double x) {
    double w = 1.0;
    for (int k = 0; k < (int)t.size(); ++k)
        if (k != j) w *= (x - t[k]) / (double)(t[j] - t[k]);
    return w;
}

// ---------------------------------------------------------------- kernels

template <int P, int B>
__global__ __launch_bounds__(256) void k_ml_p2m(const double *__restrict__ f, const double *__restrict__ W0,
                                                 double *__restrict__ M) {
    constexpr int P3 = P * P * P, B3 = B * B * B;
    __shared__ double fs[B3];
    __shared__ double w[P * B];
    const int s = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = threadIdx.x; i < B3; i += blockDim.x) fs[i] = f[(size_t)s * B3 + i];
    for (int i = threadIdx.x; i < P * B; i += blockDim.x) w[i] = W0[i];
    __syncthreads();
    const int a = threadIdx.x;
    if (a >= P3) return;
    const int ax = a % P, ay = (a / P) % P, az = a / (P * P);
    double acc = 0.0;
    for (int z = 0; z < B; ++z)
        for (int y = 0; y < B; ++y) {
            const double wzy = w[az * B + z] * w[ay * B + y];
            double r = 0.0;
#pragma unroll
            for (int x = 0; x < B; ++x) r += w[ax * B + x] * fs[(z * B + y) * B + x];
            acc += wzy * r;
        }
    M[(size_t)s * P3 + a] = acc;
}

// Wup: [2][P][P], Wup[o][j][k] = basis j of the parent at node k of a child
// whose offset in the parent is o (0 or 1) child sides.
template <int P>
__global__ __launch_bounds__(256) void k_ml_m2m(const double *__restrict__ Mc, const int *__restrict__ kids,
                                                 const double *__restrict__ Wup, double *__restrict__ Mp) {
    constexpr int P3 = P * P * P;
    __shared__ double w[2 * P * P];
    __shared__ double mc[8 * P3];
    const int c = xcd_remap(blockIdx.x, gridDim.x);
    for (int i = threadIdx.x; i < 2 * P * P; i += blockDim.x) w[i] = Wup[i];
    for (int i = threadIdx.x; i < 8 * P3; i += blockDim.x) {
        const int k = kids[c * 8 + i / P3];
        mc[i] = k >= 0 ? Mc[(size_t)k * P3 + i % P3] : 0.0;
    }
    __syncthreads();
    const int a = threadIdx.x;
    if (a >= P3) return;
    const int ax = a % P, ay = (a / P) % P, az = a / (P * P);
    double acc = 0.0;
    for (int o = 0; o < 8; ++o) {
        if (kids[c * 8 + o] < 0) continue;
        const double *wx = w + (o & 1) * P * P + ax * P;
        const double *wy = w + ((o >> 1) & 1) * P * P + ay * P;
        const double *wz = w + (o >> 2) * P * P + az * P;
        const double *m = mc + o * P3;
        for (int kz = 0; kz < P; ++kz)
            for (int ky = 0; ky < P; ++ky) {
                const double wzy = wz[kz] * wy[ky];
                double r = 0.0;
#pragma unroll
                for (int kx = 0; kx < P; ++kx) r += wx[kx] * m[(kz * P + ky) * P + kx];
                acc += wzy * r;
            }
    }
    Mp[(size_t)c * P3 + a] = acc;
}

template <int P>
__global__ __launch_bounds__(256) void k_ml_l2l(const double *__restrict__ Phip, const int *__restrict__ par,
                                                 const double *__restrict__ Wup, double *__restrict__ Phi) {
    constexpr int P3 = P * P * P;
    __shared__ double w[2 * P * P];
    __shared__ double pp[P3];
    const int c = xcd_remap(blockIdx.x, gridDim.x);
    const int pr = par[2 * c], o = par[2 * c + 1];
    for (int i = threadIdx.x; i < 2 * P * P; i += blockDim.x) w[i] = Wup[i];
    for (int i = threadIdx.x; i < P3; i += blockDim.x) pp[i] = Phip[(size_t)pr * P3 + i];
    __syncthreads();
    const int b = threadIdx.x;
    if (b >= P3) return;
    const int bx = b % P, by = (b / P) % P, bz = b / (P * P);
    const double *wx = w + (o & 1) * P * P;
    const double *wy = w + ((o >> 1) & 1) * P * P;
    const double *wz = w + (o >> 2) * P * P;
    double acc = 0.0;
    for (int kz = 0; kz < P; ++kz)
        for (int ky = 0; ky < P; ++ky) {
            const double wzy = wz[kz * P + bz] * wy[ky * P + by];
            double r = 0.0;
#pragma unroll
            for (int kx = 0; kx < P; ++kx) r += wx[kx * P + bx] * pp[(kz * P + ky) * P + kx];
            acc += wzy * r;
        }
    Phi[(size_t)c * P3 + b] = acc;
}

template <int P, typename R>
__global__ __launch_bounds__(256) void k_ml_kmat(const double *__restrict__ tab, int e1, int e2,
                                                  const int4 *__restrict__ dinfo, const int *__restrict__ nodes,
                                                  R *__restrict__ K) {
    constexpr int P3 = P * P * P;
    const int d = blockIdx.x;
    const int4 in = dinfo[d];
    const int *t = nodes + in.w * P;
    for (int i = threadIdx.x; i < P3 * P3; i += blockDim.x) {
        const int b = i / P3, a = i % P3;   // target node b, source node a
        const int ox = abs(in.x + t[b % P] - t[a % P]);
        const int oy = abs(in.y + t[(b / P) % P] - t[(a / P) % P]);
        const int oz = abs(in.z + t[b / (P * P)] - t[a / (P * P)]);
        K[(size_t)d * P3 * P3 + i] = (R)tab[((size_t)oz * (e2 + 1) + oy) * (e1 + 1) + ox];
    }
}

__global__ void k_ml_zero(double *__restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// exact sum of one neighbouring source block into a row of B target cells;
// DX = source block x - target block x, so the x offsets are compile-time
template <int B, int DX>
__device__ __forceinline__ void near_rows(const double *__restrict__ fs, const double *g, int ty, int tz, int DY,
                                          int DZ, double (&acc)[B]) {
    constexpr int G2 = 2 * B;
    for (int sz = 0; sz < B; ++sz) {
        const int dz = abs(tz - sz - B * DZ);
        for (int sy = 0; sy < B; ++sy) {
            const int dy = abs(ty - sy - B * DY);
            const double *gr = g + (dz * G2 + dy) * G2;
            double gv[G2], fv[B];
#pragma unroll
            for (int i = 0; i < G2; ++i) gv[i] = gr[i];
#pragma unroll
            for (int i = 0; i < B; ++i) fv[i] = fs[(sz * B + sy) * B + i];
#pragma unroll
            for (int tx = 0; tx < B; ++tx)
#pragma unroll
                for (int sx = 0; sx < B; ++sx) {
                    const int d = tx - sx - B * DX;
                    acc[tx] += gv[d < 0 ? -d : d] * fv[sx];
                }
        }
    }
}

// near: CSR over target blocks of int2 (source block, 9 (dz+1) + 3 (dy+1) + dx+1)
template <int P, int B, bool NEAR>
__global__ __launch_bounds__(256) void k_ml_leaf(const double *__restrict__ f, const double *__restrict__ tab, int e1,
                                                  int e2, int e3, const int *__restrict__ near_off,
                                                  const int2 *__restrict__ near_ent, const double *__restrict__ Phi0,
                                                  const double *__restrict__ W0, double scale, double *__restrict__ u,
                                                  int ntgt) {
    constexpr int P3 = P * P * P, B3 = B * B * B, R = B * B, TB = 256 / R, G2 = 2 * B;
    __shared__ double g[G2 * G2 * G2];
    __shared__ double w[P * B];
    __shared__ double ph[TB * P3];
    for (int i = threadIdx.x; i < G2 * G2 * G2; i += blockDim.x) {
        const int x = i % G2, y = (i / G2) % G2, z = i / (G2 * G2);
        g[i] = (x <= e1 && y <= e2 && z <= e3) ? tab[((size_t)z * (e2 + 1) + y) * (e1 + 1) + x] : 0.0;
    }
    for (int i = threadIdx.x; i < P * B; i += blockDim.x) w[i] = W0[i];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int lb = threadIdx.x / R;
    int t = wg * TB + lb;
    if (R % 64 == 0) t = __builtin_amdgcn_readfirstlane(t);
    const int row = threadIdx.x % R;
    if (t < ntgt)
        for (int i = row; i < P3; i += R) ph[lb * P3 + i] = Phi0[(size_t)t * P3 + i];
    __syncthreads();
    if (t >= ntgt) return;
    const int ty = row % B, tz = row / B;
    double acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = 0.0;
    const double *p = ph + lb * P3;
    for (int bz = 0; bz < P; ++bz)
        for (int by = 0; by < P; ++by) {
            const double wzy = w[bz * B + tz] * w[by * B + ty];
#pragma unroll
            for (int bx = 0; bx < P; ++bx) {
                const double c = wzy * p[(bz * P + by) * P + bx];
#pragma unroll
                for (int tx = 0; tx < B; ++tx) acc[tx] += c * w[bx * B + tx];
            }
        }
    const int e0 = NEAR ? near_off[t] : 0, e1n = NEAR ? near_off[t + 1] : 0;
    for (int e = e0; e < e1n; ++e) {
        const int2 en = near_ent[e];
        const double *fs = f + (size_t)en.x * B3;
        const int DX = en.y % 3 - 1, DY = (en.y / 3) % 3 - 1, DZ = en.y / 9 - 1;
        if (DX < 0) near_rows<B, -1>(fs, g, ty, tz, DY, DZ, acc);
        else if (DX == 0) near_rows<B, 0>(fs, g, ty, tz, DY, DZ, acc);
        else near_rows<B, 1>(fs, g, ty, tz, DY, DZ, acc);
    }
    double *ur = u + (size_t)t * B3 + (size_t)row * B;
#pragma unroll
    for (int tx = 0; tx < B; ++tx) ur[tx] = scale * acc[tx];
}

// ---- exact neighbour sum of 8^3 blocks on the matrix cores
//
// For a neighbour displacement D (source block - target block) the sum is a
// dense 512 x 512 matrix K_D[i][j] = G(x_i - y_j), i a target cell, j a source
// cell, applied to every pair with that displacement: the pairs of one D form
// a GEMM C[pair][i] = sum_j f[src(pair)][j] K_D[i][j] with gathered rows,
// whose tiles are added atomically into u (one target receives up to 27
// displacements, after the leaf kernel has stored its far-field part).

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename R>
__global__ __launch_bounds__(256) void k_ml_near_mats(const double *__restrict__ tab, int e1, int e2, int e3,
                                                       R *__restrict__ Kn) {
    const int code = blockIdx.y, i = blockIdx.x;
    const int DX = code % 3 - 1, DY = (code / 3) % 3 - 1, DZ = code / 9 - 1;
    const int tx = i & 7, ty = (i >> 3) & 7, tz = i >> 6;
    for (int j = threadIdx.x; j < 512; j += blockDim.x) {
        const int sx = j & 7, sy = (j >> 3) & 7, sz = j >> 6;
        const int dx = abs(tx - sx - 8 * DX), dy = abs(ty - sy - 8 * DY), dz = abs(tz - sz - 8 * DZ);
        Kn[((size_t)code * 512 + i) * 512 + j] =
            (R)((dx <= e1 && dy <= e2 && dz <= e3) ? tab[((size_t)dz * (e2 + 1) + dy) * (e1 + 1) + dx] : 0.0);
    }
}

// C[pair][n] = sum_k X[src(pair)][k] A_d[n][k] for the pairs of one task,
// added atomically into Y[tgt(pair)][n]: rows of X and Y hold KK and NCOL
// values, A_d is NCOL x KK.  tasks: int4 (matrix d, first pair, pair count
// <= 128, 0); grid (tasks, ceil(NCOL / TN)), TN = 64 for NCOL <= 64, else
// 128.  Four waves, each a 64 x 64 (TN = 128) or 32 x 64 (TN = 64) block of
// the tile as v_mfma_f64_16x16x4f64 products; columns past NCOL and
// contraction terms past KK are zero-filled.
// Serves the neighbour sum of 8^3 blocks (KK = NCOL = 512, A_d the cell
// kernel of a displacement) and M2L (KK = NCOL = p^3, A_d the node kernel).
// R is the product's precision: double (v_mfma_f64_16x16x4f64), or float
// (v_mfma_f32_16x16x4f32, FP32 matrix and rounded X, FP32 accumulation)
// on request; Y is FP64 either way.
template <int KK, int NCOL, typename R>
__global__ __launch_bounds__(256) void k_ml_pairs_mfma(const int4 *__restrict__ tasks, const int2 *__restrict__ pairs,
                                                        const double *__restrict__ X, const R *__restrict__ Amat,
                                                        double *__restrict__ Y, double scale) {
    constexpr bool F64 = std::is_same<R, double>::value;
    using acc_t = typename std::conditional<F64, f64x4, f32x4>::type;
    // tiles of 128 pairs x TN columns; with TN = 64 each wave takes 32 x 64
    constexpr int T = kNearTile, TN = NCOL <= 64 ? 64 : 128, KT = kNearKT;
    constexpr int FMR = TN == 64 ? 2 : 4, FMC = 4, PA = T * KT / 256, PB = TN * KT / 256;
    constexpr int KP = (KK + KT - 1) / KT * KT;
    __shared__ R As[T][KT + 1];    // [pair][k]
    __shared__ R Bs[TN][KT + 1];   // [n][k]
    __shared__ int srow[T], trow[T];
    // consecutive tasks (mostly one displacement) on one XCD, so its L2 keeps
    // the matrix slab they share
    const int4 tk = tasks[xcd_remap(blockIdx.x, gridDim.x)];
    const int n0 = blockIdx.y * TN;
    const R *A = Amat + (size_t)tk.x * NCOL * KK;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int wm = TN == 64 ? wave * 32 : (wave / 2) * 64, wn = TN == 64 ? 0 : (wave % 2) * 64;
    for (int m = tid; m < T; m += 256) {
        const int2 pr = m < tk.z ? pairs[tk.y + m] : make_int2(-1, -1);
        trow[m] = pr.x;
        srow[m] = pr.y;
    }
    __syncthreads();
    acc_t acc[FMR][FMC];
#pragma unroll
    for (int i = 0; i < FMR; ++i)
#pragma unroll
        for (int j = 0; j < FMC; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    R ra[PA], rb[PB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int e = tid + 256 * q, k = k0 + e % KT;
            const int sr = srow[e / KT];
            ra[q] = (sr >= 0 && k < KK) ? (R)X[(size_t)sr * KK + k] : (R)0;
        }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int e = tid + 256 * q, k = k0 + e % KT, n = n0 + e / KT;
            rb[q] = (n < NCOL && k < KK) ? A[(size_t)n * KK + k] : (R)0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int q = 0; q < PA; ++q) {
            const int e = tid + 256 * q;
            As[e / KT][e % KT] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int e = tid + 256 * q;
            Bs[e / KT][e % KT] = rb[q];
        }
    };
    fetch(0);
    stage();
    __syncthreads();
    // v_mfma_f64_16x16x4f64: lane l holds A[row l%16][k l/16] and B[k l/16][col
    // l%16]; the result D[row l/16 + 4q][col l%16] lands in acc[q]
    const int r = lane % 16, kq = lane / 16;
    for (int k0 = 0; k0 < KP; k0 += KT) {
        const bool more = k0 + KT < KP;
        if (more) fetch(k0 + KT);
#pragma unroll
        for (int ks = 0; ks < KT; ks += 4) {
            R a[FMR], b[FMC];
#pragma unroll
            for (int i = 0; i < FMR; ++i) a[i] = As[wm + 16 * i + r][ks + kq];
#pragma unroll
            for (int j = 0; j < FMC; ++j) b[j] = Bs[wn + 16 * j + r][ks + kq];
#pragma unroll
            for (int i = 0; i < FMR; ++i)
#pragma unroll
                for (int j = 0; j < FMC; ++j) {
                    if constexpr (F64)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
        if (more) {
            stage();
            __syncthreads();
        }
    }
    const int c = lane % 16, rq = lane / 16;
#pragma unroll
    for (int i = 0; i < FMR; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // result row of acc[q]: l/16 + 4q for the FP64 form, 4(l/16) + q for FP32
            const int t = trow[wm + 16 * i + (F64 ? rq + 4 * q : 4 * rq + q)];
            if (t < 0) continue;
#pragma unroll
            for (int j = 0; j < FMC; ++j) {
                const int n = n0 + wn + 16 * j + c;
                if (n < NCOL) unsafeAtomicAdd(&Y[(size_t)t * NCOL + n], scale * (double)acc[i][j][q]);
            }
        }
}

}  // namespace
}  // namespace lgfib

using namespace lgfib;

struct lgf_ml {
    lgfib_ctx *ctx = nullptr;
    int device = 0;   // the context's device (destroy does not touch ctx)
    lgf_table_t tbl = -1;
    int B = 0, P = 0, top = 0, nsrc = 0, ntgt = 0;
    std::vector<int> ns, nt;            // clusters per level
    std::vector<size_t> m_off, t_off;   // first cluster of each level in M / Phi
    std::vector<size_t> kid_off;        // first parent row of each level's M2M map
    std::vector<int> task_off, ntask;   // M2L tasks per level
    int64_t npairs = 0, nnear = 0, nd = 0;
    DevBuf W0, Wup, kids, par, tasks, pairs, K, near_off, near_ent, M, Phi, dinfo, nodes;
    int nntask = 0;                     // B = 8: neighbour pairs on the matrix cores
    int pair_prec = LGF_F64;            // precision of the pair products (M2L, neighbour sums)
    DevBuf nbr_tasks, nbr_pairs, Kn;
};

namespace {

template <int P, int B>
int ml_run(lgf_ml *pl, int ncomp, double dx, const double *f, double *u, hipStream_t st) {
    constexpr int P3 = P * P * P, B3 = B * B * B, TB = 256 / (B * B);
    lgfib_ctx *ctx = pl->ctx;
    const Table &tb = *ctx->tables[pl->tbl];
    double *M = pl->M.as<double>(), *Phi = pl->Phi.as<double>();
    const double *Wup = pl->Wup.as<double>();
    for (int c = 0; c < ncomp; ++c) {
        const double *fc = f + (size_t)c * pl->nsrc * B3;
        double *uc = u + (size_t)c * pl->ntgt * B3;
        {
            ProfScope ps(ctx, "k_ml_p2m", st);
            hipLaunchKernelGGL((k_ml_p2m<P, B>), dim3(pl->nsrc), dim3(256), 0, st, fc, pl->W0.as<double>(), M);
            LGF_HIP(hipGetLastError());
        }
        for (int l = 0; l < pl->top; ++l) {
            ProfScope ps(ctx, "k_ml_m2m", st);
            hipLaunchKernelGGL((k_ml_m2m<P>), dim3(pl->ns[l + 1]), dim3(P3 <= 128 ? 128 : 256), 0, st, M + pl->m_off[l] * P3,
                               pl->kids.as<int>() + pl->kid_off[l] * 8, Wup + (size_t)l * 2 * P * P,
                               M + pl->m_off[l + 1] * P3);
            LGF_HIP(hipGetLastError());
        }
        for (int l = pl->top; l >= 0; --l) {
            double *Phl = Phi + pl->t_off[l] * P3;
            if (l == pl->top) {
                const size_t n = (size_t)pl->nt[l] * P3;
                hipLaunchKernelGGL(k_ml_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Phl, n);
            } else {
                ProfScope ps(ctx, "k_ml_l2l", st);
                hipLaunchKernelGGL((k_ml_l2l<P>), dim3(pl->nt[l]), dim3(P3 <= 128 ? 128 : 256), 0, st, Phi + pl->t_off[l + 1] * P3,
                                   pl->par.as<int>() + 2 * pl->t_off[l], Wup + (size_t)l * 2 * P * P, Phl);
            }
            LGF_HIP(hipGetLastError());
            if (pl->ntask[l] > 0) {
                ProfScope ps(ctx, "k_ml_m2l", st);
                constexpr int ytiles = P3 <= 64 ? 1 : (P3 + 127) / 128;   // the kernel's column tiles
                if (pl->pair_prec == LGF_F64)
                    hipLaunchKernelGGL((k_ml_pairs_mfma<P3, P3, double>), dim3(pl->ntask[l], ytiles), dim3(256), 0,
                                       st, pl->tasks.as<int4>() + pl->task_off[l], pl->pairs.as<int2>(),
                                       M + pl->m_off[l] * P3, pl->K.as<double>(), Phl, 1.0);
                else
                    hipLaunchKernelGGL((k_ml_pairs_mfma<P3, P3, float>), dim3(pl->ntask[l], ytiles), dim3(256), 0,
                                       st, pl->tasks.as<int4>() + pl->task_off[l], pl->pairs.as<int2>(),
                                       M + pl->m_off[l] * P3, pl->K.as<float>(), Phl, 1.0);
                LGF_HIP(hipGetLastError());
            }
        }
        {
            ProfScope ps(ctx, "k_ml_leaf", st);
            hipLaunchKernelGGL((k_ml_leaf<P, B, B != 8>), dim3((pl->ntgt + TB - 1) / TB), dim3(256), 0, st, fc,
                               tb.g.as<double>(), tb.ext[0], tb.ext[1], tb.ext[2], pl->near_off.as<int>(),
                               pl->near_ent.as<int2>(), Phi, pl->W0.as<double>(), dx * dx, uc, pl->ntgt);
            LGF_HIP(hipGetLastError());
        }
        if (B == 8 && pl->nntask > 0) {
            ProfScope ps(ctx, "k_ml_near_mfma", st);
            if (pl->pair_prec == LGF_F64)
                hipLaunchKernelGGL((k_ml_pairs_mfma<512, 512, double>), dim3(pl->nntask, 512 / kNearTile), dim3(256),
                                   0, st, pl->nbr_tasks.as<int4>(), pl->nbr_pairs.as<int2>(), fc, pl->Kn.as<double>(),
                                   uc, dx * dx);
            else
                hipLaunchKernelGGL((k_ml_pairs_mfma<512, 512, float>), dim3(pl->nntask, 512 / kNearTile), dim3(256),
                                   0, st, pl->nbr_tasks.as<int4>(), pl->nbr_pairs.as<int2>(), fc, pl->Kn.as<float>(),
                                   uc, dx * dx);
            LGF_HIP(hipGetLastError());
        }
    }
    return LGFIB_OK;
}

template <typename T> int upload(DevBuf &d, const std::vector<T> &v) {
    if (v.empty()) return LGFIB_OK;
    int rc = d.reserve(v.size() * sizeof(T));
    if (rc) return rc;
    LGF_HIP(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return LGFIB_OK;
}

}  // namespace

extern "C" int lgf_ml_create(lgfib_ctx *ctx, lgf_table_t tbl, int B, int p, int pair_prec, const int32_t *src_blocks,
                             int nsrc, const int32_t *tgt_blocks, int ntgt, lgfib_stream_t stream, lgf_ml_t **out) {
    if (!out) return fail(LGFIB_EINVAL, "lgf_ml_create: null output");
    *out = nullptr;
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_ml_create: null context");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_ml_create: unknown table");
    if (B != 4 && B != 8) return fail(LGFIB_EINVAL, "lgf_ml_create: B must be 4 or 8");
    if (p < 4 || p > 6 || p > B) return fail(LGFIB_EINVAL, "lgf_ml_create: p must be 4, 5 or 6 and at most B");
    if (pair_prec != LGF_F64 && (pair_prec != LGF_F32 || B != 8))
        return fail(LGFIB_EINVAL, "lgf_ml_create: pair_prec must be LGF_F64, or LGF_F32 with B = 8");
    int rc;
    if ((rc = validate_blocks(src_blocks, nsrc, "lgf_ml_create: source blocks"))) return rc;
    if ((rc = validate_blocks(tgt_blocks, ntgt, "lgf_ml_create: target blocks"))) return rc;
    LGF_HIP(hipSetDevice(ctx->device));
    auto pl = std::make_unique<lgf_ml>();
    pl->ctx = ctx;
    pl->device = ctx->device;
    pl->tbl = tbl;
    pl->B = B;
    pl->P = p;
    pl->pair_prec = pair_prec;
    pl->nsrc = nsrc;
    pl->ntgt = ntgt;
    if (nsrc == 0 || ntgt == 0) {
        *out = pl.release();
        return LGFIB_OK;
    }
    const Table &tb = *ctx->tables[tbl];
    // top level and the table reach
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = src_blocks[a];
    for (int i = 0; i < nsrc + ntgt; ++i) {
        const int32_t *b = i < nsrc ? src_blocks + 3 * i : tgt_blocks + 3 * (i - nsrc);
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b[a]);
            hi[a] = std::max(hi[a], b[a]);
        }
    }
    int top = 0;
    for (;;) {
        bool ok = true;
        for (int a = 0; a < 3; ++a) ok = ok && (hi[a] >> top) - (lo[a] >> top) + 1 <= kTopSpan;
        if (ok) break;
        ++top;
    }
    for (int a = 0; a < 3; ++a) {
        const long need = (long)((hi[a] >> top) - (lo[a] >> top) + 1) * ((long)B << top) - 1;
        if (need > tb.ext[a])
            return fail(LGFIB_ERANGE, "lgf_ml_create: table extent " + std::to_string(tb.ext[a]) + " on axis " +
                                          std::to_string(a) + " is short of " + std::to_string(need));
    }
    pl->top = top;
    std::vector<std::vector<int>> nodes(top + 1);
    for (int l = 0; l <= top; ++l) {
        nodes[l] = cluster_nodes(B << l, p);
        if (nodes[l].empty()) return fail(LGFIB_EINVAL, "lgf_ml_create: interpolation nodes coincide");
    }
    // clusters per level
    std::vector<std::vector<CKey>> sc(top + 1), tc(top + 1);
    std::vector<CMap> smap(top + 1), tmap(top + 1);
    for (int i = 0; i < nsrc; ++i) {
        CKey k{src_blocks[3 * i], src_blocks[3 * i + 1], src_blocks[3 * i + 2]};
        smap[0][k] = i;
        sc[0].push_back(k);
    }
    for (int i = 0; i < ntgt; ++i) {
        CKey k{tgt_blocks[3 * i], tgt_blocks[3 * i + 1], tgt_blocks[3 * i + 2]};
        tmap[0][k] = i;
        tc[0].push_back(k);
    }
    std::vector<int32_t> kids, par;
    for (int l = 0; l < top; ++l) {
        for (const CKey &c : sc[l]) {
            const CKey q = parent_of(c);
            if (smap[l + 1].emplace(q, (int)sc[l + 1].size()).second) sc[l + 1].push_back(q);
        }
        const size_t k0 = kids.size();
        kids.resize(k0 + 8 * sc[l + 1].size(), -1);
        for (size_t i = 0; i < sc[l].size(); ++i)
            kids[k0 + 8 * (size_t)smap[l + 1][parent_of(sc[l][i])] + octant_of(sc[l][i])] = (int32_t)i;
        for (const CKey &c : tc[l]) {
            const CKey q = parent_of(c);
            if (tmap[l + 1].emplace(q, (int)tc[l + 1].size()).second) tc[l + 1].push_back(q);
        }
    }
    for (int l = 0; l <= top; ++l) {   // parent map of the targets (unused at the top)
        for (const CKey &c : tc[l]) {
            par.push_back(l < top ? tmap[l + 1][parent_of(c)] : -1);
            par.push_back(octant_of(c));
        }
    }
    size_t ms = 0, ts = 0, ks = 0;
    for (int l = 0; l <= top; ++l) {
        pl->ns.push_back((int)sc[l].size());
        pl->nt.push_back((int)tc[l].size());
        pl->m_off.push_back(ms);
        pl->t_off.push_back(ts);
        pl->kid_off.push_back(ks);
        ms += sc[l].size();
        ts += tc[l].size();
        if (l < top) ks += sc[l + 1].size();
    }
    // interaction lists, grouped by displacement
    std::vector<int32_t> tasks, pairs;
    std::vector<int32_t> dinfo;
    for (int l = 0; l <= top; ++l) {
        std::vector<std::vector<int32_t>> byd(343);
        auto add = [&](int ti, int si, const CKey &c, const CKey &s) {
            const int Dx = c.x - s.x, Dy = c.y - s.y, Dz = c.z - s.z;
            auto &v = byd[(Dz + 3) * 49 + (Dy + 3) * 7 + Dx + 3];
            v.push_back(ti);
            v.push_back(si);
        };
        for (int ti = 0; ti < (int)tc[l].size(); ++ti) {
            const CKey c = tc[l][ti];
            if (l == top) {
                for (int si = 0; si < (int)sc[l].size(); ++si)
                    if (!adjacent(sc[l][si], c)) add(ti, si, c, sc[l][si]);
                continue;
            }
            const CKey pc = parent_of(c);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const CKey q{pc.x + dx, pc.y + dy, pc.z + dz};
                        auto it = smap[l + 1].find(q);
                        if (it == smap[l + 1].end()) continue;
                        const int32_t *kk = kids.data() + pl->kid_off[l] * 8 + 8 * (size_t)it->second;
                        for (int o = 0; o < 8; ++o) {
                            if (kk[o] < 0) continue;
                            const CKey &s = sc[l][kk[o]];
                            if (!adjacent(s, c)) add(ti, kk[o], c, s);
                        }
                    }
        }
        pl->task_off.push_back((int)(tasks.size() / 4));
        for (int di = 0; di < 343; ++di) {
            const auto &v = byd[di];
            if (v.empty()) continue;
            const int Dx = di % 7 - 3, Dy = (di / 7) % 7 - 3, Dz = di / 49 - 3;
            const int L = B << l;
            const int d = (int)(dinfo.size() / 4);
            dinfo.insert(dinfo.end(), {Dx * L, Dy * L, Dz * L, l});
            const int np = (int)(v.size() / 2);
            for (int s0 = 0; s0 < np; s0 += kNearTile)
                tasks.insert(tasks.end(), {d, (int32_t)(pairs.size() / 2) + s0, std::min(kNearTile, np - s0), 0});
            pairs.insert(pairs.end(), v.begin(), v.end());
        }
        pl->ntask.push_back((int)(tasks.size() / 4) - pl->task_off.back());
    }
    pl->npairs = (int64_t)(pairs.size() / 2);
    pl->nd = (int64_t)(dinfo.size() / 4);
    // neighbour lists of the target blocks
    std::vector<int32_t> near_off(1, 0), near_ent;
    for (int ti = 0; ti < ntgt; ++ti) {
        const CKey c = tc[0][ti];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    auto it = smap[0].find(CKey{c.x + dx, c.y + dy, c.z + dz});
                    if (it == smap[0].end()) continue;
                    near_ent.push_back(it->second);
                    near_ent.push_back((dz + 1) * 9 + (dy + 1) * 3 + dx + 1);
                }
        near_off.push_back((int32_t)(near_ent.size() / 2));
    }
    pl->nnear = (int64_t)(near_ent.size() / 2);
    std::vector<int32_t> ntasks, npairs;
    if (B == 8) {
        std::vector<std::vector<int32_t>> byc(27);
        for (int ti = 0; ti < ntgt; ++ti)
            for (int e = near_off[ti]; e < near_off[ti + 1]; ++e) {
                byc[near_ent[2 * e + 1]].push_back(ti);
                byc[near_ent[2 * e + 1]].push_back(near_ent[2 * e]);
            }
        for (int code = 0; code < 27; ++code) {
            const int np = (int)(byc[code].size() / 2);
            for (int s0 = 0; s0 < np; s0 += kNearTile)
                ntasks.insert(ntasks.end(),
                              {code, (int32_t)(npairs.size() / 2) + s0, std::min(kNearTile, np - s0), 0});
            npairs.insert(npairs.end(), byc[code].begin(), byc[code].end());
        }
        pl->nntask = (int)(ntasks.size() / 4);
    }
    // interpolation weights
    std::vector<double> W0((size_t)p * B), Wup((size_t)std::max(top, 1) * 2 * p * p);
    for (int j = 0; j < p; ++j)
        for (int x = 0; x < B; ++x) W0[(size_t)j * B + x] = lagrange(nodes[0], j, x);
    for (int l = 0; l < top; ++l)
        for (int o = 0; o < 2; ++o)
            for (int j = 0; j < p; ++j)
                for (int k = 0; k < p; ++k)
                    Wup[(((size_t)l * 2 + o) * p + j) * p + k] =
                        lagrange(nodes[l + 1], j, (double)o * (B << l) + nodes[l][k]);
    std::vector<int32_t> nodes_flat;
    for (int l = 0; l <= top; ++l) nodes_flat.insert(nodes_flat.end(), nodes[l].begin(), nodes[l].end());
    const size_t P3 = (size_t)p * p * p;
    if ((rc = upload(pl->W0, W0)) || (rc = upload(pl->Wup, Wup)) || (rc = upload(pl->kids, kids)) ||
        (rc = upload(pl->par, par)) || (rc = upload(pl->tasks, tasks)) || (rc = upload(pl->pairs, pairs)) ||
        (rc = upload(pl->near_off, near_off)) || (rc = upload(pl->near_ent, near_ent)) ||
        (rc = upload(pl->dinfo, dinfo)) || (rc = upload(pl->nodes, nodes_flat)) ||
        (rc = upload(pl->nbr_tasks, ntasks)) || (rc = upload(pl->nbr_pairs, npairs)))
        return rc;
    if (pl->nntask > 0) {
        const bool f64 = pair_prec == LGF_F64;
        if ((rc = pl->Kn.reserve((size_t)27 * 512 * 512 * (f64 ? sizeof(double) : sizeof(float))))) return rc;
        if (f64)
            hipLaunchKernelGGL(k_ml_near_mats<double>, dim3(512, 27), dim3(256), 0, (hipStream_t)stream,
                               tb.g.as<double>(), tb.ext[0], tb.ext[1], tb.ext[2], pl->Kn.as<double>());
        else
            hipLaunchKernelGGL(k_ml_near_mats<float>, dim3(512, 27), dim3(256), 0, (hipStream_t)stream,
                               tb.g.as<double>(), tb.ext[0], tb.ext[1], tb.ext[2], pl->Kn.as<float>());
        LGF_HIP(hipGetLastError());
        LGF_HIP(hipStreamSynchronize((hipStream_t)stream));
    }
    if ((rc = pl->M.reserve(ms * P3 * sizeof(double))) || (rc = pl->Phi.reserve(ts * P3 * sizeof(double))))
        return rc;
    if (pl->nd > 0) {
        const bool f64 = pair_prec == LGF_F64;
        if ((rc = pl->K.reserve((size_t)pl->nd * P3 * P3 * (f64 ? sizeof(double) : sizeof(float))))) return rc;
        hipStream_t st = (hipStream_t)stream;
        const dim3 g((unsigned)pl->nd), b(256);
        const int4 *di = pl->dinfo.as<int4>();
        const int *nd = pl->nodes.as<int>();
        const double *tg = tb.g.as<double>();
        if (f64) {
            auto kmat = p == 4 ? k_ml_kmat<4, double> : p == 5 ? k_ml_kmat<5, double> : k_ml_kmat<6, double>;
            hipLaunchKernelGGL(kmat, g, b, 0, st, tg, tb.ext[0], tb.ext[1], di, nd, pl->K.as<double>());
        } else {
            auto kmat = p == 4 ? k_ml_kmat<4, float> : p == 5 ? k_ml_kmat<5, float> : k_ml_kmat<6, float>;
            hipLaunchKernelGGL(kmat, g, b, 0, st, tg, tb.ext[0], tb.ext[1], di, nd, pl->K.as<float>());
        }
        LGF_HIP(hipGetLastError());
        LGF_HIP(hipStreamSynchronize(st));
    }
    *out = pl.release();
    return LGFIB_OK;
}

extern "C" int lgf_ml_apply(lgfib_ctx *ctx, lgf_ml_t *pl, int ncomp, double dx, const double *f, double *u,
                            lgfib_stream_t stream) {
    if (!ctx || !pl) return fail(LGFIB_EINVAL, "lgf_ml_apply: null argument");
    if (pl->ctx != ctx) return fail(LGFIB_EINVAL, "lgf_ml_apply: the plan belongs to another context");
    if (ncomp < 1 || ncomp > 8) return fail(LGFIB_EINVAL, "lgf_ml_apply: ncomp must lie in [1, 8]");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, "lgf_ml_apply: dx must be positive");
    const size_t B3 = (size_t)pl->B * pl->B * pl->B;
    if (pl->ntgt == 0) return LGFIB_OK;
    if (!u) return fail(LGFIB_EINVAL, "lgf_ml_apply: null output");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t ubytes = (size_t)ncomp * pl->ntgt * B3 * sizeof(double);
    if (pl->nsrc == 0) {
        LGF_HIP(hipMemsetAsync(u, 0, ubytes, st));
        return LGFIB_OK;
    }
    if (!f) return fail(LGFIB_EINVAL, "lgf_ml_apply: null input");
    const size_t fbytes = (size_t)ncomp * pl->nsrc * B3 * sizeof(double);
    const char *a = (const char *)f, *b = (const char *)u;
    if (a < b + ubytes && b < a + fbytes) return fail(LGFIB_EINVAL, "lgf_ml_apply: f and u overlap");
    if (pl->B == 4) return ml_run<4, 4>(pl, ncomp, dx, f, u, st);
    if (pl->P == 4) return ml_run<4, 8>(pl, ncomp, dx, f, u, st);
    if (pl->P == 5) return ml_run<5, 8>(pl, ncomp, dx, f, u, st);
    return ml_run<6, 8>(pl, ncomp, dx, f, u, st);
}

extern "C" int lgf_ml_info(const lgf_ml_t *pl, int64_t out[6]) {
    if (!pl || !out) return fail(LGFIB_EINVAL, "lgf_ml_info: null argument");
    int64_t ns = 0, nt = 0;
    for (int v : pl->ns) ns += v;
    for (int v : pl->nt) nt += v;
    out[0] = pl->top;
    out[1] = ns;
    out[2] = nt;
    out[3] = pl->npairs;
    out[4] = pl->nnear;
    out[5] = pl->nd;
    return LGFIB_OK;
}

extern "C" void lgf_ml_destroy(lgf_ml_t *pl) {
    if (!pl) return;
    (void)hipSetDevice(pl->device);
    delete pl;
}
