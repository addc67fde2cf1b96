// ib.hip -- immersed-boundary operators on a block set: discrete delta
// regularization R and interpolation I (Sec. 2.1), the staggered gradient G
// and its adjoint G^T, and the body-block set D_body (Sec. 4.1).
//
// Positions are in lattice units; cell n has centre n + (1/2,1/2,1/2) and its
// k-th face sits at x_F^(k)(n) = n + (1/2,1/2,1/2) - e_k/2.
//
// Marker positions are fixed for a plan (a rigid body in its own frame), so
// both operators are assembled once on the host as sparse matrices with the
// tensor-product delta weights: I as rows (marker, component) over face
// indices, R as rows (face) over (marker, component) entries, each row in
// ascending column order.  Applying either is then one gather per output
// (deterministic, no atomics): a thread per face for R, a thread per
// (marker, component) for I.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <unordered_map>

#include "internal.h"

namespace lgfib {

// ------------------------------------------------------------- kernels phi

// Roma, Peskin & Berger (1999): support |r| < 3/2.
__host__ __device__ inline double phi_roma3(double r) {
    const double a = fabs(r);
    if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5) {
        const double b = 1.0 - a;
        return (5.0 - 3.0 * a - sqrt(fmax(0.0, 1.0 - 3.0 * b * b))) / 6.0;
    }
    return 0.0;
}

// Its convolution with the unit top-hat (Yang et al. 2009): support |r| < 2.
__host__ __device__ inline double phi_smooth3(double r) {
    const double a = fabs(r);
    const double s3 = 1.7320508075688772935;
    const double pi = 3.14159265358979323846;
    if (a <= 1.0) {
        return 17.0 / 48.0 + s3 * pi / 108.0 + a / 4.0 - a * a / 4.0 +
               (1.0 - 2.0 * a) / 16.0 * sqrt(fmax(0.0, -12.0 * a * a + 12.0 * a + 1.0)) -
               s3 / 12.0 * asin(fmin(1.0, fmax(-1.0, s3 / 2.0 * (2.0 * a - 1.0))));
    }
    if (a <= 2.0) {
        return 55.0 / 48.0 - s3 * pi / 108.0 - 13.0 * a / 12.0 + a * a / 4.0 +
               (2.0 * a - 3.0) / 48.0 * sqrt(fmax(0.0, -12.0 * a * a + 36.0 * a - 23.0)) +
               s3 / 36.0 * asin(fmin(1.0, fmax(-1.0, s3 / 2.0 * (2.0 * a - 3.0))));
    }
    return 0.0;
}

__host__ __device__ inline double phi_k(int kernel, double r) {
    return kernel == IB_ROMA3 ? phi_roma3(r) : phi_smooth3(r);
}

__host__ __device__ inline double half_width(int kernel) { return kernel == IB_ROMA3 ? 1.5 : 2.0; }

// ----------------------------------------------------------- host staging

static inline long long floordiv(long long a, long long b) {
    long long q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// lowest lattice index n_j with phi(n_j + c - X) != 0 possible, and count
static inline void support_range(int kernel, double X, double c, long long *lo, int *cnt) {
    const double hw = half_width(kernel);
    *lo = (long long)floor(X - c - hw) + 1;
    *cnt = (int)(2 * hw) + 1;
}

struct IbPlan {
    int kernel = 0, NL = 0, B = 0, nblk = 0;
    int lo[3] = {0, 0, 0}, nb[3] = {0, 0, 0};   // block-map box
    DevBuf X;          // double [NL][3]
    DevBuf map;        // int32 [nb2][nb1][nb0] -> slot or -1
    DevBuf blocks;     // int32 [nblk][3]
    // I: rows 3 i + k -> (face index, weight);  R: rows face -> (3 i + k, weight)
    DevBuf i_ptr, i_col, i_val;
    DevBuf r_ptr, r_col, r_val;
    int64_t nnz = 0;
};

struct IbKey {
    uint64_t h;
};

static uint64_t hash_bytes(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct IbCache {
    std::unordered_map<uint64_t, CacheEnt<IbPlan>> plans;
    std::unordered_map<uint64_t, std::vector<char>> keys;   // exact bytes of each plan's key
};

static IbCache &ib_cache(lgfib_ctx *ctx) {
    if (!ctx->ib_cache) ctx->ib_cache = std::make_shared<IbCache>();
    return *static_cast<IbCache *>(ctx->ib_cache.get());
}

static int build_ib_plan(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks, int nblk,
                         std::shared_ptr<IbPlan> &out) {
    // cache by exact bytes of (kernel, B, X, blocks)
    std::vector<char> key;
    key.resize(sizeof(int) * 2 + sizeof(double) * 3 * (size_t)NL + sizeof(int32_t) * 3 * (size_t)nblk);
    char *kp = key.data();
    memcpy(kp, &kernel, sizeof(int));
    memcpy(kp + sizeof(int), &B, sizeof(int));
    if (NL) memcpy(kp + 2 * sizeof(int), X, sizeof(double) * 3 * (size_t)NL);
    if (nblk) memcpy(kp + 2 * sizeof(int) + sizeof(double) * 3 * (size_t)NL, blocks, sizeof(int32_t) * 3 * (size_t)nblk);
    uint64_t h = hash_bytes(1469598103934665603ull, key.data(), key.size());
    IbCache &cache = ib_cache(ctx);
    for (uint64_t salt = 0;; ++salt) {
        uint64_t hh = h ^ (salt * 0x9e3779b97f4a7c15ull);
        auto it = cache.keys.find(hh);
        if (it == cache.keys.end()) {
            h = hh;
            break;
        }
        if (it->second == key) {
            auto pl = cache.plans.find(hh);
            if (pl != cache.plans.end()) {
                pl->second.tick = ++ctx->cache_tick;
                out = pl->second.v;
                return LGFIB_OK;
            }
            cache.keys.erase(it);   // a key left by a failed build: build again
            h = hh;
            break;
        }
    }
    int rc = validate_blocks(blocks, nblk, "body blocks");
    if (rc) return rc;
    for (int i = 0; i < 3 * NL; ++i)
        if (!std::isfinite(X[i]) || fabs(X[i]) > 1e6) return fail(LGFIB_EINVAL, "marker position not finite or too large");
    auto plan = std::make_shared<IbPlan>();
    plan->kernel = kernel;
    plan->NL = NL;
    plan->B = B;
    plan->nblk = nblk;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int i = 0; i < nblk; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], (int)blocks[3 * i + a]);
            hi[a] = std::max(hi[a], (int)blocks[3 * i + a]);
        }
    if (nblk == 0)
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = 0;
    size_t msize = 1;
    for (int a = 0; a < 3; ++a) {
        plan->lo[a] = lo[a];
        plan->nb[a] = hi[a] - lo[a] + 1;
        msize *= (size_t)plan->nb[a];
    }
    if (msize > (size_t)1 << 28) return fail(LGFIB_ERANGE, "body block set spans too large a box");
    std::vector<int32_t> map(msize, -1);
    for (int i = 0; i < nblk; ++i) {
        size_t idx = ((size_t)(blocks[3 * i + 2] - lo[2]) * plan->nb[1] + (blocks[3 * i + 1] - lo[1])) * plan->nb[0] +
                     (blocks[3 * i] - lo[0]);
        map[idx] = i;
    }
    auto slot_of = [&](long long bx, long long by, long long bz) -> int {
        bx -= lo[0];
        by -= lo[1];
        bz -= lo[2];
        if (bx < 0 || by < 0 || bz < 0 || bx >= plan->nb[0] || by >= plan->nb[1] || bz >= plan->nb[2]) return -1;
        return map[((size_t)bz * plan->nb[1] + by) * plan->nb[0] + bx];
    };
    // sparse I and R: the nonzero tensor-product weights of every (marker,
    // component); a support cell outside the block set is an error
    const int B3 = B * B * B;
    const int64_t nfaces = 3ll * nblk * B3;
    if (nfaces > INT32_MAX - 1 || 3ll * NL > INT32_MAX - 1) return fail(LGFIB_ERANGE, "IB operator too large");
    std::vector<int32_t> iptr(3 * (size_t)NL + 1, 0), icol;
    std::vector<double> ival;
    icol.reserve((size_t)NL * 3 * 27);
    ival.reserve((size_t)NL * 3 * 27);
    for (int i = 0; i < NL; ++i) {
        for (int k = 0; k < 3; ++k) {
            long long l[3];
            int cnt[3];
            double w[3][8];
            for (int a = 0; a < 3; ++a) {
                const double c = (a == k) ? 0.0 : 0.5;
                support_range(kernel, X[3 * i + a], c, &l[a], &cnt[a]);
                for (int q = 0; q < cnt[a]; ++q) w[a][q] = phi_k(kernel, (double)(l[a] + q) + c - X[3 * i + a]);
            }
            for (int dz = 0; dz < cnt[2]; ++dz) {
                if (w[2][dz] == 0.0) continue;
                for (int dy = 0; dy < cnt[1]; ++dy) {
                    if (w[1][dy] == 0.0) continue;
                    for (int dxx = 0; dxx < cnt[0]; ++dxx) {
                        if (w[0][dxx] == 0.0) continue;
                        const long long n[3] = {l[0] + dxx, l[1] + dy, l[2] + dz};
                        const long long bq[3] = {floordiv(n[0], B), floordiv(n[1], B), floordiv(n[2], B)};
                        const int slot = slot_of(bq[0], bq[1], bq[2]);
                        if (slot < 0)
                            return fail(LGFIB_ESUPPORT, "support of marker " + std::to_string(i) +
                                                            " leaves the block set");
                        const long long loc = ((n[2] - bq[2] * B) * B + (n[1] - bq[1] * B)) * B + (n[0] - bq[0] * B);
                        icol.push_back((int32_t)(((long long)k * nblk + slot) * B3 + loc));
                        ival.push_back(w[2][dz] * w[1][dy] * w[0][dxx]);
                    }
                }
            }
            iptr[3 * i + k + 1] = (int32_t)icol.size();
        }
    }
    // R = transpose of I: counting sort by face; rows keep ascending (3 i + k)
    const size_t nnz = icol.size();
    std::vector<int32_t> rptr((size_t)nfaces + 1, 0), rcol(std::max<size_t>(nnz, 1));
    std::vector<double> rval(std::max<size_t>(nnz, 1));
    for (size_t e = 0; e < nnz; ++e) rptr[(size_t)icol[e] + 1]++;
    for (int64_t f = 0; f < nfaces; ++f) rptr[f + 1] += rptr[f];
    {
        std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
        for (int64_t row = 0; row < 3ll * NL; ++row)
            for (int32_t e = iptr[row]; e < iptr[row + 1]; ++e) {
                const int32_t pos = fill[icol[e]]++;
                rcol[pos] = (int32_t)row;
                rval[pos] = ival[e];
            }
    }
    if (nnz == 0) {
        icol.push_back(0);
        ival.push_back(0.0);
    }
    plan->nnz = (int64_t)nnz;
    if ((rc = plan->X.reserve(sizeof(double) * 3 * std::max(NL, 1)))) return rc;
    if ((rc = plan->map.reserve(sizeof(int32_t) * map.size()))) return rc;
    if ((rc = plan->blocks.reserve(sizeof(int32_t) * 3 * std::max(nblk, 1)))) return rc;
    if ((rc = plan->i_ptr.reserve(sizeof(int32_t) * iptr.size())) || (rc = plan->i_col.reserve(4 * icol.size())) ||
        (rc = plan->i_val.reserve(8 * ival.size())) || (rc = plan->r_ptr.reserve(sizeof(int32_t) * rptr.size())) ||
        (rc = plan->r_col.reserve(4 * rcol.size())) || (rc = plan->r_val.reserve(8 * rval.size())))
        return rc;
    if (NL) LGF_HIP(hipMemcpy(plan->X.p, X, sizeof(double) * 3 * NL, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->map.p, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice));
    if (nblk) LGF_HIP(hipMemcpy(plan->blocks.p, blocks, sizeof(int32_t) * 3 * nblk, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->i_ptr.p, iptr.data(), 4 * iptr.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->i_col.p, icol.data(), 4 * icol.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->i_val.p, ival.data(), 8 * ival.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->r_ptr.p, rptr.data(), 4 * rptr.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->r_col.p, rcol.data(), 4 * rcol.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->r_val.p, rval.data(), 8 * rval.size(), hipMemcpyHostToDevice));
    out = plan;
    cache.keys[h] = std::move(key);
    cache.plans[h] = CacheEnt<IbPlan>{std::move(plan), ++ctx->cache_tick};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

size_t ib_cache_trim(lgfib_ctx *ctx, size_t cap, int64_t *left) {
    if (!ctx->ib_cache) {
        if (left) *left = 0;
        return 0;
    }
    IbCache &cache = ib_cache(ctx);
    const size_t n = cache_trim(cache.plans, cap, kNoByteCap, [&](uint64_t h, const IbPlan &) { cache.keys.erase(h); });
    if (left) *left = (int64_t)cache.plans.size();
    return n;
}

// --------------------------------------------------------------- kernels

struct BlockMapDev {
    int lo0, lo1, lo2, nb0, nb1, nb2, B;
    const int *map;
    const int *blocks;
    __device__ int slot(int bx, int by, int bz) const {
        bx -= lo0;
        by -= lo1;
        bz -= lo2;
        if (bx < 0 || by < 0 || bz < 0 || bx >= nb0 || by >= nb1 || bz >= nb2) return -1;
        return map[((size_t)bz * nb1 + by) * nb0 + bx];
    }
};

__device__ inline int fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Block sums of a grid-wide reduction go to part[block]; the last block to
// finish (a device-scope counter) adds them in block order, so the result
// does not depend on which block finishes last.  One launch per reduction.
__device__ inline void grid_sum_to(double s, double *part, unsigned *counter, double *out,
                                   double *host_out = nullptr) {
    __shared__ double sh[256];
    __shared__ bool last;
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sh[0];
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double v = 0.0;
    for (unsigned i = threadIdx.x; i < gridDim.x; i += 256) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = sh[0];
        if (host_out) *host_out = sh[0];   // pinned host memory, read after an event
        *counter = 0u;
    }
}

// y[row] = scale * sum_e val[e] x[col[e]] over the row's entries in FP64.
// R: rows are faces, columns 3 i + k, scale dx^-3
// (g^(k)(n) = dx^-3 sum_i x_i^(k) prod_j phi(x_F^(k)(n)_j - X_ij)).
// I: rows 3 i + k, columns face indices, scale 1.
// L lanes share a row (entries strided by L, then a butterfly sum), which
// keeps the dependent col -> x loads of a row short; the summation order is
// fixed, so results are reproducible.
template <typename In, typename Out, int L>
__global__ __launch_bounds__(256) void k_csr_gather(const int *__restrict__ ptr, const int *__restrict__ col,
                                                    const double *__restrict__ val, const In *__restrict__ x,
                                                    Out *__restrict__ y, int nrows, double scale) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int row = (int)(t / L), lane = (int)(t % L);
    const bool live = row < nrows;
    double acc = 0.0;
    if (live) {
        const int e1 = ptr[row + 1];
        for (int e = ptr[row] + lane; e < e1; e += L) acc += val[e] * (double)x[col[e]];
    }
#pragma unroll
    for (int m = L / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, L);
    if (live && lane == 0) y[row] = (Out)(acc * scale);
}

// I with the CG's p.Ap fused in: y = I faces, and *out = sum_row p[row] y[row]
// (rows summed per block in a fixed order, then across blocks as above)
template <typename In, int L>
__global__ __launch_bounds__(256) void k_csr_gather_dot(const int *__restrict__ ptr, const int *__restrict__ col,
                                                        const double *__restrict__ val, const In *__restrict__ x,
                                                        double *__restrict__ y, int nrows,
                                                        const double *__restrict__ p, double *part,
                                                        unsigned *counter, double *out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int row = (int)(t / L), lane = (int)(t % L);
    const bool live = row < nrows;
    double acc = 0.0;
    if (live) {
        const int e1 = ptr[row + 1];
        for (int e = ptr[row] + lane; e < e1; e += L) acc += val[e] * (double)x[col[e]];
    }
#pragma unroll
    for (int m = L / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, L);
    double contrib = 0.0;
    if (live && lane == 0) {
        y[row] = acc;
        contrib = acc * p[row];
    }
    grid_sum_to(contrib, part, counter, out);
}

// c(n) = sc sum_k u^(k)(n) - u^(k)(n + e_k)   (G^T u; faces outside are zero)
template <typename Real>
__global__ void k_grad_adjoint(BlockMapDev bm, const Real *__restrict__ u, Real *__restrict__ c, int nblk, Real sc) {
    const int B = bm.B, B3 = B * B * B;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nblk * B3) return;
    const int b = (int)(t / B3), cell = (int)(t % B3);
    const int lx = cell % B, ly = (cell / B) % B, lz = cell / (B * B);
    const int bx = bm.blocks[3 * b], by = bm.blocks[3 * b + 1], bz = bm.blocks[3 * b + 2];
    Real s = 0;
    for (int k = 0; k < 3; ++k) {
        s += u[((size_t)k * nblk + b) * B3 + cell];
        int nx = lx + (k == 0), ny = ly + (k == 1), nz = lz + (k == 2);
        int sb = b, cbx = bx, cby = by, cbz = bz;
        if (nx == B) { nx = 0; cbx += 1; }
        if (ny == B) { ny = 0; cby += 1; }
        if (nz == B) { nz = 0; cbz += 1; }
        if (cbx != bx || cby != by || cbz != bz) sb = bm.slot(cbx, cby, cbz);
        if (sb >= 0) s -= u[((size_t)k * nblk + sb) * B3 + (nz * B + ny) * B + nx];
    }
    c[t] = sc * s;
}

// e^(k)(n) += sc (d(n) - d(n - e_k))          (G d, accumulated into faces)
template <typename Real>
__global__ void k_grad_acc(BlockMapDev bm, const Real *__restrict__ d, Real *__restrict__ e, int nblk, Real sc) {
    const int B = bm.B, B3 = B * B * B;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nblk * B3) return;
    const int b = (int)(t / B3), cell = (int)(t % B3);
    const int lx = cell % B, ly = (cell / B) % B, lz = cell / (B * B);
    const int bx = bm.blocks[3 * b], by = bm.blocks[3 * b + 1], bz = bm.blocks[3 * b + 2];
    const Real dc = d[t];
    for (int k = 0; k < 3; ++k) {
        int nx = lx - (k == 0), ny = ly - (k == 1), nz = lz - (k == 2);
        int sb = b, cbx = bx, cby = by, cbz = bz;
        if (nx < 0) { nx = B - 1; cbx -= 1; }
        if (ny < 0) { ny = B - 1; cby -= 1; }
        if (nz < 0) { nz = B - 1; cbz -= 1; }
        if (cbx != bx || cby != by || cbz != bz) sb = bm.slot(cbx, cby, cbz);
        const Real dm = sb >= 0 ? d[(size_t)sb * B3 + (nz * B + ny) * B + nx] : (Real)0;
        e[((size_t)k * nblk + b) * B3 + cell] += sc * (dc - dm);
    }
}

static BlockMapDev devmap(const IbPlan &p) {
    BlockMapDev m;
    m.lo0 = p.lo[0];
    m.lo1 = p.lo[1];
    m.lo2 = p.lo[2];
    m.nb0 = p.nb[0];
    m.nb1 = p.nb[1];
    m.nb2 = p.nb[2];
    m.B = p.B;
    m.map = p.map.as<int>();
    m.blocks = p.blocks.as<int>();
    return m;
}

static unsigned nblocks(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename In, typename Out>
static int launch_regularize(lgfib_ctx *ctx, const IbPlan &p, double dx, const In *x, Out *faces, hipStream_t st) {
    if (p.nblk == 0) return LGFIB_OK;
    ProfScope ps(ctx, "k_regularize", st);
    const int nrows = 3 * p.nblk * p.B * p.B * p.B;
    hipLaunchKernelGGL((k_csr_gather<In, Out, 4>), dim3(nblocks(4 * (size_t)nrows, 256)), dim3(256), 0, st,
                       p.r_ptr.as<int>(),
                       p.r_col.as<int>(), p.r_val.as<double>(), x, faces, nrows, 1.0 / (dx * dx * dx));
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename In, typename Out>
static int launch_interpolate(lgfib_ctx *ctx, const IbPlan &p, const In *faces, Out *v, hipStream_t st) {
    if (p.NL == 0) return LGFIB_OK;
    ProfScope ps(ctx, "k_interpolate", st);
    const int nrows = 3 * p.NL;
    hipLaunchKernelGGL((k_csr_gather<In, Out, 16>), dim3(nblocks(16 * (size_t)nrows, 256)), dim3(256), 0, st,
                       p.i_ptr.as<int>(),
                       p.i_col.as<int>(), p.i_val.as<double>(), faces, v, nrows, 1.0);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real>
static int launch_grad_adjoint(lgfib_ctx *ctx, const IbPlan &p, const Real *u, Real *c, hipStream_t st,
                               Real sc = (Real)1) {
    const size_t n = (size_t)p.nblk * p.B * p.B * p.B;
    if (!n) return LGFIB_OK;
    ProfScope ps(ctx, "k_grad_adjoint", st);
    hipLaunchKernelGGL(k_grad_adjoint<Real>, dim3(nblocks(n, 256)), dim3(256), 0, st, devmap(p), u, c, p.nblk, sc);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real>
static int launch_grad_acc(lgfib_ctx *ctx, const IbPlan &p, const Real *d, Real *e, hipStream_t st,
                           Real sc = (Real)1) {
    const size_t n = (size_t)p.nblk * p.B * p.B * p.B;
    if (!n) return LGFIB_OK;
    ProfScope ps(ctx, "k_grad_acc", st);
    hipLaunchKernelGGL(k_grad_acc<Real>, dim3(nblocks(n, 256)), dim3(256), 0, st, devmap(p), d, e, p.nblk, sc);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// ------------------------------------------------------------ body blocks

static int body_blocks(int kernel, const double *X, int NL, int B, std::vector<int32_t> &out) {
    struct H {
        size_t operator()(const std::array<long long, 3> &a) const {
            return std::hash<long long>()(a[0] * 73856093ll ^ a[1] * 19349663ll ^ a[2] * 83492791ll);
        }
    };
    std::unordered_map<std::array<long long, 3>, char, H> set;
    for (int i = 0; i < NL; ++i) {
        for (int k = 0; k < 3; ++k) {
            long long l[3];
            int cnt[3];
            for (int a = 0; a < 3; ++a) support_range(kernel, X[3 * i + a], (a == k) ? 0.0 : 0.5, &l[a], &cnt[a]);
            for (int dz = 0; dz < cnt[2]; ++dz)
                for (int dy = 0; dy < cnt[1]; ++dy)
                    for (int dxx = 0; dxx < cnt[0]; ++dxx) {
                        const long long n[3] = {l[0] + dxx, l[1] + dy, l[2] + dz};
                        double w = 1.0;
                        for (int a = 0; a < 3; ++a)
                            w *= phi_k(kernel, (double)n[a] + ((a == k) ? 0.0 : 0.5) - X[3 * i + a]);
                        if (w == 0.0) continue;
                        // the support cell and its 26 neighbours
                        for (int ez = -1; ez <= 1; ++ez)
                            for (int ey = -1; ey <= 1; ++ey)
                                for (int ex = -1; ex <= 1; ++ex)
                                    set[{floordiv(n[0] + ex, B), floordiv(n[1] + ey, B), floordiv(n[2] + ez, B)}] = 1;
                    }
        }
    }
    std::vector<std::array<long long, 3>> v;
    v.reserve(set.size());
    for (auto &kv : set) v.push_back(kv.first);
    std::sort(v.begin(), v.end(), [](const std::array<long long, 3> &a, const std::array<long long, 3> &b) {
        if (a[2] != b[2]) return a[2] < b[2];
        if (a[1] != b[1]) return a[1] < b[1];
        return a[0] < b[0];
    });
    out.clear();
    for (auto &b : v) {
        for (int a = 0; a < 3; ++a) {
            if (b[a] < -(1 << 20) || b[a] >= (1 << 20)) return fail(LGFIB_ERANGE, "body block coordinate out of range");
            out.push_back((int32_t)b[a]);
        }
    }
    return LGFIB_OK;
}

}  // namespace lgfib

using namespace lgfib;

static int ib_check(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks, int nblk,
                    int prec, double dx, const char *who) {
    if (!ctx) return fail(LGFIB_EINVAL, std::string(who) + ": null context");
    if (kernel != IB_ROMA3 && kernel != IB_SMOOTH3) return fail(LGFIB_EINVAL, std::string(who) + ": unknown kernel");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, std::string(who) + ": B must be 4, 8, 16 or 32");
    if (NL < 0 || nblk < 0) return fail(LGFIB_EINVAL, std::string(who) + ": negative count");
    if (NL > 0 && !X) return fail(LGFIB_EINVAL, std::string(who) + ": null marker positions");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, std::string(who) + ": bad prec");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, std::string(who) + ": dx must be positive");
    return LGFIB_OK;
}

extern "C" int ib_body_blocks(int kernel, const double *X, int NL, int B, int32_t *out, int max, int *n) {
    if (kernel != IB_ROMA3 && kernel != IB_SMOOTH3) return fail(LGFIB_EINVAL, "ib_body_blocks: unknown kernel");
    if (B < 1 || NL < 0 || (NL > 0 && !X) || !n) return fail(LGFIB_EINVAL, "ib_body_blocks: bad argument");
    for (int i = 0; i < 3 * NL; ++i)
        if (!std::isfinite(X[i]) || fabs(X[i]) > 1e6) return fail(LGFIB_EINVAL, "ib_body_blocks: bad marker position");
    std::vector<int32_t> v;
    int rc = body_blocks(kernel, X, NL, B, v);
    if (rc) return rc;
    *n = (int)(v.size() / 3);
    if (*n > max || (*n > 0 && !out)) return fail(LGFIB_ERANGE, "ib_body_blocks: output holds fewer blocks than needed");
    std::copy(v.begin(), v.end(), out);
    return LGFIB_OK;
}

extern "C" int ib_regularize(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks,
                             int nblk, int prec, double dx, const void *x, void *faces, lgfib_stream_t stream) {
    int rc = ib_check(ctx, kernel, X, NL, B, blocks, nblk, prec, dx, "ib_regularize");
    if (rc) return rc;
    if ((NL > 0 && !x) || (nblk > 0 && !faces)) return fail(LGFIB_EINVAL, "ib_regularize: null field pointer");
    LGF_HIP(hipSetDevice(ctx->device));
    std::shared_ptr<IbPlan> p;
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, p))) return rc;
    if (prec == LGF_F64)
        return launch_regularize<double, double>(ctx, *p, dx, (const double *)x, (double *)faces, (hipStream_t)stream);
    return launch_regularize<float, float>(ctx, *p, dx, (const float *)x, (float *)faces, (hipStream_t)stream);
}

extern "C" int ib_interpolate(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks,
                              int nblk, int prec, double dx, const void *faces, void *v, lgfib_stream_t stream) {
    int rc = ib_check(ctx, kernel, X, NL, B, blocks, nblk, prec, dx, "ib_interpolate");
    if (rc) return rc;
    if ((NL > 0 && !v) || (nblk > 0 && !faces)) return fail(LGFIB_EINVAL, "ib_interpolate: null field pointer");
    LGF_HIP(hipSetDevice(ctx->device));
    std::shared_ptr<IbPlan> p;
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, p))) return rc;
    if (prec == LGF_F64)
        return launch_interpolate<double, double>(ctx, *p, (const double *)faces, (double *)v, (hipStream_t)stream);
    return launch_interpolate<float, float>(ctx, *p, (const float *)faces, (float *)v, (hipStream_t)stream);
}

// ---------------------------------------------------------- Schur system

namespace lgfib {
constexpr int kRedBlocks = 256;   // blocks of a grid-wide reduction
// partial-sum slots: a fused reduction may run one per block of its launch
inline size_t red_parts(int NL) { return std::max<size_t>(kRedBlocks, (16 * 3 * (size_t)NL + 255) / 256 + 1); }
}

struct ib_system {
    lgfib_ctx *ctx = nullptr;
    int kernel = 0, NL = 0, B = 0, nblk = 0;
    double a = 0.0;
    std::vector<double> X;
    std::vector<int32_t> blocks;
    lgf_table_t tbl = -1;
    std::shared_ptr<IbPlan> plan;   // held: pinned in the context's cache
    // work fields per precision: faces g, faces a, cells c, cells d
    DevBuf g[2], af[2], c[2], d[2];
    // CG vectors (FP64)
    DevBuf r, p, ap, x, tmp, red, scal, cnt;
    double *host_scal = nullptr;       // pinned; the CG's r.r lands in [8], [9]
    double *host_scal_dev = nullptr;   // its device address
    hipEvent_t ev[2] = {nullptr, nullptr};
    // captured CG iterations per matvec precision (index 0 FP32, 1 FP64) and
    // parity of the iteration; valid while the shared FFT workspaces stay put
    hipGraphExec_t cg_exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    const void *cg_work[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    uint64_t cg_epoch[2] = {0, 0};   // the context's cache epoch when captured
    bool cg_nograph[2] = {false, false};   // capture failed once: run eagerly
    hipStream_t cap = nullptr;
    // inverse Cholesky factor W = L^{-1} of the dense C (ib_system_factor)
    DevBuf wfac;
    bool factored = false;
    DevBuf gamma;   // R 1 on the body faces (force smoothing), built on first use
    DevBuf dense_cols;   // workspace of the column-batched dense build of C
};

namespace lgfib {

// y = C x = I [E(a) + G K^{-1} G^T] R x with the field work in Real; x and y
// may be held in another type (the FP32 matvec of the CG reads and writes its
// FP64 vectors directly).
template <typename Real, typename VIn, typename VOut>
static int schur_apply_t(ib_system *s, const VIn *x, VOut *y, hipStream_t st, const double *dot_p = nullptr,
                         double *dot_out = nullptr) {
    lgfib_ctx *ctx = s->ctx;
    const int pi = sizeof(Real) == 8 ? 1 : 0;
    const int prec = pi ? LGF_F64 : LGF_F32;
    Real *g = s->g[pi].as<Real>(), *af = s->af[pi].as<Real>(), *c = s->c[pi].as<Real>(), *d = s->d[pi].as<Real>();
    int rc;
    if ((rc = launch_regularize<VIn, Real>(ctx, *s->plan, 1.0, x, g, st))) return rc;
    if ((rc = lgf_if_apply(ctx, s->a, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, 3, prec, g, af,
                           (lgfib_stream_t)st)))
        return rc;
    if ((rc = launch_grad_adjoint<Real>(ctx, *s->plan, g, c, st))) return rc;
    if ((rc = lgf_poisson_apply(ctx, s->tbl, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, 1, prec, 1.0,
                                c, d, 0, (lgfib_stream_t)st)))
        return rc;
    if ((rc = launch_grad_acc<Real>(ctx, *s->plan, d, af, st))) return rc;
    if constexpr (std::is_same<VOut, double>::value) {
        if (dot_p) {   // y = I af with p.y fused (CG iteration)
            const IbPlan &P = *s->plan;
            const int nrows = 3 * P.NL;
            ProfScope ps(ctx, "k_interpolate", st);
            hipLaunchKernelGGL((k_csr_gather_dot<Real, 16>), dim3(nblocks(16 * (size_t)nrows, 256)), dim3(256), 0, st,
                               P.i_ptr.as<int>(), P.i_col.as<int>(), P.i_val.as<double>(), af, y, nrows, dot_p,
                               s->red.as<double>(), s->cnt.as<unsigned>(), dot_out);
            LGF_HIP(hipGetLastError());
            return LGFIB_OK;
        }
    }
    return launch_interpolate<Real, VOut>(ctx, *s->plan, af, y, st);
}

}  // namespace lgfib

extern "C" int ib_system_create(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks,
                                int nblk, double a, ib_system **out) {
    if (!out) return fail(LGFIB_EINVAL, "ib_system_create: null output");
    *out = nullptr;
    int rc = ib_check(ctx, kernel, X, NL, B, blocks, nblk, LGF_F64, 1.0, "ib_system_create");
    if (rc) return rc;
    if (B > 16) return fail(LGFIB_EINVAL, "ib_system_create: B must be 4, 8 or 16");
    if (NL < 1 || nblk < 1) return fail(LGFIB_EINVAL, "ib_system_create: need markers and blocks");
    if (!(a >= 0.0) || a > 4.0) return fail(LGFIB_EINVAL, "ib_system_create: a must lie in [0, 4]");
    LGF_HIP(hipSetDevice(ctx->device));
    auto s = std::make_unique<ib_system>();
    s->ctx = ctx;
    s->kernel = kernel;
    s->NL = NL;
    s->B = B;
    s->nblk = nblk;
    s->a = a;
    s->X.assign(X, X + 3 * (size_t)NL);
    s->blocks.assign(blocks, blocks + 3 * (size_t)nblk);
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, s->plan))) return rc;
    int ext[3];
    for (int q = 0; q < 3; ++q) ext[q] = s->plan->nb[q] * B - 1;
    if ((rc = lgf_table_build(ctx, LGF_KIND_K, a, ext, nullptr, &s->tbl))) return rc;
    const size_t B3 = (size_t)B * B * B;
    for (int pi = 0; pi < 2; ++pi) {
        const size_t es = pi ? 8 : 4;
        if ((rc = s->g[pi].reserve(3 * nblk * B3 * es))) return rc;
        if ((rc = s->af[pi].reserve(3 * nblk * B3 * es))) return rc;
        if ((rc = s->c[pi].reserve(nblk * B3 * es))) return rc;
        if ((rc = s->d[pi].reserve(nblk * B3 * es))) return rc;
    }
    const size_t nv = 3 * (size_t)NL * 8;
    if ((rc = s->r.reserve(nv)) || (rc = s->p.reserve(nv)) || (rc = s->ap.reserve(nv)) || (rc = s->x.reserve(nv)) ||
        (rc = s->tmp.reserve(nv)) || (rc = s->red.reserve(red_parts(NL) * 8)) || (rc = s->scal.reserve(64 * 8)) ||
        (rc = s->cnt.reserve(64)))
        return rc;
    LGF_HIP(hipMemset(s->cnt.p, 0, 64));
    LGF_HIP(hipHostMalloc((void **)&s->host_scal, 64 * sizeof(double), hipHostMallocDefault));
    LGF_HIP(hipHostGetDevicePointer((void **)&s->host_scal_dev, s->host_scal, 0));
    for (auto &e : s->ev) LGF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    *out = s.release();
    return LGFIB_OK;
}

extern "C" void ib_system_destroy(ib_system *sys) {
    if (!sys) return;
    (void)hipSetDevice(sys->ctx->device);
    (void)hipDeviceSynchronize();
    if (sys->host_scal) (void)hipHostFree(sys->host_scal);
    for (auto &e : sys->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &row : sys->cg_exec)
        for (auto &g : row)
            if (g) (void)hipGraphExecDestroy(g);
    if (sys->cap) (void)hipStreamDestroy(sys->cap);
    delete sys;
}

extern "C" int ib_schur_apply(lgfib_ctx *ctx, ib_system *sys, int prec, const void *x, void *y,
                              lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_schur_apply: bad context or system");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "ib_schur_apply: bad prec");
    if (!x || !y) return fail(LGFIB_EINVAL, "ib_schur_apply: null vector");
    const size_t nb = 3 * (size_t)sys->NL * (prec == LGF_F64 ? 8 : 4);
    if ((const char *)x < (const char *)y + nb && (const char *)y < (const char *)x + nb)
        return fail(LGFIB_EINVAL, "ib_schur_apply: x and y overlap");
    LGF_HIP(hipSetDevice(ctx->device));
    if (prec == LGF_F64)
        return schur_apply_t<double, double, double>(sys, (const double *)x, (double *)y, (hipStream_t)stream);
    return schur_apply_t<float, float, float>(sys, (const float *)x, (float *)y, (hipStream_t)stream);
}

// ------------------------------------------------------ conjugate gradients

namespace lgfib {

__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a, const double *__restrict__ b, size_t n,
                                             double *part, unsigned *counter, double *out) {
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) s += a[i] * b[i];
    grid_sum_to(s, part, counter, out);
}

// scal layout: [1] pAp, [2] scratch dot, [3] bb, [4] final residual,
// [6 + (j & 1)] r.r of CG iteration j (the slots alternate, so no copy is
// needed between iterations).
// x += alpha p ; r -= alpha Ap, alpha = rs / pAp (0 once the search direction
// vanishes: the host tests convergence one iteration late, so a converged
// solve may run one more, harmless, iteration); then out = r.r
__global__ __launch_bounds__(256) void k_cg_xr(double *__restrict__ x, double *__restrict__ r,
                                               const double *__restrict__ p, const double *__restrict__ ap,
                                               double *scal, int rs_slot, int out_slot, size_t n, double *part,
                                               unsigned *counter, double *host_out) {
    const double alpha = scal[1] > 0.0 ? scal[rs_slot] / scal[1] : 0.0;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * ap[i];
        r[i] = ri;
        s += ri * ri;
    }
    grid_sum_to(s, part, counter, scal + out_slot, host_out);
}

// The whole CG update for vectors small enough for one workgroup (the
// marker systems): pAp = p.Ap, alpha = rs / pAp, x += alpha p,
// r -= alpha Ap, rs_new = r.r, beta = rs_new / rs, p = r + beta p -- one
// launch, no cross-workgroup traffic, sums in a fixed order.  rs_new also
// goes to pinned host memory for the convergence test.
constexpr int kStepThreads = 1024;
constexpr size_t kStepMaxN = 65536;

// workgroup sum: butterfly within each wavefront, then across the wavefronts'
// partials (fixed order, so the result is reproducible)
__device__ inline double wg_sum(double v, double *sh) {
    constexpr int kWaves = kStepThreads / 64;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = lane < kWaves ? sh[lane] : 0.0;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    __syncthreads();   // sh is reused by the next call
    return t;
}

__global__ __launch_bounds__(kStepThreads) void k_cg_step(double *__restrict__ x, double *__restrict__ r,
                                                          double *__restrict__ p, const double *__restrict__ ap,
                                                          double *scal, int rs_slot, int new_slot, int n,
                                                          double *host_out) {
    __shared__ double sh[kStepThreads];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < n; i += kStepThreads) s += p[i] * ap[i];
    const double pap = wg_sum(s, sh);
    const double rs = scal[rs_slot];
    const double alpha = pap > 0.0 ? rs / pap : 0.0;
    double q = 0.0;
    for (int i = tid; i < n; i += kStepThreads) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * ap[i];
        r[i] = ri;
        q += ri * ri;
    }
    const double rsn = wg_sum(q, sh);
    const double beta = rs > 0.0 ? rsn / rs : 0.0;
    for (int i = tid; i < n; i += kStepThreads) p[i] = r[i] + beta * p[i];
    if (tid == 0) {
        scal[1] = pap;
        scal[new_slot] = rsn;
        if (host_out) *host_out = rsn;
    }
}

// a.b in one workgroup (small vectors)
__global__ __launch_bounds__(kStepThreads) void k_dot_small(const double *__restrict__ a,
                                                            const double *__restrict__ b, int n, double *out) {
    __shared__ double sh[kStepThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kStepThreads) s += a[i] * b[i];
    const double t = wg_sum(s, sh);
    if (threadIdx.x == 0) *out = t;
}

// p = r + beta p, beta = rs_new / rs
__global__ void k_cg_p(double *__restrict__ p, const double *__restrict__ r, const double *__restrict__ scal,
                       int rs_slot, int new_slot, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = scal[rs_slot] > 0.0 ? scal[new_slot] / scal[rs_slot] : 0.0;
    p[i] = r[i] + beta * p[i];
}

// r = b - y
__global__ void k_sub(double *__restrict__ r, const double *__restrict__ b, const double *__restrict__ y, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) r[t] = b[t] - y[t];
}

// The same update with each thread's E elements of p, Ap and r held in
// registers: every vector is read once instead of up to twice (n <= E
// kStepThreads).  Elements are visited in the same order, so the sums, and
// with them the iterates, are bitwise those of k_cg_step.
template <int E>
__global__ __launch_bounds__(kStepThreads) void k_cg_step_reg(double *__restrict__ x, double *__restrict__ r,
                                                              double *__restrict__ p, const double *__restrict__ ap,
                                                              double *scal, int rs_slot, int new_slot, int n,
                                                              double *host_out) {
    __shared__ double sh[kStepThreads];
    const int tid = threadIdx.x;
    double pv[E], av[E], rv[E];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = tid + e * kStepThreads;
        const bool in = i < n;
        pv[e] = in ? p[i] : 0.0;
        av[e] = in ? ap[i] : 0.0;
        rv[e] = in ? r[i] : 0.0;
        if (in) s += pv[e] * av[e];
    }
    const double pap = wg_sum(s, sh);
    const double rs = scal[rs_slot];
    const double alpha = pap > 0.0 ? rs / pap : 0.0;
    double q = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = tid + e * kStepThreads;
        if (i < n) {
            x[i] += alpha * pv[e];
            rv[e] = rv[e] - alpha * av[e];
            r[i] = rv[e];
            q += rv[e] * rv[e];
        }
    }
    const double rsn = wg_sum(q, sh);
    const double beta = rs > 0.0 ? rsn / rs : 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = tid + e * kStepThreads;
        if (i < n) p[i] = rv[e] + beta * pv[e];
    }
    if (tid == 0) {
        scal[1] = pap;
        scal[new_slot] = rsn;
        if (host_out) *host_out = rsn;
    }
}
constexpr int kStepRegE = 8, kStepRegE2 = 16;   // n up to 8192, then up to 16384

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, double a, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

static unsigned red_blocks(size_t n) { return (unsigned)std::min<size_t>(kRedBlocks, std::max<size_t>(1, (n + 255) / 256)); }

static int dot(ib_system *s, const double *a, const double *b, int slot, hipStream_t st) {
    const size_t n = 3 * (size_t)s->NL;
    if (n <= kStepMaxN) {
        hipLaunchKernelGGL(k_dot_small, dim3(1), dim3(kStepThreads), 0, st, a, b, (int)n, s->scal.as<double>() + slot);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    hipLaunchKernelGGL(k_dot, dim3(red_blocks(n)), dim3(256), 0, st, a, b, n, s->red.as<double>(),
                       s->cnt.as<unsigned>(), s->scal.as<double>() + slot);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

static int read_scal(ib_system *s, int slot, double *v, hipStream_t st) {
    LGF_HIP(hipMemcpyAsync(s->host_scal + slot, s->scal.as<double>() + slot, sizeof(double), hipMemcpyDeviceToHost, st));
    LGF_HIP(hipStreamSynchronize(st));
    *v = s->host_scal[slot];
    return LGFIB_OK;
}

// y = C x with an FP64 interface, field work in prec
static int matvec(ib_system *s, int prec, const double *x, double *y, hipStream_t st, double *dot_out = nullptr) {
    const double *dp = dot_out ? x : nullptr;   // fused x.y into *dot_out
    if (prec == LGF_F64) return schur_apply_t<double, double, double>(s, x, y, st, dp, dot_out);
    return schur_apply_t<float, double, double>(s, x, y, st, dp, dot_out);
}

// One CG iteration (matvec, p.Ap, x/r update with r.r, the copy of r.r to
// pinned memory, p update) for iterations of parity `par`.
static int cg_iteration(ib_system *s, int prec, int par, hipStream_t st) {
    const size_t n = 3 * (size_t)s->NL;
    double *x = s->x.as<double>(), *r = s->r.as<double>(), *p = s->p.as<double>(), *ap = s->ap.as<double>();
    double *scal = s->scal.as<double>();
    const int rs_slot = 6 + par, new_slot = 6 + (1 - par);
    int rc;
    if (n <= kStepMaxN) {
        if ((rc = matvec(s, prec, p, ap, st))) return rc;
        if (n <= (size_t)kStepRegE * kStepThreads)
            hipLaunchKernelGGL(k_cg_step_reg<kStepRegE>, dim3(1), dim3(kStepThreads), 0, st, x, r, p, ap, scal, rs_slot,
                               new_slot, (int)n, s->host_scal_dev + 8 + par);
        else if (n <= (size_t)kStepRegE2 * kStepThreads)
            hipLaunchKernelGGL(k_cg_step_reg<kStepRegE2>, dim3(1), dim3(kStepThreads), 0, st, x, r, p, ap, scal,
                               rs_slot, new_slot, (int)n, s->host_scal_dev + 8 + par);
        else
            hipLaunchKernelGGL(k_cg_step, dim3(1), dim3(kStepThreads), 0, st, x, r, p, ap, scal, rs_slot, new_slot,
                               (int)n, s->host_scal_dev + 8 + par);
        LGF_HIP(hipGetLastError());
        return LGFIB_OK;
    }
    if ((rc = matvec(s, prec, p, ap, st, scal + 1))) return rc;   // ap = C p, scal[1] = p.ap
    hipLaunchKernelGGL(k_cg_xr, dim3(red_blocks(n)), dim3(256), 0, st, x, r, p, ap, scal, rs_slot, new_slot, n,
                       s->red.as<double>(), s->cnt.as<unsigned>(), s->host_scal_dev + 8 + par);
    hipLaunchKernelGGL(k_cg_p, dim3(nblocks(n, 256)), dim3(256), 0, st, p, r, scal, rs_slot, new_slot, n);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

static bool cg_graphs_wanted() {
    const char *e = getenv("LGFIB_CG_GRAPH");
    return !(e && e[0] == '0');
}

// Capture both parities of the CG iteration into graphs (on a private
// stream, after an eager matvec has created every plan, table spectrum and
// workspace the matvec touches).  Recaptured when the context's FFT
// workspaces have been reallocated by other work.
static int cg_graphs(ib_system *s, int prec, hipStream_t st, bool *ok) {
    const int pi = prec == LGF_F64 ? 1 : 0;
    *ok = false;
    if (!cg_graphs_wanted() || s->cg_nograph[pi]) return LGFIB_OK;
    lgfib_ctx *ctx = s->ctx;
    if (s->cg_exec[pi][0] && s->cg_work[pi][0] == ctx->work1.p && s->cg_work[pi][1] == ctx->work2.p &&
        s->cg_epoch[pi] == ctx->cache_epoch) {
        *ok = true;
        return LGFIB_OK;
    }
    if (ctx->profiling) return LGFIB_OK;   // profiling events stay out of graphs
    int rc;
    if ((rc = matvec(s, prec, s->p.as<double>(), s->tmp.as<double>(), st))) return rc;
    LGF_HIP(hipStreamSynchronize(st));
    if (!s->cap) LGF_HIP(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    for (int par = 0; par < 2; ++par) {
        if (s->cg_exec[pi][par]) {
            LGF_HIP(hipGraphExecDestroy(s->cg_exec[pi][par]));
            s->cg_exec[pi][par] = nullptr;
        }
        hipGraph_t g = nullptr;
        LGF_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
        rc = cg_iteration(s, prec, par, s->cap);
        const hipError_t e = hipStreamEndCapture(s->cap, &g);
        hipError_t ei = hipErrorUnknown;
        if (!rc && e == hipSuccess && g) ei = hipGraphInstantiate(&s->cg_exec[pi][par], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {   // the eager loop runs the same kernels
            (void)hipGetLastError();
            for (auto &x : s->cg_exec[pi])
                if (x) {
                    (void)hipGraphExecDestroy(x);
                    x = nullptr;
                }
            s->cg_nograph[pi] = true;
            return LGFIB_OK;
        }
    }
    s->cg_work[pi][0] = ctx->work1.p;
    s->cg_work[pi][1] = ctx->work2.p;
    s->cg_epoch[pi] = ctx->cache_epoch;
    *ok = true;
    return LGFIB_OK;
}

}  // namespace lgfib

// column j of a row-major matrix: C[i][j] = y[i]
__global__ void k_put_column(double *__restrict__ C, long ld, int j, const double *__restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) C[(long)i * ld + j] = y[i];
}

__global__ void k_unit(double *__restrict__ e, int n, int j) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) e[i] = i == j ? 1.0 : 0.0;
}

static int direct_solve(ib_system *s, const double *b, double *f, ib_solve_stats_t *S, hipStream_t st) {
    const int n = 3 * s->NL;
    int rc;
    hipEvent_t e0, e1;
    LGF_HIP(hipEventCreate(&e0));
    LGF_HIP(hipEventCreate(&e1));
    LGF_HIP(hipEventRecord(e0, st));
    if ((rc = chol_solve_f64(s->ctx, n, s->wfac.as<double>(), n, b, f, st))) return rc;
    LGF_HIP(hipEventRecord(e1, st));
    LGF_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LGF_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (S) {
        *S = ib_solve_stats_t{};
        S->ms = ms;
        double *ap = s->ap.as<double>(), *r = s->r.as<double>();
        double bb, rr;
        if ((rc = matvec(s, LGF_F64, f, ap, st))) return rc;
        hipLaunchKernelGGL(k_sub, dim3(nblocks(n, 256)), dim3(256), 0, st, r, b, ap, (size_t)n);
        LGF_HIP(hipGetLastError());
        if ((rc = dot(s, b, b, 3, st)) || (rc = read_scal(s, 3, &bb, st))) return rc;
        if ((rc = dot(s, r, r, 4, st)) || (rc = read_scal(s, 4, &rr, st))) return rc;
        S->rel_residual = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    }
    return LGFIB_OK;
}

extern "C" int ib_force_solve(lgfib_ctx *ctx, ib_system *sys, int prec, const double *b, double *f, const double *x0,
                              double rtol, int maxit, ib_solve_stats_t *stats, lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_force_solve: bad context or system");
    if (prec == IB_SOLVE_DIRECT) {
        if (!b || !f) return fail(LGFIB_EINVAL, "ib_force_solve: null vector");
        if (!sys->factored) return fail(LGFIB_ENOTBUILT, "ib_force_solve: the system has no factor (ib_system_factor)");
        LGF_HIP(hipSetDevice(ctx->device));
        return direct_solve(sys, b, f, stats, (hipStream_t)stream);
    }
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "ib_force_solve: bad prec");
    if (!b || !f) return fail(LGFIB_EINVAL, "ib_force_solve: null vector");
    if (!(rtol > 0.0) || maxit < 1) return fail(LGFIB_EINVAL, "ib_force_solve: rtol > 0 and maxit >= 1 required");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    ib_solve_stats_t loc{};
    ib_solve_stats_t *S = stats ? stats : &loc;
    *S = ib_solve_stats_t{};
    hipEvent_t e0, e1;
    LGF_HIP(hipEventCreate(&e0));
    LGF_HIP(hipEventCreate(&e1));
    LGF_HIP(hipEventRecord(e0, st));
    const size_t n = 3 * (size_t)sys->NL;
    const unsigned gb = nblocks(n, 256);
    double *x = sys->x.as<double>(), *r = sys->r.as<double>(), *p = sys->p.as<double>(), *ap = sys->ap.as<double>(),
           *tmp = sys->tmp.as<double>(), *scal = sys->scal.as<double>();
    int rc;
    double bb;
    if ((rc = dot(sys, b, b, 3, st)) || (rc = read_scal(sys, 3, &bb, st))) return rc;
    const double bnorm = sqrt(bb);
    if (bnorm == 0.0) {
        LGF_HIP(hipMemsetAsync(f, 0, n * 8, st));
        LGF_HIP(hipStreamSynchronize(st));
        S->rel_residual = 0.0;
        return LGFIB_OK;
    }
    // initial guess
    bool use_x0 = false;
    if (x0) {
        std::vector<double> h(n);
        LGF_HIP(hipMemcpyAsync(h.data(), x0, n * 8, hipMemcpyDeviceToHost, st));
        LGF_HIP(hipStreamSynchronize(st));
        use_x0 = true;
        for (double v : h)
            if (!std::isfinite(v)) {
                use_x0 = false;
                break;
            }
    }
    double rr;
    if (use_x0) {
        LGF_HIP(hipMemcpyAsync(x, x0, n * 8, hipMemcpyDeviceToDevice, st));
        if ((rc = matvec(sys, LGF_F64, x, tmp, st))) return rc;
        hipLaunchKernelGGL(k_sub, dim3(gb), dim3(256), 0, st, r, b, tmp, n);
        if ((rc = dot(sys, r, r, 2, st)) || (rc = read_scal(sys, 2, &rr, st))) return rc;
        S->restarts++;
        if (!(sqrt(rr) <= bnorm)) use_x0 = false;
    }
    if (!use_x0) {
        S->fallback = x0 ? 1 : 0;
        LGF_HIP(hipMemsetAsync(x, 0, n * 8, st));
        LGF_HIP(hipMemcpyAsync(r, b, n * 8, hipMemcpyDeviceToDevice, st));
        rr = bb;
    }
    // CG; with an FP32 matvec the recursive residual drifts from the true one,
    // so each sweep stops after reducing it by 1e-4 (or reaching the target),
    // and the next sweep restarts from the FP64 true residual.  The recursive
    // residual of iteration j is copied to pinned memory and read by the host
    // while iteration j+1 is already queued, so the device never waits for
    // the convergence test.
    const double target = rtol * bnorm;
    double true_r = sqrt(rr);
    int it = 0;
    double rsn = rr;
    while (true_r > target && it < maxit) {
        const double sweep_stop = prec == LGF_F64 ? target : std::max(target * 0.5, true_r * 1e-4);
        LGF_HIP(hipMemcpyAsync(p, r, n * 8, hipMemcpyDeviceToDevice, st));
        if ((rc = dot(sys, r, r, 6, st))) return rc;
        bool graphs = false;
        if ((rc = cg_graphs(sys, prec, st, &graphs))) return rc;
        if (graphs) S->graphs = 1;
        int j = 0;
        bool stop = false;
        while (!stop && it < maxit) {
            if (graphs) {
                LGF_HIP(hipGraphLaunch(sys->cg_exec[prec == LGF_F64 ? 1 : 0][j & 1], st));
            } else if ((rc = cg_iteration(sys, prec, j & 1, st))) {
                return rc;
            }
            LGF_HIP(hipEventRecord(sys->ev[j & 1], st));
            ++it;
            ++j;
            if (j >= 2) {   // test iteration j-2 (0-based) while j-1 runs
                LGF_HIP(hipEventSynchronize(sys->ev[j & 1]));
                rsn = sys->host_scal[8 + (j & 1)];
                if (sqrt(rsn) <= sweep_stop || !std::isfinite(rsn)) stop = true;
            }
        }
        // the last queued iteration's residual
        LGF_HIP(hipEventSynchronize(sys->ev[(j - 1) & 1]));
        rsn = sys->host_scal[8 + ((j - 1) & 1)];
        if (prec == LGF_F64) {
            true_r = sqrt(rsn);
        } else {
            if ((rc = matvec(sys, LGF_F64, x, tmp, st))) return rc;
            hipLaunchKernelGGL(k_sub, dim3(gb), dim3(256), 0, st, r, b, tmp, n);
            if ((rc = dot(sys, r, r, 2, st)) || (rc = read_scal(sys, 2, &rr, st))) return rc;
            S->restarts++;
            true_r = sqrt(rr);
        }
        if (!std::isfinite(true_r)) break;
    }
    // final FP64 true residual (for the FP64 path too, so the report is exact)
    if (prec == LGF_F64) {
        if ((rc = matvec(sys, LGF_F64, x, tmp, st))) return rc;
        hipLaunchKernelGGL(k_sub, dim3(gb), dim3(256), 0, st, tmp, b, tmp, n);
        if ((rc = dot(sys, tmp, tmp, 4, st)) || (rc = read_scal(sys, 4, &rr, st))) return rc;
        true_r = sqrt(rr);
    }
    LGF_HIP(hipMemcpyAsync(f, x, n * 8, hipMemcpyDeviceToDevice, st));
    LGF_HIP(hipEventRecord(e1, st));
    LGF_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LGF_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    S->iterations = it;
    S->rel_residual = true_r / bnorm;
    S->ms = ms;
    if (!(true_r <= target)) {
        char msg[128];
        snprintf(msg, sizeof msg, "ib_force_solve: relative residual %.3e after %d iterations", true_r / bnorm, it);
        return fail(LGFIB_ENOCONV, msg);
    }
    return LGFIB_OK;
}

// ------------------------------------------------------------ Stokes driver
//
// One integrating-factor Euler step (one-stage IF-HERK with a11 = c1 = 1,
// H = E(a), nonlinear term omitted) of the discrete Stokes equations with a
// rigid immersed surface, by the nested projection of Sec. 3.1:
//   (ip)  d* = L^{-1}(-G^T u_k)
//   (f)   C f = I H [u_k - G d*] - u_B(t_{k+1})
//   (pc)  d  = d* + L^{-1} G^T R f
//   (vc)  u_{k+1} = H [u_k - G d - R f]
// (in (f) the faces u_k - G d* are read as the face field that H acts on).
// Velocities live on the flow blocks D_flow (which hold D_body).  The cell
// variables live on D_flow and its lower neighbours (every block b - (i,j,k),
// i,j,k in {0,1}): the divergence of a face field on D_flow reaches the layer
// of cells below its lower faces, and the gradient at those faces reads it,
// so u - G d is the unbounded lattice's projection restricted to D_flow (a
// non-expansive step).  The force solve uses the body system.  Lattice
// units, FP64 state.

struct ib_flow {
    lgfib_ctx *ctx = nullptr;
    ib_system *sys = nullptr;
    int B = 0, nflow = 0, ncell = 0;
    std::vector<int32_t> blocks;    // D_flow (faces)
    std::vector<int32_t> cblocks;   // cell blocks
    std::shared_ptr<IbPlan> plan;   // markers binned on the flow blocks (held: pinned in the cache)
    int clo[3] = {0, 0, 0}, cnb[3] = {0, 0, 0};
    DevBuf cmap, cblk;              // block map of the cell blocks
    lgf_table_t tbl = -1;           // G_L over the cell span
    DevBuf c, dstar, dd, w, h, rhs;
};

namespace lgfib {
__global__ void k_flow_rhs(double *__restrict__ b, const double *__restrict__ v, const double *__restrict__ ub,
                           size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = v[t] - ub[t];
}
__global__ void k_add(double *__restrict__ y, const double *__restrict__ x, double a, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

// face (block slot in F, local cell) of cell n's k-face, or -1 if absent
__device__ inline long face_index(const BlockMapDev &F, int nF, int k, int nx, int ny, int nz) {
    const int B = F.B;
    const int bx = fdiv(nx, B), by = fdiv(ny, B), bz = fdiv(nz, B);
    const int sl = F.slot(bx, by, bz);
    if (sl < 0) return -1;
    return ((long)k * nF + sl) * B * B * B + ((nz - bz * B) * B + (ny - by * B)) * B + (nx - bx * B);
}

// c(n) = sc sum_k u^(k)(n) - u^(k)(n + e_k) on the cell blocks A; faces u on
// the flow blocks F (zero elsewhere)
__global__ void k_div_cross(BlockMapDev F, BlockMapDev A, const double *__restrict__ u, double *__restrict__ c,
                            int nF, int nA, double sc) {
    const int B = A.B, B3 = B * B * B;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nA * B3) return;
    const int b = (int)(t / B3), cell = (int)(t % B3);
    const int nx = A.blocks[3 * b] * B + cell % B, ny = A.blocks[3 * b + 1] * B + (cell / B) % B,
              nz = A.blocks[3 * b + 2] * B + cell / (B * B);
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const long i0 = face_index(F, nF, k, nx, ny, nz);
        const long i1 = face_index(F, nF, k, nx + (k == 0), ny + (k == 1), nz + (k == 2));
        if (i0 >= 0) s += u[i0];
        if (i1 >= 0) s -= u[i1];
    }
    c[t] = sc * s;
}

// e^(k)(n) += sc (d(n) - d(n - e_k)) for faces on F; d on the cell blocks A
__global__ void k_grad_cross(BlockMapDev F, BlockMapDev A, const double *__restrict__ d, double *__restrict__ e,
                             int nF, double sc) {
    const int B = F.B, B3 = B * B * B;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nF * B3) return;
    const int b = (int)(t / B3), cell = (int)(t % B3);
    const int lx = cell % B, ly = (cell / B) % B, lz = cell / (B * B);
    const int bx = F.blocks[3 * b], by = F.blocks[3 * b + 1], bz = F.blocks[3 * b + 2];
    const int sa = A.slot(bx, by, bz);   // every flow block is a cell block
    const double dc = d[(size_t)sa * B3 + cell];
    for (int k = 0; k < 3; ++k) {
        const int nx = bx * B + lx - (k == 0), ny = by * B + ly - (k == 1), nz = bz * B + lz - (k == 2);
        const int cbx = fdiv(nx, B), cby = fdiv(ny, B), cbz = fdiv(nz, B);
        const int sb = A.slot(cbx, cby, cbz);
        const double dm = sb >= 0 ? d[(size_t)sb * B3 + ((nz - cbz * B) * B + (ny - cby * B)) * B + (nx - cbx * B)] : 0.0;
        e[((size_t)k * nF + b) * B3 + cell] += sc * (dc - dm);
    }
}
}  // namespace lgfib

extern "C" int ib_flow_create(lgfib_ctx *ctx, ib_system *sys, const int32_t *flow_blocks, int nflow,
                              ib_flow **out) {
    if (!out) return fail(LGFIB_EINVAL, "ib_flow_create: null output");
    *out = nullptr;
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_flow_create: bad context or system");
    if (nflow < 1 || !flow_blocks) return fail(LGFIB_EINVAL, "ib_flow_create: need flow blocks");
    LGF_HIP(hipSetDevice(ctx->device));
    int rc = validate_blocks(flow_blocks, nflow, "flow blocks");
    if (rc) return rc;
    // D_body must be contained in D_flow
    {
        std::unordered_map<uint64_t, int> in;
        auto key = [](const int32_t *b) {
            return ((uint64_t)(uint32_t)(b[0] + (1 << 20))) | ((uint64_t)(uint32_t)(b[1] + (1 << 20)) << 21) |
                   ((uint64_t)(uint32_t)(b[2] + (1 << 20)) << 42);
        };
        for (int i = 0; i < nflow; ++i) in[key(flow_blocks + 3 * i)] = i;
        for (int i = 0; i < sys->nblk; ++i)
            if (!in.count(key(sys->blocks.data() + 3 * i)))
                return fail(LGFIB_EINVAL, "ib_flow_create: a body block is not among the flow blocks");
    }
    auto f = std::make_unique<ib_flow>();
    f->ctx = ctx;
    f->sys = sys;
    f->B = sys->B;
    f->nflow = nflow;
    f->blocks.assign(flow_blocks, flow_blocks + 3 * (size_t)nflow);
    if ((rc = build_ib_plan(ctx, sys->kernel, sys->X.data(), sys->NL, sys->B, flow_blocks, nflow, f->plan)))
        return rc;
    // cell blocks: the flow blocks and their lower neighbours, sorted (z, y, x)
    {
        std::vector<std::array<int32_t, 3>> v;
        v.reserve(8 * (size_t)nflow);
        for (int i = 0; i < nflow; ++i)
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx)
                        v.push_back({flow_blocks[3 * i] - dx, flow_blocks[3 * i + 1] - dy, flow_blocks[3 * i + 2] - dz});
        std::sort(v.begin(), v.end(), [](const std::array<int32_t, 3> &a, const std::array<int32_t, 3> &b) {
            if (a[2] != b[2]) return a[2] < b[2];
            if (a[1] != b[1]) return a[1] < b[1];
            return a[0] < b[0];
        });
        v.erase(std::unique(v.begin(), v.end()), v.end());
        for (auto &b : v) f->cblocks.insert(f->cblocks.end(), b.begin(), b.end());
        f->ncell = (int)v.size();
    }
    if ((rc = validate_blocks(f->cblocks.data(), f->ncell, "cell blocks"))) return rc;
    {
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        for (int i = 0; i < f->ncell; ++i)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], f->cblocks[3 * i + a]);
                hi[a] = std::max(hi[a], f->cblocks[3 * i + a]);
            }
        size_t msize = 1;
        for (int a = 0; a < 3; ++a) {
            f->clo[a] = lo[a];
            f->cnb[a] = hi[a] - lo[a] + 1;
            msize *= (size_t)f->cnb[a];
        }
        if (msize > (size_t)1 << 28) return fail(LGFIB_ERANGE, "ib_flow_create: flow blocks span too large a box");
        std::vector<int32_t> map(msize, -1);
        for (int i = 0; i < f->ncell; ++i)
            map[((size_t)(f->cblocks[3 * i + 2] - lo[2]) * f->cnb[1] + (f->cblocks[3 * i + 1] - lo[1])) * f->cnb[0] +
                (f->cblocks[3 * i] - lo[0])] = i;
        if ((rc = f->cmap.reserve(map.size() * 4)) || (rc = f->cblk.reserve(f->cblocks.size() * 4))) return rc;
        LGF_HIP(hipMemcpy(f->cmap.p, map.data(), map.size() * 4, hipMemcpyHostToDevice));
        LGF_HIP(hipMemcpy(f->cblk.p, f->cblocks.data(), f->cblocks.size() * 4, hipMemcpyHostToDevice));
    }
    int ext[3];
    for (int q = 0; q < 3; ++q) ext[q] = f->cnb[q] * sys->B - 1;
    if ((rc = lgf_table_build(ctx, LGF_KIND_L, 0.0, ext, nullptr, &f->tbl))) return rc;
    const size_t B3 = (size_t)sys->B * sys->B * sys->B;
    const size_t nfc = (size_t)nflow * B3, ncc = (size_t)f->ncell * B3;
    if ((rc = f->c.reserve(ncc * 8)) || (rc = f->dstar.reserve(ncc * 8)) || (rc = f->dd.reserve(ncc * 8)) ||
        (rc = f->w.reserve(3 * nfc * 8)) || (rc = f->h.reserve(3 * nfc * 8)) ||
        (rc = f->rhs.reserve(3 * (size_t)sys->NL * 8)))
        return rc;
    *out = f.release();
    return LGFIB_OK;
}

extern "C" void ib_flow_destroy(ib_flow *flow) {
    if (!flow) return;
    (void)hipSetDevice(flow->ctx->device);
    (void)hipDeviceSynchronize();
    delete flow;
}

namespace lgfib {
__global__ void k_sum2(double *__restrict__ y, const double *__restrict__ a, const double *__restrict__ b, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = a[t] + b[t];
}
__global__ void k_scale(double *__restrict__ y, const double *__restrict__ x, double a, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = a * x[t];
}
}  // namespace lgfib

// One stage system H^{-1} u' + Q lam = u, Q^T u' = (0, u_B) by the nested
// projection; u is the right-hand side on entry and u' on return; qlam
// (nullable, faces) receives Q lam = G d + R f.
static int flow_stage(lgfib_ctx *ctx, ib_flow *fl, double *u, const double *ub, double *f, const double *x0,
                      double rtol, int maxit, int prec, ib_solve_stats_t *stats, double *b_out, double *qlam,
                      hipStream_t st) {
    ib_system *sys = fl->sys;
    const IbPlan &P = *fl->plan;
    const int B = fl->B;
    const size_t B3 = (size_t)B * B * B;
    const size_t nfc = (size_t)fl->nflow * B3, nf = 3 * nfc, ncc = (size_t)fl->ncell * B3, nl = 3 * (size_t)sys->NL;
    double *c = fl->c.as<double>(), *dstar = fl->dstar.as<double>(), *dd = fl->dd.as<double>();
    double *w = fl->w.as<double>(), *h = fl->h.as<double>(), *rhs = fl->rhs.as<double>();
    const int32_t *bl = fl->blocks.data(), *cb = fl->cblocks.data();
    const int nb = fl->nflow, nc = fl->ncell;
    const BlockMapDev Fm = devmap(P);
    BlockMapDev Am;
    Am.lo0 = fl->clo[0];
    Am.lo1 = fl->clo[1];
    Am.lo2 = fl->clo[2];
    Am.nb0 = fl->cnb[0];
    Am.nb1 = fl->cnb[1];
    Am.nb2 = fl->cnb[2];
    Am.B = B;
    Am.map = fl->cmap.as<int>();
    Am.blocks = fl->cblk.as<int>();
    int rc;
    // (ip) d* = L^{-1}(-G^T u)
    hipLaunchKernelGGL(k_div_cross, dim3(nblocks(ncc, 256)), dim3(256), 0, st, Fm, Am, (const double *)u, c, nb, nc,
                       -1.0);
    LGF_HIP(hipGetLastError());
    if ((rc = lgf_poisson_apply(ctx, fl->tbl, B, cb, nc, cb, nc, 1, LGF_F64, 1.0, c, dstar, 0, (lgfib_stream_t)st))) return rc;
    // (f) b = I E(a)[u - G d*] - u_B ;  C f = b
    LGF_HIP(hipMemcpyAsync(w, u, nf * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_grad_cross, dim3(nblocks(nfc, 256)), dim3(256), 0, st, Fm, Am, (const double *)dstar, w, nb,
                       -1.0);
    LGF_HIP(hipGetLastError());
    if ((rc = lgf_if_apply(ctx, sys->a, B, bl, nb, bl, nb, 3, LGF_F64, w, h, (lgfib_stream_t)st))) return rc;
    if ((rc = launch_interpolate<double, double>(ctx, P, h, rhs, st))) return rc;
    hipLaunchKernelGGL(k_flow_rhs, dim3(nblocks(nl, 256)), dim3(256), 0, st, rhs, rhs, ub, nl);
    LGF_HIP(hipGetLastError());
    if (b_out) LGF_HIP(hipMemcpyAsync(b_out, rhs, nl * 8, hipMemcpyDeviceToDevice, st));
    rc = ib_force_solve(ctx, sys, prec, rhs, f, x0, rtol, maxit, stats, (lgfib_stream_t)st);
    if (rc && rc != LGFIB_ENOCONV) return rc;
    const int solve_rc = rc;
    // (pc) d = d* + L^{-1} G^T R f
    if ((rc = launch_regularize<double, double>(ctx, P, 1.0, f, w, st))) return rc;   // w = R f
    hipLaunchKernelGGL(k_div_cross, dim3(nblocks(ncc, 256)), dim3(256), 0, st, Fm, Am, (const double *)w, c, nb, nc,
                       1.0);
    LGF_HIP(hipGetLastError());
    if ((rc = lgf_poisson_apply(ctx, fl->tbl, B, cb, nc, cb, nc, 1, LGF_F64, 1.0, c, dd, 0, (lgfib_stream_t)st))) return rc;
    hipLaunchKernelGGL(k_add, dim3(nblocks(ncc, 256)), dim3(256), 0, st, dstar, dd, 1.0, ncc);   // d* := d
    LGF_HIP(hipGetLastError());
    // (vc) u = E(a)[u - G d - R f]
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, w, u, -1.0, nf);   // w = R f - u
    LGF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_cross, dim3(nblocks(nfc, 256)), dim3(256), 0, st, Fm, Am, (const double *)dstar, w, nb,
                       1.0);                                                              // w += G d
    LGF_HIP(hipGetLastError());
    if (qlam) {   // Q lam = G d + R f = w + u
        hipLaunchKernelGGL(k_sum2, dim3(nblocks(nf, 256)), dim3(256), 0, st, qlam, (const double *)w, (const double *)u,
                           nf);
        LGF_HIP(hipGetLastError());
    }
    if ((rc = lgf_if_apply(ctx, sys->a, B, bl, nb, bl, nb, 3, LGF_F64, w, h, (lgfib_stream_t)st))) return rc;
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, u, u, -1.0, nf);     // u = 0
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, u, h, -1.0, nf);     // u = -E(w)
    LGF_HIP(hipGetLastError());
    LGF_HIP(hipStreamSynchronize(st));
    return solve_rc;
}

extern "C" int ib_flow_step(lgfib_ctx *ctx, ib_flow *fl, double *u, const double *ub, double *f, const double *x0,
                            double rtol, int maxit, int prec, ib_solve_stats_t *stats, double *b_out,
                            lgfib_stream_t stream) {
    if (!ctx || !fl || fl->ctx != ctx) return fail(LGFIB_EINVAL, "ib_flow_step: bad context or flow");
    if (!u || !ub || !f) return fail(LGFIB_EINVAL, "ib_flow_step: null vector");
    LGF_HIP(hipSetDevice(ctx->device));
    return flow_stage(ctx, fl, u, ub, f, x0, rtol, maxit, prec, stats, b_out, nullptr, (hipStream_t)stream);
}

// Columns j0 .. j0+K-1 of C in one pass (FP64): the operator of
// schur_apply_t on K unit vectors, with the integrating factor applied to
// the 3K face components and the K^{-1} convolution to the K cell fields in
// shared launches (each component is transformed on its own, so the columns
// are those of K separate applications).
static constexpr int kDenseCols = 8;
static int schur_dense_cols(ib_system *s, int j0, int K, double *C, long ld, hipStream_t st) {
    lgfib_ctx *ctx = s->ctx;
    const IbPlan &P = *s->plan;
    const int n = 3 * s->NL;
    const size_t nc = (size_t)s->nblk * s->B * s->B * s->B, nf = 3 * nc;
    double *base = s->dense_cols.as<double>();
    double *g = base, *af = g + kDenseCols * nf, *c = af + kDenseCols * nf, *d = c + kDenseCols * nc;
    double *e = d + kDenseCols * nc, *y = e + (size_t)kDenseCols * n;
    int rc;
    for (int k = 0; k < K; ++k) {
        hipLaunchKernelGGL(k_unit, dim3(nblocks(n, 256)), dim3(256), 0, st, e + (size_t)k * n, n, j0 + k);
        LGF_HIP(hipGetLastError());
        if ((rc = launch_regularize<double, double>(ctx, P, 1.0, e + (size_t)k * n, g + k * nf, st))) return rc;
        if ((rc = launch_grad_adjoint<double>(ctx, P, g + k * nf, c + k * nc, st))) return rc;
    }
    for (int c0 = 0; c0 < 3 * K; c0 += 8) {
        const int m = std::min(8, 3 * K - c0);
        if ((rc = lgf_if_apply(ctx, s->a, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, m, LGF_F64,
                               g + c0 * nc, af + c0 * nc, (lgfib_stream_t)st)))
            return rc;
    }
    if ((rc = lgf_poisson_apply(ctx, s->tbl, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, K, LGF_F64,
                                1.0, c, d, 0, (lgfib_stream_t)st)))
        return rc;
    for (int k = 0; k < K; ++k) {
        if ((rc = launch_grad_acc<double>(ctx, P, d + k * nc, af + k * nf, st))) return rc;
        if ((rc = launch_interpolate<double, double>(ctx, P, af + k * nf, y + (size_t)k * n, st))) return rc;
        hipLaunchKernelGGL(k_put_column, dim3(nblocks(n, 256)), dim3(256), 0, st, C, ld, j0 + k,
                           (const double *)(y + (size_t)k * n), n);
        LGF_HIP(hipGetLastError());
    }
    return LGFIB_OK;
}

extern "C" int ib_schur_dense(lgfib_ctx *ctx, ib_system *sys, double *C, int ld, lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_schur_dense: bad context or system");
    const int n = 3 * sys->NL;
    if (!C || ld < n) return fail(LGFIB_EINVAL, "ib_schur_dense: null matrix or ld < 3 NL");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t nc = (size_t)sys->nblk * sys->B * sys->B * sys->B;
    int rc;
    if ((rc = sys->dense_cols.reserve(((size_t)kDenseCols * (8 * nc + 2 * (size_t)n)) * sizeof(double)))) return rc;
    for (int j = 0; j < n; j += kDenseCols)
        if ((rc = schur_dense_cols(sys, j, std::min(kDenseCols, n - j), C, (long)ld, st))) return rc;
    LGF_HIP(hipStreamSynchronize(st));
    return LGFIB_OK;
}

extern "C" int ib_system_factor(lgfib_ctx *ctx, ib_system *sys, int enable, lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_system_factor: bad context or system");
    LGF_HIP(hipSetDevice(ctx->device));
    if (!enable) {
        sys->factored = false;
        sys->wfac.release();
        return LGFIB_OK;
    }
    const size_t n = 3 * (size_t)sys->NL;
    if (n > 46000) return fail(LGFIB_EINVAL, "ib_system_factor: more than 46000 unknowns");
    sys->factored = false;
    DevBuf C;
    int rc;
    if ((rc = C.reserve(n * n * 8)) || (rc = sys->wfac.reserve(n * n * 8))) return rc;
    if ((rc = ib_schur_dense(ctx, sys, C.as<double>(), (int)n, stream))) return rc;
    if ((rc = chol_factor_f64(ctx, (int)n, C.as<double>(), (long)n, sys->wfac.as<double>(), (long)n,
                              (hipStream_t)stream)))
        return rc;
    sys->factored = true;
    return LGFIB_OK;
}

// ------------------------------------------------------------- IF-HERK step

struct ib_herk {
    lgfib_ctx *ctx = nullptr;
    int s = 0, NL = 0, B = 0, nflow = 0;
    double A = 0.0;
    bool direct = false, have_prev = false;
    std::vector<double> at, ct, stage_a;   // shifted tableau, nodes, H parameter of each stage
    std::vector<ib_system *> systems;      // one per distinct stage parameter (owned)
    std::vector<ib_flow *> flows;
    std::vector<int> stage_k;              // system / flow of each stage
    std::vector<int32_t> fblocks;
    double conv_dt = 0.0;                  // dt / dx of the nonlinear term (0: Stokes)
    double U[3] = {0.0, 0.0, 0.0};         // frame velocity in u_a = u + U
    DevBuf fields;   // (s + 4) face fields: h, tmp, r, Q lam - g of each stage, g
    DevBuf forces;   // (s + 1) marker vectors: stage force, previous step's stage forces
};

extern "C" void ib_herk_destroy(ib_herk *hk) {
    if (!hk) return;
    for (auto *fl : hk->flows) ib_flow_destroy(fl);
    for (auto *sy : hk->systems) ib_system_destroy(sy);
    delete hk;
}

extern "C" int ib_herk_tableau(int scheme, int *s, double *at, double *ct) {
    if (!s || !at || !ct || scheme < 0 || scheme > 3) return fail(LGFIB_EINVAL, "ib_herk_tableau: bad argument");
    const double r3 = std::sqrt(3.0);
    // explicit tableaus (A, b, c) of App. B; the shifted form is
    // at_{ij} = A_{i+1,j} (i < s), at_{sj} = b_j, ct_i = c_{i+1}, ct_s = 1
    static const int ns[4] = {3, 3, 3, 4};
    double Am[4][4] = {}, b[4] = {}, c[4] = {};
    switch (scheme) {
    case 0:
        Am[1][0] = 0.5;
        Am[2][0] = r3 / 3, Am[2][1] = (3 - r3) / 3;
        b[0] = (3 + r3) / 6, b[1] = -r3 / 3, b[2] = (3 + r3) / 6;
        c[1] = 0.5, c[2] = 1.0;
        break;
    case 1:
        Am[1][0] = 1.0 / 3;
        Am[2][0] = -1.0, Am[2][1] = 2.0;
        b[1] = 0.75, b[2] = 0.25;
        c[1] = 1.0 / 3, c[2] = 1.0;
        break;
    case 2:
        Am[1][0] = 8.0 / 15;
        Am[2][0] = 0.25, Am[2][1] = 5.0 / 12;
        b[0] = 0.25, b[2] = 0.75;
        c[1] = 8.0 / 15, c[2] = 2.0 / 3;
        break;
    default:   // the classical four-stage method
        Am[1][0] = 0.5;
        Am[2][1] = 0.5;
        Am[3][2] = 1.0;
        b[0] = 1.0 / 6, b[1] = 1.0 / 3, b[2] = 1.0 / 3, b[3] = 1.0 / 6;
        c[1] = 0.5, c[2] = 0.5, c[3] = 1.0;
        break;
    }
    const int n = ns[scheme];
    *s = n;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) at[i * n + j] = i + 1 < n ? Am[i + 1][j] : b[j];
        ct[i] = i + 1 < n ? c[i + 1] : 1.0;
    }
    return LGFIB_OK;
}

extern "C" int ib_herk_create(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *body_blocks,
                              int nbody, const int32_t *flow_blocks, int nflow, double A, int s, const double *at,
                              const double *ct, int direct, ib_herk **out) {
    if (!out) return fail(LGFIB_EINVAL, "ib_herk_create: null output");
    *out = nullptr;
    if (!ctx || !at || !ct || !flow_blocks || nflow < 1) return fail(LGFIB_EINVAL, "ib_herk_create: bad argument");
    if (s < 1 || s > 8) return fail(LGFIB_EINVAL, "ib_herk_create: s must lie in [1, 8]");
    if (!(A >= 0.0) || A > 4.0) return fail(LGFIB_EINVAL, "ib_herk_create: A must lie in [0, 4]");
    double prev = 0.0;
    for (int i = 0; i < s; ++i) {
        if (!(ct[i] >= prev) || ct[i] > 1.0) return fail(LGFIB_EINVAL, "ib_herk_create: nodes must be nondecreasing in [0, 1]");
        if (!(std::fabs(at[i * s + i]) > 0.0)) return fail(LGFIB_EINVAL, "ib_herk_create: zero diagonal coefficient");
        for (int j = i + 1; j < s; ++j)
            if (at[i * s + j] != 0.0) return fail(LGFIB_EINVAL, "ib_herk_create: tableau must be lower triangular");
        prev = ct[i];
    }
    auto hk = std::unique_ptr<ib_herk, void (*)(ib_herk *)>(new ib_herk, ib_herk_destroy);
    hk->ctx = ctx;
    hk->s = s;
    hk->NL = NL;
    hk->B = B;
    hk->nflow = nflow;
    hk->A = A;
    hk->direct = direct != 0;
    hk->at.assign(at, at + s * s);
    hk->ct.assign(ct, ct + s);
    hk->fblocks.assign(flow_blocks, flow_blocks + 3 * (size_t)nflow);
    int rc;
    prev = 0.0;
    for (int i = 0; i < s; ++i) {
        const double a = (ct[i] - prev) * A;
        prev = ct[i];
        hk->stage_a.push_back(a);
        int k = -1;
        for (int q = 0; q < i; ++q)
            if (std::fabs(hk->stage_a[q] - a) <= 1e-14 * std::max(1.0, std::fabs(a))) k = hk->stage_k[q];
        if (k < 0) {
            ib_system *sy = nullptr;
            if ((rc = ib_system_create(ctx, kernel, X, NL, B, body_blocks, nbody, a, &sy))) return rc;
            hk->systems.push_back(sy);
            if (hk->direct && (rc = ib_system_factor(ctx, sy, 1, nullptr))) return rc;
            ib_flow *fl = nullptr;
            if ((rc = ib_flow_create(ctx, sy, flow_blocks, nflow, &fl))) return rc;
            hk->flows.push_back(fl);
            k = (int)hk->systems.size() - 1;
        }
        hk->stage_k.push_back(k);
    }
    const size_t nf = 3 * (size_t)nflow * B * B * B, nl = 3 * (size_t)NL;
    if ((rc = hk->fields.reserve((size_t)(s + 4) * nf * 8)) || (rc = hk->forces.reserve((size_t)(s + 1) * nl * 8)))
        return rc;
    *out = hk.release();
    return LGFIB_OK;
}

extern "C" int ib_herk_step(lgfib_ctx *ctx, ib_herk *hk, double *u, const double *ub, double *f, double rtol,
                            int maxit, int prec, ib_solve_stats_t *stats, lgfib_stream_t stream) {
    if (!ctx || !hk || hk->ctx != ctx) return fail(LGFIB_EINVAL, "ib_herk_step: bad context or step");
    if (!u || !ub || !f) return fail(LGFIB_EINVAL, "ib_herk_step: null vector");
    if (!hk->direct && prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "ib_herk_step: bad prec");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int s = hk->s, B = hk->B, nb = hk->nflow;
    const size_t nf = 3 * (size_t)nb * B * B * B, nl = 3 * (size_t)hk->NL;
    const int32_t *bl = hk->fblocks.data();
    double *base = hk->fields.as<double>();
    double *h = base, *tmp = base + nf, *r = base + 2 * nf;
    std::vector<double *> q(s);
    for (int j = 0; j < s; ++j) q[j] = base + (3 + j) * nf;
    double *g = base + (3 + s) * nf;
    const bool conv = hk->conv_dt > 0.0;
    const double *ustage = u;   // u^{i-1}: the step's input, then each stage's solution (left in r)
    double *fst = hk->forces.as<double>();
    if (stats) *stats = ib_solve_stats_t{};
    int rc, solve_rc = LGFIB_OK;
    LGF_HIP(hipMemcpyAsync(h, u, nf * 8, hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < s; ++i) {
        const double ap = i > 0 ? hk->stage_a[i - 1] : 0.0;
        if (ap > 0.0) {   // h <- H^{i-1} h, Q lam^j <- H^{i-1} Q lam^j
            if ((rc = lgf_if_apply(ctx, ap, B, bl, nb, bl, nb, 3, LGF_F64, h, tmp, stream))) return rc;
            std::swap(h, tmp);
            for (int j = 0; j < i; ++j) {
                if ((rc = lgf_if_apply(ctx, ap, B, bl, nb, bl, nb, 3, LGF_F64, q[j], tmp, stream))) return rc;
                std::swap(q[j], tmp);
            }
        }
        // g^i = -at_ii dt N~(u^{i-1}) (Eq. ibifherk_g), before r is overwritten
        if (conv && (rc = lamb_apply(ctx, B, bl, nb, hk->U, -hk->at[i * s + i] * hk->conv_dt, LGF_F64, ustage, g, st)))
            return rc;
        // r = h - sum_j (at_ij / at_jj) (Q lam^j - g^j) + g^i
        LGF_HIP(hipMemcpyAsync(r, h, nf * 8, hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < i; ++j) {
            const double cij = -hk->at[i * s + j] / hk->at[j * s + j];
            if (cij == 0.0) continue;
            hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, r, (const double *)q[j], cij, nf);
            LGF_HIP(hipGetLastError());
        }
        if (conv) {
            hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, r, (const double *)g, 1.0, nf);
            LGF_HIP(hipGetLastError());
        }
        double *fprev = fst + (1 + i) * nl;
        ib_solve_stats_t si{};
        rc = flow_stage(ctx, hk->flows[hk->stage_k[i]], r, ub + i * nl, fst,
                        (!hk->direct && hk->have_prev) ? fprev : nullptr, rtol, maxit,
                        hk->direct ? IB_SOLVE_DIRECT : prec, &si, nullptr, q[i], st);
        if (rc && rc != LGFIB_ENOCONV) return rc;
        if (rc) solve_rc = rc;
        if (conv) {   // the propagated field of this stage is Q lam^i - g^i
            hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, q[i], (const double *)g, -1.0, nf);
            LGF_HIP(hipGetLastError());
        }
        ustage = r;
        LGF_HIP(hipMemcpyAsync(fprev, fst, nl * 8, hipMemcpyDeviceToDevice, st));
        if (stats) {
            stats->iterations += si.iterations;
            stats->restarts += si.restarts;
            stats->fallback += si.fallback;
            stats->ms += si.ms;
            stats->graphs = si.graphs;
            stats->rel_residual = std::max(stats->rel_residual, si.rel_residual);
        }
    }
    LGF_HIP(hipMemcpyAsync(u, r, nf * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_scale, dim3(nblocks(nl, 256)), dim3(256), 0, st, f, (const double *)fst,
                       1.0 / hk->at[(s - 1) * s + s - 1], nl);
    LGF_HIP(hipGetLastError());
    LGF_HIP(hipStreamSynchronize(st));
    hk->have_prev = true;
    return solve_rc;
}

extern "C" int ib_herk_convection(lgfib_ctx *ctx, ib_herk *hk, double dt, const double *U) {
    if (!ctx || !hk || hk->ctx != ctx) return fail(LGFIB_EINVAL, "ib_herk_convection: bad context or step");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(LGFIB_EINVAL, "ib_herk_convection: dt must be finite and >= 0");
    if (U && !(std::isfinite(U[0]) && std::isfinite(U[1]) && std::isfinite(U[2])))
        return fail(LGFIB_EINVAL, "ib_herk_convection: non-finite frame velocity");
    hk->conv_dt = dt;
    for (int a = 0; a < 3; ++a) hk->U[a] = U ? U[a] : 0.0;
    return LGFIB_OK;
}

namespace lgfib {
// g <- g / gamma where gamma != 0, else 0
__global__ void k_div_guard(double *__restrict__ g, const double *__restrict__ gamma, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) g[t] = gamma[t] != 0.0 ? g[t] / gamma[t] : 0.0;
}
__global__ void k_fill(double *__restrict__ y, double v, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = v;
}
}  // namespace lgfib

extern "C" int ib_force_smooth(lgfib_ctx *ctx, ib_system *sys, const double *f, double *fhat, lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_force_smooth: bad context or system");
    if (!f || !fhat) return fail(LGFIB_EINVAL, "ib_force_smooth: null vector");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const IbPlan &P = *sys->plan;
    const size_t nf = 3 * (size_t)sys->nblk * sys->B * sys->B * sys->B, nl = 3 * (size_t)sys->NL;
    int rc;
    if (!sys->gamma.p) {   // gamma = R 1
        if ((rc = sys->gamma.reserve(nf * 8))) return rc;
        double *ones = sys->tmp.as<double>();
        hipLaunchKernelGGL(k_fill, dim3(nblocks(nl, 256)), dim3(256), 0, st, ones, 1.0, nl);
        LGF_HIP(hipGetLastError());
        if ((rc = launch_regularize<double, double>(ctx, P, 1.0, ones, sys->gamma.as<double>(), st))) return rc;
    }
    double *g = sys->g[1].as<double>();
    if ((rc = launch_regularize<double, double>(ctx, P, 1.0, f, g, st))) return rc;
    hipLaunchKernelGGL(k_div_guard, dim3(nblocks(nf, 256)), dim3(256), 0, st, g, (const double *)sys->gamma.as<double>(),
                       nf);
    LGF_HIP(hipGetLastError());
    return launch_interpolate<double, double>(ctx, P, g, fhat, st);
}
