// ib.hip -- immersed-boundary operators on a block set: discrete delta
// regularization R and interpolation I (Sec. 2.1), the staggered gradient G
// and its adjoint G^T, and the body-block set D_body (Sec. 4.1).
//
// Positions are in lattice units; cell n has centre n + (1/2,1/2,1/2) and its
// k-th face sits at x_F^(k)(n) = n + (1/2,1/2,1/2) - e_k/2.
//
// R is evaluated as a gather: every target block owns the list of markers
// whose delta support touches it (built on the host once per marker set), and
// each thread sums, for its faces, the contributions of that list in index
// order -- deterministic, no atomics.  I is a gather per (marker, component)
// over the marker's 3^3 (or 4^3) support.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
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
    DevBuf blk_ptr;    // int32 [nblk+1]
    DevBuf blk_mk;     // int32 marker indices per block
    DevBuf blocks;     // int32 [nblk][3]
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
    std::unordered_map<uint64_t, std::unique_ptr<IbPlan>> plans;
    std::unordered_map<uint64_t, std::vector<char>> keys;
};

static IbCache &ib_cache(lgfib_ctx *ctx) {
    static std::unordered_map<lgfib_ctx *, std::unique_ptr<IbCache>> caches;
    auto &c = caches[ctx];
    if (!c) c = std::make_unique<IbCache>();
    return *c;
}

static int build_ib_plan(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks, int nblk,
                         IbPlan **out) {
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
            *out = cache.plans[hh].get();
            return LGFIB_OK;
        }
    }
    int rc = validate_blocks(blocks, nblk, "body blocks");
    if (rc) return rc;
    for (int i = 0; i < 3 * NL; ++i)
        if (!std::isfinite(X[i]) || fabs(X[i]) > 1e6) return fail(LGFIB_EINVAL, "marker position not finite or too large");
    auto plan = std::make_unique<IbPlan>();
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
    // per-block marker lists: marker i joins every block its support touches
    std::vector<std::vector<int32_t>> lists(std::max(nblk, 1));
    for (int i = 0; i < NL; ++i) {
        long long blo[3], bhi[3];
        for (int a = 0; a < 3; ++a) {
            blo[a] = 1ll << 40;
            bhi[a] = -(1ll << 40);
        }
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                const double c = (a == k) ? 0.0 : 0.5;
                long long l;
                int cnt;
                support_range(kernel, X[3 * i + a], c, &l, &cnt);
                // only indices with phi != 0 matter; the range covers them
                blo[a] = std::min(blo[a], l);
                bhi[a] = std::max(bhi[a], l + cnt - 1);
            }
        // every support cell must be inside the block set
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
                        if (slot_of(floordiv(n[0], B), floordiv(n[1], B), floordiv(n[2], B)) < 0)
                            return fail(LGFIB_ESUPPORT, "support of marker " + std::to_string(i) +
                                                            " leaves the block set");
                    }
        }
        for (long long bz = floordiv(blo[2], B); bz <= floordiv(bhi[2], B); ++bz)
            for (long long by = floordiv(blo[1], B); by <= floordiv(bhi[1], B); ++by)
                for (long long bx = floordiv(blo[0], B); bx <= floordiv(bhi[0], B); ++bx) {
                    int s = slot_of(bx, by, bz);
                    if (s >= 0) lists[s].push_back(i);
                }
    }
    std::vector<int32_t> ptr(nblk + 1, 0), mk;
    for (int b = 0; b < nblk; ++b) {
        ptr[b + 1] = ptr[b] + (int)lists[b].size();
        mk.insert(mk.end(), lists[b].begin(), lists[b].end());
    }
    if (mk.empty()) mk.push_back(0);
    if ((rc = plan->X.reserve(sizeof(double) * 3 * std::max(NL, 1)))) return rc;
    if ((rc = plan->map.reserve(sizeof(int32_t) * map.size()))) return rc;
    if ((rc = plan->blk_ptr.reserve(sizeof(int32_t) * ptr.size()))) return rc;
    if ((rc = plan->blk_mk.reserve(sizeof(int32_t) * mk.size()))) return rc;
    if ((rc = plan->blocks.reserve(sizeof(int32_t) * 3 * std::max(nblk, 1)))) return rc;
    if (NL) LGF_HIP(hipMemcpy(plan->X.p, X, sizeof(double) * 3 * NL, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->map.p, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->blk_ptr.p, ptr.data(), sizeof(int32_t) * ptr.size(), hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->blk_mk.p, mk.data(), sizeof(int32_t) * mk.size(), hipMemcpyHostToDevice));
    if (nblk) LGF_HIP(hipMemcpy(plan->blocks.p, blocks, sizeof(int32_t) * 3 * nblk, hipMemcpyHostToDevice));
    *out = plan.get();
    cache.keys[h] = std::move(key);
    cache.plans[h] = std::move(plan);
    return LGFIB_OK;
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

// g^(k)(n) = dx^-3 sum_{i in list(block)} x_i^(k) prod_j phi(x_F^(k)(n)_j - X_ij)
template <typename Real, int KERNEL>
__global__ __launch_bounds__(256) void k_regularize(BlockMapDev bm, const double *__restrict__ X,
                                                    const int *__restrict__ ptr, const int *__restrict__ mk,
                                                    const Real *__restrict__ x, Real *__restrict__ faces, int nblk,
                                                    double inv_dx3) {
    constexpr double hw = KERNEL == IB_ROMA3 ? 1.5 : 2.0;
    const int b = blockIdx.x;
    const int B = bm.B, B3 = B * B * B;
    const int o0 = bm.blocks[3 * b] * B, o1 = bm.blocks[3 * b + 1] * B, o2 = bm.blocks[3 * b + 2] * B;
    const int m0 = ptr[b], m1 = ptr[b + 1];
    for (int cell = threadIdx.x; cell < B3; cell += blockDim.x) {
        const int lx = cell % B, ly = (cell / B) % B, lz = cell / (B * B);
        const double cx = o0 + lx + 0.5, cy = o1 + ly + 0.5, cz = o2 + lz + 0.5;
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        for (int q = m0; q < m1; ++q) {
            const int i = mk[q];
            const double rx = cx - X[3 * i], ry = cy - X[3 * i + 1], rz = cz - X[3 * i + 2];
            // face k is shifted by -1/2 along axis k
            if (fabs(rx) >= hw + 0.5 || fabs(ry) >= hw + 0.5 || fabs(rz) >= hw + 0.5) continue;
            const double px = phi_k(KERNEL, rx), py = phi_k(KERNEL, ry), pz = phi_k(KERNEL, rz);
            const double qx = phi_k(KERNEL, rx - 0.5), qy = phi_k(KERNEL, ry - 0.5), qz = phi_k(KERNEL, rz - 0.5);
            acc0 += (double)x[3 * i + 0] * qx * py * pz;
            acc1 += (double)x[3 * i + 1] * px * qy * pz;
            acc2 += (double)x[3 * i + 2] * px * py * qz;
        }
        faces[((size_t)0 * nblk + b) * B3 + cell] = (Real)(acc0 * inv_dx3);
        faces[((size_t)1 * nblk + b) * B3 + cell] = (Real)(acc1 * inv_dx3);
        faces[((size_t)2 * nblk + b) * B3 + cell] = (Real)(acc2 * inv_dx3);
    }
}

// v_i^(k) = sum_n u^(k)(n) prod_j phi(x_F^(k)(n)_j - X_ij)
template <typename Real, int KERNEL>
__global__ void k_interpolate(BlockMapDev bm, const double *__restrict__ X, const Real *__restrict__ faces,
                              Real *__restrict__ v, int NL, int nblk) {
    constexpr double hw = KERNEL == IB_ROMA3 ? 1.5 : 2.0;
    constexpr int S = KERNEL == IB_ROMA3 ? 4 : 5;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * NL) return;
    const int i = t / 3, k = t % 3;
    const int B = bm.B, B3 = B * B * B;
    double w[3][S];
    int lo[3];
    for (int a = 0; a < 3; ++a) {
        const double c = (a == k) ? 0.0 : 0.5;
        const double Xa = X[3 * i + a];
        lo[a] = (int)floor(Xa - c - hw) + 1;
        for (int s = 0; s < S; ++s) w[a][s] = phi_k(KERNEL, (double)(lo[a] + s) + c - Xa);
    }
    double acc = 0.0;
    for (int sz = 0; sz < S; ++sz) {
        if (w[2][sz] == 0.0) continue;
        const int nz = lo[2] + sz, bz = fdiv(nz, B);
        for (int sy = 0; sy < S; ++sy) {
            if (w[1][sy] == 0.0) continue;
            const int ny = lo[1] + sy, by = fdiv(ny, B);
            for (int sx = 0; sx < S; ++sx) {
                if (w[0][sx] == 0.0) continue;
                const int nx = lo[0] + sx, bx = fdiv(nx, B);
                const int slot = bm.slot(bx, by, bz);
                if (slot < 0) continue;   // excluded by the plan's support check
                const size_t idx = ((size_t)k * nblk + slot) * B3 + (size_t)((nz - bz * B) * B + (ny - by * B)) * B +
                                   (nx - bx * B);
                acc += w[2][sz] * w[1][sy] * w[0][sx] * (double)faces[idx];
            }
        }
    }
    v[3 * i + k] = (Real)acc;
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

template <typename Real>
static int launch_regularize(lgfib_ctx *ctx, const IbPlan &p, double dx, const Real *x, Real *faces, hipStream_t st) {
    if (p.nblk == 0) return LGFIB_OK;
    ProfScope ps(ctx, "k_regularize", st);
    const double inv = 1.0 / (dx * dx * dx);
    if (p.kernel == IB_ROMA3)
        hipLaunchKernelGGL((k_regularize<Real, IB_ROMA3>), dim3(p.nblk), dim3(256), 0, st, devmap(p),
                           p.X.as<double>(), p.blk_ptr.as<int>(), p.blk_mk.as<int>(), x, faces, p.nblk, inv);
    else
        hipLaunchKernelGGL((k_regularize<Real, IB_SMOOTH3>), dim3(p.nblk), dim3(256), 0, st, devmap(p),
                           p.X.as<double>(), p.blk_ptr.as<int>(), p.blk_mk.as<int>(), x, faces, p.nblk, inv);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename Real>
static int launch_interpolate(lgfib_ctx *ctx, const IbPlan &p, const Real *faces, Real *v, hipStream_t st) {
    if (p.NL == 0) return LGFIB_OK;
    ProfScope ps(ctx, "k_interpolate", st);
    if (p.kernel == IB_ROMA3)
        hipLaunchKernelGGL((k_interpolate<Real, IB_ROMA3>), dim3(nblocks(3 * (size_t)p.NL, 128)), dim3(128), 0, st,
                           devmap(p), p.X.as<double>(), faces, v, p.NL, p.nblk);
    else
        hipLaunchKernelGGL((k_interpolate<Real, IB_SMOOTH3>), dim3(nblocks(3 * (size_t)p.NL, 128)), dim3(128), 0, st,
                           devmap(p), p.X.as<double>(), faces, v, p.NL, p.nblk);
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
    IbPlan *p = nullptr;
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, &p))) return rc;
    if (prec == LGF_F64)
        return launch_regularize<double>(ctx, *p, dx, (const double *)x, (double *)faces, (hipStream_t)stream);
    return launch_regularize<float>(ctx, *p, dx, (const float *)x, (float *)faces, (hipStream_t)stream);
}

extern "C" int ib_interpolate(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *blocks,
                              int nblk, int prec, double dx, const void *faces, void *v, lgfib_stream_t stream) {
    int rc = ib_check(ctx, kernel, X, NL, B, blocks, nblk, prec, dx, "ib_interpolate");
    if (rc) return rc;
    if ((NL > 0 && !v) || (nblk > 0 && !faces)) return fail(LGFIB_EINVAL, "ib_interpolate: null field pointer");
    LGF_HIP(hipSetDevice(ctx->device));
    IbPlan *p = nullptr;
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, &p))) return rc;
    if (prec == LGF_F64)
        return launch_interpolate<double>(ctx, *p, (const double *)faces, (double *)v, (hipStream_t)stream);
    return launch_interpolate<float>(ctx, *p, (const float *)faces, (float *)v, (hipStream_t)stream);
}

// ---------------------------------------------------------- Schur system

struct ib_system {
    lgfib_ctx *ctx = nullptr;
    int kernel = 0, NL = 0, B = 0, nblk = 0;
    double a = 0.0;
    std::vector<double> X;
    std::vector<int32_t> blocks;
    lgf_table_t tbl = -1;
    IbPlan *plan = nullptr;
    // work fields per precision: faces g, faces a, cells c, cells d
    DevBuf g[2], af[2], c[2], d[2], xv[2], yv[2];
    // CG vectors (FP64)
    DevBuf r, p, ap, x, tmp, red, scal;
    double *host_scal = nullptr;
};

namespace lgfib {

template <typename Real>
static int schur_apply_t(ib_system *s, const Real *x, Real *y, hipStream_t st) {
    lgfib_ctx *ctx = s->ctx;
    const int pi = sizeof(Real) == 8 ? 1 : 0;
    const int prec = pi ? LGF_F64 : LGF_F32;
    const int B3 = s->B * s->B * s->B;
    Real *g = s->g[pi].as<Real>(), *af = s->af[pi].as<Real>(), *c = s->c[pi].as<Real>(), *d = s->d[pi].as<Real>();
    int rc;
    if ((rc = launch_regularize<Real>(ctx, *s->plan, 1.0, x, g, st))) return rc;
    if ((rc = lgf_if_apply(ctx, s->a, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, 3, prec, g, af,
                           (lgfib_stream_t)st)))
        return rc;
    if ((rc = launch_grad_adjoint<Real>(ctx, *s->plan, g, c, st))) return rc;
    if ((rc = lgf_poisson_apply(ctx, s->tbl, s->B, s->blocks.data(), s->nblk, s->blocks.data(), s->nblk, 1, prec, 1.0,
                                c, d, 0, (lgfib_stream_t)st)))
        return rc;
    if ((rc = launch_grad_acc<Real>(ctx, *s->plan, d, af, st))) return rc;
    (void)B3;
    return launch_interpolate<Real>(ctx, *s->plan, af, y, st);
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
    if ((rc = build_ib_plan(ctx, kernel, X, NL, B, blocks, nblk, &s->plan))) return rc;
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
        if ((rc = s->xv[pi].reserve(3 * (size_t)NL * es))) return rc;
        if ((rc = s->yv[pi].reserve(3 * (size_t)NL * es))) return rc;
    }
    const size_t nv = 3 * (size_t)NL * 8;
    if ((rc = s->r.reserve(nv)) || (rc = s->p.reserve(nv)) || (rc = s->ap.reserve(nv)) || (rc = s->x.reserve(nv)) ||
        (rc = s->tmp.reserve(nv)) || (rc = s->red.reserve(4096 * 8)) || (rc = s->scal.reserve(64 * 8)))
        return rc;
    LGF_HIP(hipHostMalloc((void **)&s->host_scal, 64 * sizeof(double), hipHostMallocDefault));
    *out = s.release();
    return LGFIB_OK;
}

extern "C" void ib_system_destroy(ib_system *sys) {
    if (!sys) return;
    (void)hipSetDevice(sys->ctx->device);
    (void)hipDeviceSynchronize();
    if (sys->host_scal) (void)hipHostFree(sys->host_scal);
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
    if (prec == LGF_F64) return schur_apply_t<double>(sys, (const double *)x, (double *)y, (hipStream_t)stream);
    return schur_apply_t<float>(sys, (const float *)x, (float *)y, (hipStream_t)stream);
}

// ------------------------------------------------------ conjugate gradients

namespace lgfib {

constexpr int kRedBlocks = 256;

// partial sums of a.b (fixed order: per-block tree, then one block)
__global__ void k_dot_partial(const double *__restrict__ a, const double *__restrict__ b, size_t n,
                              double *__restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) s += a[i] * b[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_dot_final(const double *__restrict__ part, int np, double *__restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// scal layout: [0] rs, [1] pAp, [2] rs_new, [3] bb, [4] scratch
// x += alpha p ; r -= alpha Ap   with alpha = rs / pAp
__global__ void k_cg_xr(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                        const double *__restrict__ ap, const double *__restrict__ scal, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha = scal[0] / scal[1];
    x[i] += alpha * p[i];
    r[i] -= alpha * ap[i];
}

// p = r + beta p, beta = rs_new / rs ; then rs = rs_new (by thread 0 after use)
__global__ void k_cg_p(double *__restrict__ p, const double *__restrict__ r, const double *__restrict__ scal,
                       size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = scal[2] / scal[0];
    p[i] = r[i] + beta * p[i];
}

__global__ void k_scal_copy(double *scal, int dst, int src) { scal[dst] = scal[src]; }

template <typename To, typename From>
__global__ void k_convert(To *__restrict__ o, const From *__restrict__ i, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) o[t] = (To)i[t];
}

// r = b - y
__global__ void k_sub(double *__restrict__ r, const double *__restrict__ b, const double *__restrict__ y, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) r[t] = b[t] - y[t];
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, double a, size_t n) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

static int dot(ib_system *s, const double *a, const double *b, int slot, hipStream_t st) {
    const size_t n = 3 * (size_t)s->NL;
    const int nb = (int)std::min<size_t>(kRedBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, st, a, b, n, s->red.as<double>());
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, s->red.as<double>(), nb, s->scal.as<double>() + slot);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

static int read_scal(ib_system *s, int slot, double *v, hipStream_t st) {
    LGF_HIP(hipMemcpyAsync(s->host_scal + slot, s->scal.as<double>() + slot, sizeof(double), hipMemcpyDeviceToHost, st));
    LGF_HIP(hipStreamSynchronize(st));
    *v = s->host_scal[slot];
    return LGFIB_OK;
}

// y = C x with an FP64 interface, matvec in prec
static int matvec(ib_system *s, int prec, const double *x, double *y, hipStream_t st) {
    const size_t n = 3 * (size_t)s->NL;
    if (prec == LGF_F64) return schur_apply_t<double>(s, x, y, st);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblocks(n, 256)), dim3(256), 0, st, s->xv[0].as<float>(), x, n);
    int rc = schur_apply_t<float>(s, s->xv[0].as<float>(), s->yv[0].as<float>(), st);
    if (rc) return rc;
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblocks(n, 256)), dim3(256), 0, st, y, s->yv[0].as<float>(), n);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

}  // namespace lgfib

extern "C" int ib_force_solve(lgfib_ctx *ctx, ib_system *sys, int prec, const double *b, double *f, const double *x0,
                              double rtol, int maxit, ib_solve_stats_t *stats, lgfib_stream_t stream) {
    if (!ctx || !sys || sys->ctx != ctx) return fail(LGFIB_EINVAL, "ib_force_solve: bad context or system");
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
    // and the next sweep restarts from the FP64 true residual.
    const double target = rtol * bnorm;
    double true_r = sqrt(rr);
    int it = 0;
    while (true_r > target && it < maxit) {
        const double sweep_stop = prec == LGF_F64 ? target : std::max(target * 0.5, true_r * 1e-4);
        LGF_HIP(hipMemcpyAsync(p, r, n * 8, hipMemcpyDeviceToDevice, st));
        if ((rc = dot(sys, r, r, 0, st))) return rc;
        double rs = rr, rsn = rr;
        while (it < maxit) {
            if ((rc = matvec(sys, prec, p, ap, st))) return rc;
            if ((rc = dot(sys, p, ap, 1, st))) return rc;
            hipLaunchKernelGGL(k_cg_xr, dim3(gb), dim3(256), 0, st, x, r, p, ap, scal, n);
            if ((rc = dot(sys, r, r, 2, st))) return rc;
            if ((rc = read_scal(sys, 2, &rsn, st))) return rc;
            ++it;
            if (sqrt(rsn) <= sweep_stop || !std::isfinite(rsn)) break;
            hipLaunchKernelGGL(k_cg_p, dim3(gb), dim3(256), 0, st, p, r, scal, n);
            hipLaunchKernelGGL(k_scal_copy, dim3(1), dim3(1), 0, st, scal, 0, 2);
            rs = rsn;
        }
        (void)rs;
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
    if (!(true_r <= target)) return fail(LGFIB_ENOCONV, "ib_force_solve: relative residual " +
                                                             std::to_string(true_r / bnorm) + " after " +
                                                             std::to_string(it) + " iterations");
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
// Every operator acts on the flow blocks D_flow (which hold D_body); the
// force solve uses the body system.  Lattice units, FP64 state.

struct ib_flow {
    lgfib_ctx *ctx = nullptr;
    ib_system *sys = nullptr;
    int B = 0, nflow = 0;
    std::vector<int32_t> blocks;
    IbPlan *plan = nullptr;   // markers binned on the flow blocks
    lgf_table_t tbl = -1;     // G_L over the flow span
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
    if ((rc = build_ib_plan(ctx, sys->kernel, sys->X.data(), sys->NL, sys->B, flow_blocks, nflow, &f->plan)))
        return rc;
    int ext[3];
    for (int q = 0; q < 3; ++q) ext[q] = f->plan->nb[q] * sys->B - 1;
    if ((rc = lgf_table_build(ctx, LGF_KIND_L, 0.0, ext, nullptr, &f->tbl))) return rc;
    const size_t nc = (size_t)nflow * sys->B * sys->B * sys->B;
    if ((rc = f->c.reserve(nc * 8)) || (rc = f->dstar.reserve(nc * 8)) || (rc = f->dd.reserve(nc * 8)) ||
        (rc = f->w.reserve(3 * nc * 8)) || (rc = f->h.reserve(3 * nc * 8)) ||
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

extern "C" int ib_flow_step(lgfib_ctx *ctx, ib_flow *fl, double *u, const double *ub, double *f, const double *x0,
                            double rtol, int maxit, int prec, ib_solve_stats_t *stats, lgfib_stream_t stream) {
    if (!ctx || !fl || fl->ctx != ctx) return fail(LGFIB_EINVAL, "ib_flow_step: bad context or flow");
    if (!u || !ub || !f) return fail(LGFIB_EINVAL, "ib_flow_step: null vector");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    ib_system *sys = fl->sys;
    const IbPlan &P = *fl->plan;
    const int B = fl->B;
    const size_t nc = (size_t)fl->nflow * B * B * B, nf = 3 * nc, nl = 3 * (size_t)sys->NL;
    double *c = fl->c.as<double>(), *dstar = fl->dstar.as<double>(), *dd = fl->dd.as<double>();
    double *w = fl->w.as<double>(), *h = fl->h.as<double>(), *rhs = fl->rhs.as<double>();
    const int32_t *bl = fl->blocks.data();
    const int nb = fl->nflow;
    int rc;
    // (ip) d* = L^{-1}(-G^T u)
    if ((rc = launch_grad_adjoint<double>(ctx, P, u, c, st, -1.0))) return rc;
    if ((rc = lgf_poisson_apply(ctx, fl->tbl, B, bl, nb, bl, nb, 1, LGF_F64, 1.0, c, dstar, 0, stream))) return rc;
    // (f) b = I E(a)[u - G d*] - u_B ;  C f = b
    LGF_HIP(hipMemcpyAsync(w, u, nf * 8, hipMemcpyDeviceToDevice, st));
    if ((rc = launch_grad_acc<double>(ctx, P, dstar, w, st, -1.0))) return rc;
    if ((rc = lgf_if_apply(ctx, sys->a, B, bl, nb, bl, nb, 3, LGF_F64, w, h, stream))) return rc;
    if ((rc = launch_interpolate<double>(ctx, P, h, rhs, st))) return rc;
    hipLaunchKernelGGL(k_flow_rhs, dim3(nblocks(nl, 256)), dim3(256), 0, st, rhs, rhs, ub, nl);
    LGF_HIP(hipGetLastError());
    rc = ib_force_solve(ctx, sys, prec, rhs, f, x0, rtol, maxit, stats, stream);
    if (rc && rc != LGFIB_ENOCONV) return rc;
    const int solve_rc = rc;
    // (pc) d = d* + L^{-1} G^T R f
    if ((rc = launch_regularize<double>(ctx, P, 1.0, f, w, st))) return rc;   // w = R f
    if ((rc = launch_grad_adjoint<double>(ctx, P, w, c, st))) return rc;
    if ((rc = lgf_poisson_apply(ctx, fl->tbl, B, bl, nb, bl, nb, 1, LGF_F64, 1.0, c, dd, 0, stream))) return rc;
    hipLaunchKernelGGL(k_add, dim3(nblocks(nc, 256)), dim3(256), 0, st, dstar, dd, 1.0, nc);   // d* := d
    LGF_HIP(hipGetLastError());
    // (vc) u = E(a)[u - G d - R f]
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, w, u, -1.0, nf);   // w = R f - u
    LGF_HIP(hipGetLastError());
    if ((rc = launch_grad_acc<double>(ctx, P, dstar, w, st, 1.0))) return rc;              // w += G d
    if ((rc = lgf_if_apply(ctx, sys->a, B, bl, nb, bl, nb, 3, LGF_F64, w, h, stream))) return rc;
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, u, u, -1.0, nf);     // u = 0
    hipLaunchKernelGGL(k_add, dim3(nblocks(nf, 256)), dim3(256), 0, st, u, h, -1.0, nf);     // u = -E(w)
    LGF_HIP(hipGetLastError());
    LGF_HIP(hipStreamSynchronize(st));
    return solve_rc;
}
