// curl.hip -- operators built on the curl C of Sec. 2.1: the nonlinear term
// in rotational form, and the velocity refresh.
//
// Velocity refresh on a finite flow domain (Sec. 4.1, Eq. vel_refresh): the vorticity w = C u is kept on the vorticity blocks and
// dropped elsewhere, the streamfunction s = -L^{-1} w is the free-space
// solution, and the velocity is replaced by C^T s on the flow blocks.
//
// The three steps run as two.  C^T and the lattice convolution are both
// translation invariant, so on the unbounded lattice
//     C^T (-G_L * w) = G_L * (-C^T w)   exactly.
// One stencil kernel therefore forms r = -C^T (C u restricted to the
// vorticity blocks) on the source side, and the box-FFT convolution returns
// G_L * r on the flow blocks: the same 3-component vector Poisson apply as
// any other, no extra layer of target cells for C^T to read, and the
// streamfunction is never stored.  r is non-zero on the vorticity blocks and
// on the top cell layer of their lower neighbours (C^T reads w at n + e_j),
// which are added to the source list.
//
// Grid placement as elsewhere in the library: face k of cell n at
// n + (1,1,1)/2 - e_k/2, edge i of cell n at n + e_i/2, so
//   (C u)^(i)(n)   = sum_jk eps_ijk [u^(k)(n) - u^(k)(n - e_j)],
//   (C^T w)^(k)(n) = sum_ij eps_ijk [w^(i)(n) - w^(i)(n + e_j)].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "conv_common.h"

namespace lgfib {
namespace {

constexpr int kNbr = 27;   // 3^3 block neighbourhood, index (dz+1)*9 + (dy+1)*3 + (dx+1)

// r = -C^T (C u |_vort) on one source block per B^3 / TPB workgroups, one
// cell per thread.  tab[28 * blk]: the flow slot of each neighbour block (-1
// if not a flow block; u is zero there), then a bit mask of the neighbours
// that are vorticity blocks (w is zero elsewhere).  Every u value is an
// unconditional load (an absent neighbour loads slot 0 and the value is then
// dropped), so the 24 distinct loads of a cell are all in flight at once;
// neighbouring threads share them through the caches.  (Staging a haloed
// tile in LDS measured slower: its index arithmetic outweighs the reuse.)
template <typename T, int B>
__global__ __launch_bounds__(256) void k_refresh_src(const T *__restrict__ u, long ustride,
                                                            const int32_t *__restrict__ tab, T *__restrict__ r,
                                                            long rstride) {
    constexpr int B3 = B * B * B;
    constexpr int TPB = B3 < 256 ? B3 : 256;
    constexpr int WPB = B3 / TPB;
    __shared__ int nb[kNbr + 1];
    // the WPB workgroups of a block (z slabs that read each other's planes)
    // and neighbouring blocks stay on one XCD, so those reads meet in its L2
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = wg / WPB;
    if (threadIdx.x <= kNbr) nb[threadIdx.x] = tab[(long)blk * (kNbr + 1) + threadIdx.x];
    __syncthreads();
    const int cell = (wg % WPB) * TPB + threadIdx.x;
    const int x = cell % B, y = (cell / B) % B, z = cell / (B * B);
    const unsigned vmask = (unsigned)nb[kNbr];
    auto U = [&](int k, int xx, int yy, int zz) -> T {
        const int s = nb[(((zz + B) / B) * 3 + (yy + B) / B) * 3 + (xx + B) / B];
        const T t = u[k * ustride + (long)(s > 0 ? s : 0) * B3 + ((zz & (B - 1)) * B + (yy & (B - 1))) * B +
                      (xx & (B - 1))];
        return s >= 0 ? t : T(0);
    };
    auto W = [&](int i, int xx, int yy, int zz) -> T {
        const int q = (((zz + B) / B) * 3 + (yy + B) / B) * 3 + (xx + B) / B;
        T w;
        if (i == 0) w = (U(2, xx, yy, zz) - U(2, xx, yy - 1, zz)) - (U(1, xx, yy, zz) - U(1, xx, yy, zz - 1));
        else if (i == 1) w = (U(0, xx, yy, zz) - U(0, xx, yy, zz - 1)) - (U(2, xx, yy, zz) - U(2, xx - 1, yy, zz));
        else w = (U(1, xx, yy, zz) - U(1, xx - 1, yy, zz)) - (U(0, xx, yy, zz) - U(0, xx, yy - 1, zz));
        return ((vmask >> q) & 1u) ? w : T(0);
    };
    const T w0 = W(0, x, y, z), w1 = W(1, x, y, z), w2 = W(2, x, y, z);
    const T rx = (w2 - W(2, x, y + 1, z)) - (w1 - W(1, x, y, z + 1));
    const T ry = (w0 - W(0, x, y, z + 1)) - (w2 - W(2, x + 1, y, z));
    const T rz = (w1 - W(1, x + 1, y, z)) - (w0 - W(0, x, y + 1, z));
    const long o = (long)blk * B3 + cell;
    r[o] = rx;
    r[rstride + o] = ry;
    r[2 * rstride + o] = rz;
}

template <typename T, int B>
int launch_src(const T *u, long ustride, const int32_t *tab, int nsrc, T *r, hipStream_t st) {
    constexpr int TPB = B * B * B < 256 ? B * B * B : 256;
    hipLaunchKernelGGL((k_refresh_src<T, B>), dim3(nsrc * (B * B * B / TPB)), dim3(TPB), 0, st, u, ustride, tab, r,
                       (long)nsrc * B * B * B);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// exact key of a block coordinate (neighbours of validated blocks may lie
// one past the validated range, so no bit packing)
struct Key3 {
    int32_t x, y, z;
    bool operator==(const Key3 &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct Key3Hash {
    size_t operator()(const Key3 &k) const {
        uint64_t h = 0xcbf29ce484222325ull;
        for (int32_t v : {k.x, k.y, k.z}) h = (h ^ (uint32_t)v) * 0x100000001b3ull;
        return (size_t)h;
    }
};
inline Key3 key3(int32_t x, int32_t y, int32_t z) { return Key3{x, y, z}; }

struct RefreshPlan {
    int B = 0;
    std::vector<int32_t> flow, vort;   // the lists the plan was made for
    std::vector<int32_t> src;          // source blocks of r
    DevBuf tab;                        // int32 [nsrc][28]
    DevBuf r;                          // [3][nsrc][B^3], FP32 or FP64
};

struct RefreshCache {
    std::map<uint64_t, CacheEnt<RefreshPlan>> plans;
};

RefreshCache &refresh_cache(lgfib_ctx *ctx) {
    if (!ctx->refresh_cache) ctx->refresh_cache = std::make_shared<RefreshCache>();
    return *static_cast<RefreshCache *>(ctx->refresh_cache.get());
}

int get_refresh_plan(lgfib_ctx *ctx, int B, const int32_t *vort, int nvort, const int32_t *flow, int nflow,
                     std::shared_ptr<RefreshPlan> &out) {
    uint64_t h = hash_blocks(0xcbf29ce484222325ull ^ (uint64_t)B, flow, nflow);
    h = hash_blocks(h ^ 0x9e3779b97f4a7c15ull, vort, nvort);
    RefreshCache &cache = refresh_cache(ctx);
    auto it = cache.plans.find(h);
    if (it != cache.plans.end()) {
        RefreshPlan &p = *it->second.v;
        if (p.B == B && p.flow.size() == 3 * (size_t)nflow && p.vort.size() == 3 * (size_t)nvort &&
            std::equal(p.flow.begin(), p.flow.end(), flow) && std::equal(p.vort.begin(), p.vort.end(), vort)) {
            it->second.tick = ++ctx->cache_tick;
            out = it->second.v;
            return LGFIB_OK;
        }
        cache.plans.erase(it);   // hash collision: rebuild for these lists
    }
    int rc = validate_blocks(flow, nflow, "flow blocks");
    if (rc) return rc;
    if ((rc = validate_blocks(vort, nvort, "vorticity blocks"))) return rc;
    std::unordered_map<Key3, int, Key3Hash> fslot;
    fslot.reserve(2 * (size_t)nflow);
    for (int i = 0; i < nflow; ++i) fslot.emplace(key3(flow[3 * i], flow[3 * i + 1], flow[3 * i + 2]), i);
    std::unordered_set<Key3, Key3Hash> vset;
    vset.reserve(2 * (size_t)nvort);
    for (int i = 0; i < nvort; ++i) {
        const Key3 k = key3(vort[3 * i], vort[3 * i + 1], vort[3 * i + 2]);
        if (!fslot.count(k))
            return fail(LGFIB_EINVAL, "lgf_velocity_refresh: vorticity block (" + std::to_string(vort[3 * i]) + "," +
                                          std::to_string(vort[3 * i + 1]) + "," + std::to_string(vort[3 * i + 2]) +
                                          ") is not a flow block");
        vset.insert(k);
    }
    auto plan = std::make_shared<RefreshPlan>();
    plan->B = B;
    plan->flow.assign(flow, flow + 3 * (size_t)nflow);
    plan->vort.assign(vort, vort + 3 * (size_t)nvort);
    // sources: the vorticity blocks, then their lower neighbours along each axis
    std::unordered_set<Key3, Key3Hash> sset(vset);
    plan->src.assign(vort, vort + 3 * (size_t)nvort);
    for (int i = 0; i < nvort; ++i)
        for (int a = 0; a < 3; ++a) {
            int32_t c[3] = {vort[3 * i], vort[3 * i + 1], vort[3 * i + 2]};
            c[a] -= 1;
            if (sset.insert(key3(c[0], c[1], c[2])).second) plan->src.insert(plan->src.end(), c, c + 3);
        }
    const int nsrc = (int)(plan->src.size() / 3);
    std::vector<int32_t> tab((size_t)nsrc * (kNbr + 1));
    for (int s = 0; s < nsrc; ++s) {
        const int32_t *b = &plan->src[3 * (size_t)s];
        uint32_t vm = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int q = ((dz + 1) * 3 + dy + 1) * 3 + dx + 1;
                    const Key3 k = key3(b[0] + dx, b[1] + dy, b[2] + dz);
                    auto f = fslot.find(k);
                    tab[(size_t)s * (kNbr + 1) + q] = f == fslot.end() ? -1 : f->second;
                    if (vset.count(k)) vm |= 1u << q;
                }
        tab[(size_t)s * (kNbr + 1) + kNbr] = (int32_t)vm;
    }
    if ((rc = plan->tab.reserve(tab.size() * sizeof(int32_t)))) return rc;
    LGF_HIP(hipMemcpy(plan->tab.p, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    out = plan;
    cache.plans[h] = CacheEnt<RefreshPlan>{std::move(plan), ++ctx->cache_tick};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

template <typename T>
int run_src(int B, const T *u, int nflow, const int32_t *tab, int nsrc, T *r, hipStream_t st) {
    const long us = (long)nflow * B * B * B;
    switch (B) {
    case 4: return launch_src<T, 4>(u, us, tab, nsrc, r, st);
    case 8: return launch_src<T, 8>(u, us, tab, nsrc, r, st);
    case 16: return launch_src<T, 16>(u, us, tab, nsrc, r, st);
    default: return launch_src<T, 32>(u, us, tab, nsrc, r, st);
    }
}

// ------------------------------------------------------------ Lamb vector

// N~^(k)(n) = scale * sum_ij eps_kij (P_ij(n) + P_ij(n + e_j)) / 2 with
// P_ij(m) = w^(i)(m) (u_a^(j)(m) + u_a^(j)(m - e_k)) / 2, w = C u, u_a = u + U
// (u zero outside the block set): the rotational nonlinear term (C u) x u_a
// with the products formed on edges.  One cell (three faces) per thread,
// unconditional loads as in k_refresh_src; tab as there (the mask word is
// unused).
template <typename T, int B>
__global__ __launch_bounds__(256) void k_lamb(const T *__restrict__ u, long ustride, const int32_t *__restrict__ tab,
                                              T *__restrict__ out, T U0, T U1, T U2, T scale) {
    constexpr int B3 = B * B * B;
    constexpr int TPB = B3 < 256 ? B3 : 256;
    constexpr int WPB = B3 / TPB;
    __shared__ int nb[kNbr + 1];
    // the WPB workgroups of a block (z slabs that read each other's planes)
    // and neighbouring blocks stay on one XCD, so those reads meet in its L2
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int blk = wg / WPB;
    if (threadIdx.x <= kNbr) nb[threadIdx.x] = tab[(long)blk * (kNbr + 1) + threadIdx.x];
    __syncthreads();
    const int cell = (wg % WPB) * TPB + threadIdx.x;
    const int x = cell % B, y = (cell / B) % B, z = cell / (B * B);
    auto Uv = [&](int k, int xx, int yy, int zz) -> T {   // block-local coordinates in [-1, B]
        const int s = nb[(((zz + B) / B) * 3 + (yy + B) / B) * 3 + (xx + B) / B];
        const T t = u[k * ustride + (long)(s > 0 ? s : 0) * B3 + ((zz & (B - 1)) * B + (yy & (B - 1))) * B +
                      (xx & (B - 1))];
        return s >= 0 ? t : T(0);
    };
    auto W = [&](int i, int xx, int yy, int zz) -> T {    // (C u)^(i), coordinates in [0, B]
        if (i == 0) return (Uv(2, xx, yy, zz) - Uv(2, xx, yy - 1, zz)) - (Uv(1, xx, yy, zz) - Uv(1, xx, yy, zz - 1));
        if (i == 1) return (Uv(0, xx, yy, zz) - Uv(0, xx, yy, zz - 1)) - (Uv(2, xx, yy, zz) - Uv(2, xx - 1, yy, zz));
        return (Uv(1, xx, yy, zz) - Uv(1, xx - 1, yy, zz)) - (Uv(0, xx, yy, zz) - Uv(0, xx, yy - 1, zz));
    };
    const T Uf[3] = {U0, U1, U2};
    // P_ij at (xx, yy, zz) with k the third index: u_a^(j) averaged along -e_k
    auto P = [&](int i, int j, int k, int xx, int yy, int zz) -> T {
        const T ub = T(0.5) * (Uv(j, xx, yy, zz) + Uv(j, xx - (k == 0), yy - (k == 1), zz - (k == 2))) + Uf[j];
        return W(i, xx, yy, zz) * ub;
    };
    const T nx = (P(1, 2, 0, x, y, z) + P(1, 2, 0, x, y, z + 1)) - (P(2, 1, 0, x, y, z) + P(2, 1, 0, x, y + 1, z));
    const T ny = (P(2, 0, 1, x, y, z) + P(2, 0, 1, x + 1, y, z)) - (P(0, 2, 1, x, y, z) + P(0, 2, 1, x, y, z + 1));
    const T nz = (P(0, 1, 2, x, y, z) + P(0, 1, 2, x, y + 1, z)) - (P(1, 0, 2, x, y, z) + P(1, 0, 2, x + 1, y, z));
    const long o = (long)blk * B3 + cell;
    const T hs = T(0.5) * scale;
    out[o] = hs * nx;
    out[ustride + o] = hs * ny;
    out[2 * ustride + o] = hs * nz;
}

// ------------------------------------------------------- block support

// Per block of the list: mu = max |w(n)| (w = C u, the three edge components
// of cell n as one vector) and nu = max |h(n)|, h = D-bar N~ the divergence of
// the nonlinear term, h(n) = sum_k N~^(k)(n + e_k) - N~^(k)(n), over the cells
// n of the block (Sec. 4.1).  N~ is formed inline from u, so faces just
// outside the block set (where N~ need not vanish) are included.  One
// workgroup per block; the maxima go through LDS.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_block_support(const T *__restrict__ u, long ustride,
                                                       const int32_t *__restrict__ tab, T U0, T U1, T U2,
                                                       double *__restrict__ mu, double *__restrict__ nu) {
    constexpr int B3 = B * B * B;
    constexpr int TPB = B3 < 256 ? B3 : 256;
    __shared__ int nb[kNbr + 1];
    __shared__ double red[2][TPB / 64];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    if (threadIdx.x <= kNbr) nb[threadIdx.x] = tab[(long)blk * (kNbr + 1) + threadIdx.x];
    __syncthreads();
    auto Uv = [&](int k, int xx, int yy, int zz) -> T {   // block-local coordinates in [-1, B]
        const int s = nb[(((zz + B) / B) * 3 + (yy + B) / B) * 3 + (xx + B) / B];
        const T t = u[k * ustride + (long)(s > 0 ? s : 0) * B3 + ((zz & (B - 1)) * B + (yy & (B - 1))) * B +
                      (xx & (B - 1))];
        return s >= 0 ? t : T(0);
    };
    auto W = [&](int i, int xx, int yy, int zz) -> T {
        if (i == 0) return (Uv(2, xx, yy, zz) - Uv(2, xx, yy - 1, zz)) - (Uv(1, xx, yy, zz) - Uv(1, xx, yy, zz - 1));
        if (i == 1) return (Uv(0, xx, yy, zz) - Uv(0, xx, yy, zz - 1)) - (Uv(2, xx, yy, zz) - Uv(2, xx - 1, yy, zz));
        return (Uv(1, xx, yy, zz) - Uv(1, xx - 1, yy, zz)) - (Uv(0, xx, yy, zz) - Uv(0, xx, yy - 1, zz));
    };
    const T Uf[3] = {U0, U1, U2};
    auto P = [&](int i, int j, int k, int xx, int yy, int zz) -> T {
        const T ub = T(0.5) * (Uv(j, xx, yy, zz) + Uv(j, xx - (k == 0), yy - (k == 1), zz - (k == 2))) + Uf[j];
        return W(i, xx, yy, zz) * ub;
    };
    // N~^(k) at face k of cell (xx, yy, zz), coordinates in [0, B]
    auto Nk = [&](int k, int xx, int yy, int zz) -> T {
        T v;
        if (k == 0)
            v = (P(1, 2, 0, xx, yy, zz) + P(1, 2, 0, xx, yy, zz + 1)) - (P(2, 1, 0, xx, yy, zz) + P(2, 1, 0, xx, yy + 1, zz));
        else if (k == 1)
            v = (P(2, 0, 1, xx, yy, zz) + P(2, 0, 1, xx + 1, yy, zz)) - (P(0, 2, 1, xx, yy, zz) + P(0, 2, 1, xx, yy, zz + 1));
        else
            v = (P(0, 1, 2, xx, yy, zz) + P(0, 1, 2, xx, yy + 1, zz)) - (P(1, 0, 2, xx, yy, zz) + P(1, 0, 2, xx + 1, yy, zz));
        return T(0.5) * v;
    };
    double m0 = 0.0, m1 = 0.0;
    for (int cell = threadIdx.x; cell < B3; cell += TPB) {
        const int x = cell % B, y = (cell / B) % B, z = cell / (B * B);
        const double w0 = (double)W(0, x, y, z), w1 = (double)W(1, x, y, z), w2 = (double)W(2, x, y, z);
        const T h = (Nk(0, x + 1, y, z) - Nk(0, x, y, z)) + (Nk(1, x, y + 1, z) - Nk(1, x, y, z)) +
                    (Nk(2, x, y, z + 1) - Nk(2, x, y, z));
        m0 = fmax(m0, sqrt(w0 * w0 + w1 * w1 + w2 * w2));
        m1 = fmax(m1, fabs((double)h));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, o, 64));
        m1 = fmax(m1, __shfl_xor(m1, o, 64));
    }
    if (threadIdx.x % 64 == 0) {
        red[0][threadIdx.x / 64] = m0;
        red[1][threadIdx.x / 64] = m1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < TPB / 64; ++q) {
            a = fmax(a, red[0][q]);
            b = fmax(b, red[1][q]);
        }
        mu[blk] = a;
        nu[blk] = b;
    }
}

struct LambPlan {
    int B = 0;
    std::vector<int32_t> blocks;
    DevBuf tab;   // int32 [nblk][28]
};

struct LambCache {
    std::map<uint64_t, CacheEnt<LambPlan>> plans;
};

int get_lamb_plan(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, std::shared_ptr<LambPlan> &out) {
    const uint64_t h = hash_blocks(0x84222325cbf29ce4ull ^ (uint64_t)B, blocks, nblk);
    if (!ctx->lamb_cache) ctx->lamb_cache = std::make_shared<LambCache>();
    LambCache &cache = *static_cast<LambCache *>(ctx->lamb_cache.get());
    auto it = cache.plans.find(h);
    if (it != cache.plans.end()) {
        LambPlan &p = *it->second.v;
        if (p.B == B && p.blocks.size() == 3 * (size_t)nblk && std::equal(p.blocks.begin(), p.blocks.end(), blocks)) {
            it->second.tick = ++ctx->cache_tick;
            out = it->second.v;
            return LGFIB_OK;
        }
        cache.plans.erase(it);
    }
    int rc = validate_blocks(blocks, nblk, "blocks");
    if (rc) return rc;
    std::unordered_map<Key3, int, Key3Hash> slot;
    slot.reserve(2 * (size_t)nblk);
    for (int i = 0; i < nblk; ++i) slot.emplace(key3(blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2]), i);
    std::vector<int32_t> tab((size_t)nblk * (kNbr + 1), 0);
    for (int b = 0; b < nblk; ++b)
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    auto f = slot.find(key3(blocks[3 * b] + dx, blocks[3 * b + 1] + dy, blocks[3 * b + 2] + dz));
                    tab[(size_t)b * (kNbr + 1) + ((dz + 1) * 3 + dy + 1) * 3 + dx + 1] = f == slot.end() ? -1 : f->second;
                }
    auto plan = std::make_shared<LambPlan>();
    plan->B = B;
    plan->blocks.assign(blocks, blocks + 3 * (size_t)nblk);
    if ((rc = plan->tab.reserve(tab.size() * sizeof(int32_t)))) return rc;
    LGF_HIP(hipMemcpy(plan->tab.p, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    out = plan;
    cache.plans[h] = CacheEnt<LambPlan>{std::move(plan), ++ctx->cache_tick};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

template <typename T, int B>
int launch_lamb(const T *u, int nblk, const int32_t *tab, T *out, const double *U, double scale, hipStream_t st) {
    constexpr int TPB = B * B * B < 256 ? B * B * B : 256;
    hipLaunchKernelGGL((k_lamb<T, B>), dim3(nblk * (B * B * B / TPB)), dim3(TPB), 0, st, u, (long)nblk * B * B * B,
                       tab, out, (T)U[0], (T)U[1], (T)U[2], (T)scale);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename T>
int run_lamb(int B, const T *u, int nblk, const int32_t *tab, T *out, const double *U, double scale, hipStream_t st) {
    switch (B) {
    case 4: return launch_lamb<T, 4>(u, nblk, tab, out, U, scale, st);
    case 8: return launch_lamb<T, 8>(u, nblk, tab, out, U, scale, st);
    case 16: return launch_lamb<T, 16>(u, nblk, tab, out, U, scale, st);
    default: return launch_lamb<T, 32>(u, nblk, tab, out, U, scale, st);
    }
}

template <typename T, int B>
int launch_support(const T *u, int nblk, const int32_t *tab, const double *U, double *mu, double *nu, hipStream_t st) {
    constexpr int TPB = B * B * B < 256 ? B * B * B : 256;
    hipLaunchKernelGGL((k_block_support<T, B>), dim3(nblk), dim3(TPB), 0, st, u, (long)nblk * B * B * B, tab, (T)U[0],
                       (T)U[1], (T)U[2], mu, nu);
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <typename T>
int run_support(int B, const T *u, int nblk, const int32_t *tab, const double *U, double *mu, double *nu,
                hipStream_t st) {
    switch (B) {
    case 4: return launch_support<T, 4>(u, nblk, tab, U, mu, nu, st);
    case 8: return launch_support<T, 8>(u, nblk, tab, U, mu, nu, st);
    case 16: return launch_support<T, 16>(u, nblk, tab, U, mu, nu, st);
    default: return launch_support<T, 32>(u, nblk, tab, U, mu, nu, st);
    }
}

}  // namespace

int lamb_apply(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, double scale, int prec,
               const void *u, void *out, hipStream_t st) {
    std::shared_ptr<LambPlan> plan;
    int rc = get_lamb_plan(ctx, B, blocks, nblk, plan);
    if (rc) return rc;
    const double zero[3] = {0.0, 0.0, 0.0};
    if (!U) U = zero;
    ProfScope ps(ctx, "k_lamb", st);
    if (prec == LGF_F64)
        return run_lamb<double>(B, (const double *)u, nblk, plan->tab.as<int32_t>(), (double *)out, U, scale, st);
    return run_lamb<float>(B, (const float *)u, nblk, plan->tab.as<int32_t>(), (float *)out, U, scale, st);
}

size_t curl_cache_trim(lgfib_ctx *ctx, size_t cap, int64_t *left) {
    size_t n = 0;
    int64_t k = 0;
    if (ctx->refresh_cache) {
        RefreshCache &rc = refresh_cache(ctx);
        n += cache_trim(rc.plans, cap);
        k += (int64_t)rc.plans.size();
    }
    if (ctx->lamb_cache) {
        LambCache &lc = *static_cast<LambCache *>(ctx->lamb_cache.get());
        n += cache_trim(lc.plans, cap);
        k += (int64_t)lc.plans.size();
    }
    if (left) *left = k;
    return n;
}

}  // namespace lgfib

using namespace lgfib;

extern "C" int lgf_lamb_vector(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, int prec,
                               const void *u, void *out, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_lamb_vector: null context");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_lamb_vector: B must be 4, 8, 16 or 32");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "lgf_lamb_vector: prec must be LGF_F32 or LGF_F64");
    if (nblk < 0) return fail(LGFIB_EINVAL, "lgf_lamb_vector: negative block count");
    if (nblk == 0) return LGFIB_OK;
    if (!blocks || !u || !out) return fail(LGFIB_EINVAL, "lgf_lamb_vector: null argument");
    if (U && !(std::isfinite(U[0]) && std::isfinite(U[1]) && std::isfinite(U[2])))
        return fail(LGFIB_EINVAL, "lgf_lamb_vector: non-finite frame velocity");
    const size_t bytes = 3 * (size_t)nblk * B * B * B * (prec == LGF_F64 ? 8 : 4);
    const char *a = (const char *)u, *b = (const char *)out;
    if (a < b + bytes && b < a + bytes) return fail(LGFIB_EINVAL, "lgf_lamb_vector: u and out overlap");
    LGF_HIP(hipSetDevice(ctx->device));
    return lamb_apply(ctx, B, blocks, nblk, U, 1.0, prec, u, out, (hipStream_t)stream);
}

extern "C" int lgf_velocity_refresh(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *vort_blocks, int nvort,
                                    const int32_t *flow_blocks, int nflow, int prec, void *u,
                                    lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: null context");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_velocity_refresh: unknown table");
    if (ctx->tables[tbl]->kind != LGF_KIND_L)
        return fail(LGFIB_EINVAL, "lgf_velocity_refresh: the refresh needs a G_L table (LGF_KIND_L)");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: B must be 4, 8, 16 or 32");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: prec must be LGF_F32 or LGF_F64");
    if (nvort < 0 || nflow < 0) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: negative block count");
    if ((nvort > 0 && !vort_blocks) || (nflow > 0 && !flow_blocks))
        return fail(LGFIB_EINVAL, "lgf_velocity_refresh: null block list");
    if (nflow == 0) {
        if (nvort > 0) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: vorticity blocks without flow blocks");
        return LGFIB_OK;
    }
    if (!u) return fail(LGFIB_EINVAL, "lgf_velocity_refresh: null velocity");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t es = prec == LGF_F64 ? 8 : 4;
    const size_t B3 = (size_t)B * B * B;
    std::shared_ptr<RefreshPlan> plan;
    int rc;
    if ((rc = get_refresh_plan(ctx, B, vort_blocks, nvort, flow_blocks, nflow, plan))) return rc;
    if (nvort == 0) {   // no vorticity: the refreshed velocity is zero
        LGF_HIP(hipMemsetAsync(u, 0, 3 * (size_t)nflow * B3 * es, st));
        return LGFIB_OK;
    }
    const int nsrc = (int)(plan->src.size() / 3);
    if ((rc = plan->r.reserve(3 * (size_t)nsrc * B3 * es))) return rc;
    {
        ProfScope ps(ctx, "k_refresh_src", st);
        rc = prec == LGF_F64 ? run_src<double>(B, (const double *)u, nflow, plan->tab.as<int32_t>(), nsrc,
                                               plan->r.as<double>(), st)
                             : run_src<float>(B, (const float *)u, nflow, plan->tab.as<int32_t>(), nsrc,
                                              plan->r.as<float>(), st);
        if (rc) return rc;
    }
    return lgf_poisson_apply(ctx, tbl, B, plan->src.data(), nsrc, flow_blocks, nflow, 3, prec, 1.0, plan->r.p, u, 0,
                             stream);
}

extern "C" int lgf_block_support(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, int prec,
                                 const void *u, double *mu, double *nu, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_block_support: null context");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_block_support: B must be 4, 8, 16 or 32");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "lgf_block_support: prec must be LGF_F32 or LGF_F64");
    if (nblk < 0) return fail(LGFIB_EINVAL, "lgf_block_support: negative block count");
    if (nblk == 0) return LGFIB_OK;
    if (!blocks || !u || !mu || !nu) return fail(LGFIB_EINVAL, "lgf_block_support: null argument");
    if (U && !(std::isfinite(U[0]) && std::isfinite(U[1]) && std::isfinite(U[2])))
        return fail(LGFIB_EINVAL, "lgf_block_support: non-finite frame velocity");
    LGF_HIP(hipSetDevice(ctx->device));
    std::shared_ptr<LambPlan> plan;
    int rc = get_lamb_plan(ctx, B, blocks, nblk, plan);
    if (rc) return rc;
    const double zero[3] = {0.0, 0.0, 0.0};
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps(ctx, "k_block_support", st);
    if (prec == LGF_F64)
        return run_support<double>(B, (const double *)u, nblk, plan->tab.as<int32_t>(), U ? U : zero, mu, nu, st);
    return run_support<float>(B, (const float *)u, nblk, plan->tab.as<int32_t>(), U ? U : zero, mu, nu, st);
}

// ------------------------------------------------------------ host: the set update

extern "C" int ib_block_weights(const double *X, int NL, int B, const int32_t *blocks, int nblk, double eta,
                                double length, double *w) {
    if (NL < 1 || !X || nblk < 0 || (nblk > 0 && (!blocks || !w)) || B < 1 || !(eta > 0.0) || !(length > 0.0))
        return fail(LGFIB_EINVAL, "ib_block_weights: bad argument");
    for (int b = 0; b < nblk; ++b) {
        double c[3];
        for (int a = 0; a < 3; ++a) c[a] = ((double)blocks[3 * b + a] + 0.5) * B;
        double d2 = INFINITY;
        for (int i = 0; i < NL; ++i) {
            const double dx = c[0] - X[3 * i], dy = c[1] - X[3 * i + 1], dz = c[2] - X[3 * i + 2];
            d2 = std::min(d2, dx * dx + dy * dy + dz * dz);
        }
        w[b] = 1.0 / std::max(eta, std::sqrt(d2) / length);
    }
    return LGFIB_OK;
}

extern "C" int ib_adapt_flow(const int32_t *xflow, int nx, const double *mu, const double *nu, const double *weights,
                             double eps, const int32_t *body, int nbody, int nbuf, int32_t *flow_out, int max_flow,
                             int *nflow, int32_t *xflow_out, int max_xflow, int *nxflow) {
    if (nx < 0 || nbody < 0 || nbuf < 0 || nbuf > 8 || !nflow || !nxflow || (nx > 0 && (!xflow || !mu || !nu || !weights)) ||
        (nbody > 0 && !body) || !(eps >= 0.0))
        return fail(LGFIB_EINVAL, "ib_adapt_flow: bad argument");
    double mg = 0.0, ng = 0.0;
    for (int b = 0; b < nx; ++b) {
        mg = std::max(mg, mu[b]);
        ng = std::max(ng, nu[b]);
    }
    std::unordered_set<Key3, Key3Hash> keep;
    for (int b = 0; b < nx; ++b) {
        double r = 0.0;
        if (mg > 0.0) r = std::max(r, mu[b] / mg);
        if (ng > 0.0) r = std::max(r, nu[b] / ng);
        if (weights[b] * r > eps) keep.insert(key3(xflow[3 * b], xflow[3 * b + 1], xflow[3 * b + 2]));
    }
    for (int b = 0; b < nbody; ++b) keep.insert(key3(body[3 * b], body[3 * b + 1], body[3 * b + 2]));
    std::unordered_set<Key3, Key3Hash> dil;
    for (const Key3 &k : keep)
        for (int dz = -nbuf; dz <= nbuf; ++dz)
            for (int dy = -nbuf; dy <= nbuf; ++dy)
                for (int dx = -nbuf; dx <= nbuf; ++dx) dil.insert(key3(k.x + dx, k.y + dy, k.z + dz));
    auto out = [](const std::unordered_set<Key3, Key3Hash> &st, int32_t *dst, int cap, int *n) {
        std::vector<Key3> v(st.begin(), st.end());
        std::sort(v.begin(), v.end(), [](const Key3 &a, const Key3 &b) {
            return a.z != b.z ? a.z < b.z : (a.y != b.y ? a.y < b.y : a.x < b.x);
        });
        *n = (int)v.size();
        if ((int)v.size() > cap || (!dst && !v.empty())) return false;
        for (size_t i = 0; i < v.size(); ++i) {
            dst[3 * i] = v[i].x;
            dst[3 * i + 1] = v[i].y;
            dst[3 * i + 2] = v[i].z;
        }
        return true;
    };
    const bool ok1 = out(keep, flow_out, max_flow, nflow);
    const bool ok2 = out(dil, xflow_out, max_xflow, nxflow);
    if (!ok1 || !ok2) return fail(LGFIB_ERANGE, "ib_adapt_flow: output lists too small (sizes returned)");
    return LGFIB_OK;
}

// ------------------------------------------------- device: the set update
//
// The same update as ib_block_weights followed by ib_adapt_flow, on the
// device: block weights by a wavefront per block over all markers, the two
// global maxima by atomics on the (non-negative) values' bit patterns, the
// kept blocks marked in a byte grid over the blocks' bounding box grown by
// nbuf, the buffer zone by three separable maximum filters, and both lists
// by a stream compaction in grid order, which is (z, y, x) order.  The
// arithmetic is the host version's, operation for operation, without fused
// multiply-adds, so that both keep exactly the same blocks.

namespace lgfib {
namespace {

constexpr int64_t kAdaptMaxCells = (int64_t)1 << 26;   // grid cap (bytes per grid)
constexpr int kCompactChunk = 4096;                    // cells per workgroup of the compaction

struct AdaptGrid {
    int x0, y0, z0, nx, ny, nz;
};

#pragma clang fp contract(off)
// w[b] and the maxima of mu and nu (as int64 bit patterns, non-negative values only)
__global__ __launch_bounds__(256) void k_adapt_weights(const double *__restrict__ X, int NL, const int32_t *__restrict__ blk,
                                                       int nx, int B, double eta, double length,
                                                       const double *__restrict__ mu, const double *__restrict__ nu,
                                                       double *__restrict__ w, unsigned long long *__restrict__ gmax) {
    const int b = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (b >= nx) return;
    double c[3];
    for (int a = 0; a < 3; ++a) c[a] = ((double)blk[3 * b + a] + 0.5) * B;
    double d2 = INFINITY;
    for (int i = lane; i < NL; i += 64) {
        const double dx = c[0] - X[3 * i], dy = c[1] - X[3 * i + 1], dz = c[2] - X[3 * i + 2];
        d2 = fmin(d2, dx * dx + dy * dy + dz * dz);
    }
    for (int o = 32; o > 0; o >>= 1) d2 = fmin(d2, __shfl_xor(d2, o));
    if (lane == 0) {
        w[b] = 1.0 / fmax(eta, sqrt(d2) / length);
        // max(0, .) of every value: negative and NaN values are left out
        if (mu[b] > 0.0) atomicMax(&gmax[0], (unsigned long long)__double_as_longlong(mu[b]));
        if (nu[b] > 0.0) atomicMax(&gmax[1], (unsigned long long)__double_as_longlong(nu[b]));
    }
}

// mark the kept blocks (W_flow > eps) and the body blocks (entries >= nx) in the grid
__global__ __launch_bounds__(256) void k_adapt_mark(const int32_t *__restrict__ blk, int nx, int nall,
                                                    const double *__restrict__ mu, const double *__restrict__ nu,
                                                    const double *__restrict__ w,
                                                    const unsigned long long *__restrict__ gmax, double eps,
                                                    AdaptGrid g, unsigned char *__restrict__ grid) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nall) return;
    bool keep = true;
    if (b < nx) {
        const double mg = __longlong_as_double((long long)gmax[0]), ng = __longlong_as_double((long long)gmax[1]);
        double r = 0.0;
        if (mg > 0.0) r = fmax(r, mu[b] / mg);
        if (ng > 0.0) r = fmax(r, nu[b] / ng);
        keep = w[b] * r > eps;
    }
    if (keep) {
        const long x = blk[3 * b] - g.x0, y = blk[3 * b + 1] - g.y0, z = blk[3 * b + 2] - g.z0;
        grid[(z * g.ny + y) * g.nx + x] = 1;
    }
}
#pragma clang fp contract(fast)

// out = maximum of in over [-r, r] along one axis (stride s, extent n)
__global__ __launch_bounds__(256) void k_adapt_dilate(const unsigned char *__restrict__ in, unsigned char *__restrict__ out,
                                                      int64_t cells, int64_t s, int n, int r) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cells) return;
    const int i = (int)((c / s) % n);
    unsigned char v = 0;
    for (int d = max(-r, -i); d <= min(r, n - 1 - i); ++d) v |= in[c + d * s];
    out[c] = v;
}

// stream compaction of a byte grid: counts per chunk, their exclusive sum,
// then the coordinates of the set cells in grid order
__global__ __launch_bounds__(256) void k_adapt_count(const unsigned char *__restrict__ grid, int64_t cells,
                                                     int *__restrict__ cnt) {
    const int64_t c0 = (int64_t)blockIdx.x * kCompactChunk;
    int n = 0;
    for (int e = threadIdx.x; e < kCompactChunk; e += 256) n += (c0 + e < cells && grid[c0 + e]) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    __shared__ int part[4];
    if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = n;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// one workgroup: off[i] = sum of cnt[0..i-1], off[nchunk] = total
__global__ __launch_bounds__(1024) void k_adapt_scan(const int *__restrict__ cnt, int nchunk, int *__restrict__ off) {
    __shared__ int tot[1024];
    const int t = threadIdx.x, per = (nchunk + 1023) / 1024, b0 = t * per;
    int s = 0;
    for (int i = b0; i < min(b0 + per, nchunk); ++i) s += cnt[i];
    tot[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan of the thread sums
        const int v = t >= o ? tot[t - o] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? tot[t - 1] : 0;
    for (int i = b0; i < min(b0 + per, nchunk); ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (t == 1023) off[nchunk] = tot[1023];
}

__global__ __launch_bounds__(256) void k_adapt_emit(const unsigned char *__restrict__ grid, int64_t cells,
                                                    const int *__restrict__ off, AdaptGrid g, int cap,
                                                    int32_t *__restrict__ out) {
    constexpr int PER = kCompactChunk / 256;   // consecutive cells per thread
    const int64_t c0 = (int64_t)blockIdx.x * kCompactChunk + threadIdx.x * PER;
    int n = 0;
    for (int e = 0; e < PER; ++e) n += (c0 + e < cells && grid[c0 + e]) ? 1 : 0;
    __shared__ int sc[256];
    sc[threadIdx.x] = n;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    int pos = off[blockIdx.x] + sc[threadIdx.x] - n;
    for (int e = 0; e < PER; ++e) {
        const int64_t c = c0 + e;
        if (c < cells && grid[c]) {
            if (pos < cap) {
                const int64_t x = c % g.nx, y = (c / g.nx) % g.ny, z = c / ((int64_t)g.nx * g.ny);
                out[3 * (int64_t)pos] = (int32_t)(x + g.x0);
                out[3 * (int64_t)pos + 1] = (int32_t)(y + g.y0);
                out[3 * (int64_t)pos + 2] = (int32_t)(z + g.z0);
            }
            ++pos;
        }
    }
}

inline unsigned nblk_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// compact `grid` into the host list dst (capacity cap); *count receives the size
int adapt_compact(const unsigned char *grid, int64_t cells, const AdaptGrid &g, int *cnt, int *off,
                  int32_t *dev_out, int cap, int32_t *dst, int *count, hipStream_t st) {
    const unsigned nchunk = nblk_of(cells, kCompactChunk);
    hipLaunchKernelGGL(k_adapt_count, dim3(nchunk), dim3(256), 0, st, grid, cells, cnt);
    hipLaunchKernelGGL(k_adapt_scan, dim3(1), dim3(1024), 0, st, cnt, (int)nchunk, off);
    hipLaunchKernelGGL(k_adapt_emit, dim3(nchunk), dim3(256), 0, st, grid, cells, off, g, cap, dev_out);
    LGF_HIP(hipGetLastError());
    int total = 0;
    LGF_HIP(hipMemcpyAsync(&total, off + nchunk, sizeof(int), hipMemcpyDeviceToHost, st));
    LGF_HIP(hipStreamSynchronize(st));
    *count = total;
    if (total > cap || (!dst && total > 0)) return LGFIB_ERANGE;
    if (total > 0)
        LGF_HIP(hipMemcpyAsync(dst, dev_out, (size_t)total * 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LGF_HIP(hipStreamSynchronize(st));
    return LGFIB_OK;
}

}  // namespace
}  // namespace lgfib

extern "C" int ib_adapt_flow_dev(lgfib_ctx *ctx, const double *X, int NL, int B, const int32_t *xflow, int nx,
                                 const double *mu, const double *nu, double eta, double length, double eps,
                                 const int32_t *body, int nbody, int nbuf, int32_t *flow_out, int max_flow, int *nflow,
                                 int32_t *xflow_out, int max_xflow, int *nxflow, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "ib_adapt_flow_dev: null context");
    if (NL < 1 || !X || nx < 0 || nbody < 0 || nbuf < 0 || nbuf > 8 || B < 1 || !nflow || !nxflow ||
        (nx > 0 && (!xflow || !mu || !nu)) || (nbody > 0 && !body) || !(eta > 0.0) || !(length > 0.0) ||
        !(eps >= 0.0) || max_flow < 0 || max_xflow < 0)
        return fail(LGFIB_EINVAL, "ib_adapt_flow_dev: bad argument");
    *nflow = *nxflow = 0;
    const int nall = nx + nbody;
    if (nall == 0) return LGFIB_OK;
    // bounding box of the listed blocks, grown by the buffer width
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int b = 0; b < nall; ++b) {
        const int32_t *k = b < nx ? xflow + 3 * b : body + 3 * (b - nx);
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min<int64_t>(lo[a], k[a]);
            hi[a] = std::max<int64_t>(hi[a], k[a]);
        }
    }
    int64_t ext[3], cells = 1;
    for (int a = 0; a < 3; ++a) {
        lo[a] -= nbuf;
        ext[a] = hi[a] + nbuf - lo[a] + 1;
        cells *= ext[a];
        if (cells > kAdaptMaxCells || lo[a] < INT32_MIN || hi[a] + nbuf > INT32_MAX)
            return fail(LGFIB_ERANGE, "ib_adapt_flow_dev: the blocks' bounding box exceeds 2^26 blocks");
    }
    const AdaptGrid g{(int)lo[0], (int)lo[1], (int)lo[2], (int)ext[0], (int)ext[1], (int)ext[2]};
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t nchunk = (cells + kCompactChunk - 1) / kCompactChunk;
    const int64_t cap_out = std::max<int64_t>(std::max(max_flow, max_xflow), 1);
    // workspace: blocks, weights, maxima, three grids, chunk counts and offsets, output list
    size_t o = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_blk = carve((size_t)nall * 3 * sizeof(int32_t)), o_w = carve((size_t)std::max(nx, 1) * 8),
                 o_max = carve(16), o_g1 = carve((size_t)cells), o_g2 = carve((size_t)cells),
                 o_g3 = carve((size_t)cells), o_cnt = carve((size_t)nchunk * 4), o_off = carve((size_t)(nchunk + 1) * 4),
                 o_out = carve((size_t)cap_out * 3 * sizeof(int32_t));
    int rc = ctx->adapt_ws.reserve(o);
    if (rc) return rc;
    char *ws = ctx->adapt_ws.as<char>();
    int32_t *dblk = (int32_t *)(ws + o_blk);
    double *w = (double *)(ws + o_w);
    unsigned long long *gmax = (unsigned long long *)(ws + o_max);
    unsigned char *g1 = (unsigned char *)(ws + o_g1), *g2 = (unsigned char *)(ws + o_g2), *g3 = (unsigned char *)(ws + o_g3);
    int *cnt = (int *)(ws + o_cnt), *off = (int *)(ws + o_off);
    int32_t *dout = (int32_t *)(ws + o_out);
    if (nx > 0) LGF_HIP(hipMemcpyAsync(dblk, xflow, (size_t)nx * 12, hipMemcpyHostToDevice, st));
    if (nbody > 0) LGF_HIP(hipMemcpyAsync(dblk + 3 * (size_t)nx, body, (size_t)nbody * 12, hipMemcpyHostToDevice, st));
    LGF_HIP(hipMemsetAsync(gmax, 0, 16, st));
    LGF_HIP(hipMemsetAsync(g1, 0, (size_t)cells, st));
    {
        ProfScope ps(ctx, "k_adapt", st);
        if (nx > 0)
            hipLaunchKernelGGL(k_adapt_weights, dim3(nblk_of(nx, 4)), dim3(256), 0, st, X, NL, dblk, nx, B, eta, length,
                               mu, nu, w, gmax);
        hipLaunchKernelGGL(k_adapt_mark, dim3(nblk_of(nall, 256)), dim3(256), 0, st, dblk, nx, nall, mu, nu, w, gmax, eps,
                           g, g1);
        const unsigned char *dil = g1;
        if (nbuf > 0) {
            const unsigned nb = nblk_of(cells, 256);
            hipLaunchKernelGGL(k_adapt_dilate, dim3(nb), dim3(256), 0, st, g1, g2, cells, (int64_t)1, g.nx, nbuf);
            hipLaunchKernelGGL(k_adapt_dilate, dim3(nb), dim3(256), 0, st, g2, g3, cells, (int64_t)g.nx, g.ny, nbuf);
            hipLaunchKernelGGL(k_adapt_dilate, dim3(nb), dim3(256), 0, st, g3, g2, cells, (int64_t)g.nx * g.ny, g.nz,
                               nbuf);
            dil = g2;
        }
        LGF_HIP(hipGetLastError());
        const int rc1 = adapt_compact(g1, cells, g, cnt, off, dout, max_flow, flow_out, nflow, st);
        if (rc1 && rc1 != LGFIB_ERANGE) return rc1;
        const int rc2 = adapt_compact(dil, cells, g, cnt, off, dout, max_xflow, xflow_out, nxflow, st);
        if (rc2 && rc2 != LGFIB_ERANGE) return rc2;
        if (rc1 || rc2) return fail(LGFIB_ERANGE, "ib_adapt_flow_dev: output lists too small (sizes returned)");
    }
    return LGFIB_OK;
}
