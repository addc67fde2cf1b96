// blockset.cpp -- host-side block-set staging: validation, bounding boxes,
// FFT box plans and integrating-factor neighbour plans.
//
// The paper partitions the unbounded grid into cubic blocks and restricts every
// non-compact operator to source and target block sets (Sec. 4.1, Table
// tab:src_trg).  Here a block list is validated once per distinct list, and the
// derived device maps are cached in the context by a hash of the lists.
#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <unordered_set>

#include "internal.h"

namespace lgfib {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

static inline uint64_t pack_coord(int32_t x, int32_t y, int32_t z) {
    const uint64_t m = (1ull << 21) - 1;
    return ((uint64_t)(x + (1 << 20)) & m) | (((uint64_t)(y + (1 << 20)) & m) << 21) |
           (((uint64_t)(z + (1 << 20)) & m) << 42);
}

int validate_blocks(const int32_t *blocks, int n, const char *what) {
    if (n < 0) return fail(LGFIB_EINVAL, std::string(what) + ": negative block count");
    if (n > 0 && !blocks) return fail(LGFIB_EINVAL, std::string(what) + ": null block list");
    std::unordered_set<uint64_t> seen;
    seen.reserve((size_t)n * 2);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            int32_t c = blocks[3 * i + a];
            if (c < -(1 << 20) || c >= (1 << 20))
                return fail(LGFIB_EINVAL, std::string(what) + ": block coordinate out of range at index " +
                                              std::to_string(i));
        }
        if (!seen.insert(pack_coord(blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2])).second)
            return fail(LGFIB_EDUP_BLOCK, std::string(what) + ": block (" + std::to_string(blocks[3 * i]) + "," +
                                              std::to_string(blocks[3 * i + 1]) + "," +
                                              std::to_string(blocks[3 * i + 2]) + ") listed twice");
    }
    return LGFIB_OK;
}

int smooth_ceil(int n) {
    for (int m = std::max(n, 1);; ++m) {
        int r = m;
        for (int p : {2, 3, 5})
            while (r % p == 0) r /= p;
        if (r == 1) return m;
    }
}

uint64_t hash_blocks(uint64_t h, const int32_t *b, int n) {
    // FNV-1a over the raw coordinates
    const unsigned char *p = reinterpret_cast<const unsigned char *>(b);
    size_t len = (size_t)n * 3 * sizeof(int32_t);
    for (size_t i = 0; i < len; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    h ^= (uint64_t)n;
    h *= 1099511628211ull;
    return h;
}

// Key = hash of (kind tag, B, extra, both lists); the stored copy of the lists
// guards against collisions.
// the stored key equals (nsrc, ntgt, extra, src..., tgt...)
static bool same_key(const std::vector<int32_t> &k, int extra, const int32_t *src, int nsrc, const int32_t *tgt,
                     int ntgt) {
    const size_t ns = 3 * (size_t)nsrc, nt = 3 * (size_t)ntgt;
    if (k.size() != 3 + ns + nt || k[0] != nsrc || k[1] != ntgt || k[2] != extra) return false;
    return (ns == 0 || memcmp(k.data() + 3, src, ns * 4) == 0) && (nt == 0 || memcmp(k.data() + 3 + ns, tgt, nt * 4) == 0);
}

static uint64_t plan_key(lgfib_ctx *ctx, int tag, int B, int extra, const int32_t *src, int nsrc,
                         const int32_t *tgt, int ntgt, bool *hit) {
    uint64_t h = 1469598103934665603ull;
    int hdr[3] = {tag, B, extra};
    h = hash_blocks(h, hdr, 1);
    h = hash_blocks(h, src, nsrc);
    h = hash_blocks(h, tgt, ntgt);
    auto make_flat = [&]() {
        std::vector<int32_t> flat;
        flat.reserve(3 + 3 * (size_t)(nsrc + ntgt));
        flat.push_back(nsrc);
        flat.push_back(ntgt);
        flat.push_back(extra);
        flat.insert(flat.end(), src, src + 3 * (size_t)nsrc);
        flat.insert(flat.end(), tgt, tgt + 3 * (size_t)ntgt);
        return flat;
    };
    // probe h, then deterministic perturbations of it on collisions
    for (uint64_t salt = 0;; ++salt) {
        const uint64_t h2 = salt ? h ^ (salt * 0x9e3779b97f4a7c15ull) : h;
        const auto k2 = std::make_tuple(tag, B, extra, 0, h2);
        auto it = ctx->plan_keys.find(k2);
        if (it == ctx->plan_keys.end()) {
            ctx->plan_keys[k2] = make_flat();
            *hit = false;
            return h2;
        }
        if (same_key(it->second, extra, src, nsrc, tgt, ntgt)) {
            *hit = true;
            return h2;
        }
    }
}

int get_box_plan(lgfib_ctx *ctx, int B, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                 std::shared_ptr<BoxPlan> &out) {
    bool hit = false;
    uint64_t key = plan_key(ctx, 1, B, 0, src, nsrc, tgt, ntgt, &hit);
    if (hit) {
        auto it = ctx->box_plans.find(key);
        if (it != ctx->box_plans.end()) {
            it->second.tick = ++ctx->cache_tick;
            out = it->second.v;
            return LGFIB_OK;
        }
    }
    int rc = validate_blocks(src, nsrc, "source blocks");
    if (rc) return rc;
    rc = validate_blocks(tgt, ntgt, "target blocks");
    if (rc) return rc;

    auto plan = std::make_shared<BoxPlan>();
    plan->B = B;
    plan->nsrc = nsrc;
    plan->ntgt = ntgt;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    auto grow = [&](const int32_t *b, int n) {
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], (int)b[3 * i + a]);
                hi[a] = std::max(hi[a], (int)b[3 * i + a]);
            }
    };
    grow(src, nsrc);
    grow(tgt, ntgt);
    for (int a = 0; a < 3; ++a) {
        plan->lo[a] = lo[a];
        plan->nb[a] = smooth_ceil(hi[a] - lo[a] + 1);
        plan->N[a] = plan->nb[a] * B;
        plan->P[a] = 2 * plan->N[a];
        if (plan->P[a] > 1024)
            return fail(LGFIB_ERANGE, "block set spans " + std::to_string(plan->N[a]) +
                                          " cells along axis " + std::to_string(a) +
                                          " after 2,3,5-smooth rounding; at most 512 are supported");
    }
    plan->Kx = plan->P[0] / 2 + 1;
    plan->Kxp = (plan->Kx + 15) / 16 * 16;

    const int nb0 = plan->nb[0], nb1 = plan->nb[1], nb2 = plan->nb[2];
    std::vector<int32_t> smap((size_t)nb0 * nb1 * nb2, -1), tmap((size_t)nb0 * nb1 * nb2, -1);
    std::vector<int32_t> srow((size_t)nb1 * nb2, 0), trow((size_t)nb1 * nb2, 0);
    for (int i = 0; i < nsrc; ++i) {
        int x = src[3 * i] - lo[0], y = src[3 * i + 1] - lo[1], z = src[3 * i + 2] - lo[2];
        smap[((size_t)z * nb1 + y) * nb0 + x] = i;
        srow[(size_t)z * nb1 + y] = 1;
    }
    for (int i = 0; i < ntgt; ++i) {
        int x = tgt[3 * i] - lo[0], y = tgt[3 * i + 1] - lo[1], z = tgt[3 * i + 2] - lo[2];
        tmap[((size_t)z * nb1 + y) * nb0 + x] = i;
        trow[(size_t)z * nb1 + y] = 1;
    }
    plan->src_mask.assign(2 * (size_t)nb2, 0ull);
    plan->tgt_mask.assign(2 * (size_t)nb2, 0ull);
    for (int z = 0; z < nb2; ++z)
        for (int y = 0; y < nb1 && y < 128; ++y) {
            if (srow[(size_t)z * nb1 + y]) plan->src_mask[2 * z + y / 64] |= 1ull << (y % 64);
            if (trow[(size_t)z * nb1 + y]) plan->tgt_mask[2 * z + y / 64] |= 1ull << (y % 64);
        }
    plan->n_src_rows = (int)std::count(srow.begin(), srow.end(), 1);
    plan->n_tgt_rows = (int)std::count(trow.begin(), trow.end(), 1);
    if ((rc = plan->src_map.reserve(smap.size() * 4))) return rc;
    if ((rc = plan->tgt_map.reserve(tmap.size() * 4))) return rc;
    if ((rc = plan->src_rows.reserve(srow.size() * 4))) return rc;
    if ((rc = plan->tgt_rows.reserve(trow.size() * 4))) return rc;
    LGF_HIP(hipMemcpy(plan->src_map.p, smap.data(), smap.size() * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->tgt_map.p, tmap.data(), tmap.size() * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->src_rows.p, srow.data(), srow.size() * 4, hipMemcpyHostToDevice));
    LGF_HIP(hipMemcpy(plan->tgt_rows.p, trow.data(), trow.size() * 4, hipMemcpyHostToDevice));
    out = plan;
    ctx->box_plans[key] = CacheEnt<BoxPlan>{std::move(plan), ++ctx->cache_tick};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

int get_if_plan(lgfib_ctx *ctx, int B, int radius, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                std::shared_ptr<IfPlan> &out) {
    int rb = (radius + B - 1) / B;
    bool hit = false;
    uint64_t key = plan_key(ctx, 2, B, rb, src, nsrc, tgt, ntgt, &hit);
    if (hit) {
        auto it = ctx->if_plans.find(key);
        if (it != ctx->if_plans.end()) {
            it->second.tick = ++ctx->cache_tick;
            out = it->second.v;
            return LGFIB_OK;
        }
    }
    int rc = validate_blocks(src, nsrc, "source blocks");
    if (rc) return rc;
    rc = validate_blocks(tgt, ntgt, "target blocks");
    if (rc) return rc;
    auto plan = std::make_shared<IfPlan>();
    plan->B = B;
    plan->nsrc = nsrc;
    plan->ntgt = ntgt;
    plan->rb = rb;
    std::unordered_map<uint64_t, int> slot;
    slot.reserve((size_t)nsrc * 2);
    for (int i = 0; i < nsrc; ++i) slot[pack_coord(src[3 * i], src[3 * i + 1], src[3 * i + 2])] = i;
    const int w = 2 * rb + 1, w3 = w * w * w;
    std::vector<int32_t> nbr((size_t)std::max(ntgt, 1) * w3, -1);
    for (int t = 0; t < ntgt; ++t)
        for (int dz = -rb; dz <= rb; ++dz)
            for (int dy = -rb; dy <= rb; ++dy)
                for (int dx = -rb; dx <= rb; ++dx) {
                    int64_t x = (int64_t)tgt[3 * t] + dx, y = (int64_t)tgt[3 * t + 1] + dy,
                            z = (int64_t)tgt[3 * t + 2] + dz;
                    if (x < -(1 << 20) || x >= (1 << 20) || y < -(1 << 20) || y >= (1 << 20) || z < -(1 << 20) ||
                        z >= (1 << 20))
                        continue;
                    auto it = slot.find(pack_coord((int32_t)x, (int32_t)y, (int32_t)z));
                    if (it != slot.end())
                        nbr[(size_t)t * w3 + ((dz + rb) * w + (dy + rb)) * w + (dx + rb)] = it->second;
                }
    if ((rc = plan->nbr.reserve(nbr.size() * 4))) return rc;
    LGF_HIP(hipMemcpy(plan->nbr.p, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice));
    out = plan;
    ctx->if_plans[key] = CacheEnt<IfPlan>{std::move(plan), ++ctx->cache_tick};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

size_t cache_trim_all(lgfib_ctx *ctx, int cap_scale) {
    const size_t sc = cap_scale ? 1 : 0;
    const size_t sb = cap_scale ? kCacheSpectraBytes : 0, pb = cap_scale ? kCachePairSpectraBytes : 0;
    int64_t nib = 0, ncurl = 0;
    ib_cache_trim(ctx, (size_t)-1, &nib);
    curl_cache_trim(ctx, (size_t)-1, &ncurl);
    const bool over = ctx->box_plans.size() > sc * kCacheBoxPlans || ctx->if_plans.size() > sc * kCacheIfPlans ||
                      cache_over(ctx->spectra, sc * kCacheSpectra, sb) ||
                      cache_over(ctx->pair_ghat, sc * kCachePairSpectra, pb) || (size_t)nib > sc * kCacheIbPlans ||
                      (size_t)ncurl > sc * kCacheCurlPlans;
    if (!over) return 0;
    // work queued earlier may still read an entry about to be freed
    (void)hipDeviceSynchronize();
    size_t n = 0;
    // a freed plan takes its collision-guard key along
    n += cache_trim(ctx->box_plans, sc * kCacheBoxPlans, kNoByteCap, [&](uint64_t h, const BoxPlan &p) {
        ctx->plan_keys.erase(std::make_tuple(1, p.B, 0, 0, h));
    });
    n += cache_trim(ctx->if_plans, sc * kCacheIfPlans, kNoByteCap, [&](uint64_t h, const IfPlan &p) {
        ctx->plan_keys.erase(std::make_tuple(2, p.B, p.rb, 0, h));
    });
    n += cache_trim(ctx->spectra, sc * kCacheSpectra, sb);
    n += cache_trim(ctx->pair_ghat, sc * kCachePairSpectra, pb);
    n += ib_cache_trim(ctx, sc * kCacheIbPlans, nullptr);
    n += curl_cache_trim(ctx, sc * kCacheCurlPlans, nullptr);
    if (n) ++ctx->cache_epoch;
    return n;
}

void cache_counts(lgfib_ctx *ctx, int64_t out[7]) {
    out[0] = (int64_t)ctx->box_plans.size();
    out[1] = (int64_t)ctx->if_plans.size();
    out[2] = (int64_t)ctx->spectra.size();
    out[3] = (int64_t)ctx->pair_ghat.size();
    ib_cache_trim(ctx, (size_t)-1, &out[4]);    // a cap above any size only counts
    curl_cache_trim(ctx, (size_t)-1, &out[5]);
    out[6] = (int64_t)ctx->cache_epoch;
}

}  // namespace lgfib
