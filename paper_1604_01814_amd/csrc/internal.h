// internal.h -- shared host-side types of the lgfib library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lgfib.h"

namespace lgfib {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define LGF_HIP(call)                                                             \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return ::lgfib::fail(LGFIB_EHIP, std::string(#call) + ": " +           \
                                                 hipGetErrorString(e_));          \
    } while (0)

// ------------------------------------------------------------ device memory
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow-only; contents are not preserved
    int reserve(size_t n) {
        if (n <= bytes) return LGFIB_OK;
        release();
        if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
            return fail(LGFIB_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
        return LGFIB_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ------------------------------------------------------------ block sets
struct BlockList {
    std::vector<int32_t> xyz;   // 3 per block
    int n() const { return (int)(xyz.size() / 3); }
};

// Validate a host block list: coordinates in range, no duplicates.
int validate_blocks(const int32_t *blocks, int n, const char *what);

// Smallest 2,3,5-smooth integer >= n.
int smooth_ceil(int n);

// A box-FFT plan for one (B, sources, targets) triple: the bounding box of the
// union, its padded FFT sizes, and device maps from box blocks to list slots.
struct BoxPlan {
    int B = 0;
    int lo[3] = {0, 0, 0};     // lowest block coordinate of the box
    int nb[3] = {0, 0, 0};     // box size in blocks (smooth-rounded)
    int N[3] = {0, 0, 0};      // box size in cells = nb * B
    int P[3] = {0, 0, 0};      // FFT length per axis = 2 N
    int Kx = 0;                // P[0]/2 + 1 retained x frequencies
    int Kxp = 0;               // Kx rounded up to the pencil tile
    int nsrc = 0, ntgt = 0;
    DevBuf src_map;            // int32 [nb2][nb1][nb0] -> source slot or -1
    DevBuf tgt_map;            // int32 [nb2][nb1][nb0] -> target slot or -1
    DevBuf tgt_rows;           // int32 list of (y, z) box rows holding targets
    int n_tgt_rows = 0;
    DevBuf src_rows;           // int32 list of (y, z) box rows holding sources
    int n_src_rows = 0;
    // per z block plane, bit y of the block rows holding sources / targets
    // (two words, y < 128), for the kernels' plane skipping
    std::vector<uint64_t> src_mask, tgt_mask;   // [nb2][2]
};

// Plan for the integrating-factor stencil: target slot -> neighbour source
// slots within the stencil's block radius.
struct IfPlan {
    int B = 0, nsrc = 0, ntgt = 0, rb = 0;   // rb: block radius of the stencil
    DevBuf nbr;                               // int32 [ntgt][(2rb+1)^3]
};

struct Table {
    int kind = 0;
    double alpha = 0.0;
    int ext[3] = {0, 0, 0};
    DevBuf g;   // double [(e3+1)(e2+1)(e1+1)]
};

struct Spectrum {
    int prec = 0;
    int P[3] = {0, 0, 0};
    int Kxp = 0;
    DevBuf ghat;   // real, [P2/2+1][P1/2+1][Kxp] of float or double
};

// ------------------------------------------------------------ plan caches
// Plans, kernel spectra and operator tables are cached per context under the
// exact lists they were made for.  Each cache keeps at most a fixed number of
// entries: once full, the least recently used entry that nothing else holds
// (shared_ptr use count 1) is freed.  Objects that keep a plan beyond one call
// (batches, IB systems) hold a shared_ptr to it, which pins it.  Freeing goes
// through hipFree, which waits for the device, so no queued kernel still
// reads an evicted plan.
template <class V> struct CacheEnt {
    std::shared_ptr<V> v;
    uint64_t tick = 0;
    size_t bytes = 0;   // device bytes the entry holds
};
// entry caps per cache, and device-byte caps for the kernel spectra
constexpr size_t kCacheBoxPlans = 256, kCacheIfPlans = 256, kCacheSpectra = 64, kCachePairSpectra = 8,
                 kCacheIbPlans = 64, kCacheCurlPlans = 64;
constexpr size_t kCacheSpectraBytes = (size_t)4 << 30, kCachePairSpectraBytes = (size_t)8 << 30;
constexpr size_t kNoByteCap = ~(size_t)0;

template <class M> size_t cache_bytes(const M &m) {
    size_t b = 0;
    for (const auto &e : m) b += e.second.bytes;
    return b;
}
template <class M> bool cache_over(const M &m, size_t cap, size_t cap_bytes) {
    return m.size() > cap || (cap_bytes != kNoByteCap && cache_bytes(m) > cap_bytes);
}
// Free the least recently used entries that nothing else holds until at
// most cap entries and cap_bytes device bytes remain (or only held entries
// are left); returns the number freed.
template <class M, class OnEvict> size_t cache_trim(M &m, size_t cap, size_t cap_bytes, OnEvict on_evict) {
    size_t n = 0;
    while (cache_over(m, cap, cap_bytes)) {
        auto victim = m.end();
        for (auto it = m.begin(); it != m.end(); ++it)
            if (it->second.v.use_count() == 1 && (victim == m.end() || it->second.tick < victim->second.tick))
                victim = it;
        if (victim == m.end()) break;   // every remaining entry is pinned
        on_evict(victim->first, *victim->second.v);
        m.erase(victim);
        ++n;
    }
    return n;
}
template <class M> size_t cache_trim(M &m, size_t cap, size_t cap_bytes = kNoByteCap) {
    return cache_trim(m, cap, cap_bytes, [](const auto &, const auto &) {});
}

}  // namespace lgfib

namespace lgfib {
struct ProfEvent {
    std::string name;
    hipEvent_t start = nullptr, stop = nullptr;
};
}  // namespace lgfib

struct lgfib_ctx {
    int device = 0;
    bool profiling = false;
    std::vector<lgfib::ProfEvent> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    std::map<std::string, std::pair<int, double>> prof_acc;
    int num_cu = 0;
    std::vector<std::unique_ptr<lgfib::Table>> tables;
    std::map<std::tuple<int, int, int, int, int>, lgfib::CacheEnt<lgfib::Spectrum>> spectra;  // (tbl, P0, P1, P2, prec)
    std::map<uint64_t, lgfib::CacheEnt<lgfib::BoxPlan>> box_plans;
    std::map<uint64_t, lgfib::CacheEnt<lgfib::IfPlan>> if_plans;
    std::map<std::tuple<int, int, int, int, uint64_t>, std::vector<int32_t>> plan_keys;  // collision guard
    lgfib::DevBuf work1, work2;   // FFT workspaces
    lgfib::DevBuf scratch;        // small per-call scratch
    std::map<std::pair<int, int>, std::unique_ptr<lgfib::DevBuf>> twiddles;   // (P, prec) -> table
    std::map<std::pair<double, int>, std::pair<int, std::unique_ptr<lgfib::DevBuf>>> if_weights;  // (a, prec) -> (r, weights)
    std::map<std::tuple<int, int, int, int>, lgfib::CacheEnt<lgfib::DevBuf>> pair_ghat;  // (tbl, span) -> spectra
    uint64_t cache_tick = 0;    // use counter of the caches (least recently used goes first)
    uint64_t cache_epoch = 0;   // bumped whenever a cached entry is freed: captured graphs check it
    std::shared_ptr<void> ib_cache;   // IB operator plans (ib.hip), freed with the context
    std::shared_ptr<void> refresh_cache;   // velocity-refresh plans (curl.hip)
    std::shared_ptr<void> lamb_cache;      // nonlinear-term plans (curl.hip)
    lgfib::DevBuf dense_ws, dense_flag, dense_solve_ws;   // dense factorisation / solve workspaces
    lgfib::DevBuf adapt_ws;   // device flow-domain update (curl.hip)
};

namespace lgfib {
// plans (blockset.cpp)
int get_box_plan(lgfib_ctx *ctx, int B, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                 std::shared_ptr<BoxPlan> &out);
int get_if_plan(lgfib_ctx *ctx, int B, int radius, const int32_t *src, int nsrc, const int32_t *tgt,
                int ntgt, std::shared_ptr<IfPlan> &out);
// trim every cache to its capacity (cap_scale 1) or empty it (0); returns the
// number of entries freed and bumps cache_epoch when any was
size_t cache_trim_all(lgfib_ctx *ctx, int cap_scale);
// the IB and curl-operator caches: trim to cap, report the entries left in *left
size_t ib_cache_trim(lgfib_ctx *ctx, size_t cap, int64_t *left);     // ib.hip
size_t curl_cache_trim(lgfib_ctx *ctx, size_t cap, int64_t *left);   // curl.hip
void cache_counts(lgfib_ctx *ctx, int64_t out[7]);
// resolve the allocation-free entry point's static scratch on a device (pair.hip)
int pair_scratch_init(int device);
uint64_t hash_blocks(uint64_t h, const int32_t *b, int n);
// tables (table.hip)
int get_spectrum(lgfib_ctx *ctx, lgf_table_t tbl, const BoxPlan &plan, int prec, hipStream_t s,
                 std::shared_ptr<Spectrum> &out);
int bessel_weights_host(double x, int nmax, std::vector<double> &out, hipStream_t s);
// FFT twiddles (conv.hip)
int get_twiddles(lgfib_ctx *ctx, int P, int prec, const void **dev);
const char *last_error_cstr();
// kernel timing: open() records a start event when profiling is on; close()
// records the stop event (both on the launch stream)
struct ProfScope {
    lgfib_ctx *ctx;
    hipStream_t st;
    int idx = -1;
    ProfScope(lgfib_ctx *c, const char *name, hipStream_t s);
    ~ProfScope();
};
// integrating-factor weights (if_apply.hip)
int get_if_weights(lgfib_ctx *ctx, double a, int prec, int *radius, const double **dev);
// dense FP64 linear algebra (dense.hip): row-major matrices with leading dimensions
// tri: which operand is lower triangular, so that its zero part is skipped
enum GemmTri { kTriNone = 0, kTriBtLower = 1, kTriBLower = 2, kTriALower = 3 };
int gemm_f64(int M, int N, int K, double alpha, const double *A, long lda, const double *B, long ldb, bool tb,
             double beta, double *C, long ldc, bool lower, int tri, hipStream_t st);
int chol_factor_f64(lgfib_ctx *ctx, int n, double *A, long lda, double *W, long ldw, hipStream_t st);
int chol_solve_f64(lgfib_ctx *ctx, int n, const double *W, long ldw, const double *b, double *x, hipStream_t st);
// nonlinear term in rotational form (curl.hip): out = scale * (C u) x (u + U)
// on the faces of the blocks, [3][nblk][B^3] of prec; U may be null (zero)
int lamb_apply(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, double scale, int prec,
               const void *u, void *out, hipStream_t st);
}  // namespace lgfib
