// ctx.cpp -- context lifetime and the thread-local error string.
#include <cstdio>

#include "internal.h"

using namespace lgfib;

extern "C" int lgfib_create(lgfib_ctx **out, int device) {
    if (!out) return fail(LGFIB_EINVAL, "lgfib_create: null output pointer");
    *out = nullptr;
    int n = 0;
    LGF_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n)
        return fail(LGFIB_EINVAL, "lgfib_create: device " + std::to_string(device) + " not present (" +
                                      std::to_string(n) + " visible)");
    LGF_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    LGF_HIP(hipGetDeviceProperties(&prop, device));
    int rc = pair_scratch_init(device);   // the static scratch's address on this device
    if (rc) return rc;
    auto *ctx = new (std::nothrow) lgfib_ctx();
    if (!ctx) return fail(LGFIB_ENOMEM, "lgfib_create: out of host memory");
    ctx->device = device;
    ctx->num_cu = prop.multiProcessorCount;
    *out = ctx;
    return LGFIB_OK;
}

static hipEvent_t prof_event(lgfib_ctx *ctx) {
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

namespace lgfib {
ProfScope::ProfScope(lgfib_ctx *c, const char *name, hipStream_t s) : ctx(c), st(s) {
    if (!ctx || !ctx->profiling) return;   // a null context times nothing
    ProfEvent ev;
    ev.name = name;
    ev.start = prof_event(ctx);
    ev.stop = prof_event(ctx);
    if (!ev.start || !ev.stop) return;
    (void)hipEventRecord(ev.start, st);
    ctx->prof_pending.push_back(ev);
    idx = (int)ctx->prof_pending.size() - 1;
}
ProfScope::~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(ctx->prof_pending[idx].stop, st);
}
}  // namespace lgfib

static int prof_drain(lgfib_ctx *ctx) {
    for (auto &ev : ctx->prof_pending) {
        LGF_HIP(hipEventSynchronize(ev.stop));
        float ms = 0.f;
        LGF_HIP(hipEventElapsedTime(&ms, ev.start, ev.stop));
        auto &a = ctx->prof_acc[ev.name];
        a.first += 1;
        a.second += ms;
        ctx->prof_pool.push_back(ev.start);
        ctx->prof_pool.push_back(ev.stop);
    }
    ctx->prof_pending.clear();
    return LGFIB_OK;
}

extern "C" int lgfib_profile_enable(lgfib_ctx *ctx, int enable) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgfib_profile_enable: null context");
    ctx->profiling = enable != 0;
    if (ctx->profiling) {
        // events are recycled after each read; create a stock up front so
        // that timed loops do not pay for event creation
        LGF_HIP(hipSetDevice(ctx->device));
        while (ctx->prof_pool.size() < 1024) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) break;
            ctx->prof_pool.push_back(e);
        }
    }
    return LGFIB_OK;
}

extern "C" int lgfib_profile_reset(lgfib_ctx *ctx) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgfib_profile_reset: null context");
    LGF_HIP(hipSetDevice(ctx->device));
    int rc = prof_drain(ctx);
    ctx->prof_acc.clear();
    return rc;
}

extern "C" int lgfib_profile_read(lgfib_ctx *ctx, int max, char *names, int *counts, double *ms, int *n) {
    if (!ctx || !n) return fail(LGFIB_EINVAL, "lgfib_profile_read: null argument");
    LGF_HIP(hipSetDevice(ctx->device));
    int rc = prof_drain(ctx);
    if (rc) return rc;
    int i = 0;
    for (auto &kv : ctx->prof_acc) {
        if (i < max && names && counts && ms) {
            snprintf(names + 64 * i, 64, "%s", kv.first.c_str());
            counts[i] = kv.second.first;
            ms[i] = kv.second.second;
        }
        ++i;
    }
    *n = i;
    return LGFIB_OK;
}

extern "C" void lgfib_destroy(lgfib_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &ev : ctx->prof_pending) {
        (void)hipEventDestroy(ev.start);
        (void)hipEventDestroy(ev.stop);
    }
    for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
    delete ctx;
}

extern "C" const char *lgfib_last_error(void) { return last_error_cstr(); }

extern "C" int lgfib_cache_release(lgfib_ctx *ctx) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgfib_cache_release: null context");
    LGF_HIP(hipSetDevice(ctx->device));
    LGF_HIP(hipDeviceSynchronize());
    cache_trim_all(ctx, 0);
    return LGFIB_OK;
}

extern "C" int lgfib_cache_info(lgfib_ctx *ctx, int64_t out[7]) {
    if (!ctx || !out) return fail(LGFIB_EINVAL, "lgfib_cache_info: null argument");
    cache_counts(ctx, out);
    return LGFIB_OK;
}
