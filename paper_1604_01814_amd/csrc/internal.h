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
    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<lgfib::Spectrum>> spectra;  // (tbl, P0, P1, P2, prec)
    std::map<uint64_t, std::unique_ptr<lgfib::BoxPlan>> box_plans;
    std::map<uint64_t, std::unique_ptr<lgfib::IfPlan>> if_plans;
    std::map<std::tuple<int, int, int, int, uint64_t>, std::vector<int32_t>> plan_keys;  // collision guard
    lgfib::DevBuf work1, work2;   // FFT workspaces
    lgfib::DevBuf scratch;        // small per-call scratch
    std::map<std::pair<int, int>, std::unique_ptr<lgfib::DevBuf>> twiddles;   // (P, prec) -> table
    std::map<double, std::pair<int, std::unique_ptr<lgfib::DevBuf>>> if_weights;  // a -> (r, weights)
    std::map<std::tuple<int, int, int, int>, std::unique_ptr<lgfib::DevBuf>> pair_ghat;  // (tbl, span) -> spectra
    std::shared_ptr<void> ib_cache;   // IB operator plans (ib.hip), freed with the context
    std::shared_ptr<void> refresh_cache;   // velocity-refresh plans (curl.hip)
    std::shared_ptr<void> lamb_cache;      // nonlinear-term plans (curl.hip)
    lgfib::DevBuf dense_ws, dense_flag, dense_solve_ws;   // dense factorisation / solve workspaces
};

namespace lgfib {
// plans (blockset.cpp)
int get_box_plan(lgfib_ctx *ctx, int B, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                 BoxPlan **out);
int get_if_plan(lgfib_ctx *ctx, int B, int radius, const int32_t *src, int nsrc, const int32_t *tgt,
                int ntgt, IfPlan **out);
uint64_t hash_blocks(uint64_t h, const int32_t *b, int n);
// tables (table.hip)
int get_spectrum(lgfib_ctx *ctx, lgf_table_t tbl, const BoxPlan &plan, int prec, hipStream_t s,
                 Spectrum **out);
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
int get_if_weights(lgfib_ctx *ctx, double a, int *radius, const double **dev);
// dense FP64 linear algebra (dense.hip): row-major matrices with leading dimensions
int gemm_f64(int M, int N, int K, double alpha, const double *A, long lda, const double *B, long ldb, bool tb,
             double beta, double *C, long ldc, bool lower, hipStream_t st);
int chol_factor_f64(lgfib_ctx *ctx, int n, double *A, long lda, double *W, long ldw, hipStream_t st);
int chol_solve_f64(lgfib_ctx *ctx, int n, const double *W, long ldw, const double *b, double *x, hipStream_t st);
// nonlinear term in rotational form (curl.hip): out = scale * (C u) x (u + U)
// on the faces of the blocks, [3][nblk][B^3] of prec; U may be null (zero)
int lamb_apply(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, double scale, int prec,
               const void *u, void *out, hipStream_t st);
}  // namespace lgfib
