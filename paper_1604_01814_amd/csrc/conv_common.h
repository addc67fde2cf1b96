// conv_common.h -- geometry shared by the generic and the specialised box-FFT
// convolution kernels.
#pragma once

#include "internal.h"

namespace lgfib {

// Workgroup ids are dispatched round-robin over the 8 XCDs (id % 8); this maps
// id L of N to a logical index so that each XCD receives one contiguous run,
// and neighbouring logical tiles (which share cache lines or halos) meet in
// the same L2.
__device__ __forceinline__ int xcd_remap(int L, int N) {
    const int q = N / 8, rem = N % 8, x = L % 8, j = L / 8;
    return x * q + min(x, rem) + j;
}

struct BoxGeo {
    int B, lb;              // block edge and log2(B)
    int nb0, nb1, nb2;      // box size in blocks
    int N0, N1, N2;         // box size in cells
    int P0, P1, P2;         // FFT lengths (2 N)
    int Kx, Kxp;            // retained x frequencies, padded row length
    int nsrc, ntgt, ncomp;
    const int *src_map;     // [nb2][nb1][nb0] -> source slot or -1
    const int *tgt_map;     // [nb2][nb1][nb0] -> target slot or -1
    const int *src_rows;    // [nb2][nb1] != 0 where a source block sits
    const int *tgt_rows;    // [nb2][nb1] != 0 where a target block sits
    // the same flags as bit masks per z block plane, passed by value so that
    // the kernels test them without memory loads (valid when masks_ok)
    static constexpr int kMaskPlanes = 64;
    int masks_ok;
    unsigned long long src_mask[kMaskPlanes][2], tgt_mask[kMaskPlanes][2];
};

// The kernels' view of a box plan for ncomp components (conv.hip).
void make_box_geo(const BoxPlan &plan, int ncomp, BoxGeo &g);

// FP32 passes specialised on the FFT length (conv_fast.hip)
bool fast_size(int P);
bool fast_x_ok(const BoxGeo &g);   // x passes need B*B rows divisible by the row tile
int launch_fast_xfwd(const BoxGeo &g, const float *f, float2 *X1, const float2 *tw, hipStream_t st);
int launch_fast_yfwd(const BoxGeo &g, const float2 *X1, float2 *X2, const float2 *tw, hipStream_t st);
int launch_fast_zconv(const BoxGeo &g, float2 *X2, const float *ghat, float scale, const float2 *tw, hipStream_t st);
// the z pass in FP64 for the specialised lengths that fit (fast_z64_size)
bool fast_z64_size(int P);
int launch_fast_zconv_f64(const BoxGeo &g, double2 *X2, const double *ghat, double scale, const double2 *tw,
                          hipStream_t st);
int launch_fast_yinv(const BoxGeo &g, const float2 *X2, float2 *X1, const float2 *tw, hipStream_t st);
// the y passes in FP64 for the specialised lengths that fit (fast_y64_size)
bool fast_y64_size(int P);
int launch_fast_yfwd_f64(const BoxGeo &g, const double2 *X1, double2 *X2, const double2 *tw, hipStream_t st);
int launch_fast_yinv_f64(const BoxGeo &g, const double2 *X2, double2 *X1, const double2 *tw, hipStream_t st);
int launch_fast_xinv(const BoxGeo &g, const float2 *X1, float *u, int accumulate, const float2 *tw, hipStream_t st);

// Batched passes (many box convolutions, one launch per pass and FFT length):
// an instance's share of one pass, in device memory.
struct FastJob {
    BoxGeo g;
    const void *in;       // f, X1, X2, X2, X1 for the passes 0..4
    void *out;            // X1, X2, X2 (in place), X1, u
    const float *ghat;    // z pass: kernel spectrum
    const float2 *tw;     // twiddles of the pass's FFT length
    float scale;          // z pass: dx^2 / (P0 P1 P2)
    int acc;              // x inverse: accumulate into u
    int n, T;             // the pass's tile count (x: chunks per block row) and tiles per workgroup
};
enum { kPassXF = 0, kPassYF = 1, kPassZ = 2, kPassYI = 3, kPassXI = 4, kNumPasses = 5 };
// Fill the five jobs of one instance (geometry g, FP32, fast sizes only) and
// the number of work items each contributes; *sm receives each pass's LDS
// bytes and *P its FFT length.  tpx / tpy: tiles per workgroup (0: defaults).
int fast_jobs(const BoxGeo &g, const float *f, float *u, float2 *X1, float2 *X2, const float *ghat, float scale,
              const float2 *const tw[3], int tpx, int tpy, FastJob jobs[kNumPasses], int items[kNumPasses],
              size_t sm[kNumPasses], int P[kNumPasses]);
// One persistent launch of pass `pass` over njobs instances of FFT length P:
// work items start[k] .. start[k + 1] - 1 belong to instance k (owner[item]
// = k); the grid pulls items from *queue, which must hold 0.
int launch_fast_batched(int pass, int P, const FastJob *jobs, const int *start, const int *owner, int njobs,
                        int total, int *queue, size_t sm, int num_cu, hipStream_t st);

// Per-thread settings of a batched launch while it enqueues one instance:
// tiles per workgroup of the x / y passes (0: the defaults) and the FFT
// workspaces to use instead of the context's (null: the context's).
struct ConvOverrides {
    int tpw_x = 0, tpw_y = 0;
    void *w1 = nullptr, *w2 = nullptr;
    size_t w1_bytes = 0, w2_bytes = 0;
};
ConvOverrides &conv_overrides();

// Bytes of the two FFT workspaces a box convolution needs.
void box_work_bytes(const BoxPlan &plan, int ncomp, int prec, size_t *w1, size_t *w2);
// The FP32 box convolution on a resolved plan and kernel spectrum.
int box_conv_f32(lgfib_ctx *ctx, const BoxPlan &plan, const Spectrum &spec, int ncomp, double dx, const float *f,
                 float *u, int accumulate, hipStream_t st);

// Block-pair form for 8^3 blocks (pair.hip): a resolved source/target pair
// set -- the kernel spectra of its span and the block lists on the device.
struct PairExec {
    int nsrc = 0, ntgt = 0, ngrp = 0;
    int D[3] = {0, 0, 0};
    std::shared_ptr<DevBuf> ghat;   // cached in the context; held here while in use
    DevBuf lists;             // int32: source / target positions, sorted source order and positions, target groups
};
int pair_prepare(lgfib_ctx *ctx, lgf_table_t tbl, const int32_t *src, int nsrc, const int32_t *tgt, int ntgt,
                 PairExec &px, hipStream_t st);
size_t pair_work_bytes(int n, int ncomp);
int pair_enqueue(lgfib_ctx *ctx, const PairExec &px, int ncomp, int dft, double dx, const float *f, float *u,
                 void *wf, void *wu, hipStream_t st);

}  // namespace lgfib
