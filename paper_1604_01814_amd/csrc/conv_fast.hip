// conv_fast.hip -- FP32 box-FFT passes specialised at compile time on the FFT
// length of their axis (the hot path of lgf_poisson_apply).  Same five passes,
// data layout and arithmetic as the generic kernels in conv.hip; the lengths
// 32..1024 with radices {2,3,4,5,8,16} are instantiated, other boxes fall back
// to the generic kernels.
#include "conv_common.h"
#include "fft_static.h"

namespace lgfib {

using C32 = float2;

// Pencils per workgroup: the largest power of two <= 16 whose LDS footprint
// (half twiddle table + pencils [+ kernel spectrum column]) fits in 64 KiB.
constexpr int kLdsBudget = 65536;
constexpr int np_fit(int P, int extra_per_pencil) {
    int np = 16;
    while (np > 1 && (P / 2 + np * P) * 8 + np * extra_per_pencil > kLdsBudget) np /= 2;
    return np;
}
template <int P> constexpr int np_rows() { return np_fit(P, 0); }
template <int P> constexpr int np_cols() { return np_fit(P, 0); }
template <int P> constexpr int np_zconv() { return np_fit(P, (P / 2 + 1) * 4); }

__device__ __forceinline__ void load_tw(C32 *dst, const C32 *__restrict__ src, int P) {
    for (int i = threadIdx.x; i < P / 2; i += kFftThreads) dst[i] = src[i];
}

// ------------------------------------------------------------------- pass 1
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_xfwd(BoxGeo g, const float *__restrict__ f, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg) {
    constexpr int NP = np_rows<P>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int c = blockIdx.y;
    const int nrows = g.N1 * g.N2;
    const int row0 = blockIdx.x * 2 * NP;
    const int lb = g.lb, B = 1 << lb, bm = B - 1;
    bool any = false;
    for (int q = 0; q < 2 * NP; ++q) {
        const int row = row0 + q;
        if (row < nrows) {
            const int y = row % g.N1, z = row / g.N1;
            any |= g.src_rows[(z >> lb) * g.nb1 + (y >> lb)] != 0;
        }
    }
    if (!any) return;
    load_tw(tw, twg, P);
    const size_t fbase = (size_t)c * g.nsrc << (3 * lb);
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx / P, x = idx % P;
        float va = 0.f, vb = 0.f;
        if (x < g.N0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = row0 + 2 * p + h;
                float v = 0.f;
                if (row < nrows) {
                    const int y = row % g.N1, z = row / g.N1;
                    const int slot = g.src_map[((z >> lb) * g.nb1 + (y >> lb)) * g.nb0 + (x >> lb)];
                    if (slot >= 0)
                        v = f[fbase + ((size_t)slot << (3 * lb)) + (((z & bm) << (2 * lb)) | ((y & bm) << lb) | (x & bm))];
                }
                if (h == 0) va = v; else vb = v;
            }
        }
        s[p * P + x] = C32{va, vb};
    }
    __syncthreads();
    sfft<C32, P, NP, P, 1, false, false>(s, tw);
    const int Kxp = g.Kxp, Kx = g.Kx;
    for (int idx = threadIdx.x; idx < NP * Kxp; idx += kFftThreads) {
        const int p = idx / Kxp, k = idx - p * Kxp;
        C32 xa = C32{0.f, 0.f}, xb = C32{0.f, 0.f};
        if (k < Kx) {
            const C32 zk = s[p * P + k];
            const C32 zm = s[p * P + (k == 0 ? 0 : P - k)];
            xa = C32{0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)};
            xb = C32{0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x)};
        }
        const int ra = row0 + 2 * p, rb = ra + 1;
        if (ra < nrows) X1[((size_t)c * nrows + ra) * Kxp + k] = xa;
        if (rb < nrows) X1[((size_t)c * nrows + rb) * Kxp + k] = xb;
    }
}

// ------------------------------------------------------------------- pass 2
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_yfwd(BoxGeo g, const C32 *__restrict__ X1, C32 *__restrict__ X2,
                                                       const C32 *__restrict__ twg) {
    constexpr int NP = np_cols<P>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int k0 = blockIdx.x * NP, z = blockIdx.y, c = blockIdx.z;
    const int lb = g.lb, Kxp = g.Kxp;
    load_tw(tw, twg, P);
    const size_t in0 = ((size_t)c * g.N2 + z) * g.N1;
    const int *srow = g.src_rows + (z >> lb) * g.nb1;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, y = idx / NP;
        C32 v = C32{0.f, 0.f};
        if (y < g.N1 && srow[y >> lb]) v = X1[(in0 + y) * Kxp + k0 + p];
        s[y * NP + p] = v;
    }
    __syncthreads();
    sfft<C32, P, NP, 1, NP, true, false>(s, tw);
    const size_t out0 = ((size_t)c * g.N2 + z) * P;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, ky = idx / NP;
        X2[(out0 + ky) * Kxp + k0 + p] = s[ky * NP + p];
    }
}

// ------------------------------------------------------------------- pass 3
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_zconv(BoxGeo g, C32 *__restrict__ X2, const float *__restrict__ ghat,
                                                        float scale, const C32 *__restrict__ twg) {
    constexpr int NP = np_zconv<P>();
    constexpr int Ph = P / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    float *gh = reinterpret_cast<float *>(s + NP * P);
    const int Kxp = g.Kxp;
    const int k0 = blockIdx.x * NP, ky = blockIdx.y;
    const int kyh = min(ky, g.P1 - ky);
    const int H1 = g.P1 / 2 + 1;
    load_tw(tw, twg, P);
    for (int idx = threadIdx.x; idx < NP * (Ph + 1); idx += kFftThreads) {
        const int p = idx % NP, kz = idx / NP;
        gh[kz * NP + p] = scale * ghat[((size_t)kz * H1 + kyh) * Kxp + k0 + p];
    }
    for (int c = 0; c < g.ncomp; ++c) {
        const size_t base = (size_t)c * g.N2 * g.P1;
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, z = idx / NP;
            C32 v = C32{0.f, 0.f};
            if (z < g.N2) v = X2[((base + (size_t)z * g.P1) + ky) * Kxp + k0 + p];
            s[z * NP + p] = v;
        }
        __syncthreads();
        sfft<C32, P, NP, 1, NP, true, false>(s, tw);
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, kz = idx / NP;
            const float w = gh[min(kz, P - kz) * NP + p];
            const C32 v = s[kz * NP + p];
            s[kz * NP + p] = C32{v.x * w, v.y * w};
        }
        __syncthreads();
        sfft<C32, P, NP, 1, NP, true, true>(s, tw);
        for (int idx = threadIdx.x; idx < NP * g.N2; idx += kFftThreads) {
            const int p = idx % NP, zz = idx / NP;
            X2[((base + (size_t)zz * g.P1) + ky) * Kxp + k0 + p] = s[zz * NP + p];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------- pass 4
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_yinv(BoxGeo g, const C32 *__restrict__ X2, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg) {
    constexpr int NP = np_cols<P>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int k0 = blockIdx.x * NP, z = blockIdx.y, c = blockIdx.z;
    const int lb = g.lb, Kxp = g.Kxp;
    const int *trow = g.tgt_rows + (z >> lb) * g.nb1;
    bool any = false;
    for (int by = 0; by < g.nb1; ++by) any |= trow[by] != 0;
    if (!any) return;
    load_tw(tw, twg, P);
    const size_t in0 = ((size_t)c * g.N2 + z) * P;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, ky = idx / NP;
        s[ky * NP + p] = X2[(in0 + ky) * Kxp + k0 + p];
    }
    __syncthreads();
    sfft<C32, P, NP, 1, NP, true, true>(s, tw);
    const size_t out0 = ((size_t)c * g.N2 + z) * g.N1;
    for (int idx = threadIdx.x; idx < NP * g.N1; idx += kFftThreads) {
        const int p = idx % NP, y = idx / NP;
        if (trow[y >> lb]) X1[(out0 + y) * Kxp + k0 + p] = s[y * NP + p];
    }
}

// ------------------------------------------------------------------- pass 5
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_xinv(BoxGeo g, const C32 *__restrict__ X1, float *__restrict__ u,
                                                       int accumulate, const C32 *__restrict__ twg) {
    constexpr int NP = np_rows<P>();
    constexpr int Ph = P / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int c = blockIdx.y;
    const int nrows = g.N1 * g.N2;
    const int row0 = blockIdx.x * 2 * NP;
    const int lb = g.lb, bm = (1 << lb) - 1;
    bool any = false;
    for (int q = 0; q < 2 * NP; ++q) {
        const int row = row0 + q;
        if (row < nrows) {
            const int y = row % g.N1, z = row / g.N1;
            any |= g.tgt_rows[(z >> lb) * g.nb1 + (y >> lb)] != 0;
        }
    }
    if (!any) return;
    load_tw(tw, twg, P);
    const int Kx = g.Kx, Kxp = g.Kxp;
    for (int idx = threadIdx.x; idx < NP * Kx; idx += kFftThreads) {
        const int p = idx / Kx, k = idx - p * Kx;
        C32 xa = C32{0.f, 0.f}, xb = C32{0.f, 0.f};
        const int ra = row0 + 2 * p, rb = ra + 1;
        if (ra < nrows && g.tgt_rows[((ra / g.N1) >> lb) * g.nb1 + ((ra % g.N1) >> lb)])
            xa = X1[((size_t)c * nrows + ra) * Kxp + k];
        if (rb < nrows && g.tgt_rows[((rb / g.N1) >> lb) * g.nb1 + ((rb % g.N1) >> lb)])
            xb = X1[((size_t)c * nrows + rb) * Kxp + k];
        if (k == 0 || k == Ph) {
            xa.y = 0.f;
            xb.y = 0.f;
        }
        s[p * P + k] = C32{xa.x - xb.y, xa.y + xb.x};
        if (k > 0 && k < Ph) s[p * P + P - k] = C32{xa.x + xb.y, xb.x - xa.y};
    }
    __syncthreads();
    sfft<C32, P, NP, P, 1, false, true>(s, tw);
    const size_t ubase = (size_t)c * g.ntgt << (3 * lb);
    for (int idx = threadIdx.x; idx < NP * g.N0; idx += kFftThreads) {
        const int p = idx / g.N0, x = idx - p * g.N0;
        const C32 v = s[p * P + x];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = row0 + 2 * p + h;
            if (row < nrows) {
                const int y = row % g.N1, z = row / g.N1;
                const int slot = g.tgt_map[((z >> lb) * g.nb1 + (y >> lb)) * g.nb0 + (x >> lb)];
                if (slot >= 0) {
                    float *dst = u + ubase + ((size_t)slot << (3 * lb)) +
                                 (((z & bm) << (2 * lb)) | ((y & bm) << lb) | (x & bm));
                    const float val = h == 0 ? v.x : v.y;
                    *dst = accumulate ? *dst + val : val;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ dispatch

#define LGF_FAST_SIZES(X) \
    X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(480) X(512) X(640) X(768) X(960) X(1024)

bool fast_size(int P) {
    switch (P) {
#define X(n) case n:
        LGF_FAST_SIZES(X)
#undef X
        return true;
    default: return false;
    }
}

int fast_np_rows(int P) { return np_fit(P, 0); }
int fast_np_cols(int P) { return np_fit(P, 0); }
int fast_np_zconv(int P) { return np_fit(P, (P / 2 + 1) * 4); }

int launch_fast_xfwd(const BoxGeo &g, const float *f, C32 *X1, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_rows(g.P0);
    const int nrows = g.N1 * g.N2;
    dim3 grid((nrows + 2 * NP - 1) / (2 * NP), g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0);
    switch (g.P0) {
#define X(n) case n: hipLaunchKernelGGL(kf_xfwd<n>, grid, dim3(kFftThreads), sm, st, g, f, X1, tw); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_yfwd(const BoxGeo &g, const C32 *X1, C32 *X2, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_cols(g.P1);
    dim3 grid(g.Kxp / NP, g.N2, g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1);
    switch (g.P1) {
#define X(n) case n: hipLaunchKernelGGL(kf_yfwd<n>, grid, dim3(kFftThreads), sm, st, g, X1, X2, tw); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised y pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_zconv(const BoxGeo &g, C32 *X2, const float *ghat, float scale, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_zconv(g.P2);
    dim3 grid(g.Kxp / NP, g.P1);
    const size_t sm = sizeof(C32) * (size_t)(g.P2 / 2 + NP * g.P2) + sizeof(float) * (size_t)NP * (g.P2 / 2 + 1);
    switch (g.P2) {
#define X(n) case n: hipLaunchKernelGGL(kf_zconv<n>, grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised z pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_yinv(const BoxGeo &g, const C32 *X2, C32 *X1, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_cols(g.P1);
    dim3 grid(g.Kxp / NP, g.N2, g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1);
    switch (g.P1) {
#define X(n) case n: hipLaunchKernelGGL(kf_yinv<n>, grid, dim3(kFftThreads), sm, st, g, X2, X1, tw); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised y pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_xinv(const BoxGeo &g, const C32 *X1, float *u, int accumulate, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_rows(g.P0);
    const int nrows = g.N1 * g.N2;
    dim3 grid((nrows + 2 * NP - 1) / (2 * NP), g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0);
    switch (g.P0) {
#define X(n) case n: hipLaunchKernelGGL(kf_xinv<n>, grid, dim3(kFftThreads), sm, st, g, X1, u, accumulate, tw); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

}  // namespace lgfib
