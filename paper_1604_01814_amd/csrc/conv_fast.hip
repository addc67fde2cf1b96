// conv_fast.hip -- FP32 box-FFT passes specialised at compile time on the FFT
// length of their axis (the hot path of lgf_poisson_apply).  Same five passes,
// data layout and arithmetic as the generic kernels in conv.hip; the lengths
// 32..1024 with radices {2,3,4,5,8,16} are instantiated, other boxes fall back
// to the generic kernels.
#include <algorithm>
#include <cstdlib>

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

// All passes walk T consecutive tiles per workgroup.  The next tile's global
// data is loaded into registers right after the current tile has been staged
// in LDS, so those loads are in flight while the current tile is transformed
// (the FFT's barriers order LDS only and do not wait for them).

// Box row r = z * N1 + y of a tile starting at row0 = z0 * N1 + y0: rows of a
// tile are consecutive, so (y, z) follows from (y0, z0) by a short wrap loop
// instead of a division per element.
struct RowPos {
    int y, z;
};
__device__ __forceinline__ RowPos row_pos(int y0, int z0, int q, int N1) {
    int y = y0 + q, z = z0;
    while (y >= N1) {
        y -= N1;
        ++z;
    }
    return RowPos{y, z};
}

// ------------------------------------------------------------------- pass 1
// Tile = 2*NP consecutive box rows (y fastest, then z) of one component.
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_xfwd(BoxGeo g, const float *__restrict__ f, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg, int ntiles, int T) {
    constexpr int NP = np_rows<P>();
    constexpr int N = P / 2;
    constexpr int NL = NP * N;   // (row pair, x) loads per tile
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int nrows = g.N1 * g.N2;
    const int ngroups = (nrows + 2 * NP - 1) / (2 * NP);
    const int lb = g.lb, bm = (1 << lb) - 1;
    load_tw(tw, twg, P);
    auto has_src_yz = [&](RowPos rp) { return g.src_rows[(rp.z >> lb) * g.nb1 + (rp.y >> lb)] != 0; };
    C32 pre[E];
    auto load = [&](int t) {
        const int c = t / ngroups, row0 = (t % ngroups) * 2 * NP;
        const int y0 = row0 % g.N1, z0 = row0 / g.N1;
        const size_t fbase = (size_t)c * g.nsrc << (3 * lb);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            float va = 0.f, vb = 0.f;
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / N, x = idx % N;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int row = row0 + 2 * p + h;
                    if (row < nrows) {
                        const RowPos rp = row_pos(y0, z0, 2 * p + h, g.N1);
                        const int y = rp.y, z = rp.z;
                        const int slot = g.src_map[((z >> lb) * g.nb1 + (y >> lb)) * g.nb0 + (x >> lb)];
                        if (slot >= 0) {
                            const float v = f[fbase + ((size_t)slot << (3 * lb)) +
                                              (((z & bm) << (2 * lb)) | ((y & bm) << lb) | (x & bm))];
                            if (h == 0) va = v; else vb = v;
                        }
                    }
                }
            }
            pre[e] = C32{va, vb};
        }
    };
    const int t0 = blockIdx.x * T;
    if (t0 < ntiles) load(t0);
    for (int i = 0; i < T; ++i) {
        const int t = t0 + i;
        if (t >= ntiles) break;
        const int c = t / ngroups, row0 = (t % ngroups) * 2 * NP;
        const int y0 = row0 % g.N1, z0 = row0 / g.N1;
        auto has_src = [&](int q) { return row0 + q < nrows && has_src_yz(row_pos(y0, z0, q, g.N1)); };
        // rows without sources are never read by pass 2: skip them
        bool active = false;
        for (int q = 0; q < 2 * NP; ++q) active |= has_src(q);
        if (!active) {
            if (i + 1 < T && t + 1 < ntiles) load(t + 1);
            continue;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) s[(idx / N) * P + idx % N] = pre[e];
        }
        for (int idx = threadIdx.x; idx < NL; idx += kFftThreads) s[(idx / N) * P + N + idx % N] = C32{0.f, 0.f};
        lds_barrier();
        if (i + 1 < T && t + 1 < ntiles) load(t + 1);
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
            if (has_src(2 * p)) X1[((size_t)c * nrows + ra) * Kxp + k] = xa;
            if (has_src(2 * p + 1)) X1[((size_t)c * nrows + rb) * Kxp + k] = xb;
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 2
// Tile = (kx tile of NP columns, z, component); kx tile fastest.
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_yfwd(BoxGeo g, const C32 *__restrict__ X1, C32 *__restrict__ X2,
                                                       const C32 *__restrict__ twg, int ntiles, int T) {
    constexpr int NP = np_cols<P>();
    constexpr int N = P / 2;
    constexpr int NL = NP * N;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int lb = g.lb, Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    load_tw(tw, twg, P);
    C32 pre[E];
    auto load = [&](int t) {
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
        const size_t in0 = ((size_t)c * g.N2 + z) * N;
        const int *srow = g.src_rows + (z >> lb) * g.nb1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            C32 v = C32{0.f, 0.f};
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx % NP, y = idx / NP;
                if (srow[y >> lb]) v = X1[(in0 + y) * Kxp + k0 + p];
            }
            pre[e] = v;
        }
    };
    const int t0 = blockIdx.x * T;
    if (t0 < ntiles) load(t0);
    for (int i = 0; i < T; ++i) {
        const int t = t0 + i;
        if (t >= ntiles) break;
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) s[idx] = pre[e];
        }
        for (int idx = threadIdx.x; idx < NL; idx += kFftThreads) s[NL + idx] = C32{0.f, 0.f};
        lds_barrier();
        if (i + 1 < T && t + 1 < ntiles) load(t + 1);
        sfft<C32, P, NP, 1, NP, true, false>(s, tw);
        const size_t out0 = ((size_t)c * g.N2 + z) * P;
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, ky = idx / NP;
            X2[(out0 + ky) * Kxp + k0 + p] = s[idx];
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 3
// Tile = (kx tile, kyh): the workgroup convolves the columns ky = kyh and
// ky = P1 - kyh (which share the kernel-spectrum column) for every component.
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_zconv(BoxGeo g, C32 *__restrict__ X2, const float *__restrict__ ghat,
                                                        float scale, const C32 *__restrict__ twg, int ntiles) {
    constexpr int NP = np_zconv<P>();
    constexpr int Ph = P / 2;
    constexpr int N = P / 2;
    constexpr int NL = NP * N;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    float *gh = reinterpret_cast<float *>(s + NP * P);
    const int Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const int k0 = (t % nkt) * NP, kyh = t / nkt;
    const int H1 = g.P1 / 2 + 1;
    const int nky = (kyh == 0 || 2 * kyh == g.P1) ? 1 : 2;
    const int nitems = nky * g.ncomp;
    load_tw(tw, twg, P);
    for (int idx = threadIdx.x; idx < NP * (Ph + 1); idx += kFftThreads) {
        const int p = idx % NP, kz = idx / NP;
        gh[kz * NP + p] = scale * ghat[((size_t)kz * H1 + kyh) * Kxp + k0 + p];
    }
    C32 pre[E];
    auto col = [&](int item, int idx) -> size_t {
        const int ky = (item / g.ncomp) == 0 ? kyh : g.P1 - kyh;
        const int c = item % g.ncomp;
        const int p = idx % NP, z = idx / NP;
        return (((size_t)c * g.N2 + z) * g.P1 + ky) * Kxp + k0 + p;
    };
    auto load = [&](int item) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) pre[e] = X2[col(item, idx)];
        }
    };
    load(0);
    for (int item = 0; item < nitems; ++item) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) s[idx] = pre[e];
        }
        for (int idx = threadIdx.x; idx < NL; idx += kFftThreads) s[NL + idx] = C32{0.f, 0.f};
        lds_barrier();
        if (item + 1 < nitems) load(item + 1);
        sfft<C32, P, NP, 1, NP, true, false>(s, tw);
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, kz = idx / NP;
            const float w = gh[min(kz, P - kz) * NP + p];
            const C32 v = s[idx];
            s[idx] = C32{v.x * w, v.y * w};
        }
        lds_barrier();
        sfft<C32, P, NP, 1, NP, true, true>(s, tw);
        for (int idx = threadIdx.x; idx < NL; idx += kFftThreads) X2[col(item, idx)] = s[idx];
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 4
// Tile = (kx tile, z, component); planes without targets are skipped.
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_yinv(BoxGeo g, const C32 *__restrict__ X2, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg, int ntiles, int T) {
    constexpr int NP = np_cols<P>();
    constexpr int N = P / 2;
    constexpr int NT = NP * P;
    constexpr int E = (NT + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int lb = g.lb, Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    load_tw(tw, twg, P);
    C32 pre[E];
    auto plane_has_targets = [&](int z) {
        const int *trow = g.tgt_rows + (z >> lb) * g.nb1;
        bool any = false;
        for (int by = 0; by < g.nb1; ++by) any |= trow[by] != 0;
        return any;
    };
    auto load = [&](int t) {
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
        const size_t in0 = ((size_t)c * g.N2 + z) * P;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NT % kFftThreads == 0 || idx < NT) pre[e] = X2[(in0 + idx / NP) * Kxp + k0 + idx % NP];
        }
    };
    const int t0 = blockIdx.x * T;
    if (t0 < ntiles && plane_has_targets((t0 / nkt) % g.N2)) load(t0);
    for (int i = 0; i < T; ++i) {
        const int t = t0 + i;
        if (t >= ntiles) break;
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
        const bool active = plane_has_targets(z);
        if (active) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int idx = threadIdx.x + e * kFftThreads;
                if (NT % kFftThreads == 0 || idx < NT) s[idx] = pre[e];
            }
        }
        lds_barrier();
        if (i + 1 < T && t + 1 < ntiles && plane_has_targets(((t + 1) / nkt) % g.N2)) load(t + 1);
        if (!active) continue;
        sfft<C32, P, NP, 1, NP, true, true>(s, tw);
        const size_t out0 = ((size_t)c * g.N2 + z) * N;
        const int *trow = g.tgt_rows + (z >> lb) * g.nb1;
        for (int idx = threadIdx.x; idx < NP * N; idx += kFftThreads) {
            const int p = idx % NP, y = idx / NP;
            if (trow[y >> lb]) X1[(out0 + y) * Kxp + k0 + p] = s[idx];
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 5
// Tile = 2*NP consecutive box rows of one component (complex-to-real).
template <int P>
__global__ __launch_bounds__(kFftThreads) void kf_xinv(BoxGeo g, const C32 *__restrict__ X1, float *__restrict__ u,
                                                       int accumulate, const C32 *__restrict__ twg, int ntiles, int T) {
    constexpr int NP = np_rows<P>();
    constexpr int Ph = P / 2;
    constexpr int Kx = Ph + 1;
    constexpr int NL = NP * Kx;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    const int nrows = g.N1 * g.N2;
    const int ngroups = (nrows + 2 * NP - 1) / (2 * NP);
    const int lb = g.lb, bm = (1 << lb) - 1;
    const int Kxp = g.Kxp;
    load_tw(tw, twg, P);
    C32 pa[E], pb[E];
    auto load = [&](int t) {
        const int c = t / ngroups, row0 = (t % ngroups) * 2 * NP;
        const int y0 = row0 % g.N1, z0 = row0 / g.N1;
        auto has_tgt = [&](int q) {
            if (row0 + q >= nrows) return false;
            const RowPos rp = row_pos(y0, z0, q, g.N1);
            return g.tgt_rows[(rp.z >> lb) * g.nb1 + (rp.y >> lb)] != 0;
        };
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            C32 xa = C32{0.f, 0.f}, xb = C32{0.f, 0.f};
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / Kx, k = idx % Kx;
                const int ra = row0 + 2 * p, rb = ra + 1;
                // rows without targets were not written by pass 4: read as zero
                if (has_tgt(2 * p)) xa = X1[((size_t)c * nrows + ra) * Kxp + k];
                if (has_tgt(2 * p + 1)) xb = X1[((size_t)c * nrows + rb) * Kxp + k];
            }
            pa[e] = xa;
            pb[e] = xb;
        }
    };
    const int t0 = blockIdx.x * T;
    if (t0 < ntiles) load(t0);
    for (int i = 0; i < T; ++i) {
        const int t = t0 + i;
        if (t >= ntiles) break;
        const int c = t / ngroups, row0 = (t % ngroups) * 2 * NP;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / Kx, k = idx % Kx;
                C32 xa = pa[e], xb = pb[e];
                if (k == 0 || k == Ph) {
                    xa.y = 0.f;
                    xb.y = 0.f;
                }
                // Z = Xa + i Xb at k;  conj(Xa) + i conj(Xb) at P - k
                s[p * P + k] = C32{xa.x - xb.y, xa.y + xb.x};
                if (k > 0 && k < Ph) s[p * P + P - k] = C32{xa.x + xb.y, xb.x - xa.y};
            }
        }
        lds_barrier();
        if (i + 1 < T && t + 1 < ntiles) load(t + 1);
        sfft<C32, P, NP, P, 1, false, true>(s, tw);
        const size_t ubase = (size_t)c * g.ntgt << (3 * lb);
        const int y0 = row0 % g.N1, z0 = row0 / g.N1;
        for (int idx = threadIdx.x; idx < NP * Ph; idx += kFftThreads) {
            const int p = idx / Ph, x = idx % Ph;
            const C32 v = s[p * P + x];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = row0 + 2 * p + h;
                if (row < nrows) {
                    const RowPos rp = row_pos(y0, z0, 2 * p + h, g.N1);
                    const int y = rp.y, z = rp.z;
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
        lds_barrier();
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

// Tiles per workgroup of the x, y and y-inverse passes (defaults; the
// environment variables LGFIB_TPW_X / LGFIB_TPW_Y override them for tuning).
static int tiles_per_wg(bool xpass) {
    static int tx = -1, ty = -1;
    if (tx < 0) {
        const char *ex = getenv("LGFIB_TPW_X"), *ey = getenv("LGFIB_TPW_Y");
        tx = ex ? std::max(1, atoi(ex)) : 2;
        ty = ey ? std::max(1, atoi(ey)) : 4;
    }
    return xpass ? tx : ty;
}

int launch_fast_xfwd(const BoxGeo &g, const float *f, C32 *X1, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_rows(g.P0);
    const int nrows = g.N1 * g.N2;
    const int ntiles = (nrows + 2 * NP - 1) / (2 * NP) * g.ncomp, T = tiles_per_wg(true);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0);
    switch (g.P0) {
#define X(n) case n: hipLaunchKernelGGL(kf_xfwd<n>, grid, dim3(kFftThreads), sm, st, g, f, X1, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_yfwd(const BoxGeo &g, const C32 *X1, C32 *X2, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_cols(g.P1);
    const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = tiles_per_wg(false);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1);
    switch (g.P1) {
#define X(n) case n: hipLaunchKernelGGL(kf_yfwd<n>, grid, dim3(kFftThreads), sm, st, g, X1, X2, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised y pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_zconv(const BoxGeo &g, C32 *X2, const float *ghat, float scale, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_zconv(g.P2);
    const int ntiles = g.Kxp / NP * (g.P1 / 2 + 1);
    dim3 grid(ntiles);
    const size_t sm = sizeof(C32) * (size_t)(g.P2 / 2 + NP * g.P2) + sizeof(float) * (size_t)NP * (g.P2 / 2 + 1);
    switch (g.P2) {
#define X(n) case n: hipLaunchKernelGGL(kf_zconv<n>, grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw, ntiles); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised z pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_yinv(const BoxGeo &g, const C32 *X2, C32 *X1, const C32 *tw, hipStream_t st) {
    const int NP = fast_np_cols(g.P1);
    const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = tiles_per_wg(false);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1);
    switch (g.P1) {
#define X(n) case n: hipLaunchKernelGGL(kf_yinv<n>, grid, dim3(kFftThreads), sm, st, g, X2, X1, tw, ntiles, T); break;
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
    const int ntiles = (nrows + 2 * NP - 1) / (2 * NP) * g.ncomp, T = tiles_per_wg(true);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0);
    switch (g.P0) {
#define X(n) case n: hipLaunchKernelGGL(kf_xinv<n>, grid, dim3(kFftThreads), sm, st, g, X1, u, accumulate, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

}  // namespace lgfib
