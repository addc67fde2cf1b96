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
// y passes: pencils plus the inverse pass's last-stage twiddle table;
// es = bytes per real
constexpr int np_fit_y(int P, int es = 4) {
    int np = 16;
    while (np > 1 && (P / 2 + np * P + P) * 2 * es > kLdsBudget) np /= 2;
    return np;
}
template <int P, int es = 4> constexpr int np_cols() { return np_fit_y(P, es); }
// z pass: pencils, the kernel-spectrum column (P/2 + 1 reals per pencil) and
// the last stage's twiddle table (fewer than P entries); es = bytes per real
constexpr int np_fit_z(int P, int es = 4) {
    int np = 16;
    while (np > 1 && (P / 2 + np * P + P) * 2 * es + np * (P / 2 + 1) * es > kLdsBudget) np /= 2;
    return np;
}
template <int P, int es = 4> constexpr int np_zconv() { return np_fit_z(P, es); }

// the real type of a complex pair
template <typename C> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };

// Spectrum pencils are read once and written once per pass, and a pass's
// whole spectrum does not fit in cache.  Each bit of LGF_FFT_NT marks one
// pass's global loads or stores as streaming (non-temporal).  The default
// (streaming loads and stores in the forward y pass, streaming loads in the
// inverse y pass, streaming source loads in the forward x pass and output
// stores in the inverse x pass) measured fastest on the plate box (0.80 ->
// 0.76 ms per three-component apply); streaming loads in the z pass made it
// slower (0.35 -> 0.37-0.41 ms), as did streaming stores of the z pass in
// the default's company.
enum : unsigned {
    kNtYfwdLd = 1u << 0, kNtYfwdSt = 1u << 1, kNtZLd = 1u << 2, kNtZSt = 1u << 3,
    kNtYinvLd = 1u << 4, kNtYinvSt = 1u << 5, kNtXfwdSt = 1u << 6, kNtXinvLd = 1u << 7,
    kNtXfwdLd = 1u << 8, kNtXinvSt = 1u << 9,
};
#ifndef LGF_FFT_NT
#define LGF_FFT_NT (kNtYfwdLd | kNtYfwdSt | kNtYinvLd | kNtXfwdLd | kNtXinvSt)
#endif
constexpr bool nt_on(unsigned bit) { return ((unsigned)(LGF_FFT_NT) & bit) != 0; }
template <bool NT, typename V> __device__ __forceinline__ V ld_vec(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename V> __device__ __forceinline__ void st_vec(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <typename R> using Vec2 = R __attribute__((ext_vector_type(2)));
using Vec4f = float __attribute__((ext_vector_type(4)));
template <bool NT, typename C> __device__ __forceinline__ C ld_pencil(const C *p) {
    using R = typename RealOf<C>::T;
    const Vec2<R> v = ld_vec<NT>(reinterpret_cast<const Vec2<R> *>(p));
    return C{v.x, v.y};
}
template <bool NT, typename C> __device__ __forceinline__ void st_pencil(C *p, C v) {
    using R = typename RealOf<C>::T;
    Vec2<R> w;
    w.x = v.x;
    w.y = v.y;
    st_vec<NT>(reinterpret_cast<Vec2<R> *>(p), w);
}
template <bool NT> __device__ __forceinline__ float4 ld_f4(const float *p) {
    const Vec4f v = ld_vec<NT>(reinterpret_cast<const Vec4f *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
template <bool NT> __device__ __forceinline__ void st_f4(float *p, float4 v) {
    Vec4f w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    st_vec<NT>(reinterpret_cast<Vec4f *>(p), w);
}

template <typename C>
__device__ __forceinline__ void load_tw(C *dst, const C *__restrict__ src, int P) {
    for (int i = threadIdx.x; i < P / 2; i += kFftThreads) dst[i] = src[i];
}

// All passes walk T consecutive tiles per workgroup.  The next tile's global
// data is loaded into registers right after the current tile has been staged
// in LDS, so those loads are in flight while the current tile is transformed
// (the FFT's barriers order LDS only and do not wait for them).

// Uniform bitmask of the block rows (by) of plane bz that hold blocks; the
// loop runs on scalar loads because its addresses are wave-uniform.
struct RowMask {
    uint64_t lo, hi;
    __device__ __forceinline__ bool test(int by) const {
        return by < 64 ? ((lo >> by) & 1ull) : ((hi >> (by - 64)) & 1ull);
    }
};
__device__ __forceinline__ RowMask plane_mask(const int *__restrict__ rows, int nb1) {
    RowMask m{0ull, 0ull};
    for (int b = 0; b < nb1; ++b)
        if (rows[b]) {
            if (b < 64) m.lo |= 1ull << b;
            else m.hi |= 1ull << (b - 64);
        }
    return m;
}
// block rows of z block plane zb holding targets (tgt) or sources
__device__ __forceinline__ RowMask plane_rows(const BoxGeo &g, bool tgt, int zb) {
    if (g.masks_ok) return tgt ? RowMask{g.tgt_mask[zb][0], g.tgt_mask[zb][1]} : RowMask{g.src_mask[zb][0], g.src_mask[zb][1]};
    return plane_mask((tgt ? g.tgt_rows : g.src_rows) + zb * g.nb1, g.nb1);
}

// padded length of a row of the x spectrum (Kx = P/2 + 1 rounded up to 16),
// as the box plan lays it out
constexpr int fast_kxp(int P) { return (P / 2 + 1 + 15) / 16 * 16; }

// ------------------------------------------------------------------- pass 1
// A workgroup owns a chunk of the B*B box rows of one block row (by, bz) of one
// component; the block row's slot table is staged in LDS once, rows come in
// tiles of 2*NP (two real rows per complex pencil), and data moves as float4
// (four consecutive x of one block row segment).
template <int P, int NPMAX>
__device__ __forceinline__ void xfwd_body(const BoxGeo &g, const float *__restrict__ f, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg, int nchunks, int T, int bid) {
    constexpr int NP = np_rows<P>() < NPMAX ? np_rows<P>() : NPMAX;
    constexpr int N = P / 2;
    constexpr int N4 = N / 4;
    constexpr int NL = NP * N4;   // float4 loads per row of pencils
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    int *slot = reinterpret_cast<int *>(s + NP * P);   // [nb0] element offsets or -1
    const int lb = g.lb, B = 1 << lb, bm = B - 1;
    const int chunk = bid % nchunks;
    const int br = (bid / nchunks) % (g.nb1 * g.nb2);
    const int c = bid / (nchunks * g.nb1 * g.nb2);
    if (!g.src_rows[br]) return;
    const int by = br % g.nb1, bz = br / g.nb1;
    load_tw(tw, twg, P);
    for (int bx = threadIdx.x; bx < g.nb0; bx += kFftThreads) {
        const int sl = g.src_map[br * g.nb0 + bx];
        slot[bx] = sl >= 0 ? (sl << (3 * lb)) : -1;
    }
    lds_barrier();
    const float *fc = f + ((size_t)c * g.nsrc << (3 * lb));
    const int nrows = g.N1 * g.N2;
    float4 pa[E], pb[E];
    auto load = [&](int q0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / N4, x = 4 * (idx % N4);
                const int q = q0 + 2 * p;                 // even row of the pair
                const int off = slot[x >> lb];
                if (off >= 0) {
                    const float *src = fc + off + (((q >> lb) << (2 * lb)) | ((q & bm) << lb) | (x & bm));
                    a = ld_f4<nt_on(kNtXfwdLd)>(src);
                    b = ld_f4<nt_on(kNtXfwdLd)>(src + B);   // row q + 1 (same z)
                }
            }
            pa[e] = a;
            pb[e] = b;
        }
    };
    const int q00 = chunk * T * 2 * NP;
    load(q00);
    for (int i = 0; i < T; ++i) {
        const int q0 = q00 + i * 2 * NP;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) {
                C32 *d = s + (idx / N4) * P + 4 * (idx % N4);
                d[0] = C32{pa[e].x, pb[e].x};
                d[1] = C32{pa[e].y, pb[e].y};
                d[2] = C32{pa[e].z, pb[e].z};
                d[3] = C32{pa[e].w, pb[e].w};
            }
        }
        lds_barrier();
        if (i + 1 < T) load(q0 + 2 * NP);
        sfft<C32, P, NP, P, 1, false, false, N, 0>(s, tw);   // x >= N is zero padding
        // two consecutive frequencies per thread, one 16-byte store per row
        // (Kxp is even and rows start 16-byte aligned); the row length is a
        // compile-time constant of P (checked on the host), so the index
        // split below needs no integer division at run time
        constexpr int Kxp = fast_kxp(P), Kx = P / 2 + 1, Kh = Kxp / 2;
        for (int idx = threadIdx.x; idx < NP * Kh; idx += kFftThreads) {
            const int p = idx / Kh, k = 2 * (idx - p * Kh);
            float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
            if (k < Kx) {
                const C32 zk = s[p * P + k];
                const C32 zm = s[p * P + (k == 0 ? 0 : P - k)];
                va.x = 0.5f * (zk.x + zm.x), va.y = 0.5f * (zk.y - zm.y);
                vb.x = 0.5f * (zk.y + zm.y), vb.y = 0.5f * (zm.x - zk.x);
            }
            if (k + 1 < Kx) {
                const C32 zk = s[p * P + k + 1];
                const C32 zm = s[p * P + P - k - 1];
                va.z = 0.5f * (zk.x + zm.x), va.w = 0.5f * (zk.y - zm.y);
                vb.z = 0.5f * (zk.y + zm.y), vb.w = 0.5f * (zm.x - zk.x);
            }
            const int q = q0 + 2 * p;
            const int row = ((bz << lb) + (q >> lb)) * g.N1 + (by << lb) + (q & bm);
            st_f4<nt_on(kNtXfwdSt)>(reinterpret_cast<float *>(X1 + ((size_t)c * nrows + row) * Kxp + k), va);
            st_f4<nt_on(kNtXfwdSt)>(reinterpret_cast<float *>(X1 + ((size_t)c * nrows + row + 1) * Kxp + k), vb);
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 2
// Tile = (kx tile of NP columns, z, component); kx tile fastest.
// C is float2 (the FP32 path) or double2 (FP64).
template <typename C, int P, int NPMAX>
__device__ __forceinline__ void yfwd_body(const BoxGeo &g, const C *__restrict__ X1, C *__restrict__ X2,
                                                       const C *__restrict__ twg, int ntiles, int T, int bid) {
    constexpr int YNP = np_cols<P, (int)sizeof(typename RealOf<C>::T)>();
    constexpr int NP = YNP < NPMAX ? YNP : NPMAX;
    constexpr int N = P / 2;
    constexpr int NL = NP * N;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tw = reinterpret_cast<C *>(smem_raw);
    C *s = tw + P / 2;
    const int lb = g.lb, Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    load_tw(tw, twg, P);
    C pre[E];
    auto load = [&](int t) {
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
        const size_t in0 = ((size_t)c * g.N2 + z) * N;
        const RowMask m = plane_rows(g, false, z >> lb);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            C v = C{};
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx % NP, y = idx / NP;
                if (m.test(y >> lb)) v = ld_pencil<nt_on(kNtYfwdLd)>(&X1[(in0 + y) * Kxp + k0 + p]);
            }
            pre[e] = v;
        }
    };
    const int t0 = bid * T;
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
        lds_barrier();
        if (i + 1 < T && t + 1 < ntiles) load(t + 1);
        sfft<C, P, NP, 1, NP, true, false, N, 0>(s, tw);   // y >= N is zero padding
        const size_t out0 = ((size_t)c * g.N2 + z) * P;
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, ky = idx / NP;
            st_pencil<nt_on(kNtYfwdSt)>(&X2[(out0 + ky) * Kxp + k0 + p], s[idx]);
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 3
// multiply by the real kernel spectrum column (symmetric in kz), applied as
// the last stage of the forward z FFT stores its outputs
template <typename C, int P, int NP> struct ZMul {
    const typename RealOf<C>::T *gh;   // [P/2 + 1][NP] in LDS
    __device__ __forceinline__ C operator()(int p, int kz, C v) const {
        const auto w = gh[min(kz, P - kz) * NP + p];
        return C{v.x * w, v.y * w};
    }
};

// Tile = (kx tile, kyh): the workgroup convolves the columns ky = kyh and
// ky = P1 - kyh (which share the kernel-spectrum column) for every component.
// Only z < P/2 holds sources and only z < P/2 is kept, so the forward FFT
// skips the zero upper half and the inverse computes the lower half only.
// C is float2 (the FP32 path) or double2 (FP64).
template <typename C, int P, int NPMAX>
__device__ __forceinline__ void zconv_body(const BoxGeo &g, C *__restrict__ X2,
                                           const typename RealOf<C>::T *__restrict__ ghat, typename RealOf<C>::T scale,
                                           const C *__restrict__ twg, int ntiles, int bid) {
    using R = typename RealOf<C>::T;
    constexpr int ZNP = np_zconv<P, (int)sizeof(R)>();
    constexpr int NP = ZNP < NPMAX ? ZNP : NPMAX;
    constexpr int Ph = P / 2;
    constexpr int N = P / 2;
    constexpr int NL = NP * N;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tw = reinterpret_cast<C *>(smem_raw);
    C *s = tw + P / 2;
    R *gh = reinterpret_cast<R *>(s + NP * P);
    C *twt = reinterpret_cast<C *>(gh + NP * (Ph + 1));   // 8-byte aligned: NP (Ph + 1) is even
    const int Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    if (bid >= ntiles) return;
    const int t = bid;
    const int k0 = (t % nkt) * NP, kyh = t / nkt;
    const int H1 = g.P1 / 2 + 1;
    const int nky = (kyh == 0 || 2 * kyh == g.P1) ? 1 : 2;
    const int nitems = nky * g.ncomp;
    // element e of a thread's column slice sits zstep * e past its first one
    // (consecutive threads walk pencils, then z)
    const size_t zrow = (size_t)g.P1 * Kxp;
    const size_t zstep = (size_t)(kFftThreads / NP) * zrow;
    const size_t lane = (size_t)(threadIdx.x / NP) * zrow + k0 + threadIdx.x % NP;
    static_assert(kFftThreads % NP == 0, "pencils must divide the workgroup");
    static_assert(NP * (Ph + 1) % 2 == 0, "twiddle table alignment");
    C pre[E];
    auto base = [&](int item) -> C * {
        const int ky = (item / g.ncomp) == 0 ? kyh : g.P1 - kyh;
        const int c = item % g.ncomp;
        return X2 + (size_t)c * g.N2 * zrow + (size_t)ky * Kxp + lane;
    };
    auto load = [&](int item) {
        const C *b = base(item);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) pre[e] = ld_pencil<nt_on(kNtZLd)>(&b[e * zstep]);
        }
    };
    load(0);   // first, so that its latency overlaps the table loads below
    load_tw(tw, twg, P);
    for (int idx = threadIdx.x; idx < NP * (Ph + 1); idx += kFftThreads) {
        const int p = idx % NP, kz = idx / NP;
        gh[kz * NP + p] = scale * ghat[((size_t)kz * H1 + kyh) * Kxp + k0 + p];
    }
    // all twiddle powers of the last stage (forward and inverse share it)
    last_stage_twiddles<C, P, RadixOf<P>::last>(twt, twg);
    for (int item = 0; item < nitems; ++item) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) s[idx] = pre[e];
        }
        lds_barrier();
        if (item + 1 < nitems) load(item + 1);
        sfft_tt<C, P, NP, 1, NP, true, false, Ph, 0>(s, tw, twt, ZMul<C, P, NP>{gh});
        sfft_tt<C, P, NP, 1, NP, true, true, 0, Ph>(s, tw, twt);
        C *b = base(item);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) st_pencil<nt_on(kNtZSt)>(&b[e * zstep], s[idx]);
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 4
// Tile = (kx tile, z, component); planes without targets are skipped.
// C is float2 (the FP32 path) or double2 (FP64).
template <typename C, int P, int NPMAX>
__device__ __forceinline__ void yinv_body(const BoxGeo &g, const C *__restrict__ X2, C *__restrict__ X1,
                                                       const C *__restrict__ twg, int ntiles, int T, int bid) {
    constexpr int YNP = np_cols<P, (int)sizeof(typename RealOf<C>::T)>();
    constexpr int NP = YNP < NPMAX ? YNP : NPMAX;
    constexpr int N = P / 2;
    constexpr int NT = NP * P;
    constexpr int E = (NT + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tw = reinterpret_cast<C *>(smem_raw);
    C *s = tw + P / 2;
    const int lb = g.lb, Kxp = g.Kxp;
    const int nkt = Kxp / NP;
    load_tw(tw, twg, P);
    // the last stage reads all its twiddle powers from a table (fewer
    // VALU products and no strided twiddle reads)
    C *twt = s + NP * P;
    lds_barrier();
    last_stage_twiddles<C, P, RadixOf<P>::last>(twt, tw);
    C pre[E];
    auto plane_has_targets = [&](int z) {
        const RowMask m = plane_rows(g, true, z >> lb);
        return (m.lo | m.hi) != 0ull;
    };
    auto load = [&](int t) {
        const int k0 = (t % nkt) * NP, z = (t / nkt) % g.N2, c = t / (nkt * g.N2);
        const size_t in0 = ((size_t)c * g.N2 + z) * P;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NT % kFftThreads == 0 || idx < NT) pre[e] = ld_pencil<nt_on(kNtYinvLd)>(&X2[(in0 + idx / NP) * Kxp + k0 + idx % NP]);
        }
    };
    const int t0 = bid * T;
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
        sfft_tt<C, P, NP, 1, NP, true, true, 0, N>(s, tw, twt);   // only y < N is kept
        const size_t out0 = ((size_t)c * g.N2 + z) * N;
        const RowMask m = plane_rows(g, true, z >> lb);
        for (int idx = threadIdx.x; idx < NP * N; idx += kFftThreads) {
            const int p = idx % NP, y = idx / NP;
            if (m.test(y >> lb)) st_pencil<nt_on(kNtYinvSt)>(&X1[(out0 + y) * Kxp + k0 + p], s[idx]);
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------------- pass 5
// Complex-to-real rows; same block-row decomposition as pass 1, cropped to the
// target blocks of the block row and stored as float4.
template <int P, int NPMAX>
__device__ __forceinline__ void xinv_body(const BoxGeo &g, const C32 *__restrict__ X1, float *__restrict__ u,
                                                       int accumulate, const C32 *__restrict__ twg, int nchunks, int T, int bid) {
    constexpr int NP = np_rows<P>() < NPMAX ? np_rows<P>() : NPMAX;
    constexpr int Ph = P / 2;
    constexpr int Kx = Ph + 1;
    constexpr int KH = (Kx + 1) / 2;   // frequency pairs; a row holds Kxp >= Kx + 1 entries
    constexpr int NL = NP * KH;
    constexpr int E = (NL + kFftThreads - 1) / kFftThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C32 *tw = reinterpret_cast<C32 *>(smem_raw);
    C32 *s = tw + P / 2;
    int *slot = reinterpret_cast<int *>(s + NP * P);
    const int lb = g.lb, B = 1 << lb, bm = B - 1;
    const int chunk = bid % nchunks;
    const int br = (bid / nchunks) % (g.nb1 * g.nb2);
    const int c = bid / (nchunks * g.nb1 * g.nb2);
    if (!g.tgt_rows[br]) return;
    const int by = br % g.nb1, bz = br / g.nb1;
    load_tw(tw, twg, P);
    for (int bx = threadIdx.x; bx < g.nb0; bx += kFftThreads) {
        const int sl = g.tgt_map[br * g.nb0 + bx];
        slot[bx] = sl >= 0 ? (sl << (3 * lb)) : -1;
    }
    const int nrows = g.N1 * g.N2;
    const int Kxp = g.Kxp;
    const size_t xbase = (size_t)c * nrows;
    auto rowidx = [&](int q) { return ((bz << lb) + (q >> lb)) * g.N1 + (by << lb) + (q & bm); };
    // two consecutive frequencies per 16-byte load (rows start 16-byte aligned)
    float4 pa[E], pb[E];
    auto load = [&](int q0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            float4 xa = make_float4(0.f, 0.f, 0.f, 0.f), xb = xa;
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / KH, k = 2 * (idx % KH);
                const int ra = rowidx(q0 + 2 * p);
                xa = ld_f4<nt_on(kNtXinvLd)>(reinterpret_cast<const float *>(X1 + (xbase + ra) * Kxp + k));
                xb = ld_f4<nt_on(kNtXinvLd)>(reinterpret_cast<const float *>(X1 + (xbase + ra + 1) * Kxp + k));
            }
            pa[e] = xa;
            pb[e] = xb;
        }
    };
    float *uc = u + ((size_t)c * g.ntgt << (3 * lb));
    const int q00 = chunk * T * 2 * NP;
    load(q00);
    for (int i = 0; i < T; ++i) {
        const int q0 = q00 + i * 2 * NP;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = threadIdx.x + e * kFftThreads;
            if (NL % kFftThreads == 0 || idx < NL) {
                const int p = idx / KH, k0 = 2 * (idx % KH);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = k0 + h;
                    if (h == 1 && k >= Kx) break;
                    C32 xa = h ? C32{pa[e].z, pa[e].w} : C32{pa[e].x, pa[e].y};
                    C32 xb = h ? C32{pb[e].z, pb[e].w} : C32{pb[e].x, pb[e].y};
                    if (k == 0 || k == Ph) {
                        xa.y = 0.f;
                        xb.y = 0.f;
                    }
                    // Z = Xa + i Xb at k;  conj(Xa) + i conj(Xb) at P - k
                    s[p * P + k] = C32{xa.x - xb.y, xa.y + xb.x};
                    if (k > 0 && k < Ph) s[p * P + P - k] = C32{xa.x + xb.y, xb.x - xa.y};
                }
            }
        }
        lds_barrier();
        if (i + 1 < T) load(q0 + 2 * NP);
        sfft<C32, P, NP, P, 1, false, true, 0, Ph>(s, tw);   // only x < P/2 is kept
        constexpr int N4 = Ph / 4;
        for (int idx = threadIdx.x; idx < NP * N4; idx += kFftThreads) {
            const int p = idx / N4, x = 4 * (idx % N4);
            const int off = slot[x >> lb];
            if (off < 0) continue;
            const C32 *v = s + p * P + x;
            const int q = q0 + 2 * p;
            float *dst = uc + off + (((q >> lb) << (2 * lb)) | ((q & bm) << lb) | (x & bm));
            float4 a = make_float4(v[0].x, v[1].x, v[2].x, v[3].x);
            float4 b = make_float4(v[0].y, v[1].y, v[2].y, v[3].y);
            if (accumulate) {
                const float4 oa = *reinterpret_cast<const float4 *>(dst);
                const float4 ob = *reinterpret_cast<const float4 *>(dst + B);
                a = make_float4(a.x + oa.x, a.y + oa.y, a.z + oa.z, a.w + oa.w);
                b = make_float4(b.x + ob.x, b.y + ob.y, b.z + ob.z, b.w + ob.w);
            }
            st_f4<nt_on(kNtXinvSt)>(dst, a);
            st_f4<nt_on(kNtXinvSt)>(dst + B, b);
        }
        lds_barrier();
    }
}


// Kernels of the single apply: one workgroup per tile (group).
template <int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kf_xfwd(BoxGeo g, const float *__restrict__ f, C32 *__restrict__ X1,
                                                       const C32 *__restrict__ twg, int nchunks, int T) {
    xfwd_body<P, NPMAX>(g, f, X1, twg, nchunks, T, (int)blockIdx.x);
}
template <typename C, int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kf_yfwd(BoxGeo g, const C *__restrict__ X1, C *__restrict__ X2,
                                                       const C *__restrict__ twg, int ntiles, int T) {
    yfwd_body<C, P, NPMAX>(g, X1, X2, twg, ntiles, T, (int)blockIdx.x);
}
// neighbouring kx tiles of the z pass share cache lines when NP * 8 bytes is
// below a line: the tiles are remapped so that each XCD takes a contiguous run
template <typename C, int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kf_zconv(BoxGeo g, C *__restrict__ X2,
                                                        const typename RealOf<C>::T *__restrict__ ghat,
                                                        typename RealOf<C>::T scale, const C *__restrict__ twg,
                                                        int ntiles) {
    if ((int)blockIdx.x >= ntiles) return;
    zconv_body<C, P, NPMAX>(g, X2, ghat, scale, twg, ntiles, xcd_remap(blockIdx.x, ntiles));
}
template <typename C, int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kf_yinv(BoxGeo g, const C *__restrict__ X2, C *__restrict__ X1,
                                                       const C *__restrict__ twg, int ntiles, int T) {
    yinv_body<C, P, NPMAX>(g, X2, X1, twg, ntiles, T, (int)blockIdx.x);
}
template <int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kf_xinv(BoxGeo g, const C32 *__restrict__ X1, float *__restrict__ u,
                                                       int accumulate, const C32 *__restrict__ twg, int nchunks, int T) {
    xinv_body<P, NPMAX>(g, X1, u, accumulate, twg, nchunks, T, (int)blockIdx.x);
}


// ------------------------------------------------------------ batched passes
// One pass of many independent convolutions of one FFT length in one
// persistent launch: workgroups pull work items (an instance's tile groups,
// numbered consecutively over the instances) from a device counter until all
// are taken, look up the item's instance, and run the pass body on that
// instance's geometry and buffers.
template <int PASS, int P, int NPMAX>
__device__ __forceinline__ void kb_item(const FastJob *__restrict__ jobs, const int *__restrict__ start,
                                        const int *__restrict__ owner, int item) {
    const int k = __builtin_amdgcn_readfirstlane(owner[item]);
    const FastJob &J = jobs[k];
    const int bid = item - start[k];
    if constexpr (PASS == kPassXF)
        xfwd_body<P, NPMAX>(J.g, (const float *)J.in, (C32 *)J.out, J.tw, J.n, J.T, bid);
    else if constexpr (PASS == kPassYF)
        yfwd_body<C32, P, NPMAX>(J.g, (const C32 *)J.in, (C32 *)J.out, J.tw, J.n, J.T, bid);
    else if constexpr (PASS == kPassZ)
        zconv_body<C32, P, NPMAX>(J.g, (C32 *)J.out, J.ghat, J.scale, J.tw, J.n, bid);
    else if constexpr (PASS == kPassYI)
        yinv_body<C32, P, NPMAX>(J.g, (const C32 *)J.in, (C32 *)J.out, J.tw, J.n, J.T, bid);
    else
        xinv_body<P, NPMAX>(J.g, (const C32 *)J.in, (float *)J.out, J.acc, J.tw, J.n, J.T, bid);
}

// persistent form: workgroups pull items from *queue until all are taken; the
// next item is claimed while the current one runs
template <int PASS, int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kb_pass(const FastJob *__restrict__ jobs, const int *__restrict__ start,
                                                      const int *__restrict__ owner, int total, int *__restrict__ queue) {
    __shared__ int next[2];
    if (threadIdx.x == 0) next[0] = atomicAdd(queue, 1);
    __syncthreads();
    for (int r = 0;; r ^= 1) {
        const int item = __builtin_amdgcn_readfirstlane(next[r]);
        if (item >= total) return;
        if (threadIdx.x == 0) next[r ^ 1] = atomicAdd(queue, 1);
        kb_item<PASS, P, NPMAX>(jobs, start, owner, item);
        __syncthreads();   // the next item rewrites LDS; next[r ^ 1] is visible
    }
}

// one workgroup per item
template <int PASS, int P, int NPMAX>
__global__ __launch_bounds__(kFftThreads) void kb_pass_grid(const FastJob *__restrict__ jobs,
                                                           const int *__restrict__ start,
                                                           const int *__restrict__ owner, int total) {
    if ((int)blockIdx.x >= total) return;
    // each XCD takes a contiguous run of items: an instance's neighbouring
    // tiles share cache lines in that XCD's L2
    kb_item<PASS, P, NPMAX>(jobs, start, owner, xcd_remap(blockIdx.x, total));
}

// ------------------------------------------------------------------ dispatch

#define LGF_FAST_SIZES(X) \
    X(16) X(32) X(48) X(64) X(80) X(96) X(128) X(144) X(160) X(192) X(240) X(256) X(288) X(320) X(384) X(480) \
    X(512) X(576) X(640) X(768) X(960) X(1024)

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
int fast_np_cols(int P) { return np_fit_y(P); }
int fast_np_zconv(int P) { return np_fit_z(P); }
int fast_np_zconv_f64(int P) { return np_fit_z(P, 8); }

// Tiles per workgroup of the x, y and y-inverse passes (defaults; the
// environment variables LGFIB_TPW_X / LGFIB_TPW_Y override them for tuning).
ConvOverrides &conv_overrides() {
    static thread_local ConvOverrides o;
    return o;
}

// tiles per workgroup: x passes 2; y passes 2, except the FP32 forward y
// pass with 4 (0.143 -> 0.138 ms on the plate box; 4 in the inverse y pass
// measured slower, 0.143 -> 0.149 ms)
static int tiles_per_wg(bool xpass, bool xinv = false, bool yfwd = false) {
    const ConvOverrides &o = conv_overrides();
    if (xpass && o.tpw_x > 0) return o.tpw_x;
    if (!xpass && o.tpw_y > 0) return o.tpw_y;
    static int tx = -1, txi = -1, ty = -1, tyf = -1;
    if (tx < 0) {
        const char *ex = getenv("LGFIB_TPW_X"), *exi = getenv("LGFIB_TPW_XI"), *ey = getenv("LGFIB_TPW_Y"),
                   *eyf = getenv("LGFIB_TPW_YF");
        tx = ex ? std::max(1, atoi(ex)) : 2;
        txi = exi ? std::max(1, atoi(exi)) : 2;
        ty = ey ? std::max(1, atoi(ey)) : 2;
        tyf = eyf ? std::max(1, atoi(eyf)) : (ey ? ty : 4);
    }
    return xpass ? (xinv ? txi : tx) : (yfwd ? tyf : ty);
}

// Small boxes lower the grouping until the launch has enough workgroups to
// occupy the chip (kMinGroups).
constexpr long kMinGroups = 2048;

// y passes: ntiles tiles grouped T per workgroup
static int y_group(int ntiles, bool fwd32 = false) {
    int t = tiles_per_wg(false, false, fwd32);
    if (conv_overrides().tpw_y > 0) return std::max(1, std::min(t, ntiles));
    while (t > 1 && (ntiles + t - 1) / t < kMinGroups) --t;
    return t;
}

// x passes: a block row of B*B box rows splits into B*B/(2 NP) tiles, grouped
// T per workgroup (T dividing that count).
static int x_tiles(const BoxGeo &g, int NP, int *T, bool inv) {
    const int tpb = (g.B * g.B) / (2 * NP);
    const long rows = (long)g.nb1 * g.nb2 * g.ncomp;
    int t = std::min(tiles_per_wg(true, inv), tpb);
    const bool fixed = conv_overrides().tpw_x > 0;
    while (t > 1 && (tpb % t || (!fixed && rows * (tpb / t) < kMinGroups))) --t;
    *T = t;
    return tpb / t;   // chunks per block row
}

static int x_np_cap(bool fwd);
static int x_np(int P, bool fwd) { return std::min(fast_np_rows(P), x_np_cap(fwd)); }

bool fast_x_ok(const BoxGeo &g) {
    // the x passes move frequencies in pairs: a spectrum row needs room for
    // Kx + 1; the forward pass takes the row length as fast_kxp(P0)
    return fast_size(g.P0) && g.Kxp >= g.Kx + 1 && g.Kxp % 2 == 0 && g.Kxp == fast_kxp(g.P0) && (g.B * g.B) % (2 * x_np(g.P0, true)) == 0 &&
           (g.B * g.B) % (2 * x_np(g.P0, false)) == 0 && g.nb1 <= 128;
}

template <int P, bool FWD, typename... Args>
static void launch_x_np(int cap, dim3 grid, size_t sm, hipStream_t st, Args... args) {
    if constexpr (FWD) {
        if (cap == 4) hipLaunchKernelGGL((kf_xfwd<P, 4>), grid, dim3(kFftThreads), sm, st, args...);
        else if (cap == 8) hipLaunchKernelGGL((kf_xfwd<P, 8>), grid, dim3(kFftThreads), sm, st, args...);
        else hipLaunchKernelGGL((kf_xfwd<P, 16>), grid, dim3(kFftThreads), sm, st, args...);
    } else {
        if (cap == 4) hipLaunchKernelGGL((kf_xinv<P, 4>), grid, dim3(kFftThreads), sm, st, args...);
        else if (cap == 8) hipLaunchKernelGGL((kf_xinv<P, 8>), grid, dim3(kFftThreads), sm, st, args...);
        else hipLaunchKernelGGL((kf_xinv<P, 16>), grid, dim3(kFftThreads), sm, st, args...);
    }
}

int launch_fast_xfwd(const BoxGeo &g, const float *f, C32 *X1, const C32 *tw, hipStream_t st) {
    const int cap = x_np_cap(true);
    const int NP = x_np(g.P0, true);
    int T = 1;
    const int nchunks = x_tiles(g, NP, &T, false);
    dim3 grid(nchunks * g.nb1 * g.nb2 * g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0) + sizeof(int) * (size_t)g.nb0;
    switch (g.P0) {
#define X(n) case n: launch_x_np<n, true>(cap, grid, sm, st, g, f, X1, tw, nchunks, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

template <int P, bool FWD>
static void launch_y_np(int cap, dim3 grid, size_t sm, hipStream_t st, const BoxGeo &g, const C32 *in, C32 *out,
                        const C32 *tw, int ntiles, int T) {
#define LGF_YL(NPM)                                                                                               \
    if (FWD) hipLaunchKernelGGL((kf_yfwd<C32, P, NPM>), grid, dim3(kFftThreads), sm, st, g, in, out, tw, ntiles, T); \
    else hipLaunchKernelGGL((kf_yinv<C32, P, NPM>), grid, dim3(kFftThreads), sm, st, g, in, out, tw, ntiles, T);
    if (cap == 4) {
        LGF_YL(4)
    } else if (cap == 8) {
        LGF_YL(8)
    } else {
        LGF_YL(16)
    }
#undef LGF_YL
}

static int y_np_cap();

int launch_fast_yfwd(const BoxGeo &g, const C32 *X1, C32 *X2, const C32 *tw, hipStream_t st) {
    const int cap = y_np_cap();
    const int NP = std::min(fast_np_cols(g.P1), cap);
    const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = y_group(ntiles, true);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1);
    switch (g.P1) {
#define X(n) case n: launch_y_np<n, true>(cap, grid, sm, st, g, X1, X2, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised y pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// pencils per workgroup of the z and y passes: the LDS fit, capped at 8 for
// the z pass (its smaller LDS footprint lets more workgroups share a CU:
// 0.62 -> 0.50 ms on the plate set) and 16 for the y passes (measured
// best); the environment variables LGFIB_ZNP / LGFIB_YNP = 4, 8 or 16
// override them
static int np_cap(const char *var, int dflt) {
    const char *e = getenv(var);
    const int cap = e ? atoi(e) : dflt;
    return (cap == 4 || cap == 8 || cap == 16) ? cap : dflt;
}
static int z_np_cap() {
    static int cap = np_cap("LGFIB_ZNP", 8);
    return cap;
}
static int y_np_cap() {
    static int cap = np_cap("LGFIB_YNP", 16);
    return cap;
}
// x passes: both run best with four pencils per workgroup (LDS for more
// workgroups in flight: 0.079 -> 0.071 ms forward, 0.082 -> 0.073 inverse on
// the 640-point rows of the plate box)
static int x_np_cap(bool fwd) {
    static int capf = np_cap("LGFIB_XNP", 4), capi = np_cap("LGFIB_XINP", 4);
    return fwd ? capf : capi;
}

template <int P>
static void launch_zconv_np(int cap, dim3 grid, size_t sm, hipStream_t st, const BoxGeo &g, C32 *X2,
                            const float *ghat, float scale, const C32 *tw, int ntiles) {
    if (cap == 4)
        hipLaunchKernelGGL((kf_zconv<C32, P, 4>), grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw, ntiles);
    else if (cap == 8)
        hipLaunchKernelGGL((kf_zconv<C32, P, 8>), grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw, ntiles);
    else
        hipLaunchKernelGGL((kf_zconv<C32, P, 16>), grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw, ntiles);
}

int launch_fast_zconv(const BoxGeo &g, C32 *X2, const float *ghat, float scale, const C32 *tw, hipStream_t st) {
    const int NP = std::min(fast_np_zconv(g.P2), z_np_cap());
    const int ntiles = g.Kxp / NP * (g.P1 / 2 + 1);
    dim3 grid(ntiles);
    const size_t sm = sizeof(C32) * (size_t)(g.P2 / 2 + NP * g.P2 + g.P2) + sizeof(float) * (size_t)NP * (g.P2 / 2 + 1);
    const int cap = z_np_cap();
    switch (g.P2) {
#define X(n) case n: launch_zconv_np<n>(cap, grid, sm, st, g, X2, ghat, scale, tw, ntiles); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised z pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// The z pass in FP64 (the drivers' and the dense build's convolutions):
// the same kernel on double2 pencils, at most 8 per workgroup; lengths whose
// FP64 tile would hold a single pencil stay on the generic kernel.
template <int P> constexpr bool z64_ok() { return np_zconv<P, 8>() >= 2; }

bool fast_z64_size(int P) {
    switch (P) {
#define X(n) case n: return z64_ok<n>();
        LGF_FAST_SIZES(X)
#undef X
    default: return false;
    }
}

template <int P>
static void launch_z64(dim3 grid, size_t sm, hipStream_t st, const BoxGeo &g, double2 *X2, const double *ghat,
                       double scale, const double2 *tw, int ntiles) {
    if constexpr (z64_ok<P>())
        hipLaunchKernelGGL((kf_zconv<double2, P, 8>), grid, dim3(kFftThreads), sm, st, g, X2, ghat, scale, tw, ntiles);
}

int launch_fast_zconv_f64(const BoxGeo &g, double2 *X2, const double *ghat, double scale, const double2 *tw,
                          hipStream_t st) {
    if (!fast_z64_size(g.P2)) return fail(LGFIB_EINVAL, "no specialised FP64 z pass");
    const int NP = std::min(fast_np_zconv_f64(g.P2), 8);
    const int ntiles = g.Kxp / NP * (g.P1 / 2 + 1);
    const size_t sm = sizeof(double2) * (size_t)(g.P2 / 2 + NP * g.P2 + g.P2) + sizeof(double) * (size_t)NP * (g.P2 / 2 + 1);
    switch (g.P2) {
#define X(n) case n: launch_z64<n>(dim3(ntiles), sm, st, g, X2, ghat, scale, tw, ntiles); break;
        LGF_FAST_SIZES(X)
#undef X
    default: break;
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// The y passes in FP64: the same kernels on double2 pencils (at most 8 per
// workgroup by the LDS fit at the plate lengths); lengths whose FP64 tile
// would hold a single pencil stay on the generic kernels.
template <int P> constexpr bool y64_ok() { return np_cols<P, 8>() >= 2; }

bool fast_y64_size(int P) {
    switch (P) {
#define X(n) case n: return y64_ok<n>();
        LGF_FAST_SIZES(X)
#undef X
    default: return false;
    }
}

template <int P, bool FWD>
static void launch_y64(dim3 grid, size_t sm, hipStream_t st, const BoxGeo &g, const double2 *in, double2 *out,
                       const double2 *tw, int ntiles, int T) {
    if constexpr (y64_ok<P>()) {
        if (FWD) hipLaunchKernelGGL((kf_yfwd<double2, P, 16>), grid, dim3(kFftThreads), sm, st, g, in, out, tw, ntiles, T);
        else hipLaunchKernelGGL((kf_yinv<double2, P, 16>), grid, dim3(kFftThreads), sm, st, g, in, out, tw, ntiles, T);
    }
}

static int launch_fast_y_f64(const BoxGeo &g, const double2 *in, double2 *out, const double2 *tw, bool fwd,
                             hipStream_t st) {
    if (!fast_y64_size(g.P1)) return fail(LGFIB_EINVAL, "no specialised FP64 y pass");
    const int NP = std::min(np_fit_y(g.P1, 8), 16);
    const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = y_group(ntiles);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(double2) * (size_t)(g.P1 / 2 + NP * g.P1 + (fwd ? 0 : g.P1));
    switch (g.P1) {
#define X(n) case n: if (fwd) launch_y64<n, true>(grid, sm, st, g, in, out, tw, ntiles, T); else launch_y64<n, false>(grid, sm, st, g, in, out, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: break;
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_yfwd_f64(const BoxGeo &g, const double2 *X1, double2 *X2, const double2 *tw, hipStream_t st) {
    return launch_fast_y_f64(g, X1, X2, tw, true, st);
}
int launch_fast_yinv_f64(const BoxGeo &g, const double2 *X2, double2 *X1, const double2 *tw, hipStream_t st) {
    return launch_fast_y_f64(g, X2, X1, tw, false, st);
}

int launch_fast_yinv(const BoxGeo &g, const C32 *X2, C32 *X1, const C32 *tw, hipStream_t st) {
    const int cap = y_np_cap();
    const int NP = std::min(fast_np_cols(g.P1), cap);
    const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = y_group(ntiles);
    dim3 grid((ntiles + T - 1) / T);
    const size_t sm = sizeof(C32) * (size_t)(g.P1 / 2 + NP * g.P1 + g.P1);
    switch (g.P1) {
#define X(n) case n: launch_y_np<n, false>(cap, grid, sm, st, g, X2, X1, tw, ntiles, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised y pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

int launch_fast_xinv(const BoxGeo &g, const C32 *X1, float *u, int accumulate, const C32 *tw, hipStream_t st) {
    const int cap = x_np_cap(false);
    const int NP = x_np(g.P0, false);
    int T = 1;
    const int nchunks = x_tiles(g, NP, &T, true);
    dim3 grid(nchunks * g.nb1 * g.nb2 * g.ncomp);
    const size_t sm = sizeof(C32) * (size_t)(g.P0 / 2 + NP * g.P0) + sizeof(int) * (size_t)g.nb0;
    switch (g.P0) {
#define X(n) case n: launch_x_np<n, false>(cap, grid, sm, st, g, X1, u, accumulate, tw, nchunks, T); break;
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised x pass");
    }
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

// ------------------------------------------------------ batched dispatch

// pencils per workgroup of the batched passes (x forward 16, x inverse 4,
// y 16, z 8)
static constexpr int kBatchNP[kNumPasses] = {16, 16, 8, 16, 4};

static size_t pass_lds(int pass, const BoxGeo &g, int *NP) {
    switch (pass) {
    case kPassXF: *NP = std::min(fast_np_rows(g.P0), kBatchNP[pass]);
        return sizeof(C32) * (size_t)(g.P0 / 2 + *NP * g.P0) + sizeof(int) * (size_t)g.nb0;
    case kPassXI: *NP = std::min(fast_np_rows(g.P0), kBatchNP[pass]);
        return sizeof(C32) * (size_t)(g.P0 / 2 + *NP * g.P0) + sizeof(int) * (size_t)g.nb0;
    case kPassYF: *NP = std::min(fast_np_cols(g.P1), kBatchNP[pass]);
        return sizeof(C32) * (size_t)(g.P1 / 2 + *NP * g.P1);
    case kPassYI: *NP = std::min(fast_np_cols(g.P1), kBatchNP[pass]);
        return sizeof(C32) * (size_t)(g.P1 / 2 + *NP * g.P1 + g.P1);
    default: *NP = std::min(fast_np_zconv(g.P2), kBatchNP[pass]);
        return sizeof(C32) * (size_t)(g.P2 / 2 + *NP * g.P2 + g.P2) + sizeof(float) * (size_t)*NP * (g.P2 / 2 + 1);
    }
}

int fast_jobs(const BoxGeo &g, const float *f, float *u, C32 *X1, C32 *X2, const float *ghat, float scale,
              const C32 *const tw[3], int tpx, int tpy, FastJob jobs[kNumPasses], int items[kNumPasses],
              size_t sm[kNumPasses], int P[kNumPasses]) {
    if (!(fast_x_ok(g) && fast_size(g.P1) && fast_size(g.P2)))
        return fail(LGFIB_EINVAL, "batched passes need specialised FFT lengths on every axis");
    ConvOverrides &ov = conv_overrides();
    const ConvOverrides saved = ov;
    ov.tpw_x = tpx;
    ov.tpw_y = tpy;
    for (int pass = 0; pass < kNumPasses; ++pass) {
        FastJob &J = jobs[pass];
        J.g = g;
        J.ghat = nullptr;
        J.scale = 0.f;
        J.acc = 0;
        int NP = 1;
        sm[pass] = pass_lds(pass, g, &NP);
        switch (pass) {
        case kPassXF:
        case kPassXI: {
            int T = 1;
            const int nchunks = x_tiles(g, NP, &T, pass == kPassXI);
            J.n = nchunks;
            J.T = T;
            items[pass] = nchunks * g.nb1 * g.nb2 * g.ncomp;
            J.tw = tw[0];
            J.in = pass == kPassXF ? (const void *)f : (const void *)X1;
            J.out = pass == kPassXF ? (void *)X1 : (void *)u;
            P[pass] = g.P0;
            break;
        }
        case kPassYF:
        case kPassYI: {
            const int ntiles = g.Kxp / NP * g.N2 * g.ncomp, T = y_group(ntiles);
            J.n = ntiles;
            J.T = T;
            items[pass] = (ntiles + T - 1) / T;
            J.tw = tw[1];
            J.in = pass == kPassYF ? (const void *)X1 : (const void *)X2;
            J.out = pass == kPassYF ? (void *)X2 : (void *)X1;
            P[pass] = g.P1;
            break;
        }
        default: {
            const int ntiles = g.Kxp / NP * (g.P1 / 2 + 1);
            J.n = ntiles;
            J.T = 1;
            items[pass] = ntiles;
            J.tw = tw[2];
            J.in = X2;
            J.out = X2;
            J.ghat = ghat;
            J.scale = scale;
            P[pass] = g.P2;
        }
        }
    }
    ov = saved;
    return LGFIB_OK;
}

// one workgroup per item (default: measured faster, it keeps the XCD-aware
// item order), or the persistent queue form with LGFIB_BATCH_PERSIST=1
static bool batch_persistent() {
    static const bool on = [] {
        const char *e = getenv("LGFIB_BATCH_PERSIST");
        return e && e[0] == '1';
    }();
    return on;
}

template <int PASS, int P>
static int launch_batched_p(const FastJob *jobs, const int *start, const int *owner, int njobs, int total, int *queue,
                            size_t sm, int num_cu, hipStream_t st) {
    constexpr int NPM = kBatchNP[PASS];
    (void)njobs;
    if (!batch_persistent()) {
        hipLaunchKernelGGL((kb_pass_grid<PASS, P, NPM>), dim3(total), dim3(kFftThreads), sm, st, jobs, start, owner,
                           total);
        return LGFIB_OK;
    }
    auto kern = kb_pass<PASS, P, NPM>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kFftThreads, sm) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int grid = std::max(1, std::min(total, per_cu * std::max(num_cu, 1)));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFftThreads), sm, st, jobs, start, owner, total, queue);
    return LGFIB_OK;
}

template <int PASS>
static int launch_batched_pass(int P, const FastJob *jobs, const int *start, const int *owner, int njobs, int total,
                               int *queue, size_t sm, int num_cu, hipStream_t st) {
    switch (P) {
#define X(n) case n: return launch_batched_p<PASS, n>(jobs, start, owner, njobs, total, queue, sm, num_cu, st);
        LGF_FAST_SIZES(X)
#undef X
    default: return fail(LGFIB_EINVAL, "no specialised batched pass for this length");
    }
}

int launch_fast_batched(int pass, int P, const FastJob *jobs, const int *start, const int *owner, int njobs,
                        int total, int *queue, size_t sm, int num_cu, hipStream_t st) {
    if (total <= 0) return LGFIB_OK;
    int rc;
    switch (pass) {
    case kPassXF: rc = launch_batched_pass<kPassXF>(P, jobs, start, owner, njobs, total, queue, sm, num_cu, st); break;
    case kPassYF: rc = launch_batched_pass<kPassYF>(P, jobs, start, owner, njobs, total, queue, sm, num_cu, st); break;
    case kPassZ: rc = launch_batched_pass<kPassZ>(P, jobs, start, owner, njobs, total, queue, sm, num_cu, st); break;
    case kPassYI: rc = launch_batched_pass<kPassYI>(P, jobs, start, owner, njobs, total, queue, sm, num_cu, st); break;
    default: rc = launch_batched_pass<kPassXI>(P, jobs, start, owner, njobs, total, queue, sm, num_cu, st); break;
    }
    if (rc) return rc;
    LGF_HIP(hipGetLastError());
    return LGFIB_OK;
}

}  // namespace lgfib
