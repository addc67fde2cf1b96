// conv.hip -- block-wise LGF convolution u = dx^2 G * f by a zero-padded FFT
// over the bounding box of the active blocks (Sec. 2.2, Eq. dpoisson_conv).
//
// The convolution of sources on a box of N cells per axis with an even kernel,
// evaluated at targets in the same box, equals a circular convolution of
// length P = 2N per axis (offsets span -(N-1)..N-1, which fit without
// wrap-around).  The kernel's spectrum on that box is real and even (built in
// table.hip).  Five passes, each streaming through HBM once:
//   1. x: real rows of the box -> x-spectrum (two real rows per complex FFT),
//      reading only active source blocks (empty rows are never read later);
//   2. y: columns of the x-spectrum, zero-padded to P1 -> xy-spectrum;
//   3. z: columns zero-padded to P2, FFT, times the kernel spectrum, inverse
//      FFT, keep the first N2 -- one fused pass, all components per workgroup;
//   4. y inverse, keeping the first N1 rows, only rows that hold targets;
//   5. x inverse (complex-to-real, two rows per FFT), cropped to the target
//      blocks and written in the caller's block layout.
#include <algorithm>
#include <cmath>

#include "conv_common.h"
#include "fft_lds.h"

namespace lgfib {

static void make_fft_plan(int P, FftPlan1D &pl) {
    pl.P = P;
    pl.nst = 0;
    int r = P;
    int e2 = 0;
    while (r % 2 == 0) {
        r /= 2;
        ++e2;
    }
    while (r % 5 == 0) {
        pl.rad[pl.nst++] = 5;
        r /= 5;
    }
    while (r % 3 == 0) {
        pl.rad[pl.nst++] = 3;
        r /= 3;
    }
    int n8 = e2 / 3, rem = e2 % 3;
    if (rem == 1 && n8 > 0) {
        --n8;
        pl.rad[pl.nst++] = 4;
        pl.rad[pl.nst++] = 4;
    } else if (rem == 1) {
        pl.rad[pl.nst++] = 2;
    } else if (rem == 2) {
        pl.rad[pl.nst++] = 4;
    }
    for (int i = 0; i < n8; ++i) pl.rad[pl.nst++] = 8;
}

int get_twiddles(lgfib_ctx *ctx, int P, int prec, const void **dev) {
    auto key = std::make_pair(P, prec);
    auto it = ctx->twiddles.find(key);
    if (it != ctx->twiddles.end()) {
        *dev = it->second->p;
        return LGFIB_OK;
    }
    auto buf = std::make_unique<DevBuf>();
    int rc;
    std::vector<double> c(P), s(P);
    for (int m = 0; m < P; ++m) {
        // exp(-2 pi i m / P) via the octant-reduced angle for accuracy
        int mm = m;
        double sign_s = 1.0;
        if (2 * mm > P) {   // sin odd, cos even about P/2
            mm = P - mm;
            sign_s = -1.0;
        }
        double cv, sv;
        if (4 * mm <= P) {
            double a = 2.0 * M_PI * mm / P;
            cv = cos(a);
            sv = sin(a);
        } else {
            double a = 2.0 * M_PI * (P / 2.0 - mm) / P;   // angle = pi - a
            cv = -cos(a);
            sv = sin(a);
        }
        c[m] = cv;
        s[m] = -sign_s * sv;
    }
    if (prec == LGF_F64) {
        std::vector<double2> h(P);
        for (int m = 0; m < P; ++m) h[m] = double2{c[m], s[m]};
        if ((rc = buf->reserve(P * sizeof(double2)))) return rc;
        LGF_HIP(hipMemcpy(buf->p, h.data(), P * sizeof(double2), hipMemcpyHostToDevice));
    } else {
        std::vector<float2> h(P);
        for (int m = 0; m < P; ++m) h[m] = float2{(float)c[m], (float)s[m]};
        if ((rc = buf->reserve(P * sizeof(float2)))) return rc;
        LGF_HIP(hipMemcpy(buf->p, h.data(), P * sizeof(float2), hipMemcpyHostToDevice));
    }
    *dev = buf->p;
    ctx->twiddles[key] = std::move(buf);
    return LGFIB_OK;
}

template <typename Real> struct Tune;
template <> struct Tune<float> { static constexpr int MAXV = 32; };
template <> struct Tune<double> { static constexpr int MAXV = 16; };

// ------------------------------------------------------------------- pass 1
// Rows r = z * N1 + y; a workgroup takes 2*NP consecutive rows, packing row
// 2p in the real and row 2p+1 in the imaginary part of pencil p.
template <typename Real>
__global__ __launch_bounds__(kFftThreads) void k_xfwd(BoxGeo g, FftPlan1D pl, int NP, const Real *__restrict__ f,
                                                      typename CplxOf<Real>::T *__restrict__ X1,
                                                      const typename CplxOf<Real>::T *__restrict__ tw) {
    using C = typename CplxOf<Real>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *s = reinterpret_cast<C *>(smem_raw);
    const int c = blockIdx.y;
    const int nrows = g.N1 * g.N2;
    const int row0 = blockIdx.x * 2 * NP;
    const int B = g.B, B2 = B * B, B3 = B2 * B;
    // skip the workgroup if none of its rows holds a source
    bool any = false;
    for (int q = 0; q < 2 * NP; ++q) {
        const int row = row0 + q;
        if (row < nrows) {
            const int y = row % g.N1, z = row / g.N1;
            any |= g.src_rows[(z / B) * g.nb1 + y / B] != 0;
        }
    }
    if (!any) return;
    const int P = g.P0;
    const size_t fbase = (size_t)c * g.nsrc * B3;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx / P, x = idx - p * P;
        Real va = 0, vb = 0;
        if (x < g.N0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = row0 + 2 * p + h;
                Real v = 0;
                if (row < nrows) {
                    const int y = row % g.N1, z = row / g.N1;
                    const int slot = g.src_map[((z / B) * g.nb1 + y / B) * g.nb0 + x / B];
                    if (slot >= 0) v = f[fbase + (size_t)slot * B3 + (z % B) * B2 + (y % B) * B + (x % B)];
                }
                if (h == 0) va = v; else vb = v;
            }
        }
        s[p * P + x] = C{va, vb};
    }
    __syncthreads();
    fft_lds<C, Tune<Real>::MAXV, false, false>(s, pl, NP, P, 1, tw);
    // split the two real spectra: Xa = (Z_k + conj Z_{-k})/2, Xb = -i (Z_k - conj Z_{-k})/2
    const int Kxp = g.Kxp, Kx = g.Kx;
    for (int idx = threadIdx.x; idx < NP * Kxp; idx += kFftThreads) {
        const int p = idx / Kxp, k = idx - p * Kxp;
        C xa = C{0, 0}, xb = C{0, 0};
        if (k < Kx) {
            const C zk = s[p * P + k];
            const C zm = s[p * P + (k == 0 ? 0 : P - k)];
            xa = C{(Real)0.5 * (zk.x + zm.x), (Real)0.5 * (zk.y - zm.y)};
            xb = C{(Real)0.5 * (zk.y + zm.y), (Real)0.5 * (zm.x - zk.x)};
        }
        const int ra = row0 + 2 * p, rb = ra + 1;
        if (ra < nrows) X1[((size_t)c * nrows + ra) * Kxp + k] = xa;
        if (rb < nrows) X1[((size_t)c * nrows + rb) * Kxp + k] = xb;
    }
}

// ------------------------------------------------------------------- pass 2
template <typename Real>
__global__ __launch_bounds__(kFftThreads) void k_yfwd(BoxGeo g, FftPlan1D pl, int NP,
                                                      const typename CplxOf<Real>::T *__restrict__ X1,
                                                      typename CplxOf<Real>::T *__restrict__ X2,
                                                      const typename CplxOf<Real>::T *__restrict__ tw) {
    using C = typename CplxOf<Real>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *s = reinterpret_cast<C *>(smem_raw);
    const int k0 = blockIdx.x * NP, z = blockIdx.y, c = blockIdx.z;
    const int P = g.P1, B = g.B, Kxp = g.Kxp;
    const size_t in0 = ((size_t)c * g.N2 + z) * g.N1;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, y = idx / NP;
        C v = C{0, 0};
        if (y < g.N1 && g.src_rows[(z / B) * g.nb1 + y / B]) v = X1[(in0 + y) * Kxp + k0 + p];
        s[y * NP + p] = v;
    }
    __syncthreads();
    fft_lds<C, Tune<Real>::MAXV, false, true>(s, pl, NP, 1, NP, tw);
    const size_t out0 = ((size_t)c * g.N2 + z) * P;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, ky = idx / NP;
        X2[(out0 + ky) * Kxp + k0 + p] = s[ky * NP + p];
    }
}

// ------------------------------------------------------------------- pass 3
template <typename Real>
__global__ __launch_bounds__(kFftThreads) void k_zconv(BoxGeo g, FftPlan1D pl, int NP,
                                                       typename CplxOf<Real>::T *__restrict__ X2,
                                                       const Real *__restrict__ ghat, Real scale,
                                                       const typename CplxOf<Real>::T *__restrict__ tw) {
    using C = typename CplxOf<Real>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *s = reinterpret_cast<C *>(smem_raw);
    const int P = g.P2, Kxp = g.Kxp, Ph = P / 2;
    Real *gh = reinterpret_cast<Real *>(smem_raw + sizeof(C) * (size_t)NP * P);
    const int k0 = blockIdx.x * NP, ky = blockIdx.y;
    const int kyh = min(ky, g.P1 - ky);
    const int H1 = g.P1 / 2 + 1;
    for (int idx = threadIdx.x; idx < NP * (Ph + 1); idx += kFftThreads) {
        const int p = idx % NP, kz = idx / NP;
        gh[kz * NP + p] = scale * ghat[((size_t)kz * H1 + kyh) * Kxp + k0 + p];
    }
    for (int c = 0; c < g.ncomp; ++c) {
        const size_t base = (size_t)c * g.N2 * g.P1;
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, z = idx / NP;
            C v = C{0, 0};
            if (z < g.N2) v = X2[((base + (size_t)z * g.P1) + ky) * Kxp + k0 + p];
            s[z * NP + p] = v;
        }
        __syncthreads();
        fft_lds<C, Tune<Real>::MAXV, false, true>(s, pl, NP, 1, NP, tw);
        for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
            const int p = idx % NP, kz = idx / NP;
            const Real w = gh[min(kz, P - kz) * NP + p];
            C v = s[kz * NP + p];
            s[kz * NP + p] = C{v.x * w, v.y * w};
        }
        __syncthreads();
        fft_lds<C, Tune<Real>::MAXV, true, true>(s, pl, NP, 1, NP, tw);
        for (int idx = threadIdx.x; idx < NP * g.N2; idx += kFftThreads) {
            const int p = idx % NP, z = idx / NP;
            X2[((base + (size_t)z * g.P1) + ky) * Kxp + k0 + p] = s[z * NP + p];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------- pass 4
template <typename Real>
__global__ __launch_bounds__(kFftThreads) void k_yinv(BoxGeo g, FftPlan1D pl, int NP,
                                                      const typename CplxOf<Real>::T *__restrict__ X2,
                                                      typename CplxOf<Real>::T *__restrict__ X1,
                                                      const typename CplxOf<Real>::T *__restrict__ tw) {
    using C = typename CplxOf<Real>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *s = reinterpret_cast<C *>(smem_raw);
    const int k0 = blockIdx.x * NP, z = blockIdx.y, c = blockIdx.z;
    const int P = g.P1, B = g.B, Kxp = g.Kxp;
    bool any = false;
    for (int by = 0; by < g.nb1; ++by) any |= g.tgt_rows[(z / B) * g.nb1 + by] != 0;
    if (!any) return;
    const size_t in0 = ((size_t)c * g.N2 + z) * P;
    for (int idx = threadIdx.x; idx < NP * P; idx += kFftThreads) {
        const int p = idx % NP, ky = idx / NP;
        s[ky * NP + p] = X2[(in0 + ky) * Kxp + k0 + p];
    }
    __syncthreads();
    fft_lds<C, Tune<Real>::MAXV, true, true>(s, pl, NP, 1, NP, tw);
    const size_t out0 = ((size_t)c * g.N2 + z) * g.N1;
    for (int idx = threadIdx.x; idx < NP * g.N1; idx += kFftThreads) {
        const int p = idx % NP, y = idx / NP;
        if (g.tgt_rows[(z / B) * g.nb1 + y / B]) X1[(out0 + y) * Kxp + k0 + p] = s[y * NP + p];
    }
}

// ------------------------------------------------------------------- pass 5
template <typename Real>
__global__ __launch_bounds__(kFftThreads) void k_xinv(BoxGeo g, FftPlan1D pl, int NP,
                                                      const typename CplxOf<Real>::T *__restrict__ X1,
                                                      Real *__restrict__ u, int accumulate,
                                                      const typename CplxOf<Real>::T *__restrict__ tw) {
    using C = typename CplxOf<Real>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *s = reinterpret_cast<C *>(smem_raw);
    const int c = blockIdx.y;
    const int nrows = g.N1 * g.N2;
    const int row0 = blockIdx.x * 2 * NP;
    const int B = g.B, B2 = B * B, B3 = B2 * B;
    bool any = false;
    for (int q = 0; q < 2 * NP; ++q) {
        const int row = row0 + q;
        if (row < nrows) {
            const int y = row % g.N1, z = row / g.N1;
            any |= g.tgt_rows[(z / B) * g.nb1 + y / B] != 0;
        }
    }
    if (!any) return;
    const int P = g.P0, Kx = g.Kx, Kxp = g.Kxp, Ph = P / 2;
    for (int idx = threadIdx.x; idx < NP * Kx; idx += kFftThreads) {
        const int p = idx / Kx, k = idx - p * Kx;
        C xa = C{0, 0}, xb = C{0, 0};
        const int ra = row0 + 2 * p, rb = ra + 1;
        // rows without targets were not written by pass 4: read them as zero
        // (their garbage would leak into the partner row through the FFT)
        if (ra < nrows && g.tgt_rows[((ra / g.N1) / B) * g.nb1 + (ra % g.N1) / B])
            xa = X1[((size_t)c * nrows + ra) * Kxp + k];
        if (rb < nrows && g.tgt_rows[((rb / g.N1) / B) * g.nb1 + (rb % g.N1) / B])
            xb = X1[((size_t)c * nrows + rb) * Kxp + k];
        if (k == 0 || k == Ph) {
            xa.y = 0;
            xb.y = 0;
        }
        // Z = Xa + i Xb  at k;  conj(Xa) + i conj(Xb)  at P - k
        s[p * P + k] = C{xa.x - xb.y, xa.y + xb.x};
        if (k > 0 && k < Ph) s[p * P + P - k] = C{xa.x + xb.y, xb.x - xa.y};
    }
    __syncthreads();
    fft_lds<C, Tune<Real>::MAXV, true, false>(s, pl, NP, P, 1, tw);
    const size_t ubase = (size_t)c * g.ntgt * B3;
    for (int idx = threadIdx.x; idx < NP * g.N0; idx += kFftThreads) {
        const int p = idx / g.N0, x = idx - p * g.N0;
        const C v = s[p * P + x];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = row0 + 2 * p + h;
            if (row < nrows) {
                const int y = row % g.N1, z = row / g.N1;
                const int slot = g.tgt_map[((z / B) * g.nb1 + y / B) * g.nb0 + x / B];
                if (slot >= 0) {
                    Real *dst = u + ubase + (size_t)slot * B3 + (z % B) * B2 + (y % B) * B + (x % B);
                    const Real val = h == 0 ? v.x : v.y;
                    *dst = accumulate ? *dst + val : val;
                }
            }
        }
    }
}

template <typename Real> __global__ void k_fill(Real *p, size_t n, Real v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static int pick_np(int P, int maxv, int cap) {
    int np = cap;
    while (np > 1 && np * P > kFftThreads * maxv) np /= 2;
    return np;
}

void make_box_geo(const BoxPlan &plan, int ncomp, BoxGeo &g) {
    g.B = plan.B;
    g.lb = plan.B == 4 ? 2 : plan.B == 8 ? 3 : plan.B == 16 ? 4 : 5;
    g.nb0 = plan.nb[0];
    g.nb1 = plan.nb[1];
    g.nb2 = plan.nb[2];
    g.N0 = plan.N[0];
    g.N1 = plan.N[1];
    g.N2 = plan.N[2];
    g.P0 = plan.P[0];
    g.P1 = plan.P[1];
    g.P2 = plan.P[2];
    g.Kx = plan.Kx;
    g.Kxp = plan.Kxp;
    g.nsrc = plan.nsrc;
    g.ntgt = plan.ntgt;
    g.ncomp = ncomp;
    g.src_map = plan.src_map.as<int>();
    g.tgt_map = plan.tgt_map.as<int>();
    g.src_rows = plan.src_rows.as<int>();
    g.tgt_rows = plan.tgt_rows.as<int>();
    g.masks_ok = g.nb2 <= BoxGeo::kMaskPlanes && g.nb1 <= 128;
    for (int z = 0; z < BoxGeo::kMaskPlanes; ++z)
        for (int w = 0; w < 2; ++w) {
            const bool in = g.masks_ok && z < g.nb2;
            g.src_mask[z][w] = in ? plan.src_mask[2 * z + w] : 0ull;
            g.tgt_mask[z][w] = in ? plan.tgt_mask[2 * z + w] : 0ull;
        }

}

template <typename Real>
static int run_box_conv(lgfib_ctx *ctx, const BoxPlan &plan, const Spectrum &spec, int ncomp, double dx,
                        const Real *f, Real *u, int accumulate, hipStream_t st) {
    using C = typename CplxOf<Real>::T;
    const int prec = sizeof(Real) == 8 ? LGF_F64 : LGF_F32;
    BoxGeo g;
    make_box_geo(plan, ncomp, g);

    const size_t n1 = (size_t)ncomp * g.N2 * g.N1 * g.Kxp;
    const size_t n2 = (size_t)ncomp * g.N2 * g.P1 * g.Kxp;
    int rc;
    C *X1, *X2;
    const ConvOverrides &ov = conv_overrides();
    if (ov.w1 && ov.w2) {
        if (ov.w1_bytes < n1 * sizeof(C) || ov.w2_bytes < n2 * sizeof(C))
            return fail(LGFIB_EINVAL, "box convolution: external workspace too small");
        X1 = (C *)ov.w1;
        X2 = (C *)ov.w2;
    } else {
        if ((rc = ctx->work1.reserve(n1 * sizeof(C)))) return rc;
        if ((rc = ctx->work2.reserve(n2 * sizeof(C)))) return rc;
        X1 = ctx->work1.as<C>();
        X2 = ctx->work2.as<C>();
    }
    const void *tw0, *tw1, *tw2;
    if ((rc = get_twiddles(ctx, g.P0, prec, &tw0))) return rc;
    if ((rc = get_twiddles(ctx, g.P1, prec, &tw1))) return rc;
    if ((rc = get_twiddles(ctx, g.P2, prec, &tw2))) return rc;
    FftPlan1D p0, p1, p2;
    make_fft_plan(g.P0, p0);
    make_fft_plan(g.P1, p1);
    make_fft_plan(g.P2, p2);
    const int maxv = Tune<Real>::MAXV;
    const int npx = pick_np(g.P0, maxv, 16);
    const int npy = pick_np(g.P1, maxv, 16);
    const int npz = pick_np(g.P2, maxv, 16);
    const int nrows = g.N1 * g.N2;
    const Real scale = (Real)(dx * dx / ((double)g.P0 * g.P1 * g.P2));

    const bool fast = sizeof(Real) == 4;
    {
        ProfScope ps(ctx, "k_xfwd", st);
        if (fast && fast_x_ok(g)) {
            if ((rc = launch_fast_xfwd(g, (const float *)f, (float2 *)X1, (const float2 *)tw0, st))) return rc;
        } else {
            hipLaunchKernelGGL(k_xfwd<Real>, dim3((nrows + 2 * npx - 1) / (2 * npx), ncomp), dim3(kFftThreads),
                               sizeof(C) * npx * g.P0, st, g, p0, npx, f, X1, (const C *)tw0);
            LGF_HIP(hipGetLastError());
        }
    }
    {
        ProfScope ps(ctx, "k_yfwd", st);
        if (fast && fast_size(g.P1)) {
            if ((rc = launch_fast_yfwd(g, (const float2 *)X1, (float2 *)X2, (const float2 *)tw1, st))) return rc;
        } else if (!fast && fast_y64_size(g.P1)) {
            if ((rc = launch_fast_yfwd_f64(g, (const double2 *)X1, (double2 *)X2, (const double2 *)tw1, st)))
                return rc;
        } else {
            hipLaunchKernelGGL(k_yfwd<Real>, dim3(g.Kxp / npy, g.N2, ncomp), dim3(kFftThreads),
                               sizeof(C) * npy * g.P1, st, g, p1, npy, (const C *)X1, X2, (const C *)tw1);
            LGF_HIP(hipGetLastError());
        }
    }
    {
        ProfScope ps(ctx, "k_zconv", st);
        if (fast && fast_size(g.P2)) {
            if ((rc = launch_fast_zconv(g, (float2 *)X2, (const float *)spec.ghat.p, (float)scale,
                                        (const float2 *)tw2, st)))
                return rc;
        } else if (!fast && fast_z64_size(g.P2)) {
            if ((rc = launch_fast_zconv_f64(g, (double2 *)X2, (const double *)spec.ghat.p, (double)scale,
                                            (const double2 *)tw2, st)))
                return rc;
        } else {
            hipLaunchKernelGGL(k_zconv<Real>, dim3(g.Kxp / npz, g.P1), dim3(kFftThreads),
                               sizeof(C) * npz * g.P2 + sizeof(Real) * npz * (g.P2 / 2 + 1), st, g, p2, npz, X2,
                               spec.ghat.as<Real>(), scale, (const C *)tw2);
            LGF_HIP(hipGetLastError());
        }
    }
    {
        ProfScope ps(ctx, "k_yinv", st);
        if (fast && fast_size(g.P1)) {
            if ((rc = launch_fast_yinv(g, (const float2 *)X2, (float2 *)X1, (const float2 *)tw1, st))) return rc;
        } else if (!fast && fast_y64_size(g.P1)) {
            if ((rc = launch_fast_yinv_f64(g, (const double2 *)X2, (double2 *)X1, (const double2 *)tw1, st)))
                return rc;
        } else {
            hipLaunchKernelGGL(k_yinv<Real>, dim3(g.Kxp / npy, g.N2, ncomp), dim3(kFftThreads),
                               sizeof(C) * npy * g.P1, st, g, p1, npy, (const C *)X2, X1, (const C *)tw1);
            LGF_HIP(hipGetLastError());
        }
    }
    {
        ProfScope ps(ctx, "k_xinv", st);
        if (fast && fast_x_ok(g)) {
            if ((rc = launch_fast_xinv(g, (const float2 *)X1, (float *)u, accumulate, (const float2 *)tw0, st)))
                return rc;
        } else {
            hipLaunchKernelGGL(k_xinv<Real>, dim3((nrows + 2 * npx - 1) / (2 * npx), ncomp), dim3(kFftThreads),
                               sizeof(C) * npx * g.P0, st, g, p0, npx, (const C *)X1, u, accumulate,
                               (const C *)tw0);
            LGF_HIP(hipGetLastError());
        }
    }
    return LGFIB_OK;
}

void box_work_bytes(const BoxPlan &plan, int ncomp, int prec, size_t *w1, size_t *w2) {
    const size_t cs = prec == LGF_F64 ? 16 : 8;
    *w1 = (size_t)ncomp * plan.N[2] * plan.N[1] * plan.Kxp * cs;
    *w2 = (size_t)ncomp * plan.N[2] * plan.P[1] * plan.Kxp * cs;
}

int box_conv_f32(lgfib_ctx *ctx, const BoxPlan &plan, const Spectrum &spec, int ncomp, double dx, const float *f,
                 float *u, int accumulate, hipStream_t st) {
    return run_box_conv<float>(ctx, plan, spec, ncomp, dx, f, u, accumulate, st);
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace lgfib

using namespace lgfib;

extern "C" int lgf_poisson_apply(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *src_blocks, int nsrc,
                                 const int32_t *tgt_blocks, int ntgt, int ncomp, int prec, double dx, const void *f,
                                 void *u, int accumulate, lgfib_stream_t stream) {
    if (!ctx) return fail(LGFIB_EINVAL, "lgf_poisson_apply: null context");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_poisson_apply: unknown table");
    if (B != 4 && B != 8 && B != 16 && B != 32) return fail(LGFIB_EINVAL, "lgf_poisson_apply: B must be 4, 8, 16 or 32");
    if (ncomp < 1 || ncomp > 8) return fail(LGFIB_EINVAL, "lgf_poisson_apply: ncomp must lie in [1, 8]");
    if (prec != LGF_F32 && prec != LGF_F64) return fail(LGFIB_EINVAL, "lgf_poisson_apply: prec must be LGF_F32 or LGF_F64");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LGFIB_EINVAL, "lgf_poisson_apply: dx must be positive");
    if (nsrc < 0 || ntgt < 0) return fail(LGFIB_EINVAL, "lgf_poisson_apply: negative block count");
    const size_t es = prec == LGF_F64 ? 8 : 4;
    const size_t B3 = (size_t)B * B * B;
    const size_t fbytes = (size_t)ncomp * nsrc * B3 * es, ubytes = (size_t)ncomp * ntgt * B3 * es;
    if ((nsrc > 0 && !f) || (ntgt > 0 && !u)) return fail(LGFIB_EINVAL, "lgf_poisson_apply: null field pointer");
    if (nsrc > 0 && ntgt > 0 && overlaps(f, fbytes, u, ubytes))
        return fail(LGFIB_EINVAL, "lgf_poisson_apply: f and u overlap");
    LGF_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    // block lists are validated when their plan is built (a cached plan
    // matched the same lists before)
    if ((nsrc > 0 && !src_blocks) || (ntgt > 0 && !tgt_blocks)) return fail(LGFIB_EINVAL, "null block list");
    int rc = LGFIB_OK;
    if (ntgt == 0) return LGFIB_OK;
    if (nsrc == 0) {
        if (!accumulate) LGF_HIP(hipMemsetAsync(u, 0, ubytes, st));
        return LGFIB_OK;
    }
    std::shared_ptr<BoxPlan> plan;
    if ((rc = get_box_plan(ctx, B, src_blocks, nsrc, tgt_blocks, ntgt, plan))) return rc;
    // the table must reach every offset between cells of the blocks' span
    const Table &tb = *ctx->tables[tbl];
    {
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        for (const int32_t *bl : {src_blocks, tgt_blocks}) {
            const int n = bl == src_blocks ? nsrc : ntgt;
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], (int)bl[3 * i + a]);
                    hi[a] = std::max(hi[a], (int)bl[3 * i + a]);
                }
        }
        for (int a = 0; a < 3; ++a)
            if (tb.ext[a] < (hi[a] - lo[a] + 1) * B - 1)
                return fail(LGFIB_ERANGE, "lgf_poisson_apply: table extent " + std::to_string(tb.ext[a]) +
                                              " along axis " + std::to_string(a) + " is below the needed " +
                                              std::to_string((hi[a] - lo[a] + 1) * B - 1));
    }
    std::shared_ptr<Spectrum> spec;
    if ((rc = get_spectrum(ctx, tbl, *plan, prec, st, spec))) return rc;
    if (prec == LGF_F64)
        return run_box_conv<double>(ctx, *plan, *spec, ncomp, dx, (const double *)f, (double *)u, accumulate, st);
    return run_box_conv<float>(ctx, *plan, *spec, ncomp, dx, (const float *)f, (float *)u, accumulate, st);
}
