// table.hip -- FP64 construction of the lattice Green's functions on the GPU
// and of their cosine spectra on a padded FFT box.
//
// App. A expresses the LGFs through the scaled modified Bessel functions
// g_n(t) = e^{-2t} I_n(2t):
//   G_E(a)(n) = prod_q g_{n_q}(a)                       (Eq. lgf_intfac)
//   G_L(n)    = - int_0^inf prod_q g_{n_q}(t) dt        (Eq. lgf_lap)
//   G_K(a)(n) = G_L(n) + int_0^a prod_q g_{n_q}(t) dt   (partition of G_K)
// The t-integral is done here by composite Gauss-Legendre panels (linear on
// [0,1], logarithmic in t on [1,T]) plus the analytic integral of the large-t
// series of the product on [T, inf).  The Bessel vectors at all quadrature
// nodes are computed once, so a table entry is a 3-way contraction over the
// nodes.  Beyond max|n_i| > 256 the far-field expansion of G_L is used (its
// leading term is -1/(4 pi |n|)); G_K - G_L is below 1e-30 there.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace lgfib {

static constexpr int kQuadRadius = 256;   // quadrature for max|n| <= this
static constexpr int kRRadius = 64;       // R(a) kept for max|n| <= this (a <= 4)
static constexpr int kGL = 20;            // Gauss-Legendre points per panel

// ------------------------------------------------------------------ Bessel

// e^{-x} I_n(x) for n = 0..nmax into out[0..nmax] (stride 1).
// Large x (>= 30 nmax^2 + 200): Hankel's asymptotic series, whose terms then
// shrink by >= 60x per order.  Otherwise Miller's backward recurrence
// I_{n-1} = (2n/x) I_n + I_{n+1}, started far enough above nmax that the
// dominant solution is reached, normalised by e^{-x}(I_0 + 2 sum I_n) = 1.
__host__ __device__ static void bessel_scaled_vec(double x, int nmax, double *out) {
    if (x <= 0.0) {
        out[0] = 1.0;
        for (int n = 1; n <= nmax; ++n) out[n] = 0.0;
        return;
    }
    if (x >= 30.0 * (double)nmax * (double)nmax + 200.0) {
        const double pre = 1.0 / sqrt(2.0 * M_PI * x);
        for (int n = 0; n <= nmax; ++n) {
            const double mu = 4.0 * (double)n * (double)n;
            double term = 1.0, sum = 1.0;
            for (int k = 1; k < 40; ++k) {
                term *= -(mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k * x);
                sum += term;
                if (fabs(term) < 1e-18 * fabs(sum)) break;
            }
            out[n] = pre * sum;
        }
        return;
    }
    const int N0 = nmax + 24 + (int)ceil(sqrt(80.0 * x));
    double ip1 = 0.0, i0 = 1e-280, sum = 0.0;
    for (int n = N0; n >= 1; --n) {
        // i0 = I_n, ip1 = I_{n+1} (up to a common factor)
        if (n <= nmax) out[n] = i0;
        sum += i0;
        const double im1 = (2.0 * n / x) * i0 + ip1;
        ip1 = i0;
        i0 = im1;
        if (i0 > 1e250) {
            i0 *= 1e-250;
            ip1 *= 1e-250;
            sum *= 1e-250;
            for (int k = n; k <= nmax; ++k) out[k] *= 1e-250;
        }
    }
    out[0] = i0;
    const double inv = 1.0 / (i0 + 2.0 * sum);
    for (int n = 0; n <= nmax; ++n) out[n] *= inv;
}

__global__ void k_bessel_nodes(const double *__restrict__ t, int nodes, int nmax, double *__restrict__ bes) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nodes) return;
    bessel_scaled_vec(2.0 * t[j], nmax, bes + (size_t)j * (nmax + 1));
}

// ------------------------------------------------------------ quadrature

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-17) break;
        }
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// Composite rule for int_0^T: linear panels on [0, 1], log panels of width
// 0.5 in ln t on [1, T].  Weights include the Jacobian.
static void lgf_nodes(double T, std::vector<double> &t, std::vector<double> &w) {
    std::vector<double> gx, gw;
    gauss_legendre(kGL, gx, gw);
    t.clear();
    w.clear();
    for (int p = 0; p < 4; ++p) {
        double a = 0.25 * p, b = 0.25 * (p + 1);
        for (int i = 0; i < kGL; ++i) {
            t.push_back(0.5 * (a + b) + 0.5 * (b - a) * gx[i]);
            w.push_back(0.5 * (b - a) * gw[i]);
        }
    }
    const double sT = log(T);
    const int np = (int)ceil(sT / 0.5);
    for (int p = 0; p < np; ++p) {
        double a = sT * p / np, b = sT * (p + 1) / np;
        for (int i = 0; i < kGL; ++i) {
            double s = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
            double tt = exp(s);
            t.push_back(tt);
            w.push_back(0.5 * (b - a) * gw[i] * tt);
        }
    }
}

static void r_nodes(double alpha, std::vector<double> &t, std::vector<double> &w) {
    std::vector<double> gx, gw;
    gauss_legendre(kGL, gx, gw);
    t.clear();
    w.clear();
    const int np = 8;
    for (int p = 0; p < np; ++p) {
        double a = alpha * p / np, b = alpha * (p + 1) / np;
        for (int i = 0; i < kGL; ++i) {
            t.push_back(0.5 * (a + b) + 0.5 * (b - a) * gx[i]);
            w.push_back(0.5 * (b - a) * gw[i]);
        }
    }
}

// --------------------------------------------------------- table kernels

// coefficients of the large-argument series e^{-x} I_n(x) ~ (2 pi x)^{-1/2} sum_k a_k x^{-k}
__device__ static void hankel_coeffs(int n, double *a, int K) {
    const double mu = 4.0 * (double)n * (double)n;
    a[0] = 1.0;
    for (int k = 1; k <= K; ++k) a[k] = -a[k - 1] * (mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (8.0 * k);
}

// Far-field expansion of G_L (lattice units), three terms:
//   -1/(4 pi r) + (3 r^4 - 5 sum n^4)/(32 pi r^7)
//   - (23 S8 - 244 S62 + 621 S44 - 228 S422)/(128 pi r^13)
// obtained by expanding 1/sigma(xi) about xi = 0 in homogeneous terms and
// inverting each with the 3D transforms of |xi|^-2, |xi|^-4, |xi|^-6.
__device__ static double lgf_far(int a, int b, int c) {
    const double x = a, y = b, z = c;
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double r2 = x2 + y2 + z2, r = sqrt(r2);
    const double s4 = x2 * x2 + y2 * y2 + z2 * z2;
    const double s8 = x2 * x2 * x2 * x2 + y2 * y2 * y2 * y2 + z2 * z2 * z2 * z2;
    const double s62 = x2 * x2 * x2 * (y2 + z2) + y2 * y2 * y2 * (x2 + z2) + z2 * z2 * z2 * (x2 + y2);
    const double s44 = x2 * x2 * y2 * y2 + x2 * x2 * z2 * z2 + y2 * y2 * z2 * z2;
    const double s422 = x2 * y2 * z2 * (x2 + y2 + z2);
    const double r4 = r2 * r2, r7 = r4 * r2 * r, r13 = r7 * r4 * r2;
    return -1.0 / (4.0 * M_PI * r) + (3.0 * r4 - 5.0 * s4) / (32.0 * M_PI * r7) -
           (23.0 * s8 - 244.0 * s62 + 621.0 * s44 - 228.0 * s422) / (128.0 * M_PI * r13);
}

// Dense table entry (n1, n2, n3) of G_L.
__global__ void k_lgf_contract(const double *__restrict__ bes, const double *__restrict__ wq, int nodes, int nb,
                               double T, int e1, int e2, int e3, double *__restrict__ out) {
    const size_t total = (size_t)(e1 + 1) * (e2 + 1) * (e3 + 1);
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int n1 = (int)(idx % (e1 + 1));
    const int n2 = (int)((idx / (e1 + 1)) % (e2 + 1));
    const int n3 = (int)(idx / ((size_t)(e1 + 1) * (e2 + 1)));
    const int m = max(n1, max(n2, n3));
    if (m > kQuadRadius) {
        out[idx] = lgf_far(n1, n2, n3);
        return;
    }
    // compensated (Kahan-Babuska) sum of a positive integrand
    double s = 0.0, c = 0.0;
    for (int j = 0; j < nodes; ++j) {
        const double *bj = bes + (size_t)j * nb;
        const double v = wq[j] * bj[n1] * bj[n2] * bj[n3];
        const double t = s + v;
        c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
        s = t;
    }
    // tail on [T, inf): prod_q (4 pi t)^{-1/2} sum_k a_k(n_q) (2t)^{-k}
    //   = (4 pi t)^{-3/2} sum_K A_K (2t)^{-K};  int_T^inf -> T^{-K-1/2}/(K+1/2)
    constexpr int K = 6;
    double a1[K + 1], a2[K + 1], a3[K + 1];
    hankel_coeffs(n1, a1, K);
    hankel_coeffs(n2, a2, K);
    hankel_coeffs(n3, a3, K);
    double tail = 0.0, p2t = 1.0;
    const double inv2T = 1.0 / (2.0 * T);
    for (int k = 0; k <= K; ++k) {
        double A = 0.0;
        for (int i = 0; i <= k; ++i)
            for (int j = 0; i + j <= k; ++j) A += a1[i] * a2[j] * a3[k - i - j];
        tail += A * p2t / (k + 0.5);
        p2t *= inv2T;
    }
    tail *= pow(4.0 * M_PI, -1.5) / sqrt(T);
    out[idx] = -((s + c) + tail);
}

// Adds R(a)(n) = int_0^a prod g dt to entries with max n <= kRRadius.
__global__ void k_r_contract(const double *__restrict__ bes, const double *__restrict__ wq, int nodes, int nb,
                             int e1, int e2, int e3, double *__restrict__ out) {
    const size_t total = (size_t)(e1 + 1) * (e2 + 1) * (e3 + 1);
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int n1 = (int)(idx % (e1 + 1));
    const int n2 = (int)((idx / (e1 + 1)) % (e2 + 1));
    const int n3 = (int)(idx / ((size_t)(e1 + 1) * (e2 + 1)));
    if (max(n1, max(n2, n3)) > kRRadius) return;
    double s = 0.0, c = 0.0;
    for (int j = 0; j < nodes; ++j) {
        const double *bj = bes + (size_t)j * nb;
        const double v = wq[j] * bj[n1] * bj[n2] * bj[n3];
        const double t = s + v;
        c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
        s = t;
    }
    out[idx] += s + c;
}

// ------------------------------------------------------ kernel spectra
//
// On a box of N cells per axis padded to P = 2N, the circulant embedding of an
// even kernel g has a real, even DFT:
//   ghat(k) = g(0) + 2 sum_{n=1}^{N-1} g(n) cos(2 pi k n / P) + g(N) cos(pi k),
// separable over the axes.  One pass per axis, one thread per output value.

// in: [d2][d1][d0_in] (d0 fastest), out: [d2][d1][d0_out]; transform along the
// fastest axis of length Nin (entries n >= valid are treated as zero).
__global__ void k_cos_axis0(const double *__restrict__ in, int d0_in, int valid, int d1, int d2, int Nh,
                            const double *__restrict__ ctab, int P, double *__restrict__ out, int d0_out) {
    const size_t total = (size_t)d0_out * d1 * d2;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int k = (int)(idx % d0_out);
    const size_t row = idx / d0_out;
    if (k > Nh) {
        out[idx] = 0.0;
        return;
    }
    const double *src = in + row * d0_in;
    const int nmax = min(Nh, valid - 1);
    double s = 0.0;
    int ph = 0;
    for (int n = 0; n <= nmax; ++n) {
        const double cw = (n == 0 || n == Nh) ? 1.0 : 2.0;
        s += cw * src[n] * ctab[ph];
        ph += k;
        if (ph >= P) ph -= P;
    }
    out[idx] = s;
}

// Transform along a strided (non-fastest) axis: in/out indexed
// [outer][n][inner]; n runs over the transformed axis.
__global__ void k_cos_axis_strided(const double *__restrict__ in, int n_in, int valid, int inner, int outer, int Nh,
                                   const double *__restrict__ ctab, int P, double *__restrict__ out, int n_out) {
    const size_t total = (size_t)inner * n_out * outer;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int i = (int)(idx % inner);
    const int k = (int)((idx / inner) % n_out);
    const size_t o = idx / ((size_t)inner * n_out);
    const double *src = in + o * (size_t)n_in * inner + i;
    const int nmax = min(Nh, valid - 1);
    double s = 0.0;
    int ph = 0;
    for (int n = 0; n <= nmax; ++n) {
        const double cw = (n == 0 || n == Nh) ? 1.0 : 2.0;
        s += cw * src[(size_t)n * inner] * ctab[ph];
        ph += k;
        if (ph >= P) ph -= P;
    }
    out[idx] = s;
}

__global__ void k_to_float(const double *__restrict__ in, float *__restrict__ out, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

static unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int bessel_weights_host(double x, int nmax, std::vector<double> &out, hipStream_t s) {
    DevBuf t, b;
    int rc;
    if ((rc = t.reserve(sizeof(double)))) return rc;
    if ((rc = b.reserve(sizeof(double) * (nmax + 1)))) return rc;
    double hx = 0.5 * x;   // kernel evaluates at 2 t
    LGF_HIP(hipMemcpyAsync(t.p, &hx, sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bessel_nodes, dim3(1), dim3(1), 0, s, t.as<double>(), 1, nmax, b.as<double>());
    LGF_HIP(hipGetLastError());
    out.resize(nmax + 1);
    LGF_HIP(hipMemcpyAsync(out.data(), b.p, sizeof(double) * (nmax + 1), hipMemcpyDeviceToHost, s));
    LGF_HIP(hipStreamSynchronize(s));
    return LGFIB_OK;
}

static int build_table(Table &tb, hipStream_t s) {
    const int e1 = tb.ext[0], e2 = tb.ext[1], e3 = tb.ext[2];
    const size_t total = (size_t)(e1 + 1) * (e2 + 1) * (e3 + 1);
    int rc;
    if ((rc = tb.g.reserve(total * sizeof(double)))) return rc;
    const int nq = std::min(std::max(e1, std::max(e2, e3)), kQuadRadius);
    const double T = std::max(1.0e8, 1000.0 * nq * nq);
    std::vector<double> t, w;
    lgf_nodes(T, t, w);
    DevBuf dt, dw, db;
    const int nodes = (int)t.size(), nb = nq + 1;
    if ((rc = dt.reserve(nodes * sizeof(double)))) return rc;
    if ((rc = dw.reserve(nodes * sizeof(double)))) return rc;
    if ((rc = db.reserve((size_t)nodes * nb * sizeof(double)))) return rc;
    LGF_HIP(hipMemcpyAsync(dt.p, t.data(), nodes * sizeof(double), hipMemcpyHostToDevice, s));
    LGF_HIP(hipMemcpyAsync(dw.p, w.data(), nodes * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bessel_nodes, dim3(nblk(nodes, 64)), dim3(64), 0, s, dt.as<double>(), nodes, nq,
                       db.as<double>());
    LGF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lgf_contract, dim3(nblk(total)), dim3(256), 0, s, db.as<double>(), dw.as<double>(), nodes,
                       nb, T, e1, e2, e3, tb.g.as<double>());
    LGF_HIP(hipGetLastError());
    if (tb.kind == LGF_KIND_K && tb.alpha > 0.0) {
        const int nr = std::min(std::max(e1, std::max(e2, e3)), kRRadius);
        std::vector<double> rt, rw;
        r_nodes(tb.alpha, rt, rw);
        DevBuf rdt, rdw, rdb;
        const int rn = (int)rt.size();
        if ((rc = rdt.reserve(rn * sizeof(double)))) return rc;
        if ((rc = rdw.reserve(rn * sizeof(double)))) return rc;
        if ((rc = rdb.reserve((size_t)rn * (nr + 1) * sizeof(double)))) return rc;
        LGF_HIP(hipMemcpyAsync(rdt.p, rt.data(), rn * sizeof(double), hipMemcpyHostToDevice, s));
        LGF_HIP(hipMemcpyAsync(rdw.p, rw.data(), rn * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_bessel_nodes, dim3(nblk(rn, 64)), dim3(64), 0, s, rdt.as<double>(), rn, nr,
                           rdb.as<double>());
        LGF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_r_contract, dim3(nblk(total)), dim3(256), 0, s, rdb.as<double>(), rdw.as<double>(), rn,
                           nr + 1, e1, e2, e3, tb.g.as<double>());
        LGF_HIP(hipGetLastError());
        LGF_HIP(hipStreamSynchronize(s));
    }
    LGF_HIP(hipStreamSynchronize(s));
    return LGFIB_OK;
}

int get_spectrum(lgfib_ctx *ctx, lgf_table_t tbl, const BoxPlan &plan, int prec, hipStream_t s,
                 std::shared_ptr<Spectrum> &out) {
    auto key = std::make_tuple((int)tbl, plan.P[0], plan.P[1], plan.P[2], prec);
    auto it = ctx->spectra.find(key);
    if (it != ctx->spectra.end()) {
        it->second.tick = ++ctx->cache_tick;
        out = it->second.v;
        return LGFIB_OK;
    }
    const Table &tb = *ctx->tables[tbl];
    const int N0 = plan.N[0], N1 = plan.N[1], N2 = plan.N[2];
    const int Kxp = plan.Kxp;
    // valid entries per axis (n beyond the table is never reached by a
    // source/target pair inside the box, so it may be taken as zero)
    const int v0 = std::min(tb.ext[0] + 1, N0 + 1), v1 = std::min(tb.ext[1] + 1, N1 + 1),
              v2 = std::min(tb.ext[2] + 1, N2 + 1);
    int rc;
    // cosine tables per axis
    // cos(2 pi m / P) with the angle reduced to [0, pi/2] by symmetry
    auto ctab = [&](int P, std::vector<double> &c) {
        c.resize(P);
        for (int m = 0; m < P; ++m) {
            const int mm = std::min(m, P - m);   // cos is even
            c[m] = (4 * mm <= P) ? cos(2.0 * M_PI * mm / P) : -cos(2.0 * M_PI * (P / 2 - mm) / P);
        }
    };
    std::vector<double> c0, c1, c2;
    ctab(plan.P[0], c0);
    ctab(plan.P[1], c1);
    ctab(plan.P[2], c2);
    DevBuf dc0, dc1, dc2, A, Bf;
    if ((rc = dc0.reserve(c0.size() * 8))) return rc;
    if ((rc = dc1.reserve(c1.size() * 8))) return rc;
    if ((rc = dc2.reserve(c2.size() * 8))) return rc;
    LGF_HIP(hipMemcpyAsync(dc0.p, c0.data(), c0.size() * 8, hipMemcpyHostToDevice, s));
    LGF_HIP(hipMemcpyAsync(dc1.p, c1.data(), c1.size() * 8, hipMemcpyHostToDevice, s));
    LGF_HIP(hipMemcpyAsync(dc2.p, c2.data(), c2.size() * 8, hipMemcpyHostToDevice, s));
    // pass 0: table [v2][v1][ext0+1] -> A [v2][v1][Kxp]; the table rows have
    // stride ext0+1, and only planes/rows below v2/v1 are read.
    // (rows beyond v1/v2 are zero and are handled by the later passes' valid)
    const size_t nA = (size_t)(N2 + 1) * (N1 + 1) * Kxp;
    if ((rc = A.reserve(nA * 8))) return rc;
    if ((rc = Bf.reserve(nA * 8))) return rc;
    // step 0: gather table rows into A0 [v2][v1][ext0+1] is the table itself
    // when v1 == ext1+1; to keep strides simple we transform row by row of the
    // table and then pick rows.
    {
        // transform all rows of the table along axis 0 into Bf laid out
        // [e3+1][e2+1][Kxp] if it fits, else do it in the needed sub-box
        const int t1 = tb.ext[1] + 1, t2 = tb.ext[2] + 1;
        DevBuf T0;
        const size_t nT0 = (size_t)v2 * v1 * Kxp;
        if ((rc = T0.reserve(nT0 * 8))) return rc;
        // rows (n2 < v1, n3 < v2) of the table: launch per plane n3 to honour
        // the table's row stride (t1 rows per plane)
        for (int n3 = 0; n3 < v2; ++n3) {
            const double *src = tb.g.as<double>() + (size_t)n3 * t1 * (tb.ext[0] + 1);
            double *dst = T0.as<double>() + (size_t)n3 * v1 * Kxp;
            hipLaunchKernelGGL(k_cos_axis0, dim3(nblk((size_t)Kxp * v1)), dim3(256), 0, s, src, tb.ext[0] + 1, v0,
                               v1, 1, N0, dc0.as<double>(), plan.P[0], dst, Kxp);
        }
        LGF_HIP(hipGetLastError());
        (void)t2;
        // pass 1 (axis 1): T0 [v2][v1][Kxp] -> A [v2][N1+1][Kxp]
        hipLaunchKernelGGL(k_cos_axis_strided, dim3(nblk((size_t)Kxp * (N1 + 1) * v2)), dim3(256), 0, s,
                           T0.as<double>(), v1, v1, Kxp, v2, N1, dc1.as<double>(), plan.P[1], A.as<double>(), N1 + 1);
        LGF_HIP(hipGetLastError());
        // pass 2 (axis 2): A [v2][N1+1][Kxp] viewed as [1][v2][(N1+1) Kxp] -> Bf [N2+1][(N1+1) Kxp]
        hipLaunchKernelGGL(k_cos_axis_strided, dim3(nblk((size_t)Kxp * (N1 + 1) * (N2 + 1))), dim3(256), 0, s,
                           A.as<double>(), v2, v2, Kxp * (N1 + 1), 1, N2, dc2.as<double>(), plan.P[2],
                           Bf.as<double>(), N2 + 1);
        LGF_HIP(hipGetLastError());
        LGF_HIP(hipStreamSynchronize(s));
    }
    auto sp = std::make_shared<Spectrum>();
    sp->prec = prec;
    sp->Kxp = Kxp;
    for (int a = 0; a < 3; ++a) sp->P[a] = plan.P[a];
    if (prec == LGF_F64) {
        if ((rc = sp->ghat.reserve(nA * 8))) return rc;
        LGF_HIP(hipMemcpyAsync(sp->ghat.p, Bf.p, nA * 8, hipMemcpyDeviceToDevice, s));
    } else {
        if ((rc = sp->ghat.reserve(nA * 4))) return rc;
        hipLaunchKernelGGL(k_to_float, dim3(nblk(nA)), dim3(256), 0, s, Bf.as<double>(), sp->ghat.as<float>(), nA);
        LGF_HIP(hipGetLastError());
    }
    LGF_HIP(hipStreamSynchronize(s));
    out = sp;
    const size_t sp_bytes = sp->ghat.bytes;
    ctx->spectra[key] = CacheEnt<Spectrum>{std::move(sp), ++ctx->cache_tick, sp_bytes};
    cache_trim_all(ctx, 1);
    return LGFIB_OK;
}

}  // namespace lgfib

using namespace lgfib;

extern "C" int lgf_table_build(lgfib_ctx *ctx, int kind, double alpha, const int32_t extent[3],
                               lgfib_stream_t stream, lgf_table_t *out) {
    if (!ctx || !extent || !out) return fail(LGFIB_EINVAL, "lgf_table_build: null argument");
    if (kind != LGF_KIND_L && kind != LGF_KIND_K) return fail(LGFIB_EINVAL, "lgf_table_build: unknown kind");
    if (!(alpha >= 0.0) || alpha > 4.0)
        return fail(LGFIB_EINVAL, "lgf_table_build: alpha must lie in [0, 4]");
    if (kind == LGF_KIND_L && alpha != 0.0)
        return fail(LGFIB_EINVAL, "lgf_table_build: alpha must be 0 for LGF_KIND_L");
    for (int a = 0; a < 3; ++a)
        if (extent[a] < 0 || extent[a] > 4096) return fail(LGFIB_EINVAL, "lgf_table_build: extent out of [0, 4096]");
    LGF_HIP(hipSetDevice(ctx->device));
    for (size_t i = 0; i < ctx->tables.size(); ++i) {
        const Table &t = *ctx->tables[i];
        if (t.kind == kind && t.alpha == alpha && t.ext[0] == extent[0] && t.ext[1] == extent[1] &&
            t.ext[2] == extent[2]) {
            *out = (lgf_table_t)i;
            return LGFIB_OK;
        }
    }
    auto tb = std::make_unique<Table>();
    tb->kind = kind;
    tb->alpha = alpha;
    for (int a = 0; a < 3; ++a) tb->ext[a] = extent[a];
    int rc = build_table(*tb, (hipStream_t)stream);
    if (rc) return rc;
    ctx->tables.push_back(std::move(tb));
    *out = (lgf_table_t)(ctx->tables.size() - 1);
    return LGFIB_OK;
}

extern "C" int lgf_table_upload(lgfib_ctx *ctx, const int32_t extent[3], const double *host_src, int64_t count,
                                lgf_table_t *out) {
    if (!ctx || !extent || !host_src || !out) return fail(LGFIB_EINVAL, "lgf_table_upload: null argument");
    for (int a = 0; a < 3; ++a)
        if (extent[a] < 0 || extent[a] > 4096) return fail(LGFIB_EINVAL, "lgf_table_upload: extent out of [0, 4096]");
    const int64_t n = (int64_t)(extent[0] + 1) * (extent[1] + 1) * (extent[2] + 1);
    if (count != n) return fail(LGFIB_EINVAL, "lgf_table_upload: count must be " + std::to_string(n));
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host_src[i])) return fail(LGFIB_EINVAL, "lgf_table_upload: non-finite value");
    LGF_HIP(hipSetDevice(ctx->device));
    auto tb = std::make_unique<Table>();
    tb->kind = LGF_KIND_USER;
    for (int a = 0; a < 3; ++a) tb->ext[a] = extent[a];
    int rc = tb->g.reserve((size_t)n * sizeof(double));
    if (rc) return rc;
    LGF_HIP(hipMemcpy(tb->g.p, host_src, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
    ctx->tables.push_back(std::move(tb));
    *out = (lgf_table_t)(ctx->tables.size() - 1);
    return LGFIB_OK;
}

extern "C" int lgf_table_copy(lgfib_ctx *ctx, lgf_table_t tbl, double *host_dst, int64_t count) {
    if (!ctx || !host_dst) return fail(LGFIB_EINVAL, "lgf_table_copy: null argument");
    if (tbl < 0 || (size_t)tbl >= ctx->tables.size()) return fail(LGFIB_ENOTBUILT, "lgf_table_copy: unknown table");
    const Table &t = *ctx->tables[tbl];
    const int64_t n = (int64_t)(t.ext[0] + 1) * (t.ext[1] + 1) * (t.ext[2] + 1);
    if (count != n) return fail(LGFIB_EINVAL, "lgf_table_copy: count must be " + std::to_string(n));
    LGF_HIP(hipSetDevice(ctx->device));
    LGF_HIP(hipMemcpy(host_dst, t.g.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    return LGFIB_OK;
}

extern "C" int lgf_if_weights(lgfib_ctx *ctx, double a, double cutoff, double *w, int wmax, int *radius) {
    if (!ctx || !radius) return fail(LGFIB_EINVAL, "lgf_if_weights: null argument");
    if (!(a >= 0.0) || a > 64.0) return fail(LGFIB_EINVAL, "lgf_if_weights: a must lie in [0, 64]");
    if (!(cutoff > 0.0) || cutoff >= 1.0) return fail(LGFIB_EINVAL, "lgf_if_weights: cutoff must lie in (0, 1)");
    LGF_HIP(hipSetDevice(ctx->device));
    std::vector<double> v;
    int nmax = 32;
    for (;;) {
        int rc = bessel_weights_host(2.0 * a, nmax, v, nullptr);
        if (rc) return rc;
        int r = -1;
        for (int j = 0; j <= nmax; ++j)
            if (v[j] < cutoff) {
                r = j - 1;
                break;
            }
        if (r >= 0 || (a == 0.0)) {
            if (a == 0.0) r = 0;
            *radius = r;
            if (w && wmax > r)
                for (int j = 0; j <= r; ++j) w[j] = v[j];
            return LGFIB_OK;
        }
        nmax *= 2;
        if (nmax > 4096) return fail(LGFIB_ERANGE, "lgf_if_weights: kernel wider than 4096");
    }
}
