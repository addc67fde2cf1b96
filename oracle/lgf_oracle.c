/*
 * lgf_oracle.c -- plain, slow FP64 reference for the lattice Green's function
 * (LGF) immersed-boundary hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * What it computes (Liska & Colonius, "A fast immersed boundary method for
 * external incompressible viscous flows using lattice Green's functions"):
 *
 *   - the scaled modified Bessel function  g_n(x) = exp(-x) I_n(x): ascending
 *     power series for x <= 64; the integral representation
 *     I_n(x) = (1/pi) int_0^pi exp(x cos th) cos(n th) dth by the periodic
 *     trapezoid rule (geometric convergence) for moderate x; the classical
 *     large-argument (Hankel) series when x >> n^2;
 *   - the 1D integrating-factor weights e^{-2a} I_j(2a), whose product over the
 *     three axes is the LGF of E(a) = exp(aL)            (App. A, Eq. lgf_intfac);
 *   - the LGF of the 7-point Laplacian, G_L(n) = - int_0^inf prod_q g_{n_q}(2t) dt
 *     (App. A, Eq. lgf_lap), by a double-exponential (exp-sinh) quadrature in t;
 *   - R(a)(n) = int_0^a prod_q g_{n_q}(2t) dt by adaptive Gauss-Kronrod (7/15),
 *     so that G_K(a) = G_L + R(a)                         (App. A, partition of G_K);
 *   - the discrete convolution u(n) = sum_m K(n - m) f(m) (Sec. 2.2,
 *     Eq. dpoisson_conv) by direct summation with Neumaier compensation.
 *
 * Lattice units (dx = 1) throughout; callers scale by dx^2 where the paper does.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------- */
/* Scaled modified Bessel functions g_n(x) = e^{-x} I_n(x), n = 0..nmax.      */
/* ------------------------------------------------------------------------- */

/* Large-argument series (Abramowitz & Stegun 9.7.1):
 *   e^{-x} I_n(x) ~ (2 pi x)^{-1/2} sum_k (-1)^k prod_{j=1..k}(4n^2-(2j-1)^2) / (k! (8x)^k)
 * used only when x >= 50 n^2 + 1000, where the terms fall by >= 100x per step
 * and the exponentially small companion term e^{-2x} is far below rounding. */
static double hankel_scaled(int n, double x)
{
    double mu = 4.0 * (double)n * (double)n;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 60; ++k) {
        double c = (mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (k * 8.0 * x);
        term *= -c;
        sum += term;
        if (fabs(term) < 1e-19 * fabs(sum)) break;
    }
    return sum / sqrt(2.0 * OR_PI * x);
}

/* Ascending series (Abramowitz & Stegun 9.6.10):
 *   I_n(x) = sum_k (x/2)^{2k+n} / (k! (n+k)!)
 * all terms positive, so every order keeps its relative accuracy; used for
 * x <= 64, where it converges in under ~120 terms. */
static double series_scaled(int n, double x)
{
    double h = 0.5 * x;
    double lt = (double)n * log(h) - lgamma((double)n + 1.0) - x;
    if (lt < -745.0) return 0.0;
    double term = exp(lt), sum = term;
    for (int k = 0; k < 400; ++k) {
        term *= h * h / ((double)(k + 1) * (double)(k + 1 + n));
        sum += term;
        if (term < 1e-19 * sum) break;
    }
    return sum;
}

static int hankel_ok(int nmax, double x)
{
    return x >= 50.0 * (double)nmax * (double)nmax + 1000.0;
}

/* Fill out[0..nmax] with e^{-x} I_n(x), x >= 0. */
void oracle_bessel_scaled_vec(double x, int nmax, double *out)
{
    if (x == 0.0) {
        out[0] = 1.0;
        for (int n = 1; n <= nmax; ++n) out[n] = 0.0;
        return;
    }
    if (x <= 64.0) {
        for (int n = 0; n <= nmax; ++n) out[n] = series_scaled(n, x);
        return;
    }
    if (hankel_ok(nmax, x)) {
        for (int n = 0; n <= nmax; ++n) out[n] = hankel_scaled(n, x);
        return;
    }
    /* Trapezoid rule on the full period of exp(x(cos th - 1)) cos(n th).
     * It returns sum_k g_{n+kM}(x); M is chosen so g_{M-nmax}(x) < 1e-18.
     * The integrand is even about th = pi, so only th_j = 2 pi j / M for
     * j = 0..M/2 is evaluated (doubling the interior nodes): near th = 2 pi
     * the half-angle sine would lose its relative accuracy, and x amplifies
     * that loss in the exponent. */
    int M = nmax + (int)ceil(sqrt(83.0 * x)) + 24;
    if (M & 1) ++M;
    int H = M / 2;
    double *E = (double *)malloc(sizeof(double) * (size_t)(H + 1));
    double *C = (double *)malloc(sizeof(double) * (size_t)M);
    for (int j = 0; j < M; ++j) C[j] = cos(2.0 * OR_PI * (double)j / (double)M);
    for (int j = 0; j <= H; ++j) {
        double sh = sin(OR_PI * (double)j / (double)M);
        double w = (j == 0 || j == H) ? 1.0 : 2.0;
        E[j] = w * exp(-2.0 * x * sh * sh); /* x (cos th - 1) without cancellation */
    }
    for (int n = 0; n <= nmax; ++n) {
        /* cos(n th_j) = C[(n j) mod M]: exact index arithmetic, no recurrence */
        double s = 0.0, comp = 0.0;
        long long idx = 0;
        for (int j = 0; j <= H; ++j) {
            double v = E[j] * C[idx];
            double t = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - t) + v; else comp += (v - t) + s;
            s = t;
            idx += n;
            if (idx >= M) idx %= M;
        }
        out[n] = (s + comp) / (double)M;
    }
    free(E);
    free(C);
}

double oracle_bessel_scaled(int n, double x)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    oracle_bessel_scaled_vec(x, n, v);
    double r = v[n];
    free(v);
    return r;
}

/* 1D integrating-factor weights w[j] = e^{-2a} I_j(2a), j = 0..rmax. */
void oracle_if_factors(double a, int rmax, double *w)
{
    oracle_bessel_scaled_vec(2.0 * a, rmax, w);
}

/* ------------------------------------------------------------------------- */
/* LGF of the 7-point Laplacian by exp-sinh quadrature in t.                  */
/* ------------------------------------------------------------------------- */

/* Dense even table G[n3][n2][n1] for 0 <= n1 <= e1, 0 <= n2 <= e2, 0 <= n3 <= e3
 * (so out has (e1+1)(e2+1)(e3+1) doubles, n1 fastest).
 *
 * G(n) = - int_0^inf prod_q g_{n_q}(2t) dt, with t = exp((pi/2) sinh u),
 * dt = (pi/2) cosh(u) t du, trapezoid in u with step h on |u| <= 4.7.  The
 * transformed integrand decays double-exponentially at both ends (it behaves
 * like t near t = 0 and like t^{-1/2} as t -> inf).  h = 1/128 is the default.
 *
 * The LGF is invariant under permutation and sign changes of n, so only sorted
 * triples n1 >= n2 >= n3 >= 0 are integrated and then copied out.
 * Returns 0 on success. */
int oracle_lgf_table(int e1, int e2, int e3, double h, double *out)
{
    if (e1 < 0 || e2 < 0 || e3 < 0 || !(h > 0.0)) return -1;
    int nmax = e1;
    if (e2 > nmax) nmax = e2;
    if (e3 > nmax) nmax = e3;
    const double U = 4.7;
    int K = (int)ceil(U / h);
    int nodes = 2 * K + 1;
    double *wt = (double *)malloc(sizeof(double) * (size_t)nodes);
    double *bes = (double *)malloc(sizeof(double) * (size_t)nodes * (size_t)(nmax + 1));
    if (!wt || !bes) { free(wt); free(bes); return -2; }

#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < nodes; ++k) {
        double u = (double)(k - K) * h;
        double t = exp(0.5 * OR_PI * sinh(u));
        wt[k] = h * 0.5 * OR_PI * cosh(u) * t;
        oracle_bessel_scaled_vec(2.0 * t, nmax, bes + (size_t)k * (size_t)(nmax + 1));
    }

    /* sorted triples a >= b >= c, each bounded by nmax */
    size_t nn = (size_t)(nmax + 1);
    size_t stride2 = (size_t)(e1 + 1), stride3 = (size_t)(e1 + 1) * (size_t)(e2 + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a <= nmax; ++a) {
        for (int b = 0; b <= a; ++b) {
            for (int c = 0; c <= b; ++c) {
                /* is any permutation of (a,b,c) inside the requested box? */
                int p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
                int need = 0;
                for (int q = 0; q < 6; ++q)
                    if (p[q][0] <= e1 && p[q][1] <= e2 && p[q][2] <= e3) need = 1;
                if (!need) continue;
                double s = 0.0, comp = 0.0;
                for (int k = 0; k < nodes; ++k) {
                    const double *bk = bes + (size_t)k * nn;
                    double v = wt[k] * bk[a] * bk[b] * bk[c];
                    double tt = s + v;
                    if (fabs(s) >= fabs(v)) comp += (s - tt) + v; else comp += (v - tt) + s;
                    s = tt;
                }
                double g = -(s + comp);
                for (int q = 0; q < 6; ++q)
                    if (p[q][0] <= e1 && p[q][1] <= e2 && p[q][2] <= e3)
                        out[(size_t)p[q][2] * stride3 + (size_t)p[q][1] * stride2 + (size_t)p[q][0]] = g;
            }
        }
    }
    free(wt);
    free(bes);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* R(a)(n) = int_0^a prod_q g_{n_q}(2t) dt by adaptive Gauss-Kronrod 7/15.    */
/* ------------------------------------------------------------------------- */

/* Kronrod 15-point nodes/weights and embedded Gauss 7-point weights
 * (standard published values, e.g. QUADPACK's qk15). */
static const double gk_x[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double gk_wk[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double gk_wg[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

static double r_integrand(const int n[3], double t)
{
    int m = n[0];
    if (n[1] > m) m = n[1];
    if (n[2] > m) m = n[2];
    double *v = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    oracle_bessel_scaled_vec(2.0 * t, m, v);
    double r = v[n[0]] * v[n[1]] * v[n[2]];
    free(v);
    return r;
}

static double gk15(const int n[3], double a, double b, double *err)
{
    double c = 0.5 * (a + b), hl = 0.5 * (b - a);
    double fc = r_integrand(n, c);
    double rk = fc * gk_wk[7], rg = fc * gk_wg[3];
    for (int j = 0; j < 7; ++j) {
        double dx = hl * gk_x[j];
        double f1 = r_integrand(n, c - dx), f2 = r_integrand(n, c + dx);
        rk += gk_wk[j] * (f1 + f2);
        if (j & 1) rg += gk_wg[j / 2] * (f1 + f2);
    }
    *err = fabs((rk - rg) * hl);
    return rk * hl;
}

static double gk_adapt(const int n[3], double a, double b, double tol, int depth)
{
    double err;
    double r = gk15(n, a, b, &err);
    if (err <= tol || depth >= 40) return r;
    double m = 0.5 * (a + b);
    return gk_adapt(n, a, m, 0.5 * tol, depth + 1) + gk_adapt(n, m, b, 0.5 * tol, depth + 1);
}

/* Dense even table R[n3][n2][n1] for 0 <= n_i <= e_i; entries with
 * max(n) > rcut are set to zero (R decays faster than any exponential;
 * the caller picks rcut so that the dropped values are below rounding). */
int oracle_lgf_r_table(double alpha, int e1, int e2, int e3, int rcut, double *out)
{
    if (alpha < 0.0 || e1 < 0 || e2 < 0 || e3 < 0) return -1;
    size_t stride2 = (size_t)(e1 + 1), stride3 = (size_t)(e1 + 1) * (size_t)(e2 + 1);
    size_t total = stride3 * (size_t)(e3 + 1);
    memset(out, 0, sizeof(double) * total);
    if (alpha == 0.0) return 0;
    int nmax = e1;
    if (e2 > nmax) nmax = e2;
    if (e3 > nmax) nmax = e3;
    if (rcut < nmax) nmax = rcut;
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a <= nmax; ++a) {
        for (int b = 0; b <= a; ++b) {
            for (int c = 0; c <= b; ++c) {
                int p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
                int need = 0;
                for (int q = 0; q < 6; ++q)
                    if (p[q][0] <= e1 && p[q][1] <= e2 && p[q][2] <= e3) need = 1;
                if (!need) continue;
                int n[3] = {a, b, c};
                double r = gk_adapt(n, 0.0, alpha, 1e-19, 0);
                for (int q = 0; q < 6; ++q)
                    if (p[q][0] <= e1 && p[q][1] <= e2 && p[q][2] <= e3)
                        out[(size_t)p[q][2] * stride3 + (size_t)p[q][1] * stride2 + (size_t)p[q][0]] = r;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Direct-sum discrete convolution u(n) = sum_m K(n - m) f(m).                */
/* ------------------------------------------------------------------------- */

/* Kernel is an even dense table K[k3][k2][k1], |d_i| <= ke_i (n1 fastest),
 * taken as zero outside.  Sources: ns cells (int32 xyz triples) with values
 * f[ns]; targets: nt cells.  u[nt] is overwritten.  Neumaier-compensated sum,
 * OpenMP over targets.  Sources with f == 0 are skipped (they add nothing). */
int oracle_conv_direct(const double *ktab, int ke1, int ke2, int ke3,
                       const int32_t *src, const double *f, long long ns,
                       const int32_t *tgt, long long nt, double *u)
{
    if (ke1 < 0 || ke2 < 0 || ke3 < 0 || ns < 0 || nt < 0) return -1;
    size_t s2 = (size_t)(ke1 + 1), s3 = (size_t)(ke1 + 1) * (size_t)(ke2 + 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (long long i = 0; i < nt; ++i) {
        int tx = tgt[3 * i], ty = tgt[3 * i + 1], tz = tgt[3 * i + 2];
        double s = 0.0, comp = 0.0;
        for (long long j = 0; j < ns; ++j) {
            double fj = f[j];
            if (fj == 0.0) continue;
            int dx = abs(tx - src[3 * j]), dy = abs(ty - src[3 * j + 1]), dz = abs(tz - src[3 * j + 2]);
            if (dx > ke1 || dy > ke2 || dz > ke3) continue;
            double v = ktab[(size_t)dz * s3 + (size_t)dy * s2 + (size_t)dx] * fj;
            double t = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - t) + v; else comp += (v - t) + s;
            s = t;
        }
        u[i] = s + comp;
    }
    return 0;
}

/* Windowed direct sum for a compactly supported even kernel (|d_i| <= r_i)
 * over a dense source box f[nz][ny][nx] (x fastest) whose cell (0,0,0) sits at
 * lattice point org.  Targets are lattice points; sources outside the box are
 * zero.  Same compensated summation. */
int oracle_conv_window(const double *ktab, int r1, int r2, int r3,
                       const double *fbox, const int32_t org[3], int nx, int ny, int nz,
                       const int32_t *tgt, long long nt, double *u)
{
    if (r1 < 0 || r2 < 0 || r3 < 0 || nx < 0 || ny < 0 || nz < 0 || nt < 0) return -1;
    size_t s2 = (size_t)(r1 + 1), s3 = (size_t)(r1 + 1) * (size_t)(r2 + 1);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long i = 0; i < nt; ++i) {
        int tx = tgt[3 * i] - org[0], ty = tgt[3 * i + 1] - org[1], tz = tgt[3 * i + 2] - org[2];
        double s = 0.0, comp = 0.0;
        for (int dz = -r3; dz <= r3; ++dz) {
            int z = tz - dz;
            if (z < 0 || z >= nz) continue;
            for (int dy = -r2; dy <= r2; ++dy) {
                int y = ty - dy;
                if (y < 0 || y >= ny) continue;
                for (int dx = -r1; dx <= r1; ++dx) {
                    int x = tx - dx;
                    if (x < 0 || x >= nx) continue;
                    double v = ktab[(size_t)abs(dz) * s3 + (size_t)abs(dy) * s2 + (size_t)abs(dx)] *
                               fbox[((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x];
                    double t = s + v;
                    if (fabs(s) >= fabs(v)) comp += (s - t) + v; else comp += (v - t) + s;
                    s = t;
                }
            }
        }
        u[i] = s + comp;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
