/*
 * lgfib.h -- C ABI of the MI355X (gfx950) lattice-Green's-function library.
 *
 * The library evaluates, on one GPU, the operators that every projection step
 * and every viscous integrating-factor application of the immersed-boundary
 * LGF method of Liska & Colonius (arXiv:1604.01814) reduces to:
 *
 *   u = G * f     discrete convolution with the LGF of the 7-point Laplacian
 *                 on the active blocks of an unbounded grid (Sec. 2.2,
 *                 Eq. dpoisson_conv), or with the LGF of K = E(-a) L;
 *   u = E(a) f    the integrating factor exp(aL) (Sec. 2.3; its LGF is the
 *                 Bessel product of App. A, Eq. lgf_intfac);
 *   R, I          regularization / interpolation with a discrete delta
 *                 (Sec. 2.1);
 *   C f = r       the rigid-body force Schur complement (Sec. 3.1,
 *                 Eq. force_schur) solved by conjugate gradients (Sec. 3.2).
 *
 * Conventions shared by every entry point
 *   - Lattice units: a cell n in Z^3 has centre n + (1/2,1/2,1/2); its k-th
 *     face sits on the cell's lower k-side.  Grid spacing dx only scales.
 *   - Block sets are HOST arrays of int32 triples (bx, by, bz), one per block,
 *     each block covering cells b*B + [0,B)^3.  Coordinates must lie in
 *     [-2^20, 2^20) and be unique within a list (else LGFIB_EDUP_BLOCK).
 *     Lists may be in any order; results follow the caller's order.
 *   - Fields are DEVICE arrays owned by the caller, laid out
 *     [ncomp][nblk][B][B][B] with x fastest (element (c, i, z, y, x) at
 *     ((c*nblk + i)*B + z)*B*B + y*B + x), float (LGF_F32) or double (LGF_F64).
 *   - Every compute call is asynchronous on the given stream (a hipStream_t;
 *     NULL = the null stream).  Host arrays may be reused on return.
 *   - Return value: 0 on success, a negative LGFIB_E* code on error; then
 *     lgfib_last_error() (thread-local) describes it.  Nothing is launched
 *     when an argument check fails.  No C++ exception crosses the ABI.
 *   - A context is bound to one device; calls on one context must not
 *     overlap in time from several host threads.
 */
#ifndef LGFIB_H
#define LGFIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgfib_ctx lgfib_ctx;
typedef void *lgfib_stream_t;   /* hipStream_t */
typedef int32_t lgf_table_t;    /* handle of a table held by a context */

enum {
    LGFIB_OK = 0,
    LGFIB_EINVAL = -1,      /* bad argument (sizes, kinds, aliasing, null) */
    LGFIB_EDUP_BLOCK = -2,  /* a block appears twice in one list */
    LGFIB_ENOMEM = -3,      /* device or host allocation failed */
    LGFIB_ENOTBUILT = -4,   /* table handle unknown */
    LGFIB_ENOCONV = -5,     /* iterative solve stopped at maxit */
    LGFIB_EHIP = -6,        /* a HIP runtime call failed */
    LGFIB_ESUPPORT = -7,    /* a delta support leaves the block set */
    LGFIB_ERANGE = -8,      /* table extent smaller than the geometry needs */
    LGFIB_ENOTSPD = -9      /* a Cholesky pivot was not positive */
};

enum { LGF_KIND_L = 0, LGF_KIND_K = 1, LGF_KIND_USER = 2 };   /* G_L, G_K(a) = G_L + R(a), or uploaded */
enum { LGF_F32 = 0, LGF_F64 = 1 };
enum { IB_ROMA3 = 0, IB_SMOOTH3 = 1 };     /* discrete delta kernels */

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  It owns tables, spectra,
 * workspaces and plans, all freed by lgfib_destroy. */
int lgfib_create(lgfib_ctx **out, int device);
void lgfib_destroy(lgfib_ctx *ctx);
const char *lgfib_last_error(void);

/* Kernel timing (tracing aid).  With enable != 0 every kernel launched by the
 * convolution, integrating-factor and IB paths of this context is bracketed
 * by two HIP events recorded on the stream it is launched on.
 * lgfib_profile_read waits for the recorded events and reports, per kernel
 * name (at most max entries, names as NUL-terminated strings of up to 63
 * characters in names[64*i]), the launch count and the summed milliseconds
 * accumulated since the last lgfib_profile_reset.  *n receives the number of
 * distinct kernels. */
int lgfib_profile_enable(lgfib_ctx *ctx, int enable);
int lgfib_profile_reset(lgfib_ctx *ctx);
int lgfib_profile_read(lgfib_ctx *ctx, int max, char *names, int *counts, double *ms, int *n);

/* Plan caches.  The context caches, under the exact block lists or marker
 * positions they were made for, the box-FFT plans (at most 256), the
 * integrating-factor plans (256), the kernel spectra of box FFTs (64, within
 * 4 GiB of device memory) and of the block-pair form (8, within 8 GiB), the IB
 * operator plans I and R (64) and the curl-operator plans (64 of each
 * kind).  When a cache is full the least
 * recently used entry that no live batch, IB system, flow or HERK driver
 * holds is freed, so a moving body (new I and R every step) or an adapting
 * flow domain (Sec. 2.1, Sec. 4.1) does not grow memory without bound.
 * lgfib_cache_release frees every entry that nothing holds now (it waits for
 * the device first).  lgfib_cache_info writes the entry counts
 * out[0..5] = (box plans, IF plans, box spectra, pair spectra, IB plans,
 * curl plans) and out[6] = the number of trims that freed something.  Tables
 * (lgf_table_build) are handles and are not cached this way. */
int lgfib_cache_release(lgfib_ctx *ctx);
int lgfib_cache_info(lgfib_ctx *ctx, int64_t out[7]);

/* ----------------------------------------------------------------- tables */

/* Build the FP64 lattice Green's function on the device for every offset
 * 0 <= n_i <= extent[i] (the function is even in each axis), as in App. A:
 *   kind LGF_KIND_L:  G_L(n) = - int_0^inf prod_q e^{-2t} I_{n_q}(2t) dt
 *                     (Eq. lgf_lap), in lattice units (dx = 1);
 *   kind LGF_KIND_K:  G_K(a)(n) = G_L(n) + int_0^a prod_q e^{-2t} I_{n_q}(2t) dt
 *                     (the partition of G_K in App. A; K^{-1} = E(a) L^{-1}).
 * Computed once by Gauss-Legendre quadrature of the t-integral plus its
 * large-t asymptotic tail, with the far-field expansion of G_L for
 * max|n_i| > 256.  The result is cached in the context by (kind, alpha,
 * extent); *out receives the handle.  extent[i] in [0, 4096];
 * alpha >= 0 (must be 0 for LGF_KIND_L).  Synchronous with respect to
 * `stream`: on return the table is ready for work later on that stream. */
int lgf_table_build(lgfib_ctx *ctx, int kind, double alpha, const int32_t extent[3],
                    lgfib_stream_t stream, lgf_table_t *out);

/* Copy a built table to host memory (count = (e1+1)(e2+1)(e3+1) doubles,
 * layout [n3][n2][n1], n1 fastest).  Blocks until the copy has landed. */
int lgf_table_copy(lgfib_ctx *ctx, lgf_table_t tbl, double *host_dst, int64_t count);

/* Register a caller-supplied even kernel K(n) = host_src[|n3|][|n2|][|n1|]
 * (count = (e1+1)(e2+1)(e3+1) FP64 values, n1 fastest, copied before
 * return) as a table of kind LGF_KIND_USER.  Every convolution of Eq.
 * dpoisson_conv (Sec. 2.2) accepts it in place of G_L or G_K; entry points
 * that need G_L itself reject it.  Each call adds a new table. */
int lgf_table_upload(lgfib_ctx *ctx, const int32_t extent[3], const double *host_src, int64_t count,
                     lgf_table_t *out);

/* Cutoffs of the integrating-factor kernel used by lgf_if_apply: weights
 * below them are dropped (FP64 applies, FP32 applies). */
#define LGF_IF_CUTOFF_F64 1e-14
#define LGF_IF_CUTOFF_F32 0x1p-28

/* Half-width r of the integrating-factor kernel: the largest j with
 * e^{-2a} I_j(2a) >= cutoff (the 1D factor of Eq. lgf_intfac), and (if w is
 * not NULL and wmax > r) the weights w[0..r] in FP64. */
int lgf_if_weights(lgfib_ctx *ctx, double a, double cutoff, double *w, int wmax, int *radius);

/* ------------------------------------------------------------ convolutions */

/* u(n) = dx^2 * sum_{m in S} G(n - m) f(m)  for every cell n of the target
 * blocks, S the cells of the source blocks (Sec. 2.2, Eq. dpoisson_conv; the
 * dx^2 places G in physical units as in Eq. lgf_lap).  With a G_L table this
 * is the free-space solution of L u = f restricted to the targets; with a
 * G_K(a) table it is K^{-1} f = E(a) L^{-1} f.
 *   f: device [ncomp][nsrc][B^3], u: device [ncomp][ntgt][B^3], same prec.
 *   accumulate != 0 adds into u instead of overwriting it.
 *   B in {4, 8, 16, 32}; 1 <= ncomp <= 8; nsrc, ntgt >= 0 (nothing to do if
 *   either is 0, beyond zeroing u when accumulate == 0).
 *   f and u must not overlap.  The table extent must cover every offset
 *   between the blocks' bounding box corners, else LGFIB_ERANGE.
 * Evaluated exactly (no far-field approximation beyond the table's) by a
 * zero-padded FFT over the blocks' bounding box; spectra of the kernel are
 * cached per (table, box shape, prec). */
int lgf_poisson_apply(lgfib_ctx *ctx, lgf_table_t tbl, int B,
                      const int32_t *src_blocks, int nsrc,
                      const int32_t *tgt_blocks, int ntgt,
                      int ncomp, int prec, double dx,
                      const void *f, void *u, int accumulate, lgfib_stream_t stream);

/* u(n) = sum_{m in S} prod_q w[|n_q - m_q|] f(m), n in the target blocks:
 * the integrating factor E(a) = exp(aL) (Sec. 2.3, App. A Eq. lgf_intfac)
 * with w[j] = e^{-2a} I_j(2a) truncated where w < LGF_IF_CUTOFF_F64 = 1e-14
 * for LGF_F64 and w < LGF_IF_CUTOFF_F32 = 2^-28 for LGF_F32 (half-width from
 * lgf_if_weights with that cutoff;
 * in FP32 the dropped tail stays below the unit roundoff 2^-24 relative to
 * max |f|).  a = nu dt / dx^2 is dimensionless, a >= 0 (a = 0 copies).
 * Same layouts, limits and aliasing rule as lgf_poisson_apply. */
int lgf_if_apply(lgfib_ctx *ctx, double a, int B,
                 const int32_t *src_blocks, int nsrc,
                 const int32_t *tgt_blocks, int ntgt,
                 int ncomp, int prec, const void *f, void *u, lgfib_stream_t stream);

/* The nonlinear term in rotational form (Sec. 2.1: N~ approximates
 * (curl u) x u_a), out = (C u) x u_a with u_a = u + U, on the faces of the
 * blocks, u zero outside them (so u_a = U there).  The paper leaves the
 * stencil open; this one forms the products on the edges and averages them
 * to the faces:
 *   P_ij(m)   = w^(i)(m) (u_a^(j)(m) + u_a^(j)(m - e_k)) / 2,  w = C u,
 *   out^(k)(n) = sum_ij eps_kij (P_ij(n) + P_ij(n + e_j)) / 2,
 * k the third index of (i, j); the two averages are transposes of each
 * other, so sum u . out = 0 for U = 0 (the term does no work).  Face and
 * edge placement as for lgf_velocity_refresh; lattice units (divide by dx).
 *   u, out: device [3][nblk][B^3], FP32 or FP64 by prec, must not overlap
 *   (LGFIB_EINVAL).  blocks: host int32 [nblk][3] (duplicates give
 *   LGFIB_EDUP_BLOCK).  U: host double[3] or NULL (zero).  B in
 *   {4, 8, 16, 32}.  The neighbour table is cached in the context by the
 *   block list.  Asynchronous on stream. */
int lgf_lamb_vector(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, int prec,
                    const void *u, void *out, lgfib_stream_t stream);

/* Support of the flow for the adaptive flow domain (Sec. 4.1, Eq.
 * weight_fun): for each block B of the list, on device,
 *   mu[B] = max over the cells n of B of |w(n)|, w = C u (the three edge
 *           components of cell n as one vector, Euclidean norm),
 *   nu[B] = max over the cells n of B of |h(n)|, h = D-bar N~ the divergence
 *           of the nonlinear term of lgf_lamb_vector (frame velocity U),
 *           h(n) = sum_k N~^(k)(n + e_k) - N~^(k)(n).
 * u is zero outside the blocks; N~ is formed from u wherever the divergence
 * reads it, faces just outside the blocks included.
 *   u: device [3][nblk][B^3], FP32 or FP64 by prec.  mu, nu: device double
 *   [nblk].  blocks: host int32 [nblk][3] (duplicates give
 *   LGFIB_EDUP_BLOCK).  U: host double[3] or NULL.  B in {4, 8, 16, 32}.
 *   Asynchronous on stream. */
int lgf_block_support(lgfib_ctx *ctx, int B, const int32_t *blocks, int nblk, const double *U, int prec,
                      const void *u, double *mu, double *nu, lgfib_stream_t stream);

/* Block weights of Eq. weight_fun_modifer, host only:
 *   w[B] = 1 / max(eta, dist(pos(B))), pos(B) the block's centre in lattice
 *   units and dist the distance from it to the nearest of the NL points X
 *   (host double [NL][3]) divided by `length`.
 * eta > 0, length > 0, NL >= 1, else LGFIB_EINVAL. */
int ib_block_weights(const double *X, int NL, int B, const int32_t *blocks, int nblk, double eta, double length,
                     double *w);

/* The flow-domain update of Sec. 4.1, host only.  Over the blocks of D_xflow
 * (xflow, host int32 [nx][3]) with host mu, nu (from lgf_block_support) and
 * weights (ib_block_weights):
 *   W_flow(B) = weights[B] max(mu[B] / mu_global, nu[B] / nu_global)
 * (a global maximum of zero leaves its ratio out); the new D_flow is every
 * block with W_flow > eps together with the body blocks (host int32
 * [nbody][3]), and the new D_xflow every block within nbuf (0..8) blocks of
 * D_flow along each axis.  Both lists are written sorted by (z, y, x) to
 * flow_out (capacity max_flow blocks) and xflow_out (max_xflow); *nflow and
 * *nxflow receive their sizes, also when a capacity is too small, which
 * returns LGFIB_ERANGE. */
int ib_adapt_flow(const int32_t *xflow, int nx, const double *mu, const double *nu, const double *weights,
                  double eps, const int32_t *body, int nbody, int nbuf, int32_t *flow_out, int max_flow, int *nflow,
                  int32_t *xflow_out, int max_xflow, int *nxflow);

/* The flow-domain update of Sec. 4.1 with its block weights
 * (Eq. weight_fun_modifer) on the device, in one call: the result of
 * ib_block_weights(X, NL, B, xflow, nx, eta, length, w) followed by
 * ib_adapt_flow(xflow, nx, mu, nu, w, eps, body, nbody, nbuf, ...), block
 * for block (the same floating-point operations, without fused
 * multiply-adds).
 *   X: device double [NL][3] (lattice units); xflow: host int32 [nx][3];
 *   mu, nu: device double [nx] (lgf_block_support); body: host int32
 *   [nbody][3].  The output lists, sizes and LGFIB_ERANGE on too small a
 *   capacity are as in ib_adapt_flow.  The blocks' bounding box grown by nbuf
 *   may hold at most 2^26 blocks (else LGFIB_ERANGE); the context keeps three
 *   byte grids of that size as workspace.  Returns after the lists are on the
 *   host (the stream is synchronised). */
int ib_adapt_flow_dev(lgfib_ctx *ctx, const double *X, int NL, int B, const int32_t *xflow, int nx, const double *mu,
                      const double *nu, double eta, double length, double eps, const int32_t *body, int nbody,
                      int nbuf, int32_t *flow_out, int max_flow, int *nflow, int32_t *xflow_out, int max_xflow,
                      int *nxflow, lgfib_stream_t stream);

/* Velocity refresh on a finite flow domain (Sec. 4.1, Eq. vel_refresh; the
 * curl C and its transpose of Sec. 2.1), in place:
 *   w = C u on the edges of the vorticity blocks (zero elsewhere),
 *   s = -L^{-1} w (free-space solution, G_L table `tbl`),
 *   u <- C^T s on the faces of the flow blocks.
 * For a divergence-free u whose vorticity lies in the vorticity blocks this
 * returns u; errors of u away from the vorticity are replaced by the
 * velocity the vorticity induces.  The sign of s follows from
 * L_F = -G G^T - C^T C (Sec. 2.1).  Face k of cell n sits at
 * n + (1,1,1)/2 - e_k/2, edge i at n + e_i/2:
 *   (C u)^(i)(n) = sum_jk eps_ijk [u^(k)(n) - u^(k)(n - e_j)].
 * u outside the flow blocks is taken as zero.  Lattice units (the grid
 * spacing cancels).
 *   u: device [3][nflow][B^3], FP32 or FP64 by prec, x fastest in a block.
 *   vort_blocks: host int32 [nvort][3], each also a flow block, else
 *   LGFIB_EINVAL; flow_blocks: host int32 [nflow][3]; duplicates give
 *   LGFIB_EDUP_BLOCK.  nvort == 0 zeroes u.  B in {4, 8, 16, 32}.
 *   tbl must be an LGF_KIND_L table reaching the span of the flow blocks and
 *   of the vorticity blocks' lower neighbours, else LGFIB_ERANGE.
 * Runs as one stencil kernel (r = -C^T of the restricted w) and the
 * 3-component box-FFT apply of G_L * r (C^T commutes with the convolution);
 * the plan and its FP32/FP64 workspace of 3 x (source blocks) x B^3 values
 * are cached in the context by the two block lists.  Asynchronous on stream. */
int lgf_velocity_refresh(lgfib_ctx *ctx, lgf_table_t tbl, int B,
                         const int32_t *vort_blocks, int nvort,
                         const int32_t *flow_blocks, int nflow,
                         int prec, void *u, lgfib_stream_t stream);


/* ------------------------------------------------------ immersed boundary */

/* D_body (Sec. 4.1): the blocks of edge B holding a cell at most one cell
 * away (in every axis) from a cell n whose face (n, k) lies in the support of
 * some delta(x_F^(k)(n) - X_i).  X: HOST double [NL][3] in lattice units.
 * Writes up to max block triples to out (sorted by z, then y, then x) and
 * their count to *n; LGFIB_ERANGE if max is too small (*n then holds the
 * count needed).  Host-side staging; no device work. */
int ib_body_blocks(int kernel, const double *X, int NL, int B, int32_t *out, int max, int *n);

/* Regularization g = R x (Sec. 2.1):
 *   g^(k)(n) = dx^-3 sum_i x_i^(k) prod_j phi(x_F^(k)(n)_j - X_ij),
 * phi the 3-point kernel (IB_ROMA3: Roma, Peskin & Berger 1999; IB_SMOOTH3:
 * its smoothed version, Yang et al. 2009, support 4), x_F^(k)(n) =
 * n + (1/2,1/2,1/2) - e_k/2.  X: HOST double [NL][3] (lattice units; the
 * marker binning is built once per distinct (X, blocks) and cached);
 * x: DEVICE [NL][3]; faces: DEVICE [3][nblk][B^3], overwritten on every
 * face of the block set.  Every marker's support must lie inside the block
 * set, else LGFIB_ESUPPORT.  Deterministic (gather over per-block marker
 * lists; no atomics). */
int ib_regularize(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B,
                  const int32_t *blocks, int nblk, int prec, double dx,
                  const void *x, void *faces, lgfib_stream_t stream);

/* Interpolation v = I u = dx^3 R^T u (Sec. 2.1):
 *   v_i^(k) = sum_n u^(k)(n) prod_j phi(x_F^(k)(n)_j - X_ij).
 * Same arguments; faces is read, v: DEVICE [NL][3] overwritten. */
int ib_interpolate(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B,
                   const int32_t *blocks, int nblk, int prec, double dx,
                   const void *faces, void *v, lgfib_stream_t stream);

/* A rigid-body force system: markers, kernel, body blocks and a = nu dt/dx^2.
 * Builds the G_K(a) table over the body blocks' span and every plan the
 * Schur complement needs.  X: HOST [NL][3]; blocks: HOST (e.g. from
 * ib_body_blocks); B in {4, 8, 16}. */
typedef struct ib_system ib_system;
int ib_system_create(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B,
                     const int32_t *blocks, int nblk, double a, ib_system **out);
void ib_system_destroy(ib_system *sys);

/* y = C x with the force Schur complement of a rigid body (Sec. 3.1,
 * Eq. force_schur with I^{i-1} = I^i):  C = I [E(a) + G K^{-1} G^T] I^T,
 * G the staggered gradient (G q)^(k)(n) = q(n) - q(n - e_k), K^{-1} the
 * G_K(a) convolution, every operator restricted to the body blocks (Table
 * tab:src_trg).  Lattice units (C does not depend on dx).  x, y: DEVICE
 * [NL][3] in prec; they must not overlap. */
int ib_schur_apply(lgfib_ctx *ctx, ib_system *sys, int prec, const void *x, void *y,
                   lgfib_stream_t stream);

typedef struct {
    int iterations;        /* CG iterations (inner iterations summed) */
    int restarts;          /* outer FP64 residual evaluations */
    int fallback;          /* 1 if x0 was rejected (NaN/Inf or worse than 0) */
    double rel_residual;   /* final ||b - C f|| / ||b|| from an FP64 matvec */
    double ms;             /* wall time of the solve */
    int graphs;            /* 1: CG iterations ran as captured HIP graphs */
} ib_solve_stats_t;

/* Solve C f = b by conjugate gradients (C is SPD for a rigid body, Sec. 3.2).
 * The matvec runs in prec; all dot products, the iterate and the residual
 * in FP64.  With prec == LGF_F32 the solve is refined: inner FP32-matvec CG
 * sweeps are restarted from the FP64 true residual b - C f until
 * ||b - C f|| / ||b|| <= rtol (FP64 matvec).  x0 (DEVICE [NL][3] double, may
 * be NULL for a cold start) is the initial guess; a guess containing NaN/Inf
 * or whose residual exceeds ||b|| is replaced by 0 and stats->fallback = 1.
 * b, f: DEVICE double [NL][3].  Returns LGFIB_ENOCONV (with f holding the
 * last iterate) if maxit iterations do not reach rtol.  Synchronous.
 * Convergence is tested one iteration late (the device never waits for the
 * host), so a solve may run one iteration past the one that met the test.
 * Each iteration is replayed from a captured HIP graph unless the
 * environment sets LGFIB_CG_GRAPH=0 (then the same kernels are launched one
 * by one; results are identical).
 * prec == IB_SOLVE_DIRECT instead solves with the system's inverse Cholesky
 * factor (ib_system_factor; LGFIB_ENOTBUILT without one): f = W^T (W b),
 * x0, rtol and maxit are ignored, stats->iterations = 0, and when stats is
 * given one FP64 matvec fills stats->rel_residual. */
enum { IB_SOLVE_DIRECT = 2 };
int ib_force_solve(lgfib_ctx *ctx, ib_system *sys, int prec, const double *b, double *f,
                   const double *x0, double rtol, int maxit, ib_solve_stats_t *stats,
                   lgfib_stream_t stream);

/* Boundary-force post-processing of the sphere results (Sec. 5, flow around
 * spheres): the smoothed force fhat = I W R f, with W = 1 / gamma where
 * gamma = R 1 (the regularized all-ones marker vector) is nonzero and 0
 * elsewhere, on the system's body blocks (a weighted moving average with
 * the discrete delta as kernel).  f, fhat: DEVICE double [NL][3]; they may
 * alias.  gamma is built on the first call.  Asynchronous on stream; uses
 * the system's work fields, so calls on one system are ordered by the
 * caller. */
int ib_force_smooth(lgfib_ctx *ctx, ib_system *sys, const double *f, double *fhat, lgfib_stream_t stream);

/* ------------------------------------------- dense force solve (Sec. 3.2) */

/* The force Schur complement as a dense matrix, built as the paper's
 * pre-processing does: column j = C e_j by the FP64 matvec of
 * ib_schur_apply, for j < n = 3 NL (unknown i*3 + k is component k of
 * marker i).  C: DEVICE double [n][ld] row-major, ld >= n, caller-owned.
 * Costs n matvecs.  Synchronous. */
int ib_schur_dense(lgfib_ctx *ctx, ib_system *sys, double *C, int ld, lgfib_stream_t stream);

/* Cholesky factorisation of a symmetric positive definite matrix, C = L L^T,
 * and the inverse of its factor W = L^{-1} (Sec. 3.2: computed once, then
 * every solve is two matrix-vector products).  FP64; recursive on halves,
 * so the work is FP64 matrix-core products apart from 64 x 64 diagonal
 * leaves.  A: DEVICE double [n][lda] row-major; only its lower triangle is
 * read; on return the lower triangle (with the diagonal) holds L and the
 * strict upper triangle is unspecified.  W: DEVICE double [n][ldw] receives
 * L^{-1} (lower triangular, strict upper triangle zero); A and W must not
 * overlap.  Uses a context workspace of about n^2/4 doubles.  Returns
 * LGFIB_ENOTSPD when a pivot is not positive (L and W then hold NaN).
 * Synchronous. */
int ib_chol_factor(lgfib_ctx *ctx, int n, double *A, int lda, double *W, int ldw, lgfib_stream_t stream);

/* x = W^T (W b) for a lower-triangular W (the inverse Cholesky factor from
 * ib_chol_factor: x = C^{-1} b).  W: DEVICE double [n][ldw]; b, x: DEVICE
 * double [n] (may alias).  Reads each half of W once.  Asynchronous on
 * stream; uses a context workspace of 33 n doubles, so concurrent calls on
 * one context must be ordered by the caller. */
int ib_chol_solve(lgfib_ctx *ctx, int n, const double *W, int ldw, const double *b, double *x,
                  lgfib_stream_t stream);

/* With enable != 0: build the system's dense C (ib_schur_dense), factor it
 * (ib_chol_factor) and keep W inside the system (8 n^2 bytes, n = 3 NL);
 * from then on ib_force_solve and ib_flow_step accept IB_SOLVE_DIRECT.
 * enable == 0 releases the factor.  Synchronous.  Returns LGFIB_ENOTSPD if
 * C is not positive definite. */
int ib_system_factor(lgfib_ctx *ctx, ib_system *sys, int enable, lgfib_stream_t stream);

/* Force-history driver: one integrating-factor Euler step (a one-stage
 * IF-HERK scheme, Sec. 2.3, with the nonlinear term omitted: a Stokes flow)
 * of the discrete equations with the rigid body of `sys`, solved by the
 * nested projection of Sec. 3.1, Eq. nested_proj (ip, f, pc, vc) with
 * H = E(a):  d* = L^{-1}(-G^T u);  C f = I H[u - G d*] - u_B;
 * d = d* + L^{-1} G^T R f;  u <- H[u - G d - R f].  Every operator is
 * restricted to the flow blocks, which must contain the body blocks.
 * u: DEVICE double faces [3][nflow][B^3] (updated in place); u_B: DEVICE
 * double [NL][3], the marker velocity at the new time; f: DEVICE double
 * [NL][3] receives the force; x0 (nullable) warm-starts the force solve,
 * which runs as ib_force_solve(prec, rtol, maxit) (prec may be
 * IB_SOLVE_DIRECT for a factored system); b_out (nullable, DEVICE
 * double [NL][3]) receives that solve's right-hand side
 * b = I H[u - G d*] - u_B.  Synchronous. */
typedef struct ib_flow ib_flow;
int ib_flow_create(lgfib_ctx *ctx, ib_system *sys, const int32_t *flow_blocks, int nflow, ib_flow **out);
void ib_flow_destroy(ib_flow *flow);
int ib_flow_step(lgfib_ctx *ctx, ib_flow *flow, double *u, const double *u_B, double *f, const double *x0,
                 double rtol, int maxit, int prec, ib_solve_stats_t *stats, double *b_out, lgfib_stream_t stream);

/* ------------------------------------------ IF-HERK step (Sec. 2.3, App. B) */

/* The shifted tableau of the HERK schemes of App. B (scheme 0..3 = A..D):
 * for an explicit tableau (A, b, c) with s rows, at[i][j] = A[i+1][j] for
 * i < s - 1, at[s-1][j] = b[j], ct[i] = c[i+1], ct[s-1] = 1 (stage i ends at
 * node ct[i]).  Scheme D is the classical four-stage method.  at: HOST double
 * [16] (row-major [s][s]), ct: HOST double [4]; *s receives 3 or 4. */
int ib_herk_tableau(int scheme, int *s, double *at, double *ct);

/* An s-stage integrating-factor half-explicit Runge-Kutta step of the Stokes
 * driver (Sec. 2.3, the nonlinear term omitted) on the flow blocks.  Stage i
 * solves the system of Eq. ibifherk_linsys, H_i^{-1} u_i + Q lam_i = r_i,
 * Q^T u_i = (0, u_B(t + ct_i dt)), Q = [G, R], by the nested projection of
 * ib_flow_step with H_i = E((ct_i - ct_{i-1}) A) (ct_{-1} = 0); the
 * right-hand side is r_i = h_i - sum_{j<i} (at_ij / at_jj) P_ij Q lam_j, with
 * h_0 = u_k, h_i = H_{i-1} h_{i-1} and P_ij = H_{i-1} ... H_j (the dt factors
 * of the scheme cancel).  u_{k+1} = u_s and the reported force is
 * lam_f,s / at_ss.  A = nu dt / dx^2, the integrating-factor parameter of a
 * whole step.  Stages with equal parameters share one force system (and, with
 * direct != 0, one dense factor: their force solves are then direct).
 * at: HOST double [s][s], lower triangular with a nonzero diagonal; ct: HOST
 * double [s], nondecreasing in [0, 1].  X, blocks as ib_system_create and
 * ib_flow_create (the flow blocks contain the body blocks).  Synchronous. */
typedef struct ib_herk ib_herk;
int ib_herk_create(lgfib_ctx *ctx, int kernel, const double *X, int NL, int B, const int32_t *body_blocks, int nbody,
                   const int32_t *flow_blocks, int nflow, double A, int s, const double *at, const double *ct,
                   int direct, ib_herk **out);
/* One step: u: DEVICE double faces [3][nflow][B^3], updated in place; ub:
 * DEVICE double [s][NL][3], the marker velocity at t_k + ct_i dt; f: DEVICE
 * double [NL][3] receives the force.  Without a dense factor the force solves
 * are CG (prec, rtol, maxit), warm-started from the same stage of the
 * previous step.  stats (nullable) sums iterations, restarts, fallbacks and
 * ms over the stages and keeps the largest residual.  Returns LGFIB_ENOCONV
 * if a stage's solve stopped at maxit (the step still completes).
 * Synchronous. */
int ib_herk_step(lgfib_ctx *ctx, ib_herk *hk, double *u, const double *ub, double *f, double rtol, int maxit,
                 int prec, ib_solve_stats_t *stats, lgfib_stream_t stream);

/* Turn the nonlinear term on in ib_herk_step (Sec. 2.3, Eq. ibifherk_g):
 * stage i adds g^i = -a~_ii dt N~(u^{i-1}), u^0 the step's input and u^{i-1}
 * the previous stage's solution, and propagates Q lam^j - g^j in place of
 * Q lam^j, which makes the step the Navier-Stokes step on the fixed flow set.
 * N~ is lgf_lamb_vector's term with frame velocity U on the flow blocks.
 *   dt: the time step over the grid spacing, in the velocity's units (the
 *   convective Courant number is dt |u|); dt = 0 turns the term off (Stokes).
 *   U: host double[3] or NULL (zero).  dt < 0 or non-finite values give
 *   LGFIB_EINVAL.  Host-side only; applies to the following steps. */
int ib_herk_convection(lgfib_ctx *ctx, ib_herk *hk, double dt, const double *U);
void ib_herk_destroy(ib_herk *hk);

/* ------------------------------------------ block-pair form (8^3 blocks) */

/* Transforms of the block-pair form: */
enum {
    LGF_DFT_FFT32 = 0,    /* 16-point DFTs in FP32 registers */
    LGF_DFT_BF16X3 = 1    /* DFTs as 16 x 16 complex matrix products on the
                             matrix cores, both operands split into three BF16
                             terms (hi + mid + lo), the six products down to
                             relative size 2^-16, FP32 accumulation */
};
/* u = dx^2 G * f (Eq. dpoisson_conv) evaluated block pair by block pair for
 * blocks of 8^3: per source block the zero-padded 16^3 spectrum, per target
 * block U_t(k) = sum_s Ghat_{t-s}(k) F_s(k) with Ghat_d the spectrum of the
 * kernel over the offsets of block distance d (FP64 transform, cached per
 * table and span), then the inverse kept on the block.  Exact (no
 * truncation); cost grows with the number of block pairs.  FP32 fields
 * [ncomp][n][8^3] as lgf_poisson_apply (B must be 8); dft selects the
 * per-block transforms.  Asynchronous on stream (the block lists are
 * copied before return). */
int lgf_pair_apply(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *src_blocks, int nsrc,
                   const int32_t *tgt_blocks, int ntgt, int ncomp, int dft, double dx, const float *f, float *u,
                   lgfib_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * apply as lgf_pair_apply, same arguments and results, with every
 * intermediate (the pair lists, the kernel spectra of the span, the source
 * and target spectra) in a static device array of 64 MiB that each device
 * using the library holds until the process ends; the call makes no device
 * allocation.  The kernel spectra are transformed on every call (nothing is
 * cached).  A set needing more than 64 MiB
 * (lists + (2D+1)^3 * 18 KiB for a span of D blocks per axis +
 * ncomp * (nsrc + ntgt) * 18 KiB) returns LGFIB_ERANGE before anything is
 * launched.  All calls on one device share that array: calls that overlap on
 * one device (two streams, two threads, or two contexts) race and must be
 * ordered by the caller.  The caller still owns f and u; the table must have
 * been built.  Synchronous with respect to `stream` on return (the host lists
 * are copied through it). */
int lgf_pair_apply_noalloc(lgfib_ctx *ctx, lgf_table_t tbl, int B, const int32_t *src_blocks, int nsrc,
                           const int32_t *tgt_blocks, int ntgt, int ncomp, int dft, double dx, const float *f,
                           float *u, lgfib_stream_t stream);

/* ------------------------------------------- multilevel (far-field) form */

/* u ~= dx^2 G * f (Eq. dpoisson_conv) by a multilevel interpolation method,
 * the kind of evaluator Sec. 2.2 names for these convolutions (kernel
 * independent, interpolation based, linear in the number of blocks); the
 * paper gives no steps, so these are this library's:
 *   - blocks of B^3 cells are the leaves; level l groups 2^l blocks per axis
 *     into a cluster of side L = B 2^l; the top level is the first at which
 *     sources and targets together span at most 4 clusters per axis;
 *   - each cluster has p^3 nodes on lattice points, the tensor product of
 *     t_j = floor((L-1)/2 (1 - cos(pi (2j+1)/(2p))) + 1/2);
 *   - sources are anterpolated to their block's nodes and up the levels with
 *     the Lagrange basis of the receiving cluster; clusters interact node to
 *     node at the finest level where they are not neighbours (Chebyshev
 *     distance of the cluster indices > 1) but their parents are (at the top
 *     level: every non-neighbour pair); node values are interpolated down to
 *     the cells; neighbouring blocks (the block itself included) are summed
 *     exactly.
 * The result is exact for kernels that are polynomials of degree < p in
 * each coordinate; for G_L its error falls with p: on the sets of 8^3
 * blocks tested (random sparse sets and sphere shells of up to 26,120
 * blocks) it stays below 5e-4 of the largest value at p = 4, 1e-4 at
 * p = 5 and 2e-5 at p = 6.
 *
 * lgf_ml_create plans one (table, B, p, sources, targets):
 *   B in {4, 8}; p in {4, 5, 6} with p <= B; pair_prec LGF_F64, or LGF_F32
 *   (B = 8 only) to run the node-to-node products and the exact neighbour
 *   sum as FP32 matrix products (FP32 kernel matrices, rounded node charges
 *   and sources, FP32 accumulation; results about 1e-6 of the largest
 *   value from the FP64 form, below the interpolation error at these p); src_blocks / tgt_blocks: HOST int32
 *   [n][3] block coordinates (copied; no duplicates within a list; either
 *   may be empty).  The table extent must reach (c+1) B 2^top - 1 on each
 *   axis, c the span of the top-level cluster indices (the top clusters'
 *   nodes reach beyond the blocks), else LGFIB_ERANGE.  Builds the
 *   node-to-node matrices from the table on `stream` and waits for them.
 *   *out receives the plan (release with lgf_ml_destroy, before the
 *   context).
 * lgf_ml_apply evaluates: f DEVICE double [ncomp][nsrc][B^3] (cells z, y, x
 *   within a block, blocks in list order), u DEVICE double
 *   [ncomp][ntgt][B^3], overwritten; 1 <= ncomp <= 8; dx > 0; f and u must
 *   not overlap; u must be ordinary (coarse-grained) device memory, since
 *   the pair products add into it with hardware floating-point atomics.
 *   Asynchronous on `stream`; one apply at a time per plan (the plan holds
 *   the node values).  Results differ from run to run in the last bits
 *   (pair products are accumulated atomically).
 * lgf_ml_info: levels above the blocks (top), source and target clusters
 *   over all levels, node-to-node pairs, neighbour block pairs and distinct
 *   node-to-node matrices, in out[0..5]. */
typedef struct lgf_ml lgf_ml_t;
int lgf_ml_create(lgfib_ctx *ctx, lgf_table_t tbl, int B, int p, int pair_prec, const int32_t *src_blocks,
                  int nsrc, const int32_t *tgt_blocks, int ntgt, lgfib_stream_t stream, lgf_ml_t **out);
int lgf_ml_apply(lgfib_ctx *ctx, lgf_ml_t *plan, int ncomp, double dx, const double *f, double *u,
                 lgfib_stream_t stream);
int lgf_ml_info(const lgf_ml_t *plan, int64_t out[6]);
void lgf_ml_destroy(lgf_ml_t *plan);

/* ------------------------------------------------------- batched applies */

/* Many independent FP32 scalar Poisson applies u_i = dx^2 G * f_i on block sets
 * S_i (targets = sources, Eq. dpoisson_conv) run as one HIP-graph launch.
 * blocks: HOST int32 [nblk][3] (blocks of B^3); f, u: DEVICE float
 * [nblk][B^3] in the block order of `blocks` (caller-owned, must stay valid
 * and at the same address while the batch exists; u must not overlap f). */
typedef struct {
    int nblk;
    const int32_t *blocks;
    const float *f;
    float *u;
} lgf_instance_t;
typedef struct lgf_batch lgf_batch_t;
/* flags of lgf_batch_create (a bit set; 1 alone keeps the meaning "autotune") */
enum {
    LGF_BATCH_AUTOTUNE = 1,   /* time the candidates of every instance, keep the fastest */
    LGF_BATCH_PASSES = 2      /* box instances run as batched passes (below) */
};
/* Plans the batch: with LGF_BATCH_AUTOTUNE each instance is timed for the
 * block size its box is built from (B, B/2 or 2B, re-blocking the fields
 * exactly), the tiles per workgroup of the FFT passes and, for sets of at
 * most 400 blocks of 8^3, the block-pair form (lgf_pair_apply), and the
 * fastest is kept.  Without LGF_BATCH_PASSES every instance runs its own
 * kernels: instances are bin-packed by time onto nbranch (1..16) concurrent
 * graph branches, each with its own FFT workspace.  With LGF_BATCH_PASSES the
 * box instances whose FFT lengths have specialised passes share launches:
 * one launch per (pass, FFT length) over all of them, in pass order, with one
 * workgroup per (instance, tile group) work item taken in an XCD-aware order
 * (or, with the environment variable LGFIB_BATCH_PERSIST=1, a persistent grid
 * whose workgroups pull the items from a device counter), each instance with
 * its own workspace; the other instances run on the branches beside them.  Either way the batch is captured into one graph.  The table
 * tbl (a G_L table) must cover every instance's span at every block size
 * tried (ERANGE otherwise, after trying the others).  The autotuner runs the
 * applies, so f must hold valid data.  Synchronous. */
int lgf_batch_create(lgfib_ctx *ctx, lgf_table_t tbl, int B, int ninst, const lgf_instance_t *inst, double dx,
                     int flags, int nbranch, lgf_batch_t **out);
/* eager == 0: one hipGraphLaunch of the captured batch on `stream`;
 * eager != 0: the same kernels launched one after another on `stream`. */
int lgf_batch_run(lgfib_ctx *ctx, lgf_batch_t *batch, int eager, lgfib_stream_t stream);
/* The autotuner's choice for instance i: block size, x / y tiles per
 * workgroup (0: defaults), branch, its timed ms (0 without autotune) and the
 * form (0 box FFT, 1 block pairs).  Null outputs are skipped. */
int lgf_batch_info(lgf_batch_t *batch, int i, int *block, int *tiles_x, int *tiles_y, int *branch,
                   double *tuned_ms, int *path);
void lgf_batch_destroy(lgf_batch_t *batch);
/* One-shot form: plans the instances without autotuning (each at block size
 * B with the default tiles, spread over four branches), runs them as one
 * graph launch on `stream`, waits, and releases the plan.  For repeated
 * applies on the same sets keep a batch from lgf_batch_create instead.
 * Synchronous. */
int lgf_poisson_apply_batched(lgfib_ctx *ctx, lgf_table_t tbl, int B, int ninst, const lgf_instance_t *inst,
                              double dx, lgfib_stream_t stream);

/* ------------------------------------------------- learned warm start (MLP) */

/* A per-marker network nin -> nh -> nh -> nout with tanh hidden layers that
 * corrects the linear extrapolation of a marker's force history, used to
 * warm-start the force solve (x0_i = 2 f_{k-1,i} - f_{k-2,i} + MLP(features_i);
 * the CG iteration it starts still decides convergence, see
 * ib_force_solve).  Not part of the paper's method.
 *   y = out_shift + out_scale * (W3 tanh(W2 tanh(W1 xh + b1) + b2) + b3),
 *   xh = (x - in_shift) / in_scale.
 * params (HOST float, copied): W1 [nh][nin], b1 [nh], W2 [nh][nh], b2 [nh],
 * W3 [nout][nh], b3 [nout] (FP32 master weights, row-major).  Matrix products
 * round both operands to BF16 (round to nearest even) and accumulate in FP32
 * on the matrix cores. */
typedef struct ib_mlp ib_mlp;
int ib_mlp_create(lgfib_ctx *ctx, int nin, int nh, int nout, const float *params, const float *in_shift,
                  const float *in_scale, const float *out_shift, const float *out_scale, ib_mlp **out);
void ib_mlp_destroy(ib_mlp *m);
int ib_mlp_get_params(ib_mlp *m, float *host, int64_t n);
/* y = MLP(x): x DEVICE float [M][nin], y DEVICE float [M][nout]. */
int ib_mlp_forward(lgfib_ctx *ctx, ib_mlp *m, const float *x, int M, float *y, lgfib_stream_t stream);
/* Gradient of 0.5/M sum_m ||o_m - (t_m - out_shift)/out_scale||^2 with respect
 * to the parameters (o the normalised output), copied to grad_host (nparam
 * floats, same layout as params); *loss receives the loss.  Synchronous. */
int ib_mlp_grad(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, float *grad_host, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss. */
int ib_mlp_train_step(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, float lr,
                      lgfib_stream_t stream);
int ib_mlp_last_loss(ib_mlp *m, int M, double *loss);
/* epochs x (M / batch) Adam steps over rows shuffled per epoch by a splitmix64
 * stream seeded with seed (rows beyond the last full batch are skipped that
 * epoch); *final_loss = loss of the last batch.  Synchronous. */
int ib_mlp_train(lgfib_ctx *ctx, ib_mlp *m, const float *x, const float *t, int M, int epochs, int batch, float lr,
                 uint64_t seed, double *final_loss);
/* Features of marker i for the solve of step k (DEVICE float [NL][12]):
 * [normal_i (3), U_{k+1} - U_k, U_k - U_{k-1}, U_{k-1} - U_{k-2},
 *  f_{k-1,i} (3), f_{k-1,i} - f_{k-2,i} (3)], with ustate = (U_{k+1}, U_k,
 * U_{k-1}, U_{k-2}) (HOST 4 doubles: the body velocity history); normals, f1,
 * f2: DEVICE double [NL][3]. */
int ib_mlp_features(lgfib_ctx *ctx, const double *normals, const double *ustate, const double *f1, const double *f2,
                    int NL, float *feats, lgfib_stream_t stream);
/* x0 = 2 f1 - f2 + MLP(feats) (f1, f2, x0: DEVICE double [NL][3]); the
 * network must map 12 -> 3. */
int ib_mlp_warmstart(lgfib_ctx *ctx, ib_mlp *m, const float *feats, const double *f1, const double *f2, int NL,
                     double *x0, lgfib_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LGFIB_H */
