"""Pins of the FP64 oracle's Bessel factors, LGF tables and direct sums against
facts the paper and the mathematics fix (closed forms, identities, library
evaluations of the defining integrals, brute force).  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads


# --------------------------------------------------------------------------
# Bessel factors e^{-x} I_n(x)  (App. A, Eq. lgf_intfac)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("x", [1e-3, 0.1, 1.0, 10.0, 63.0, 100.0, 1000.0, 8.0e4, 1.0e6])
def test_bessel_matches_library(x):
    """Against mpmath.besseli (an independent library routine) at 30 digits;
    the three oracle branches (series, trapezoid, Hankel) are all exercised.
    The trapezoid branch is accurate to ~1e-17 absolute (its terms are bounded
    by 1), so tiny high orders there are held to that, not to a relative bound."""
    mp.mp.dps = 30
    v = oracle.bessel_scaled(x, 40)
    for n in (0, 1, 5, 20, 40):
        ref = mp.exp(-x) * mp.besseli(n, x)
        if ref < 1e-280:
            continue
        assert abs(v[n] - float(ref)) <= 5e-14 * float(ref) + 2e-17, (n, x, v[n], ref)


@pytest.mark.parametrize("alpha", [0.02, 0.05, 0.1, 0.5, 1.0])
def test_if_kernel_sums_to_one(alpha):
    """sum_j e^{-2a} I_j(2a) = 1 (generating function of I_n at theta = 0), so the
    3D kernel of E(a) sums to one."""
    w = oracle.bessel_scaled(2 * alpha, 80)
    assert abs(w[0] + 2 * w[1:].sum() - 1.0) < 1e-15


@pytest.mark.parametrize("a,b", [(0.02, 0.05), (0.1, 0.5)])
def test_if_semigroup(a, b):
    """E(a) E(b) = E(a + b): the 1D weights convolve into the weights of a + b
    (Neumann's addition theorem for I_n)."""
    N = 60
    wa = oracle.bessel_scaled(2 * a, N)
    wb = oracle.bessel_scaled(2 * b, N)
    wab = oracle.bessel_scaled(2 * (a + b), N)
    fa = np.concatenate([wa[:0:-1], wa])
    fb = np.concatenate([wb[:0:-1], wb])
    conv = np.convolve(fa, fb)
    mid = len(conv) // 2
    assert np.max(np.abs(conv[mid:mid + 20] - wab[:20])) < 1e-15


def test_if_truncation_radius():
    """The 1e-14 cut of e^{-2a} I_j(2a): r is the last j at or above the cut."""
    mp.mp.dps = 30
    for a in (0.02, 0.05, 0.1, 0.5):
        r = oracle.if_radius(a)
        assert mp.exp(-2 * a) * mp.besseli(r, 2 * a) >= 1e-14
        assert mp.exp(-2 * a) * mp.besseli(r + 1, 2 * a) < 1e-14


@pytest.mark.parametrize("a", [0.001, 0.02, 0.05, 0.1, 0.5, 1.0, 4.0])
def test_if_fp32_cut_drops_less_than_roundoff(a):
    """The FP32 applies cut e^{-2a} I_j(2a) below 2^-28: the weights dropped on
    both sides of all three axes sum to less than FP32's unit roundoff 2^-24
    (the 3D kernel is the product of three 1D kernels that each sum to 1, so
    the dropped mass of the product is at most the sum over the axes)."""
    mp.mp.dps = 40
    w = lambda j: mp.exp(-2 * a) * mp.besseli(j, 2 * a)
    r = 0
    while w(r + 1) >= mp.mpf(2) ** -28:
        r += 1
    assert w(r) >= mp.mpf(2) ** -28 or r == 0
    tail, j = mp.mpf(0), r + 1
    while True:
        t = w(j)
        tail += t
        if t < mp.mpf(10) ** -30:
            break
        j += 1
    assert 3 * 2 * tail < mp.mpf(2) ** -24, (a, r, float(tail))


# --------------------------------------------------------------------------
# LGF of the 7-point Laplacian (Sec. 2.2, App. A Eq. lgf_lap)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def gtab():
    return oracle.lgf_table(48, 40, 40)


def _G(tab, n):
    a = sorted((abs(int(v)) for v in n), reverse=True)
    return tab[a[2], a[1], a[0]]


def test_origin_watson_closed_form(gtab):
    """G(0) = -W/6 with W = sqrt(6)/(32 pi^3) Gamma(1/24) Gamma(5/24) Gamma(7/24)
    Gamma(11/24) (Watson's integral for the simple cubic lattice)."""
    mp.mp.dps = 30
    W = mp.sqrt(6) / (32 * mp.pi ** 3) * mp.gamma(mp.mpf(1) / 24) * mp.gamma(mp.mpf(5) / 24) \
        * mp.gamma(mp.mpf(7) / 24) * mp.gamma(mp.mpf(11) / 24)
    assert abs(gtab[0, 0, 0] - float(-W / 6)) < 2e-16


def test_first_neighbour(gtab):
    """(L G)(0) = 1 with six equal neighbours gives G(e1) = G(0) + 1/6."""
    assert abs(gtab[0, 0, 1] - (gtab[0, 0, 0] + 1.0 / 6.0)) < 2e-16


def test_laplacian_of_lgf_is_delta(gtab):
    """L G = delta (G is the fundamental solution of the 7-point L, Eq. dpoisson)."""
    R = 12
    idx = np.arange(-R, R + 1)
    box = np.array([[[_G(gtab, (x, y, z)) for x in idx] for y in idx] for z in idx])
    lap = oracle.laplacian_7pt(box)
    delta = np.zeros_like(lap)
    delta[R - 1, R - 1, R - 1] = 1.0
    assert np.max(np.abs(lap - delta)) < 2e-15


@pytest.mark.parametrize("n", [(1, 1, 0), (3, 2, 1), (8, 4, 2)])
def test_against_library_quadrature(gtab, n):
    """G(n) = -int_0^inf prod_q e^{-2t} I_{n_q}(2t) dt evaluated independently by
    mpmath's adaptive quadrature and Bessel routine.  That evaluation itself
    carries ~1.3e-16 absolute error (it misses -W/6 by that much), hence 5e-16."""
    mp.mp.dps = 25
    f = lambda t: mp.fprod([mp.besseli(q, 2 * t) * mp.exp(-2 * t) for q in n])
    pts = [0] + [mp.mpf(2) ** k for k in range(-1, 20)] + [mp.inf]
    ref = -mp.quad(f, pts)
    assert abs(_G(gtab, n) - float(ref)) < 5e-16


def _far_field(n):
    """Asymptotic expansion of G_L for large |n| (leading term -1/(4 pi |n|),
    App. A footnote), derived from the small-xi expansion of 1/sigma:
      1/sigma = -1/|xi|^2 - (P4/12)/|xi|^4 - [(P4/12)^2/|xi|^6 - (P6/360)/|xi|^4] - ...
    with P_k = sum xi_i^k, each term inverted through the 3D transforms of
    |xi|^-2, |xi|^-4, |xi|^-6 (1/(4 pi r), -r/(8 pi), r^3/(96 pi))."""
    x = np.asarray(n, dtype=np.float64)
    r = math.sqrt(float(np.sum(x * x)))
    s4 = float(np.sum(x ** 4))
    t0 = -1.0 / (4 * math.pi * r)
    t1 = (3 * r ** 4 - 5 * s4) / (32 * math.pi * r ** 7)
    s8 = float(np.sum(x ** 8))
    s62 = sum(x[i] ** 6 * x[j] ** 2 for i in range(3) for j in range(3) if i != j)
    s44 = sum(x[i] ** 4 * x[j] ** 4 for i in range(3) for j in range(3) if i < j)
    s422 = sum(x[i] ** 4 * x[(i + 1) % 3] ** 2 * x[(i + 2) % 3] ** 2 for i in range(3))
    t2 = -(23 * s8 - 244 * s62 + 621 * s44 - 228 * s422) / (128 * math.pi * r ** 13)
    return t0, t1, t2


def test_far_field_convergence():
    """Each further asymptotic term shrinks the gap to the quadrature by the
    expected power of |n|; with three terms the gap is at rounding level for
    |n| >= 150 off-axis."""
    tab = oracle.lgf_table(160, 90, 60)
    for n, tol in [((160, 0, 0), 1e-12), ((120, 90, 60), 5e-14), ((64, 64, 0), 3e-12)]:
        g = tab[n[2], n[1], n[0]]
        t0, t1, t2 = _far_field(n)
        e0 = abs(t0 - g) / abs(g)
        e1 = abs(t0 + t1 - g) / abs(g)
        e2 = abs(t0 + t1 + t2 - g) / abs(g)
        assert e0 < 3e-5 and e1 < e0 * 1e-2 and e2 < e1 * 1e-2 and e2 < tol, (n, e0, e1, e2)


def test_quadrature_step_converged():
    """Halving the exp-sinh step leaves the table unchanged to rounding."""
    a = oracle.lgf_table(24, 16, 8, h=1.0 / 128)
    b = oracle.lgf_table(24, 16, 8, h=1.0 / 256)
    assert np.max(np.abs(a - b)) < 2e-17


# --------------------------------------------------------------------------
# G_K(a) = G_L + R(a)  (App. A)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [0.05, 0.5])
def test_r_origin_library(alpha):
    """R(a)(0) = int_0^a (e^{-2t} I_0(2t))^3 dt by mpmath."""
    mp.mp.dps = 25
    ref = mp.quad(lambda t: (mp.exp(-2 * t) * mp.besseli(0, 2 * t)) ** 3, [0, alpha])
    R = oracle.lgf_r_table(alpha, 2, 2, 2)
    assert abs(R[0, 0, 0] - float(ref)) < 1e-17


@pytest.mark.parametrize("alpha", [0.05, 0.5])
def test_laplacian_of_gk_is_if_kernel(alpha):
    """L G_K(a) = G_E(a): differentiate G_E(t) = exp(tL) delta in t and integrate
    over [0, a]; so L R(a) = G_E(a) - delta and L G_K(a) = G_E(a)."""
    R = oracle.lgf_r_table(alpha, 10, 10, 10)
    G = oracle.lgf_table(10, 10, 10)
    w = oracle.bessel_scaled(2 * alpha, 12)
    n = 8
    idx = np.arange(-n, n + 1)
    gk = np.array([[[G[abs(z), abs(y), abs(x)] + R[abs(z), abs(y), abs(x)] for x in idx]
                    for y in idx] for z in idx])
    lap = oracle.laplacian_7pt(gk)
    ii = np.abs(np.arange(-n + 1, n))
    ge = w[ii][:, None, None] * w[ii][None, :, None] * w[ii][None, None, :]
    assert np.max(np.abs(lap - ge)) < 3e-15


def test_decay_bounds_footnote():
    """Sec. 2.2 footnote: for a in [0, 1] and |n| > 10, |G_E(n)|/|G_E(0)| < 1e-7 and
    |G_K(n) - G_L(n)|/|G_L(0)| < 1e-9 (checked at the worst case a = 1 on the axis)."""
    w = oracle.bessel_scaled(2.0, 12)
    assert w[11] / w[0] < 1e-7
    R = oracle.lgf_r_table(1.0, 12, 0, 0)
    G0 = oracle.lgf_table(0, 0, 0)[0, 0, 0]
    assert abs(R[0, 0, 11]) / abs(G0) < 1e-9


# --------------------------------------------------------------------------
# Direct sums (Sec. 2.2, Eq. dpoisson_conv)
# --------------------------------------------------------------------------

def test_conv_direct_brute_force():
    """The C direct sum equals a pure-Python double loop on a tiny random set."""
    g = np.random.Generator(np.random.PCG64(7))
    src = g.integers(-4, 5, size=(30, 3))
    tgt = g.integers(-6, 7, size=(25, 3))
    f = g.standard_normal(30)
    K = g.standard_normal((7, 6, 5))
    u = oracle.conv_direct(K, src, f, tgt)
    ref = np.zeros(25)
    for i in range(25):
        for j in range(30):
            d = np.abs(tgt[i] - src[j])
            if d[0] <= 4 and d[1] <= 5 and d[2] <= 6:
                ref[i] += K[d[2], d[1], d[0]] * f[j]
    assert np.max(np.abs(u - ref)) < 1e-13


def test_conv_window_matches_direct():
    g = np.random.Generator(np.random.PCG64(8))
    box = g.standard_normal((6, 7, 8))
    org = np.array([3, -2, 5])
    K = oracle.if_kernel_table(0.1)
    z, y, x = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    src = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + org
    tgt = src[::5] + np.array([1, 0, -1])
    a = oracle.conv_window(K, box, org, tgt)
    b = oracle.conv_direct(K, src, box.ravel(), tgt)
    assert np.max(np.abs(a - b)) < 1e-14


def test_poisson_solution_small_cube():
    """u = G * f solves L u = f (Eq. dpoisson) everywhere: with f on the 16^3
    cube of 2x2x2 blocks of 8^3 (seeded N(0,1)), L u - f vanishes to rounding
    on an 18^3 box around it."""
    B = 8
    blocks = workloads.cube_blocks(2)
    f = workloads.normal_sources(len(blocks), B).reshape(-1)
    src = workloads.block_cells(blocks, B)
    G = oracle.lgf_table(17, 17, 17)
    idx = np.arange(-1, 17)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    tgt = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    u = oracle.conv_direct(G, src, f, tgt).reshape(18, 18, 18)
    org, fbox, _ = workloads.dense_box(blocks, B, f.reshape(-1, B, B, B))
    res = oracle.laplacian_7pt(u)
    fpad = np.zeros((16, 16, 16))
    fpad[:] = fbox
    assert np.max(np.abs(res - fpad)) < 2e-13 * np.max(np.abs(u))
