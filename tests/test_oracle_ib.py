"""Pins of the oracle's immersed-boundary operators: discrete delta moments,
the smoothed kernel against a numerical convolution, adjointness of I and R,
mimetic identities, and symmetry / definiteness of the force Schur complement
for a small sphere (Sec. 2.1, Sec. 3.1-3.2).  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads
from oracle.ib import ROMA3, SMOOTH3


@pytest.mark.parametrize("kernel", [ROMA3, SMOOTH3])
def test_delta_moments(kernel):
    """sum_j phi(x - j) = 1 and sum_j (x - j) phi(x - j) = 0 for every shift x
    (the defining moment conditions of both 3-point kernels)."""
    xs = np.random.Generator(np.random.PCG64(3)).uniform(-0.5, 0.5, 200)
    j = np.arange(-3, 4)
    for x in xs:
        w = oracle.phi(kernel, x - j)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(np.sum((x - j) * w)) < 1e-14


def test_roma_sum_of_squares():
    """Roma's kernel has the extra property sum_j phi(x - j)^2 = 1/2."""
    j = np.arange(-3, 4)
    for x in np.linspace(-0.5, 0.5, 41):
        assert abs(np.sum(oracle.phi_roma3(x - j) ** 2) - 0.5) < 1e-14


def test_smooth_kernel_is_roma_convolved_with_top_hat():
    """The smoothed kernel equals int_{r-1/2}^{r+1/2} phi_roma(s) ds (computed by
    scipy quad), and phi_smooth(0) = 5/12 + pi/(9 sqrt 3)."""
    for r in [0.0, 0.13, 0.5, 0.77, 1.0, 1.31, 1.5, 1.9, 2.0, 2.3]:
        brk = [p for p in (-1.5, -0.5, 0.5, 1.5) if r - 0.5 < p < r + 0.5]
        ref, _ = integrate.quad(lambda s: float(oracle.phi_roma3(s)), r - 0.5, r + 0.5,
                                points=brk or None, epsabs=1e-15, epsrel=1e-14)
        assert abs(float(oracle.phi_smooth3(r)) - ref) < 1e-13, r
    assert abs(float(oracle.phi_smooth3(0.0)) - (5.0 / 12.0 + math.pi / (9.0 * math.sqrt(3.0)))) < 1e-15


@pytest.mark.parametrize("kernel", [ROMA3, SMOOTH3])
def test_interpolate_regularize_adjoint(kernel):
    """I = dx^3 R^T (Sec. 2.1): <I v, g> = dx^3 <v, R g>."""
    g = np.random.Generator(np.random.PCG64(11))
    X = g.uniform(6.0, 10.0, size=(17, 3))
    gm = g.standard_normal((17, 3))
    shape = (16, 16, 16)
    v = g.standard_normal((3,) + shape)
    dx = 0.5
    Rg = oracle.regularize(X, gm, kernel, (0, 0, 0), shape, dx=dx)
    Iv = oracle.interpolate(X, v, kernel, (0, 0, 0), dx=dx)
    lhs = np.sum(Iv * gm) * dx ** 3 / dx ** 3
    rhs = dx ** 3 * np.sum(v * Rg)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_interpolate_reproduces_linear_fields():
    """Interpolating a linear face field returns its value at the marker
    (the zeroth and first moment conditions), with x_F^(k)(n) = n + 1/2 - e_k/2."""
    X = np.array([[7.3, 8.1, 6.6], [9.9, 7.45, 8.5]])
    shape = (16, 16, 16)
    z, y, x = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    a = np.array([0.3, -1.2, 0.7])
    u = np.zeros((3,) + shape)
    for k in range(3):
        pos = [x + 0.5, y + 0.5, z + 0.5]
        pos[k] = pos[k] - 0.5
        u[k] = 2.0 + a[0] * pos[0] + a[1] * pos[1] + a[2] * pos[2]
    v = oracle.interpolate(X, u, ROMA3, (0, 0, 0))
    for k in range(3):
        assert np.allclose(v[:, k], 2.0 + X @ a, atol=1e-13)


def test_mimetic_laplacian():
    """L_C = -G^T G (Sec. 2.1): the 7-point Laplacian on interior cells."""
    g = np.random.Generator(np.random.PCG64(5))
    q = np.zeros((12, 12, 12))
    q[2:-2, 2:-2, 2:-2] = g.standard_normal((8, 8, 8))
    lhs = -oracle.grad_adjoint(oracle.grad(q))[1:-1, 1:-1, 1:-1]
    assert np.max(np.abs(lhs - oracle.laplacian_7pt(q))) < 1e-13


@pytest.fixture(scope="module")
def small_sphere():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    blocks = oracle.body_blocks(X, ROMA3, 8)
    origin, mask = oracle.block_mask(blocks, 8)
    ext = np.array(mask.shape[::-1])
    alpha = 0.05
    gk = oracle.lgf_k_table(alpha, *ext)
    return X, blocks, origin, mask, alpha, gk


# Two Roma markers with B = 4, worked by hand (Sec. 2.1 places face k of cell n
# at n + (1/2)(1,1,1) - (1/2)e_k; Sec. 4.1 takes D_body as the blocks within one
# cell of the delta's support).  Per axis j and face component k the support is
# {n : |n + c - X_j| < 3/2} with c = 0 on the face's own axis, 1/2 elsewhere;
# dilating by one cell and dividing by B = 4 gives block ranges per axis, and
# D_body is the union over k of their products.
#   marker (5.25, 6.0, 9.7): x -> {0,1} for every k; (y, z) -> k=0 {1}x{1,2},
#     k=1 {1,2}x{1,2}, k=2 {1}x{2,3}: 5 (y,z) pairs, so 10 blocks; (y,z)=(2,3)
#     is NOT in the set (no single k reaches both).
#   marker (2.0, 1.6, 10.5): k=0 {0,1}x{-1,0}x{2,3}, k=1 {0}x{0,1}x{2,3},
#     k=2 {0}x{-1,0}x{2,3}: 10 blocks, two of them shared with the first marker.
BODY_MARKERS = np.array([[5.25, 6.0, 9.7], [2.0, 1.6, 10.5]])
BODY_BLOCKS_B4 = sorted(set(
    [(x, y, z) for x in (0, 1) for (y, z) in ((1, 1), (2, 1), (1, 2), (2, 2), (1, 3))]
    + [(x, y, z) for x in (0, 1) for y in (-1, 0) for z in (2, 3)]
    + [(0, 1, 2), (0, 1, 3)]))
assert len(BODY_BLOCKS_B4) == 18


def _body_blocks_pins(fn):
    """Every pin of D_body for a candidate implementation fn(X, kernel, B):
    the hand-worked set above, coverage of every support cell's neighbours, and
    minimality (each block holds a cell within one cell of a support cell)."""
    got = sorted(set(map(tuple, fn(BODY_MARKERS, ROMA3, 4).tolist())))
    assert got == BODY_BLOCKS_B4, "hand-worked D_body differs"
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    for B in (4, 8):
        blocks = {tuple(b) for b in fn(X, ROMA3, B).tolist()}
        sc = oracle.support_cells(X, ROMA3)
        near = {tuple(c) for d in np.ndindex(3, 3, 3) for c in (sc + (np.array(d) - 1)).tolist()}
        need = {tuple(np.floor_divide(c, B)) for c in near}
        assert need <= blocks, "a support cell's neighbour is outside D_body"
        assert blocks <= need, "D_body holds a block with no cell near the support"


def test_body_blocks_cover_support_with_margin(small_sphere):
    """D_body holds every cell within one cell of a delta support cell (Sec. 4.1)."""
    X, blocks, origin, mask, _, _ = small_sphere
    sc = oracle.support_cells(X, ROMA3)
    bset = {tuple(b) for b in blocks}
    for d in np.ndindex(3, 3, 3):
        for c in sc + (np.array(d) - 1):
            assert tuple(np.floor_divide(c, 8)) in bset


def test_body_blocks_hand_worked_and_minimal():
    """D_body (Sec. 4.1) equals the hand-worked two-marker set and holds no
    block without a cell next to the support."""
    _body_blocks_pins(oracle.body_blocks)


def _planted_double_dilation(X, kernel, B):
    sc = oracle.support_cells(X, kernel)
    cells = {tuple(c) for d in np.ndindex(5, 5, 5) for c in (sc + (np.array(d) - 2)).tolist()}
    return np.array(sorted({tuple(np.floor_divide(c, B)) for c in cells}), dtype=np.int64)


def _planted_axis_product(X, kernel, B):
    """Per-axis block ranges multiplied out: a superset of the union over k."""
    sc = oracle.support_cells(X, kernel)
    out = set()
    for i in range(X.shape[0]):
        one = oracle.support_cells(X[i:i + 1], kernel)
        ax = [sorted({int(np.floor_divide(v + d, B)) for v in one[:, j] for d in (-1, 0, 1)}) for j in range(3)]
        out |= {(a, b, c) for a in ax[0] for b in ax[1] for c in ax[2]}
    return np.array(sorted(out), dtype=np.int64)


def _planted_no_dilation(X, kernel, B):
    sc = oracle.support_cells(X, kernel)
    return np.array(sorted({tuple(np.floor_divide(c, B)) for c in sc.tolist()}), dtype=np.int64)


@pytest.mark.parametrize("planted", [_planted_double_dilation, _planted_axis_product, _planted_no_dilation])
def test_body_blocks_pins_reject_planted_mistakes(planted):
    """The pins above fail for a dilation by two cells, for per-axis ranges
    multiplied out, and for no dilation at all."""
    with pytest.raises(AssertionError):
        _body_blocks_pins(planted)


def test_schur_symmetric_positive_definite(small_sphere):
    """For a rigid body the force Schur complement is symmetric positive
    definite (Sec. 3.2), built column by column from basis vectors."""
    X, blocks, origin, mask, alpha, gk = small_sphere
    C = oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    asym = np.max(np.abs(C - C.T)) / np.max(np.abs(C))
    assert asym < 1e-12
    ev = np.linalg.eigvalsh(0.5 * (C + C.T))
    assert ev.min() > 0.0
    # Cholesky solve (the paper's pre-processing) reproduces a known solution
    xs = np.random.Generator(np.random.PCG64(2)).standard_normal(C.shape[0])
    L = np.linalg.cholesky(C)
    sol = np.linalg.solve(L.T, np.linalg.solve(L, C @ xs))
    assert np.max(np.abs(sol - xs)) < 1e-8 * np.max(np.abs(xs)) * ev.max() / ev.min()


def test_schur_rows_match_full_matvec(small_sphere):
    """The sampled-row evaluation used at full size equals the full matvec."""
    X, blocks, origin, mask, alpha, gk = small_sphere
    x = np.random.Generator(np.random.PCG64(4)).standard_normal(X.shape)
    full = oracle.schur_matvec(x, X, ROMA3, alpha, gk, mask, origin)
    rows = [0, 7, 31, 59]
    part = oracle.schur_matvec_rows(x, X, ROMA3, alpha, gk, mask, origin, rows)
    assert np.max(np.abs(part - full[rows])) < 1e-13 * np.max(np.abs(full))


def test_stokes_step_noslip_and_divergence_free(small_sphere):
    """One nested-projection step of the Stokes driver (Sec. 3.1) enforces the
    no-slip constraint I u' = u_B at the markers and leaves u' discretely
    divergence-free wherever neither the projection nor E(a) reaches the
    edge of the flow box (G^T u' = 0 there); a body at rest in fluid at rest
    stays at rest."""
    X, blocks, origin, mask, alpha, gk = small_sphere
    C = oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    fmask = np.ones((24, 24, 24), dtype=bool)
    forigin = np.zeros(3, dtype=np.int64)
    gl = oracle.lgf_table(24, 24, 24)
    g = np.random.Generator(np.random.PCG64(12))
    ub = np.zeros(X.shape)
    ub[:, 1] = 0.3
    u = np.zeros((3,) + fmask.shape)
    u, f = oracle.stokes_if_euler_step(u, X, ub, ROMA3, alpha, gl, C, fmask, forigin)
    v = oracle.interpolate(X, u, ROMA3, forigin)
    assert np.max(np.abs(v - ub)) < 1e-10
    r = oracle.if_radius(alpha) + 2
    div = oracle.grad_adjoint(u)[r:-r, r:-r, r:-r]
    assert np.max(np.abs(div)) < 1e-11 * np.max(np.abs(u))
    assert np.max(np.abs(f)) > 0.01
    # second step from a state with a random, not solenoidal, part: the
    # projection removes its divergence
    ub2 = ub * 0.5 + g.standard_normal(X.shape) * 1e-3
    u2, f2 = oracle.stokes_if_euler_step(u + 0.1 * g.standard_normal(u.shape), X, ub2, ROMA3, alpha, gl, C, fmask,
                                         forigin)
    assert np.max(np.abs(oracle.interpolate(X, u2, ROMA3, forigin) - ub2)) < 1e-10
    div2 = oracle.grad_adjoint(u2)[r:-r, r:-r, r:-r]
    assert np.max(np.abs(div2)) < 1e-11 * np.max(np.abs(u2))
    # rest stays rest
    u0, f0 = oracle.stokes_if_euler_step(np.zeros_like(u), X, np.zeros(X.shape), ROMA3, alpha, gl, C, fmask,
                                         forigin)
    assert np.max(np.abs(u0)) == 0.0 and np.max(np.abs(f0)) == 0.0


def test_stokes_step_energy_decays_with_body_at_rest(small_sphere):
    """With the body at rest each step is a projection onto divergence-free
    fields that satisfy no-slip, followed by the contraction E(a) and the
    restriction to the flow set, so the discrete kinetic energy cannot grow
    (Sec. 3.1; E(a) has symbol exp(a sigma) <= 1).  A random start loses
    energy every step and no-slip holds after each."""
    X, blocks, origin, mask, alpha, gk = small_sphere
    C = oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    fmask = np.ones((24, 24, 24), dtype=bool)
    forigin = np.zeros(3, dtype=np.int64)
    gl = oracle.lgf_table(24, 24, 24)
    u = np.random.Generator(np.random.PCG64(13)).standard_normal((3,) + fmask.shape)
    n0 = np.linalg.norm(u)
    for _ in range(3):
        u, f = oracle.stokes_if_euler_step(u, X, np.zeros(X.shape), ROMA3, alpha, gl, C, fmask, forigin)
        n1 = np.linalg.norm(u)
        assert n1 < n0
        assert np.max(np.abs(oracle.interpolate(X, u, ROMA3, forigin))) < 1e-12 * n1
        n0 = n1


def test_force_smoothing_keeps_constants_and_is_symmetric(small_sphere):
    """f^ = I W R f: a uniform force is returned unchanged (I reproduces the
    constant 1 wherever gamma = R 1 is positive), the operator is symmetric
    (<x, S y> = <S x, y>, since I = R^T and W is diagonal), and it damps an
    alternating marker pattern."""
    X, blocks, origin, mask, _, _ = small_sphere
    c = np.array([0.3, -1.2, 2.5])
    f = np.tile(c, (X.shape[0], 1))
    got = oracle.force_smooth(X, f, ROMA3, mask, origin)
    assert np.max(np.abs(got - f)) < 1e-13
    g = np.random.Generator(np.random.PCG64(9))
    x, y = g.standard_normal(X.shape), g.standard_normal(X.shape)
    sx, sy = oracle.force_smooth(X, x, ROMA3, mask, origin), oracle.force_smooth(X, y, ROMA3, mask, origin)
    assert abs(np.sum(x * sy) - np.sum(sx * y)) < 1e-12 * np.sum(np.abs(x * sy))
    alt = np.where(np.arange(X.shape[0])[:, None] % 2 == 0, 1.0, -1.0) * np.ones((1, 3))
    assert np.linalg.norm(oracle.force_smooth(X, alt, ROMA3, mask, origin)) < np.linalg.norm(alt)
