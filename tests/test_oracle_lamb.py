"""Pins of the oracle's nonlinear term in rotational form, N~ = (C u) x u_a
(Sec. 2.1), and of the IF-HERK step carrying it (Sec. 2.3, Eq. ibifherk_g).

What fixes them, independently of the code under test:
- a rigid rotation (a linear field) gets the exact Lamb vector, with and
  without a frame velocity;
- a potential flow (u = G q) has no vorticity, so N~ = 0;
- the stencil does no work: sum u . N~(u) = 0 for any u (frame velocity 0);
- on a smooth field the stencil converges to (curl u) x u at second order;
- with exact operators the HERK step keeps its orders on a constrained
  system with a quadratic nonlinearity.
"""
import numpy as np
import pytest

import oracle


def _rand(shape, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


@pytest.mark.parametrize("U", [(0.0, 0.0, 0.0), (0.3, -0.7, 0.2)])
def test_rigid_rotation_gets_the_exact_lamb_vector(U):
    nz, ny, nx = 7, 8, 9
    om = 0.41
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[0] = -om * (y + 0.5)          # face x of cell n at (n_x, n_y + 1/2, n_z + 1/2)
    u[1] = om * (x + 0.5)           # face y at (n_x + 1/2, n_y, n_z + 1/2)
    N = oracle.lamb_vector(u, U)
    # (0, 0, 2 om) x (u + U) at each face's position
    want_x = -2 * om * (om * x + U[1])
    want_y = 2 * om * (-om * y + U[0])
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.max(np.abs(N[0][inner] - want_x[inner])) < 1e-13
    assert np.max(np.abs(N[1][inner] - want_y[inner])) < 1e-13
    assert np.max(np.abs(N[2][inner])) < 1e-13


def test_box_edges_do_not_truncate_the_term():
    """u is zero outside the box: the result equals that of the same field
    placed in a larger zero box (faces on the upper side take the edges one
    cell beyond, where w and u_a are not zero)."""
    u = _rand((3, 6, 7, 8), 3)
    U = (0.3, -0.2, 0.7)
    big = np.zeros((3, 10, 11, 12))
    big[:, 2:8, 2:9, 2:10] = u
    ref = oracle.lamb_vector(big, U)[:, 2:8, 2:9, 2:10]
    assert np.max(np.abs(oracle.lamb_vector(u, U) - ref)) < 1e-14


def test_potential_flow_has_no_lamb_vector():
    q = _rand((9, 10, 11), 1)
    N = oracle.lamb_vector(oracle.grad(q), (0.2, 0.1, -0.4))
    assert np.max(np.abs(N[:, 2:-2, 2:-2, 2:-2])) < 1e-13


def test_the_term_does_no_work():
    u = _rand((3, 8, 9, 10), 2)
    N = oracle.lamb_vector(u)
    assert abs(np.sum(u * N)) < 1e-12 * np.sum(np.abs(u) * np.abs(N))
    # a non-zero frame velocity does work in general
    N = oracle.lamb_vector(u, (0.5, 0.0, 0.0))
    assert abs(np.sum(u * N)) > 1e-3


def _smooth_error(h):
    n = int(round(2.0 / h))
    idx = np.arange(n)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = [x * h, y * h, z * h]
    half = 0.5 * h

    def field(px, py, pz):
        return (np.sin(py) * np.cos(pz), np.sin(pz) * np.cos(px), np.sin(px) * np.cos(py))

    def lamb(px, py, pz):
        ux, uy, uz = field(px, py, pz)
        wx = -np.sin(px) * np.sin(py) - np.cos(pz) * np.cos(px)
        wy = -np.sin(py) * np.sin(pz) - np.cos(px) * np.cos(py)
        wz = -np.sin(pz) * np.sin(px) - np.cos(py) * np.cos(pz)
        return (wy * uz - wz * uy, wz * ux - wx * uz, wx * uy - wy * ux)

    u = np.zeros((3, n, n, n))
    want = np.zeros((3, n, n, n))
    for k in range(3):   # face k of cell n at n + (1,1,1)/2 - e_k/2, times h
        p = [pos[a] + (0.0 if a == k else half) for a in range(3)]
        u[k] = field(*p)[k]
        want[k] = lamb(*p)[k]
    N = oracle.lamb_vector(u) / h
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    return np.max(np.abs(N[inner] - want[inner]))


def test_second_order_on_a_smooth_field():
    e1, e2 = _smooth_error(0.1), _smooth_error(0.05)
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def _dense_dae(n=8, m=2, seed=5):
    from scipy.linalg import expm
    g = np.random.Generator(np.random.PCG64(seed))
    M = g.standard_normal((n, n))
    L = -(M @ M.T / n + np.eye(n))
    Q = g.standard_normal((n, m))
    B1 = 0.3 * g.standard_normal((n, n))
    B2 = 0.3 * g.standard_normal((n, n))

    def zeta(t):
        return np.array([np.sin(1.3 * t), np.cos(0.7 * t) - 1.0])

    def nonlinear(u):
        return (B1 @ u) * (B2 @ u)

    def propagate(a, x):
        return expm(a * L) @ x

    def make_stage(ts):
        def stage_solve(i, a, r):
            Hinv = expm(-a * L)
            K = np.block([[Hinv, Q], [Q.T, np.zeros((m, m))]])
            sol = np.linalg.solve(K, np.concatenate([r, zeta(ts[i])]))
            return sol[:n], sol[n:], Q @ sol[n:]
        return stage_solve
    return Q, zeta, nonlinear, propagate, make_stage


def _integrate(scheme, nsteps, T=1.0):
    """u' = L u - N(u) - Q z, Q^T u = zeta(t) with exact operators."""
    Q, zeta, nonlinear, propagate, make_stage = _dense_dae()
    at, ct = oracle.herk_tableau(scheme)
    dt = T / nsteps
    u = Q @ np.linalg.solve(Q.T @ Q, zeta(0.0)) + 0.5
    u = u - Q @ np.linalg.solve(Q.T @ Q, Q.T @ u - zeta(0.0))
    for k in range(nsteps):
        ts = [(k + c) * dt for c in ct]
        u, lam = oracle.herk_step(u, propagate, make_stage(ts), at, ct, dt, nonlinear, dt)
    return u, lam / dt


@pytest.mark.parametrize("scheme,pu,pz", [("A", 2, 2), ("B", 3, 2), ("C", 2, 1)])
def test_herk_orders_with_a_nonlinear_term(scheme, pu, pz):
    ref_u, ref_z = _integrate(scheme, 512)
    eu, ez = [], []
    for n in (8, 16, 32):
        u, z = _integrate(scheme, n)
        eu.append(np.max(np.abs(u - ref_u)))
        ez.append(np.max(np.abs(z - ref_z)))
    ru = [np.log2(eu[i] / eu[i + 1]) for i in range(2)]
    rz = [np.log2(ez[i] / ez[i + 1]) for i in range(2)]
    assert min(ru) > pu - 0.3, (scheme, eu, ru)
    assert min(rz) > pz - 0.3, (scheme, ez, rz)


def test_a_wrong_nonlinear_stage_argument_loses_the_order():
    """The order test can tell: evaluating N at the start of the step in every
    stage (instead of at the previous stage's u) drops Scheme B to first
    order."""
    Q, zeta, nonlinear, propagate, make_stage = _dense_dae()
    at, ct = oracle.herk_tableau("B")

    def run(nsteps):
        dt = 1.0 / nsteps
        u = Q @ np.linalg.solve(Q.T @ Q, zeta(0.0)) + 0.5
        u = u - Q @ np.linalg.solve(Q.T @ Q, Q.T @ u - zeta(0.0))
        for k in range(nsteps):
            ts = [(k + c) * dt for c in ct]
            u0 = u.copy()
            u, _ = oracle.herk_step(u, propagate, make_stage(ts), at, ct, dt, lambda _x: nonlinear(u0), dt)
        return u
    ref = run(512)
    e = [np.max(np.abs(run(n) - ref)) for n in (16, 32)]
    assert np.log2(e[0] / e[1]) < 1.5
