"""Pins of the oracle's IF-HERK step (Sec. 2.3, App. B): the transcribed
tableaus satisfy the classical order conditions of the orders the paper
lists for problems without an immersed surface, the one-stage tableau
reproduces the integrating-factor Euler step, and a Scheme A step of the
Stokes driver meets the no-slip and divergence constraints at its end.
CPU only."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.ib import ROMA3

ODE_ORDER = {"A": 2, "B": 3, "C": 3, "D": 4}


def _unshift(at, ct):
    s = len(ct)
    A = np.zeros((s, s))
    A[1:] = at[:s - 1]
    return A, at[s - 1], np.concatenate([[0.0], ct[:s - 1]])


@pytest.mark.parametrize("name", "ABCD")
def test_tableau_order_conditions(name):
    at, ct = oracle.herk_tableau(name)
    A, b, c = _unshift(at, ct)
    p = ODE_ORDER[name]
    assert np.allclose(A.sum(1), c, atol=1e-15)          # row sums give the nodes
    assert np.allclose(np.tril(A, -1), A)                 # explicit
    conds = [(b.sum(), 1.0), (b @ c, 0.5)]
    if p >= 3:
        conds += [(b @ c ** 2, 1 / 3), (b @ A @ c, 1 / 6)]
    if p >= 4:
        conds += [(b @ c ** 3, 1 / 4), (b @ (c * (A @ c)), 1 / 8), (b @ A @ c ** 2, 1 / 12), (b @ A @ A @ c, 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 1e-14, (name, got, want)
    if p == 2:   # Scheme A is exactly second order: the third-order condition fails
        assert abs(b @ c ** 2 - 1 / 3) > 1e-3


def test_distinct_integrating_factors():
    """Schemes A and D need two distinct integrating factors, one of them the
    identity; B and C need three (App. B)."""
    for name, n in (("A", 2), ("B", 3), ("C", 3), ("D", 2)):
        _, ct = oracle.herk_tableau(name)
        steps = np.round(np.diff(np.concatenate([[0.0], ct])), 12)
        assert len(set(steps)) == n, name
        if name in "AD":
            assert 0.0 in set(steps)


@pytest.fixture(scope="module")
def tiny():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    B = 8
    blocks = oracle.body_blocks(X, ROMA3, B)
    origin, mask = oracle.block_mask(blocks, B)
    flow = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    forigin, fmask = oracle.block_mask(flow, B)
    gl = oracle.lgf_table(*np.array(fmask.shape[::-1]))

    def C_of(alpha):
        gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
        return oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    return X, flow, forigin, fmask, gl, C_of


def test_one_stage_tableau_is_the_euler_step(tiny):
    X, flow, forigin, fmask, gl, C_of = tiny
    a = 0.05
    C = C_of(a)
    g = np.random.Generator(np.random.PCG64(4))
    u = g.standard_normal((3,) + fmask.shape) * fmask[None]
    ub = np.zeros(X.shape)
    ub[:, 1] = 0.2
    ue, fe = oracle.stokes_if_euler_step(u, X, ub, ROMA3, a, gl, C, fmask, forigin)
    uh, fh = oracle.stokes_ifherk_step(u, X, [ub], ROMA3, a, np.ones((1, 1)), np.ones(1), gl, [C], fmask, forigin)
    assert np.array_equal(ue, uh) and np.array_equal(fe, fh)


def test_scheme_a_step_meets_the_constraints(tiny):
    """After a Scheme A step the velocity is discretely divergence free on the
    interior of the flow set and interpolates to the marker velocity at
    t_{k+1} (the last stage's constraint equations)."""
    X, flow, forigin, fmask, gl, C_of = tiny
    A = 0.05
    at, ct = oracle.herk_tableau("A")
    Cs = {}
    stage_C = []
    prev = 0.0
    for c in ct:
        al = round((c - prev) * A, 14)
        if al not in Cs:
            Cs[al] = C_of(al)
        stage_C.append(Cs[al])
        prev = c
    assert len(Cs) == 2
    g = np.random.Generator(np.random.PCG64(6))
    u = g.standard_normal((3,) + fmask.shape) * fmask[None]
    ubs = []
    for c in ct:
        ub = np.zeros(X.shape)
        ub[:, 1] = 0.3 * np.sin(0.7 + c)
        ubs.append(ub)
    u1, f1 = oracle.stokes_ifherk_step(u, X, ubs, ROMA3, A, at, ct, gl, stage_C, fmask, forigin)
    v = oracle.interpolate(X, u1, ROMA3, forigin)
    assert np.max(np.abs(v - ubs[-1])) < 1e-10
    div = oracle.grad_adjoint(u1)
    inner = fmask.copy()
    inner[0, :, :] = inner[-1, :, :] = False
    inner[:, 0, :] = inner[:, -1, :] = False
    inner[:, :, 0] = inner[:, :, -1] = False
    assert np.max(np.abs(div[inner])) < 1e-10 * np.max(np.abs(u))


def _dense_dae(n=8, m=2, seed=5):
    """u' = L u - Q z, Q^T u = zeta(t) with a negative definite L: the linear
    index-2 system the IF-HERK scheme integrates, with exact operators
    (E(a) = expm(a L), stage systems solved densely)."""
    from scipy.linalg import expm
    g = np.random.Generator(np.random.PCG64(seed))
    M = g.standard_normal((n, n))
    L = -(M @ M.T / n + np.eye(n))
    Q = g.standard_normal((n, m))

    def zeta(t):
        return np.array([np.sin(1.3 * t), np.cos(0.7 * t) - 1.0])

    def propagate(a, x):
        return expm(a * L) @ x

    def make_stage(ts):
        def stage_solve(i, a, r):
            Hinv = expm(-a * L)
            K = np.block([[Hinv, Q], [Q.T, np.zeros((m, m))]])
            sol = np.linalg.solve(K, np.concatenate([r, zeta(ts[i])]))
            return sol[:n], sol[n:], Q @ sol[n:]
        return stage_solve
    return L, Q, zeta, propagate, make_stage


def _integrate(scheme, nsteps, T=1.0):
    L, Q, zeta, propagate, make_stage = _dense_dae()
    if scheme == "E":
        at, ct = np.ones((1, 1)), np.ones(1)
    else:
        at, ct = oracle.herk_tableau(scheme)
    dt = T / nsteps
    # consistent start: the minimal-norm u with Q^T u = zeta(0)
    u = Q @ np.linalg.solve(Q.T @ Q, zeta(0.0))
    for k in range(nsteps):
        ts = [(k + c) * dt for c in ct]
        u, lam = oracle.herk_step(u, propagate, make_stage(ts), at, ct, dt)
    return u, lam / dt


@pytest.mark.parametrize("scheme,pu,pz", [("E", 1, 1), ("A", 2, 2), ("B", 3, 2), ("C", 2, 1)])
def test_herk_orders_on_a_dense_linear_system(scheme, pu, pz):
    """With exact operators the step converges at the orders Table
    tab:ifherk_schemes lists for the velocity (y) and the constraint
    variables (z): errors against a 16x finer run fall by ~2^p per halving."""
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
