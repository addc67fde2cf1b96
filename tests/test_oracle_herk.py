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
