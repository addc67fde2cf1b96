"""GPU parity of the IF-HERK step of the Stokes driver (Sec. 2.3, App. B)
against the FP64 oracle through the C ABI: the tableaus, the one-stage
tableau as the integrating-factor Euler step, and Schemes A, B and D against
the oracle's step.  (The orders of the scheme itself are pinned on the oracle
with exact operators; on a finite flow set the restricted operators add a
first-order term, so the lattice runs are not an order test.)"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.ib import ROMA3

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def case():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    B = 8
    blocks = oracle.body_blocks(X, ROMA3, B)
    flow = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    return X, B, blocks, flow


def _rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _blocks_to_box(field, blocks, B, origin, shape):
    box = np.zeros((field.shape[0],) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def _box_to_blocks(box, blocks, B, origin):
    out = np.zeros((box.shape[0], len(blocks), B, B, B))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        out[:, i] = box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B]
    return out


def test_tableau_matches_oracle():
    for name in "ABCD":
        at, ct = lg.ib_herk_tableau(name)
        at_o, ct_o = oracle.herk_tableau(name)
        assert np.allclose(at, at_o, rtol=0, atol=1e-15) and np.allclose(ct, ct_o, rtol=0, atol=1e-15)


def test_one_stage_tableau_is_the_flow_step(ctx, case):
    X, B, blocks, flow = case
    a = 0.05
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, blocks, flow, a, np.ones((1, 1)), np.ones(1), direct=True)
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, a)
    lg.ib_system_factor(ctx, sys)
    fl = lg.ib_flow_create(ctx, sys, flow)
    g = np.random.Generator(np.random.PCG64(2))
    u0 = torch.from_numpy(g.standard_normal((3, len(flow), B, B, B))).cuda()
    u1, u2 = u0.clone(), u0.clone()
    for k in range(2):
        ub = torch.zeros((1, len(X), 3), dtype=torch.float64, device="cuda")
        ub[0, :, 1] = 0.2 + 0.1 * k
        f1 = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
        f2 = torch.zeros_like(f1)
        lg.ib_herk_step(ctx, hk, u1, ub, f1)
        lg.ib_flow_step(ctx, fl, u2, ub[0], f2, prec=lg.IB_SOLVE_DIRECT)
        assert torch.equal(u1, u2) and torch.equal(f1, f2)
    fl.close()
    sys.close()
    hk.close()


def _stage_C(X, blocks, B, A, ct):
    origin, mask = oracle.block_mask(blocks, B)
    cache, out, prev = {}, [], 0.0
    for c in ct:
        al = round((c - prev) * A, 14)
        if al not in cache:
            gk = oracle.lgf_k_table(al, *np.array(mask.shape[::-1]))
            cache[al] = oracle.schur_dense(X, ROMA3, al, gk, mask, origin)
        out.append(cache[al])
        prev = c
    return out


@pytest.mark.parametrize("scheme,direct", [("A", True), ("A", False), ("D", True), ("B", True)])
def test_herk_steps_match_oracle(ctx, case, scheme, direct):
    """Two steps from a random field with a moving body, against the oracle's
    step (dense Cholesky force solves): Scheme A (two distinct integrating
    factors, one the identity), D (four stages, identity stages in between)
    and B (three distinct factors), with direct and CG force solves."""
    X, B, blocks, flow = case
    A = 0.05
    at, ct = lg.ib_herk_tableau(scheme)
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, blocks, flow, A, at, ct, direct=direct)
    forigin, fmask = oracle.block_mask(flow, B)
    gl = oracle.lgf_table(*np.array(fmask.shape[::-1]))
    Cs = _stage_C(X, blocks, B, A, ct)
    g = np.random.Generator(np.random.PCG64(3))
    ubox = g.standard_normal((3,) + fmask.shape) * fmask[None]
    u = torch.from_numpy(_box_to_blocks(ubox, flow, B, forigin)).cuda()
    for k in range(2):
        ubs = np.zeros((len(ct), len(X), 3))
        for i, c in enumerate(ct):
            ubs[i, :, 1] = 0.3 * math.sin(0.4 * (k + c))
        f = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
        st = lg.ib_herk_step(ctx, hk, u, torch.from_numpy(ubs).cuda(), f, rtol=1e-12, maxit=4000, prec=lg.LGF_F64)
        ubox, fref = oracle.stokes_ifherk_step(ubox, X, list(ubs), ROMA3, A, at, ct, gl, Cs, fmask, forigin)
        got = _blocks_to_box(u.cpu().numpy(), flow, B, forigin, fmask.shape)
        assert _rel(got, ubox) < 1e-9, (k, scheme, direct)
        assert _rel(f.cpu().numpy(), fref) < 1e-8, (k, scheme, direct)
        if direct:
            assert st["iterations"] == 0
    hk.close()
