"""GPU parity of the rotational nonlinear term (Sec. 2.1) and of the IF-HERK
step that carries it (Sec. 2.3, Eq. ibifherk_g) against the FP64 oracle
through the C ABI.

Bars: the stencil in FP64 <= 1e-13 and in FP32 <= 1e-5 (relative max-norm
per component); the HERK steps <= 1e-9 (velocity) and 1e-8 (forces), as for
the Stokes steps."""
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


def _rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _to_box(field, blocks, B, origin, shape):
    box = np.zeros((3,) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def _from_box(box, blocks, B, origin):
    out = np.zeros((3, len(blocks), B, B, B))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        out[:, i] = box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B]
    return out


def _ragged(seed, B):
    g = np.random.Generator(np.random.PCG64(seed))
    allb = np.array(list(np.ndindex(4, 3, 5)), dtype=np.int32)[:, ::-1] + np.array([-1, 2, 0], dtype=np.int32)
    return allb[np.sort(g.choice(len(allb), len(allb) - 11, replace=False))]


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-13), (np.float32, 1e-5)])
@pytest.mark.parametrize("B", [4, 8])
def test_lamb_vector_matches_oracle(ctx, dtype, tol, B):
    blocks = _ragged(40 + B, B)
    U = (0.3, -0.2, 0.7)
    u = np.random.Generator(np.random.PCG64(B)).standard_normal((3, len(blocks), B, B, B))
    u = u.astype(dtype).astype(np.float64)
    ud = torch.from_numpy(u.astype(dtype)).cuda()
    out = torch.empty_like(ud)
    lg.lgf_lamb_vector(ctx, B, blocks, ud, out, U)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    origin, mask = oracle.block_mask(blocks, B)
    ref = _from_box(oracle.lamb_vector(_to_box(u, blocks, B, origin, mask.shape), U), blocks, B, origin)
    for c in range(3):
        assert _rel(got[c], ref[c]) < tol, c


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-13), (np.float32, 1e-5)])
@pytest.mark.parametrize("B", [16, 32])
def test_lamb_vector_large_blocks(ctx, dtype, tol, B):
    """Blocks of 16^3 and 32^3 (several workgroups per block), a small
    L-shaped set, against the oracle on every face."""
    blocks = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, -1]], dtype=np.int32)
    U = (-0.2, 0.4, 0.1)
    u = np.random.Generator(np.random.PCG64(B + 1)).standard_normal((3, len(blocks), B, B, B))
    u = u.astype(dtype).astype(np.float64)
    ud = torch.from_numpy(u.astype(dtype)).cuda()
    out = torch.empty_like(ud)
    lg.lgf_lamb_vector(ctx, B, blocks, ud, out, U)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    origin, mask = oracle.block_mask(blocks, B)
    ref = _from_box(oracle.lamb_vector(_to_box(u, blocks, B, origin, mask.shape), U), blocks, B, origin)
    for c in range(3):
        assert _rel(got[c], ref[c]) < tol, c


def test_lamb_vector_does_no_work_on_the_gpu(ctx):
    B = 8
    blocks = _ragged(9, B)
    u = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).standard_normal((3, len(blocks), B, B, B))).cuda()
    out = torch.empty_like(u)
    lg.lgf_lamb_vector(ctx, B, blocks, u, out)
    assert abs(float((u * out).sum())) < 1e-12 * float((u.abs() * out.abs()).sum())


def test_lamb_vector_argument_checks(ctx):
    B = 4
    blocks = workloads.cube_blocks(2)
    u = torch.zeros((3, len(blocks), B, B, B), dtype=torch.float64, device="cuda")
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_lamb_vector(ctx, B, blocks, u, u)
    assert e.value.code == lg.LGFIB_EINVAL
    dup = np.concatenate([blocks, blocks[:1]])
    u2 = torch.zeros((3, len(dup), B, B, B), dtype=torch.float64, device="cuda")
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_lamb_vector(ctx, B, dup, u2, torch.zeros_like(u2))
    assert e.value.code == lg.LGFIB_EDUP_BLOCK


@pytest.fixture(scope="module")
def case():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    B = 8
    blocks = oracle.body_blocks(X, ROMA3, B)
    flow = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    return X, B, blocks, flow


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


@pytest.mark.parametrize("scheme,direct", [("A", True), ("D", True), ("A", False)])
def test_navier_stokes_herk_steps_match_oracle(ctx, case, scheme, direct):
    """Two steps with the nonlinear term (dt / dx = 0.4, a frame velocity)
    from a random field with a moving body, against the oracle's step."""
    X, B, blocks, flow = case
    A, dtc, U = 0.05, 0.4, (0.25, 0.0, -0.1)
    at, ct = lg.ib_herk_tableau(scheme)
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, blocks, flow, A, at, ct, direct=direct)
    lg.ib_herk_convection(ctx, hk, dtc, U)
    forigin, fmask = oracle.block_mask(flow, B)
    gl = oracle.lgf_table(*np.array(fmask.shape[::-1]))
    Cs = _stage_C(X, blocks, B, A, ct)
    g = np.random.Generator(np.random.PCG64(13))
    ubox = g.standard_normal((3,) + fmask.shape) * fmask[None]
    u = torch.from_numpy(_from_box(ubox, flow, B, forigin)).cuda()
    for k in range(2):
        ubs = np.zeros((len(ct), len(X), 3))
        for i, c in enumerate(ct):
            ubs[i, :, 1] = 0.3 * math.sin(0.4 * (k + c))
        f = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
        lg.ib_herk_step(ctx, hk, u, torch.from_numpy(ubs).cuda(), f, rtol=1e-12, maxit=4000, prec=lg.LGF_F64)
        ubox, fref = oracle.stokes_ifherk_step(ubox, X, list(ubs), ROMA3, A, at, ct, gl, Cs, fmask, forigin,
                                               dt=dtc, frame_velocity=U)
        got = _to_box(u.cpu().numpy(), flow, B, forigin, fmask.shape)
        assert _rel(got, ubox) < 1e-9, (k, scheme, direct)
        assert _rel(f.cpu().numpy(), fref) < 1e-8, (k, scheme, direct)
    # the term matters at this step size: the Stokes step differs
    lg.ib_herk_convection(ctx, hk, 0.0)
    u2 = torch.from_numpy(_from_box(ubox, flow, B, forigin)).cuda()
    u3 = u2.clone()
    ubs_t = torch.from_numpy(ubs).cuda()
    f = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
    lg.ib_herk_step(ctx, hk, u2, ubs_t, f, rtol=1e-12, maxit=4000, prec=lg.LGF_F64)
    lg.ib_herk_convection(ctx, hk, dtc, U)
    lg.ib_herk_step(ctx, hk, u3, ubs_t, f, rtol=1e-12, maxit=4000, prec=lg.LGF_F64)
    assert _rel(u3.cpu().numpy(), u2.cpu().numpy()) > 1e-3
    hk.close()


def test_lamb_vector_plate_wake_full_size(ctx):
    """The 1272-block plate-and-wake set, blocks of 16^3, FP32: the launch
    configuration the benchmark times, against the oracle on every face."""
    B = 16
    blocks = workloads.plate_blocks(B)
    u = workloads.plate_sources(blocks, B, ncomp=3).astype(np.float32)
    U = (0.1, 0.0, 0.0)
    ud = torch.from_numpy(u).cuda()
    out = torch.empty_like(ud)
    lg.lgf_lamb_vector(ctx, B, blocks, ud, out, U)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    origin, mask = oracle.block_mask(blocks, B)
    ref = _from_box(oracle.lamb_vector(_to_box(u.astype(np.float64), blocks, B, origin, mask.shape), U),
                    blocks, B, origin)
    for c in range(3):
        assert _rel(got[c], ref[c]) < 1e-5, c


def test_navier_stokes_step_at_full_size_meets_the_constraints(ctx):
    """Config 5 at full size (sphere of diameter 32 with 2200 markers, 1728
    flow blocks of 8^3, a = 0.05, dt / dx = 1): after each Scheme A step with
    the nonlinear term the velocity interpolated to the markers is the body
    velocity and the interior of the flow set is discretely divergence-free,
    properties the oracle's operators check at any size."""
    X = workloads.sphere_markers(32.0, 2200)
    B = 8
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    flow = np.array([(x, y, z) for z in range(-1, 11) for y in range(-1, 11) for x in range(-1, 11)], dtype=np.int32)
    at, ct = lg.ib_herk_tableau("A")
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, blocks, flow, 0.05, at, ct, direct=True)
    lg.ib_herk_convection(ctx, hk, 1.0, (0.05, 0.0, 0.0))
    origin, fmask = oracle.block_mask(flow, B)
    inner = np.zeros_like(fmask)
    inner[1:-1, 1:-1, 1:-1] = True
    u = torch.zeros((3, len(flow), B, B, B), dtype=torch.float64, device="cuda")
    f = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
    for k in range(3):
        ubs = np.zeros((len(ct), len(X), 3))
        for i, c in enumerate(ct):
            ubs[i, :, 1] = workloads.heave_velocity(k + c, 32.0)
        lg.ib_herk_step(ctx, hk, u, torch.from_numpy(ubs).cuda(), f)
        ubox = _to_box(u.cpu().numpy(), flow, B, origin, fmask.shape)
        v = oracle.interpolate(X, ubox, ROMA3, origin)
        assert np.max(np.abs(v - ubs[-1])) < 1e-9 * max(1e-3, np.max(np.abs(ubs[-1]))), k
        div = oracle.grad_adjoint(ubox)
        assert np.max(np.abs(div[inner])) < 1e-10 * np.max(np.abs(ubox)), k
    assert float(u.abs().max()) > 0.0
    hk.close()
