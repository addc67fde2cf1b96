"""GPU parity of the immersed-boundary operators (regularize, interpolate, body
blocks), the force Schur complement and the CG force solve against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.ib import ROMA3, SMOOTH3

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


def _relerr(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def _markers(seed, n, lo=20.0, hi=36.0):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, size=(n, 3))


def _box_to_blocks(box, origin, blocks, B):
    """Gather a dense face box [3, z, y, x] onto blocks -> [3, nblk, B, B, B]."""
    out = np.zeros((box.shape[0], len(blocks), B, B, B))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        out[:, i] = box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B]
    return out


@pytest.mark.parametrize("kernel", [ROMA3, SMOOTH3])
@pytest.mark.parametrize("B", [4, 8])
def test_body_blocks_bit_exact(kernel, B):
    X = _markers(1 + kernel, 40)
    got = lg.ib_body_blocks(kernel, X, B)
    ref = oracle.body_blocks(X, kernel, B)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("kernel", [ROMA3, SMOOTH3])
def test_regularize_interpolate(ctx, dtype, kernel):
    B = 8
    X = _markers(7, 50)
    blocks = oracle.body_blocks(X, kernel, B)
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((50, 3))
    origin, mask = oracle.block_mask(blocks, B)
    for dx in (1.0, 0.5):
        ref = _box_to_blocks(oracle.regularize(X, x, kernel, origin, mask.shape, dx=dx), origin, blocks, B)
        faces = torch.zeros((3, len(blocks), B, B, B), dtype=getattr(torch, np.dtype(dtype).name), device="cuda")
        lg.ib_regularize(ctx, kernel, X, B, blocks, torch.from_numpy(x.astype(dtype)).cuda(), faces, dx=dx)
        tol = 1e-13 if dtype == np.float64 else 1e-6
        assert _relerr(faces.cpu().numpy(), ref) < tol
    # interpolation of a random face field on the blocks
    u = rng.standard_normal((3, len(blocks), B, B, B))
    ubox = np.zeros((3,) + mask.shape)
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - origin
        ubox[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = u[:, i]
    ref = oracle.interpolate(X, ubox, kernel, origin)
    v = torch.zeros((50, 3), dtype=getattr(torch, np.dtype(dtype).name), device="cuda")
    lg.ib_interpolate(ctx, kernel, X, B, blocks, torch.from_numpy(u.astype(dtype)).cuda(), v)
    tol = 1e-13 if dtype == np.float64 else 1e-6
    assert _relerr(v.cpu().numpy(), ref) < tol


def test_support_outside_blocks_rejected(ctx):
    B = 8
    X = _markers(9, 10)
    blocks = oracle.body_blocks(X, ROMA3, B)[1:]   # drop one block
    faces = torch.zeros((3, len(blocks), B, B, B), dtype=torch.float64, device="cuda")
    x = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(lg.LgfibError) as e:
        lg.ib_regularize(ctx, ROMA3, X, B, blocks, x, faces)
    assert e.value.code == lg.LGFIB_ESUPPORT


@pytest.fixture(scope="module")
def small_sphere():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    B, alpha = 8, 0.05
    blocks = oracle.body_blocks(X, ROMA3, B)
    origin, mask = oracle.block_mask(blocks, B)
    gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
    C = oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    return X, B, alpha, blocks, origin, mask, gk, C


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_schur_matvec_small_sphere(ctx, small_sphere, dtype):
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    x = np.random.Generator(np.random.PCG64(5)).standard_normal(X.shape)
    tdt = getattr(torch, np.dtype(dtype).name)
    y = torch.zeros(X.shape, dtype=tdt, device="cuda")
    lg.ib_schur_apply(ctx, sys, torch.from_numpy(x.astype(dtype)).cuda(), y)
    ref = (C @ x.reshape(-1)).reshape(X.shape)
    assert _relerr(y.cpu().numpy(), ref) < (1e-12 if dtype == np.float64 else 1e-5)
    sys.close()


@pytest.mark.parametrize("prec", [lg.LGF_F64, lg.LGF_F32])
def test_force_solve_matches_cholesky(ctx, small_sphere, prec):
    """CG on the SPD Schur complement reaches 1e-8 relative residual (FP64 true
    residual) and agrees with the paper's dense Cholesky solve."""
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    b = np.random.Generator(np.random.PCG64(6)).standard_normal(X.shape)
    L = np.linalg.cholesky(C)
    ref = np.linalg.solve(L.T, np.linalg.solve(L, b.reshape(-1))).reshape(X.shape)
    bd = torch.from_numpy(b).cuda()
    f = torch.zeros_like(bd)
    st = lg.ib_force_solve(ctx, sys, bd, f, rtol=1e-8, maxit=500, prec=prec)
    assert st["converged"] and st["rel_residual"] <= 1e-8
    got = f.cpu().numpy()
    res = np.linalg.norm(b.reshape(-1) - C @ got.reshape(-1)) / np.linalg.norm(b)
    assert res < 2e-8
    kappa = np.linalg.cond(C)
    assert _relerr(got, ref) < 1e-8 * kappa
    # warm start at the solution: no iterations; NaN warm start falls back
    f2 = torch.zeros_like(bd)
    st2 = lg.ib_force_solve(ctx, sys, bd, f2, x0=torch.from_numpy(ref).cuda(), rtol=1e-8, prec=prec)
    assert st2["iterations"] == 0 and st2["fallback"] == 0
    bad = torch.full_like(bd, float("nan"))
    st3 = lg.ib_force_solve(ctx, sys, bd, f2, x0=bad, rtol=1e-8, maxit=500, prec=prec)
    assert st3["fallback"] == 1 and st3["converged"]
    sys.close()


def test_force_solve_reports_noconv(ctx, small_sphere):
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    bd = torch.from_numpy(np.random.Generator(np.random.PCG64(7)).standard_normal(X.shape)).cuda()
    f = torch.zeros_like(bd)
    with pytest.raises(lg.LgfibError) as e:
        lg.ib_force_solve(ctx, sys, bd, f, rtol=1e-12, maxit=2, prec=lg.LGF_F64)
    assert e.value.code == lg.LGFIB_ENOCONV
    sys.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_schur_matvec_sphere_full_size(ctx, dtype):
    """Sphere of diameter 32 cells with 4000 markers, blocks of 8^3, a = 0.05:
    rows of C x for 12 seeded markers against the oracle (full size)."""
    X = workloads.sphere_markers(32.0, 4000)
    B, alpha = 8, 0.05
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    x = np.random.Generator(np.random.PCG64(8)).standard_normal(X.shape)
    y = torch.zeros(X.shape, dtype=getattr(torch, np.dtype(dtype).name), device="cuda")
    lg.ib_schur_apply(ctx, sys, torch.from_numpy(x.astype(dtype)).cuda(), y)
    origin, mask = oracle.block_mask(blocks, B)
    gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
    rows = np.random.Generator(np.random.PCG64(9)).choice(4000, 12, replace=False)
    ref = oracle.schur_matvec_rows(x, X, ROMA3, alpha, gk, mask, origin, rows)
    got = y.cpu().numpy()[rows]
    assert _relerr(got, ref) < (1e-12 if dtype == np.float64 else 1e-5)
    sys.close()


@pytest.mark.parametrize("prec", [lg.LGF_F64, lg.LGF_F32])
def test_force_solve_listed_sphere(ctx, prec):
    """CG on the listed sphere (diameter 32, 4000 markers, 12,000 unknowns:
    the register-resident update for up to 16,384 unknowns, kappa ~3e4)
    reaches 1e-8, checked by the library's FP64 matvec in norm and by the
    oracle's rows of C f at 12 seeded markers."""
    X = workloads.sphere_markers(32.0, 4000)
    B, alpha = 8, 0.05
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    b = np.random.Generator(np.random.PCG64(10)).standard_normal(X.shape)
    bd = torch.from_numpy(b).cuda()
    f = torch.zeros_like(bd)
    st = lg.ib_force_solve(ctx, sys, bd, f, rtol=1e-8, maxit=30000, prec=prec)
    assert st["converged"] and st["rel_residual"] <= 1e-8
    y = torch.zeros_like(bd)
    lg.ib_schur_apply(ctx, sys, f, y)
    assert np.linalg.norm((bd - y).cpu().numpy()) / np.linalg.norm(b) < 2e-8
    origin, mask = oracle.block_mask(blocks, B)
    gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
    rows = np.random.Generator(np.random.PCG64(11)).choice(4000, 12, replace=False)
    cf = oracle.schur_matvec_rows(f.cpu().numpy(), X, ROMA3, alpha, gk, mask, origin, rows)
    assert np.max(np.abs(cf - b[rows])) < 1e-8 * np.linalg.norm(b)
    sys.close()


def _blocks_to_box(field, blocks, B, origin, shape):
    box = np.zeros((field.shape[0],) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def test_stokes_driver_steps_match_oracle(ctx, small_sphere):
    """Two integrating-factor Euler steps of the Stokes driver (nested
    projection, Sec. 3.1) on 3^3 flow blocks of 8^3 around a small sphere moving
    at a prescribed velocity, against the oracle's dense implementation."""
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    flow = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    forigin, fmask = oracle.block_mask(flow, B)
    gl = oracle.lgf_table(*np.array(fmask.shape[::-1]))
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    fl = lg.ib_flow_create(ctx, sys, flow)
    u = torch.zeros((3, len(flow), B, B, B), dtype=torch.float64, device="cuda")
    ubox = np.zeros((3,) + fmask.shape)
    for step, U in enumerate([0.3, 0.25]):
        ub = np.zeros(X.shape)
        ub[:, 1] = U
        f = torch.zeros(X.shape, dtype=torch.float64, device="cuda")
        st = lg.ib_flow_step(ctx, fl, u, torch.from_numpy(ub).cuda(), f, rtol=1e-11, maxit=2000, prec=lg.LGF_F64)
        assert st["converged"]
        ubox, fref = oracle.stokes_if_euler_step(ubox, X, ub, ROMA3, alpha, gl, C, fmask, forigin)
        got_u = _blocks_to_box(u.cpu().numpy(), flow, B, forigin, fmask.shape)
        assert _relerr(f.cpu().numpy(), fref) < 1e-8, step
        assert _relerr(got_u, ubox) < 1e-8, step
        # no-slip holds at the markers: I u' = u_B
        v = oracle.interpolate(X, got_u, ROMA3, forigin)
        assert np.max(np.abs(v - ub)) < 1e-8
    fl.close()
    sys.close()


@pytest.mark.parametrize("prec", [lg.LGF_F32, lg.LGF_F64])
def test_force_solve_graph_replay_matches_eager(ctx, small_sphere, prec, monkeypatch):
    """CG iterations replayed from captured HIP graphs give bit-identical
    iterates and iteration counts to the same kernels launched one by one,
    over repeated solves with eager work in between."""
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    g = np.random.Generator(np.random.PCG64(17))
    runs = []
    for mode in ("1", "0", "1", "0", "1"):
        monkeypatch.setenv("LGFIB_CG_GRAPH", mode)
        b = torch.from_numpy(g.standard_normal(X.shape)).cuda() if not runs else runs[0][0]
        f = torch.zeros_like(b)
        st = lg.ib_force_solve(ctx, sys, b, f, rtol=1e-9, maxit=1000, prec=prec)
        assert st["converged"]
        assert st["graphs"] == (1 if mode == "1" else 0)
        # eager work on the same stream between solves
        y = torch.zeros_like(b)
        lg.ib_schur_apply(ctx, sys, f, y)
        runs.append((b, f.cpu().numpy(), st["iterations"], y.cpu().numpy()))
    for b, f, its, y in runs[1:]:
        assert its == runs[0][2]
        assert np.array_equal(f, runs[0][1])
        assert np.array_equal(y, runs[0][3])
    sys.close()


def test_stokes_driver_energy_decays(ctx, small_sphere):
    """Body at rest, random initial velocity on 4^3 flow blocks: the GPU
    driver's steps are non-expansive (kinetic energy decreases every step)
    and keep no-slip at the markers."""
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    flow = np.array([(x, y, z) for z in range(4) for y in range(4) for x in range(4)], dtype=np.int32)
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    fl = lg.ib_flow_create(ctx, sys, flow)
    g = torch.Generator(device="cuda").manual_seed(3)
    u = torch.randn((3, len(flow), B, B, B), dtype=torch.float64, device="cuda", generator=g)
    ub = torch.zeros(X.shape, dtype=torch.float64, device="cuda")
    f = torch.zeros_like(ub)
    n0 = float(torch.linalg.vector_norm(u))
    forigin, fmask = oracle.block_mask(flow, B)
    for _ in range(5):
        st = lg.ib_flow_step(ctx, fl, u, ub, f, rtol=1e-10, maxit=3000, prec=lg.LGF_F64)
        assert st["converged"]
        n1 = float(torch.linalg.vector_norm(u))
        assert n1 < n0
        n0 = n1
    v = oracle.interpolate(X, _blocks_to_box(u.cpu().numpy(), flow, B, forigin, fmask.shape), ROMA3, forigin)
    assert np.max(np.abs(v)) < 1e-8 * n0
    fl.close()
    sys.close()


def test_force_smoothing_matches_oracle(ctx, small_sphere):
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    g = np.random.Generator(np.random.PCG64(12))
    for rep in range(2):   # the second call reuses gamma
        f = g.standard_normal(X.shape)
        out = torch.zeros(X.shape, dtype=torch.float64, device="cuda")
        fd = torch.from_numpy(f).cuda()
        lg.ib_force_smooth(ctx, sys, fd, out)
        ref = oracle.force_smooth(X, f, ROMA3, mask, origin)
        assert _relerr(out.cpu().numpy(), ref) < 1e-13
    lg.ib_force_smooth(ctx, sys, fd, fd)   # in place
    assert torch.equal(fd, out)
    sys.close()
