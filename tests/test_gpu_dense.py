"""GPU parity of the dense force solve (Sec. 3.2: C built column by column,
FP64 Cholesky factor and its inverse computed once, each solve two
triangular matrix-vector products) against the FP64 oracle, through the
C ABI.

Tolerance of the factor: the computed Cholesky factor of an SPD matrix
satisfies L L^T = C + dC with |dC| of order n eps |L||L^T|, which bounds the
forward error of L (and of its inverse) by about n eps kappa(C); the tests
allow 4 n eps kappa (relative to the largest entry)."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.ib import ROMA3

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


def _rel(a, ref):
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _factor(ctx, C, pad=0):
    n = C.shape[0]
    A = torch.zeros((n, n + pad), dtype=torch.float64, device="cuda")
    A[:, :n] = torch.from_numpy(C).cuda()
    W = torch.full((n, n + pad), 7.0, dtype=torch.float64, device="cuda")   # garbage the factor must overwrite
    lg.ib_chol_factor(ctx, A[:, :n], W[:, :n])
    return A[:, :n].cpu().numpy(), W[:, :n].cpu().numpy()


@pytest.mark.parametrize("n,pad", [(1, 0), (5, 3), (64, 0), (65, 1), (127, 0), (200, 5), (513, 0), (777, 2)])
def test_factor_and_inverse_match_oracle(ctx, n, pad):
    """Leaves only (n <= 64), one split, and several levels of the recursion,
    with ragged sizes and padded leading dimensions."""
    kappa = 1e3
    C = workloads.spd_matrix(n, kappa, seed=n)
    A, W = _factor(ctx, C, pad)
    L_ref, W_ref = oracle.chol_factor(C)
    tol = 4 * max(n, 8) * EPS * kappa
    assert _rel(np.tril(A), L_ref) < tol
    assert _rel(W, W_ref) < tol
    assert np.all(np.triu(W, 1) == 0.0)


def test_solve_matches_oracle_and_allows_aliasing(ctx):
    n = 300
    C = workloads.spd_matrix(n, 1e4, seed=3)
    _, W_ref = oracle.chol_factor(C)
    A, W = _factor(ctx, C)
    b = np.random.Generator(np.random.PCG64(5)).standard_normal(n)
    ref = oracle.chol_solve(W_ref, b)
    Wd = torch.from_numpy(W).cuda()
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    lg.ib_chol_solve(ctx, Wd, bd, x)
    assert _rel(x.cpu().numpy(), ref) < 4 * n * EPS * 1e4
    lg.ib_chol_solve(ctx, Wd, bd, bd)      # in place
    assert np.array_equal(bd.cpu().numpy(), x.cpu().numpy())


def test_indefinite_matrix_reports_enotspd(ctx):
    n = 70
    C = workloads.spd_matrix(n, 10.0, seed=4)
    C[40, 40] = -5.0
    A = torch.from_numpy(C).cuda()
    W = torch.zeros_like(A)
    with pytest.raises(lg.LgfibError) as e:
        lg.ib_chol_factor(ctx, A, W)
    assert e.value.code == lg.LGFIB_ENOTSPD


def test_empty_matrix(ctx):
    A = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    lg.ib_chol_factor(ctx, A, A.clone())


@pytest.fixture(scope="module")
def small_sphere():
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    B, alpha = 8, 0.05
    blocks = oracle.body_blocks(X, ROMA3, B)
    origin, mask = oracle.block_mask(blocks, B)
    gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
    C = oracle.schur_dense(X, ROMA3, alpha, gk, mask, origin)
    return X, B, alpha, blocks, origin, mask, gk, C


def test_schur_dense_matches_oracle(ctx, small_sphere):
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    n = 3 * len(X)
    Cd = torch.zeros((n, n + 3), dtype=torch.float64, device="cuda")
    lg.ib_schur_dense(ctx, sys, Cd[:, :n])
    got = Cd.cpu().numpy()
    assert _rel(got[:, :n], C) < 1e-12
    assert np.all(got[:, n:] == 0.0)
    sys.close()


def test_direct_force_solve_matches_oracle(ctx, small_sphere):
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    b = np.random.Generator(np.random.PCG64(8)).standard_normal(X.shape)
    f = torch.zeros(X.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(lg.LgfibError) as e:
        lg.ib_force_solve(ctx, sys, torch.from_numpy(b).cuda(), f, prec=lg.IB_SOLVE_DIRECT)
    assert e.value.code == lg.LGFIB_ENOTBUILT
    lg.ib_system_factor(ctx, sys)
    st = lg.ib_force_solve(ctx, sys, torch.from_numpy(b).cuda(), f, prec=lg.IB_SOLVE_DIRECT)
    _, W_ref = oracle.chol_factor(C)
    ref = oracle.chol_solve(W_ref, b.reshape(-1)).reshape(X.shape)
    kappa = np.linalg.cond(C)
    assert _rel(f.cpu().numpy(), ref) < 4 * C.shape[0] * EPS * kappa
    assert st["iterations"] == 0 and st["rel_residual"] < 1e-12
    lg.ib_system_factor(ctx, sys, False)
    with pytest.raises(lg.LgfibError):
        lg.ib_force_solve(ctx, sys, torch.from_numpy(b).cuda(), f, prec=lg.IB_SOLVE_DIRECT)
    sys.close()


def _blocks_to_box(field, blocks, B, origin, shape):
    box = np.zeros((field.shape[0],) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def test_stokes_driver_with_direct_solve_matches_oracle(ctx, small_sphere):
    """Two driver steps (Eq. nested_proj) with the force system solved by the
    factor, against the oracle's step (which solves with a dense Cholesky)."""
    X, B, alpha, blocks, origin, mask, gk, C = small_sphere
    flow = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    forigin, fmask = oracle.block_mask(flow, B)
    gl = oracle.lgf_table(*np.array(fmask.shape[::-1]))
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    lg.ib_system_factor(ctx, sys)
    fl = lg.ib_flow_create(ctx, sys, flow)
    u = torch.zeros((3, len(flow), B, B, B), dtype=torch.float64, device="cuda")
    ubox = np.zeros((3,) + fmask.shape)
    for step, U in enumerate([0.3, 0.25]):
        ub = np.zeros(X.shape)
        ub[:, 1] = U
        f = torch.zeros(X.shape, dtype=torch.float64, device="cuda")
        st = lg.ib_flow_step(ctx, fl, u, torch.from_numpy(ub).cuda(), f, prec=lg.IB_SOLVE_DIRECT)
        assert st["iterations"] == 0
        ubox, fref = oracle.stokes_if_euler_step(ubox, X, ub, ROMA3, alpha, gl, C, fmask, forigin)
        got_u = _blocks_to_box(u.cpu().numpy(), flow, B, forigin, fmask.shape)
        assert _rel(f.cpu().numpy(), fref) < 1e-10, step
        assert _rel(got_u, ubox) < 1e-10, step
    fl.close()
    sys.close()


def test_full_size_sphere_direct_solve(ctx):
    """Sphere of diameter 32 with 2200 markers (6600 unknowns): sampled entries
    of the dense C against the oracle's rows of C e_j, symmetry, and the
    direct solve against a tight FP64 CG solve and its own FP64 residual."""
    X = workloads.sphere_markers(diameter=32.0, n=2200)
    B, alpha = 8, 0.05
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    sys = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    n = 3 * len(X)
    Cd = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    lg.ib_schur_dense(ctx, sys, Cd)
    g = np.random.Generator(np.random.PCG64(21))
    cols = g.choice(n, 3, replace=False)
    rows = np.unique(np.concatenate([g.choice(len(X), 12, replace=False), cols // 3]))
    origin, mask = oracle.block_mask(blocks, B)
    gk = oracle.lgf_k_table(alpha, *np.array(mask.shape[::-1]))
    Cs = Cd.cpu().numpy()
    for j in cols:
        e = np.zeros(X.shape)
        e[j // 3, j % 3] = 1.0
        ref = oracle.schur_matvec_rows(e, X, ROMA3, alpha, gk, mask, origin, rows)
        got = Cs[:, j].reshape(X.shape)[rows]
        assert _rel(got, ref) < 1e-12
    assert np.max(np.abs(Cs - Cs.T)) < 1e-13 * np.max(np.abs(Cs))
    del Cd, Cs
    lg.ib_system_factor(ctx, sys)
    b = torch.from_numpy(g.standard_normal(X.shape)).cuda()
    f = torch.zeros_like(b)
    st = lg.ib_force_solve(ctx, sys, b, f, prec=lg.IB_SOLVE_DIRECT)
    assert st["rel_residual"] < 1e-11
    fc = torch.zeros_like(b)
    stc = lg.ib_force_solve(ctx, sys, b, fc, rtol=1e-12, maxit=5000, prec=lg.LGF_F64)
    assert stc["converged"]
    assert _rel(f.cpu().numpy(), fc.cpu().numpy()) < 1e-8
    sys.close()
