"""GPU parity of the flow support that drives the adaptive flow domain
(Sec. 4.1): per-block max |C u| and max |D-bar N~| against the FP64 oracle
through the C ABI, on ragged sets and on the config-5 flow set after
Navier-Stokes steps, and the resulting domain update.

Bars: mu and nu relative to their largest value, FP64 <= 1e-12; FP32
<= 1e-5 for mu and 1e-4 for nu (a divergence of FP32 products)."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


def _to_box(field, blocks, B, origin, shape):
    box = np.zeros((3,) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def _gpu_support(ctx, B, blocks, u, U, dtype):
    ud = torch.from_numpy(np.ascontiguousarray(u, dtype=dtype)).cuda()
    mu = torch.zeros(len(blocks), dtype=torch.float64, device="cuda")
    nu = torch.zeros_like(mu)
    lg.lgf_block_support(ctx, B, blocks, ud, mu, nu, U)
    torch.cuda.synchronize()
    return mu.cpu().numpy(), nu.cpu().numpy()


@pytest.mark.parametrize("dtype,tmu,tnu", [(np.float64, 1e-12, 1e-12), (np.float32, 1e-5, 1e-4)])
@pytest.mark.parametrize("B", [4, 8])
def test_block_support_matches_oracle(ctx, dtype, tmu, tnu, B):
    g = np.random.Generator(np.random.PCG64(60 + B))
    allb = np.array(list(np.ndindex(4, 3, 5)), dtype=np.int32)[:, ::-1] + np.array([1, -2, 0], dtype=np.int32)
    blocks = allb[np.sort(g.choice(len(allb), len(allb) - 12, replace=False))]
    u = g.standard_normal((3, len(blocks), B, B, B)).astype(dtype).astype(np.float64)
    U = (0.2, -0.1, 0.3)
    mu, nu = _gpu_support(ctx, B, blocks, u, U, dtype)
    origin, mask = oracle.block_mask(blocks, B)
    mo, no = oracle.block_support(_to_box(u, blocks, B, origin, mask.shape), blocks, B, origin, U)
    assert np.max(np.abs(mu - mo)) < tmu * np.max(mo)
    assert np.max(np.abs(nu - no)) < tnu * np.max(no)


@pytest.mark.parametrize("B", [16, 32])
def test_block_support_large_blocks(ctx, B):
    """Blocks of 16^3 and 32^3 (the reduction over many cells per block),
    FP64, against the oracle."""
    blocks = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 0, 1]], dtype=np.int32)
    u = np.random.Generator(np.random.PCG64(B + 7)).standard_normal((3, len(blocks), B, B, B))
    U = (0.1, 0.0, -0.3)
    mu, nu = _gpu_support(ctx, B, blocks, u, U, np.float64)
    origin, mask = oracle.block_mask(blocks, B)
    mo, no = oracle.block_support(_to_box(u, blocks, B, origin, mask.shape), blocks, B, origin, U)
    assert np.max(np.abs(mu - mo)) < 1e-12 * np.max(mo)
    assert np.max(np.abs(nu - no)) < 1e-12 * np.max(no)


def test_support_and_domain_update_after_navier_stokes_steps(ctx):
    """Config 5 (sphere of diameter 32, 2200 markers, 1728 flow blocks of
    8^3): two Scheme A steps with the nonlinear term from rest, then the
    support on the flow set against the oracle, and the new D_flow / D_xflow
    from it (blocks whose W_flow lies within 1e-9 of the threshold may go
    either way)."""
    X = workloads.sphere_markers(32.0, 2200)
    B = 8
    body = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    flow = np.array([(x, y, z) for z in range(-1, 11) for y in range(-1, 11) for x in range(-1, 11)], dtype=np.int32)
    at, ct = lg.ib_herk_tableau("A")
    hk = lg.ib_herk_create(ctx, lg.IB_ROMA3, X, B, body, flow, 0.05, at, ct, direct=True)
    lg.ib_herk_convection(ctx, hk, 1.0)
    u = torch.zeros((3, len(flow), B, B, B), dtype=torch.float64, device="cuda")
    f = torch.zeros((len(X), 3), dtype=torch.float64, device="cuda")
    for k in range(2):
        ubs = np.zeros((len(ct), len(X), 3))
        for i, c in enumerate(ct):
            ubs[i, :, 1] = workloads.heave_velocity(k + c, 32.0)
        lg.ib_herk_step(ctx, hk, u, torch.from_numpy(ubs).cuda(), f)
    hk.close()
    uh = u.cpu().numpy()
    mu, nu = _gpu_support(ctx, B, flow, uh, (0.0, 0.0, 0.0), np.float64)
    origin, mask = oracle.block_mask(flow, B)
    mo, no = oracle.block_support(_to_box(uh, flow, B, origin, mask.shape), flow, B, origin)
    assert np.max(np.abs(mu - mo)) < 1e-12 * np.max(mo)
    assert np.max(np.abs(nu - no)) < 1e-12 * np.max(no)
    w = lg.ib_block_weights(X, B, flow, 1.0, 32.0)
    eps = 1e-3
    fg, xg = lg.ib_adapt_flow(flow, mu, nu, w, eps, body, 1)
    fo, xo = oracle.adapt_flow(flow, mo, no, oracle.block_weights(flow, B, X, 1.0, 32.0), eps, body, 1)
    wf = w * np.maximum(mo / mo.max(), no / no.max())
    near = {tuple(b) for b, v in zip(flow.tolist(), wf) if abs(v - eps) <= 1e-9 * eps}
    assert {tuple(b) for b in fg.tolist()} ^ {tuple(b) for b in fo.tolist()} <= near
    # the body blocks are kept, the far field is dropped
    assert {tuple(b) for b in body.tolist()} <= {tuple(b) for b in fg.tolist()}
    assert 0 < len(fg) < len(flow)
