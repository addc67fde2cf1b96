"""GPU parity of the flow support that drives the adaptive flow domain
(Sec. 4.1): per-block max |C u| and max |D-bar N~| against the FP64 oracle
through the C ABI, on ragged sets and on the config-5 flow set after
Navier-Stokes steps, and the resulting domain update.

Bars: mu and nu relative to their largest value, FP64 <= 1e-12, FP32
<= 1e-5 (measured 5e-8 and 9e-8)."""
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


@pytest.mark.parametrize("dtype,tmu,tnu", [(np.float64, 1e-12, 1e-12), (np.float32, 1e-5, 1e-5)])
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
    # the device form of the update gives the same lists, in the same order
    fd, xd = lg.ib_adapt_flow_dev(ctx, torch.from_numpy(X).cuda(), B, flow, torch.from_numpy(mu).cuda(),
                                  torch.from_numpy(nu).cuda(), 1.0, 32.0, eps, body, 1)
    assert np.array_equal(fd, fg) and np.array_equal(xd, xg)


def _host_update(X, B, xflow, mu, nu, eta, length, eps, body, nbuf):
    w = lg.ib_block_weights(X, B, xflow, eta, length)
    return lg.ib_adapt_flow(xflow, mu, nu, w, eps, body, nbuf)


@pytest.mark.parametrize("nbuf", [0, 1, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_adapt_flow_dev_matches_host_and_oracle(ctx, nbuf, seed):
    """The device update (weights, W_flow, D_flow, D_xflow) against the host
    one and the oracle: a ragged set of blocks around negative coordinates,
    markers off the lattice, support values with zeros, the threshold inside
    the range of W_flow."""
    g = np.random.Generator(np.random.PCG64(900 + seed))
    B = 8
    allb = np.array(list(np.ndindex(9, 7, 6)), dtype=np.int32)[:, ::-1] + np.array([-4, -3, -2], dtype=np.int32)
    xflow = allb[np.sort(g.choice(len(allb), 250, replace=False))]
    X = g.uniform(-20.0, 30.0, (37, 3))
    mu = g.uniform(0.0, 1.0, len(xflow)) ** 3
    nu = g.uniform(0.0, 1.0, len(xflow)) ** 3
    mu[::7] = 0.0
    nu[::5] = 0.0
    body = np.array([[0, 0, 0], [1, 0, 0], [30, -9, 4]], dtype=np.int32)   # one far from the rest
    w = lg.ib_block_weights(X, B, xflow, 0.5, 16.0)
    wf = w * np.maximum(mu / mu.max(), nu / nu.max())
    eps = float(np.median(wf))
    fh, xh = lg.ib_adapt_flow(xflow, mu, nu, w, eps, body, nbuf)
    fd, xd = lg.ib_adapt_flow_dev(ctx, torch.from_numpy(X).cuda(), B, xflow, torch.from_numpy(mu).cuda(),
                                  torch.from_numpy(nu).cuda(), 0.5, 16.0, eps, body, nbuf)
    assert np.array_equal(fd, fh) and np.array_equal(xd, xh)
    fo, xo = oracle.adapt_flow(xflow, mu, nu, oracle.block_weights(xflow, B, X, 0.5, 16.0), eps, body, nbuf)
    assert {tuple(b) for b in fd.tolist()} == {tuple(b) for b in np.asarray(fo).tolist()}
    assert {tuple(b) for b in xd.tolist()} == {tuple(b) for b in np.asarray(xo).tolist()}


def test_adapt_flow_dev_edge_cases(ctx):
    """No flow blocks (body only), support that is zero everywhere (nothing
    but the body is kept), and too small output lists (LGFIB_ERANGE with the
    sizes returned)."""
    import ctypes
    X = torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64, device="cuda")
    body = np.array([[2, 2, 2], [-1, 0, 5]], dtype=np.int32)
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    f, x = lg.ib_adapt_flow_dev(ctx, X, 4, np.zeros((0, 3), np.int32), empty, empty, 1.0, 1.0, 0.1, body, 1)
    fh, xh = lg.ib_adapt_flow(np.zeros((0, 3), np.int32), [], [], [], 0.1, body, 1)
    assert np.array_equal(f, fh) and np.array_equal(x, xh) and len(x) == 54
    xflow = np.array([[0, 0, 0], [1, 0, 0], [2, 2, 2]], dtype=np.int32)
    z = torch.zeros(3, dtype=torch.float64, device="cuda")
    f, x = lg.ib_adapt_flow_dev(ctx, X, 4, xflow, z, z, 1.0, 1.0, 0.0, body, 0)
    assert np.array_equal(f, body[np.lexsort(body.T)])
    lib = lg.load_library()
    xb = np.ascontiguousarray(xflow)
    bb = np.ascontiguousarray(body)
    fo = np.zeros((1, 3), np.int32)
    xo = np.zeros((1, 3), np.int32)
    nf, nx = ctypes.c_int(), ctypes.c_int()
    rc = lib.ib_adapt_flow_dev(ctx.handle, ctypes.c_void_p(X.data_ptr()), 1, 4, xb.ctypes.data_as(ctypes.c_void_p), 3,
                               ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()), 1.0, 1.0, 0.0,
                               bb.ctypes.data_as(ctypes.c_void_p), 2, 1, fo.ctypes.data_as(ctypes.c_void_p), 1,
                               ctypes.byref(nf), xo.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(nx),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == lg.LGFIB_ERANGE and nf.value == 2 and nx.value == 54
