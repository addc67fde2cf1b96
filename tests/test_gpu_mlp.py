"""GPU parity of the warm-start network kernels (BF16 matrix-core products,
FP32 accumulate) against the FP64 oracle with the same BF16 rounding of the
product operands, through the C ABI."""
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


def _problem(nin, nh, nout, M, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    p = oracle.mlp_init(nin, nh, nout, seed).astype(np.float32).astype(np.float64)
    nb1 = nh * nin
    p[nb1:nb1 + nh] = (g.standard_normal(nh) * 0.2).astype(np.float32)
    x = (g.standard_normal((M, nin)) * 1.5 + 0.3).astype(np.float32)
    t = (g.standard_normal((M, nout)) * 0.7).astype(np.float32)
    nm = dict(in_shift=(g.standard_normal(nin) * 0.1).astype(np.float32),
              in_scale=g.uniform(0.5, 2.0, nin).astype(np.float32),
              out_shift=(g.standard_normal(nout) * 0.1).astype(np.float32),
              out_scale=g.uniform(0.5, 2.0, nout).astype(np.float32))
    return p, x, t, nm


def _onm(nm):
    return {k: v.astype(np.float64) for k, v in nm.items()}


def _make(ctx, nin, nh, nout, p, nm):
    return lg.ib_mlp_create(ctx, nin, nh, nout, p, nm["in_shift"], nm["in_scale"], nm["out_shift"],
                            nm["out_scale"])


# (nin, nh, nout, M): the warm-start shape over several 64-row tiles with a
# ragged tail, and a shape whose widths are not multiples of the 16-deep slices
SHAPES = [(12, 256, 3, 1000), (5, 40, 3, 77), (12, 256, 3, 1)]


@pytest.mark.parametrize("nin,nh,nout,M", SHAPES)
def test_forward_matches_oracle(ctx, nin, nh, nout, M):
    p, x, t, nm = _problem(nin, nh, nout, M, 11)
    net = _make(ctx, nin, nh, nout, p, nm)
    y = torch.zeros((M, nout), dtype=torch.float32, device="cuda")
    lg.ib_mlp_forward(ctx, net, torch.from_numpy(x).cuda(), y)
    ref = oracle.mlp_forward(p, x.astype(np.float64), nin, nh, nout, bf16=True, **_onm(nm))
    got = y.cpu().numpy().astype(np.float64)
    # measured <= 2.8e-4 (max) and 2.2e-5 (norm): an activation rounded to
    # BF16 from FP32 here and from FP64 in the oracle may differ by one step
    assert np.max(np.abs(got - ref)) <= 1e-3 * np.max(np.abs(ref))
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    net.close()


@pytest.mark.parametrize("nin,nh,nout,M", SHAPES[:2])
def test_gradient_matches_oracle(ctx, nin, nh, nout, M):
    p, x, t, nm = _problem(nin, nh, nout, M, 12)
    net = _make(ctx, nin, nh, nout, p, nm)
    g, loss = lg.ib_mlp_grad(ctx, net, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    lref, gref = oracle.mlp_loss_grad(p, x.astype(np.float64), t.astype(np.float64), nin, nh, nout, bf16=True,
                                      **_onm(nm))
    assert abs(loss - lref) <= 1e-5 * lref
    # per parameter block (W1, b1, W2, b2, W3, b3), element by element against
    # the block's largest entry (measured <= 1.5e-4: the oracle rounds FP64
    # activations to BF16, the kernels FP32 ones, so an activation may land
    # one BF16 step, 2^-8 relative, away), and in norm
    sizes = [nh * nin, nh, nh * nh, nh, nout * nh, nout]
    o = 0
    for s in sizes:
        a, b = g[o:o + s].astype(np.float64), gref[o:o + s]
        assert np.max(np.abs(a - b)) <= 5e-4 * np.max(np.abs(b)), (o, s)
        assert np.linalg.norm(a - b) <= 2e-4 * np.linalg.norm(b), (o, s)
        o += s
    net.close()


def test_adam_step_matches_oracle(ctx):
    nin, nh, nout, M = 12, 256, 3, 300
    p, x, t, nm = _problem(nin, nh, nout, M, 13)
    net = _make(ctx, nin, nh, nout, p, nm)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    p0 = lg.ib_mlp_get_params(net).astype(np.float64)
    g, _ = lg.ib_mlp_grad(ctx, net, xd, td)
    lg.ib_mlp_train_step(ctx, net, xd, td, 1e-3)
    p1 = lg.ib_mlp_get_params(net).astype(np.float64)
    ref, m1, m2 = oracle.adam_step(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    assert np.max(np.abs(p1 - ref)) <= 1e-9 + 1e-6 * np.max(np.abs(p0))
    # second step: moments carried over
    g2, _ = lg.ib_mlp_grad(ctx, net, xd, td)
    lg.ib_mlp_train_step(ctx, net, xd, td, 1e-3)
    p2 = lg.ib_mlp_get_params(net).astype(np.float64)
    ref2, _, _ = oracle.adam_step(p1, g2.astype(np.float64), m1, m2, 2, 1e-3)
    assert np.max(np.abs(p2 - ref2)) <= 1e-9 + 1e-6 * np.max(np.abs(p0))
    net.close()


def test_training_fits_smooth_map(ctx):
    """The hand-written backward + Adam kernels reduce the loss of a smooth
    12 -> 3 regression by more than an order of magnitude, and the trained net
    predicts held-out rows (generalisation, not memorisation)."""
    nin, nh, nout = 12, 256, 3
    g = np.random.Generator(np.random.PCG64(21))
    A = g.standard_normal((nin, nout)) / np.sqrt(nin)
    C = g.standard_normal((nin, nout)) / np.sqrt(nin)

    def target(x):
        return np.tanh(x @ A) + 0.3 * np.sin(x @ C)

    X = g.standard_normal((6000, nin)).astype(np.float32)
    T = target(X.astype(np.float64)).astype(np.float32)
    Xv = g.standard_normal((1000, nin)).astype(np.float32)
    Tv = target(Xv.astype(np.float64))
    p = oracle.mlp_init(nin, nh, nout, 22).astype(np.float32)
    one, zero = np.ones(nin, np.float32), np.zeros(nin, np.float32)
    net = lg.ib_mlp_create(ctx, nin, nh, nout, p, zero, one, np.zeros(3, np.float32), np.ones(3, np.float32))
    yv = torch.zeros((1000, nout), dtype=torch.float32, device="cuda")
    lg.ib_mlp_forward(ctx, net, torch.from_numpy(Xv).cuda(), yv)
    err0 = np.mean((yv.cpu().numpy() - Tv) ** 2)
    loss = lg.ib_mlp_train(ctx, net, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), epochs=40, batch=250,
                           lr=2e-3, seed=5)
    lg.ib_mlp_forward(ctx, net, torch.from_numpy(Xv).cuda(), yv)
    err1 = np.mean((yv.cpu().numpy() - Tv) ** 2)
    assert np.isfinite(loss) and err1 < 0.05 * err0, (err0, err1, loss)
    net.close()


def test_features_and_warmstart(ctx):
    NL = 333
    g = np.random.Generator(np.random.PCG64(31))
    n = g.standard_normal((NL, 3))
    f1, f2 = g.standard_normal((NL, 3)), g.standard_normal((NL, 3))
    us = (0.1, -0.2, 0.3, 0.25)
    feats = torch.zeros((NL, 12), dtype=torch.float32, device="cuda")
    lg.ib_mlp_features(ctx, torch.from_numpy(n).cuda(), us, torch.from_numpy(f1).cuda(), torch.from_numpy(f2).cuda(),
                       feats)
    ref = oracle.warm_features(n, us, f1, f2).astype(np.float32)
    assert np.array_equal(feats.cpu().numpy(), ref)
    p, _, _, nm = _problem(12, 64, 3, 1, 32)
    net = _make(ctx, 12, 64, 3, p, nm)
    y = torch.zeros((NL, 3), dtype=torch.float32, device="cuda")
    lg.ib_mlp_forward(ctx, net, feats, y)
    x0 = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    lg.ib_mlp_warmstart(ctx, net, feats, torch.from_numpy(f1).cuda(), torch.from_numpy(f2).cuda(), x0)
    want = oracle.warm_start(y.cpu().numpy().astype(np.float64), f1, f2)
    assert np.max(np.abs(x0.cpu().numpy() - want)) <= 1e-6 * np.max(np.abs(want))
    net.close()


def test_bad_arguments(ctx):
    p = np.zeros(lg.mlp_param_count(4, 8, 2), np.float32)
    with pytest.raises(lg.LgfibError):
        lg.ib_mlp_create(ctx, 4, 8, 2, p, np.zeros(4), np.zeros(4), np.zeros(2), np.ones(2))   # zero in_scale
    net = lg.ib_mlp_create(ctx, 4, 8, 2, p, np.zeros(4), np.ones(4), np.zeros(2), np.ones(2))
    feats = torch.zeros((5, 12), dtype=torch.float32, device="cuda")
    with pytest.raises(lg.LgfibError):
        lg.ib_mlp_warmstart(ctx, net, feats, torch.zeros((5, 3), dtype=torch.float64, device="cuda"),
                            torch.zeros((5, 3), dtype=torch.float64, device="cuda"),
                            torch.zeros((5, 3), dtype=torch.float64, device="cuda"))
    net.close()


def test_learned_start_beats_cold_cg(ctx):
    """The trained network's gain over the method without it: a heaving
    sphere (D = 12 cells, 400 markers, Roma kernel, a = 0.05) generates a
    force history with the Stokes driver (Sec. 3.1); the network is trained
    on its steps 20-149 and warm-starts the force solves C f = b_k of steps
    150-199.  Plain CG is the judge: cold and learned starts both reach a true
    FP64 relative residual of 1e-8, and the learned start needs fewer
    iterations."""
    B, alpha, D, NL, period = 8, 0.05, 12.0, 400, 50
    X = workloads.fibonacci_sphere(NL, D / 2, (24.37, 24.21, 24.13))
    normals = torch.from_numpy((X - np.array([24.37, 24.21, 24.13])) / (D / 2)).cuda()
    blocks = lg.ib_body_blocks(lg.IB_ROMA3, X, B)
    sys_ = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, alpha)
    fb = np.array([(x, y, z) for z in range(6) for y in range(6) for x in range(6)], dtype=np.int32)
    fl = lg.ib_flow_create(ctx, sys_, fb)
    nsteps, ntrain, skip = 200, 150, 20
    U = [workloads.heave_velocity(k, D, period=period) for k in range(nsteps + 2)]
    u = torch.zeros((3, len(fb), B, B, B), dtype=torch.float64, device="cuda")
    F = torch.zeros((nsteps, NL, 3), dtype=torch.float64, device="cuda")
    Bk = torch.zeros_like(F)
    ub = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    for k in range(nsteps):
        ub[:, 1] = U[k + 1]
        st = lg.ib_flow_step(ctx, fl, u, ub, F[k], x0=F[k - 1] if k else None, rtol=1e-10, maxit=4000,
                             prec=lg.LGF_F64, b_out=Bk[k])
        assert st["converged"], k
    nin, nh, nout = 12, 256, 3
    rows = list(range(skip, ntrain))
    Xtr = torch.zeros((len(rows) * NL, nin), dtype=torch.float32, device="cuda")
    for i, k in enumerate(rows):
        lg.ib_mlp_features(ctx, normals, (U[k + 1], U[k], U[k - 1], U[k - 2]), F[k - 1], F[k - 2],
                           Xtr[i * NL:(i + 1) * NL])
    Ttr = (F[rows] - 2.0 * F[[k - 1 for k in rows]] + F[[k - 2 for k in rows]]).reshape(-1, 3).float().contiguous()
    ins, inc = Xtr.mean(0), Xtr.std(0).clamp_min(1e-6)
    ots, otc = Ttr.mean(0), Ttr.std(0).clamp_min(1e-12)
    p = oracle.mlp_init(nin, nh, nout, 7).astype(np.float32)
    net = lg.ib_mlp_create(ctx, nin, nh, nout, p, ins.cpu().numpy(), inc.cpu().numpy(), ots.cpu().numpy(),
                           otc.cpu().numpy())
    lg.ib_mlp_train(ctx, net, Xtr, Ttr, epochs=30, batch=2048, lr=1e-3, seed=3)
    feats = torch.zeros((NL, nin), dtype=torch.float32, device="cuda")
    x0 = torch.zeros((NL, 3), dtype=torch.float64, device="cuda")
    f = torch.zeros_like(x0)
    its = {"cold": [], "mlp": []}
    for k in range(ntrain, nsteps, 5):
        for m in its:
            guess = None
            if m == "mlp":
                lg.ib_mlp_features(ctx, normals, (U[k + 1], U[k], U[k - 1], U[k - 2]), F[k - 1], F[k - 2], feats)
                lg.ib_mlp_warmstart(ctx, net, feats, F[k - 1], F[k - 2], x0)
                guess = x0
            st = lg.ib_force_solve(ctx, sys_, Bk[k], f, x0=guess, rtol=1e-8, maxit=4000, prec=lg.LGF_F32)
            assert st["rel_residual"] <= 1e-8 and st["fallback"] == 0, (k, m, st)
            its[m].append(st["iterations"])
            err = float(torch.linalg.vector_norm(f - F[k]) / torch.linalg.vector_norm(F[k]))
            assert err < 1e-5, (k, m, err)
    print("iterations cold %s learned %s" % (its["cold"], its["mlp"]))
    assert np.mean(its["mlp"]) < 0.7 * np.mean(its["cold"])
    net.close()
    fl.close()
    sys_.close()
