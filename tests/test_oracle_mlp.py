"""Pins of the warm-start network oracle: bfloat16 rounding against torch's
conversion and hand-checked ties, the forward pass and its gradient against
torch.nn / autograd and central finite differences, Adam against its
first-step closed form and torch.optim.Adam."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")

NIN, NH, NOUT = 5, 7, 3


def _setup(seed=0, M=9):
    g = np.random.Generator(np.random.PCG64(seed))
    p = oracle.mlp_init(NIN, NH, NOUT, seed)
    p[NH * NIN:NH * NIN + NH] = g.standard_normal(NH) * 0.3          # nonzero biases
    p[-NOUT:] = g.standard_normal(NOUT) * 0.3
    x = g.standard_normal((M, NIN)) * 2.0 + 0.5
    t = g.standard_normal((M, NOUT))
    norm = dict(in_shift=g.standard_normal(NIN) * 0.1, in_scale=g.uniform(0.5, 2.0, NIN),
                out_shift=g.standard_normal(NOUT) * 0.1, out_scale=g.uniform(0.5, 2.0, NOUT))
    return p, x, t, norm


def test_bf16_round_ties_and_torch():
    # halfway cases round to the even neighbour
    assert oracle.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert oracle.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert oracle.bf16_round(-(1.0 + 2.0 ** -8)) == -1.0
    assert oracle.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -30) == 1.0 + 2.0 ** -7
    x = (np.random.Generator(np.random.PCG64(1)).standard_normal(200000) *
         np.exp(np.random.Generator(np.random.PCG64(2)).uniform(-30, 30, 200000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.bf16_round(x.astype(np.float64)), ref)


def _torch_net(p):
    W1, b1, W2, b2, W3, b3 = oracle.mlp_unpack(p, NIN, NH, NOUT)
    net = torch.nn.Sequential(torch.nn.Linear(NIN, NH), torch.nn.Tanh(), torch.nn.Linear(NH, NH), torch.nn.Tanh(),
                              torch.nn.Linear(NH, NOUT)).double()
    with torch.no_grad():
        for lin, (W, b) in zip((net[0], net[2], net[4]), ((W1, b1), (W2, b2), (W3, b3))):
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
    return net


def test_forward_and_grad_match_torch_autograd():
    p, x, t, nm = _setup()
    y = oracle.mlp_forward(p, x, NIN, NH, NOUT, **nm)
    net = _torch_net(p)
    xh = torch.from_numpy((x - nm["in_shift"]) / nm["in_scale"])
    o = net(xh)
    yref = nm["out_shift"] + nm["out_scale"] * o.detach().numpy()
    assert np.max(np.abs(y - yref)) < 1e-14
    that = torch.from_numpy((t - nm["out_shift"]) / nm["out_scale"])
    loss_t = 0.5 * ((o - that) ** 2).sum() / x.shape[0]
    loss_t.backward()
    gref = np.concatenate([torch.cat([lin.weight.grad.reshape(-1), lin.bias.grad]).numpy()
                           for lin in (net[0], net[2], net[4])])
    loss, g = oracle.mlp_loss_grad(p, x, t, NIN, NH, NOUT, **nm)
    assert abs(loss - loss_t.item()) < 1e-14 * max(1.0, loss)
    assert np.max(np.abs(g - gref)) < 1e-13 * np.max(np.abs(gref))


def test_grad_central_differences():
    p, x, t, nm = _setup(3)
    _, g = oracle.mlp_loss_grad(p, x, t, NIN, NH, NOUT, **nm)
    h = 1e-5
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = oracle.mlp_loss_grad(p + e, x, t, NIN, NH, NOUT, **nm)
        lm, _ = oracle.mlp_loss_grad(p - e, x, t, NIN, NH, NOUT, **nm)
        fd[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * np.max(np.abs(g))


def test_bf16_mode_rounds_product_operands_only():
    """With weights and inputs already on the bfloat16 grid the only change
    bf16 mode makes is rounding the hidden activations; with one hidden unit
    active per layer the result is computable by hand."""
    p, x, t, nm = _setup(4)
    nm = dict(in_shift=np.zeros(NIN), in_scale=np.ones(NIN), out_shift=np.zeros(NOUT), out_scale=np.ones(NOUT))
    W1, b1, W2, b2, W3, b3 = [a.copy() for a in oracle.mlp_unpack(p, NIN, NH, NOUT)]
    W1[:] = 0
    W1[2, 1] = 0.75
    W2[:] = 0
    W2[4, 2] = 1.5
    W3[:] = 0
    W3[1, 4] = -0.625
    b1[:] = 0
    b2[:] = 0
    b3[:] = [0.5, 0.25, -1.0]
    q = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    xs = oracle.bf16_round(x)
    y = oracle.mlp_forward(q, xs, NIN, NH, NOUT, bf16=True, **nm)
    h1 = oracle.bf16_round(np.tanh(0.75 * xs[:, 1]))
    h2 = oracle.bf16_round(np.tanh(1.5 * h1))
    assert np.array_equal(y[:, 0], np.full(len(xs), 0.5))
    assert np.allclose(y[:, 1], 0.25 - 0.625 * h2, rtol=0, atol=1e-15)
    assert np.array_equal(y[:, 2], np.full(len(xs), -1.0))
    # and the unrounded pass differs from it (the rounding is really applied)
    y64 = oracle.mlp_forward(q, xs, NIN, NH, NOUT, **nm)
    assert np.max(np.abs(y64 - y)) > 1e-5


def test_adam_first_step_and_torch():
    g = np.random.Generator(np.random.PCG64(5))
    p0 = g.standard_normal(50)
    grads = [g.standard_normal(50) for _ in range(4)]
    p1, m1, m2 = oracle.adam_step(p0, grads[0], np.zeros(50), np.zeros(50), 1, 1e-3)
    # bias-corrected first step moves every weight by lr g/(|g| + eps)
    assert np.max(np.abs(p1 - (p0 - 1e-3 * grads[0] / (np.abs(grads[0]) + 1e-8)))) < 1e-15
    w = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m1, m2 = p0.copy(), np.zeros(50), np.zeros(50)
    for k, gr in enumerate(grads, start=1):
        w.grad = torch.from_numpy(gr.copy())
        opt.step()
        p, m1, m2 = oracle.adam_step(p, gr, m1, m2, k, 1e-3)
    assert np.max(np.abs(p - w.detach().numpy())) < 1e-14


def test_warm_features_layout():
    n = np.arange(12.0).reshape(4, 3)
    f1 = n + 100
    f2 = n + 200
    F = oracle.warm_features(n, (7.0, 8.5, 9.0, 11.0), f1, f2)
    assert F.shape == (4, 12)
    assert np.array_equal(F[2], [6, 7, 8, -1.5, -0.5, -2.0, 106, 107, 108, -100, -100, -100])
    assert np.array_equal(oracle.warm_start(np.ones((4, 3)), f1, f2), 2 * f1 - f2 + 1)
