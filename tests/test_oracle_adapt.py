"""Pins of the oracle's adaptive flow-domain update (Sec. 4.1, Eqs.
weight_fun and weight_fun_modifer).

What fixes them, independently of the code under test:
- a rigid rotation has |w| = 2 W and h = div((curl u) x u) = -4 W^2 exactly
  (linear fields), so the interior block's mu and nu are known in closed form;
- a compact solenoidal field has no vorticity and no Lamb vector two blocks
  away, so mu = nu = 0 there;
- the set update against a hand-worked case and a brute-force Chebyshev
  dilation;
- the weight is 1/eta next to the surface and 1/dist far from it.
"""
import numpy as np

import oracle


def test_rigid_rotation_support_in_closed_form():
    B, om = 4, 0.37
    blocks = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)])
    origin, mask = oracle.block_mask(blocks, B)
    z, y, x = np.meshgrid(*[np.arange(n) for n in mask.shape], indexing="ij")
    u = np.zeros((3,) + mask.shape)
    u[0] = -om * (y + 0.5)
    u[1] = om * (x + 0.5)
    mu, nu = oracle.block_support(u, blocks, B, origin)
    c = [i for i, b in enumerate(blocks.tolist()) if b == [1, 1, 1]][0]
    assert abs(mu[c] - 2 * om) < 1e-13
    assert abs(nu[c] - 4 * om ** 2) < 1e-13


def test_compact_solenoidal_field_has_no_support_far_away():
    B = 4
    blocks = np.array([(x, y, z) for z in range(5) for y in range(5) for x in range(5)])
    origin, mask = oracle.block_mask(blocks, B)
    psi = np.zeros((3,) + mask.shape)
    psi[:, 9:11, 9:11, 9:11] = np.random.Generator(np.random.PCG64(1)).standard_normal((3, 2, 2, 2))
    u = oracle.curl_adjoint(psi)
    mu, nu = oracle.block_support(u, blocks, B, origin, (0.2, 0.0, 0.1))
    far = np.array([np.max(np.abs(b - 2)) >= 2 for b in blocks])
    assert np.all(mu[far] == 0.0) and np.all(nu[far] == 0.0)
    assert mu[[i for i, b in enumerate(blocks.tolist()) if b == [2, 2, 2]][0]] > 0.0


def test_adapt_flow_hand_case_and_brute_force_dilation():
    xflow = np.array([(x, 0, 0) for x in range(6)], dtype=np.int32)
    mu = np.array([0.0, 0.5, 2.0, 0.1, 0.0, 0.0])
    nu = np.array([0.0, 0.0, 0.0, 0.0, 3.0, 0.3])
    w = np.array([1.0, 1.0, 1.0, 1.0, 0.5, 1.0])
    # ratios max(mu/2, nu/3) = [0, .25, 1, .05, 1, .1]; times w = [0, .25, 1, .05, .5, .1]
    flow, xf = oracle.adapt_flow(xflow, mu, nu, w, 0.2, np.array([[0, 5, 0]]), 1)
    assert sorted(map(tuple, flow.tolist())) == sorted([(1, 0, 0), (2, 0, 0), (4, 0, 0), (0, 5, 0)])
    want = {(x + dx, y + dy, z + dz) for (x, y, z) in map(tuple, flow.tolist())
            for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)}
    assert set(map(tuple, xf.tolist())) == want
    # sorted by (z, y, x)
    key = [(b[2], b[1], b[0]) for b in xf.tolist()]
    assert key == sorted(key)
    # no support at all keeps only the body blocks
    flow, _ = oracle.adapt_flow(xflow, np.zeros(6), np.zeros(6), w, 0.2, np.array([[9, 9, 9]]), 2)
    assert flow.tolist() == [[9, 9, 9]]


def test_block_weights_near_and_far():
    B = 8
    X = np.array([[4.0, 4.0, 4.0]])
    blocks = np.array([[0, 0, 0], [10, 0, 0]])
    w = oracle.block_weights(blocks, B, X, eta=2.0, length=8.0)
    assert abs(w[0] - 0.5) < 1e-15
    d = np.linalg.norm(np.array([84.0, 4.0, 4.0]) - X[0]) / 8.0
    assert abs(w[1] - 1.0 / d) < 1e-15
