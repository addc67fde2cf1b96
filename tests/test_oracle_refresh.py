"""Pins of the oracle's curl, its adjoint and the velocity refresh (Sec. 2.1
operators C and C^T; Sec. 4.1, Eq. vel_refresh).

What fixes them, independently of the code under test:
- the orientation and the face/edge placement of C: a rigid rotation with
  angular velocity W has vorticity 2W;
- the mimetic identity L_F = -G G^T - C^T C of Sec. 2.1 against the textbook
  7-point Laplacian, per component;
- Im(G) in Null(C) and div curl = 0;
- a solenoidal field u = C^T psi with compact support comes back exactly from
  its vorticity, also where it is zero, and errors placed away from the
  vorticity are removed.
"""
import numpy as np
import pytest

import oracle

EPS = 1e-13


def _rand(shape, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


def test_rigid_rotation_has_vorticity_twice_the_rate():
    nz, ny, nx = 6, 7, 8
    om = 0.37
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    # rotation about the z axis: face x of cell n sits at (n_x, n_y + 1/2, n_z + 1/2),
    # face y at (n_x + 1/2, n_y, n_z + 1/2)
    u[0] = -om * (y + 0.5)
    u[1] = om * (x + 0.5)
    w = oracle.curl(u)
    inner = (slice(1, None), slice(1, None), slice(1, None))
    assert np.max(np.abs(w[2][inner] - 2.0 * om)) < EPS
    assert np.max(np.abs(w[0][inner])) < EPS and np.max(np.abs(w[1][inner])) < EPS
    # the same rotation about the x axis
    u[:] = 0.0
    u[1] = -om * (z + 0.5)
    u[2] = om * (y + 0.5)
    w = oracle.curl(u)
    assert np.max(np.abs(w[0][inner] - 2.0 * om)) < EPS
    assert np.max(np.abs(w[1][inner])) < EPS and np.max(np.abs(w[2][inner])) < EPS


def test_mimetic_identity_gives_the_7pt_laplacian():
    u = _rand((3, 10, 11, 12), 1)
    lhs = -oracle.grad(oracle.grad_adjoint(u)) - oracle.curl_adjoint(oracle.curl(u))
    for k in range(3):
        ref = oracle.laplacian_7pt(u[k])[1:-1, 1:-1, 1:-1]
        assert np.max(np.abs(lhs[k][2:-2, 2:-2, 2:-2] - ref)) < 1e-12


def test_curl_of_gradient_and_divergence_of_curl_vanish():
    q = _rand((9, 10, 11), 2)
    assert np.max(np.abs(oracle.curl(oracle.grad(q))[:, 1:, 1:, 1:])) < 1e-13
    w = _rand((3, 9, 10, 11), 3)
    assert np.max(np.abs(oracle.grad_adjoint(oracle.curl_adjoint(w))[:-1, :-1, :-1])) < 1e-13


def test_curl_adjoint_is_the_transpose():
    u = _rand((3, 5, 6, 7), 4)
    w = _rand((3, 5, 6, 7), 5)
    assert abs(np.sum(oracle.curl(u) * w) - np.sum(u * oracle.curl_adjoint(w))) < 1e-11


@pytest.fixture(scope="module")
def refresh_case():
    B = 4
    flow = np.array([(x, y, z) for z in range(4) for y in range(4) for x in range(4)])
    vort = np.array([(x, y, z) for z in (1, 2) for y in (1, 2) for x in (1, 2)])
    origin, fmask = oracle.block_mask(flow, B)
    _, vsub = oracle.block_mask(vort, B)
    vmask = np.zeros_like(fmask)
    vmask[4:12, 4:12, 4:12] = vsub
    gl = oracle.lgf_table(16, 16, 16)
    psi = np.zeros((3,) + fmask.shape)
    psi[:, 6:10, 6:10, 6:10] = _rand((3, 4, 4, 4), 6)
    u = oracle.curl_adjoint(psi)
    return B, flow, vort, origin, fmask, vmask, gl, u


def test_refresh_reproduces_a_compact_solenoidal_field(refresh_case):
    B, flow, vort, origin, fmask, vmask, gl, u = refresh_case
    # the vorticity C C^T psi stays inside the vorticity blocks
    assert np.all(vmask[np.any(oracle.curl(u) != 0.0, axis=0)])
    out = oracle.velocity_refresh(u, fmask, vmask, origin, gl)
    assert np.max(np.abs(out - u)) < 1e-11 * np.max(np.abs(u))


def test_refresh_removes_errors_away_from_the_vorticity(refresh_case):
    B, flow, vort, origin, fmask, vmask, gl, u = refresh_case
    err = _rand(u.shape, 7)
    # faces whose cell is at least two cells from every vorticity cell never
    # enter C u on a vorticity edge
    far = np.ones(fmask.shape, dtype=bool)
    far[2:14, 2:14, 2:14] = False
    out = oracle.velocity_refresh(u + err * far[None], fmask, vmask, origin, gl)
    assert np.max(np.abs(out - u)) < 1e-11 * np.max(np.abs(u))


def test_refresh_of_a_gradient_is_zero(refresh_case):
    B, flow, vort, origin, fmask, vmask, gl, u = refresh_case
    q = np.zeros(fmask.shape)
    q[5:11, 5:11, 5:11] = _rand((6, 6, 6), 8)
    out = oracle.velocity_refresh(oracle.grad(q), fmask, vmask, origin, gl)
    assert np.max(np.abs(out)) < 1e-12


def test_sampled_refresh_matches_the_dense_one(refresh_case):
    B, flow, vort, origin, fmask, vmask, gl, u = refresh_case
    g = np.random.Generator(np.random.PCG64(9))
    u2 = u + 0.1 * g.standard_normal(u.shape)
    full = oracle.velocity_refresh(u2, fmask, vmask, origin, gl)
    idx = g.choice(fmask.size, 40, replace=False)
    z, y, x = np.unravel_index(idx, fmask.shape)
    cells = np.stack([x, y, z], axis=1) + np.asarray(origin)[None, :]
    got = oracle.velocity_refresh_at(u2, fmask, vmask, origin, gl, cells)
    assert np.max(np.abs(got - full[:, z, y, x].T)) < 1e-13 * np.max(np.abs(full))
