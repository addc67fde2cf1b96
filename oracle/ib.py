"""Immersed-boundary part of the FP64 oracle (test infrastructure only).

Discrete delta function, interpolation / regularization, the staggered
gradient and its adjoint, the body-block set, the force Schur complement and
its dense Cholesky solve, written out from Liska & Colonius Sec. 2.1
(operators I and R), Sec. 3.1 (Eq. force_schur) and Sec. 3.2 (dense
pre-processing).  Fields live in dense boxes: a box has an integer ``origin``
(lattice point of its (0,0,0) cell) and arrays indexed [z, y, x]; face fields
carry a leading component axis of length 3.  Values outside the block set are
zero.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "phi_roma3", "phi_smooth3", "phi", "delta_halfwidth", "support_cells",
    "body_blocks", "block_mask", "regularize", "interpolate", "grad", "grad_adjoint",
    "if_apply_faces", "kinv_apply_cells", "schur_matvec", "schur_matvec_rows", "schur_dense",
    "stokes_if_euler_step", "stokes_stage_solve", "herk_tableau", "herk_step", "stokes_ifherk_step", "chol_factor", "chol_solve", "force_smooth",
    "curl", "curl_adjoint", "velocity_refresh", "velocity_refresh_at", "lamb_vector",
    "block_support", "block_weights", "adapt_flow",
]

ROMA3, SMOOTH3 = 0, 1


def phi_roma3(r):
    """Roma, Peskin & Berger (1999) 3-point kernel (the kernel named in Sec. 5):
    (1 + sqrt(1 - 3 r^2)) / 3 for |r| <= 1/2,
    (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6 for 1/2 <= |r| <= 3/2, else 0."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    m2 = (a > 0.5) & (a <= 1.5)
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] ** 2)) / 3.0
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[m2]) ** 2))) / 6.0
    return out


def phi_smooth3(r):
    """Smoothed 3-point kernel (Yang et al. 2009, used by the paper's runs,
    Sec. 5): the Roma kernel convolved with the unit top-hat, in closed form."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    s3 = math.sqrt(3.0)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a <= 2.0)
    x = a[m1]
    out[m1] = (17.0 / 48.0 + s3 * math.pi / 108.0 + x / 4.0 - x ** 2 / 4.0
               + (1.0 - 2.0 * x) / 16.0 * np.sqrt(np.maximum(0.0, -12.0 * x ** 2 + 12.0 * x + 1.0))
               - s3 / 12.0 * np.arcsin(np.clip(s3 / 2.0 * (2.0 * x - 1.0), -1.0, 1.0)))
    x = a[m2]
    out[m2] = (55.0 / 48.0 - s3 * math.pi / 108.0 - 13.0 * x / 12.0 + x ** 2 / 4.0
               + (2.0 * x - 3.0) / 48.0 * np.sqrt(np.maximum(0.0, -12.0 * x ** 2 + 36.0 * x - 23.0))
               + s3 / 36.0 * np.arcsin(np.clip(s3 / 2.0 * (2.0 * x - 3.0), -1.0, 1.0)))
    return out


def phi(kernel: int, r):
    return phi_roma3(r) if kernel == ROMA3 else phi_smooth3(r)


def delta_halfwidth(kernel: int) -> float:
    """phi vanishes for |r| >= this value."""
    return 1.5 if kernel == ROMA3 else 2.0


def _face_offset(k: int) -> np.ndarray:
    """x_F^(k)(n) - n: the k-th face sits on the lower k-side of cell n."""
    c = np.full(3, 0.5)
    c[k] = 0.0
    return c


def _marker_stencil(X: np.ndarray, k: int, kernel: int):
    """For every marker, the lattice indices n (per axis) with phi != 0 at face
    component k, and the 1D weights.  Returns (base[N,3], w[N,3,S])."""
    hw = delta_halfwidth(kernel)
    S = int(2 * hw) + 1
    c = _face_offset(k)
    # smallest n_j with n_j + c_j > X_j - hw
    base = np.floor(X - c - hw).astype(np.int64) + 1
    idx = base[:, :, None] + np.arange(S)[None, None, :]
    r = idx + c[None, :, None] - X[:, :, None]
    w = phi(kernel, r)
    return base, w


def support_cells(X: np.ndarray, kernel: int) -> np.ndarray:
    """Cells n with a face (n, k) inside the support of some delta_h(x - X_i)."""
    cells = set()
    for k in range(3):
        base, w = _marker_stencil(X, k, kernel)
        S = w.shape[2]
        for i in range(X.shape[0]):
            for a in range(S):
                if w[i, 2, a] == 0.0:
                    continue
                for b in range(S):
                    if w[i, 1, b] == 0.0:
                        continue
                    for c in range(S):
                        if w[i, 0, c] == 0.0:
                            continue
                        cells.add((base[i, 0] + c, base[i, 1] + b, base[i, 2] + a))
    return np.array(sorted(cells), dtype=np.int64).reshape(-1, 3)


def body_blocks(X: np.ndarray, kernel: int, B: int) -> np.ndarray:
    """D_body (Sec. 4.1): the blocks of edge B holding a cell at most one cell
    away (in every axis) from a support cell.  Sorted (z, y, x) block coords."""
    sc = support_cells(X, kernel)
    blocks = set()
    for d in np.ndindex(3, 3, 3):
        cc = sc + (np.array(d) - 1)
        for b in map(tuple, np.floor_divide(cc, B)):
            blocks.add(b)
    arr = np.array(sorted(blocks, key=lambda b: (b[2], b[1], b[0])), dtype=np.int64)
    return arr.reshape(-1, 3)


def block_mask(blocks: np.ndarray, B: int):
    """Dense box covering the blocks: returns (origin, mask[z, y, x] bool)."""
    lo = blocks.min(axis=0) * B
    hi = (blocks.max(axis=0) + 1) * B
    shape = tuple((hi - lo)[::-1])
    m = np.zeros(shape, dtype=bool)
    for b in blocks:
        o = b * B - lo
        m[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = True
    return lo, m


def regularize(X: np.ndarray, g: np.ndarray, kernel: int, origin, shape, dx: float = 1.0) -> np.ndarray:
    """[R g]^(k)(n) = sum_i g^(k)(i) delta_dx(x_F^(k)(n) - X_i)  (Sec. 2.1),
    delta_h(x) = h^-3 prod phi(x_j / h); X in lattice units.  Returns faces
    [3, z, y, x] on the box (origin, shape=(nz, ny, nx))."""
    out = np.zeros((3,) + tuple(shape), dtype=np.float64)
    org = np.asarray(origin, dtype=np.int64)
    for k in range(3):
        base, w = _marker_stencil(X, k, kernel)
        S = w.shape[2]
        for i in range(X.shape[0]):
            blk = (w[i, 2][:, None, None] * w[i, 1][None, :, None] * w[i, 0][None, None, :]) * g[i, k]
            o = base[i] - org
            if np.any(o < 0) or o[2] + S > shape[0] or o[1] + S > shape[1] or o[0] + S > shape[2]:
                raise ValueError("marker support leaves the box")
            out[k, o[2]:o[2] + S, o[1]:o[1] + S, o[0]:o[0] + S] += blk
    return out / dx ** 3


def interpolate(X: np.ndarray, u: np.ndarray, kernel: int, origin, dx: float = 1.0) -> np.ndarray:
    """[I v]^(k)(i) = dx^3 sum_n v^(k)(n) delta_dx(x_F^(k)(n) - X_i)  (Sec. 2.1);
    I = dx^3 R^T.  u is a face box [3, z, y, x]; returns [N, 3]."""
    org = np.asarray(origin, dtype=np.int64)
    out = np.zeros((X.shape[0], 3), dtype=np.float64)
    shape = u.shape[1:]
    for k in range(3):
        base, w = _marker_stencil(X, k, kernel)
        S = w.shape[2]
        for i in range(X.shape[0]):
            o = base[i] - org
            if np.any(o < 0) or o[2] + S > shape[0] or o[1] + S > shape[1] or o[0] + S > shape[2]:
                raise ValueError("marker support leaves the box")
            blk = w[i, 2][:, None, None] * w[i, 1][None, :, None] * w[i, 0][None, None, :]
            out[i, k] = np.sum(blk * u[k, o[2]:o[2] + S, o[1]:o[1] + S, o[0]:o[0] + S])
    return out


def grad(q: np.ndarray) -> np.ndarray:
    """(G q)^(k)(n) = q(n) - q(n - e_k), zero outside the box (Sec. 2.1)."""
    out = np.zeros((3,) + q.shape, dtype=np.float64)
    # axis order of q is [z, y, x]; component k = 0, 1, 2 is x, y, z
    for k, ax in enumerate((2, 1, 0)):
        sh = np.zeros_like(q)
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(None, -1)
        sh[tuple(sl_dst)] = q[tuple(sl_src)]
        out[k] = q - sh
    return out


def grad_adjoint(u: np.ndarray) -> np.ndarray:
    """(G^T u)(n) = sum_k u^(k)(n) - u^(k)(n + e_k) = -(D-bar u)(n) (Sec. 2.1)."""
    out = np.zeros(u.shape[1:], dtype=np.float64)
    for k, ax in enumerate((2, 1, 0)):
        sh = np.zeros_like(u[k])
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax] = slice(None, -1)
        sl_src[ax] = slice(1, None)
        sh[tuple(sl_dst)] = u[k][tuple(sl_src)]
        out += u[k] - sh
    return out


def _cells_of(mask: np.ndarray, origin) -> np.ndarray:
    z, y, x = np.nonzero(mask)
    return np.stack([x, y, z], axis=1) + np.asarray(origin, dtype=np.int64)[None, :]


def if_apply_faces(u: np.ndarray, alpha: float, mask: np.ndarray, origin) -> np.ndarray:
    """E(a) applied per face component with sources and targets on the block
    set (Table tab:src_trg, the H_F column of force_schur): direct 3D sum of
    the product kernel prod_q e^{-2a} I_{n_q}(2a) truncated at 1e-14."""
    from . import conv_direct, if_kernel_table
    ker = if_kernel_table(alpha)
    tgt = _cells_of(mask, origin)
    out = np.zeros_like(u)
    for k in range(3):
        nz = np.nonzero((u[k] != 0.0) & mask)
        if nz[0].size == 0:
            continue
        src = np.stack([nz[2], nz[1], nz[0]], axis=1) + np.asarray(origin)[None, :]
        vals = conv_direct(ker, src, u[k][nz], tgt)
        out[k][mask] = vals
    return out


def kinv_apply_cells(c: np.ndarray, gk_table: np.ndarray, mask: np.ndarray, origin) -> np.ndarray:
    """K^{-1} c = G_K(a) * c with sources and targets on the block set
    (Table tab:src_trg, the K^{-1} column of force_schur)."""
    from . import conv_direct
    tgt = _cells_of(mask, origin)
    out = np.zeros_like(c)
    nz = np.nonzero((c != 0.0) & mask)
    if nz[0].size == 0:
        return out
    src = np.stack([nz[2], nz[1], nz[0]], axis=1) + np.asarray(origin)[None, :]
    out[mask] = conv_direct(gk_table, src, c[nz], tgt)
    return out


def schur_matvec(x: np.ndarray, X: np.ndarray, kernel: int, alpha: float, gk_table: np.ndarray,
                 mask: np.ndarray, origin) -> np.ndarray:
    """Force Schur complement C x = I [H_F + G K_C^{-1} G^T] I^T x for a rigid
    body (Eq. force_schur with I^{i-1} = I^i; dx = 1 so I^T = R).  Every
    operator keeps its sources and targets on D_body."""
    g = regularize(X, x, kernel, origin, mask.shape)
    g *= mask[None]
    a = if_apply_faces(g, alpha, mask, origin)
    c = grad_adjoint(g) * mask
    d = kinv_apply_cells(c, gk_table, mask, origin)
    e = grad(d) * mask[None]
    return interpolate(X, a + e, kernel, origin)


def schur_dense(X: np.ndarray, kernel: int, alpha: float, gk_table: np.ndarray,
                mask: np.ndarray, origin) -> np.ndarray:
    """Dense matrix of C built column by column from basis vectors, the paper's
    pre-processing step (Sec. 3.2).  Unknown ordering: i * 3 + k."""
    n = X.shape[0] * 3
    C = np.zeros((n, n), dtype=np.float64)
    e = np.zeros((X.shape[0], 3), dtype=np.float64)
    for j in range(n):
        e[j // 3, j % 3] = 1.0
        C[:, j] = schur_matvec(e, X, kernel, alpha, gk_table, mask, origin).reshape(-1)
        e[j // 3, j % 3] = 0.0
    return C


def schur_matvec_rows(x: np.ndarray, X: np.ndarray, kernel: int, alpha: float, gk_table: np.ndarray,
                      mask: np.ndarray, origin, rows) -> np.ndarray:
    """Rows ``rows`` of C x (same operator as schur_matvec), evaluating E(a) and
    K^{-1} only at the faces/cells that those markers' interpolation reads."""
    from . import conv_direct, if_kernel_table
    org = np.asarray(origin, dtype=np.int64)
    g = regularize(X, x, kernel, origin, mask.shape) * mask[None]
    c = grad_adjoint(g) * mask
    nzc = np.nonzero(c)
    src_c = np.stack([nzc[2], nzc[1], nzc[0]], axis=1) + org[None, :]
    cv = c[nzc]
    ker = if_kernel_table(alpha)

    def inside(cells):
        o = cells - org[None, :]
        ok = np.all(o >= 0, axis=1) & (o[:, 0] < mask.shape[2]) & (o[:, 1] < mask.shape[1]) & (o[:, 2] < mask.shape[0])
        res = np.zeros(len(cells), dtype=bool)
        res[ok] = mask[o[ok, 2], o[ok, 1], o[ok, 0]]
        return res

    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), 3))
    for k in range(3):
        base, w = _marker_stencil(X[rows], k, kernel)
        S = w.shape[2]
        off = np.array(list(np.ndindex(S, S, S)))[:, ::-1]          # (dx, dy, dz), x fastest
        faces = (base[:, None, :] + off[None, :, :]).reshape(-1, 3)
        wts = (w[:, 0, :][:, off[:, 0]] * w[:, 1, :][:, off[:, 1]] * w[:, 2, :][:, off[:, 2]]).reshape(-1)
        nzg = np.nonzero(g[k])
        src_g = np.stack([nzg[2], nzg[1], nzg[0]], axis=1) + org[None, :]
        a = conv_direct(ker, src_g, g[k][nzg], faces) * inside(faces)
        ek = np.zeros(3, dtype=np.int64)
        ek[k] = 1
        dn = conv_direct(gk_table, src_c, cv, faces) * inside(faces)
        dm = conv_direct(gk_table, src_c, cv, faces - ek[None, :]) * inside(faces - ek[None, :])
        vals = a + (dn - dm) * inside(faces)
        out[:, k] = np.sum((wts * vals).reshape(len(rows), -1), axis=1)
    return out


def _embed(field, src_origin, dst_origin, dst_shape):
    """Copy a dense box (leading component axes allowed) into a larger box."""
    out = np.zeros(field.shape[:-3] + tuple(dst_shape))
    o = np.asarray(src_origin) - np.asarray(dst_origin)
    nz, ny, nx = field.shape[-3:]
    out[..., o[2]:o[2] + nz, o[1]:o[1] + ny, o[0]:o[0] + nx] = field
    return out


def stokes_if_euler_step(u, X, ub, kernel, alpha, gl_table, C, flow_mask, flow_origin):
    """One integrating-factor Euler step (one-stage IF-HERK): the stage solve
    below with r = u.  Returns (u', f)."""
    u2, f, _ = stokes_stage_solve(u, X, ub, kernel, alpha, gl_table, C, flow_mask, flow_origin)
    return u2, f


def stokes_stage_solve(u, X, ub, kernel, alpha, gl_table, C, flow_mask, flow_origin):
    """One stage system of the integrating-factor HERK scheme for the discrete
    Stokes equations with a rigid immersed surface (Sec. 2.3, Eq.
    ibifherk_linsys with the nonlinear term omitted): H^{-1} u' + Q lam = u,
    Q^T u' = (0, u_B), Q = [G, R], solved by the nested projection of Sec. 3.1
    (Eq. nested_proj):
      (ip) d* = L^{-1}(-G^T u);  (f) C f = I H[u - G d*] - u_B;
      (pc) d = d* + L^{-1} G^T R f;  (vc) u' = H[u - G d - R f],  H = E(a).
    Velocities (faces) live on the flow box cells in ``flow_mask``, zero
    outside.  The cell variables d*, d live on those cells and on the layer of
    cells just below them (cells n with n + e_k in the set): that layer carries
    part of the divergence of a face field on the set, and the gradient at the
    set's lower faces reads it, so u - G d is the unbounded lattice's
    projection restricted to the set.  C is the dense force Schur complement
    (solved by Cholesky, Sec. 3.2).
    u: faces [3, z, y, x] on the flow box (the stage right-hand side).
    Returns (u', f, Q lam) with Q lam = G d + R f on the set."""
    from . import conv_direct
    org = np.asarray(flow_origin)
    m = flow_mask
    corg = org - 1                       # cell box: one more layer below
    mp = np.zeros(tuple(n + 1 for n in m.shape), dtype=bool)
    mp[1:, 1:, 1:] = m
    cm = mp.copy()
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(None, -1)
        hi[ax] = slice(1, None)
        cm[tuple(lo)] |= mp[tuple(hi)]

    def pad(w):
        out = np.zeros((3,) + mp.shape)
        out[:, 1:, 1:, 1:] = w
        return out

    def grad_on_set(q):
        return grad(q)[:, 1:, 1:, 1:] * m[None]

    def linv(c):
        nz = np.nonzero(c * cm)
        if nz[0].size == 0:
            return np.zeros_like(c)
        src = np.stack([nz[2], nz[1], nz[0]], axis=1) + corg[None, :]
        out = np.zeros_like(c)
        out[cm] = conv_direct(gl_table, src, c[nz], _cells_of(cm, corg))
        return out

    dstar = linv(-grad_adjoint(pad(u * m[None])))
    w = (u - grad_on_set(dstar)) * m[None]
    h = if_apply_faces(w, alpha, m, org)
    b = interpolate(X, h, kernel, org) - ub
    L = np.linalg.cholesky(C)
    f = np.linalg.solve(L.T, np.linalg.solve(L, b.reshape(-1))).reshape(b.shape)
    g = regularize(X, f, kernel, org, m.shape) * m[None]
    d = dstar + linv(grad_adjoint(pad(g)))
    gd = grad_on_set(d)
    u2 = if_apply_faces((u - gd - g) * m[None], alpha, m, org)
    return u2, f, (gd + g) * m[None]


def herk_tableau(name: str):
    """Shifted coefficients (a~, c~) of the HERK schemes of App. B: for an
    explicit tableau (A, b, c) with s rows, a~_{i,j} = A_{i+1,j} for i < s,
    a~_{s,j} = b_j and c~_i = c_{i+1}, c~_s = 1 (row i of a~ is the stage
    that ends at node c~_i).  Returns (a~ [s][s] lower triangular, c~ [s])."""
    r3 = math.sqrt(3.0)
    tab = {
        "A": ([[0, 0, 0], [0.5, 0, 0], [r3 / 3, (3 - r3) / 3, 0]], [(3 + r3) / 6, -r3 / 3, (3 + r3) / 6],
              [0.0, 0.5, 1.0]),
        "B": ([[0, 0, 0], [1 / 3, 0, 0], [-1.0, 2.0, 0]], [0.0, 0.75, 0.25], [0.0, 1 / 3, 1.0]),
        "C": ([[0, 0, 0], [8 / 15, 0, 0], [0.25, 5 / 12, 0]], [0.25, 0.0, 0.75], [0.0, 8 / 15, 2 / 3]),
        # the classical four-stage method (its last row reads garbled in the
        # printed tableau; the text names the scheme)
        "D": ([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]], [1 / 6, 1 / 3, 1 / 3, 1 / 6],
              [0.0, 0.5, 0.5, 1.0]),
    }[name]
    A, b, c = (np.asarray(v, dtype=np.float64) for v in tab)
    s = len(b)
    at = np.zeros((s, s))
    at[:s - 1] = A[1:]
    at[s - 1] = b
    ct = np.append(c[1:], 1.0)
    return at, ct


def herk_step(u, propagate, stage_solve, at, ct, A, nonlinear=None, dt=0.0):
    """One s-stage IF-HERK step (Sec. 2.3) for a constrained system, written
    once for any operators: propagate(a, x) applies the integrating factor
    E(a) to a field, stage_solve(i, a, r) solves stage i's system
    H^{-1} u' + Q lam = r, Q^T u' = zeta_i with H = E(a) and returns
    (u', lam, Q lam).  Stage i uses a_i = (c~_i - c~_{i-1}) A (c~_0 = 0) and
    the right-hand side r^i = h^i + dt sum_{j<i} a~_{ij} w^{ij} + g^i, with
    h^{i+1} = H^i h^i, w^{i+1,j} = H^i w^{ij},
    w^{ii} = (a~_{ii} dt)^{-1} (g^i - Q lam^i) and
    g^i = -a~_{ii} dt N(u^{i-1}) (Eq. ibifherk_g; u^0 = u, and g = 0 without
    a nonlinear term).  The dt factors of the sums cancel:
    dt a~_{ij} w^{ij} = (a~_{ij} / a~_{jj}) (propagated g^j - Q lam^j).
    Returns (u_s, lam^s / a~_{ss})."""
    s = len(ct)
    h = np.array(u, dtype=np.float64)
    ustage = h
    q = []   # propagated Q lam^j - g^j
    prev = 0.0
    for i in range(s):
        if i > 0:
            ap = (ct[i - 1] - (ct[i - 2] if i >= 2 else 0.0)) * A
            if ap != 0.0:
                h = propagate(ap, h)
                q = [propagate(ap, qj) for qj in q]
        g = None if nonlinear is None else -at[i, i] * dt * nonlinear(ustage)
        r = h.copy()
        for j in range(i):
            r = r - (at[i, j] / at[j, j]) * q[j]
        if g is not None:
            r = r + g
        ui, li, qi = stage_solve(i, (ct[i] - prev) * A, r)
        q.append(qi if g is None else qi - g)
        ustage = ui
        prev = ct[i]
    return ui, li / at[s - 1, s - 1]


def stokes_ifherk_step(u, X, ub_stages, kernel, A, at, ct, gl_table, stage_C, flow_mask, flow_origin,
                       dt=0.0, frame_velocity=None):
    """The IF-HERK step (herk_step) of the discrete Stokes equations with a
    rigid immersed surface: stage i is stokes_stage_solve with the marker
    velocity ub_stages[i] (at t_k + c~_i dt) and its own force Schur
    complement stage_C[i] (for parameter (c~_i - c~_{i-1}) A); the
    integrating factor is E on the flow set.  A = dt / (dx^2 Re).
    Returns (u_{k+1}, f_{k+1}) with f_{k+1} = lam_f^s / a~_{ss} (in the units
    of the one-stage step's force).  With dt > 0 the step carries the
    nonlinear term N~ = lamb_vector(u, frame_velocity) on the flow faces
    (the Navier-Stokes step); dt is the time step over the grid spacing."""
    org = np.asarray(flow_origin)
    m = flow_mask
    nonlinear = None
    if dt > 0.0:
        U = np.zeros(3) if frame_velocity is None else np.asarray(frame_velocity, dtype=np.float64)

        def nonlinear(x):
            return lamb_vector(x * m[None], U) * m[None]

    def propagate(a, x):
        return if_apply_faces(x, a, m, org)

    def stage_solve(i, a, r):
        return stokes_stage_solve(r, X, ub_stages[i], kernel, a, gl_table, stage_C[i], m, org)

    return herk_step(u, propagate, stage_solve, at, ct, A, nonlinear, dt)


def chol_factor(C: np.ndarray):
    """The paper's pre-processing of the force system (Sec. 3.2): the Cholesky
    factor L of the SPD matrix C (C = L L^T, L lower triangular with a
    positive diagonal) and its inverse W = L^{-1}, so that C^{-1} = W^T W.
    Raises numpy.linalg.LinAlgError when C is not positive definite."""
    from scipy.linalg import solve_triangular
    L = np.linalg.cholesky(C)
    W = solve_triangular(L, np.eye(C.shape[0]), lower=True)
    return L, W


def chol_solve(W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """f = C^{-1} b evaluated with the inverse factor as two matrix-vector
    products, f = W^T (W b) (Sec. 3.2)."""
    return W.T @ (W @ b)


def force_smooth(X: np.ndarray, f: np.ndarray, kernel: int, mask: np.ndarray, origin) -> np.ndarray:
    """Boundary-force post-processing of the sphere results (Sec. 5, flow
    around spheres): the smoothed force f^ = I W R f with W(n) = 1 / gamma(n)
    where gamma = R 1 (the regularized all-ones marker vector) is nonzero,
    and W(n) = 0 elsewhere (dx = 1, so I^T = R).  f: [NL, 3]."""
    g = regularize(X, f, kernel, origin, mask.shape)
    gamma = regularize(X, np.ones_like(f), kernel, origin, mask.shape)
    w = np.zeros_like(g)
    nz = gamma != 0
    w[nz] = g[nz] / gamma[nz]
    return interpolate(X, w, kernel, origin)


# --------------------------------------------------------------------------
# Curl and the velocity refresh (Sec. 2.1 operators C and C^T; Sec. 4.1,
# Eq. vel_refresh)
# --------------------------------------------------------------------------

# (i, j, k, eps_ijk) for the six non-zero Levi-Civita symbols
_LEVI = ((0, 1, 2, 1.0), (1, 2, 0, 1.0), (2, 0, 1, 1.0), (0, 2, 1, -1.0), (2, 1, 0, -1.0), (1, 0, 2, -1.0))
_AXIS = (2, 1, 0)   # array axis of lattice direction 0, 1, 2 (arrays are [z, y, x])


def _shifted(a: np.ndarray, ax: int, d: int) -> np.ndarray:
    """b(n) = a(n + d e) along array axis ax, zero where n + d e leaves the box."""
    out = np.zeros_like(a)
    dst = [slice(None)] * 3
    src = [slice(None)] * 3
    if d > 0:
        dst[ax], src[ax] = slice(None, -d), slice(d, None)
    else:
        dst[ax], src[ax] = slice(-d, None), slice(None, d)
    out[tuple(dst)] = a[tuple(src)]
    return out


def curl(u: np.ndarray) -> np.ndarray:
    """Faces to edges: (C u)^(i)(n) = sum_jk eps_ijk [u^(k)(n) - u^(k)(n - e_j)],
    the circulation of the face values around edge i of cell n.  With face k
    of cell n at n + (1,1,1)/2 - e_k/2, edge i lies at n + e_i/2, so every
    difference is a centred one.  Zero outside the box (Sec. 2.1)."""
    w = np.zeros_like(u, dtype=np.float64)
    for i, j, k, e in _LEVI:
        w[i] += e * (u[k] - _shifted(u[k], _AXIS[j], -1))
    return w


def curl_adjoint(w: np.ndarray) -> np.ndarray:
    """Edges to faces, the transpose of ``curl`` on the box:
    (C^T w)^(k)(n) = sum_ij eps_ijk [w^(i)(n) - w^(i)(n + e_j)]."""
    u = np.zeros_like(w, dtype=np.float64)
    for i, j, k, e in _LEVI:
        u[k] += e * (w[i] - _shifted(w[i], _AXIS[j], +1))
    return u


def velocity_refresh(u: np.ndarray, flow_mask: np.ndarray, vort_mask: np.ndarray, origin,
                     gl_table: np.ndarray) -> np.ndarray:
    """Velocity refresh (Sec. 4.1, Eq. vel_refresh) on a finite flow domain:
    the vorticity w = C u is kept on the edges of the vorticity cells
    (``vort_mask``, inside ``flow_mask``) and dropped elsewhere, the
    streamfunction s = -L^{-1} w is the free-space solution by direct LGF sums,
    and the new velocity C^T s is returned on the faces of the flow cells.

    Sign: for a divergence-free u the identity L_F = -G G^T - C^T C of Sec. 2.1
    gives L_F u = -C^T C u, and since C^T L_E = L_F C^T, u = C^T (-L_E^{-1} C u);
    the refresh therefore uses s = -L^{-1} w (lattice units; the grid spacing
    cancels between C, L^{-1} and C^T).  Values of u outside the flow cells are
    taken as zero.  ``gl_table`` must reach offsets up to the box extent."""
    from . import conv_direct
    u = np.asarray(u, dtype=np.float64) * flow_mask[None]
    w = curl(u) * vort_mask[None]
    nz, ny, nx = flow_mask.shape
    # s is needed on the flow cells and on their upper neighbours (C^T reads n + e_j)
    need = np.zeros((nz + 1, ny + 1, nx + 1), dtype=bool)
    need[:nz, :ny, :nx] |= flow_mask
    need[1:, :ny, :nx] |= flow_mask
    need[:nz, 1:, :nx] |= flow_mask
    need[:nz, :ny, 1:] |= flow_mask
    tgt = _cells_of(need, origin)
    s = np.zeros((3,) + need.shape)
    for i in range(3):
        nzi = np.nonzero(w[i])
        if nzi[0].size == 0:
            continue
        src = np.stack([nzi[2], nzi[1], nzi[0]], axis=1) + np.asarray(origin)[None, :]
        s[i][need] = -conv_direct(gl_table, src, w[i][nzi], tgt)
    return curl_adjoint(s)[:, :nz, :ny, :nx] * flow_mask[None]


def velocity_refresh_at(u: np.ndarray, flow_mask: np.ndarray, vort_mask: np.ndarray, origin,
                        gl_table: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """The refreshed velocity of ``velocity_refresh`` at the faces of the given
    flow cells only (int (N, 3) xyz lattice coordinates): the streamfunction is
    summed at just the edges C^T reads there, s^(i) at n and at n + e_j.
    Returns [N, 3]."""
    from . import conv_direct
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    u = np.asarray(u, dtype=np.float64) * flow_mask[None]
    w = curl(u) * vort_mask[None]
    unit = np.eye(3, dtype=np.int64)
    out = np.zeros((cells.shape[0], 3))
    for i in range(3):
        nzi = np.nonzero(w[i])
        if nzi[0].size == 0:
            continue
        src = np.stack([nzi[2], nzi[1], nzi[0]], axis=1) + np.asarray(origin)[None, :]
        # s^(i) at n, n + e_0, n + e_1, n + e_2 (the one along e_i is unused)
        pts = np.concatenate([cells + d for d in (np.zeros(3, dtype=np.int64), unit[0], unit[1], unit[2])])
        si = -conv_direct(gl_table, src, w[i][nzi], pts).reshape(4, -1)
        for ii, j, k, e in _LEVI:
            if ii == i:
                out[:, k] += e * (si[0] - si[1 + j])
    inside = flow_mask[tuple((cells - np.asarray(origin)[None, :])[:, ::-1].T)]
    return out * inside[:, None]


def lamb_vector(u: np.ndarray, U=(0.0, 0.0, 0.0)) -> np.ndarray:
    """The nonlinear term in rotational form, N~(u) = (C u) x u_a with
    u_a = u + U (Sec. 2.1: N~ approximates (curl u) x u_a), on the faces of a
    box (u zero outside it, so u_a = U there), in lattice units.  The paper
    leaves the stencils open; this one forms the products on the edges and
    averages them to the faces:
        P_ij(m)    = w^(i)(m) (u_a^(j)(m) + u_a^(j)(m - e_k)) / 2,
        N~^(k)(n)  = sum_ij eps_kij (P_ij(n) + P_ij(n + e_j)) / 2,
    w = C u on edge i of cell m, k the third index of (i, j).  The two
    averages are transposes of each other, so sum_faces u . N~(u) = 0 for
    U = 0 on any box: the term does no work, as in the continuum."""
    U = np.asarray(U, dtype=np.float64)
    nz, ny, nx = u.shape[1:]
    # a face on the upper side of the box also takes the products on the
    # edges one cell beyond it, where u = 0 but w = C u and u_a = U are not
    up = np.pad(np.asarray(u, dtype=np.float64), ((0, 0), (0, 1), (0, 1), (0, 1)))
    w = curl(up)
    out = np.zeros_like(up)
    for i, j, k, e in _LEVI:
        ubar = 0.5 * (up[j] + _shifted(up[j], _AXIS[k], -1)) + U[j]
        P = w[i] * ubar
        out[k] += e * 0.5 * (P + _shifted(P, _AXIS[j], +1))
    return out[:, :nz, :ny, :nx]


# --------------------------------------------------------------------------
# Adaptive flow domain (Sec. 4.1, Eqs. weight_fun and weight_fun_modifer)
# --------------------------------------------------------------------------

def block_support(u: np.ndarray, blocks: np.ndarray, B: int, origin, U=(0.0, 0.0, 0.0)):
    """Per block B of the list: mu(B) = max |w(n)| and nu(B) = max |h(n)| over
    the cells n of the block, w = C u (the three edge components of cell n
    taken as one vector, Euclidean norm) and h = D-bar N~(u), the divergence of
    the nonlinear term (lamb_vector with frame velocity U),
    h(n) = sum_k N~^(k)(n + e_k) - N~^(k)(n).  u is a face field on the box
    (zero outside it).  Returns (mu, nu) as float64 arrays."""
    w = curl(u)
    wn = np.sqrt(w[0] ** 2 + w[1] ** 2 + w[2] ** 2)
    # the divergence reads N~ at n + e_k: evaluate N~ on a box one cell larger
    nz, ny, nx = u.shape[1:]
    up = np.pad(np.asarray(u, dtype=np.float64), ((0, 0), (0, 1), (0, 1), (0, 1)))
    N = lamb_vector(up, U)
    h = -grad_adjoint(N)[:nz, :ny, :nx]
    mu = np.zeros(len(blocks))
    nu = np.zeros(len(blocks))
    for i, b in enumerate(np.asarray(blocks).reshape(-1, 3)):
        o = b * B - np.asarray(origin)
        sl = (slice(o[2], o[2] + B), slice(o[1], o[1] + B), slice(o[0], o[0] + B))
        mu[i] = np.max(wn[sl])
        nu[i] = np.max(np.abs(h[sl]))
    return mu, nu


def block_weights(blocks: np.ndarray, B: int, X: np.ndarray, eta: float, length: float) -> np.ndarray:
    """W(pos(B)) = 1 / max(eta, dist(pos(B))) (Eq. weight_fun_modifer): pos(B)
    is the block's centre, dist the distance from it to the nearest
    Lagrangian point divided by the reference length."""
    c = (np.asarray(blocks, dtype=np.float64).reshape(-1, 3) + 0.5) * B
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    d = np.sqrt(((c[:, None, :] - X[None, :, :]) ** 2).sum(-1)).min(axis=1) / length
    return 1.0 / np.maximum(eta, d)


def adapt_flow(xflow: np.ndarray, mu: np.ndarray, nu: np.ndarray, weights: np.ndarray, eps: float,
               body: np.ndarray, nbuf: int):
    """The flow-domain update of Sec. 4.1: W_flow(B) = W(pos(B)) max(mu(B) /
    mu_global, nu(B) / nu_global) over the blocks of D_xflow (a global maximum
    of zero leaves its ratio out); the new D_flow is every block of D_xflow
    with W_flow > eps, together with D_body; D_xflow is every block within
    nbuf blocks of D_flow in each direction.  Returns (D_flow, D_xflow) as
    int32 [n][3] arrays sorted by (z, y, x)."""
    xflow = np.asarray(xflow, dtype=np.int64).reshape(-1, 3)
    mg, ng = float(np.max(mu)) if len(mu) else 0.0, float(np.max(nu)) if len(nu) else 0.0
    r = np.zeros(len(xflow))
    if mg > 0.0:
        r = np.maximum(r, np.asarray(mu) / mg)
    if ng > 0.0:
        r = np.maximum(r, np.asarray(nu) / ng)
    keep = {tuple(b) for b, wf in zip(xflow.tolist(), np.asarray(weights) * r) if wf > eps}
    keep |= {tuple(b) for b in np.asarray(body, dtype=np.int64).reshape(-1, 3).tolist()}
    dil = set()
    for (x, y, z) in keep:
        for dz in range(-nbuf, nbuf + 1):
            for dy in range(-nbuf, nbuf + 1):
                for dx in range(-nbuf, nbuf + 1):
                    dil.add((x + dx, y + dy, z + dz))

    def srt(st):
        a = np.array(sorted(st, key=lambda t: (t[2], t[1], t[0])), dtype=np.int32).reshape(-1, 3)
        return a
    return srt(keep), srt(dil)
