"""Multilevel interpolation evaluator of the lattice convolution (Sec. 2.2,
Eq. dpoisson_conv): the plain FP64 form the GPU evaluator is checked against.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper evaluates these convolutions with a kernel-independent,
interpolation-based fast multipole method on the block-structured grid
(Sec. 2.2) and gives no further steps.  The steps below are this project's
reading of such a method, written for checking, not speed:

  * blocks of B^3 cells are the leaves; level l groups 2^l x 2^l x 2^l blocks
    into a cluster of side L = B 2^l cells, cluster index floor(block / 2^l);
  * each cluster carries p^3 interpolation nodes on lattice points, the
    tensor product of the 1D nodes t_j = floor((L-1)/2 (1 - cos(pi (2j+1) /
    (2p))) + 1/2) (Chebyshev points rounded to the lattice, so the kernel is
    only ever needed at lattice offsets);
  * sources are anterpolated to the nodes of their block (P2M) and up the
    levels (M2M) with the tensor Lagrange basis of the receiving cluster;
  * two clusters interact through their nodes (M2L) at the finest level at
    which they are not neighbours (Chebyshev distance of the cluster indices
    > 1) while their parents are neighbours or equal; at the top level every
    non-neighbour pair interacts;
  * node values are interpolated down (L2L) and to the cells (L2P);
  * neighbouring blocks (including the block itself) are summed exactly
    (P2P);
  * the top level is the first at which the sources and targets together
    span at most 4 clusters on every axis.

Every pair of a source block and a target block is counted exactly once
(neighbourhood at a level implies neighbourhood of the parents), so for a
kernel that is a polynomial of degree < p in each coordinate the result is
the exact sum: that is the pin of the tree logic.
"""
from __future__ import annotations

import numpy as np

TOP_SPAN = 4


def ml_nodes(L: int, p: int) -> np.ndarray:
    """The p lattice nodes of a cluster side of L cells, as offsets in [0, L)."""
    if p < 1 or p > L:
        raise ValueError("need 1 <= p <= L")
    j = np.arange(p)
    t = np.floor((L - 1) / 2.0 * (1.0 - np.cos(np.pi * (2 * j + 1) / (2 * p))) + 0.5).astype(np.int64)
    if len(np.unique(t)) != p:
        raise ValueError("rounded nodes coincide for L=%d, p=%d" % (L, p))
    return t


def lagrange(t: np.ndarray, x) -> np.ndarray:
    """W[j, m] = prod_{k != j} (x_m - t_k) / (t_j - t_k)."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    t = np.asarray(t, dtype=np.float64)
    W = np.ones((len(t), len(x)))
    for j in range(len(t)):
        for k in range(len(t)):
            if k != j:
                W[j] *= (x - t[k]) / (t[j] - t[k])
    return W


def ml_top_level(blocks: np.ndarray) -> int:
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    lev = 0
    while True:
        c = np.floor_divide(b, 1 << lev)
        if np.all(c.max(0) - c.min(0) + 1 <= TOP_SPAN):
            return lev
        lev += 1


def ml_table_extent(blocks, B: int) -> np.ndarray:
    """Largest |offset| per axis (xyz) the evaluator reads the kernel at: the
    nodes of the top-level clusters reach beyond the blocks themselves."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    top = ml_top_level(b)
    c = np.floor_divide(b, 1 << top)
    return (c.max(0) - c.min(0) + 1) * (B << top) - 1


def _adjacent(a, b) -> bool:
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]), abs(a[2] - b[2])) <= 1


def _parent(c):
    return (c[0] >> 1, c[1] >> 1, c[2] >> 1)


def _node_positions(c, L: int, t: np.ndarray) -> np.ndarray:
    """xyz lattice positions of a cluster's nodes, node a = (az p + ay) p + ax."""
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + np.asarray(c, dtype=np.int64) * L


def _tensor(Wz, Wy, Wx, a):
    """r[i, j, k] = sum Wz[i, l] Wy[j, m] Wx[k, n] a[l, m, n]."""
    return np.einsum("il,jm,kn,lmn->ijk", Wz, Wy, Wx, a)


def even_table_kernel(tab: np.ndarray):
    """Kernel K(d) = tab[|dz|, |dy|, |dx|] of an even table (as G_L, G_K)."""
    tab = np.asarray(tab, dtype=np.float64)

    def kern(d):
        d = np.abs(np.asarray(d, dtype=np.int64))
        return tab[d[..., 2], d[..., 1], d[..., 0]]
    return kern


def ml_conv(kern, src_blocks, f, tgt_blocks, B: int, p: int, dx: float = 1.0) -> np.ndarray:
    """u(n) ~= dx^2 sum_m K(n - m) f(m) on the target blocks by the multilevel
    evaluator above.  f: [nsrc, B, B, B] (z, y, x); returns [ntgt, B, B, B]."""
    src = [tuple(int(v) for v in b) for b in np.asarray(src_blocks).reshape(-1, 3)]
    tgt = [tuple(int(v) for v in b) for b in np.asarray(tgt_blocks).reshape(-1, 3)]
    f = np.asarray(f, dtype=np.float64).reshape(len(src), B, B, B)
    u = np.zeros((len(tgt), B, B, B))
    if not src or not tgt:
        return u
    top = ml_top_level(np.array(src + tgt))
    nodes = [ml_nodes(B << lev, p) for lev in range(top + 1)]

    # upward: P2M at the blocks, then M2M level by level
    M = [dict() for _ in range(top + 1)]
    W0 = lagrange(nodes[0], np.arange(B))
    for i, b in enumerate(src):
        M[0][b] = M[0].get(b, 0.0) + _tensor(W0, W0, W0, f[i])
    for lev in range(top):
        L = B << lev
        for c, m in M[lev].items():
            par = _parent(c)
            off = [c[k] * L - par[k] * 2 * L for k in range(3)]
            W = [lagrange(nodes[lev + 1], off[k] + nodes[lev]) for k in range(3)]
            M[lev + 1][par] = M[lev + 1].get(par, 0.0) + _tensor(W[2], W[1], W[0], m)

    # downward: L2L from the parent, plus M2L over the interaction list
    Phi = [dict() for _ in range(top + 1)]
    for lev in range(top, -1, -1):
        L = B << lev
        tclus = sorted({(b[0] >> lev, b[1] >> lev, b[2] >> lev) for b in tgt})
        for c in tclus:
            phi = np.zeros((p, p, p))
            if lev < top:
                par = _parent(c)
                off = [c[k] * L - par[k] * 2 * L for k in range(3)]
                W = [lagrange(nodes[lev + 1], off[k] + nodes[lev]) for k in range(3)]
                phi += _tensor(W[2].T, W[1].T, W[0].T, Phi[lev + 1][par])
            yc = _node_positions(c, L, nodes[lev])
            for s, m in M[lev].items():
                if _adjacent(s, c):
                    continue
                if lev < top and not _adjacent(_parent(s), _parent(c)):
                    continue
                K = kern(yc[:, None, :] - _node_positions(s, L, nodes[lev])[None, :, :])
                phi += (K @ m.reshape(-1)).reshape(p, p, p)
            Phi[lev][c] = phi

    # leaves: L2P plus the exact sum over neighbouring source blocks
    z, y, x = np.meshgrid(np.arange(B), np.arange(B), np.arange(B), indexing="ij")
    loc = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    for i, b in enumerate(tgt):
        u[i] = _tensor(W0.T, W0.T, W0.T, Phi[0][b])
        xt = loc + np.asarray(b) * B
        for j, s in enumerate(src):
            if _adjacent(s, b):
                K = kern(xt[:, None, :] - (loc + np.asarray(s) * B)[None, :, :])
                u[i] += (K @ f[j].reshape(-1)).reshape(B, B, B)
    return dx * dx * u


def ml_counts(src_blocks, tgt_blocks) -> dict:
    """The tree the evaluator above walks, counted: levels above the blocks,
    source and target clusters over all levels, node-to-node pairs and
    neighbouring block pairs (by the same definitions as ml_conv)."""
    src = {tuple(int(v) for v in b) for b in np.asarray(src_blocks).reshape(-1, 3)}
    tgt = {tuple(int(v) for v in b) for b in np.asarray(tgt_blocks).reshape(-1, 3)}
    top = ml_top_level(np.array(sorted(src | tgt)))
    ns = nt = m2l = 0
    for lev in range(top + 1):
        sc = {(b[0] >> lev, b[1] >> lev, b[2] >> lev) for b in src}
        tc = {(b[0] >> lev, b[1] >> lev, b[2] >> lev) for b in tgt}
        ns += len(sc)
        nt += len(tc)
        for c in tc:
            for s in sc:
                if not _adjacent(s, c) and (lev == top or _adjacent(_parent(s), _parent(c))):
                    m2l += 1
    near = sum(1 for t in tgt for s in src if _adjacent(s, t))
    return {"levels": top, "source_clusters": ns, "target_clusters": nt, "m2l_pairs": m2l, "near_pairs": near}


def direct_conv(kern, src_blocks, f, tgt_blocks, B: int, dx: float = 1.0) -> np.ndarray:
    """The exact sum dx^2 sum_m K(n - m) f(m) by brute force (small sets)."""
    src = np.asarray(src_blocks, dtype=np.int64).reshape(-1, 3)
    tgt = np.asarray(tgt_blocks, dtype=np.int64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(len(src), -1)
    z, y, x = np.meshgrid(np.arange(B), np.arange(B), np.arange(B), indexing="ij")
    loc = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    u = np.zeros((len(tgt), B ** 3))
    for i, b in enumerate(tgt):
        xt = loc + b * B
        for j, s in enumerate(src):
            u[i] += kern(xt[:, None, :] - (loc + s * B)[None, :, :]) @ f[j]
    return dx * dx * u.reshape(len(tgt), B, B, B)
