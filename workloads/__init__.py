"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method itself: it only builds block
sets (lists of integer block coordinates), source fields drawn from seeded
normal distributions, and marker positions.  Shapes follow the workloads of
Liska & Colonius: block-wise grids around a low-aspect-ratio flat plate at
incidence with its near wake (Sec. 5.3 geometry), spheres covered by
near-uniform Lagrangian markers (Sec. 5.4), and many small uneven block sets.

Conventions
  * block coordinates are int32 (bx, by, bz); a block of edge B covers cells
    b * B + [0, B)^3;
  * a field on a block set is float64 [ncomp, nblk, B, B, B] indexed
    [c, block, z, y, x] (x fastest), matching the library's device layout;
  * blocks are listed in (bz, by, bx) lexicographic order unless shuffled.
All randomness comes from numpy PCG64 seeded with 1604 + config number.
"""
from __future__ import annotations

import math

import numpy as np

SEED = 1604


def rng(config: int, extra: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED + config + 1000 * extra))


def sort_blocks(blocks: np.ndarray) -> np.ndarray:
    b = np.asarray(blocks, dtype=np.int32).reshape(-1, 3)
    order = np.lexsort((b[:, 0], b[:, 1], b[:, 2]))
    return np.ascontiguousarray(b[order])


def block_cells(blocks: np.ndarray, B: int) -> np.ndarray:
    """Lattice coordinates (x, y, z) of every cell, in [block, z, y, x] order."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    z, y, x = np.meshgrid(np.arange(B), np.arange(B), np.arange(B), indexing="ij")
    loc = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    cells = b[:, None, :] * B + loc[None, :, :]
    return cells.reshape(-1, 3)


def dense_box(blocks: np.ndarray, B: int, field: np.ndarray):
    """Scatter a [nblk, B, B, B] field into its bounding box; returns
    (origin xyz, box[z, y, x], mask)."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    lo = b.min(axis=0) * B
    hi = (b.max(axis=0) + 1) * B
    shape = tuple((hi - lo)[::-1])
    box = np.zeros(shape, dtype=np.float64)
    mask = np.zeros(shape, dtype=bool)
    f = np.asarray(field).reshape(-1, B, B, B)
    for i, bb in enumerate(b):
        o = bb * B - lo
        box[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = f[i]
        mask[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = True
    return lo, box, mask


# ----------------------------------------------------------------------------
# Small dense cube: 2 x 2 x 2 blocks of 8^3 cells
# ----------------------------------------------------------------------------

def cube_blocks(nb: int = 2) -> np.ndarray:
    return sort_blocks(np.array(list(np.ndindex(nb, nb, nb)), dtype=np.int32)[:, ::-1])


def normal_sources(nblk: int, B: int, ncomp: int = 1, config: int = 1, extra: int = 0) -> np.ndarray:
    return rng(config, extra).standard_normal((ncomp, nblk, B, B, B))


# ----------------------------------------------------------------------------
# Flat plate (aspect ratio 2, chord 64 cells, 30 deg incidence) with its wake
# ----------------------------------------------------------------------------

PLATE_CENTER = np.array([64.0, 96.0, 96.0])
PLATE_CHORD, PLATE_SPAN, PLATE_INCIDENCE_DEG = 64.0, 128.0, 30.0
PLATE_BOX_BLOCKS = (20, 12, 12)          # 320 x 192 x 192 cells at B = 16
ELLIPSOID_SEMI = np.array([64.0, 48.0, 96.0])
CONE_APEX_UPSTREAM, CONE_HALF_ANGLE_DEG = 64.0, 15.0


def _in_plate_region(p: np.ndarray) -> np.ndarray:
    v = (p - PLATE_CENTER) / ELLIPSOID_SEMI
    ell = np.sum(v * v, axis=-1) <= 1.0
    apex = PLATE_CENTER - np.array([CONE_APEX_UPSTREAM, 0.0, 0.0])
    w = p - apex
    rad = np.sqrt(w[..., 1] ** 2 + w[..., 2] ** 2)
    cone = (w[..., 0] > 0) & (rad <= w[..., 0] * math.tan(math.radians(CONE_HALF_ANGLE_DEG)))
    return ell | cone


def plate_blocks(B: int = 16) -> np.ndarray:
    """Blocks of the 320 x 192 x 192-cell box with a corner or the centre inside
    an ellipsoid around the plate or a downstream cone (1272 blocks at B=16)."""
    cells_box = np.array(PLATE_BOX_BLOCKS) * 16
    nb = cells_box // B
    out = []
    corners = np.array(list(np.ndindex(2, 2, 2)), dtype=np.float64)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                o = np.array([bx, by, bz], dtype=np.float64) * B
                pts = np.concatenate([o + corners * B, (o + B / 2.0)[None]], axis=0)
                if np.any(_in_plate_region(pts)):
                    out.append((bx, by, bz))
    return sort_blocks(np.array(out, dtype=np.int32))


def plate_distance(p: np.ndarray) -> np.ndarray:
    """Euclidean distance from points to the (zero-thickness) plate rectangle."""
    a = math.radians(PLATE_INCIDENCE_DEG)
    d = np.array([math.cos(a), -math.sin(a), 0.0])
    e = np.array([0.0, 0.0, 1.0])
    nrm = np.cross(d, e)
    v = p - PLATE_CENTER
    s = np.abs(v @ d) - PLATE_CHORD / 2.0
    w = np.abs(v @ e) - PLATE_SPAN / 2.0
    return np.sqrt(np.maximum(s, 0.0) ** 2 + np.maximum(w, 0.0) ** 2 + (v @ nrm) ** 2)


def plate_sources(blocks: np.ndarray, B: int = 16, ncomp: int = 3, config: int = 2) -> np.ndarray:
    """N(0,1) on cells whose centre lies within 4 cells of the plate, 1e-3 N(0,1)
    elsewhere; independent draws per component.  [ncomp, nblk, B, B, B]."""
    cells = block_cells(blocks, B).astype(np.float64) + 0.5
    near = (plate_distance(cells) <= 4.0).reshape(len(blocks), B, B, B)
    g = rng(config)
    out = np.empty((ncomp, len(blocks), B, B, B))
    for c in range(ncomp):
        z = g.standard_normal((len(blocks), B, B, B))
        out[c] = np.where(near, z, 1e-3 * z)
    return out


def lower_closed_blocks(blocks: np.ndarray) -> np.ndarray:
    """The blocks of a set whose neighbours at -e_x, -e_y and -e_z are also in
    the set (in the set's order)."""
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    have = set(map(tuple, b.tolist()))
    keep = [i for i, (x, y, z) in enumerate(b.tolist())
            if (x - 1, y, z) in have and (x, y - 1, z) in have and (x, y, z - 1) in have]
    return np.ascontiguousarray(b[keep].astype(np.int32))


def plate_near_blocks(blocks: np.ndarray, B: int = 16, count: int = 8) -> np.ndarray:
    """Indices (into ``blocks``) of the ``count`` blocks closest to the plate."""
    ctr = np.asarray(blocks, dtype=np.float64) * B + B / 2.0
    return np.argsort(plate_distance(ctr), kind="stable")[:count]


def sample_targets(nblk: int, B: int, n: int, must_blocks=(), config: int = 2) -> np.ndarray:
    """Seeded sample of flat cell indices (block * B^3 + local) containing every
    cell of ``must_blocks`` plus random others; sorted, unique."""
    g = rng(config, extra=7)
    must = np.concatenate([np.arange(B ** 3) + int(b) * B ** 3 for b in must_blocks]) \
        if len(must_blocks) else np.zeros(0, dtype=np.int64)
    rest = max(0, n - must.size)
    extra = g.choice(nblk * B ** 3, size=rest, replace=False) if rest else np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate([must, extra]).astype(np.int64))


# ----------------------------------------------------------------------------
# Batches of uneven compact blobs
# ----------------------------------------------------------------------------

def blob_instances(n_inst: int = 64, kmin: int = 1, kmax: int = 400, region: int = 16, config: int = 4):
    """n_inst block sets; instance i holds K_i = round(exp(U[ln kmin, ln kmax]))
    blocks: the K_i blocks of a region^3 block grid nearest a random centre in a
    metric with random axis weights U[0.5, 2]."""
    g = rng(config)
    out = []
    grid = np.array(list(np.ndindex(region, region, region)), dtype=np.float64)[:, ::-1]
    for _ in range(n_inst):
        k = int(round(math.exp(g.uniform(math.log(kmin), math.log(kmax)))))
        ctr = g.uniform(0.3 * region, 0.7 * region, size=3)
        wts = g.uniform(0.5, 2.0, size=3)
        d = np.sum(((grid + 0.5 - ctr) * wts) ** 2, axis=1)
        pick = np.argsort(d, kind="stable")[:k]
        out.append(sort_blocks(grid[pick].astype(np.int32)))
    return out


# ----------------------------------------------------------------------------
# Spheres of Lagrangian markers
# ----------------------------------------------------------------------------

def fibonacci_sphere(n: int, radius: float, center) -> np.ndarray:
    """n near-uniform points on a sphere (Fibonacci lattice), float64 [n, 3]."""
    i = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = math.pi * (3.0 - math.sqrt(5.0)) * i
    pts = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)
    return pts * radius + np.asarray(center, dtype=np.float64)[None, :]


SPHERE_CENTER = np.array([40.37, 40.21, 40.13])


def sphere_markers(diameter: float = 32.0, n: int = 4000, center=None) -> np.ndarray:
    c = SPHERE_CENTER if center is None else np.asarray(center, dtype=np.float64)
    return fibonacci_sphere(n, diameter / 2.0, c)


def heave_velocity(step: int, diameter: float = 32.0, amplitude: float = 0.25,
                   period: int = 200) -> float:
    """Body velocity for y(t) = amplitude * D * sin(2 pi t / period), in cells
    per step (the Lagrangian points move rigidly; the grid moves with them)."""
    return amplitude * diameter * (2.0 * math.pi / period) * math.cos(2.0 * math.pi * step / period)


def shell_blocks(diameter: float, B: int = 8, center=None) -> np.ndarray:
    """Blocks of B^3 whose centre lies within B of a sphere surface of the
    given diameter (a near-surface source / target region two blocks thick,
    sparse in its bounding box), sorted by (z, y, x)."""
    c = np.zeros(3) if center is None else np.asarray(center, dtype=np.float64)
    R = diameter / 2.0
    n = int(math.ceil((R + 2 * B) / B))
    g = np.arange(-n - 1, n + 1)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    b = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    d = np.linalg.norm((b + 0.5) * B - c[None, :], axis=1)
    return sort_blocks(b[np.abs(d - R) <= B])


def spd_matrix(n: int, cond: float = 1e3, seed: int = 0) -> np.ndarray:
    """Seeded symmetric positive definite test matrix [n, n] (float64): a
    random orthogonal basis (QR of a normal matrix) with eigenvalues spaced
    geometrically from 1 to ``cond``.  Input data for the dense force-solve
    tests; the matrices of the method itself come from the Schur operator."""
    g = np.random.Generator(np.random.PCG64(1604 + 7 * 1000 + seed))
    if n == 0:
        return np.zeros((0, 0))
    q, r = np.linalg.qr(g.standard_normal((n, n)))
    q *= np.sign(np.diag(r))[None, :]
    lam = np.geomspace(1.0, cond, n) if n > 1 else np.ones(1)
    a = (q * lam[None, :]) @ q.T
    return 0.5 * (a + a.T)
