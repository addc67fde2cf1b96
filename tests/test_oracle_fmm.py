"""Pins of the oracle's multilevel interpolation evaluator of the lattice
convolution (Sec. 2.2, Eq. dpoisson_conv).

What fixes them, independently of the code under test:
- the rounded Chebyshev nodes are distinct lattice points of the cluster and
  the Lagrange weights reproduce polynomials of degree < p;
- for a kernel that is a polynomial of degree < p in each coordinate every
  interpolation step is exact, so the evaluator equals the brute-force sum:
  a pair counted twice or missed, a wrong node offset or a wrong parent
  offset in M2M / L2L breaks it;
- with every block a neighbour of every other there is no far field and the
  result is the exact sum;
- on G_L the error against the exact sum (the C direct sum) falls as p
  grows and is small at p = 4.
"""
import numpy as np
import pytest

import oracle
from oracle import fmm


def _rand_set(seed, n, region):
    g = np.random.Generator(np.random.PCG64(seed))
    allb = np.array(list(np.ndindex(*region)), dtype=np.int64)[:, ::-1] - np.array([3, 1, 2])
    return allb[np.sort(g.choice(len(allb), n, replace=False))], g


@pytest.mark.parametrize("L,p", [(4, 4), (8, 4), (8, 5), (8, 6), (16, 4), (64, 5), (512, 4)])
def test_nodes_and_weights(L, p):
    t = fmm.ml_nodes(L, p)
    assert len(set(t.tolist())) == p and t.min() >= 0 and t.max() <= L - 1
    x = np.arange(L)
    W = fmm.lagrange(t, x)
    for k in range(p):
        assert np.max(np.abs(W.T @ (t.astype(float) / L) ** k - (x / L) ** k)) < 1e-9
    # interpolating at the nodes is the identity
    assert np.max(np.abs(fmm.lagrange(t, t) - np.eye(p))) < 1e-13


def test_top_level_rule():
    assert fmm.ml_top_level(np.array([[0, 0, 0], [3, 3, 3]])) == 0
    assert fmm.ml_top_level(np.array([[0, 0, 0], [4, 0, 0]])) == 1
    assert fmm.ml_top_level(np.array([[-9, 0, 0], [9, 2, 1]])) == 3
    # clusters of 8 blocks from -16 to 15 on x: 4 clusters of 64 cells
    assert fmm.ml_table_extent(np.array([[-9, 0, 0], [9, 2, 1]]), 8).tolist() == [255, 63, 63]


def test_tree_counts_hand_case():
    two = np.array([[0, 0, 0], [3, 0, 0]])
    assert fmm.ml_counts(two, two) == {"levels": 0, "source_clusters": 2, "target_clusters": 2,
                                       "m2l_pairs": 2, "near_pairs": 2}
    # x from 0 to 5: one level of clusters (0..2 on x); blocks 0 and 5 have the
    # parents 0 and 2, which are not neighbours, so the pair is counted once,
    # at the top level (each direction)
    ends = np.array([[0, 0, 0], [5, 0, 0]])
    c = fmm.ml_counts(ends, ends)
    assert c["levels"] == 1 and c["source_clusters"] == 4 and c["m2l_pairs"] == 2 and c["near_pairs"] == 2


def _poly_kernel(d):
    d = np.asarray(d, dtype=np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    return 0.7 + 0.3 * x - 0.2 * y * y + 0.1 * x * y * z + 0.05 * z ** 3 - 0.01 * x * x * z * z


@pytest.mark.parametrize("B,p,seed", [(4, 4, 1), (8, 4, 2), (8, 5, 3)])
def test_exact_for_a_polynomial_kernel(B, p, seed):
    n = 30 if B == 4 else 14
    src, g = _rand_set(seed, n, (9, 6, 7))
    tgt, _ = _rand_set(seed + 10, n - 4, (9, 6, 7))
    tgt = tgt + np.array([1, 0, -1])        # targets partly outside the sources
    assert fmm.ml_top_level(np.concatenate([src, tgt])) >= 1
    f = g.standard_normal((len(src), B, B, B))
    got = fmm.ml_conv(_poly_kernel, src, f, tgt, B, p, dx=0.5)
    ref = fmm.direct_conv(_poly_kernel, src, f, tgt, B, dx=0.5)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_a_dropped_pair_breaks_the_polynomial_pin():
    """The pin can tell: a reference that leaves one source block out (a
    pair missed) fails it."""
    B, p = 4, 4
    src, g = _rand_set(7, 20, (8, 5, 6))
    f = g.standard_normal((len(src), B, B, B))
    got = fmm.ml_conv(_poly_kernel, src, f, src, B, p)
    f2 = f.copy()
    f2[3] *= 0.0
    ref = fmm.direct_conv(_poly_kernel, src, f2, src, B)
    assert np.max(np.abs(got - ref)) > 1e-3 * np.max(np.abs(ref))


def test_no_far_field_is_exact():
    B = 4
    blocks = np.array(list(np.ndindex(2, 2, 2)), dtype=np.int64)
    f = np.random.Generator(np.random.PCG64(4)).standard_normal((8, B, B, B))
    tab = oracle.lgf_table(7, 7, 7)
    kern = fmm.even_table_kernel(tab)
    got = fmm.ml_conv(kern, blocks, f, blocks, B, 3)
    cells = np.concatenate([np.stack(np.meshgrid(np.arange(B), np.arange(B), np.arange(B), indexing="ij")[::-1], -1)
                            .reshape(-1, 3) + b * B for b in blocks])
    ref = oracle.conv_direct(tab, cells, f.reshape(-1), cells)
    assert np.max(np.abs(got.reshape(-1) - ref)) < 1e-12 * np.max(np.abs(ref))


def test_error_on_the_lattice_green_function_falls_with_p():
    """A sparse set of 8^3 blocks spread over several levels of clusters: the
    error against the exact sum at p = 3, 4, 5, 6."""
    B = 8
    g = np.random.Generator(np.random.PCG64(9))
    src = np.unique(g.integers(-6, 7, size=(14, 3)), axis=0)
    tgt = np.unique(np.concatenate([src[:6], g.integers(-6, 7, size=(4, 3))]), axis=0)
    f = g.standard_normal((len(src), B, B, B))
    tab = oracle.lgf_table(*[int(v) for v in fmm.ml_table_extent(np.concatenate([src, tgt]), B)])
    kern = fmm.even_table_kernel(tab)
    ref = fmm.direct_conv(kern, src, f, tgt, B)
    err = []
    for p in (3, 4, 5, 6):
        got = fmm.ml_conv(kern, src, f, tgt, B, p)
        err.append(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err[0] > err[1] > err[2] > err[3], err
    assert err[1] < 3e-4 and err[2] < 1e-4 and err[3] < 5e-6, err
