"""GPU parity of the LGF tables, the block-wise Poisson / K^{-1} convolution and
the integrating factor against the FP64 oracle (all calls through the C ABI).

Bars: FP64 paths <= 1e-12 and FP32 paths <= 1e-5 in relative max-norm error
||u - u_ref||_inf / ||u_ref||_inf per component."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _relerr(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def _span_ext(src, tgt, B):
    allb = np.concatenate([np.asarray(src).reshape(-1, 3), np.asarray(tgt).reshape(-1, 3)])
    return tuple(int(v) for v in ((allb.max(0) - allb.min(0) + 1) * B - 1))


# ------------------------------------------------------------------ tables

def test_table_L_matches_oracle(ctx):
    ext = (40, 30, 20)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    g = lg.lgf_table_copy(ctx, t, ext)
    ref = oracle.lgf_table(*ext)
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-13


def test_table_far_field_region(ctx):
    """Entries beyond the quadrature radius use the far-field expansion."""
    ext = (300, 6, 4)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    g = lg.lgf_table_copy(ctx, t, ext)
    ref = oracle.lgf_table(*ext)
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-13


@pytest.mark.parametrize("alpha", [0.05, 0.5])
def test_table_K_matches_oracle(ctx, alpha):
    ext = (20, 20, 20)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_K, alpha, ext)
    g = lg.lgf_table_copy(ctx, t, ext)
    ref = oracle.lgf_k_table(alpha, *ext)
    assert np.max(np.abs(g - ref)) < 1e-16


@pytest.mark.parametrize("a", [0.02, 0.05, 0.1, 0.5])
def test_if_weights(ctx, a):
    """GPU Miller recurrence vs the oracle's series/trapezoid: a few ulp relative
    (the recurrence's rounding grows mildly with the order)."""
    r, w = lg.lgf_if_weights(ctx, a)
    ref = oracle.if_factors(a)
    assert r == len(ref) - 1
    assert np.all(np.abs(w - ref) <= 1e-14 * ref + 1e-25)
    # the FP32 applies' radius: the last factor at or above 2^-28
    r32, w32 = lg.lgf_if_weights(ctx, a, lg.IF_CUTOFF_F32)
    assert r32 == int(np.max(np.nonzero(ref >= 2.0 ** -28)[0]))
    assert np.array_equal(w32, w[:r32 + 1])


# ------------------------------------------------------------- Poisson

def _poisson(ctx, B, src, tgt, f, dtype, kind=lg.LGF_KIND_L, alpha=0.0, dx=1.0):
    ext = _span_ext(src, tgt, B)
    t = lg.lgf_table_build(ctx, kind, alpha, ext)
    fd = _dev(f, dtype)
    ud = torch.zeros((f.shape[0], len(tgt), B, B, B), dtype=fd.dtype, device="cuda")
    lg.lgf_poisson_apply(ctx, t, B, src, tgt, fd, ud, dx=dx)
    torch.cuda.synchronize()
    return ud.cpu().numpy().astype(np.float64)


def _oracle_poisson(B, src, tgt, f, table):
    sc = workloads.block_cells(src, B)
    tc = workloads.block_cells(tgt, B)
    out = np.empty((f.shape[0], len(tgt), B, B, B))
    for c in range(f.shape[0]):
        out[c] = oracle.conv_direct(table, sc, f[c].reshape(-1), tc).reshape(len(tgt), B, B, B)
    return out


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_poisson_small_cube(ctx, dtype):
    """2x2x2 blocks of 8^3 (16^3 cells), f ~ N(0,1): u = G * f, and L u = f on
    the 14^3 interior."""
    B = 8
    blocks = workloads.cube_blocks(2)
    f = workloads.normal_sources(len(blocks), B)
    u = _poisson(ctx, B, blocks, blocks, f, dtype)
    G = oracle.lgf_table(15, 15, 15)
    ref = _oracle_poisson(B, blocks, blocks, f, G)
    assert _relerr(u, ref) < TOL[dtype]
    if dtype == np.float64:
        _, ubox, _ = workloads.dense_box(blocks, B, u[0])
        _, fbox, _ = workloads.dense_box(blocks, B, f[0])
        res = oracle.laplacian_7pt(ubox) - fbox[1:-1, 1:-1, 1:-1]
        assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(ubox))


def _random_sets(seed, B, nsrc, ntgt, region):
    g = np.random.Generator(np.random.PCG64(seed))
    allb = np.array(list(np.ndindex(*region)), dtype=np.int32)[:, ::-1] + np.array([-3, 2, -1], dtype=np.int32)
    s = allb[g.choice(len(allb), nsrc, replace=False)]
    t = allb[g.choice(len(allb), ntgt, replace=False)]
    return s, t


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("B", [4, 8])
def test_poisson_ragged_sets(ctx, dtype, B):
    """Disconnected, non-convex source and target sets that differ; 2 components;
    a box that is not 2,3,5-smooth in blocks (7 along z) so it gets padded."""
    src, tgt = _random_sets(11 + B, B, 17, 13, (5, 6, 7))
    f = np.random.Generator(np.random.PCG64(3)).standard_normal((2, len(src), B, B, B))
    u = _poisson(ctx, B, src, tgt, f, dtype)
    ext = _span_ext(src, tgt, B)
    G = oracle.lgf_table(*ext)
    ref = _oracle_poisson(B, src, tgt, f, G)
    for c in range(2):
        assert _relerr(u[c], ref[c]) < TOL[dtype]


def test_poisson_order_invariance_and_accumulate(ctx):
    B = 4
    src, tgt = _random_sets(5, B, 9, 11, (4, 4, 4))
    g = np.random.Generator(np.random.PCG64(9))
    f = g.standard_normal((1, len(src), B, B, B))
    u1 = _poisson(ctx, B, src, tgt, f, np.float64)
    ps = g.permutation(len(src))
    pt = g.permutation(len(tgt))
    u2 = _poisson(ctx, B, src[ps], tgt[pt], f[:, ps], np.float64)
    assert np.array_equal(u2, u1[:, pt])
    # accumulate adds into u
    ext = _span_ext(src, tgt, B)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    u0 = g.standard_normal((1, len(tgt), B, B, B))
    ud = _dev(u0, np.float64)
    lg.lgf_poisson_apply(ctx, t, B, src, tgt, _dev(f, np.float64), ud, accumulate=True)
    assert np.max(np.abs(ud.cpu().numpy() - (u0 + u1))) < 1e-13


def test_poisson_dx_scaling(ctx):
    B = 4
    src, tgt = _random_sets(6, B, 5, 5, (3, 3, 3))
    f = np.random.Generator(np.random.PCG64(1)).standard_normal((1, len(src), B, B, B))
    u1 = _poisson(ctx, B, src, tgt, f, np.float64)
    u2 = _poisson(ctx, B, src, tgt, f, np.float64, dx=0.5)
    assert np.max(np.abs(u2 - 0.25 * u1)) < 1e-15 * np.max(np.abs(u1)) * 10


def test_kinv_matches_oracle(ctx):
    """K^{-1} f = G_K(a) * f with the G_K table (Sec. 2.2)."""
    B, alpha = 8, 0.05
    src, tgt = _random_sets(8, B, 6, 7, (3, 3, 3))
    f = np.random.Generator(np.random.PCG64(4)).standard_normal((1, len(src), B, B, B))
    u = _poisson(ctx, B, src, tgt, f, np.float64, kind=lg.LGF_KIND_K, alpha=alpha)
    ext = _span_ext(src, tgt, B)
    ref = _oracle_poisson(B, src, tgt, f, oracle.lgf_k_table(alpha, *ext))
    assert _relerr(u, ref) < 1e-12


def test_poisson_edge_cases(ctx):
    B = 4
    blk = np.array([[0, 0, 0], [1, 0, 0]], dtype=np.int32)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (7, 3, 3))
    f = torch.ones((1, 2, B, B, B), dtype=torch.float64, device="cuda")
    u = torch.full((1, 2, B, B, B), 7.0, dtype=torch.float64, device="cuda")
    # no sources: u is zeroed
    lg.lgf_poisson_apply(ctx, t, B, np.zeros((0, 3), np.int32), blk,
                         torch.zeros((1, 0, B, B, B), dtype=torch.float64, device="cuda"), u)
    assert float(u.abs().max()) == 0.0
    # duplicate blocks
    dup = np.array([[0, 0, 0], [0, 0, 0]], dtype=np.int32)
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_poisson_apply(ctx, t, B, dup, blk, f, u)
    assert e.value.code == lg.LGFIB_EDUP_BLOCK
    # table too small for the span
    far = np.array([[0, 0, 0], [5, 0, 0]], dtype=np.int32)
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_poisson_apply(ctx, t, B, far, far, f, u)
    assert e.value.code == lg.LGFIB_ERANGE
    # aliasing
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_poisson_apply(ctx, t, B, blk, blk, f, f)
    assert e.value.code == lg.LGFIB_EINVAL


@pytest.fixture(scope="module")
def plate():
    B = 16
    blocks = workloads.plate_blocks(B)
    f = workloads.plate_sources(blocks, B, ncomp=3)
    near = workloads.plate_near_blocks(blocks, B, 8)
    g = np.random.Generator(np.random.PCG64(77))
    picks = [int(b) * B ** 3 + int(v) for b in near for v in g.choice(B ** 3, 4, replace=False)]
    rnd = g.choice(len(blocks) * B ** 3, 96, replace=False)
    sample = np.unique(np.concatenate([picks, rnd]).astype(np.int64))
    G = oracle.lgf_table(*_span_ext(blocks, blocks, B))
    cells = workloads.block_cells(blocks, B)
    refs = [oracle.conv_direct(G, cells, f[c].reshape(-1), cells[sample]) for c in range(3)]
    return B, blocks, f, sample, refs


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_poisson_plate_wake_full_size(ctx, plate, dtype):
    """The 1272-block plate-and-wake set (5.2M cells per component, 3
    components) at full size, in the launch configuration the benchmark
    times; checked on a seeded sample of 128 target cells (32 next to the
    plate) against the direct sum."""
    B, blocks, f, sample, refs = plate
    assert len(blocks) == 1272
    u = _poisson(ctx, B, blocks, blocks, f, dtype)
    for c in range(3):
        got = u[c].reshape(-1)[sample]
        assert _relerr(got, refs[c]) < TOL[dtype], c


@pytest.mark.parametrize("B", [8, 16])
def test_poisson_tall_z_box(ctx, B):
    """A ragged column of blocks 192 cells tall (z FFT length 384, the
    benchmark's z pass) with a few blocks beside it, so the x and y spectra
    hold the zero and Nyquist rows of ky; two components, FP32, against the
    direct sum on every cell of three target blocks and a seeded sample."""
    nz = 192 // B
    col = [(0, 0, z) for z in range(nz) if z not in (3, nz - 5)]
    src = np.array(col + [(1, 0, 2), (0, 1, nz - 3)], dtype=np.int32)
    tgt = np.array(col[::2] + [(1, 1, 5), (1, 0, 2)], dtype=np.int32)
    g = np.random.Generator(np.random.PCG64(97 + B))
    f = g.standard_normal((2, len(src), B, B, B))
    u = _poisson(ctx, B, src, tgt, f, np.float32)
    G = oracle.lgf_table(*_span_ext(src, tgt, B))
    sc, tc = workloads.block_cells(src, B), workloads.block_cells(tgt, B)
    pick = np.unique(np.concatenate([np.arange(B ** 3) + B ** 3 * i for i in (0, len(tgt) - 2, len(tgt) - 1)]
                                    + [g.choice(len(tc), 256, replace=False)]))
    for c in range(2):
        ref = oracle.conv_direct(G, sc, f[c].reshape(-1), tc[pick])
        assert _relerr(u[c].reshape(-1)[pick], ref) < TOL[np.float32], c


@pytest.mark.parametrize("B,nb", [(8, (1, 1, 1)), (8, (5, 9, 15)), (16, (9, 1, 2)), (32, (9, 1, 1))])
def test_poisson_box_lengths(ctx, B, nb):
    """Boxes whose FFT lengths take the less common radix plans (16; 80, 144,
    240; 288; 576 points): a sparse set spanning nb blocks per axis, one
    component, FP32, against the direct sum on a seeded sample."""
    g = np.random.Generator(np.random.PCG64(sum(nb) + B))
    cand = [(x, 0, 0) for x in range(nb[0])] + [(0, y, 0) for y in range(nb[1])] + \
           [(0, 0, z) for z in range(nb[2])] + [(nb[0] - 1, nb[1] - 1, nb[2] - 1)]
    blocks = np.array(sorted(set(cand), key=lambda b: (b[2], b[1], b[0])), dtype=np.int32)
    f = g.standard_normal((1, len(blocks), B, B, B))
    u = _poisson(ctx, B, blocks, blocks, f, np.float32)
    G = oracle.lgf_table(*_span_ext(blocks, blocks, B))
    cells = workloads.block_cells(blocks, B)
    pick = np.unique(g.choice(len(cells), min(len(cells), 384), replace=False))
    ref = oracle.conv_direct(G, cells, f[0].reshape(-1), cells[pick])
    assert _relerr(u[0].reshape(-1)[pick], ref) < TOL[np.float32]


# ----------------------------------------------------- integrating factor

def _oracle_if(B, src, tgt, f, a):
    ker = oracle.if_kernel_table(a)
    sc = workloads.block_cells(src, B)
    tc = workloads.block_cells(tgt, B)
    out = np.empty((f.shape[0], len(tgt), B, B, B))
    for c in range(f.shape[0]):
        out[c] = oracle.conv_direct(ker, sc, f[c].reshape(-1), tc).reshape(len(tgt), B, B, B)
    return out


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("a", [0.005, 0.02, 0.1, 0.2, 0.3, 0.5])
def test_if_apply_cube(ctx, dtype, a):
    """FP32 radii 3, 4, 5, 6, 7 and 8 (FP64 radii 5 to 12) on 8^3 blocks."""
    B = 8
    blocks = workloads.cube_blocks(2)
    f = workloads.normal_sources(len(blocks), B, ncomp=1, config=3)
    fd = _dev(f, dtype)
    ud = torch.zeros_like(fd)
    lg.lgf_if_apply(ctx, a, B, blocks, blocks, fd, ud)
    u = ud.cpu().numpy().astype(np.float64)
    ref = _oracle_if(B, blocks, blocks, f, a)
    assert _relerr(u, ref) < TOL[dtype]


@pytest.mark.parametrize("B", [4, 8, 16])
def test_if_apply_ragged(ctx, B):
    """Radius 12 (a = 0.5) reaches two blocks away for B = 4 and 8."""
    src, tgt = _random_sets(21 + B, B, 14, 10, (4, 5, 4))
    f = np.random.Generator(np.random.PCG64(8)).standard_normal((2, len(src), B, B, B))
    for a in (0.05, 0.5):
        fd = _dev(f, np.float64)
        ud = torch.zeros((2, len(tgt), B, B, B), dtype=torch.float64, device="cuda")
        lg.lgf_if_apply(ctx, a, B, src, tgt, fd, ud)
        ref = _oracle_if(B, src, tgt, f, a)
        assert _relerr(ud.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("a", [0.005, 0.02, 0.05, 0.1, 0.2, 0.3, 0.5])
def test_if_apply_b16_fp32_ragged(ctx, a):
    """B = 16 in FP32 (FP32 radii 3 to 8, every thread count and LDS plane
    stride of the row-register kernel) on disconnected source and target sets
    that differ, against the oracle's kernel at the full FP64 radius."""
    B = 16
    src, tgt = _random_sets(31, B, 10, 8, (4, 5, 4))
    f = np.random.Generator(np.random.PCG64(9)).standard_normal((1, len(src), B, B, B))
    fd = _dev(f, np.float32)
    ud = torch.zeros((1, len(tgt), B, B, B), dtype=torch.float32, device="cuda")
    lg.lgf_if_apply(ctx, a, B, src, tgt, fd, ud)
    ref = _oracle_if(B, src, tgt, f, a)
    assert _relerr(ud.cpu().numpy().astype(np.float64), ref) < TOL[np.float32]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_if_apply_plate_wake_full_size(ctx, plate, dtype):
    """E(0.1) on the 1272-block plate-and-wake set, 3 components, in the
    launch configuration the benchmark times, on the seeded sample of target
    cells against the windowed direct sum of the product kernel."""
    B, blocks, f, sample, _ = plate
    fd = _dev(f, dtype)
    ud = torch.zeros_like(fd)
    lg.lgf_if_apply(ctx, 0.1, B, blocks, blocks, fd, ud)
    u = ud.cpu().numpy().astype(np.float64)
    ker = oracle.if_kernel_table(0.1)
    cells = workloads.block_cells(blocks, B)[sample]
    for c in range(3):
        lo, box, _ = workloads.dense_box(blocks, B, f[c])
        ref = oracle.conv_window(ker, box, lo, cells)
        assert _relerr(u[c].reshape(-1)[sample], ref) < TOL[dtype], c


def test_if_apply_zero_is_identity(ctx):
    B = 8
    blocks = workloads.cube_blocks(2)
    f = workloads.normal_sources(len(blocks), B)
    fd = _dev(f, np.float64)
    ud = torch.zeros_like(fd)
    lg.lgf_if_apply(ctx, 0.0, B, blocks, blocks, fd, ud)
    assert torch.equal(ud, fd)
