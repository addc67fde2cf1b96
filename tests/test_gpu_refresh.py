"""GPU parity of the velocity refresh (Sec. 4.1, Eq. vel_refresh) against the
FP64 oracle through the C ABI: ragged flow and vorticity sets with B = 4 and
8 (vorticity blocks on the lower boundary of the flow set, so the source side
reaches outside it), exact reproduction of a compact solenoidal field, the
argument checks, and the 1272-block plate-and-wake set at full size on
sampled cells.

Bars as for the Poisson apply the refresh runs on: FP64 <= 1e-12 and FP32 <=
1e-5 in relative max-norm error per component."""
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


def _rel(a, ref):
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def _sources(vort):
    """Vorticity blocks and their lower neighbours: the blocks the refresh's
    source term occupies (it decides the table extent the call needs)."""
    v = np.asarray(vort).reshape(-1, 3)
    return np.concatenate([v] + [v - np.eye(3, dtype=v.dtype)[a] for a in range(3)])


def _ext(blocks_a, blocks_b, B):
    allb = np.concatenate([np.asarray(blocks_a).reshape(-1, 3), np.asarray(blocks_b).reshape(-1, 3)])
    return tuple(int(v) for v in ((allb.max(0) - allb.min(0) + 1) * B - 1))


def _to_box(field, blocks, B, origin, shape):
    box = np.zeros((3,) + tuple(shape))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = field[:, i]
    return box


def _from_box(box, blocks, B, origin):
    out = np.zeros((3, len(blocks), B, B, B))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        out[:, i] = box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B]
    return out


def _oracle(u_blocks, flow, vort, B):
    origin, fmask = oracle.block_mask(flow, B)
    vmask = np.zeros_like(fmask)
    for b in vort:
        o = np.asarray(b) * B - origin
        vmask[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = True
    gl = oracle.lgf_table(*fmask.shape[::-1])
    ubox = _to_box(u_blocks, flow, B, origin, fmask.shape)
    out = oracle.velocity_refresh(ubox, fmask, vmask, origin, gl)
    return _from_box(out, flow, B, origin)


def _gpu(ctx, u_blocks, flow, vort, B, dtype):
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, _ext(_sources(vort), flow, B))
    u = torch.from_numpy(np.ascontiguousarray(u_blocks, dtype=dtype)).cuda()
    lg.lgf_velocity_refresh(ctx, t, B, vort, flow, u)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64)


def _ragged(seed, region, drop, nvort):
    g = np.random.Generator(np.random.PCG64(seed))
    allb = np.array(list(np.ndindex(*region)), dtype=np.int32)[:, ::-1] + np.array([2, -1, 0], dtype=np.int32)
    flow = allb[np.sort(g.choice(len(allb), len(allb) - drop, replace=False))]
    vort = flow[g.choice(len(flow), nvort, replace=False)]
    return flow, vort


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("B", [4, 8])
def test_refresh_ragged_sets_match_oracle(ctx, dtype, B):
    flow, vort = _ragged(20 + B, (4, 3, 5), 9, 14)
    lo = flow.min(0)
    # at least one vorticity block on the lower boundary of the flow set
    assert np.any(np.any(vort == lo[None, :], axis=1))
    u = np.random.Generator(np.random.PCG64(B)).standard_normal((3, len(flow), B, B, B))
    u = u.astype(dtype).astype(np.float64)
    got = _gpu(ctx, u, flow, vort, B, dtype)
    ref = _oracle(u, flow, vort, B)
    for c in range(3):
        assert _rel(got[c], ref[c]) < TOL[dtype], c


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_refresh_b32_on_sampled_cells(ctx, dtype):
    """Blocks of 32^3, which the kernel splits into several tiles per block;
    checked on a seeded sample of cells, tile edges included."""
    B = 32
    flow = np.array([(x, y, z) for z in range(2) for y in range(2) for x in range(2)], dtype=np.int32)[:7]
    vort = flow[[0, 3, 6]]
    g = np.random.Generator(np.random.PCG64(32))
    u = g.standard_normal((3, len(flow), B, B, B)).astype(dtype).astype(np.float64)
    got = _gpu(ctx, u, flow, vort, B, dtype)
    origin, fmask = oracle.block_mask(flow, B)
    vmask = np.zeros_like(fmask)
    for b in vort:
        o = np.asarray(b) * B - origin
        vmask[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = True
    edges = [i * B ** 3 + (z * B + y) * B + x for i in range(len(flow)) for (x, y, z) in
             ((15, 3, 9), (16, 16, 16), (0, 31, 15), (31, 0, 16), (7, 15, 31))]
    sample = np.unique(np.concatenate([edges, g.choice(len(flow) * B ** 3, 150, replace=False)]))
    cells = workloads.block_cells(flow, B)[sample]
    ref = oracle.velocity_refresh_at(_to_box(u, flow, B, origin, fmask.shape), fmask, vmask, origin,
                                     oracle.lgf_table(*fmask.shape[::-1]), cells)
    for c in range(3):
        assert _rel(got[c].reshape(-1)[sample], ref[:, c]) < TOL[dtype], c


def test_refresh_reproduces_a_compact_solenoidal_field(ctx):
    B = 8
    flow = np.array([(x, y, z) for z in range(4) for y in range(4) for x in range(4)], dtype=np.int32)
    vort = np.array([(x, y, z) for z in (1, 2) for y in (1, 2) for x in (1, 2)], dtype=np.int32)
    origin, fmask = oracle.block_mask(flow, B)
    psi = np.zeros((3,) + fmask.shape)
    psi[:, 11:21, 10:22, 12:20] = np.random.Generator(np.random.PCG64(4)).standard_normal((3, 10, 12, 8))
    ubox = oracle.curl_adjoint(psi)
    u = _from_box(ubox, flow, B, origin)
    got = _gpu(ctx, u, flow, vort, B, np.float64)
    assert _rel(got, u) < 1e-11
    # an error two or more cells away from the vorticity blocks (cells 8..23
    # on each axis) never enters C u there, and the refresh removes it
    err = np.random.Generator(np.random.PCG64(5)).standard_normal((3,) + fmask.shape)
    err[:, 6:26, 6:26, 6:26] = 0.0
    noisy = u + _from_box(err, flow, B, origin)
    got = _gpu(ctx, noisy, flow, vort, B, np.float64)
    assert _rel(got, u) < 1e-11


def test_refresh_argument_checks(ctx):
    B = 4
    flow = workloads.cube_blocks(2)
    t = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (15, 15, 15))
    u = torch.ones((3, len(flow), B, B, B), dtype=torch.float64, device="cuda")
    # no vorticity: the refreshed velocity is zero
    lg.lgf_velocity_refresh(ctx, t, B, np.zeros((0, 3), np.int32), flow, u)
    assert float(u.abs().max()) == 0.0
    with pytest.raises(lg.LgfibError) as e:   # vorticity block outside the flow set
        lg.lgf_velocity_refresh(ctx, t, B, np.array([[5, 5, 5]], np.int32), flow, u)
    assert e.value.code == lg.LGFIB_EINVAL
    with pytest.raises(lg.LgfibError) as e:   # duplicate flow block
        lg.lgf_velocity_refresh(ctx, t, B, flow[:1], np.concatenate([flow, flow[:1]]),
                                torch.zeros((3, len(flow) + 1, B, B, B), dtype=torch.float64, device="cuda"))
    assert e.value.code == lg.LGFIB_EDUP_BLOCK
    tk = lg.lgf_table_build(ctx, lg.LGF_KIND_K, 0.05, (15, 15, 15))
    with pytest.raises(lg.LgfibError) as e:   # needs G_L
        lg.lgf_velocity_refresh(ctx, tk, B, flow[:1], flow, u)
    assert e.value.code == lg.LGFIB_EINVAL
    ts = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (7, 7, 7))
    with pytest.raises(lg.LgfibError) as e:   # table shorter than the span
        lg.lgf_velocity_refresh(ctx, ts, B, flow[:1], flow, u)
    assert e.value.code == lg.LGFIB_ERANGE


@pytest.fixture(scope="module")
def plate_refresh():
    B = 16
    flow = workloads.plate_blocks(B)
    vort = workloads.lower_closed_blocks(flow)
    u = workloads.plate_sources(flow, B, ncomp=3).astype(np.float32).astype(np.float64)
    g = np.random.Generator(np.random.PCG64(78))
    near = workloads.plate_near_blocks(flow, B, 8)
    vset = set(map(tuple, vort.tolist()))
    edge = [i for i, b in enumerate(flow.tolist()) if tuple(b) not in vset]
    picks = [int(b) * B ** 3 + int(v) for b in near for v in g.choice(B ** 3, 4, replace=False)]
    picks += [int(b) * B ** 3 + int(v) for b in g.choice(edge, 8, replace=False) for v in g.choice(B ** 3, 4, replace=False)]
    rnd = g.choice(len(flow) * B ** 3, 64, replace=False)
    sample = np.unique(np.concatenate([picks, rnd]).astype(np.int64))
    origin, fmask = oracle.block_mask(flow, B)
    vmask = np.zeros_like(fmask)
    for b in vort:
        o = np.asarray(b) * B - origin
        vmask[o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B] = True
    gl = oracle.lgf_table(*fmask.shape[::-1])
    ubox = _to_box(u, flow, B, origin, fmask.shape)
    cells = workloads.block_cells(flow, B)[sample]
    ref = oracle.velocity_refresh_at(ubox, fmask, vmask, origin, gl, cells)
    return B, flow, vort, u, sample, ref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_refresh_plate_wake_full_size(ctx, plate_refresh, dtype):
    """The 1272-block plate-and-wake set with the vorticity kept on the blocks
    whose lower neighbours are flow blocks (the benchmark's configuration),
    on a seeded sample of cells: next to the plate, in blocks outside the
    vorticity set, and random."""
    B, flow, vort, u, sample, ref = plate_refresh
    assert len(flow) == 1272
    got = _gpu(ctx, u, flow, vort, B, dtype)
    for c in range(3):
        assert _rel(got[c].reshape(-1)[sample], ref[:, c]) < TOL[dtype], c
