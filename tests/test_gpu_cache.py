"""The context's plan caches stay bounded when the geometry changes every
call (a moving body rebuilds I and R each step, Sec. 2.1; an adapting flow
domain changes the block set, Sec. 4.1), evicted plans are rebuilt exactly,
and objects that hold a plan (an IB system and its captured CG iterations)
keep working while other work cycles the caches."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.ib import ROMA3

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu


def _relerr(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def _box_to_blocks(box, origin, blocks, B):
    out = np.zeros((box.shape[0], len(blocks), B, B, B))
    for i, b in enumerate(blocks):
        o = np.asarray(b) * B - np.asarray(origin)
        out[:, i] = box[:, o[2]:o[2] + B, o[1]:o[1] + B, o[0]:o[0] + B]
    return out


def test_moving_markers_keep_the_ib_cache_bounded():
    """1000 regularizations, each with the sphere moved a little: at most 64
    IB plans stay cached, and the last result equals the oracle's."""
    ctx = lg.Context(0)
    try:
        B = 8
        X0 = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
        # one block set that holds the support of every shifted sphere
        hull = np.concatenate([X0, X0 + 1000 * np.array([0.0031, -0.0017, 0.0023])])
        blocks = oracle.body_blocks(hull, ROMA3, B)
        x = np.random.Generator(np.random.PCG64(11)).standard_normal((60, 3))
        xd = torch.from_numpy(x).cuda()
        faces = torch.zeros((3, len(blocks), B, B, B), dtype=torch.float64, device="cuda")
        peak = 0
        for k in range(1000):
            X = X0 + k * np.array([0.0031, -0.0017, 0.0023])
            lg.ib_regularize(ctx, lg.IB_ROMA3, X, B, blocks, xd, faces)
            if k % 50 == 0:
                peak = max(peak, lg.lgfib_cache_info(ctx)["ib_plans"])
        info = lg.lgfib_cache_info(ctx)
        assert max(peak, info["ib_plans"]) <= 64 and info["trims"] > 0
        origin, mask = oracle.block_mask(blocks, B)
        ref = _box_to_blocks(oracle.regularize(X, x, ROMA3, origin, mask.shape), origin, blocks, B)
        assert _relerr(faces.cpu().numpy(), ref) < 1e-13
        # a position used long ago (its plan evicted) is rebuilt exactly
        lg.ib_regularize(ctx, lg.IB_ROMA3, X0, B, blocks, xd, faces)
        ref0 = _box_to_blocks(oracle.regularize(X0, x, ROMA3, origin, mask.shape), origin, blocks, B)
        assert _relerr(faces.cpu().numpy(), ref0) < 1e-13
        lg.lgfib_cache_release(ctx)
        assert lg.lgfib_cache_info(ctx)["ib_plans"] == 0
    finally:
        ctx.close()


def test_changing_block_sets_keep_box_and_if_caches_bounded():
    """300 distinct block sets through the Poisson and E(a) applies: at most
    256 box plans, 256 IF plans and 64 spectra stay cached; results against
    the oracle's direct sums on the last set."""
    ctx = lg.Context(0)
    try:
        B = 4
        g = np.random.Generator(np.random.PCG64(12))
        allb = np.array(list(np.ndindex(4, 4, 4)), dtype=np.int32)
        tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (4 * B - 1,) * 3)
        peak = {}
        for k in range(300):
            nb = int(g.integers(3, 12))
            blocks = np.ascontiguousarray(allb[np.sort(g.choice(len(allb), nb, replace=False))])
            f = g.standard_normal((1, nb, B, B, B))
            fd = torch.from_numpy(f).cuda()
            ud = torch.zeros_like(fd)
            lg.lgf_poisson_apply(ctx, tbl, B, blocks, blocks, fd, ud)
            ed = torch.zeros_like(fd)
            lg.lgf_if_apply(ctx, 0.05, B, blocks, blocks, fd, ed)
            info = lg.lgfib_cache_info(ctx)
            for key in ("box_plans", "if_plans", "box_spectra"):
                peak[key] = max(peak.get(key, 0), info[key])
        assert peak["box_plans"] <= 256 and peak["if_plans"] <= 256 and peak["box_spectra"] <= 64
        assert lg.lgfib_cache_info(ctx)["trims"] > 0
        cells = workloads.block_cells(blocks, B)
        ref = oracle.conv_direct(oracle.lgf_table(4 * B - 1, 4 * B - 1, 4 * B - 1), cells, f.reshape(-1), cells)
        assert _relerr(ud.cpu().numpy().reshape(-1), ref) < 1e-12
        lo, box, _ = workloads.dense_box(blocks, B, f[0])
        eref = oracle.conv_window(oracle.if_kernel_table(0.05), box, lo, cells)
        assert _relerr(ed.cpu().numpy().reshape(-1), eref) < 1e-12
    finally:
        ctx.close()


def test_ib_system_survives_cache_cycling():
    """An IB system pins its operator plan; the convolution plans its captured
    CG iterations use may be evicted by other work, and the iterations are
    then captured again: the second solve equals the first bit for bit."""
    ctx = lg.Context(0)
    try:
        B = 8
        X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
        blocks = oracle.body_blocks(X, ROMA3, B)
        sys_ = lg.ib_system_create(ctx, lg.IB_ROMA3, X, B, blocks, 0.05)
        b = torch.from_numpy(np.random.Generator(np.random.PCG64(13)).standard_normal((60, 3))).cuda()
        f1 = torch.zeros_like(b)
        s1 = lg.ib_force_solve(ctx, sys_, b, f1, rtol=1e-8)
        # cycle every cache with other geometry
        g = np.random.Generator(np.random.PCG64(14))
        allb = np.array(list(np.ndindex(4, 4, 4)), dtype=np.int32)
        tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (15, 15, 15))
        for k in range(80):
            nb = int(g.integers(2, 9))
            bl = np.ascontiguousarray(allb[np.sort(g.choice(len(allb), nb, replace=False))])
            fd = torch.from_numpy(g.standard_normal((1, nb, 4, 4, 4))).cuda()
            ud = torch.zeros_like(fd)
            lg.lgf_poisson_apply(ctx, tbl, 4, bl, bl, fd, ud)
            lg.lgf_if_apply(ctx, 0.05, 4, bl, bl, fd, ud)
            Xk = X + 0.01 * (k + 1)
            lg.ib_regularize(ctx, lg.IB_ROMA3, Xk, B, oracle.body_blocks(Xk, ROMA3, B),
                             torch.zeros((60, 3), dtype=torch.float64, device="cuda"),
                             torch.zeros((3, len(oracle.body_blocks(Xk, ROMA3, B)), B, B, B), dtype=torch.float64,
                                         device="cuda"))
        assert lg.lgfib_cache_info(ctx)["trims"] > 0
        f2 = torch.zeros_like(b)
        s2 = lg.ib_force_solve(ctx, sys_, b, f2, rtol=1e-8)
        assert s2["iterations"] == s1["iterations"]
        assert torch.equal(f1, f2)
        lg.lgfib_cache_release(ctx)
        assert lg.lgfib_cache_info(ctx)["ib_plans"] == 1   # the system's own, still held
        f3 = torch.zeros_like(b)
        lg.ib_force_solve(ctx, sys_, b, f3, rtol=1e-8)
        assert torch.equal(f1, f3)
        sys_.close()
    finally:
        ctx.close()
