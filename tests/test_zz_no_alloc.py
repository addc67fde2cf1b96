"""The allocation-free variant of the block-pair apply (lgf_pair_apply_noalloc)
against lgf_pair_apply, through the C ABI: two calls in a row, the second on a
smaller set (the static scratch keeps the first call's contents), both
transform variants; and its size limit."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu
B = 8


def _case(g, nb_side, ncomp):
    allb = np.array(list(np.ndindex(nb_side, nb_side, nb_side)), dtype=np.int32)[:, ::-1]
    src = allb[np.sort(g.choice(len(allb), max(1, (2 * len(allb)) // 3), replace=False))]
    tgt = allb[np.sort(g.choice(len(allb), max(1, len(allb) // 2), replace=False))]
    f = torch.from_numpy(g.standard_normal((ncomp, len(src), B, B, B)).astype(np.float32)).cuda()
    return np.ascontiguousarray(src), np.ascontiguousarray(tgt), f


@pytest.mark.parametrize("dft", [lg.LGF_DFT_FFT32, lg.LGF_DFT_BF16X3])
def test_noalloc_pair_apply_matches_pair_apply(dft):
    ctx = lg.Context(0)
    try:
        tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (47, 47, 47))
        g = np.random.Generator(np.random.PCG64(91 + dft))
        for nb_side, ncomp in ((6, 3), (3, 1)):   # the second call is smaller
            src, tgt, f = _case(g, nb_side, ncomp)
            want = torch.zeros((ncomp, len(tgt), B, B, B), dtype=torch.float32, device="cuda")
            got = torch.full_like(want, float("nan"))
            lg.lgf_pair_apply(ctx, tbl, B, src, tgt, f, want, dft=dft, dx=0.5)
            lg.lgf_pair_apply_noalloc(ctx, tbl, B, src, tgt, f, got, dft=dft, dx=0.5)
            torch.cuda.synchronize()
            w, h = want.cpu().numpy().astype(np.float64), got.cpu().numpy().astype(np.float64)
            assert np.all(np.isfinite(h))
            err = float(np.max(np.abs(h - w)) / np.max(np.abs(w)))
            print("blocks %d -> %d, ncomp %d: rel diff %.3e, bitwise %s" % (len(src), len(tgt), ncomp, err,
                                                                        np.array_equal(h, w)))
            assert err <= 1e-5
    finally:
        ctx.close()


def test_noalloc_pair_apply_rejects_sets_beyond_the_scratch():
    ctx = lg.Context(0)
    try:
        tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (127, 127, 127))
        allb = np.ascontiguousarray(np.array(list(np.ndindex(16, 16, 16)), dtype=np.int32)[:, ::-1])
        f = torch.zeros((1, len(allb), B, B, B), dtype=torch.float32, device="cuda")
        u = torch.zeros_like(f)
        with pytest.raises(lg.LgfibError) as e:
            lg.lgf_pair_apply_noalloc(ctx, tbl, B, allb, allb, f, u)
        assert e.value.code == lg.LGFIB_ERANGE and "scratch" in str(e.value)
        # an empty source set writes zeros with no scratch at all
        one = np.array([[0, 0, 0]], dtype=np.int32)
        u1 = torch.ones((1, 1, B, B, B), dtype=torch.float32, device="cuda")
        lg.lgf_pair_apply_noalloc(ctx, tbl, B, np.zeros((0, 3), np.int32), one,
                                  torch.zeros((1, 0, B, B, B), dtype=torch.float32, device="cuda"), u1)
        torch.cuda.synchronize()
        assert float(u1.abs().max()) == 0.0
    finally:
        ctx.close()
