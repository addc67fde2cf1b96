"""GPU parity of the block-pair form of the LGF convolution (blocks of 8^3,
per-block zero-padded 16^3 spectra, pair multiply-accumulate) against the
FP64 oracle, in both transform variants: FP32 register DFTs and split-BF16
matrix-core DFTs."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_1604_01814_amd as lg  # noqa: E402

pytestmark = pytest.mark.gpu
B = 8


@pytest.fixture(scope="module")
def ctx():
    c = lg.Context(0)
    yield c
    c.close()


def _relerr(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def case():
    g = np.random.Generator(np.random.PCG64(61))
    allb = np.array(list(np.ndindex(4, 5, 4)), dtype=np.int32)[:, ::-1] + np.array([-2, 1, -1], dtype=np.int32)
    src = allb[g.choice(len(allb), 12, replace=False)]
    tgt = allb[g.choice(len(allb), 9, replace=False)]
    f = g.standard_normal((2, len(src), B, B, B))
    lo = np.minimum(src.min(0), tgt.min(0))
    hi = np.maximum(src.max(0), tgt.max(0))
    ext = tuple(int(v) for v in (hi - lo + 1) * B - 1)
    G = oracle.lgf_table(*ext)
    sc, tc = workloads.block_cells(src, B), workloads.block_cells(tgt, B)
    ref = np.stack([oracle.conv_direct(G, sc, f[c].reshape(-1), tc) for c in range(2)])
    return src, tgt, f, ext, ref.reshape(2, len(tgt), B, B, B)


@pytest.mark.parametrize("dft,tol", [(lg.LGF_DFT_FFT32, 1e-5), (lg.LGF_DFT_BF16X3, 1e-5)])
def test_pair_apply_matches_oracle(ctx, case, dft, tol):
    src, tgt, f, ext, ref = case
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    fd = torch.from_numpy(f.astype(np.float32)).cuda()
    ud = torch.zeros((2, len(tgt), B, B, B), dtype=torch.float32, device="cuda")
    lg.lgf_pair_apply(ctx, tbl, B, src, tgt, fd, ud, dft=dft)
    u = ud.cpu().numpy().astype(np.float64)
    for c in range(2):
        err = _relerr(u[c], ref[c])
        print("dft %d component %d: rel err %.3e" % (dft, c, err))
        assert err < tol


def test_pair_apply_matches_box_fft(ctx, case):
    """Both exact forms of the same sum agree to FP32 rounding."""
    src, tgt, f, ext, ref = case
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, ext)
    fd = torch.from_numpy(f.astype(np.float32)).cuda()
    ua = torch.zeros((2, len(tgt), B, B, B), dtype=torch.float32, device="cuda")
    ub = torch.zeros_like(ua)
    lg.lgf_pair_apply(ctx, tbl, B, src, tgt, fd, ua, dx=0.5)
    lg.lgf_poisson_apply(ctx, tbl, B, src, tgt, fd, ub, dx=0.5)
    assert _relerr(ua.cpu().numpy().astype(np.float64), ub.cpu().numpy().astype(np.float64)) < 2e-6


def test_pair_apply_edges(ctx):
    tbl = lg.lgf_table_build(ctx, lg.LGF_KIND_L, 0.0, (15, 15, 15))
    far = np.array([[0, 0, 0], [3, 0, 0]], dtype=np.int32)
    f = torch.zeros((1, 2, B, B, B), dtype=torch.float32, device="cuda")
    u = torch.zeros_like(f)
    with pytest.raises(lg.LgfibError) as e:
        lg.lgf_pair_apply(ctx, tbl, B, far, far, f, u)
    assert e.value.code == lg.LGFIB_ERANGE
    one = np.array([[0, 0, 0]], dtype=np.int32)
    f1 = torch.zeros((1, 1, B, B, B), dtype=torch.float32, device="cuda")
    f1[0, 0, 3, 4, 5] = 1.0
    u1 = torch.zeros_like(f1)
    lg.lgf_pair_apply(ctx, tbl, B, one, one, f1, u1)
    G = oracle.lgf_table(7, 7, 7)
    # a unit source reproduces the table: u(n) = G(n - m)
    n = np.array(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"))   # z, y, x
    want = G[np.abs(n[0] - 3), np.abs(n[1] - 4), np.abs(n[2] - 5)]
    assert _relerr(u1[0, 0].cpu().numpy().astype(np.float64), want) < 1e-6
