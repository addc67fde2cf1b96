"""MI355X (gfx950) lattice-Green's-function hot path of the immersed-boundary
LGF method (Liska & Colonius, arXiv:1604.01814).

Thin ctypes binding over the C ABI declared in ``include/lgfib.h``: every
function here only marshals arguments (torch device tensors -> raw pointers,
numpy block lists -> host int32 arrays, the current HIP stream) and forwards
to the native library of the same name.  All arithmetic runs in the HIP
kernels of ``liblgfib.so``; there is no fallback path.  If the library has
not been built, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgfib.so")

LGFIB_OK, LGFIB_EINVAL, LGFIB_EDUP_BLOCK, LGFIB_ENOMEM, LGFIB_ENOTBUILT = 0, -1, -2, -3, -4
LGFIB_ENOCONV, LGFIB_EHIP, LGFIB_ESUPPORT, LGFIB_ERANGE, LGFIB_ENOTSPD = -5, -6, -7, -8, -9
LGF_KIND_L, LGF_KIND_K, LGF_KIND_USER = 0, 1, 2
LGF_F32, LGF_F64 = 0, 1
IF_CUTOFF_F64, IF_CUTOFF_F32 = 1e-14, 2.0 ** -28   # LGF_IF_CUTOFF_F64 / _F32 of the header
IB_SOLVE_DIRECT = 2
LGF_BATCH_AUTOTUNE, LGF_BATCH_PASSES = 1, 2
IB_ROMA3, IB_SMOOTH3 = 0, 1

_ERRNAMES = {0: "OK", -1: "EINVAL", -2: "EDUP_BLOCK", -3: "ENOMEM", -4: "ENOTBUILT", -5: "ENOCONV",
             -6: "EHIP", -7: "ESUPPORT", -8: "ERANGE", -9: "ENOTSPD"}


class LgfibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


class LgfInstance(ctypes.Structure):
    _fields_ = [("nblk", ctypes.c_int), ("blocks", ctypes.c_void_p), ("f", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class IbSolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("fallback", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("ms", ctypes.c_double), ("graphs", ctypes.c_int)]


def load_library():
    """Load liblgfib.so (built by ``paper_1604_01814_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblgfib.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1604_01814_amd.build); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    p, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    pi = ctypes.POINTER(ctypes.c_int)
    sig = {
        "lgfib_create": (i, [ctypes.POINTER(p), i]),
        "lgfib_destroy": (None, [p]),
        "lgfib_last_error": (ctypes.c_char_p, []),
        "lgf_table_build": (i, [p, i, d, p, p, ctypes.POINTER(ctypes.c_int32)]),
        "lgf_table_copy": (i, [p, ctypes.c_int32, p, i64]),
        "lgf_table_upload": (i, [p, p, p, i64, ctypes.POINTER(ctypes.c_int32)]),
        "lgf_ml_create": (i, [p, ctypes.c_int32, i, i, i, p, i, p, i, p, ctypes.POINTER(p)]),
        "lgf_ml_apply": (i, [p, p, i, d, p, p, p]),
        "lgf_ml_info": (i, [p, p]),
        "lgf_ml_destroy": (None, [p]),
        "lgf_if_weights": (i, [p, d, d, p, i, pi]),
        "lgf_poisson_apply": (i, [p, ctypes.c_int32, i, p, i, p, i, i, i, d, p, p, i, p]),
        "lgf_if_apply": (i, [p, d, i, p, i, p, i, i, i, p, p, p]),
        "lgfib_profile_enable": (i, [p, i]),
        "lgfib_profile_reset": (i, [p]),
        "lgfib_profile_read": (i, [p, i, p, p, p, pi]),
        "lgfib_cache_release": (i, [p]),
        "lgfib_cache_info": (i, [p, p]),
        "ib_body_blocks": (i, [i, p, i, i, p, i, pi]),
        "ib_regularize": (i, [p, i, p, i, i, p, i, i, d, p, p, p]),
        "ib_interpolate": (i, [p, i, p, i, i, p, i, i, d, p, p, p]),
        "ib_system_create": (i, [p, i, p, i, i, p, i, d, ctypes.POINTER(p)]),
        "ib_system_destroy": (None, [p]),
        "ib_schur_apply": (i, [p, p, i, p, p, p]),
        "ib_force_solve": (i, [p, p, i, p, p, p, d, i, ctypes.POINTER(IbSolveStats), p]),
        "ib_flow_create": (i, [p, p, p, i, ctypes.POINTER(p)]),
        "ib_flow_destroy": (None, [p]),
        "ib_flow_step": (i, [p, p, p, p, p, p, d, i, i, ctypes.POINTER(IbSolveStats), p, p]),
        "lgf_pair_apply": (i, [p, i, i, p, i, p, i, i, i, d, p, p, p]),
        "lgf_pair_apply_noalloc": (i, [p, i, i, p, i, p, i, i, i, d, p, p, p]),
        "lgf_batch_create": (i, [p, i, i, i, p, d, i, i, ctypes.POINTER(p)]),
        "lgf_batch_run": (i, [p, p, i, p]),
        "lgf_batch_info": (i, [p, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                               ctypes.POINTER(d), ctypes.POINTER(i)]),
        "lgf_batch_destroy": (None, [p]),
        "lgf_poisson_apply_batched": (i, [p, i, i, i, p, d, p]),
        "lgf_velocity_refresh": (i, [p, ctypes.c_int32, i, p, i, p, i, i, p, p]),
        "lgf_lamb_vector": (i, [p, i, p, i, p, i, p, p, p]),
        "lgf_block_support": (i, [p, i, p, i, p, i, p, p, p, p]),
        "ib_block_weights": (i, [p, i, i, p, i, d, d, p]),
        "ib_adapt_flow": (i, [p, i, p, p, p, d, p, i, i, p, i, pi, p, i, pi]),
        "ib_adapt_flow_dev": (i, [p, p, i, i, p, i, p, p, d, d, d, p, i, i, p, i, pi, p, i, pi, p]),
        "ib_herk_convection": (i, [p, p, d, p]),
        "ib_herk_tableau": (i, [i, ctypes.POINTER(i), p, p]),
        "ib_herk_create": (i, [p, i, p, i, i, p, i, p, i, d, i, p, p, i, ctypes.POINTER(p)]),
        "ib_herk_step": (i, [p, p, p, p, p, d, i, i, ctypes.POINTER(IbSolveStats), p]),
        "ib_herk_destroy": (None, [p]),
        "ib_force_smooth": (i, [p, p, p, p, p]),
        "ib_schur_dense": (i, [p, p, p, i, p]),
        "ib_chol_factor": (i, [p, i, p, i, p, i, p]),
        "ib_chol_solve": (i, [p, i, p, i, p, p, p]),
        "ib_system_factor": (i, [p, p, i, p]),
        "ib_mlp_create": (i, [p, i, i, i, p, p, p, p, p, ctypes.POINTER(p)]),
        "ib_mlp_destroy": (None, [p]),
        "ib_mlp_get_params": (i, [p, p, i64]),
        "ib_mlp_forward": (i, [p, p, p, i, p, p]),
        "ib_mlp_grad": (i, [p, p, p, p, i, p, ctypes.POINTER(d)]),
        "ib_mlp_train_step": (i, [p, p, p, p, i, ctypes.c_float, p]),
        "ib_mlp_last_loss": (i, [p, i, ctypes.POINTER(d)]),
        "ib_mlp_train": (i, [p, p, p, p, i, i, i, ctypes.c_float, ctypes.c_uint64, ctypes.POINTER(d)]),
        "ib_mlp_features": (i, [p, p, p, p, p, i, p, p]),
        "ib_mlp_warmstart": (i, [p, p, p, p, p, i, p, p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load_library().lgfib_last_error()
        raise LgfibError(rc, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _blocks(b):
    a = np.ascontiguousarray(np.asarray(b, dtype=np.int32).reshape(-1, 3))
    return a, a.shape[0]


def _field(t, name, prec_expected=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA/HIP torch tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dtype == torch.float32:
        prec = LGF_F32
    elif t.dtype == torch.float64:
        prec = LGF_F64
    else:
        raise TypeError("%s must be float32 or float64" % name)
    if prec_expected is not None and prec != prec_expected:
        raise TypeError("%s dtype differs from the other field" % name)
    return prec


class Context:
    """Owns an ``lgfib_ctx`` (tables, spectra, plans, workspaces) on one device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.lgfib_create(ctypes.byref(h), int(device)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load_library().lgfib_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def lgf_table_build(ctx: Context, kind: int, alpha: float, extent, stream=None) -> int:
    ext = (ctypes.c_int32 * 3)(*[int(e) for e in extent])
    out = ctypes.c_int32()
    _check(load_library().lgf_table_build(ctx.handle, int(kind), float(alpha), ext, _stream(stream),
                                          ctypes.byref(out)))
    return out.value


def lgf_table_copy(ctx: Context, tbl: int, extent) -> np.ndarray:
    e = [int(v) for v in extent]
    out = np.empty((e[2] + 1, e[1] + 1, e[0] + 1), dtype=np.float64)
    _check(load_library().lgf_table_copy(ctx.handle, int(tbl), out.ctypes.data_as(ctypes.c_void_p), out.size))
    return out


def lgf_table_upload(ctx: Context, table: np.ndarray) -> int:
    """Register an even kernel given as a host array [n3 + 1][n2 + 1][n1 + 1]
    (values at |offset|); returns the table handle."""
    t = np.ascontiguousarray(table, dtype=np.float64)
    if t.ndim != 3:
        raise ValueError("the table must be a 3-D array [n3][n2][n1]")
    ext = (ctypes.c_int32 * 3)(t.shape[2] - 1, t.shape[1] - 1, t.shape[0] - 1)
    out = ctypes.c_int32()
    _check(load_library().lgf_table_upload(ctx.handle, ext, t.ctypes.data_as(ctypes.c_void_p), t.size,
                                           ctypes.byref(out)))
    return out.value


def lgf_if_weights(ctx: Context, a: float, cutoff: float = 1e-14):
    r = ctypes.c_int()
    w = np.zeros(4097, dtype=np.float64)
    _check(load_library().lgf_if_weights(ctx.handle, float(a), float(cutoff), w.ctypes.data_as(ctypes.c_void_p),
                                         w.size, ctypes.byref(r)))
    return r.value, w[: r.value + 1].copy()


def lgf_poisson_apply(ctx: Context, tbl: int, B: int, src_blocks, tgt_blocks, f, u, dx: float = 1.0,
                      accumulate: bool = False, stream=None):
    """u = dx^2 G * f on the target blocks; f [ncomp, nsrc, B, B, B], u [ncomp, ntgt, B, B, B]."""
    sb, ns = _blocks(src_blocks)
    tb, nt = _blocks(tgt_blocks)
    prec = _field(f, "f")
    _field(u, "u", prec)
    ncomp = f.shape[0]
    if tuple(f.shape) != (ncomp, ns, B, B, B) or tuple(u.shape) != (ncomp, nt, B, B, B):
        raise ValueError("field shapes must be [ncomp, nblk, B, B, B]")
    _check(load_library().lgf_poisson_apply(
        ctx.handle, int(tbl), int(B), sb.ctypes.data_as(ctypes.c_void_p), ns,
        tb.ctypes.data_as(ctypes.c_void_p), nt, int(ncomp), prec, float(dx),
        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), int(bool(accumulate)), _stream(stream)))


def lgf_lamb_vector(ctx: Context, B: int, blocks, u, out, U=(0.0, 0.0, 0.0), stream=None):
    """out = (C u) x (u + U) on the faces of the blocks (rotational nonlinear
    term, lattice units); u and out [3, nblk, B, B, B], same dtype."""
    bl, n = _blocks(blocks)
    prec = _field(u, "u")
    _field(out, "out", prec)
    if tuple(u.shape) != (3, n, B, B, B) or tuple(out.shape) != (3, n, B, B, B):
        raise ValueError("u and out must be [3, nblk, B, B, B]")
    Ua = (ctypes.c_double * 3)(*[float(v) for v in U])
    _check(load_library().lgf_lamb_vector(ctx.handle, int(B), bl.ctypes.data_as(ctypes.c_void_p), n, Ua, prec,
                                          ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          _stream(stream)))


def lgf_block_support(ctx: Context, B: int, blocks, u, mu, nu, U=(0.0, 0.0, 0.0), stream=None):
    """Per-block max |C u| and max |D-bar N~| into the float64 device tensors
    mu, nu [nblk] (Sec. 4.1); u [3, nblk, B, B, B]."""
    import torch
    bl, n = _blocks(blocks)
    prec = _field(u, "u")
    if tuple(u.shape) != (3, n, B, B, B):
        raise ValueError("u must be [3, nblk, B, B, B]")
    for t, nm in ((mu, "mu"), (nu, "nu")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or t.numel() != n \
                or not t.is_contiguous():
            raise TypeError("%s must be a contiguous float64 device tensor of nblk values" % nm)
    Ua = (ctypes.c_double * 3)(*[float(v) for v in U])
    _check(load_library().lgf_block_support(ctx.handle, int(B), bl.ctypes.data_as(ctypes.c_void_p), n, Ua, prec,
                                            ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
                                            ctypes.c_void_p(nu.data_ptr()), _stream(stream)))


def ib_block_weights(X, B: int, blocks, eta: float, length: float) -> np.ndarray:
    """W(pos(B)) = 1 / max(eta, dist / length) per block (host)."""
    Xa, nl = _markers(X)
    bl, n = _blocks(blocks)
    w = np.zeros(n)
    _check(load_library().ib_block_weights(Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B),
                                           bl.ctypes.data_as(ctypes.c_void_p), n, float(eta), float(length),
                                           w.ctypes.data_as(ctypes.c_void_p)))
    return w


def ib_adapt_flow(xflow, mu, nu, weights, eps: float, body, nbuf: int):
    """New (D_flow, D_xflow) block lists from the support of the flow on D_xflow
    (host arrays; Sec. 4.1)."""
    xb, nx = _blocks(xflow)
    bb, nbd = _blocks(body)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    wt = np.ascontiguousarray(weights, dtype=np.float64)
    if mu.size != nx or nu.size != nx or wt.size != nx:
        raise ValueError("mu, nu and weights need one value per xflow block")
    lib = load_library()
    cap_f, cap_x = nx + nbd, max(1, (nx + nbd) * (2 * int(nbuf) + 1) ** 3)
    fo = np.zeros((cap_f, 3), dtype=np.int32)
    xo = np.zeros((cap_x, 3), dtype=np.int32)
    nf, nxo = ctypes.c_int(), ctypes.c_int()
    _check(lib.ib_adapt_flow(xb.ctypes.data_as(ctypes.c_void_p), nx, mu.ctypes.data_as(ctypes.c_void_p),
                             nu.ctypes.data_as(ctypes.c_void_p), wt.ctypes.data_as(ctypes.c_void_p), float(eps),
                             bb.ctypes.data_as(ctypes.c_void_p), nbd, int(nbuf), fo.ctypes.data_as(ctypes.c_void_p),
                             cap_f, ctypes.byref(nf), xo.ctypes.data_as(ctypes.c_void_p), cap_x, ctypes.byref(nxo)))
    return fo[:nf.value].copy(), xo[:nxo.value].copy()


def ib_adapt_flow_dev(ctx: Context, X, B: int, xflow, mu, nu, eta: float, length: float, eps: float, body,
                      nbuf: int, stream=None):
    """Block weights and the new (D_flow, D_xflow) lists on the device (Sec. 4.1):
    X [NL, 3] FP64 marker positions and mu, nu [nx] FP64 on the device, block
    lists on the host; the same lists as ib_block_weights + ib_adapt_flow."""
    for t, name in ((X, "X"), (mu, "mu"), (nu, "nu")):
        if _field(t, name) != LGF_F64:
            raise TypeError("%s must be float64" % name)
    if X.dim() != 2 or X.shape[1] != 3:
        raise ValueError("X must be [NL, 3]")
    xb, nx = _blocks(xflow)
    bb, nbd = _blocks(body)
    if mu.numel() != nx or nu.numel() != nx:
        raise ValueError("mu and nu need one value per xflow block")
    cap_f, cap_x = nx + nbd, max(1, (nx + nbd) * (2 * int(nbuf) + 1) ** 3)
    fo = np.zeros((cap_f, 3), dtype=np.int32)
    xo = np.zeros((cap_x, 3), dtype=np.int32)
    nf, nxo = ctypes.c_int(), ctypes.c_int()
    _check(load_library().ib_adapt_flow_dev(ctx.handle, ctypes.c_void_p(X.data_ptr()), int(X.shape[0]), int(B),
                                            xb.ctypes.data_as(ctypes.c_void_p), nx, ctypes.c_void_p(mu.data_ptr()),
                                            ctypes.c_void_p(nu.data_ptr()), float(eta), float(length), float(eps),
                                            bb.ctypes.data_as(ctypes.c_void_p), nbd, int(nbuf),
                                            fo.ctypes.data_as(ctypes.c_void_p), cap_f, ctypes.byref(nf),
                                            xo.ctypes.data_as(ctypes.c_void_p), cap_x, ctypes.byref(nxo),
                                            _stream(stream)))
    return fo[:nf.value].copy(), xo[:nxo.value].copy()


def lgf_velocity_refresh(ctx: Context, tbl: int, B: int, vort_blocks, flow_blocks, u, stream=None):
    """Velocity refresh in place: u [3, nflow, B, B, B] on the faces of the
    flow blocks becomes C^T s with s = -L^{-1} (C u) kept on the vorticity
    blocks (a subset of the flow blocks); tbl is a G_L table."""
    vb, nv = _blocks(vort_blocks)
    fb, nf = _blocks(flow_blocks)
    prec = _field(u, "u")
    if tuple(u.shape) != (3, nf, B, B, B):
        raise ValueError("u must be [3, nflow, B, B, B]")
    _check(load_library().lgf_velocity_refresh(
        ctx.handle, int(tbl), int(B), vb.ctypes.data_as(ctypes.c_void_p), nv, fb.ctypes.data_as(ctypes.c_void_p), nf,
        prec, ctypes.c_void_p(u.data_ptr()), _stream(stream)))


LGF_DFT_FFT32, LGF_DFT_BF16X3 = 0, 1


def lgf_pair_apply(ctx: Context, tbl: int, B: int, src_blocks, tgt_blocks, f, u, dft: int = LGF_DFT_FFT32,
                   dx: float = 1.0, stream=None, _entry: str = "lgf_pair_apply"):
    """Block-pair form of u = dx^2 G * f for blocks of 8^3 (FP32 fields
    [ncomp, n, 8, 8, 8]); dft selects FP32 or split-BF16 matrix-core DFTs."""
    import torch
    sb, ns = _blocks(src_blocks)
    tb, nt = _blocks(tgt_blocks)
    prec = _field(f, "f")
    _field(u, "u", prec)
    if f.dtype != torch.float32:
        raise TypeError("the block-pair form takes float32 fields")
    ncomp = f.shape[0]
    if tuple(f.shape) != (ncomp, ns, B, B, B) or tuple(u.shape) != (ncomp, nt, B, B, B):
        raise ValueError("field shapes must be [ncomp, nblk, B, B, B]")
    _check(getattr(load_library(), _entry)(
        ctx.handle, int(tbl), int(B), sb.ctypes.data_as(ctypes.c_void_p), ns, tb.ctypes.data_as(ctypes.c_void_p), nt,
        int(ncomp), int(dft), float(dx), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
        _stream(stream)))


def lgf_pair_apply_noalloc(ctx: Context, tbl: int, B: int, src_blocks, tgt_blocks, f, u, dft: int = LGF_DFT_FFT32,
                           dx: float = 1.0, stream=None):
    """lgf_pair_apply with every intermediate in the library's static device
    scratch (64 MiB per device): no device allocation in the call."""
    lgf_pair_apply(ctx, tbl, B, src_blocks, tgt_blocks, f, u, dft=dft, dx=dx, stream=stream,
                   _entry="lgf_pair_apply_noalloc")


def lgf_if_apply(ctx: Context, a: float, B: int, src_blocks, tgt_blocks, f, u, stream=None):
    """u = E(a) f on the target blocks (separable Bessel-product kernel)."""
    sb, ns = _blocks(src_blocks)
    tb, nt = _blocks(tgt_blocks)
    prec = _field(f, "f")
    _field(u, "u", prec)
    ncomp = f.shape[0]
    if tuple(f.shape) != (ncomp, ns, B, B, B) or tuple(u.shape) != (ncomp, nt, B, B, B):
        raise ValueError("field shapes must be [ncomp, nblk, B, B, B]")
    _check(load_library().lgf_if_apply(
        ctx.handle, float(a), int(B), sb.ctypes.data_as(ctypes.c_void_p), ns,
        tb.ctypes.data_as(ctypes.c_void_p), nt, int(ncomp), prec,
        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), _stream(stream)))


class LgfMultilevel:
    """Owns an ``lgf_ml`` plan: the multilevel interpolation evaluator of
    u = dx^2 G * f on FP64 fields [ncomp, nblk, B, B, B]."""

    def __init__(self, ctx: Context, tbl: int, B: int, p: int, src_blocks, tgt_blocks, stream=None,
                 pair_prec: int = LGF_F64):
        sb, ns = _blocks(src_blocks)
        tb, nt = _blocks(tgt_blocks)
        h = ctypes.c_void_p()
        _check(load_library().lgf_ml_create(ctx.handle, int(tbl), int(B), int(p), int(pair_prec),
                                            sb.ctypes.data_as(ctypes.c_void_p),
                                            ns, tb.ctypes.data_as(ctypes.c_void_p), nt, _stream(stream),
                                            ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.B, self.nsrc, self.ntgt = int(B), ns, nt

    def apply(self, f, u, dx: float = 1.0, stream=None):
        import torch
        for t, nm, n in ((f, "f", self.nsrc), (u, "u", self.ntgt)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
                raise TypeError("%s must be a contiguous float64 device tensor" % nm)
            if t.dim() != 5 or tuple(t.shape[1:]) != (n, self.B, self.B, self.B):
                raise ValueError("%s must be [ncomp, %d, B, B, B]" % (nm, n))
        if f.shape[0] != u.shape[0]:
            raise ValueError("f and u differ in ncomp")
        _check(load_library().lgf_ml_apply(self.ctx.handle, self._h, int(f.shape[0]), float(dx),
                                           ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                           _stream(stream)))

    def info(self) -> dict:
        out = (ctypes.c_int64 * 6)()
        _check(load_library().lgf_ml_info(self._h, out))
        return dict(zip(("levels", "source_clusters", "target_clusters", "m2l_pairs", "near_pairs", "matrices"),
                        [int(v) for v in out]))

    def close(self):
        if self._h is not None and self._h.value:
            load_library().lgf_ml_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lgf_ml_create(ctx, tbl, B, p, src_blocks, tgt_blocks, stream=None, pair_prec=None) -> LgfMultilevel:
    return LgfMultilevel(ctx, tbl, B, p, src_blocks, tgt_blocks, stream, LGF_F64 if pair_prec is None else pair_prec)


def lgf_ml_apply(ctx, plan: LgfMultilevel, f, u, dx: float = 1.0, stream=None):
    if plan.ctx is not ctx:
        raise ValueError("the plan belongs to another context")
    plan.apply(f, u, dx, stream)


def lgf_ml_info(plan: LgfMultilevel) -> dict:
    return plan.info()


def lgf_ml_destroy(plan: LgfMultilevel):
    plan.close()


class LgfBatch:
    """Owns an ``lgf_batch`` (many FP32 Poisson applies in one graph launch).
    Keeps references to the block lists and field tensors it was planned on."""

    def __init__(self, ctx: Context, tbl: int, B: int, instances, dx: float = 1.0, autotune: bool = True,
                 nbranch: int = 4, passes: bool = False):
        import torch
        self._keep = []
        arr = (LgfInstance * len(instances))()
        for k, (blocks, f, u) in enumerate(instances):
            bl, n = _blocks(blocks)
            for t, nm in ((f, "f"), (u, "u")):
                if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32:
                    raise TypeError("%s must be a contiguous float32 device tensor" % nm)
                if t.numel() != n * B ** 3:
                    raise ValueError("%s must hold [nblk, B, B, B] values" % nm)
            self._keep += [bl, f, u]
            arr[k] = LgfInstance(n, bl.ctypes.data_as(ctypes.c_void_p).value, f.data_ptr(), u.data_ptr())
        h = ctypes.c_void_p()
        flags = (LGF_BATCH_AUTOTUNE if autotune else 0) | (LGF_BATCH_PASSES if passes else 0)
        _check(load_library().lgf_batch_create(ctx.handle, int(tbl), int(B), len(instances), arr, float(dx),
                                               flags, int(nbranch), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.n = len(instances)

    def run(self, eager: bool = False, stream=None):
        _check(load_library().lgf_batch_run(self.ctx.handle, self._h, int(bool(eager)), _stream(stream)))

    def info(self, i: int) -> dict:
        b, tx, ty, br, ms, pa = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double(),
                                 ctypes.c_int())
        _check(load_library().lgf_batch_info(self._h, int(i), ctypes.byref(b), ctypes.byref(tx), ctypes.byref(ty),
                                             ctypes.byref(br), ctypes.byref(ms), ctypes.byref(pa)))
        return {"block": b.value, "tiles_x": tx.value, "tiles_y": ty.value, "branch": br.value, "tuned_ms": ms.value,
                "path": "pair" if pa.value == 1 else "box"}

    def close(self):
        if getattr(self, "_h", None):
            load_library().lgf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lgf_batch_create(ctx, tbl, B, instances, dx=1.0, autotune=True, nbranch=4, passes=False) -> LgfBatch:
    return LgfBatch(ctx, tbl, B, instances, dx, autotune, nbranch, passes)


def lgf_batch_run(ctx, batch: LgfBatch, eager: bool = False, stream=None):
    batch.run(eager, stream)


def lgf_batch_info(batch: LgfBatch, i: int) -> dict:
    return batch.info(i)


def lgf_batch_destroy(batch: LgfBatch):
    batch.close()


def lgf_poisson_apply_batched(ctx, tbl, B, instances, dx=1.0, stream=None):
    """One-shot batched apply (no autotuning): instances as for LgfBatch."""
    import torch
    keep = []
    arr = (LgfInstance * len(instances))()
    for k, (blocks, f, u) in enumerate(instances):
        bl, n = _blocks(blocks)
        for t, nm in ((f, "f"), (u, "u")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32:
                raise TypeError("%s must be a contiguous float32 device tensor" % nm)
            if t.numel() != n * B ** 3:
                raise ValueError("%s must hold [nblk, B, B, B] values" % nm)
        keep += [bl, f, u]
        arr[k] = LgfInstance(n, bl.ctypes.data_as(ctypes.c_void_p).value, f.data_ptr(), u.data_ptr())
    _check(load_library().lgf_poisson_apply_batched(ctx.handle, int(tbl), int(B), len(instances), arr, float(dx),
                                                    _stream(stream)))


def lgfib_profile_enable(ctx: Context, enable: bool = True):
    _check(load_library().lgfib_profile_enable(ctx.handle, int(bool(enable))))


def lgfib_profile_reset(ctx: Context):
    _check(load_library().lgfib_profile_reset(ctx.handle))


def lgfib_profile_read(ctx: Context, max_kernels: int = 64) -> dict:
    """{kernel name: (launches, total ms)} accumulated since the last reset."""
    names = ctypes.create_string_buffer(64 * max_kernels)
    counts = np.zeros(max_kernels, dtype=np.int32)
    ms = np.zeros(max_kernels, dtype=np.float64)
    n = ctypes.c_int()
    _check(load_library().lgfib_profile_read(ctx.handle, max_kernels, names, counts.ctypes.data_as(ctypes.c_void_p),
                                             ms.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    out = {}
    for i in range(min(n.value, max_kernels)):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (int(counts[i]), float(ms[i]))
    return out


def lgfib_cache_release(ctx: Context):
    """Free every cached plan and spectrum that no live object holds."""
    _check(load_library().lgfib_cache_release(ctx.handle))


def lgfib_cache_info(ctx: Context) -> dict:
    """Entry counts of the context's plan caches."""
    out = np.zeros(7, dtype=np.int64)
    _check(load_library().lgfib_cache_info(ctx.handle, out.ctypes.data_as(ctypes.c_void_p)))
    keys = ("box_plans", "if_plans", "box_spectra", "pair_spectra", "ib_plans", "curl_plans", "trims")
    return {k: int(v) for k, v in zip(keys, out)}


# ------------------------------------------------------------ immersed boundary

def _markers(X):
    a = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(-1, 3))
    return a, a.shape[0]


def _vec(t, name, n, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError("%s must be a contiguous CUDA/HIP tensor" % name)
    if t.numel() != 3 * n:
        raise ValueError("%s must hold [NL, 3] values" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


def ib_body_blocks(kernel: int, X, B: int) -> np.ndarray:
    """D_body: blocks within one cell of every delta support cell (host staging)."""
    Xa, nl = _markers(X)
    n = ctypes.c_int()
    lib = load_library()
    rc = lib.ib_body_blocks(int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B), None, 0, ctypes.byref(n))
    if rc not in (0, LGFIB_ERANGE):
        _check(rc)
    out = np.zeros((max(n.value, 1), 3), dtype=np.int32)
    _check(lib.ib_body_blocks(int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B),
                              out.ctypes.data_as(ctypes.c_void_p), out.shape[0], ctypes.byref(n)))
    return out[: n.value]


def ib_regularize(ctx: Context, kernel: int, X, B: int, blocks, x, faces, dx: float = 1.0, stream=None):
    """faces = R x on the block set; x [NL, 3], faces [3, nblk, B, B, B] (device)."""
    Xa, nl = _markers(X)
    bl, nb = _blocks(blocks)
    prec = _field(faces, "faces")
    _vec(x, "x", nl, faces.dtype)
    if tuple(faces.shape) != (3, nb, B, B, B):
        raise ValueError("faces must be [3, nblk, B, B, B]")
    _check(load_library().ib_regularize(ctx.handle, int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B),
                                        bl.ctypes.data_as(ctypes.c_void_p), nb, prec, float(dx),
                                        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(faces.data_ptr()),
                                        _stream(stream)))


def ib_interpolate(ctx: Context, kernel: int, X, B: int, blocks, faces, v, dx: float = 1.0, stream=None):
    """v = I faces; faces [3, nblk, B, B, B], v [NL, 3] (device)."""
    Xa, nl = _markers(X)
    bl, nb = _blocks(blocks)
    prec = _field(faces, "faces")
    _vec(v, "v", nl, faces.dtype)
    if tuple(faces.shape) != (3, nb, B, B, B):
        raise ValueError("faces must be [3, nblk, B, B, B]")
    _check(load_library().ib_interpolate(ctx.handle, int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B),
                                         bl.ctypes.data_as(ctypes.c_void_p), nb, prec, float(dx),
                                         ctypes.c_void_p(faces.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                         _stream(stream)))


class IbSystem:
    """Owns an ``ib_system`` (rigid-body force Schur complement)."""

    def __init__(self, ctx: Context, kernel: int, X, B: int, blocks, a: float):
        Xa, nl = _markers(X)
        bl, nb = _blocks(blocks)
        h = ctypes.c_void_p()
        _check(load_library().ib_system_create(ctx.handle, int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl,
                                               int(B), bl.ctypes.data_as(ctypes.c_void_p), nb, float(a),
                                               ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.NL = nl
        self.B = int(B)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ib_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ib_system_create(ctx: Context, kernel: int, X, B: int, blocks, a: float) -> IbSystem:
    return IbSystem(ctx, kernel, X, B, blocks, a)


def ib_schur_apply(ctx: Context, sys: IbSystem, x, y, stream=None):
    """y = C x (force Schur complement); x, y [NL, 3] float32 or float64."""
    prec = _field(x, "x")
    _field(y, "y", prec)
    _vec(x, "x", sys.NL)
    _vec(y, "y", sys.NL)
    _check(load_library().ib_schur_apply(ctx.handle, sys.handle, prec, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), _stream(stream)))


def ib_force_solve(ctx: Context, sys: IbSystem, b, f, x0=None, rtol: float = 1e-8, maxit: int = 2000,
                   prec: int = LGF_F32, stream=None, raise_on_noconv: bool = True) -> dict:
    """Solve C f = b by CG (FP64 vectors; matvec in ``prec``); returns stats."""
    import torch
    _vec(b, "b", sys.NL, torch.float64)
    _vec(f, "f", sys.NL, torch.float64)
    x0p = None if x0 is None else _vec(x0, "x0", sys.NL, torch.float64)
    st = IbSolveStats()
    rc = load_library().ib_force_solve(ctx.handle, sys.handle, int(prec), ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(f.data_ptr()), x0p, float(rtol), int(maxit),
                                       ctypes.byref(st), _stream(stream))
    if rc != 0 and (rc != LGFIB_ENOCONV or raise_on_noconv):
        _check(rc)
    return {"iterations": st.iterations, "restarts": st.restarts, "fallback": st.fallback,
            "rel_residual": st.rel_residual, "ms": st.ms, "graphs": st.graphs, "converged": rc == 0}


def ib_system_destroy(sys: IbSystem):
    sys.close()


class IbFlow:
    """Owns an ``ib_flow`` (Stokes IF-Euler driver on the flow blocks)."""

    def __init__(self, ctx: Context, sys: IbSystem, flow_blocks):
        bl, nb = _blocks(flow_blocks)
        h = ctypes.c_void_p()
        _check(load_library().ib_flow_create(ctx.handle, sys.handle, bl.ctypes.data_as(ctypes.c_void_p), nb,
                                             ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.sys = sys
        self.nflow = nb
        self.B = sys.B

    def close(self):
        if getattr(self, "_h", None):
            load_library().ib_flow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ib_flow_create(ctx: Context, sys: IbSystem, flow_blocks) -> IbFlow:
    return IbFlow(ctx, sys, flow_blocks)


def ib_flow_destroy(flow: IbFlow):
    flow.close()


def ib_flow_step(ctx: Context, flow: IbFlow, u, u_b, f, x0=None, rtol: float = 1e-8, maxit: int = 2000,
                 prec: int = LGF_F32, stream=None, raise_on_noconv: bool = True, b_out=None) -> dict:
    """One IF-Euler Stokes step: u (faces [3, nflow, B, B, B], float64) in place;
    u_b, f, x0, b_out: [NL, 3] float64 device tensors (b_out receives the
    force-solve right-hand side).  Returns the force-solve stats."""
    import torch
    if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous():
        raise TypeError("u must be a contiguous float64 device tensor")
    if u.numel() != 3 * flow.nflow * flow.B ** 3:
        raise ValueError("u must hold [3, nflow, B, B, B] values")
    nl = flow.sys.NL
    _vec(u_b, "u_b", nl, torch.float64)
    _vec(f, "f", nl, torch.float64)
    x0p = None if x0 is None else _vec(x0, "x0", nl, torch.float64)
    bp = None if b_out is None else _vec(b_out, "b_out", nl, torch.float64)
    st = IbSolveStats()
    rc = load_library().ib_flow_step(ctx.handle, flow.handle, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(u_b.data_ptr()), ctypes.c_void_p(f.data_ptr()), x0p,
                                     float(rtol), int(maxit), int(prec), ctypes.byref(st), bp, _stream(stream))
    if rc != 0 and (rc != LGFIB_ENOCONV or raise_on_noconv):
        _check(rc)
    return {"iterations": st.iterations, "restarts": st.restarts, "fallback": st.fallback,
            "rel_residual": st.rel_residual, "ms": st.ms, "graphs": st.graphs, "converged": rc == 0}


# ------------------------------------------------------------------ IF-HERK step

HERK_SCHEMES = {"A": 0, "B": 1, "C": 2, "D": 3}


def ib_herk_tableau(scheme) -> tuple:
    """(at [s, s], ct [s]) of App. B's scheme 'A'..'D' (shifted form)."""
    k = HERK_SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    s = ctypes.c_int()
    at = np.zeros(16)
    ct = np.zeros(4)
    _check(load_library().ib_herk_tableau(k, ctypes.byref(s), at.ctypes.data_as(ctypes.c_void_p),
                                          ct.ctypes.data_as(ctypes.c_void_p)))
    n = s.value
    return at[:n * n].reshape(n, n).copy(), ct[:n].copy()


class IbHerk:
    """Owns an ``ib_herk`` (s-stage IF-HERK step of the Stokes driver)."""

    def __init__(self, ctx: Context, kernel: int, X, B: int, body_blocks, flow_blocks, A: float, at, ct,
                 direct: bool = False):
        Xa, nl = _markers(X)
        bb, nbb = _blocks(body_blocks)
        fb, nfb = _blocks(flow_blocks)
        at = np.ascontiguousarray(at, dtype=np.float64)
        ct = np.ascontiguousarray(ct, dtype=np.float64)
        s = len(ct)
        if at.shape != (s, s):
            raise ValueError("at must be [s, s]")
        h = ctypes.c_void_p()
        _check(load_library().ib_herk_create(ctx.handle, int(kernel), Xa.ctypes.data_as(ctypes.c_void_p), nl, int(B),
                                             bb.ctypes.data_as(ctypes.c_void_p), nbb,
                                             fb.ctypes.data_as(ctypes.c_void_p), nfb, float(A), s,
                                             at.ctypes.data_as(ctypes.c_void_p), ct.ctypes.data_as(ctypes.c_void_p),
                                             int(bool(direct)), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.NL = nl
        self.s = s
        self.nflow = nfb
        self.B = int(B)

    def close(self):
        if getattr(self, "_h", None):
            load_library().ib_herk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ib_herk_create(ctx, kernel, X, B, body_blocks, flow_blocks, A, at, ct, direct=False) -> IbHerk:
    return IbHerk(ctx, kernel, X, B, body_blocks, flow_blocks, A, at, ct, direct)


def ib_herk_step(ctx: Context, hk: IbHerk, u, u_b, f, rtol: float = 1e-8, maxit: int = 2000, prec: int = LGF_F32,
                 stream=None, raise_on_noconv: bool = True) -> dict:
    """One IF-HERK step: u (faces, float64) in place; u_b [s, NL, 3] and f
    [NL, 3] float64 device tensors.  Returns the summed solve stats."""
    import torch
    if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous():
        raise TypeError("u must be a contiguous float64 device tensor")
    if u.numel() != 3 * hk.nflow * hk.B ** 3:
        raise ValueError("u must hold [3, nflow, B, B, B] values")
    if (u_b.dtype != torch.float64 or not u_b.is_cuda or not u_b.is_contiguous()
            or tuple(u_b.shape) != (hk.s, hk.NL, 3)):
        raise TypeError("u_b must be a contiguous float64 device tensor [s, NL, 3]")
    _vec(f, "f", hk.NL, torch.float64)
    st = IbSolveStats()
    rc = load_library().ib_herk_step(ctx.handle, hk.handle, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(u_b.data_ptr()), ctypes.c_void_p(f.data_ptr()), float(rtol),
                                     int(maxit), int(prec), ctypes.byref(st), _stream(stream))
    if rc != 0 and (rc != LGFIB_ENOCONV or raise_on_noconv):
        _check(rc)
    return {"iterations": st.iterations, "restarts": st.restarts, "fallback": st.fallback,
            "rel_residual": st.rel_residual, "ms": st.ms, "graphs": st.graphs, "converged": rc == 0}


def ib_herk_convection(ctx: Context, hk: IbHerk, dt: float, U=(0.0, 0.0, 0.0)):
    """Carry the nonlinear term (C u) x (u + U) in the following HERK steps;
    dt is the time step over the grid spacing (0 turns it off)."""
    Ua = (ctypes.c_double * 3)(*[float(v) for v in U])
    _check(load_library().ib_herk_convection(ctx.handle, hk.handle, float(dt), Ua))


def ib_herk_destroy(hk: IbHerk):
    hk.close()


def ib_force_smooth(ctx: Context, sys: IbSystem, f, fhat, stream=None):
    """fhat = I W R f (smoothed boundary force); f, fhat [NL, 3] float64."""
    import torch
    _vec(f, "f", sys.NL, torch.float64)
    _vec(fhat, "fhat", sys.NL, torch.float64)
    _check(load_library().ib_force_smooth(ctx.handle, sys.handle, ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(fhat.data_ptr()), _stream(stream)))


# ------------------------------------------------------------ dense force solve

def _matrix(a, name, n=None):
    import torch
    if a.dtype != torch.float64 or not a.is_cuda or a.dim() != 2 or a.stride(1) != 1:
        raise TypeError("%s must be a 2-D float64 device tensor with unit column stride" % name)
    if a.shape[0] != a.shape[1] and n is None:
        raise ValueError("%s must be square" % name)
    if a.shape[0] > 0 and a.stride(0) < a.shape[1]:
        raise ValueError("%s: row stride below the row length" % name)
    return max(int(a.stride(0)), 1)


def ib_schur_dense(ctx: Context, sys: IbSystem, C, stream=None):
    """C[:, :] = dense force Schur complement (3 NL x 3 NL, FP64 matvecs)."""
    ld = _matrix(C, "C")
    if C.shape[0] != 3 * sys.NL:
        raise ValueError("C must be %d x %d" % (3 * sys.NL, 3 * sys.NL))
    _check(load_library().ib_schur_dense(ctx.handle, sys.handle, ctypes.c_void_p(C.data_ptr()), ld, _stream(stream)))


def ib_chol_factor(ctx: Context, A, W, stream=None):
    """A = L L^T in place (lower triangle; the strict upper triangle becomes
    unspecified) and W = L^{-1}; A, W square float64 device tensors."""
    lda, ldw = _matrix(A, "A"), _matrix(W, "W")
    if A.shape != W.shape:
        raise ValueError("A and W must have the same shape")
    _check(load_library().ib_chol_factor(ctx.handle, int(A.shape[0]), ctypes.c_void_p(A.data_ptr()), lda,
                                         ctypes.c_void_p(W.data_ptr()), ldw, _stream(stream)))


def ib_chol_solve(ctx: Context, W, b, x, stream=None):
    """x = W^T (W b) for lower-triangular W; b, x float64 device vectors."""
    import torch
    ldw = _matrix(W, "W")
    n = int(W.shape[0])
    for v, nm in ((b, "b"), (x, "x")):
        if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous() or v.numel() != n:
            raise TypeError("%s must be a contiguous float64 device vector of %d values" % (nm, n))
    _check(load_library().ib_chol_solve(ctx.handle, n, ctypes.c_void_p(W.data_ptr()), ldw,
                                        ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        _stream(stream)))


def ib_system_factor(ctx: Context, sys: IbSystem, enable: bool = True, stream=None):
    """Build, factor and keep the system's dense C (enable) or drop it."""
    _check(load_library().ib_system_factor(ctx.handle, sys.handle, int(bool(enable)), _stream(stream)))


# ---------------------------------------------------------- learned warm start

def mlp_param_count(nin: int, nh: int, nout: int) -> int:
    return nh * nin + nh + nh * nh + nh + nout * nh + nout


class IbMlp:
    """Owns an ``ib_mlp`` (per-marker warm-start network)."""

    def __init__(self, ctx: Context, nin: int, nh: int, nout: int, params, in_shift, in_scale, out_shift,
                 out_scale):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
                for a in (params, in_shift, in_scale, out_shift, out_scale)]
        if arrs[0].size != mlp_param_count(nin, nh, nout):
            raise ValueError("params must hold %d floats" % mlp_param_count(nin, nh, nout))
        h = ctypes.c_void_p()
        _check(load_library().ib_mlp_create(ctx.handle, int(nin), int(nh), int(nout),
                                            *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs], ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.nin, self.nh, self.nout = nin, nh, nout

    def close(self):
        if getattr(self, "_h", None):
            load_library().ib_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ib_mlp_create(ctx, nin, nh, nout, params, in_shift, in_scale, out_shift, out_scale) -> IbMlp:
    return IbMlp(ctx, nin, nh, nout, params, in_shift, in_scale, out_shift, out_scale)


def ib_mlp_destroy(m: IbMlp):
    m.close()


def ib_mlp_get_params(m: IbMlp) -> np.ndarray:
    out = np.empty(mlp_param_count(m.nin, m.nh, m.nout), dtype=np.float32)
    _check(load_library().ib_mlp_get_params(m.handle, out.ctypes.data_as(ctypes.c_void_p), out.size))
    return out


def _f32(t, name, width):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32:
        raise TypeError("%s must be a contiguous float32 device tensor" % name)
    if t.numel() % width:
        raise ValueError("%s must have rows of %d" % (name, width))
    return ctypes.c_void_p(t.data_ptr()), t.numel() // width


def ib_mlp_forward(ctx: Context, m: IbMlp, x, y, stream=None):
    xp, M = _f32(x, "x", m.nin)
    yp, My = _f32(y, "y", m.nout)
    if M != My:
        raise ValueError("x and y row counts differ")
    _check(load_library().ib_mlp_forward(ctx.handle, m.handle, xp, M, yp, _stream(stream)))


def ib_mlp_grad(ctx: Context, m: IbMlp, x, t):
    xp, M = _f32(x, "x", m.nin)
    tp, Mt = _f32(t, "t", m.nout)
    if M != Mt:
        raise ValueError("x and t row counts differ")
    g = np.empty(mlp_param_count(m.nin, m.nh, m.nout), dtype=np.float32)
    loss = ctypes.c_double()
    _check(load_library().ib_mlp_grad(ctx.handle, m.handle, xp, tp, M, g.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(loss)))
    return g, loss.value


def ib_mlp_train_step(ctx: Context, m: IbMlp, x, t, lr: float, stream=None):
    xp, M = _f32(x, "x", m.nin)
    tp, _ = _f32(t, "t", m.nout)
    _check(load_library().ib_mlp_train_step(ctx.handle, m.handle, xp, tp, M, ctypes.c_float(lr), _stream(stream)))


def ib_mlp_last_loss(m: IbMlp, M: int) -> float:
    loss = ctypes.c_double()
    _check(load_library().ib_mlp_last_loss(m.handle, int(M), ctypes.byref(loss)))
    return loss.value


def ib_mlp_train(ctx: Context, m: IbMlp, x, t, epochs: int, batch: int, lr: float, seed: int) -> float:
    xp, M = _f32(x, "x", m.nin)
    tp, Mt = _f32(t, "t", m.nout)
    if M != Mt:
        raise ValueError("x and t row counts differ")
    loss = ctypes.c_double()
    _check(load_library().ib_mlp_train(ctx.handle, m.handle, xp, tp, M, int(epochs), int(batch), ctypes.c_float(lr),
                                       ctypes.c_uint64(seed), ctypes.byref(loss)))
    return loss.value


def ib_mlp_features(ctx: Context, normals, ustate, f1, f2, feats, stream=None):
    """Warm-start features; ustate = (U_{k+1}, U_k, U_{k-1}, U_{k-2})."""
    import torch
    nl = normals.shape[0]
    if len(ustate) != 4:
        raise ValueError("ustate must hold U_{k+1}, U_k, U_{k-1}, U_{k-2}")
    us = (ctypes.c_double * 4)(*[float(v) for v in ustate])
    for t, nm in ((normals, "normals"), (f1, "f1"), (f2, "f2")):
        _vec(t, nm, nl, torch.float64)
    fp, M = _f32(feats, "feats", 12)
    if M != nl:
        raise ValueError("feats must have NL rows")
    _check(load_library().ib_mlp_features(ctx.handle, ctypes.c_void_p(normals.data_ptr()), us,
                                          ctypes.c_void_p(f1.data_ptr()), ctypes.c_void_p(f2.data_ptr()), nl, fp,
                                          _stream(stream)))


def ib_mlp_warmstart(ctx: Context, m: IbMlp, feats, f1, f2, x0, stream=None):
    """x0 = 2 f1 - f2 + MLP(feats)."""
    import torch
    fp, nl = _f32(feats, "feats", 12)
    _vec(f1, "f1", nl, torch.float64)
    _vec(f2, "f2", nl, torch.float64)
    _vec(x0, "x0", nl, torch.float64)
    _check(load_library().ib_mlp_warmstart(ctx.handle, m.handle, fp, ctypes.c_void_p(f1.data_ptr()),
                                           ctypes.c_void_p(f2.data_ptr()), nl, ctypes.c_void_p(x0.data_ptr()),
                                           _stream(stream)))
