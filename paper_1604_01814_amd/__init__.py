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
LGFIB_ENOCONV, LGFIB_EHIP, LGFIB_ESUPPORT, LGFIB_ERANGE = -5, -6, -7, -8
LGF_KIND_L, LGF_KIND_K = 0, 1
LGF_F32, LGF_F64 = 0, 1
IB_ROMA3, IB_SMOOTH3 = 0, 1

_ERRNAMES = {0: "OK", -1: "EINVAL", -2: "EDUP_BLOCK", -3: "ENOMEM", -4: "ENOTBUILT", -5: "ENOCONV",
             -6: "EHIP", -7: "ESUPPORT", -8: "ERANGE"}


class LgfibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


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
        "lgf_if_weights": (i, [p, d, d, p, i, pi]),
        "lgf_poisson_apply": (i, [p, ctypes.c_int32, i, p, i, p, i, i, i, d, p, p, i, p]),
        "lgf_if_apply": (i, [p, d, i, p, i, p, i, i, i, p, p, p]),
        "lgfib_profile_enable": (i, [p, i]),
        "lgfib_profile_reset": (i, [p]),
        "lgfib_profile_read": (i, [p, i, p, p, p, pi]),
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
