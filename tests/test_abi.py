"""CPU checks of the C ABI: the shared library loads without a GPU and exports
every function that include/lgfib.h declares; the Python binding carries the
same names; host-side argument checks fail before anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1604_01814_amd as lg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lgfib.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("lgf", "ib_"))))


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ["lgfib_create", "lgfib_destroy", "lgfib_last_error", "lgf_table_build", "lgf_table_copy",
              "lgf_if_weights", "lgf_poisson_apply", "lgf_if_apply"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = lg.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_same_names():
    for n in _declared():
        if n.startswith("lgfib_"):
            continue
        assert hasattr(lg, n), n


def test_null_context_rejected_without_gpu():
    lib = lg.load_library()
    ext = (ctypes.c_int32 * 3)(1, 1, 1)
    out = ctypes.c_int32()
    rc = lib.lgf_table_build(None, 0, 0.0, ext, None, ctypes.byref(out))
    assert rc == lg.LGFIB_EINVAL
    assert b"null" in lib.lgfib_last_error()


def test_multilevel_entry_points_reject_bad_arguments_without_gpu():
    lib = lg.load_library()
    ext = (ctypes.c_int32 * 3)(1, 1, 1)
    out = ctypes.c_int32()
    vals = np.zeros(8)
    assert lib.lgf_table_upload(None, ext, vals.ctypes.data_as(ctypes.c_void_p), 8, ctypes.byref(out)) == lg.LGFIB_EINVAL
    h = ctypes.c_void_p()
    blk = np.zeros((1, 3), np.int32)
    rc = lib.lgf_ml_create(None, 0, 8, 4, lg.LGF_F64, blk.ctypes.data_as(ctypes.c_void_p), 1,
                           blk.ctypes.data_as(ctypes.c_void_p), 1, None, ctypes.byref(h))
    assert rc == lg.LGFIB_EINVAL and not h.value
    assert lib.lgf_ml_apply(None, None, 1, 1.0, None, None, None) == lg.LGFIB_EINVAL
    assert lib.lgf_ml_info(None, None) == lg.LGFIB_EINVAL
    lib.lgf_ml_destroy(None)


def test_dense_solve_entry_points_reject_bad_arguments_without_gpu():
    lib = lg.load_library()
    assert lib.ib_chol_factor(None, 4, None, 4, None, 4, None) == lg.LGFIB_EINVAL
    assert lib.ib_chol_solve(None, 4, None, 4, None, None, None) == lg.LGFIB_EINVAL
    assert lib.ib_system_factor(None, None, 1, None) == lg.LGFIB_EINVAL
    assert lib.ib_schur_dense(None, None, None, 0, None) == lg.LGFIB_EINVAL


def test_herk_and_smoothing_entry_points_reject_bad_arguments_without_gpu():
    lib = lg.load_library()
    s = ctypes.c_int()
    at = (ctypes.c_double * 16)()
    ct = (ctypes.c_double * 4)()
    assert lib.ib_herk_tableau(7, ctypes.byref(s), at, ct) == lg.LGFIB_EINVAL
    assert lib.ib_herk_tableau(0, ctypes.byref(s), at, ct) == 0 and s.value == 3
    assert lib.ib_herk_tableau(3, ctypes.byref(s), at, ct) == 0 and s.value == 4
    out = ctypes.c_void_p()
    assert lib.ib_herk_create(None, 0, None, 0, 8, None, 0, None, 0, 0.05, 3, at, ct, 0, ctypes.byref(out)) \
        == lg.LGFIB_EINVAL
    assert lib.ib_herk_step(None, None, None, None, None, 1e-8, 10, 0, None, None) == lg.LGFIB_EINVAL
    assert lib.ib_force_smooth(None, None, None, None, None) == lg.LGFIB_EINVAL
    assert lib.lgf_poisson_apply_batched(None, 0, 8, 0, None, 1.0, None) != 0
    assert lib.lgf_velocity_refresh(None, 0, 8, None, 0, None, 0, 0, None, None) == lg.LGFIB_EINVAL
    assert lib.lgf_lamb_vector(None, 8, None, 1, None, 0, None, None, None) == lg.LGFIB_EINVAL
    assert lib.ib_herk_convection(None, None, 0.1, None) == lg.LGFIB_EINVAL
    assert lib.lgf_block_support(None, 8, None, 1, None, 0, None, None, None, None) == lg.LGFIB_EINVAL


def test_adapt_flow_host_update_matches_the_oracle():
    """The host set update (no GPU) against the oracle on seeded supports."""
    import numpy as np
    import oracle
    g = np.random.Generator(np.random.PCG64(4))
    xflow = np.array([(x, y, z) for z in range(-2, 4) for y in range(-1, 5) for x in range(0, 7)], dtype=np.int32)
    mu = g.exponential(1.0, len(xflow)) ** 3
    nu = g.exponential(1.0, len(xflow)) ** 3
    X = g.uniform(8, 40, (30, 3))
    for eta, eps, nbuf in ((1.0, 0.05, 1), (2.0, 0.01, 2), (1.5, 0.2, 0)):
        w = lg.ib_block_weights(X, 8, xflow, eta, 16.0)
        assert np.allclose(w, oracle.block_weights(xflow, 8, X, eta, 16.0), rtol=1e-14, atol=0)
        body = xflow[[3, 40]]
        f, xf = lg.ib_adapt_flow(xflow, mu, nu, w, eps, body, nbuf)
        fo, xfo = oracle.adapt_flow(xflow, mu, nu, w, eps, body, nbuf)
        assert np.array_equal(f, fo) and np.array_equal(xf, xfo)
    f, xf = lg.ib_adapt_flow(xflow, np.zeros(len(xflow)), np.zeros(len(xflow)), np.ones(len(xflow)), 0.1,
                             xflow[:1], 1)
    assert f.tolist() == xflow[:1].tolist() and len(xf) == 27


def test_herk_tableaus_from_the_library_match_the_oracle():
    import numpy as np
    import oracle
    for name in "ABCD":
        at, ct = lg.ib_herk_tableau(name)
        at_o, ct_o = oracle.herk_tableau(name)
        assert np.allclose(at, at_o, rtol=0, atol=1e-15) and np.allclose(ct, ct_o, rtol=0, atol=1e-15)


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No fallback: with the shared library absent every entry point raises."""
    import numpy as np
    monkeypatch.setattr(lg, "_lib", None)
    monkeypatch.setattr(lg, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "liblgfib.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        lg.load_library()
    with pytest.raises(RuntimeError, match="no fallback"):
        lg.ib_block_weights(np.zeros((1, 3)), 8, np.zeros((1, 3), np.int32), 1.0, 1.0)


def test_body_blocks_from_the_library_match_the_hand_worked_set():
    """ib_body_blocks runs on the host: the two-marker set worked by hand
    (Sec. 4.1, B = 4) and the oracle's set for a small sphere, with no GPU."""
    import numpy as np
    import oracle
    import workloads
    from test_oracle_ib import BODY_BLOCKS_B4, BODY_MARKERS
    got = sorted(map(tuple, lg.ib_body_blocks(lg.IB_ROMA3, BODY_MARKERS, 4).tolist()))
    assert got == sorted(BODY_BLOCKS_B4)
    X = workloads.sphere_markers(diameter=6.0, n=60, center=(12.37, 12.21, 12.13))
    for kernel in (lg.IB_ROMA3, lg.IB_SMOOTH3):
        for B in (4, 8):
            assert np.array_equal(lg.ib_body_blocks(kernel, X, B), oracle.body_blocks(X, kernel, B))
