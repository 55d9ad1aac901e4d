"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/dg_hgks.h, and rejects invalid arguments before touching
the device (dg_hgks_init launches nothing and allocates nothing)."""
import ctypes
import re

import numpy as np
import pytest

from paper_2202_13821_amd import _lib

L = None


@pytest.fixture(scope="module", autouse=True)
def lib():
    global L
    L = _lib.load()
    return L


def _params(**kw):
    base = dict(shape=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1), degree=2, nq=0, gamma=1.4, mu=0.0, prandtl=1.0,
                precision=_lib.DG_HGKS_FP64)
    base.update(kw)
    return _lib.make_params(base["shape"], base["lo"], base["hi"], base["degree"], base["nq"], base["gamma"],
                            base["mu"], base["prandtl"], base["precision"], base.get("widths"))


def test_every_declared_symbol_is_exported():
    text = open(_lib.HEADER).read()
    names = set(re.findall(r"\b(dg_hgks_[a-z_]+)\s*\(", text))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n
    assert names == set(_lib.SIGNATURES), names ^ set(_lib.SIGNATURES)


def test_params_struct_size():
    assert ctypes.sizeof(_lib.dg_hgks_params) == 112


def test_nmodes():
    assert [L.dg_hgks_nmodes(k) for k in (1, 2, 3)] == [4, 10, 20]
    assert L.dg_hgks_nmodes(0) == -1 and L.dg_hgks_nmodes(4) == -1


def test_workspace_bytes():
    p = _params()
    b0 = L.dg_hgks_workspace_bytes(ctypes.byref(p), 0)
    b1 = L.dg_hgks_workspace_bytes(ctypes.byref(p), 3)
    assert b0 > 0 and b1 > b0 and b0 % 256 == 0
    # FP32-bulk keeps a float copy and float records
    pf = _params(precision=_lib.DG_HGKS_FP32_BULK)
    assert L.dg_hgks_workspace_bytes(ctypes.byref(pf), 0) > 0
    assert L.dg_hgks_workspace_bytes(ctypes.byref(_params(degree=5)), 0) == 0
    assert L.dg_hgks_workspace_bytes(ctypes.byref(p), -1) == 0


BAD = [
    dict(shape=(0, 8, 8)), dict(shape=(8, -1, 8)), dict(lo=(1, 0, 0), hi=(1, 1, 1)), dict(degree=0),
    dict(degree=4), dict(nq=5), dict(gamma=1.0), dict(gamma=float("nan")), dict(mu=-1e-3),
    dict(prandtl=0.0), dict(precision=7),
]


@pytest.mark.parametrize("kw", BAD)
def test_init_rejects_invalid_params(kw):
    p = _params(**kw)
    ctx = ctypes.c_void_p()
    rc = L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), 1 << 30, ctypes.byref(ctx))
    assert rc == _lib.DG_HGKS_EINVAL
    assert not ctx.value
    assert L.dg_hgks_last_error(None)


def test_init_unsupported_and_workspace_errors():
    ctx = ctypes.c_void_p()
    p = _params(degree=2, nq=4)
    assert L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), 1 << 30, ctypes.byref(ctx)) \
        == _lib.DG_HGKS_EUNSUPPORTED
    p = _params()
    need = L.dg_hgks_workspace_bytes(ctypes.byref(p), 0)
    assert L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), need - 256, ctypes.byref(ctx)) \
        == _lib.DG_HGKS_ENOMEM
    assert L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p((1 << 20) + 8), need, ctypes.byref(ctx)) \
        == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_init(ctypes.byref(p), None, None, need, ctypes.byref(ctx)) == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_init(None, None, ctypes.c_void_p(1 << 20), need, ctypes.byref(ctx)) == _lib.DG_HGKS_EINVAL
    bad = _params()
    bad.struct_size = 8
    assert L.dg_hgks_init(ctypes.byref(bad), None, ctypes.c_void_p(1 << 20), need, ctypes.byref(ctx)) \
        == _lib.DG_HGKS_EINVAL


def test_calls_reject_invalid_arguments_without_device_work():
    """Init only records the workspace pointer, so a dummy address is safe
    here as long as no call reaches a launch."""
    p = _params()
    need = L.dg_hgks_workspace_bytes(ctypes.byref(p), 2)
    ctx = ctypes.c_void_p()
    assert L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), need, ctypes.byref(ctx)) == 0
    q = ctypes.c_void_p(1 << 24)
    E = _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_step(ctx, None, 1e-3, 1, None, 0) == E
    assert L.dg_hgks_step(ctx, q, 0.0, 1, None, 0) == E
    assert L.dg_hgks_step(ctx, q, float("inf"), 1, None, 0) == E
    assert L.dg_hgks_step(ctx, q, 1e-3, -1, None, 0) == E
    assert L.dg_hgks_step(ctx, q, 1e-3, 1, q, 0) == E
    assert b"dt" in L.dg_hgks_last_error(ctx) or b"stride" in L.dg_hgks_last_error(ctx)
    assert L.dg_hgks_residual(ctx, q, -1.0, q, q) == E
    assert L.dg_hgks_residual(ctx, None, 1e-3, q, q) == E
    mb = ctypes.c_double()
    assert L.dg_hgks_adjoint(ctx, q, 0, 1e-3, 2, q, q, ctypes.byref(mb)) == E
    assert L.dg_hgks_adjoint(ctx, q, 3, 1e-3, 2, q, q, ctypes.byref(mb)) == _lib.DG_HGKS_ENOMEM
    assert L.dg_hgks_adjoint(ctx, None, 1, 1e-3, 2, q, q, ctypes.byref(mb)) == E
    assert L.dg_hgks_set_mu(ctx, -1.0) == E
    assert L.dg_hgks_set_mu(ctx, 0.01) == 0
    assert L.dg_hgks_point_face_flux(ctx, q, 4, 3, 1e-3, q, q) == E
    assert L.dg_hgks_point_volume_flux(ctx, None, 4, q, q) == E
    out = (ctypes.c_double * 2)()
    assert L.dg_hgks_diagnostics(ctx, None, out, None) == E
    assert L.dg_hgks_diagnostics(ctx, q, None, None) == E
    assert L.dg_hgks_destroy(ctx) == 0
    assert L.dg_hgks_destroy(None) == E


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5):
        assert L.dg_hgks_strerror(code)
    assert L.dg_hgks_strerror(123) == b"unknown status"


def test_init_validates_cell_widths():
    """Separable meshes: every width finite and > 0, each axis summing to
    hi - lo; the array is copied, so it may be freed after init."""
    shape, hi = (3, 2, 2), (1.5, 1.0, 2.0)
    good = np.array([0.4, 0.6, 0.5, 0.3, 0.7, 1.5, 0.5])
    ctx = ctypes.c_void_p()
    for w, rc in ((good, 0), (np.array([0.4, 0.6, 0.5, 0.3, 0.7, 1.4, 0.5]), _lib.DG_HGKS_EINVAL),
                  (np.array([0.4, 0.6, 0.5, -0.3, 1.3, 1.5, 0.5]), _lib.DG_HGKS_EINVAL),
                  (np.array([0.4, 0.6, 0.5, np.nan, 0.7, 1.5, 0.5]), _lib.DG_HGKS_EINVAL)):
        p = _params(shape=shape, hi=hi, widths=np.ascontiguousarray(w))
        need = L.dg_hgks_workspace_bytes(ctypes.byref(p), 0)
        assert (need > 0) == (rc == 0)
        got = L.dg_hgks_init(ctypes.byref(p), None, ctypes.c_void_p(1 << 20), 1 << 30, ctypes.byref(ctx))
        assert got == rc, (w, got)
        if rc == 0:
            assert L.dg_hgks_destroy(ctx) == 0


def test_noalloc_step_validates_before_touching_the_device():
    """dg_hgks_step_noalloc rejects bad arguments, non-uniform meshes and
    grids beyond its static scratch before any HIP call."""
    q = ctypes.c_void_p(256)  # never dereferenced: every case fails validation
    p = _params()
    assert L.dg_hgks_step_noalloc(None, None, q, 1e-3, 1, None) == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_step_noalloc(ctypes.byref(_params(degree=5)), None, q, 1e-3, 1, None) == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_step_noalloc(ctypes.byref(p), None, None, 1e-3, 1, None) == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_step_noalloc(ctypes.byref(p), None, q, 0.0, 1, None) == _lib.DG_HGKS_EINVAL
    assert L.dg_hgks_step_noalloc(ctypes.byref(p), None, q, 1e-3, -1, None) == _lib.DG_HGKS_EINVAL
    w = np.full(24, 1.0 / 8)
    pw = _params(widths=w)
    assert L.dg_hgks_step_noalloc(ctypes.byref(pw), None, q, 1e-3, 1, None) == _lib.DG_HGKS_EINVAL
    assert b"uniform" in L.dg_hgks_last_error(None)
    big = _params(shape=(64, 64, 64))
    assert L.dg_hgks_step_noalloc(ctypes.byref(big), None, q, 1e-3, 1, None) == _lib.DG_HGKS_ENOMEM
    assert b"scratch" in L.dg_hgks_last_error(None)
    # 32^3 P2 fits in both precisions
    for prec in (_lib.DG_HGKS_FP64, _lib.DG_HGKS_FP32_BULK):
        assert L.dg_hgks_workspace_bytes(ctypes.byref(_params(shape=(32, 32, 32), precision=prec)), 0) <= 96 << 20

