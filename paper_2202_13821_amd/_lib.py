"""ctypes binding of libdg_hgks.so (include/dg_hgks.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Importing this module never builds anything; if the
library is missing, :func:`load` raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdg_hgks.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "dg_hgks.h")

DG_HGKS_OK = 0
DG_HGKS_EINVAL = -1
DG_HGKS_ENOMEM = -2
DG_HGKS_EHIP = -3
DG_HGKS_ENONPHYS = -4
DG_HGKS_EUNSUPPORTED = -5
DG_HGKS_FP64 = 0
DG_HGKS_FP32_BULK = 1


class dg_hgks_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("degree", ctypes.c_int32), ("nq", ctypes.c_int32),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("cell_widths", ctypes.c_void_p),
    ]


class DGHGKSError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"dg_hgks error {status}: {message}")
        self.status = status


_lib = None

_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double

SIGNATURES = {
    "dg_hgks_nmodes": (_i64, [_i32]),
    "dg_hgks_workspace_bytes": (ctypes.c_size_t, [_P(dg_hgks_params), _i32]),
    "dg_hgks_init": (ctypes.c_int, [_P(dg_hgks_params), _vp, _vp, ctypes.c_size_t, _P(_vp)]),
    "dg_hgks_step": (ctypes.c_int, [_vp, _vp, _d, _i32, _vp, _i32]),
    "dg_hgks_step_noalloc": (ctypes.c_int, [_P(dg_hgks_params), _vp, _vp, _d, _i32, _vp]),
    "dg_hgks_residual": (ctypes.c_int, [_vp, _vp, _d, _vp, _vp]),
    "dg_hgks_adjoint": (ctypes.c_int, [_vp, _vp, _i32, _d, _i32, _vp, _vp, _P(_d)]),
    "dg_hgks_set_mu": (ctypes.c_int, [_vp, _d]),
    "dg_hgks_set_stream": (ctypes.c_int, [_vp, _vp]),
    "dg_hgks_check": (ctypes.c_int, [_vp]),
    "dg_hgks_point_face_flux": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp]),
    "dg_hgks_point_volume_flux": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "dg_hgks_diagnostics": (ctypes.c_int, [_vp, _vp, _P(_d), _vp]),
    "dg_hgks_set_timing": (ctypes.c_int, [_vp, _i32]),
    "dg_hgks_get_timing": (ctypes.c_int, [_vp, _P(_d), _P(_i64), _i32]),
    "dg_hgks_last_error": (ctypes.c_char_p, [_vp]),
    "dg_hgks_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dg_hgks_destroy": (ctypes.c_int, [_vp]),
}


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2202_13821_amd.build` "
                "(hipcc, gfx950). There is no fallback path.")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, ctx=None):
    if status != DG_HGKS_OK:
        lib = load()
        msg = lib.dg_hgks_last_error(ctx)
        raise DGHGKSError(status, (msg or b"").decode() or lib.dg_hgks_strerror(status).decode())
    return status


def make_params(shape, lo, hi, degree, nq=0, gamma=1.4, mu=0.0, prandtl=1.0, precision=DG_HGKS_FP64,
                widths=None):
    """widths: None, or a contiguous float64 numpy array of nx + ny + nz cell
    widths that the caller keeps alive until dg_hgks_init has returned."""
    p = dg_hgks_params()
    p.struct_size = ctypes.sizeof(dg_hgks_params)
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    for e in range(3):
        p.lo[e] = float(lo[e])
        p.hi[e] = float(hi[e])
    p.degree = int(degree)
    p.nq = int(nq)
    p.gamma = float(gamma)
    p.mu = float(mu)
    p.prandtl = float(prandtl)
    p.precision = int(precision)
    p.cell_widths = None if widths is None else widths.ctypes.data
    return p
