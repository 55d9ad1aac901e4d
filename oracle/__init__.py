"""ctypes front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The product package never does.

Every array is float64 with the layout ``q[var][mode][z][y][x]`` (5 conservative
variables rho, rho U, rho V, rho W, rho E; modes in the order of
:func:`modes`).  See ``dg_oracle.cpp`` for the passages of the paper each
routine follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))


class Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("k", ctypes.c_int32), ("nq", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("widths", ctypes.c_void_p),
    ]


def make_cfg(shape, k, nq=None, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             gamma=1.4, mu=0.0, prandtl=1.0, widths=None):
    """shape = (nx, ny, nz).  widths: optional separable mesh, the nx + ny + nz
    cell widths (x, then y, then z), each axis summing to hi - lo; None for
    the uniform mesh."""
    c = Cfg()
    c.nx, c.ny, c.nz = (int(s) for s in shape)
    c.k = int(k)
    c.nq = int(nq if nq else k + 1)
    for e in range(3):
        c.lo[e] = float(lo[e])
        c.hi[e] = float(hi[e])
    c.gamma, c.mu, c.prandtl = float(gamma), float(mu), float(prandtl)
    c.widths = None
    if widths is not None:
        w = np.ascontiguousarray(widths, dtype=np.float64)
        if w.shape != (c.nx + c.ny + c.nz,) or not np.all(w > 0):
            raise ValueError("widths: nx + ny + nz positive cell widths")
        c._widths = w  # keeps the array alive as long as the configuration
        c.widths = w.ctypes.data
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        dp = P(d)
        cp = P(Cfg)
        sig = {
            "orc_num_threads": (i, []),
            "orc_gauss": (None, [i, dp, dp]),
            "orc_legendre": (None, [i, d, dp, dp]),
            "orc_nmodes": (i, [i]),
            "orc_modes": (None, [i, P(i)]),
            "orc_moments": (None, [d, d, d, i, dp, dp]),
            "orc_slope": (None, [dp, d, d, dp, dp, dp]),
            "orc_time_integrals": (None, [d, d, dp]),
            "orc_volume_flux": (None, [cp, dp, dp, dp, dp]),
            "orc_face_flux": (None, [cp, d, i, dp, dp, dp, dp, dp, dp]),
            "orc_mass_entry": (d, [i, i, i]),
            "orc_residual": (None, [cp, dp, d, dp, dp]),
            "orc_residual_cells": (None, [cp, dp, d, P(i64), i64, dp, dp]),
            "orc_residual_slab": (None, [cp, dp, d, i, i, dp, dp]),
            "orc_step": (None, [cp, dp, d, i]),
            "orc_step_cells": (None, [cp, dp, d, P(i64), i64, dp]),
            "orc_project": (None, [cp, i, dp]),
            "orc_kinetic_energy": (d, [cp, dp]),
            "orc_enstrophy": (d, [cp, dp]),
            "orc_advection_error": (d, [cp, dp, d, i, i]),
            "orc_step_jvp": (None, [cp, dp, dp, d, d, i, dp, dp]),
            "orc_ke_jvp": (None, [cp, dp, dp, dp, dp]),
            "orc_volume_flux_jvp": (None, [cp, dp, dp, dp, dp, d, dp, dp, dp, dp]),
            "orc_face_flux_jvp": (None, [cp, d, i, dp, dp, d, dp, dp, dp, dp]),
            "orc_s2o4_linear": (d, [d, d, i]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads():
    return lib().orc_num_threads()


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss(n, _p(x), _p(w))
    return x, w


def legendre(lmax, x):
    P = np.zeros(lmax + 1)
    dP = np.zeros(lmax + 1)
    lib().orc_legendre(lmax, float(x), _p(P), _p(dP))
    return P, dP


def nmodes(k):
    return lib().orc_nmodes(k)


def modes(k):
    n = nmodes(k)
    out = (ctypes.c_int * (3 * n))()
    lib().orc_modes(k, out)
    return np.array(list(out), dtype=np.int64).reshape(n, 3)


def moments(U, lam, K, side=0):
    """Normalised 1-D moments <c^0..c^8> (side 0 full, +1 u>0, -1 u<0) and <xi^0,2,4>."""
    u = np.zeros(9)
    x = np.zeros(3)
    lib().orc_moments(float(U), float(lam), float(K), int(side), _p(u), _p(x))
    return u, x


def slope(U, lam, K, b):
    Uv = _f64(U, (3,))
    bv = _f64(b, (5,))
    a = np.zeros(5)
    M = np.zeros(25)
    lib().orc_slope(_p(Uv), float(lam), float(K), _p(bv), _p(a), _p(M))
    return a, M.reshape(5, 5)


def time_integrals(tau, delta):
    c = np.zeros(6)
    lib().orc_time_integrals(float(tau), float(delta), _p(c))
    return c


def volume_flux(cfg, q, dq):
    q = _f64(q, (5,))
    dq = _f64(dq, (3, 5))
    F = np.zeros((3, 5))
    Ft = np.zeros((3, 5))
    lib().orc_volume_flux(ctypes.byref(cfg), _p(q), _p(dq), _p(F), _p(Ft))
    return F, Ft


def face_flux(cfg, dt, d, qL, dqL, qR, dqR):
    qL, qR = _f64(qL, (5,)), _f64(qR, (5,))
    dqL, dqR = _f64(dqL, (3, 5)), _f64(dqR, (3, 5))
    F = np.zeros(5)
    Ft = np.zeros(5)
    lib().orc_face_flux(ctypes.byref(cfg), float(dt), int(d), _p(qL), _p(dqL), _p(qR), _p(dqR), _p(F), _p(Ft))
    return F, Ft


def mass_entry(k, n1, n2):
    return lib().orc_mass_entry(k, n1, n2)


def field_shape(cfg):
    return (5, nmodes(cfg.k), cfg.nz, cfg.ny, cfg.nx)


def residual(cfg, q, dt):
    q = _f64(q, field_shape(cfg))
    L = np.zeros_like(q)
    Lt = np.zeros_like(q)
    lib().orc_residual(ctypes.byref(cfg), _p(q), float(dt), _p(L), _p(Lt))
    return L, Lt


def residual_cells(cfg, q, dt, cells):
    """L, L_t of the listed flat cell indices; output shape (ncells, 5, nmodes)."""
    q = _f64(q, field_shape(cfg))
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    nm = nmodes(cfg.k)
    L = np.zeros((len(cells), 5, nm))
    Lt = np.zeros_like(L)
    lib().orc_residual_cells(ctypes.byref(cfg), _p(q), float(dt),
                             cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cells), _p(L), _p(Lt))
    return L, Lt


def residual_slab(cfg, q, dt, k0, k1):
    q = _f64(q, field_shape(cfg))
    nm = nmodes(cfg.k)
    n = cfg.nx * cfg.ny * (k1 - k0)
    L = np.zeros((n, 5, nm))
    Lt = np.zeros_like(L)
    lib().orc_residual_slab(ctypes.byref(cfg), _p(q), float(dt), int(k0), int(k1), _p(L), _p(Lt))
    return L, Lt


def step_cells(cfg, q, dt, cells):
    """Q^{n+1} of one step at the listed flat cell indices; shape (ncells, 5, nmodes)."""
    q = _f64(q, field_shape(cfg))
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
    out = np.zeros((len(cells), 5, nmodes(cfg.k)))
    lib().orc_step_cells(ctypes.byref(cfg), _p(q), float(dt), cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         len(cells), _p(out))
    return out


def step(cfg, q, dt, nsteps=1):
    q = _f64(q, field_shape(cfg)).copy()
    lib().orc_step(ctypes.byref(cfg), _p(q), float(dt), int(nsteps))
    return q


def project(cfg, problem):
    """L2 projection of analytic initial data.  problem: 'advection' (3-D
    diagonal), 'tgv', or 'advection_x' / 'advection_y' / 'advection_z'."""
    which = {"advection": 0, "tgv": 1, "advection_x": 2, "advection_y": 3, "advection_z": 4}[problem]
    q = np.zeros(field_shape(cfg))
    lib().orc_project(ctypes.byref(cfg), which, _p(q))
    return q


def kinetic_energy(cfg, q):
    q = _f64(q, field_shape(cfg))
    return lib().orc_kinetic_energy(ctypes.byref(cfg), _p(q))


def enstrophy(cfg, q):
    """sum over cells of |K| sum_q w_q |curl U|^2 / 2 on the volume Gauss rule."""
    q = _f64(q, field_shape(cfg))
    return lib().orc_enstrophy(ctypes.byref(cfg), _p(q))


def advection_error(cfg, q, t, problem="advection", nqe=5):
    which = {"advection": 0, "advection_x": 2, "advection_y": 3, "advection_z": 4}[problem]
    q = _f64(q, field_shape(cfg))
    return lib().orc_advection_error(ctypes.byref(cfg), _p(q), float(t), which, int(nqe))


def step_jvp(cfg, q, dq, dmu, dt, nsteps):
    q = _f64(q, field_shape(cfg))
    dq = _f64(dq, field_shape(cfg))
    qo = np.zeros_like(q)
    dqo = np.zeros_like(q)
    lib().orc_step_jvp(ctypes.byref(cfg), _p(q), _p(dq), float(dmu), float(dt), int(nsteps), _p(qo), _p(dqo))
    return qo, dqo


def ke_jvp(cfg, q, dq):
    q = _f64(q, field_shape(cfg))
    dq = _f64(dq, field_shape(cfg))
    J = ctypes.c_double()
    dJ = ctypes.c_double()
    lib().orc_ke_jvp(ctypes.byref(cfg), _p(q), _p(dq), ctypes.byref(J), ctypes.byref(dJ))
    return J.value, dJ.value


def volume_flux_jvp(cfg, q, dq, tq, tdq, tmu):
    q, tq = _f64(q, (5,)), _f64(tq, (5,))
    dq, tdq = _f64(dq, (3, 5)), _f64(tdq, (3, 5))
    F, dF, Ft, dFt = (np.zeros((3, 5)) for _ in range(4))
    lib().orc_volume_flux_jvp(ctypes.byref(cfg), _p(q), _p(dq), _p(tq), _p(tdq), float(tmu),
                              _p(F), _p(dF), _p(Ft), _p(dFt))
    return F, dF, Ft, dFt


def face_flux_jvp(cfg, dt, d, x, tx, tmu):
    x, tx = _f64(x, (40,)), _f64(tx, (40,))
    F, dF, Ft, dFt = (np.zeros(5) for _ in range(4))
    lib().orc_face_flux_jvp(ctypes.byref(cfg), float(dt), int(d), _p(x), _p(tx), float(tmu),
                            _p(F), _p(dF), _p(Ft), _p(dFt))
    return F, dF, Ft, dFt


def s2o4_linear(z, dt, nsteps):
    return lib().orc_s2o4_linear(float(z), float(dt), int(nsteps))
