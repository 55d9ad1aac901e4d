"""Python front end of the C-ABI: a Solver bound to one HIP stream, and a
torch.autograd.Function around the forward step and its hand-written adjoint.

torch provides device memory and the stream; every operation of the method
runs in libdg_hgks.so.
"""
import ctypes
import math

import numpy as np
import torch

from . import _lib
from .problems import nmodes

PRECISIONS = {"fp64": _lib.DG_HGKS_FP64, "fp32_bulk": _lib.DG_HGKS_FP32_BULK}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One DG-HGKS discretisation on a periodic box.

    q tensors: float64, shape (5, nmodes, nz, ny, nx), contiguous, on `device`.
    """

    def __init__(self, shape, lo, hi, degree, nq=0, gamma=1.4, mu=0.0, prandtl=1.0, precision="fp64",
                 device="cuda", max_stride=0, widths=None):
        """widths: optional separable mesh, the nx + ny + nz cell widths (x,
        then y, then z), each axis summing to hi - lo (see problems.mapped_widths);
        None for uniform cells."""
        self.lib = _lib.load()
        self.shape = tuple(int(s) for s in shape)
        self.lo, self.hi = tuple(lo), tuple(hi)
        self.degree = int(degree)
        self.nq = int(nq) if nq else self.degree + 1
        self.gamma, self.prandtl = float(gamma), float(prandtl)
        self._mu = float(mu)
        self.precision = precision
        self.device = torch.device(device)
        self.widths = None if widths is None else np.ascontiguousarray(widths, dtype=np.float64).ravel()
        self.params = _lib.make_params(self.shape, lo, hi, degree, nq, gamma, mu, prandtl, PRECISIONS[precision],
                                       self.widths)
        nbytes = self.lib.dg_hgks_workspace_bytes(ctypes.byref(self.params), int(max_stride))
        if nbytes == 0:
            raise _lib.DGHGKSError(_lib.DG_HGKS_EINVAL, "invalid parameters")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = self.lib.dg_hgks_init(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                                   _ptr(self.workspace), int(nbytes), ctypes.byref(ctx))
        _lib.check(rc, None)
        self.ctx = ctx
        self.max_stride = int(max_stride)

    # -- helpers -------------------------------------------------------------
    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (5, nmodes(self.degree), nz, ny, nx)

    @property
    def mu(self):
        return self._mu

    def _chk(self, rc):
        return _lib.check(rc, self.ctx)

    def _field(self, q, name="q"):
        if q.dtype != torch.float64 or q.device != self.device or not q.is_contiguous() \
                or tuple(q.shape) != self.field_shape:
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {self.field_shape} on "
                             f"{self.device}")
        return q

    # -- C-ABI calls -----------------------------------------------------------
    def set_mu(self, mu):
        self._chk(self.lib.dg_hgks_set_mu(self.ctx, float(mu)))
        self._mu = float(mu)

    def step(self, q, dt, nsteps=1, ckpt=None, ckpt_stride=0):
        """Advance q in place by nsteps S2O4 steps."""
        self._field(q)
        cp = _ptr(ckpt) if ckpt is not None else None
        self._chk(self.lib.dg_hgks_step(self.ctx, _ptr(q), float(dt), int(nsteps), cp, int(ckpt_stride)))
        return q

    def residual(self, q, dt):
        self._field(q)
        L = torch.empty_like(q)
        Lt = torch.empty_like(q)
        self._chk(self.lib.dg_hgks_residual(self.ctx, _ptr(q), float(dt), _ptr(L), _ptr(Lt)))
        return L, Lt

    def adjoint(self, ckpt, ckpt_stride, dt, nsteps, qN_bar):
        """Returns (q0_bar, mu_bar)."""
        self._field(qN_bar, "qN_bar")
        q0_bar = torch.empty_like(qN_bar)
        mu_bar = ctypes.c_double()
        self._chk(self.lib.dg_hgks_adjoint(self.ctx, _ptr(ckpt), int(ckpt_stride), float(dt), int(nsteps),
                                           _ptr(qN_bar), _ptr(q0_bar), ctypes.byref(mu_bar)))
        return q0_bar, mu_bar.value

    def check(self):
        self._chk(self.lib.dg_hgks_check(self.ctx))

    def point_face_flux(self, x, axis, dt):
        x = x.contiguous()
        n = x.shape[0]
        F = torch.empty((n, 5), dtype=torch.float64, device=self.device)
        Ft = torch.empty_like(F)
        self._chk(self.lib.dg_hgks_point_face_flux(self.ctx, _ptr(x), n, int(axis), float(dt), _ptr(F), _ptr(Ft)))
        return F, Ft

    def point_volume_flux(self, x):
        x = x.contiguous()
        n = x.shape[0]
        F = torch.empty((n, 3, 5), dtype=torch.float64, device=self.device)
        Ft = torch.empty_like(F)
        self._chk(self.lib.dg_hgks_point_volume_flux(self.ctx, _ptr(x), n, _ptr(F), _ptr(Ft)))
        return F, Ft

    def diagnostics(self, q, grad=False):
        """((kinetic energy, enstrophy), dE_k/dq or None) of the state q on the
        volume Gauss rule (Section 5.3 Taylor-Green diagnostics, FP64)."""
        q = q.detach().contiguous()
        out = (ctypes.c_double * 2)()
        g = torch.empty_like(q) if grad else None
        self._chk(self.lib.dg_hgks_diagnostics(self.ctx, _ptr(q), out, _ptr(g) if grad else None))
        return (out[0], out[1]), g

    def set_timing(self, enable=True):
        self._chk(self.lib.dg_hgks_set_timing(self.ctx, 1 if enable else 0))

    def get_timing(self):
        """{'face': (ms, launches), 'volume': ..., 'convert': ..., 'adj_face': ..., 'adj_volume': ...}"""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int64 * 5)()
        rc = self.lib.dg_hgks_get_timing(self.ctx, ms, cnt, 5)
        if rc < 0:
            self._chk(rc)
        names = ["face", "volume", "convert", "adj_face", "adj_volume"]
        return {k: (ms[i], cnt[i]) for i, k in enumerate(names)}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dg_hgks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- time integration with checkpoints -------------------------------------
    def checkpoint_stride(self, nsteps):
        return max(1, int(math.ceil(math.sqrt(nsteps))))

    def new_checkpoints(self, nsteps, stride):
        nslots = (nsteps + stride - 1) // stride
        return torch.empty((max(nslots, 1),) + self.field_shape, dtype=torch.float64, device=self.device)


def step_noalloc(q, dt, nsteps, shape, lo, hi, degree, nq=0, gamma=1.4, mu=0.0, prandtl=1.0, precision="fp64",
                 nonphys=None):
    """dg_hgks_step_noalloc: advance q (contiguous float64 (5, nmodes, nz, ny,
    nx) on the current CUDA device) in place by nsteps S2O4 steps on a uniform
    mesh, on torch's current stream, without a context or workspace (the
    library's static device scratch, at most 96 MiB: 32^3 cells at P2 in
    both precisions).  nonphys: optional int32 device tensor of one element
    that receives 1 if a non-physical state was met, else 0."""
    lib = _lib.load()
    nx, ny, nz = (int(x) for x in shape)
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() \
            or tuple(q.shape) != (5, nmodes(degree), nz, ny, nx):
        raise ValueError("q must be a contiguous float64 CUDA tensor of shape (5, nmodes, nz, ny, nx)")
    if nonphys is not None and (nonphys.dtype != torch.int32 or not nonphys.is_cuda or nonphys.numel() < 1):
        raise ValueError("nonphys must be an int32 CUDA tensor")
    params = _lib.make_params((nx, ny, nz), lo, hi, degree, nq, gamma, mu, prandtl, PRECISIONS[precision])
    stream = torch.cuda.current_stream(q.device)
    with torch.cuda.device(q.device):
        rc = lib.dg_hgks_step_noalloc(ctypes.byref(params), ctypes.c_void_p(stream.cuda_stream), _ptr(q), float(dt),
                                      int(nsteps), _ptr(nonphys) if nonphys is not None else None)
    _lib.check(rc, None)
    return q


class _KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, solver):
        need = bool(ctx.needs_input_grad[0])
        (ek, _), grad = solver.diagnostics(q, grad=need)
        if need:
            ctx.save_for_backward(grad)
        return torch.tensor(ek, dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return gout * grad, None


def kinetic_energy(q, solver):
    """Domain-integrated kinetic energy J = sum_K |K| sum_q w_q |rho U|^2/(2 rho)
    on the volume Gauss rule of the solver, evaluated on the device
    (dg_hgks_diagnostics), differentiable in q through the device gradient."""
    return _KineticEnergy.apply(q, solver)


class DGHGKSSteps(torch.autograd.Function):
    """q_N = S2O4^n(q_0; mu) with gradients from the hand-written adjoint.

    forward(q0, mu_tensor, solver, dt, nsteps) stores sqrt(n)-spaced
    checkpoints; backward recomputes each segment and runs the adjoint.
    """

    @staticmethod
    def forward(ctx, q0, mu, solver, dt, nsteps):
        mu_f = float(mu.item())
        solver.set_mu(mu_f)
        stride = solver.checkpoint_stride(nsteps)
        if stride > solver.max_stride:
            raise ValueError(f"solver built with max_stride={solver.max_stride} < {stride}")
        ckpt = solver.new_checkpoints(nsteps, stride)
        q = q0.detach().clone().contiguous()
        solver.step(q, dt, nsteps, ckpt, stride)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.stride, ctx.mu = solver, dt, nsteps, stride, mu_f
        ctx.save_for_backward(ckpt)
        return q

    @staticmethod
    def backward(ctx, gq):
        (ckpt,) = ctx.saved_tensors
        solver = ctx.solver
        # the reverse sweep recomputes the segments and differentiates tau =
        # mu / p with the viscosity of this forward call, whatever the solver
        # holds now (another forward, or a set_mu, may have changed it)
        mu_now = solver.mu
        solver.set_mu(ctx.mu)
        try:
            q0_bar, mu_bar = solver.adjoint(ckpt, ctx.stride, ctx.dt, ctx.nsteps, gq.contiguous())
        finally:
            solver.set_mu(mu_now)
        mu_grad = torch.tensor(mu_bar, dtype=torch.float64, device=gq.device)
        return q0_bar, mu_grad, None, None, None


def steps(q0, mu, solver, dt, nsteps):
    return DGHGKSSteps.apply(q0, mu, solver, dt, nsteps)


def tgv_history(solver, q, dt, nsteps, every=1):
    """Advance q in place by nsteps S2O4 steps of size dt and record, at
    t = 0, every*dt, 2*every*dt, ... (and at the final time), the kinetic
    energy and the enstrophy of the state (device diagnostics, FP64), and the
    kinetic-energy dissipation rate eps = -dE_k/dt from central differences of
    E_k in time (one-sided at the two ends): the Taylor-Green curves of
    Section 5.3.  Values are domain integrals; divide by the box volume for
    the per-volume curves.  For a nearly incompressible flow eps tracks
    2 (mu / rho) times the enstrophy."""
    import numpy as np

    if nsteps < 1 or every < 1:
        raise ValueError("nsteps and every must be >= 1")
    t, ek, en = [0.0], [], []
    (e, w), _ = solver.diagnostics(q)
    ek.append(e)
    en.append(w)
    done = 0
    while done < nsteps:
        m = min(every, nsteps - done)
        solver.step(q, dt, m)
        done += m
        (e, w), _ = solver.diagnostics(q)
        t.append(done * dt)
        ek.append(e)
        en.append(w)
    solver.check()
    t, ek, en = np.array(t), np.array(ek), np.array(en)
    eps = -np.gradient(ek, t) if len(t) > 2 else -np.diff(ek) / np.diff(t) * np.ones(len(t))
    return {"t": t, "kinetic_energy": ek, "enstrophy": en, "dissipation": eps}
