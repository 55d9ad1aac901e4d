"""Initial data of the paper's test problems as modal DG coefficients.

Problem setup, outside the hot path.  Both problems are sums of separable
products f(x) g(y) h(z), so the L2 projection on the P_k Legendre basis
(6-point Gauss rule per direction, the tensor-product rule) factorises into
one-dimensional projections.

* advection (Section 5.1): rho = 1 + 0.2 sin(pi (x + y + z)), U = V = W = 1,
  p = 1 on [0, 2]^3; exact solution rho(x - 3 t).
* Taylor-Green vortex (Section 5.3, with rho = 1): u = sin x cos y cos z,
  v = -cos x sin y cos z, w = 0, p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16
  on [-pi, pi]^3.
"""
import math

import numpy as np

NQ_INIT = 6


def modes(degree):
    """(nx, ny, nz) of every mode, ordered as in the C-ABI."""
    out = []
    for s in range(degree + 1):
        for a in range(s, -1, -1):
            for b in range(s - a, -1, -1):
                out.append((a, b, s - a - b))
    return out


def nmodes(degree):
    return (degree + 1) * (degree + 2) * (degree + 3) // 6


def _legendre(l, x):
    return np.polynomial.legendre.legval(x, [0.0] * l + [1.0])


def _project_1d(f, n, lo, hi, degree):
    """P[l][i] = sum_g w_g f(x_g) P_l(xi_g) over cell i (weights sum to 1)."""
    xg, wg = np.polynomial.legendre.leggauss(NQ_INIT)
    wg = wg / 2.0
    dx = (hi - lo) / n
    centers = lo + (np.arange(n) + 0.5) * dx
    x = centers[:, None] + 0.5 * dx * xg[None, :]
    fx = f(x)
    return np.stack([(fx * (wg * _legendre(l, xg))[None, :]).sum(axis=1) for l in range(degree + 1)])


def project_separable(terms, shape, lo, hi, degree):
    """terms[var] = list of (coef, fx, fy, fz); returns q[5][nmodes][nz][ny][nx]."""
    nx, ny, nz = shape
    md = modes(degree)
    q = np.zeros((5, len(md), nz, ny, nx))
    for v, tl in enumerate(terms):
        for coef, fx, fy, fz in tl:
            px = _project_1d(fx, nx, lo[0], hi[0], degree)
            py = _project_1d(fy, ny, lo[1], hi[1], degree)
            pz = _project_1d(fz, nz, lo[2], hi[2], degree)
            for n, (a, b, c) in enumerate(md):
                scale = coef * (2 * a + 1) * (2 * b + 1) * (2 * c + 1)
                q[v, n] += scale * pz[c][:, None, None] * py[b][None, :, None] * px[a][None, None, :]
    return q


one = lambda x: np.ones_like(x)


def tgv(shape, degree, gamma=1.4, mach=0.1):
    p0 = 1.0 / (gamma * mach * mach)
    sin, cos = np.sin, np.cos
    c2 = lambda x: np.cos(2 * x)
    sq = lambda f: (lambda x: f(x) ** 2)
    g1 = 1.0 / (gamma - 1.0)
    terms = [
        [(1.0, one, one, one)],
        [(1.0, sin, cos, cos)],
        [(-1.0, cos, sin, cos)],
        [],
        [(g1 * p0, one, one, one),
         (g1 / 16.0, c2, one, c2), (g1 * 2.0 / 16.0, c2, one, one),
         (g1 / 16.0, one, c2, c2), (g1 * 2.0 / 16.0, one, c2, one),
         (0.5, sq(sin), sq(cos), sq(cos)), (0.5, sq(cos), sq(sin), sq(cos))],
    ]
    lo, hi = (-math.pi,) * 3, (math.pi,) * 3
    return project_separable(terms, shape, lo, hi, degree), lo, hi


def advection(shape, degree, gamma=1.4):
    pi = math.pi
    s = lambda x: np.sin(pi * x)
    c = lambda x: np.cos(pi * x)
    # sin(a + b + c) = s c c + c s c + c c s - s s s
    rho = [(1.0, one, one, one), (0.2, s, c, c), (0.2, c, s, c), (0.2, c, c, s), (-0.2, s, s, s)]
    energy = [(1.0 / (gamma - 1.0), one, one, one)] + [(1.5 * k, fx, fy, fz) for k, fx, fy, fz in rho]
    terms = [rho, rho, rho, rho, energy]
    lo, hi = (0.0,) * 3, (2.0,) * 3
    return project_separable(terms, shape, lo, hi, degree), lo, hi


def cfl_dt(cfl, dx_min, max_speed):
    """dt = CFL * min dx / max(|U_d| + c) (the time-step rule whose values
    match the Taylor-Green step sizes quoted with the paper's timings)."""
    return cfl * dx_min / max_speed


def tgv_dt(n, cfl=0.15, gamma=1.4, mach=0.1):
    p_max = 1.0 / (gamma * mach * mach) + 2.0 * 3.0 / 16.0
    return cfl_dt(cfl, 2 * math.pi / n, 1.0 + math.sqrt(gamma * p_max))


def advection_dt(n, cfl=0.1, gamma=1.4):
    rho_min = 0.8
    return cfl_dt(cfl, 2.0 / n, 1.0 + math.sqrt(gamma * 1.0 / rho_min))
