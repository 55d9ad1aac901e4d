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


def mapped_widths(n, lo=0.0, hi=2.0, amp=0.05):
    """Cell widths of the non-uniform mesh of Section 5.1 along one axis: the
    nodes of n uniform cells, xi_i = lo + i (hi - lo) / n, mapped by
    x = xi + amp (hi - lo) / 2 sin(2 pi (xi - lo) / (hi - lo)) (on [0, 2]:
    x = xi + 0.05 sin(pi xi)); the end nodes stay at lo and hi."""
    L = hi - lo
    xi = lo + np.arange(n + 1) * (L / n)
    x = xi + amp * L / 2.0 * np.sin(2.0 * np.pi * (xi - lo) / L)
    x[0], x[-1] = lo, hi
    return np.diff(x)


def _project_1d(f, n, lo, hi, degree, widths=None):
    """P[l][i] = sum_g w_g f(x_g) P_l(xi_g) over cell i (weights sum to 1)."""
    xg, wg = np.polynomial.legendre.leggauss(NQ_INIT)
    wg = wg / 2.0
    if widths is None:
        dx = (hi - lo) / n
        centers = lo + (np.arange(n) + 0.5) * dx
    else:
        dx = np.asarray(widths, dtype=np.float64)
        centers = lo + np.concatenate([[0.0], np.cumsum(dx)[:-1]]) + 0.5 * dx
        dx = dx[:, None]
    x = centers[:, None] + 0.5 * dx * xg[None, :]
    fx = f(x)
    return np.stack([(fx * (wg * _legendre(l, xg))[None, :]).sum(axis=1) for l in range(degree + 1)])


def split_widths(shape, widths):
    """(wx, wy, wz) of a concatenated widths array, or (None,) * 3."""
    if widths is None:
        return (None, None, None)
    w = np.asarray(widths, dtype=np.float64).ravel()
    nx, ny, nz = shape
    return (w[:nx], w[nx:nx + ny], w[nx + ny:])


def project_separable(terms, shape, lo, hi, degree, widths=None):
    """terms[var] = list of (coef, fx, fy, fz); returns q[5][nmodes][nz][ny][nx].
    widths: optional nx + ny + nz cell widths of a separable mesh."""
    nx, ny, nz = shape
    wx, wy, wz = split_widths(shape, widths)
    md = modes(degree)
    q = np.zeros((5, len(md), nz, ny, nx))
    for v, tl in enumerate(terms):
        for coef, fx, fy, fz in tl:
            px = _project_1d(fx, nx, lo[0], hi[0], degree, wx)
            py = _project_1d(fy, ny, lo[1], hi[1], degree, wy)
            pz = _project_1d(fz, nz, lo[2], hi[2], degree, wz)
            for n, (a, b, c) in enumerate(md):
                scale = coef * (2 * a + 1) * (2 * b + 1) * (2 * c + 1)
                q[v, n] += scale * pz[c][:, None, None] * py[b][None, :, None] * px[a][None, None, :]
    return q


one = lambda x: np.ones_like(x)


def tgv(shape, degree, gamma=1.4, mach=0.1, widths=None):
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
    return project_separable(terms, shape, lo, hi, degree, widths), lo, hi


def advection(shape, degree, gamma=1.4, widths=None):
    pi = math.pi
    s = lambda x: np.sin(pi * x)
    c = lambda x: np.cos(pi * x)
    # sin(a + b + c) = s c c + c s c + c c s - s s s
    rho = [(1.0, one, one, one), (0.2, s, c, c), (0.2, c, s, c), (0.2, c, c, s), (-0.2, s, s, s)]
    energy = [(1.0 / (gamma - 1.0), one, one, one)] + [(1.5 * k, fx, fy, fz) for k, fx, fy, fz in rho]
    terms = [rho, rho, rho, rho, energy]
    lo, hi = (0.0,) * 3, (2.0,) * 3
    return project_separable(terms, shape, lo, hi, degree, widths), lo, hi


def cfl_dt(cfl, dx_min, max_speed):
    """dt = CFL * min dx / max(|U_d| + c) (the time-step rule whose values
    match the Taylor-Green step sizes quoted with the paper's timings)."""
    return cfl * dx_min / max_speed


def tgv_dt(n, cfl=0.15, gamma=1.4, mach=0.1):
    p_max = 1.0 / (gamma * mach * mach) + 2.0 * 3.0 / 16.0
    return cfl_dt(cfl, 2 * math.pi / n, 1.0 + math.sqrt(gamma * p_max))


def advection_dt(n, cfl=0.1, gamma=1.4, dx_min=None):
    rho_min = 0.8
    return cfl_dt(cfl, 2.0 / n if dx_min is None else dx_min, 1.0 + math.sqrt(gamma * 1.0 / rho_min))


def paper_mesh(n, lo=0.0, hi=2.0):
    """Concatenated widths of the Section 5.1 mapped mesh, n cells per axis."""
    w = mapped_widths(n, lo, hi)
    return np.concatenate([w, w, w])
