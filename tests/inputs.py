"""Seeded synthetic inputs shared by the oracle and the HIP path in tests.

This module holds no arithmetic of the method: it only draws random numbers in
stated ranges.  Point states are drawn directly in conservative form through
(rho, U, internal energy density), so no equation of state is used here.
"""
import numpy as np


def point_state(rng, low_mach=False):
    """Conservative state (rho, rho U, rho V, rho W, rho E)."""
    rho = rng.uniform(0.5, 2.0)
    U = rng.uniform(-1.5, 1.5, size=3)
    if low_mach:
        eint = rng.uniform(170.0, 190.0)  # p ~ 71 with gamma = 1.4
    else:
        eint = rng.uniform(0.75, 7.5)  # p in [0.3, 3] with gamma = 1.4
    return np.array([rho, rho * U[0], rho * U[1], rho * U[2], eint + 0.5 * rho * U @ U])


def point_gradient(rng, scale=0.5):
    """dQ/dx_e for e = 0,1,2 as a (3, 5) array."""
    return rng.normal(0.0, scale, size=(3, 5))


def random_field(rng, shape, nmodes, amp=0.02, low_mach=False):
    """Random modal field q[5][nmodes][nz][ny][nx] (shape = (nx, ny, nz)).

    Mode 0 is a smooth random mean state per cell; higher modes are small
    random perturbations of relative size `amp`, so every point value stays
    physical.
    """
    nx, ny, nz = shape
    q = np.zeros((5, nmodes, nz, ny, nx))
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, size=8)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * y + ph[1]) + 0.1 * np.sin(2 * np.pi * z + ph[2])
    U = 0.5 * np.sin(2 * np.pi * (y + z) + ph[3])
    V = 0.4 * np.cos(2 * np.pi * (x - z) + ph[4])
    W = 0.3 * np.sin(2 * np.pi * (x + y) + ph[5])
    eint = (180.0 if low_mach else 2.5) * (1.0 + 0.1 * np.cos(2 * np.pi * (x + y + z) + ph[6]))
    q[0, 0] = rho
    q[1, 0] = rho * U
    q[2, 0] = rho * V
    q[3, 0] = rho * W
    q[4, 0] = eint + 0.5 * rho * (U * U + V * V + W * W)
    for v in range(5):
        scale = np.abs(q[v, 0]).mean() + 0.1
        q[v, 1:] = amp * scale * rng.uniform(-1.0, 1.0, size=q[v, 1:].shape)
    return q


def random_direction(rng, like):
    return rng.normal(0.0, 1.0, size=like.shape)


def mapped_widths(n, lo=0.0, hi=2.0, amp=0.05):
    """Cell widths along one axis of the Section 5.1 non-uniform mesh: nodes
    xi_i = lo + i (hi - lo) / n mapped by x = xi + amp (hi - lo) / 2
    sin(2 pi (xi - lo) / (hi - lo)), i.e. x = xi + 0.05 sin(pi xi) on [0, 2]."""
    L = hi - lo
    xi = lo + np.arange(n + 1) * (L / n)
    x = xi + amp * L / 2.0 * np.sin(2.0 * np.pi * (xi - lo) / L)
    x[0], x[-1] = lo, hi
    return np.diff(x)


def random_widths(rng, shape, lo, hi, spread=0.4):
    """nx + ny + nz random cell widths, uniform in [1 - spread, 1 + spread]
    times the mean width, each axis summing to hi - lo."""
    out = []
    for e, n in enumerate(shape):
        w = rng.uniform(1.0 - spread, 1.0 + spread, n)
        out.append(w * (hi[e] - lo[e]) / w.sum())
    return np.concatenate(out)
