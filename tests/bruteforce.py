"""Brute-force velocity-space quadrature of the BGK distribution functions.

Test-only pins for the oracle.  Nothing here shares code with the oracle or the
HIP library: every moment is a numerical integral over a tensor grid in
(u, v, w, s = xi^2) -- Gauss-Hermite nodes for the full Gaussian directions,
Gauss-Legendre nodes on a truncated half line for half-space integrals, and a
generalised Gauss-Laguerre rule for s, whose law for K internal degrees of
freedom is Gamma(K/2, scale 1/lambda).  The 5x5 slope systems are solved with
``numpy.linalg.solve`` and the time integrals with ``scipy.integrate.quad_vec``.
"""
import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from scipy import integrate
from scipy.special import roots_genlaguerre


class MaxwellQuad:
    """Expectation over the normalised Maxwellian of (rho, U, V, W, lambda).

    half = 0: whole velocity space; +1: u > 0 only; -1: u < 0 only.
    """

    def __init__(self, U, V, W, lam, K, half=0, n_gh=24, n_half=240, n_s=4):
        sig = 1.0 / np.sqrt(2.0 * lam)
        x, w = hermegauss(n_gh)
        w = w / np.sqrt(2.0 * np.pi)
        vn, wn = V + sig * x, W + sig * x
        if half == 0:
            un, uw = U + sig * x, w
        else:
            if half > 0:
                a, b = 0.0, max(U + 16.0 * sig, 16.0 * sig * 1e-3)
            else:
                a, b = min(U - 16.0 * sig, -16.0 * sig * 1e-3), 0.0
            xl, wl = np.polynomial.legendre.leggauss(n_half)
            un = 0.5 * (b - a) * xl + 0.5 * (b + a)
            uw = 0.5 * (b - a) * wl * np.exp(-((un - U) ** 2) / (2 * sig * sig)) / (np.sqrt(2 * np.pi) * sig)
        xs, ws = roots_genlaguerre(n_s, K / 2.0 - 1.0)
        ws = ws / ws.sum()
        sn = xs / lam
        self.u, self.v, self.w, self.s = np.meshgrid(un, vn, wn, sn, indexing="ij", sparse=True)
        self.wt = uw[:, None, None, None] * w[None, :, None, None] * w[None, None, :, None] * ws[None, None, None, :]
        self.vel = (self.u, self.v, self.w)

    def mean(self, h):
        return float(np.sum(self.wt * h))

    def psi(self):
        u, v, w, s = self.u, self.v, self.w, self.s
        return [np.ones_like(u), u, v, w, 0.5 * (u * u + v * v + w * w + s)]

    def mean_psi(self, h):
        """<h psi_k>, k = 0..4."""
        return np.array([self.mean(h * p) for p in self.psi()])

    def poly(self, a):
        """sum_j a_j psi_j evaluated on the grid."""
        return sum(aj * p for aj, p in zip(a, self.psi()))

    def m5(self):
        ps = self.psi()
        return np.array([[self.mean(pi * pj) for pj in ps] for pi in ps])


def primitives(Q, gamma):
    rho = Q[0]
    U = Q[1:4] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * U @ U)
    return rho, U, p, rho / (2.0 * p)


def kdof(gamma):
    return (5.0 - 3.0 * gamma) / (gamma - 1.0)


def _slopes(Qf, rho, dq):
    """a_i from <a_i psi> = dQ/dn_i / rho, and A from compatibility."""
    M = Qf.m5()
    a = [np.linalg.solve(M, dq[i] / rho) for i in range(3)]
    rhs = -sum(Qf.mean_psi(Qf.vel[i] * Qf.poly(a[i])) for i in range(3))
    A = np.linalg.solve(M, rhs)
    return a, A


def volume_flux(gamma, mu, prandtl, q, dq):
    """f = g (1 - tau (a.u + A) + A t) (global frame); returns F[3,5], Ft[3,5]."""
    K = kdof(gamma)
    rho, U, p, lam = primitives(np.asarray(q, float), gamma)
    G = MaxwellQuad(U[0], U[1], U[2], lam, K)
    a, A = _slopes(G, rho, np.asarray(dq, float))
    tau = mu / p
    X = sum(G.vel[e] * G.poly(a[e]) for e in range(3)) + G.poly(A)
    F = np.zeros((3, 5))
    Ft = np.zeros((3, 5))
    c2 = sum((G.vel[e] - U[e]) ** 2 for e in range(3)) + G.s
    for d in range(3):
        ud = G.vel[d]
        F[d] = rho * G.mean_psi(ud * (1.0 - tau * X))
        Ft[d] = rho * G.mean_psi(ud * G.poly(A))
        q_heat = -tau * rho * G.mean((ud - U[d]) * 0.5 * c2 * X)
        F[d, 4] += (1.0 / prandtl - 1.0) * q_heat
    return F, Ft


def face_flux_local(gamma, mu, prandtl, dt, qL, dqL, qR, dqR):
    """Eq. (flux) in the local frame (normal = first velocity component).

    dqL[i] is the derivative along local direction i.  Returns F[5], Ft[5] from
    the linear-in-time fit of the integrated flux over [0, dt] and [0, dt/2].
    """
    K = kdof(gamma)
    sides = []
    for s, (q, dq) in enumerate(((qL, dqL), (qR, dqR))):
        rho, U, p, lam = primitives(np.asarray(q, float), gamma)
        Gf = MaxwellQuad(U[0], U[1], U[2], lam, K)
        Gh = MaxwellQuad(U[0], U[1], U[2], lam, K, half=(+1 if s == 0 else -1))
        a, A = _slopes(Gf, rho, np.asarray(dq, float))
        sides.append((rho, Gh, a, A))
    Q0 = sum(rho * Gh.mean_psi(1.0) for rho, Gh, a, A in sides)
    dQ0 = [sum(rho * Gh.mean_psi(Gh.poly(a[i])) for rho, Gh, a, A in sides) for i in range(3)]
    rho0, U0, p0, lam0 = primitives(Q0, gamma)
    G0 = MaxwellQuad(U0[0], U0[1], U0[2], lam0, K)
    abar, Abar = _slopes(G0, rho0, np.array(dQ0))
    tau = mu / p0
    u0 = G0.u
    V1 = rho0 * G0.mean_psi(u0)
    V2 = rho0 * G0.mean_psi(u0 * sum(G0.vel[i] * G0.poly(abar[i]) for i in range(3)))
    V3 = rho0 * G0.mean_psi(u0 * G0.poly(Abar))
    W0 = sum(rho * Gh.mean_psi(Gh.u) for rho, Gh, a, A in sides)
    W1 = sum(rho * Gh.mean_psi(Gh.u * sum(Gh.vel[i] * Gh.poly(a[i]) for i in range(3))) for rho, Gh, a, A in sides)
    W2 = sum(rho * Gh.mean_psi(Gh.u * Gh.poly(A)) for rho, Gh, a, A in sides)

    def flux(t):
        e = np.exp(-t / tau) if tau > 0 else 0.0
        return ((1 - e) * V1 + ((t + tau) * e - tau) * V2 + (t - tau + tau * e) * V3
                + e * (W0 - (tau + t) * W1 - tau * W2))

    def time_integral(T):
        pts = [x for x in (tau, 10 * tau, 50 * tau) if 0 < x < T]
        val, _ = integrate.quad_vec(flux, 0.0, T, epsabs=0.0, epsrel=1e-14, points=pts or None, limit=400)
        return val

    I1, I2 = time_integral(dt), time_integral(0.5 * dt)
    Msys = np.array([[dt, 0.5 * dt * dt], [0.5 * dt, dt * dt / 8.0]])
    sol = np.linalg.solve(Msys, np.vstack([I1, I2]))
    F, Ft = sol[0].copy(), sol[1].copy()
    c2 = sum((G0.vel[e] - U0[e]) ** 2 for e in range(3)) + G0.s
    X = sum(G0.vel[i] * G0.poly(abar[i]) for i in range(3)) + G0.poly(Abar)
    q_heat = -tau * rho0 * G0.mean((u0 - U0[0]) * 0.5 * c2 * X)
    F[4] += (1.0 / prandtl - 1.0) * q_heat
    return F, Ft


def to_local(d, q, dq):
    """Global -> local frame with normal axis d; axes (d, d+1, d+2) mod 3."""
    ax = [d, (d + 1) % 3, (d + 2) % 3]
    q = np.asarray(q, float)
    dq = np.asarray(dq, float)
    ql = np.array([q[0], q[1 + ax[0]], q[1 + ax[1]], q[1 + ax[2]], q[4]])
    dql = np.array([[dq[ax[i]][0], dq[ax[i]][1 + ax[0]], dq[ax[i]][1 + ax[1]], dq[ax[i]][1 + ax[2]], dq[ax[i]][4]]
                    for i in range(3)])
    return ql, dql


def from_local(d, Fl):
    ax = [d, (d + 1) % 3, (d + 2) % 3]
    F = np.zeros(5)
    F[0], F[4] = Fl[0], Fl[4]
    for i in range(3):
        F[1 + ax[i]] = Fl[1 + i]
    return F


def face_flux(gamma, mu, prandtl, dt, d, qL, dqL, qR, dqR):
    qLl, dqLl = to_local(d, qL, dqL)
    qRl, dqRl = to_local(d, qR, dqR)
    F, Ft = face_flux_local(gamma, mu, prandtl, dt, qLl, dqLl, qRl, dqRl)
    return from_local(d, F), from_local(d, Ft)


def euler_flux(Q, d, gamma):
    """Textbook Euler flux along axis d (works with complex Q for complex-step)."""
    rho = Q[0]
    m = Q[1:4]
    E = Q[4]
    p = (gamma - 1.0) * (E - 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / rho)
    out = [m[d]]
    for i in range(3):
        out.append(m[d] * m[i] / rho + (p if i == d else 0.0))
    out.append((E + p) * m[d] / rho)
    return np.array(out)


def euler_jvp(Q, d, v, gamma, h=1e-30):
    """Complex-step directional derivative J_d(Q) v, exact to round-off."""
    Qc = np.asarray(Q, complex) + 1j * h * np.asarray(v, float)
    return np.imag(euler_flux(Qc, d, gamma)) / h


def ns_flux(gamma, mu, prandtl, q, dq):
    """Navier-Stokes flux from the Chapman-Enskog expansion of BGK with K
    internal degrees of freedom: stress mu (dU_i/dx_j + dU_j/dx_i -
    2/(K+3) delta_ij div U), heat flux -(c_p mu / Pr) grad T, c_p = (K+5)/2,
    T = p / rho (R = 1).  Returns F[3,5]."""
    K = kdof(gamma)
    q = np.asarray(q, float)
    dq = np.asarray(dq, float)
    rho = q[0]
    U = q[1:4] / rho
    p = (gamma - 1.0) * (q[4] - 0.5 * rho * U @ U)
    T = p / rho
    dU = np.zeros((3, 3))  # dU[e][i] = dU_i/dx_e
    dT = np.zeros(3)
    for e in range(3):
        drho = dq[e][0]
        dm = dq[e][1:4]
        dU[e] = (dm - U * drho) / rho
        dp = (gamma - 1.0) * (dq[e][4] - (q[1:4] @ dm) / rho + 0.5 * (q[1:4] @ q[1:4]) * drho / rho ** 2)
        dT[e] = (dp - T * drho) / rho
    div = np.trace(dU)
    cp = (K + 5.0) / 2.0
    F = np.zeros((3, 5))
    for d in range(3):
        sig = np.array([mu * (dU[d][i] + dU[i][d] - (2.0 / (K + 3.0)) * (div if i == d else 0.0)) for i in range(3)])
        F[d] = euler_flux(q, d, gamma)
        F[d, 1:4] -= sig
        F[d, 4] -= U @ sig + cp * mu / prandtl * dT[d]
    return F
