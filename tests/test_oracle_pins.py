"""Pins of the FP64 CPU oracle against things other than itself.

Each test ties one part of the oracle to a library routine, a closed form, an
invariant, or an independent brute-force quadrature (tests/bruteforce.py), so
that a dropped term, a wrong sign, a swapped side or a transposed operand in
the oracle fails at least one of them.  No GPU needed.
"""
import numpy as np
import pytest
from scipy import integrate

import bruteforce as BF
import inputs as IN

GAMMA = 1.4
K_DOF = (5.0 - 3.0 * GAMMA) / (GAMMA - 1.0)


# --------------------------------------------------------------------------
# Quadrature, Legendre basis, mode order, mass matrix (Section 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_matches_numpy(orc, n):
    x, w = orc.gauss(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


def test_legendre_matches_numpy(orc):
    from numpy.polynomial import legendre as npl

    for x in np.linspace(-1, 1, 11):
        P, dP = orc.legendre(5, x)
        for l in range(6):
            c = np.zeros(l + 1)
            c[l] = 1.0
            assert abs(P[l] - npl.legval(x, c)) < 1e-14
            assert abs(dP[l] - npl.legval(x, npl.legder(c))) < 1e-13


def test_mode_order_and_counts(orc):
    # dim P_k = (k+1)(k+2)(k+3)/6 (P1: 4, P2: 10, P3: 20)
    for k in (1, 2, 3):
        assert orc.nmodes(k) == (k + 1) * (k + 2) * (k + 3) // 6
    m2 = orc.modes(2).tolist()
    assert m2 == [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 0, 0], [1, 1, 0], [1, 0, 1], [0, 2, 0],
                  [0, 1, 1], [0, 0, 2]]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_mass_matrix_is_orthogonality(orc, k):
    md = orc.modes(k)
    for a in range(len(md)):
        for b in range(len(md)):
            M = orc.mass_entry(k, a, b)
            expect = 1.0 / np.prod(2 * md[a] + 1) if a == b else 0.0
            assert abs(M - expect) < 1e-15


# --------------------------------------------------------------------------
# Maxwellian moments (Section 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.2, 2.0), (0.0, 0.25), (1.4, 0.007)])
def test_moments_vs_scipy_quad(orc, U, lam):
    dens = lambda u: np.sqrt(lam / np.pi) * np.exp(-lam * (u - U) ** 2)
    for side, (a, b) in ((0, (-np.inf, np.inf)), (1, (0.0, np.inf)), (-1, (-np.inf, 0.0))):
        mu, mx = orc.moments(U, lam, K_DOF, side)
        for n in range(9):
            ref, _ = integrate.quad(lambda u: u ** n * dens(u), a, b, epsabs=1e-15, epsrel=1e-13, limit=200)
            scale = max(1.0, abs(ref))
            assert abs(mu[n] - ref) <= 2e-12 * scale, (side, n, mu[n], ref)
    # half spaces add to the full space
    f, _ = orc.moments(U, lam, K_DOF, 0)
    p, _ = orc.moments(U, lam, K_DOF, 1)
    m, _ = orc.moments(U, lam, K_DOF, -1)
    np.testing.assert_allclose(p + m, f, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("K", [1.0, 2.0, 3.0])
def test_internal_dof_moments_vs_brute_force(orc, K):
    # xi = (xi_1..xi_K) i.i.d. N(0, 1/(2 lambda)): <xi^2>, <xi^4> by Gauss-Hermite
    lam = 0.8
    from numpy.polynomial.hermite_e import hermegauss

    x, w = hermegauss(12)
    w = w / w.sum()
    s = 1.0 / np.sqrt(2 * lam)
    grids = np.meshgrid(*([s * x] * int(K)), indexing="ij")
    wt = np.ones_like(grids[0])
    for g in np.meshgrid(*([w] * int(K)), indexing="ij"):
        wt = wt * g
    xi2 = sum(g * g for g in grids)
    _, mx = orc.moments(0.0, lam, K, 0)
    assert abs(mx[0] - 1.0) < 1e-15
    assert abs(mx[1] - np.sum(wt * xi2)) < 1e-13
    assert abs(mx[2] - np.sum(wt * xi2 ** 2)) < 1e-13


def test_slope_solve_vs_dense_quadrature(orc):
    rng = np.random.default_rng(11)
    for _ in range(6):
        U = rng.uniform(-1.5, 1.5, 3)
        lam = rng.uniform(0.1, 2.0)
        b = rng.normal(size=5)
        a, M = orc.slope(U, lam, K_DOF, b)
        G = BF.MaxwellQuad(U[0], U[1], U[2], lam, K_DOF)
        Mq = G.m5()
        np.testing.assert_allclose(M, Mq, rtol=1e-12, atol=1e-12)
        aq = np.linalg.solve(Mq, b)
        np.testing.assert_allclose(a, aq, rtol=1e-9, atol=1e-10 * np.abs(aq).max())
        np.testing.assert_allclose(Mq @ a, b, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# Time integrals of Eq. (flux) and the linear-in-time fit
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau,delta", [(1e-3, 1e-2), (2e-2, 1e-2), (1e-1, 1e-2), (5e-6, 6.7e-4)])
def test_time_integrals_vs_quad(orc, tau, delta):
    factors = [
        lambda t: 1 - np.exp(-t / tau),
        lambda t: (t + tau) * np.exp(-t / tau) - tau,
        lambda t: t - tau + tau * np.exp(-t / tau),
        lambda t: np.exp(-t / tau),
        lambda t: (t + tau) * np.exp(-t / tau),
        lambda t: tau * np.exp(-t / tau),
    ]
    c = orc.time_integrals(tau, delta)
    for i, f in enumerate(factors):
        ref, _ = integrate.quad(f, 0, delta, epsabs=1e-17, epsrel=1e-13, points=[min(tau, delta / 2)], limit=200)
        assert abs(c[i] - ref) <= 1e-11 * max(abs(ref), delta * tau, 1e-300), (i, c[i], ref)


def test_time_integrals_inviscid_limit(orc):
    d = 0.01
    np.testing.assert_allclose(orc.time_integrals(0.0, d), [d, 0, d * d / 2, 0, 0, 0], atol=0, rtol=0)


# --------------------------------------------------------------------------
# Volume flux, Eq. (flux-2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("low_mach", [False, True])
def test_volume_flux_vs_bruteforce(orc, low_mach):
    rng = np.random.default_rng(3 + low_mach)
    for mu, pr in ((0.0, 1.0), (0.02, 1.0), (1 / 1600, 0.72), (0.3, 0.72)):
        c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=pr)
        for _ in range(3):
            q = IN.point_state(rng, low_mach)
            dq = IN.point_gradient(rng)
            F, Ft = orc.volume_flux(c, q, dq)
            Fb, Ftb = BF.volume_flux(GAMMA, mu, pr, q, dq)
            assert np.abs(F - Fb).max() <= 1e-13 * np.abs(Fb).max()
            assert np.abs(Ft - Ftb).max() <= 1e-12 * np.abs(Ftb).max()


@pytest.mark.parametrize("mu,pr", [(0.0, 1.0), (0.05, 1.0), (0.05, 0.72), (1 / 1600, 0.72)])
def test_volume_flux_recovers_navier_stokes(orc, mu, pr):
    rng = np.random.default_rng(5)
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=pr)
    for lm in (False, True):
        for _ in range(4):
            q = IN.point_state(rng, lm)
            dq = IN.point_gradient(rng)
            F, _ = orc.volume_flux(c, q, dq)
            Fn = BF.ns_flux(GAMMA, mu, pr, q, dq)
            assert np.abs(F - Fn).max() <= 1e-12 * np.abs(Fn).max()


def test_volume_flux_time_derivative_is_euler_jacobian(orc):
    rng = np.random.default_rng(6)
    c = orc.make_cfg((1, 1, 1), 2, mu=0.01, prandtl=0.72)
    for lm in (False, True):
        for _ in range(4):
            q = IN.point_state(rng, lm)
            dq = IN.point_gradient(rng)
            _, Ft = orc.volume_flux(c, q, dq)
            qt = -sum(BF.euler_jvp(q, e, dq[e], GAMMA) for e in range(3))
            for d in range(3):
                ref = BF.euler_jvp(q, d, qt, GAMMA)
                assert np.abs(Ft[d] - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


# --------------------------------------------------------------------------
# Face flux, Eq. (flux) + slopes + time fit
# --------------------------------------------------------------------------
FACE_CASES = [(0.0, 1.0, 1e-2), (1e-6, 1.0, 1e-2), (1e-4, 0.72, 1e-2), (1e-2, 0.72, 1e-2), (0.1, 0.72, 1e-3)]


@pytest.mark.parametrize("mu,pr,dt", FACE_CASES)
def test_face_flux_vs_bruteforce(orc, mu, pr, dt):
    rng = np.random.default_rng(int(1e6 * mu) + 17)
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=pr)
    for d in range(3):
        qL, qR = IN.point_state(rng), IN.point_state(rng)
        dqL, dqR = IN.point_gradient(rng), IN.point_gradient(rng)
        F, Ft = orc.face_flux(c, dt, d, qL, dqL, qR, dqR)
        Fb, Ftb = BF.face_flux(GAMMA, mu, pr, dt, d, qL, dqL, qR, dqR)
        assert np.abs(F - Fb).max() <= 1e-12 * np.abs(Fb).max(), (d, F, Fb)
        assert np.abs(Ft - Ftb).max() <= 1e-10 * np.abs(Ftb).max(), (d, Ft, Ftb)


def test_face_flux_low_mach_vs_bruteforce(orc):
    rng = np.random.default_rng(23)
    mu, pr, dt = 1 / 1600, 0.72, 6.67782e-4
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=pr)
    for d in range(3):
        qL = IN.point_state(rng, True)
        qR = qL + rng.normal(0, 0.01, 5)  # nearly continuous, as in a smooth flow
        dqL, dqR = IN.point_gradient(rng), IN.point_gradient(rng)
        F, Ft = orc.face_flux(c, dt, d, qL, dqL, qR, dqR)
        Fb, Ftb = BF.face_flux(GAMMA, mu, pr, dt, d, qL, dqL, qR, dqR)
        assert np.abs(F - Fb).max() <= 1e-12 * np.abs(Fb).max()
        assert np.abs(Ft - Ftb).max() <= 1e-8 * np.abs(Ftb).max()


@pytest.mark.parametrize("mu", [0.0, 1e-4, 0.05, 2.0])
def test_face_flux_equal_states_is_euler_flux(orc, mu):
    rng = np.random.default_rng(7)
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=0.72)
    z = np.zeros((3, 5))
    for lm in (False, True):
        q = IN.point_state(rng, lm)
        for d in range(3):
            F, Ft = orc.face_flux(c, 1e-2, d, q, z, q, z)
            ref = BF.euler_flux(q, d, GAMMA)
            assert np.abs(F - ref).max() <= 1e-13 * np.abs(ref).max()
            assert np.abs(Ft).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("mu,pr", [(0.0, 1.0), (1e-3, 0.72), (0.05, 0.72)])
def test_face_flux_continuous_data_equals_volume_flux(orc, mu, pr):
    # With q_L = q_R and equal gradients all e^{-t/tau} terms cancel and the
    # face distribution reduces to the volume form g0 (1 - tau (a.u + A) + A t).
    rng = np.random.default_rng(8)
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=pr)
    for lm in (False, True):
        q = IN.point_state(rng, lm)
        dq = IN.point_gradient(rng)
        Fv, Ftv = orc.volume_flux(c, q, dq)
        for d in range(3):
            F, Ft = orc.face_flux(c, 1e-2, d, q, dq, q, dq)
            assert np.abs(F - Fv[d]).max() <= 1e-12 * np.abs(Fv[d]).max()
            assert np.abs(Ft - Ftv[d]).max() <= 2e-9 * np.abs(Ftv[d]).max()


# --------------------------------------------------------------------------
# Grid-level invariants (Section 3 operator, Eq. (two-stage))
# --------------------------------------------------------------------------
def _uniform(orc, cfg, Q):
    q = np.zeros(orc.field_shape(cfg))
    q[:, 0] = np.asarray(Q)[:, None, None, None]
    return q


@pytest.mark.parametrize("k", [1, 2, 3])
def test_free_stream_preservation(orc, k):
    c = orc.make_cfg((4, 3, 5), k, lo=(0, 0, 0), hi=(1, 2, 3), mu=0.01, prandtl=0.72)
    Q = [1.2, 0.3, -0.4, 0.5, 3.0]
    q = _uniform(orc, c, Q)
    L, Lt = orc.residual(c, q, 1e-2)
    # rounding of O(|Q| (2k+1) / dx) volume and face terms that cancel exactly
    tol = 1e-15 * max(abs(v) for v in Q) * orc.nmodes(k) * (2 * k + 1) / (1.0 / 4)
    assert np.abs(L).max() < tol and np.abs(Lt).max() < tol
    q2 = orc.step(c, q, 1e-2, 3)
    assert np.abs(q2 - q).max() < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3])
def test_conservation(orc, k):
    rng = np.random.default_rng(9)
    c = orc.make_cfg((5, 4, 6), k, lo=(0, 0, 0), hi=(1, 1.5, 2), mu=0.01, prandtl=0.72)
    q = IN.random_field(rng, (5, 4, 6), orc.nmodes(k), amp=0.05)
    tot0 = q[:, 0].sum(axis=(1, 2, 3))
    q2 = orc.step(c, q, 2e-3, 3)
    tot1 = q2[:, 0].sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0).max())


def test_s2o4_amplification(orc):
    for z in (-0.3, 0.7, -2.0, 1.1):
        dt = 0.5
        zd = z * dt
        assert abs(orc.s2o4_linear(z, dt, 1) - (1 + zd + zd ** 2 / 2 + zd ** 3 / 6 + zd ** 4 / 24)) < 1e-15


def _order_run(orc, k, N, axis, t_end=0.5, cfl=0.2):
    shape = [1, 1, 1]
    shape[axis] = N
    c = orc.make_cfg(shape, k, lo=(0, 0, 0), hi=(2, 2, 2))
    prob = "advection_" + "xyz"[axis]
    q = orc.project(c, prob)
    amax = 1.0 + np.sqrt(GAMMA / 0.8)
    n = int(np.ceil(t_end / (cfl * (2.0 / N) / amax)))
    q = orc.step(c, q, t_end / n, n)
    return orc.advection_error(c, q, t_end, prob)


@pytest.mark.parametrize("k,axis", [(1, 0), (2, 0), (2, 1), (2, 2), (3, 0), (3, 2)])
def test_convergence_order_1d_advection(orc, k, axis):
    # exact solution rho = 1 + 0.2 sin(pi (x - t)), Section 5.1 in one axis;
    # P3 needs the smaller CFL number (the DG limit falls like 1 / (2k + 1))
    cfl = 0.2 if k < 3 else 0.1
    e = [_order_run(orc, k, N, axis, cfl=cfl) for N in (8, 16, 32)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(orders - (k + 1)) < 0.3), orders


def test_convergence_order_3d_advection(orc):
    # Section 5.1 3-D problem, rho = 1 + 0.2 sin(pi (x + y + z - 3 t)), P2
    errs = []
    for N in (4, 8):
        c = orc.make_cfg((N, N, N), 2, lo=(0, 0, 0), hi=(2, 2, 2))
        q = orc.project(c, "advection")
        amax = 1.0 + np.sqrt(GAMMA / 0.8)
        n = int(np.ceil(0.25 / (0.2 * (2.0 / N) / amax)))
        q = orc.step(c, q, 0.25 / n, n)
        errs.append(orc.advection_error(c, q, 0.25))
    assert abs(np.log2(errs[0] / errs[1]) - 3.0) < 0.3


def test_tgv_initial_kinetic_energy(orc):
    c = orc.make_cfg((16, 16, 16), 2, lo=(-np.pi,) * 3, hi=(np.pi,) * 3)
    q = orc.project(c, "tgv")
    Ek = orc.kinetic_energy(c, q) / (2 * np.pi) ** 3
    assert abs(Ek - 0.125) < 1e-4


def test_tgv_initial_kinetic_energy_converges_to_closed_form(orc):
    """E_k of the Taylor-Green initial field (rho = 1) is pi^3 on [-pi, pi]^3;
    the L^2-projected P2 field converges to it at high order."""
    errs = []
    for n in (8, 16):
        c = orc.make_cfg((n, n, n), 2, lo=(-np.pi,) * 3, hi=(np.pi,) * 3)
        errs.append(abs(orc.kinetic_energy(c, orc.project(c, "tgv")) - np.pi ** 3))
    assert errs[1] < 1e-3 and errs[0] / errs[1] > 16


def test_tgv_initial_enstrophy_converges_to_closed_form(orc):
    """curl U of the Taylor-Green initial field is (-cos x sin y sin z,
    -sin x cos y sin z, 2 sin x sin y cos z), so int |curl U|^2 / 2 = 3 pi^3;
    the P2 gradients converge at second order."""
    errs = []
    for n in (8, 16, 32):
        c = orc.make_cfg((n, n, n), 2, lo=(-np.pi,) * 3, hi=(np.pi,) * 3)
        errs.append(abs(orc.enstrophy(c, orc.project(c, "tgv")) - 3 * np.pi ** 3))
    assert errs[2] < 0.2 and errs[0] / errs[1] > 2 and errs[1] / errs[2] > 3


def _linear_field(orc, shape, k, lo, hi, rho, grad_u):
    """Modal coefficients of rho = const and rho U = rho (grad_u @ x), which
    every P_k (k >= 1) represents exactly: per cell, mode 0 holds the value at
    the centre and mode e_d (P_1 along axis d) half the cell width times the
    slope along d."""
    nm = orc.nmodes(k)
    modes = orc.modes(k)
    q = np.zeros((5, nm) + tuple(reversed(shape)))
    dx = [(hi[d] - lo[d]) / shape[d] for d in range(3)]
    xc = [lo[d] + (np.arange(shape[d]) + 0.5) * dx[d] for d in range(3)]
    Z, Y, X = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    centre = [X, Y, Z]
    unit = {tuple(int(d == e) for d in range(3)): e for e in range(3)}
    n_of = {tuple(m): i for i, m in enumerate(modes)}
    q[0, 0] = rho
    q[4, 0] = 10.0
    for j in range(3):
        q[1 + j, 0] = rho * sum(grad_u[j][e] * centre[e] for e in range(3))
        for e_vec, e in unit.items():
            q[1 + j, n_of[e_vec]] = rho * grad_u[j][e] * dx[e] / 2
    return q


def test_enstrophy_and_kinetic_energy_of_linear_fields_exact(orc):
    """Constant rho and U = A x: curl U = (A32 - A23, A13 - A31, A21 - A12),
    so the enstrophy is |curl U|^2 V / 2 exactly; the kinetic energy
    rho int |A x|^2 / 2 over the box is a quadratic the 3-point rule
    integrates exactly."""
    lo, hi, shape, rho = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0), (3, 4, 2), 1.7
    A = np.array([[0.0, -0.8, 0.3], [0.8, 0.1, 0.0], [0.0, 0.45, -0.2]])
    q = _linear_field(orc, shape, 2, lo, hi, rho, A)
    c = orc.make_cfg(shape, 2, lo=lo, hi=hi)
    V = np.prod(np.subtract(hi, lo))
    w = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    assert abs(orc.enstrophy(c, q) - 0.5 * w @ w * V) < 1e-12 * V
    # int x_a x_b over the box
    m1 = [(hi[d] ** 2 - lo[d] ** 2) / 2 for d in range(3)]
    m2 = [(hi[d] ** 3 - lo[d] ** 3) / 3 for d in range(3)]
    L = [hi[d] - lo[d] for d in range(3)]
    Mx = np.empty((3, 3))
    for a in range(3):
        for b in range(3):
            if a == b:
                Mx[a, b] = m2[a] * np.prod([L[d] for d in range(3) if d != a])
            else:
                Mx[a, b] = m1[a] * m1[b] * np.prod([L[d] for d in range(3) if d not in (a, b)])
    ek = 0.5 * rho * np.trace(A @ Mx @ A.T)
    assert abs(orc.kinetic_energy(c, q) - ek) < 1e-12 * abs(ek)


def test_projection_cell_average(orc):
    c = orc.make_cfg((3, 3, 3), 2, lo=(-np.pi,) * 3, hi=(np.pi,) * 3)
    q = orc.project(c, "tgv")
    dx = 2 * np.pi / 3
    i, j, k = 1, 2, 0
    x0, y0, z0 = -np.pi + i * dx, -np.pi + j * dx, -np.pi + k * dx
    f = lambda z, y, x: np.sin(x) * np.cos(y) * np.cos(z)
    ref, _ = integrate.tplquad(f, x0, x0 + dx, y0, y0 + dx, z0, z0 + dx, epsabs=1e-13)
    assert abs(q[1, 0, k, j, i] - ref / dx ** 3) < 1e-9


def _swap_xy(orc, q, k):
    md = orc.modes(k).tolist()
    perm = [md.index([m[1], m[0], m[2]]) for m in md]
    out = q[:, perm].transpose(0, 1, 2, 4, 3).copy()
    out[[1, 2]] = out[[2, 1]]
    return out


def test_axis_permutation_symmetry(orc):
    rng = np.random.default_rng(12)
    k = 2
    c = orc.make_cfg((4, 4, 3), k, lo=(0, 0, 0), hi=(1, 1, 0.8), mu=0.01, prandtl=0.72)
    q = IN.random_field(rng, (4, 4, 3), orc.nmodes(k), amp=0.05)
    L, Lt = orc.residual(c, q, 1e-2)
    Ls, Lts = orc.residual(c, _swap_xy(orc, q, k), 1e-2)
    assert np.abs(Ls - _swap_xy(orc, L, k)).max() <= 1e-12 * np.abs(L).max()
    assert np.abs(Lts - _swap_xy(orc, Lt, k)).max() <= 1e-12 * np.abs(Lt).max()


def test_residual_cells_and_slab_match_full_grid(orc):
    rng = np.random.default_rng(13)
    c = orc.make_cfg((5, 4, 6), 2, lo=(0, 0, 0), hi=(1, 1, 1), mu=0.01, prandtl=0.72)
    q = IN.random_field(rng, (5, 4, 6), 10)
    L, Lt = orc.residual(c, q, 1e-2)
    cells = [0, 7, 19, 119, 60]
    Lc, Ltc = orc.residual_cells(c, q, 1e-2, cells)
    Lf = L.reshape(5, 10, -1)
    Ltf = Lt.reshape(5, 10, -1)
    for t, cc in enumerate(cells):
        assert np.array_equal(Lc[t], Lf[:, :, cc])
        assert np.array_equal(Ltc[t], Ltf[:, :, cc])
    Ls, Lts = orc.residual_slab(c, q, 1e-2, 2, 4)
    n = 5 * 4
    assert np.array_equal(Ls, Lf[:, :, 2 * n:4 * n].transpose(2, 0, 1))
    assert np.array_equal(Lts, Ltf[:, :, 2 * n:4 * n].transpose(2, 0, 1))


def test_step_cells_matches_full_grid_step(orc):
    """The sampled one-step oracle (stage 1 on the listed cells and their face
    neighbours, stage 2 on the listed cells) equals the full-grid S2O4 step
    of Eq. (two-stage) at those cells, bit for bit; corner and edge cells
    exercise the periodic wrap."""
    rng = np.random.default_rng(21)
    shape = (5, 4, 6)
    c = orc.make_cfg(shape, 2, lo=(0, 0, 0), hi=(1, 1.1, 0.9), mu=0.01, prandtl=0.72)
    q = IN.random_field(rng, shape, 10)
    dt = 2e-3
    full = orc.step(c, q, dt, 1).reshape(5, 10, -1)
    cells = [0, 4, 19, 60, 119, 77]
    got = orc.step_cells(c, q, dt, cells)
    for t, cc in enumerate(cells):
        assert np.array_equal(got[t], full[:, :, cc])


def test_advection_error_norm_closed_forms(orc):
    """The Section 5.1 error norm sqrt(int (rho_h - rho_exact)^2 dV) against
    closed forms on [0,2]^3: rho_h = 0 gives sqrt(8 + 0.04 * 4) (the sine
    squared averages 1/2 over whole periods), rho_h = 1 gives 0.4; and the
    exact solution moves at speed 3 along the diagonal: the projection of the
    t = 0 state has its own small error at t = 2/3 (one period later) and
    ||2 * 0.2 sin|| = 0.8 at t = 1/3 (half a period)."""
    N = 8
    c = orc.make_cfg((N, N, N), 2, lo=(0, 0, 0), hi=(2, 2, 2))
    q = np.zeros(orc.field_shape(c))
    assert abs(orc.advection_error(c, q, 0.3) - np.sqrt(8.16)) <= 1e-9
    q[0, 0] = 1.0
    assert abs(orc.advection_error(c, q, 0.7) - 0.4) <= 1e-9
    assert abs(orc.advection_error(c, q, 0.2, "advection_y") - 0.4) <= 1e-9
    qp = orc.project(c, "advection")
    e0 = orc.advection_error(c, qp, 0.0)
    assert e0 < 1e-2
    assert abs(orc.advection_error(c, qp, 2.0 / 3.0) - e0) <= 1e-12
    assert abs(orc.advection_error(c, qp, 1.0 / 3.0) - 0.8) <= 2 * e0


# --------------------------------------------------------------------------
# Forward-mode dual numbers (the oracle gradient) against central differences
# --------------------------------------------------------------------------
def test_dual_point_fluxes_vs_central_differences(orc):
    rng = np.random.default_rng(14)
    mu = 0.01
    c = orc.make_cfg((1, 1, 1), 2, mu=mu, prandtl=0.72)
    q, dq = IN.point_state(rng), IN.point_gradient(rng)
    tq, tdq, tmu = rng.normal(size=5), rng.normal(size=(3, 5)), 0.3
    F, dF, Ft, dFt = orc.volume_flux_jvp(c, q, dq, tq, tdq, tmu)
    h = 1e-6
    cp = orc.make_cfg((1, 1, 1), 2, mu=mu + h * tmu, prandtl=0.72)
    cm = orc.make_cfg((1, 1, 1), 2, mu=mu - h * tmu, prandtl=0.72)
    Fp, Ftp = orc.volume_flux(cp, q + h * tq, dq + h * tdq)
    Fm, Ftm = orc.volume_flux(cm, q - h * tq, dq - h * tdq)
    np.testing.assert_allclose(dF, (Fp - Fm) / (2 * h), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(dFt, (Ftp - Ftm) / (2 * h), rtol=1e-6, atol=1e-7)
    x = np.concatenate([IN.point_state(rng), IN.point_gradient(rng).ravel(), IN.point_state(rng),
                        IN.point_gradient(rng).ravel()])
    tx = rng.normal(size=40)
    dt = 1e-2
    for d in range(3):
        F, dF, Ft, dFt = orc.face_flux_jvp(c, dt, d, x, tx, tmu)
        xp, xm = x + h * tx, x - h * tx
        Fp, Ftp = orc.face_flux(cp, dt, d, xp[:5], xp[5:20], xp[20:25], xp[25:])
        Fm, Ftm = orc.face_flux(cm, dt, d, xm[:5], xm[5:20], xm[20:25], xm[25:])
        np.testing.assert_allclose(dF, (Fp - Fm) / (2 * h), rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(dFt, (Ftp - Ftm) / (2 * h), rtol=1e-5, atol=1e-5)


def test_dual_step_and_energy_vs_central_differences(orc):
    rng = np.random.default_rng(15)
    mu = 0.01
    shape = (4, 3, 3)
    mk = lambda m: orc.make_cfg(shape, 1, lo=(0, 0, 0), hi=(1, 1, 1), mu=m, prandtl=0.72)
    c = mk(mu)
    q = IN.random_field(rng, shape, orc.nmodes(1), amp=0.05)
    v = IN.random_direction(rng, q) * 1e-2
    dt, n = 2e-3, 2
    # direction in the coefficients (h = 1e-3) and in mu (h = 1e-6): the
    # step sizes keep truncation and round-off of the differences below 1e-8
    for tmu, vv, h in ((0.0, v, 1e-3), (0.5, 0 * v, 1e-6)):
        qN, dqN = orc.step_jvp(c, q, vv, tmu, dt, n)
        assert np.array_equal(qN, orc.step(c, q, dt, n))
        J, dJ = orc.ke_jvp(c, qN, dqN)
        assert abs(J - orc.kinetic_energy(c, qN)) <= 1e-15 * abs(J)
        Jp = orc.kinetic_energy(c, orc.step(mk(mu + h * tmu), q + h * vv, dt, n))
        Jm = orc.kinetic_energy(c, orc.step(mk(mu - h * tmu), q - h * vv, dt, n))
        assert abs(dJ - (Jp - Jm) / (2 * h)) <= 1e-8 * abs(dJ)


# ---------------------------------------------------------------------------
# separable non-uniform meshes (Section 5.1 mapped meshes)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 3])
def test_nonuniform_free_stream_and_conservation(orc, k):
    rng = np.random.default_rng(30 + k)
    shape, lo, hi = (5, 3, 4), (0.0, 0.0, 0.0), (1.0, 2.0, 3.0)
    w = IN.random_widths(rng, shape, lo, hi)
    c = orc.make_cfg(shape, k, lo=lo, hi=hi, mu=0.01, prandtl=0.72, widths=w)
    Q = [1.2, 0.3, -0.4, 0.5, 3.0]
    q = _uniform(orc, c, Q)
    L, Lt = orc.residual(c, q, 1e-2)
    tol = 1e-15 * max(abs(v) for v in Q) * orc.nmodes(k) * (2 * k + 1) / w.min()
    assert np.abs(L).max() < tol and np.abs(Lt).max() < tol
    # conservation: the integral of each variable is sum_K |K| Q_0(K)
    q = IN.random_field(rng, shape, orc.nmodes(k), amp=0.05)
    nx, ny = shape[0], shape[1]
    vol = w[nx + ny:][:, None, None] * w[nx:nx + ny][None, :, None] * w[:nx][None, None, :]
    tot0 = (q[:, 0] * vol).sum(axis=(1, 2, 3))
    q2 = orc.step(c, q, 2e-3, 3)
    tot1 = (q2[:, 0] * vol).sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0).max())


def test_nonuniform_equal_widths_reproduce_uniform_mesh(orc):
    rng = np.random.default_rng(41)
    shape, lo, hi = (4, 3, 5), (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
    w = np.concatenate([np.full(n, (hi[e] - lo[e]) / n) for e, n in enumerate(shape)])
    q = IN.random_field(rng, shape, 10, amp=0.05)
    a = orc.residual(orc.make_cfg(shape, 2, lo=lo, hi=hi, mu=0.01, prandtl=0.72), q, 1e-2)
    b = orc.residual(orc.make_cfg(shape, 2, lo=lo, hi=hi, mu=0.01, prandtl=0.72, widths=w), q, 1e-2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_nonuniform_transverse_widths_do_not_change_a_one_dimensional_flow(orc):
    """A field that varies along x only has equal states on both faces of
    every y and z face pair, whose terms then cancel whatever the y and z
    widths: the residual is that of the 1-D grid.  A width taken from the
    wrong axis (normal derivative, face area, mass matrix) breaks this."""
    rng = np.random.default_rng(42)
    nx, lo, hi = 6, (0.0, 0.0, 0.0), (2.0, 1.0, 1.5)
    wx = IN.random_widths(rng, (nx,), lo[:1], hi[:1])
    q1 = IN.random_field(rng, (nx, 1, 1), 10, amp=0.05)
    # keep only modes constant in y and z (e_y = e_z = 0): modes 0, 1 (x), 4 (x^2) of P2
    md = orc.modes(2)
    keep = [n for n in range(10) if md[n][1] == 0 and md[n][2] == 0]
    q1[:, [n for n in range(10) if n not in keep]] = 0.0
    c1 = orc.make_cfg((nx, 1, 1), 2, lo=lo, hi=hi, mu=0.01, prandtl=0.72,
                      widths=np.concatenate([wx, [1.0], [1.5]]))
    L1, Lt1 = orc.residual(c1, q1, 1e-2)
    shape = (nx, 3, 4)
    w = np.concatenate([wx, IN.random_widths(rng, (3, 4), lo[1:], hi[1:])])
    c3 = orc.make_cfg(shape, 2, lo=lo, hi=hi, mu=0.01, prandtl=0.72, widths=w)
    q3 = np.broadcast_to(q1, (5, 10, 4, 3, nx)).copy()
    L3, Lt3 = orc.residual(c3, q3, 1e-2)
    for L, ref in ((L3, L1), (Lt3, Lt1)):
        scale = np.abs(ref).max()
        assert np.abs(L - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("k,axis", [(2, 0), (3, 1)])
def test_nonuniform_convergence_order_1d(orc, k, axis):
    """Section 5.1 mapped mesh x = xi + 0.05 sin(pi xi) along the flow: order k + 1."""
    e = []
    for N in (8, 16, 32):
        shape = [1, 1, 1]
        shape[axis] = N
        ws = [np.array([2.0])] * 3
        ws[axis] = IN.mapped_widths(N)
        c = orc.make_cfg(shape, k, lo=(0, 0, 0), hi=(2, 2, 2), widths=np.concatenate(ws))
        prob = "advection_" + "xyz"[axis]
        q = orc.project(c, prob)
        amax = 1.0 + np.sqrt(GAMMA / 0.8)
        n = int(np.ceil(0.5 / (0.1 * ws[axis].min() / amax)))
        q = orc.step(c, q, 0.5 / n, n)
        e.append(orc.advection_error(c, q, 0.5, prob))
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(orders - (k + 1)) < 0.3), orders


def test_mapped_mesh_error_ratio_matches_paper_tables(orc):
    """3-D advection, P2 with the paper's 2 Gauss points per direction, 8^3:
    the L2 error on the mapped mesh over the error on the uniform mesh.  The
    paper's tables of the 3-D P2 accuracy test give 1.6035e-2 (mapped) and
    1.4834e-2 (uniform; printed as 1.4834e-3, read as e-2 since the printed
    order 3.6965 to the 16^3 value 1.1441e-3 requires it): a ratio of 1.081.
    The final time is not stated with the tables, so the ratio (insensitive
    to it) is compared, within 3%."""
    errs = []
    for w in (None, np.tile(IN.mapped_widths(8), 3)):
        c = orc.make_cfg((8, 8, 8), 2, nq=2, lo=(0, 0, 0), hi=(2, 2, 2), widths=w)
        q = orc.project(c, "advection")
        dxm = 0.25 if w is None else w.min()
        n = int(np.ceil(0.5 / (0.1 * dxm / (1.0 + np.sqrt(GAMMA / 0.8)))))
        q = orc.step(c, q, 0.5 / n, n)
        errs.append(orc.advection_error(c, q, 0.5))
    ratio = errs[1] / errs[0]
    assert abs(ratio / (1.6035e-2 / 1.4834e-2) - 1.0) < 0.03, ratio
