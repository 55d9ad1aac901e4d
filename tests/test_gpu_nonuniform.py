"""Separable non-uniform meshes (Section 5.1 mapped meshes and random cell
widths) on the GPU path against the FP64 oracle: the same bars as on uniform
meshes (FP64 relative L2 <= 1e-11 for one operator evaluation, <= 1e-10 over
a few steps; FP32-bulk stated tolerance; adjoint against the oracle's dual
numbers), plus the convergence order k + 1 on the mapped mesh and the ratio
of mapped-mesh to uniform-mesh errors printed in the paper's 3-D tables."""
import math

import numpy as np
import pytest
import torch

import inputs as IN
import oracle as O
from gpu_util import pair, rel_l2, rel_l2_groups, say, to_dev, to_np
from paper_2202_13821_amd import kinetic_energy, problems as P

pytestmark = pytest.mark.gpu

LO, HI = (0.0, -0.5, 0.2), (1.0, 1.0, 1.1)
AMAX = 1.0 + math.sqrt(1.4 / 0.8)  # max |U_d| + c of the advection problem


@pytest.mark.parametrize("k,nq,shape", [(1, 2, (5, 4, 3)), (2, 3, (7, 5, 6)), (2, 3, (67, 2, 3)), (2, 2, (4, 6, 5)),
                                        (3, 4, (4, 3, 5)), (3, 3, (5, 4, 3))])
def test_nonuniform_residual_fp64(k, nq, shape):
    say("nonuniform residual fp64", k, nq, shape)
    rng = np.random.default_rng(900 + 10 * k + nq)
    w = IN.random_widths(rng, shape, LO, HI)
    q = IN.random_field(rng, shape, P.nmodes(k), amp=0.03)
    s, c = pair(shape, k, LO, HI, nq=nq, mu=0.01, pr=0.72, widths=w)
    L, Lt = s.residual(to_dev(q), 3e-3)
    Lo, Lto = O.residual(c, q, 3e-3)
    eL, eLt = rel_l2_groups(to_np(L), Lo), rel_l2_groups(to_np(Lt), Lto)
    say("  rel L2 of L, Lt:", eL, eLt)
    assert eL <= 1e-11 and eLt <= 1e-10
    s.check()


@pytest.mark.parametrize("k,nq", [(2, 3), (3, 4)])
def test_nonuniform_residual_fp32_bulk(k, nq):
    say("nonuniform residual fp32", k, nq)
    rng = np.random.default_rng(910 + k)
    shape = (6, 5, 4)
    w = IN.random_widths(rng, shape, LO, HI)
    q = IN.random_field(rng, shape, P.nmodes(k), amp=0.03)
    s, c = pair(shape, k, LO, HI, nq=nq, mu=0.01, pr=0.72, precision="fp32_bulk", widths=w)
    L, Lt = s.residual(to_dev(q), 3e-3)
    Lo, Lto = O.residual(c, q, 3e-3)
    eL, eLt = rel_l2_groups(to_np(L), Lo), rel_l2_groups(to_np(Lt), Lto)
    say("  rel L2 of L, Lt:", eL, eLt)
    assert eL <= 1e-4 and eLt <= 1e-3


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("precision,tol,told", [("fp64", 1e-10, 1e-9), ("fp32_bulk", 1e-5, 5e-2)])
def test_nonuniform_steps(precision, tol, told, k):
    """Also P3: the FP64 stage-1 pass then runs as its two launches (L_t pass,
    then F pass and update) on the non-uniform kernels."""
    say("nonuniform steps", precision, "P%d" % k)
    rng = np.random.default_rng(920 + k)
    shape = (7, 3, 5)
    w = IN.random_widths(rng, shape, LO, HI)
    q0 = IN.random_field(rng, shape, P.nmodes(k), amp=0.03)
    s, c = pair(shape, k, LO, HI, mu=0.005, pr=0.72, precision=precision, widths=w)
    q = to_dev(q0)
    s.step(q, 1e-3, 3)
    qo = O.step(c, q0, 1e-3, 3)
    e, ed = rel_l2(to_np(q), qo), rel_l2(to_np(q) - q0, qo - q0)
    say("  rel L2 of q, of q - q0:", e, ed)
    assert e <= tol and ed <= told
    s.check()


def test_nonuniform_free_stream_and_conservation():
    rng = np.random.default_rng(930)
    shape = (6, 5, 4)
    w = IN.random_widths(rng, shape, LO, HI)
    s, _ = pair(shape, 2, LO, HI, mu=0.01, pr=0.72, widths=w)
    q0 = IN.random_field(rng, shape, 10, amp=0.03)
    nx, ny = shape[0], shape[1]
    vol = w[nx + ny:][:, None, None] * w[nx:nx + ny][None, :, None] * w[:nx][None, None, :]
    q = to_dev(q0)
    s.step(q, 1e-3, 4)
    tot0 = (q0[:, 0] * vol).sum(axis=(1, 2, 3))
    tot1 = (to_np(q)[:, 0] * vol).sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0).max())
    qu = np.zeros_like(q0)
    qu[:, 0] = np.array([1.1, 0.2, -0.3, 0.4, 2.9])[:, None, None, None]
    q = to_dev(qu)
    s.step(q, 1e-3, 4)
    assert np.abs(to_np(q) - qu).max() <= 1e-12


@pytest.mark.parametrize("k,nq", [(2, 3), (3, 3), (2, 2)])
def test_nonuniform_adjoint_vs_oracle_dual_fp64(k, nq):
    say("nonuniform adjoint", k, nq)
    rng = np.random.default_rng(940 + k)
    shape, n, stride = (4, 3, 3), 3, 2
    w = IN.random_widths(rng, shape, LO, HI)
    q0 = IN.random_field(rng, shape, P.nmodes(k), amp=0.04)
    mu, dt = 0.02, 1e-3
    s, c = pair(shape, k, LO, HI, nq=nq, mu=mu, pr=0.72, max_stride=stride, widths=w)
    ck = s.new_checkpoints(n, stride)
    q = to_dev(q0)
    s.step(q, dt, n, ck, stride)
    qN = q.detach().clone().requires_grad_(True)
    J = kinetic_energy(qN, s)
    (g,) = torch.autograd.grad(J, qN)
    q0b, mub = s.adjoint(ck, stride, dt, n, g.contiguous())
    q0b = to_np(q0b)
    Jo = O.kinetic_energy(c, O.step(c, q0, dt, n))
    assert abs(J.item() - Jo) <= 1e-12 * abs(Jo)
    for t in range(3):
        v = IN.random_direction(rng, q0)
        qNo, dqN = O.step_jvp(c, q0, v, 0.0, dt, n)
        _, dJ = O.ke_jvp(c, qNo, dqN)
        got = float((q0b * v).sum())
        say("  direction", t, got, dJ)
        assert abs(got - dJ) <= 1e-10 * max(abs(dJ), 1e-12 * np.abs(q0b).sum())
    qNo, dqN = O.step_jvp(c, q0, np.zeros_like(q0), 1.0, dt, n)
    _, dJmu = O.ke_jvp(c, qNo, dqN)
    say("  mu", mub, dJmu)
    assert abs(mub - dJmu) <= 1e-10 * abs(dJmu)


def test_nonuniform_diagnostics():
    rng = np.random.default_rng(950)
    shape = (7, 5, 6)
    w = IN.random_widths(rng, shape, LO, HI)
    q0 = IN.random_field(rng, shape, 10, amp=0.05)
    s, c = pair(shape, 2, LO, HI, widths=w)
    (ek, en), g = s.diagnostics(to_dev(q0), grad=True)
    eko, eno = O.kinetic_energy(c, q0), O.enstrophy(c, q0)
    say(f"  E_k {ek:.15e} oracle {eko:.15e}; enstrophy {en:.15e} oracle {eno:.15e}")
    assert abs(ek - eko) <= 1e-12 * abs(eko)
    assert abs(en - eno) <= 1e-11 * abs(eno)
    g = to_np(g)
    for t in range(3):
        v = IN.random_direction(rng, q0)
        _, dJ = O.ke_jvp(c, q0, v)
        assert abs(float((g * v).sum()) - dJ) <= 1e-11 * max(abs(dJ), 1e-12 * np.abs(g).sum())


def _advection_error(k, nq, n, widths, t_end=0.5):
    shape = (n, n, n)
    q0, lo, hi = P.advection(shape, k, widths=widths)
    s, c = pair(shape, k, lo, hi, nq=nq, widths=widths)
    dxm = 2.0 / n if widths is None else float(np.min(widths))
    nst = int(math.ceil(t_end / (0.1 * dxm / AMAX)))
    q = to_dev(q0)
    s.step(q, t_end / nst, nst)
    s.check()
    return O.advection_error(c, to_np(q), t_end)


@pytest.mark.parametrize("k,nq,ns", [(2, 3, (8, 16, 32)), (2, 2, (8, 16, 32)), (3, 4, (8, 16)), (3, 3, (8, 16))])
def test_mapped_mesh_convergence_order(k, nq, ns):
    """Section 5.1 3-D advection on x = xi + 0.05 sin(pi xi) along every
    axis, to t = 0.5 at CFL 0.1: order k + 1 (pre-asymptotic at the coarsest
    pair; the paper's own orders there are 3.70 for P2 and 4.22 for P3)."""
    say("mapped mesh order", k, nq, ns)
    em = [_advection_error(k, nq, n, np.tile(IN.mapped_widths(n), 3)) for n in ns]
    orders = np.log2(np.array(em[:-1]) / np.array(em[1:]))
    say("  mapped-mesh errors", em, "orders", orders)
    assert np.all(orders > k + 0.7) and abs(orders[-1] - (k + 1)) < 0.45


@pytest.mark.parametrize("k,paper_ratio", [
    # the paper's 3-D tables at 8^3: L2 error on the mapped mesh / uniform mesh
    (2, 1.6035e-2 / 1.4834e-2),
    (3, 1.0100e-3 / 8.9026e-4),
])
def test_mapped_mesh_error_ratio_matches_paper(k, paper_ratio):
    """With the paper's quadrature (k Gauss points per direction), 8^3: the
    mapped/uniform error ratio within 3% of the paper's.  The final time of
    the tables is not stated; the ratio is insensitive to it.  The uniform
    P2 entry is printed as 1.4834e-3 and read as e-2, which its printed
    order 3.6965 requires.  (At 16^3 and finer the paper's P3 ratio falls to
    1.02 and 1.00; ours stays near 1.13, printed here for the record.)"""
    say("mapped mesh ratio", k)
    ratios = []
    for n in (8, 16):
        eu = _advection_error(k, k, n, None)
        em = _advection_error(k, k, n, np.tile(IN.mapped_widths(n), 3))
        ratios.append(em / eu)
    say("  ratios (8^3, 16^3)", ratios, "paper 8^3", paper_ratio)
    assert abs(ratios[0] / paper_ratio - 1.0) < 0.03


def test_nonuniform_adjoint_fp32_bulk_vs_fp64():
    """FP32-bulk adjoint on a random non-uniform mesh against the FP64 adjoint
    (the bar of the uniform-mesh FP32-bulk adjoint)."""
    rng = np.random.default_rng(960)
    shape, n, stride = (6, 5, 4), 4, 2
    w = IN.random_widths(rng, shape, LO, HI)
    q0 = IN.random_field(rng, shape, 10, amp=0.04)
    out = {}
    for prec in ("fp64", "fp32_bulk"):
        s, _ = pair(shape, 2, LO, HI, mu=0.01, pr=0.72, precision=prec, max_stride=stride, widths=w)
        ck = s.new_checkpoints(n, stride)
        q = to_dev(q0)
        s.step(q, 1e-3, n, ck, stride)
        qN = q.detach().clone().requires_grad_(True)
        (g,) = torch.autograd.grad(kinetic_energy(qN, s), qN)
        q0b, mub = s.adjoint(ck, stride, 1e-3, n, g.contiguous())
        out[prec] = (to_np(q0b), mub)
    g32, g64 = out["fp32_bulk"][0], out["fp64"][0]
    e = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    emu = abs(out["fp32_bulk"][1] - out["fp64"][1]) / abs(out["fp64"][1])
    say("  full-gradient rel L2, rel dJ/dmu:", e, emu)
    assert e <= 1e-3 and emu <= 1e-3
