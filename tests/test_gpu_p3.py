"""Degree-3 (P3) DG-HGKS on the GPU path against the FP64 oracle.

Both compiled P3 rules: 4 Gauss points per direction (exact mass matrix and
the usual k+1 rule) and 3 points per direction (the reduced rule the paper
uses for P2 carried one degree up).  Same bars as the P2 parity tests:
FP64 relative L2 <= 1e-11 for one operator evaluation and <= 1e-10 over a
few steps; FP32-bulk within its stated tolerance; P3 advection converges at
order ~4 on the GPU as the oracle does (CFL 0.1: the DG stability limit falls
like 1 / (2k + 1)); the adjoint matches the oracle's dual numbers.
"""
import math

import numpy as np
import pytest
import torch

import inputs as IN
import oracle as O
from gpu_util import pair, rel_l2, rel_l2_groups, say, to_dev, to_np
from paper_2202_13821_amd import kinetic_energy, problems as P

pytestmark = pytest.mark.gpu

NM3 = P.nmodes(3)
LO, HI = (0.0, 0.0, 0.0), (1.0, 1.3, 0.7)


@pytest.mark.parametrize("nq", [4, 3])
@pytest.mark.parametrize("shape,mu,pr", [((5, 4, 3), 0.01, 0.72), ((3, 1, 2), 0.0, 1.0), ((67, 2, 1), 0.02, 0.72)])
def test_p3_residual_fp64(nq, shape, mu, pr):
    say("p3 residual fp64", nq, shape, mu)
    rng = np.random.default_rng(800 + nq)
    q = IN.random_field(rng, shape, NM3, amp=0.03)
    s, c = pair(shape, 3, LO, HI, nq=nq, mu=mu, pr=pr)
    L, Lt = s.residual(to_dev(q), 3e-3)
    Lo, Lto = O.residual(c, q, 3e-3)
    eL, eLt = rel_l2_groups(to_np(L), Lo), rel_l2_groups(to_np(Lt), Lto)
    say("  rel L2 of L, Lt:", eL, eLt)
    assert eL <= 1e-11 and eLt <= 1e-10
    s.check()


@pytest.mark.parametrize("nq", [4, 3])
def test_p3_residual_fp32_bulk(nq):
    say("p3 residual fp32", nq)
    rng = np.random.default_rng(810 + nq)
    shape = (6, 5, 4)
    q = IN.random_field(rng, shape, NM3, amp=0.03)
    s, c = pair(shape, 3, LO, HI, nq=nq, mu=0.01, pr=0.72, precision="fp32_bulk")
    L, Lt = s.residual(to_dev(q), 3e-3)
    Lo, Lto = O.residual(c, q, 3e-3)
    eL, eLt = rel_l2_groups(to_np(L), Lo), rel_l2_groups(to_np(Lt), Lto)
    say("  rel L2 of L, Lt:", eL, eLt)
    assert eL <= 1e-4 and eLt <= 1e-3


@pytest.mark.parametrize("nq", [4, 3])
@pytest.mark.parametrize("precision,tol,told", [("fp64", 1e-10, 1e-9), ("fp32_bulk", 1e-5, 5e-2)])
def test_p3_steps_ragged(nq, precision, tol, told):
    say("p3 steps", precision, nq)
    rng = np.random.default_rng(820 + nq)
    shape = (7, 3, 5)
    q0 = IN.random_field(rng, shape, NM3, amp=0.03)
    s, c = pair(shape, 3, LO, HI, nq=nq, mu=0.005, pr=0.72, precision=precision)
    q = to_dev(q0)
    s.step(q, 1e-3, 2)
    qo = O.step(c, q0, 1e-3, 2)
    e, ed = rel_l2(to_np(q), qo), rel_l2(to_np(q) - q0, qo - q0)
    say("  rel L2 of q, of q - q0:", e, ed)
    assert e <= tol and ed <= told
    s.check()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32_bulk", 1e-5)])
def test_p3_tgv_8(precision, tol):
    say("p3 tgv8", precision)
    shape = (8, 8, 8)
    q0, lo, hi = P.tgv(shape, 3)
    s, c = pair(shape, 3, lo, hi, mu=1 / 1600, pr=0.72, precision=precision)
    dt = P.tgv_dt(8, cfl=0.08)
    q = to_dev(q0)
    s.step(q, dt, 2)
    qo = O.step(c, q0, dt, 2)
    e, ed = rel_l2_groups(to_np(q), qo), rel_l2_groups(to_np(q) - q0, qo - q0)
    say("  rel L2 of q, of q - q0:", e, ed)
    assert e <= tol
    assert ed <= (1e-9 if precision == "fp64" else 5e-2)
    s.check()


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_p3_conservation_and_free_stream(precision):
    say("p3 conservation", precision)
    rng = np.random.default_rng(830)
    shape = (6, 5, 4)
    q0 = IN.random_field(rng, shape, NM3, amp=0.03)
    s, _ = pair(shape, 3, (0, 0, 0), (1, 1, 1), mu=0.01, pr=0.72, precision=precision)
    q = to_dev(q0)
    s.step(q, 1e-3, 4)
    tot0 = q0[:, 0].sum(axis=(1, 2, 3))
    tot1 = to_np(q)[:, 0].sum(axis=(1, 2, 3))
    tol = 1e-13 if precision == "fp64" else 1e-7
    assert np.all(np.abs(tot1 - tot0) <= tol * np.abs(tot0).max())
    qu = np.zeros_like(q0)
    qu[:, 0] = np.array([1.1, 0.2, -0.3, 0.4, 2.9])[:, None, None, None]
    q = to_dev(qu)
    s.step(q, 1e-3, 4)
    assert np.abs(to_np(q) - qu).max() <= (1e-12 if precision == "fp64" else 1e-6)


def test_p3_convergence_order():
    """Section 5.1 3-D advection to t = 0.5 with P3 (4 points): order ~ 4."""
    say("order p3")
    errs = []
    for n in (4, 8, 16):
        q0, lo, hi = P.advection((n, n, n), 3)
        s, c = pair((n, n, n), 3, lo, hi)
        dt0 = P.advection_dt(n)
        nst = int(math.ceil(0.5 / dt0))
        q = to_dev(q0)
        s.step(q, 0.5 / nst, nst)
        errs.append(O.advection_error(c, to_np(q), 0.5))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    say("errors", errs, "orders", orders)
    assert orders[-1] > 3.6 and np.all(orders > 3.3)


@pytest.mark.parametrize("nq", [4, 3])
def test_p3_adjoint_vs_oracle_dual_fp64(nq):
    say("p3 adjoint", nq)
    rng = np.random.default_rng(840 + nq)
    shape, n, stride = (3, 4, 2), 3, 2
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.2, 0.9)
    q0 = IN.random_field(rng, shape, NM3, amp=0.04)
    mu, dt = 0.02, 1e-3
    s, c = pair(shape, 3, lo, hi, nq=nq, mu=mu, pr=0.72, max_stride=stride)
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


def test_p3_adjoint_fp32_bulk_vs_fp64():
    say("p3 adjoint fp32")
    rng = np.random.default_rng(850)
    shape, n, stride = (6, 5, 4), 4, 2
    q0 = IN.random_field(rng, shape, NM3, amp=0.04)
    out = {}
    for prec in ("fp64", "fp32_bulk"):
        s, _ = pair(shape, 3, (0, 0, 0), (1, 1, 1), mu=0.01, pr=0.72, precision=prec, max_stride=stride)
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
    # the bar of the P2 FP32-bulk adjoint (float32 VJPs, FP64 accumulation)
    assert e <= 1e-3 and emu <= 1e-3
