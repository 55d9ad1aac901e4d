"""The five benchmark configurations on the GPU path.

C1  P1 advection 8^3, 10 steps         FP64 vs live oracle            <= 1e-10
C2  P2 advection 32^3, 100 steps       FP64 vs oracle golden          <= 1e-10; FP32-bulk stated below
C3  P2 Taylor-Green 64^3               FP64 vs oracle golden (10 steps) <= 1e-10; 200 steps FP32-bulk vs FP64
C4  P2 Taylor-Green 128^3, 100 steps   FP32-bulk vs FP64 (stated), FP64 conservation
C5  adjoint                            tests/test_gpu_adjoint.py

Error measure: max over (rho, momentum vector, rho E) of ||diff|| / ||ref||.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import pair, rel_l2_groups, say, to_dev, to_np
from paper_2202_13821_amd import problems as P

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# stated FP32-bulk tolerances (float32 fluxes/projections, FP64 accumulation)
TOL32 = {"c2": 1e-6, "c3_10": 1e-5, "c3_200": 1e-4, "c4_100": 1e-4}


def _golden(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}.json")) as f:
        return json.load(f)


def _groups_err(sample, ref):
    """sample/ref: (ncells, 5, nmodes)."""
    a = np.transpose(np.asarray(sample), (1, 0, 2)).reshape(5, -1)
    b = np.transpose(np.asarray(ref), (1, 0, 2)).reshape(5, -1)
    return rel_l2_groups(a, b)


def _run(shape, k, problem, precision, mu, pr, dt, steps):
    if problem == "tgv":
        q0, lo, hi = P.tgv(shape, k)
    else:
        q0, lo, hi = P.advection(shape, k)
    s, c = pair(shape, k, lo, hi, mu=mu, pr=pr, precision=precision)
    q = to_dev(q0)
    s.step(q, dt, steps)
    s.check()
    return to_np(q), q0, c


def test_c1_p1_advection_fp64_vs_oracle():
    say("C1")
    q, q0, c = _run((8, 8, 8), 1, "advection", "fp64", 0.0, 1.0, P.advection_dt(8), 10)
    e = rel_l2_groups(q, O.step(c, q0, P.advection_dt(8), 10))
    say("  rel L2", e)
    assert e <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_c2_p2_advection_vs_oracle_golden(precision):
    g = _golden("c2")
    say("C2", precision)
    shape = tuple(g["shape"])
    q, q0, c = _run(shape, 2, "advection", precision, 0.0, 1.0, g["dt"], g["steps"])
    qf = q.reshape(5, 10, -1)
    sample = np.stack([qf[:, :, cc] for cc in g["cells"]])
    e = _groups_err(sample, np.array(g["coeffs"]))
    ss = np.array([(qf[v] ** 2).sum() for v in range(5)])
    ess = np.max(np.abs(ss - np.array(g["sumsq"])) / np.array(g["sumsq"]))
    err_exact = O.advection_error(c, q, g["steps"] * g["dt"])
    say(f"  sampled rel {e:.3e}, sum-of-squares rel {ess:.3e}, rho L2 vs exact {err_exact:.6e} "
        f"(oracle {g['rho_l2_error_vs_exact']:.6e})")
    tol = 1e-10 if precision == "fp64" else TOL32["c2"]
    assert e <= tol and ess <= 2 * tol
    assert abs(err_exact - g["rho_l2_error_vs_exact"]) <= max(tol, 1e-12) * 1e3 * g["rho_l2_error_vs_exact"] + 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_c3_tgv64_first_steps_vs_oracle_golden(precision):
    g = _golden("c3")
    say("C3 golden", precision)
    shape = tuple(g["shape"])
    q, q0, c = _run(shape, 2, "tgv", precision, g["mu"], g["prandtl"], g["dt"], g["steps"])
    qf = q.reshape(5, 10, -1)
    sample = np.stack([qf[:, :, cc] for cc in g["cells"]])
    ref = np.array(g["coeffs"])
    e = _groups_err(sample, ref)
    q0f = q0.reshape(5, 10, -1)
    d0 = np.stack([q0f[:, :, cc] for cc in g["cells"]])
    ed = _groups_err(sample - d0, ref - d0)
    say(f"  sampled rel {e:.3e}, rel of the change since t=0 {ed:.3e}")
    assert e <= (1e-10 if precision == "fp64" else TOL32["c3_10"])
    if precision == "fp64":
        assert ed <= 1e-8


def _fp32_vs_fp64(shape, steps):
    q0, lo, hi = P.tgv(shape, 2)
    dt = P.tgv_dt(shape[0])
    out = {}
    for prec in ("fp64", "fp32_bulk"):
        s, _ = pair(shape, 2, lo, hi, mu=1 / 1600, pr=0.72, precision=prec)
        q = to_dev(q0)
        s.step(q, dt, steps)
        s.check()
        out[prec] = to_np(q)
        del s
    tot0 = q0[:, 0].sum(axis=(1, 2, 3))
    tot64 = out["fp64"][:, 0].sum(axis=(1, 2, 3))
    cons = np.max(np.abs(tot64 - tot0)) / np.abs(tot0).max()
    e = rel_l2_groups(out["fp32_bulk"], out["fp64"])
    ed = rel_l2_groups(out["fp32_bulk"] - q0, out["fp64"] - q0)
    return e, ed, cons


def test_c3_tgv64_200_steps_fp32_bulk_vs_fp64():
    say("C3 200 steps")
    e, ed, cons = _fp32_vs_fp64((64, 64, 64), 200)
    say(f"  FP32-bulk vs FP64 rel {e:.3e} (of the change {ed:.3e}); FP64 conservation {cons:.2e}")
    assert e <= TOL32["c3_200"] and cons <= 1e-13


def test_c4_tgv128_100_steps_fp32_bulk_vs_fp64():
    say("C4 100 steps")
    e, ed, cons = _fp32_vs_fp64((128, 128, 128), 100)
    say(f"  FP32-bulk vs FP64 rel {e:.3e} (of the change {ed:.3e}); FP64 conservation {cons:.2e}")
    assert e <= TOL32["c4_100"] and cons <= 1e-13
