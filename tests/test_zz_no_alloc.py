"""The allocation-free step (dg_hgks_step_noalloc: static device scratch, no
context, no workspace) against dg_hgks_step on the same inputs: the same
kernels in the same launch configuration, so the results agree bit for bit.
Two calls in a row, the second on a smaller grid (the scratch keeps the first
call's contents), in both precisions."""
import numpy as np
import pytest
import torch

import inputs as IN
from gpu_util import say, to_dev
from paper_2202_13821_amd import DGHGKSError, Solver, problems as P, step_noalloc

pytestmark = pytest.mark.gpu


def _cases():
    # 32^3 P2 Taylor-Green (the largest grid whose FP64 buffers fit the
    # 96 MiB scratch), then a random 7 x 5 x 4 field with another viscosity
    q0, lo, hi = P.tgv((32, 32, 32), 2)
    yield (32, 32, 32), q0, lo, hi, 1 / 1600, 0.72, P.tgv_dt(32), 3
    rng = np.random.default_rng(1234)
    q1 = IN.random_field(rng, (7, 5, 4), 10, amp=0.03)
    yield (7, 5, 4), q1, (0.0, 0.0, 0.0), (1.0, 0.8, 0.6), 0.02, 1.0, 2e-3, 2


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_noalloc_step_matches_workspace_step(precision):
    for shape, q0, lo, hi, mu, pr, dt, n in _cases():
        say(f"no-alloc step {precision} {shape}, {n} steps")
        s = Solver(shape, lo, hi, 2, mu=mu, prandtl=pr, precision=precision, device="cuda:0")
        qa = to_dev(q0)
        s.step(qa, dt, n)
        s.check()
        qb = to_dev(q0)
        flag = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        step_noalloc(qb, dt, n, shape, lo, hi, 2, mu=mu, prandtl=pr, precision=precision, nonphys=flag)
        torch.cuda.synchronize()
        assert flag.item() == 0
        assert torch.equal(qa, qb)
        del s


def test_noalloc_step_rejects_grids_beyond_its_scratch():
    q = torch.zeros((5, 10, 64, 64, 64), dtype=torch.float64, device="cuda:0")
    with pytest.raises(DGHGKSError, match="scratch"):
        step_noalloc(q, 1e-3, 1, (64, 64, 64), (0, 0, 0), (1, 1, 1), 2)


@pytest.mark.parametrize("k,nq", [(1, 2), (3, 4), (3, 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_noalloc_step_other_rules(precision, k, nq):
    """P1 and P3 (FP64 P3 also uses the L_t buffer of the two-launch stage-1
    pass, placed in the static scratch) on a small ragged grid."""
    shape, lo, hi = (6, 4, 5), (0.0, -0.5, 0.2), (1.0, 1.0, 1.1)
    say(f"no-alloc step {precision} P{k} nq {nq} {shape}")
    rng = np.random.default_rng(4321 + 10 * k + nq)
    q0 = IN.random_field(rng, shape, P.nmodes(k), amp=0.03)
    s = Solver(shape, lo, hi, k, nq=nq, mu=0.01, prandtl=0.72, precision=precision, device="cuda:0")
    qa = to_dev(q0)
    s.step(qa, 2e-3, 2)
    s.check()
    qb = to_dev(q0)
    flag = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    step_noalloc(qb, 2e-3, 2, shape, lo, hi, k, nq=nq, mu=0.01, prandtl=0.72, precision=precision, nonphys=flag)
    torch.cuda.synchronize()
    assert flag.item() == 0
    assert torch.equal(qa, qb)
    del s
