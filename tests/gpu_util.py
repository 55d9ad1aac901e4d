"""Helpers shared by the GPU tests (no method arithmetic)."""
import numpy as np
import torch

import oracle as O
from paper_2202_13821_amd import Solver


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    """max over variables of ||a - b|| / ||b|| (plain coefficient norm)."""
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    return max(np.linalg.norm(a[v] - b[v]) / max(np.linalg.norm(b[v]), 1e-300) for v in range(5))


def rel_l2_groups(a, b):
    """max over (rho, momentum vector, rho E) of ||a - b|| / ||b||: the error
    measure stated for both precisions (momentum is normed as one vector so a
    component that is small in the flow, e.g. rho W of the Taylor-Green
    vortex, is measured against the momentum scale)."""
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    out = []
    for grp in ((0,), (1, 2, 3), (4,)):
        out.append(np.linalg.norm(a[list(grp)] - b[list(grp)]) / max(np.linalg.norm(b[list(grp)]), 1e-300))
    return max(out)


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def pair(shape, k, lo, hi, nq=0, mu=0.0, pr=1.0, gamma=1.4, precision="fp64", max_stride=0, widths=None):
    s = Solver(shape, lo, hi, k, nq=nq, gamma=gamma, mu=mu, prandtl=pr, precision=precision, device="cuda:0",
               max_stride=max_stride, widths=widths)
    c = O.make_cfg(shape, k, nq=nq or k + 1, lo=lo, hi=hi, gamma=gamma, mu=mu, prandtl=pr, widths=widths)
    return s, c


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
