"""Write oracle reference results for the multi-step configurations whose
oracle runs take too long for a test (calls only oracle/).

python tests/golden/make_golden.py c2 [c4 c3 ...]

c2: 3-D density advection (Section 5.1), [0,2]^3, 32^3 cells, P2, 3-point
    Gauss rules, gamma 1.4, inviscid, dt = 0.1 dx / max(|U| + c) = 2.690630e-3,
    100 steps.
c3: Taylor-Green vortex (Section 5.3, rho = 1), [-pi,pi]^3, 64^3 cells, P2,
    3-point rules, Re 1600 (mu = 1/1600), Ma 0.1, Pr 0.72, dt = 0.15 dx /
    max(|U| + c) = 1.335564e-3, 200 steps.
c4: the same Taylor-Green vortex on 128^3 cells, dt = 6.677819e-4, the first
    10 of its 100 steps (one oracle step takes about ten minutes on eight
    cores).

The initial state is the oracle's own L2 projection.  Stored, at the initial
state and at each checkpoint step: per-variable sums of squares of all
coefficients and of the change since the initial state, and every coefficient
of 64 sampled cells (seeded choice, the first and last cell included).  The
file is rewritten after every checkpoint, so a run cut short still leaves the
checkpoints it reached.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402


def _tgv_dt(n, cfl=0.15, gamma=1.4, mach=0.1):
    # dt = CFL dx / max(|U_d| + c) over the analytic initial data: |U_d| <= 1
    # and the largest pressure is 1/(gamma Ma^2) + 6/16 (rho = 1).
    return cfl * (2 * math.pi / n) / (1.0 + math.sqrt(gamma * (1.0 / (gamma * mach * mach) + 6.0 / 16.0)))


CASES = {
    "c2": dict(shape=(32, 32, 32), k=2, problem="advection", lo=(0.0,) * 3, hi=(2.0,) * 3, mu=0.0, pr=1.0,
               dt=0.1 * (2.0 / 32) / (1.0 + math.sqrt(1.4 / 0.8)), checkpoints=(10, 50, 100)),
    "c3": dict(shape=(64, 64, 64), k=2, problem="tgv", lo=(-math.pi,) * 3, hi=(math.pi,) * 3, mu=1 / 1600, pr=0.72,
               dt=_tgv_dt(64), checkpoints=(10, 50, 100, 150, 200)),
    "c4": dict(shape=(128, 128, 128), k=2, problem="tgv", lo=(-math.pi,) * 3, hi=(math.pi,) * 3, mu=1 / 1600,
               pr=0.72, dt=_tgv_dt(128), checkpoints=(1, 5, 10)),
}
NSAMPLE = 64


def _sample(qf, cells):
    return [qf[:, :, cc].tolist() for cc in cells]


def _sumsq(qf):
    return [float((qf[v] ** 2).sum()) for v in range(5)]


def main(name):
    cs = CASES[name]
    c = O.make_cfg(cs["shape"], cs["k"], lo=cs["lo"], hi=cs["hi"], mu=cs["mu"], prandtl=cs["pr"])
    q0 = O.project(c, cs["problem"])
    N = int(np.prod(cs["shape"]))
    rng = np.random.default_rng(2022)
    cells = sorted(set([0, N - 1] + rng.integers(0, N, NSAMPLE - 2).tolist()))
    q0f = q0.reshape(5, q0.shape[1], -1)
    out = {
        "case": name, "shape": cs["shape"], "k": cs["k"], "problem": cs["problem"], "lo": cs["lo"], "hi": cs["hi"],
        "mu": cs["mu"], "prandtl": cs["pr"], "gamma": 1.4, "dt": cs["dt"],
        "cells": cells, "sumsq0": _sumsq(q0f), "coeffs0": _sample(q0f, cells),
        "checkpoints": [], "oracle_threads": O.num_threads(),
    }
    path = os.path.join(HERE, f"oracle_{name}.json")
    t0 = time.time()
    q = q0
    done = 0
    for target in cs["checkpoints"]:
        for s in range(done, target):
            q = O.step(c, q, cs["dt"], 1)
            print(f"{name}: step {s + 1}/{cs['checkpoints'][-1]} ({time.time() - t0:.0f} s)", flush=True)
        done = target
        qf = q.reshape(5, q.shape[1], -1)
        cp = {"steps": target, "sumsq": _sumsq(qf), "sumsq_inc": _sumsq(qf - q0f), "coeffs": _sample(qf, cells),
              "seconds": time.time() - t0}
        if cs["problem"] == "advection":
            cp["rho_l2_error_vs_exact"] = O.advection_error(c, q, target * cs["dt"])
        out["checkpoints"].append(cp)
        with open(path + ".tmp", "w") as f:
            json.dump(out, f)
        os.replace(path + ".tmp", path)
        print(f"wrote {name} at step {target}", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        main(arg)
