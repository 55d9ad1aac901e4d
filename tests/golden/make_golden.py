"""Write oracle reference results for the multi-step configurations whose
oracle runs take too long for a test (calls only oracle/).

python tests/golden/make_golden.py c2|c3

c2: 3-D density advection (Section 5.1), [0,2]^3, 32^3 cells, P2, 3-point
    Gauss rules, gamma 1.4, inviscid, dt = 0.1 dx / max(|U| + c) = 2.690630e-3,
    100 steps.
c3: Taylor-Green vortex (Section 5.3, rho = 1), [-pi,pi]^3, 64^3 cells, P2,
    3-point rules, Re 1600 (mu = 1/1600), Ma 0.1, Pr 0.72, dt = 0.15 dx /
    max(|U| + c) = 1.335564e-3, first 10 of its 200 steps.

Stored: per-variable sums of squares of the final coefficients, the density L2
error against the exact advection solution (c2), and all coefficients of 48
sampled cells (seeded choice).
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

CASES = {
    "c2": dict(shape=(32, 32, 32), k=2, problem="advection", lo=(0.0,) * 3, hi=(2.0,) * 3, mu=0.0, pr=1.0,
               dt=0.1 * (2.0 / 32) / (1.0 + math.sqrt(1.4 / 0.8)), steps=100),
    "c3": dict(shape=(64, 64, 64), k=2, problem="tgv", lo=(-math.pi,) * 3, hi=(math.pi,) * 3, mu=1 / 1600, pr=0.72,
               dt=0.15 * (2 * math.pi / 64) / (1.0 + math.sqrt(1.4 * (1.0 / (1.4 * 0.01) + 6.0 / 16.0))),
               steps=10),
}


def main(name):
    cs = CASES[name]
    c = O.make_cfg(cs["shape"], cs["k"], lo=cs["lo"], hi=cs["hi"], mu=cs["mu"], prandtl=cs["pr"])
    q0 = O.project(c, cs["problem"])
    t0 = time.time()
    q = q0.copy()
    for s in range(cs["steps"]):
        q = O.step(c, q, cs["dt"], 1)
        print(f"{name}: step {s + 1}/{cs['steps']} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(2022)
    N = int(np.prod(cs["shape"]))
    cells = sorted(set([0, N - 1] + rng.integers(0, N, 46).tolist()))
    qf = q.reshape(5, q.shape[1], -1)
    out = {
        "case": name, "shape": cs["shape"], "k": cs["k"], "problem": cs["problem"], "lo": cs["lo"], "hi": cs["hi"],
        "mu": cs["mu"], "prandtl": cs["pr"], "gamma": 1.4, "dt": cs["dt"], "steps": cs["steps"],
        "sumsq": [float((qf[v] ** 2).sum()) for v in range(5)],
        "cells": cells, "coeffs": [qf[:, :, cc].tolist() for cc in cells],
        "oracle_threads": O.num_threads(), "seconds": time.time() - t0,
    }
    if cs["problem"] == "advection":
        out["rho_l2_error_vs_exact"] = O.advection_error(c, q, cs["steps"] * cs["dt"])
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f)
    print("wrote", name, flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
