"""The FP64 exp of the face kernels' time coefficients (exp_neg_tab: Cody-Waite
reduction by ln 2, degree-13 Taylor polynomial, scaling by 2^-k), built for
the host from the kernels' own header and compared with exp(-x) evaluated to
40 digits: at most 2 ulp over the whole range of arguments the scheme produces
(x = dt / (2 tau) >= 0), exact at x = 0, and 0 beyond the underflow."""
import os
import random
import subprocess
from decimal import Decimal, getcontext

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_13821_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r'''
#include <cstdio>
#include "gks_point.hpp"
int main() {
  double x;
  while (scanf("%lf", &x) == 1) printf("%a\n", dgk::exp_neg_tab(x, dgk::ExpTabHolder<>::t.c));
  return 0;
}
'''


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("exp")
    src, out = d / "t.hip", d / "t"
    src.write_text(SRC)
    subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, "-o", str(out), str(src)],
                   check=True, capture_output=True)
    return str(out)


def _run(exe, xs):
    r = subprocess.run([exe], input="\n".join(repr(x) for x in xs), capture_output=True, text=True, check=True)
    return [float.fromhex(v) for v in r.stdout.split()]


def test_exp_neg_tab_accuracy(exe):
    rng = random.Random(7)
    xs = [0.0, 1e-300, 1e-17, 1e-8, 0.34657359027997264, 0.34657359027997270, 0.5, 1.0, 2.0, 30.0, 700.0, 708.0]
    xs += [rng.uniform(0.0, 1.0) for _ in range(4000)] + [rng.uniform(0.0, 50.0) for _ in range(4000)]
    xs += [10 ** rng.uniform(-12, 2.8) for _ in range(4000)]
    got = _run(exe, xs)
    getcontext().prec = 40
    worst = 0.0
    for x, g in zip(xs, got):
        ref = float((-Decimal(x)).exp())
        if ref < 2.3e-308:  # subnormal results: absolute check
            assert abs(g - ref) <= 2 * 5e-324
            continue
        ulp = abs(ref) * 2.0 ** -52
        worst = max(worst, abs(g - ref) / ulp)
    assert got[0] == 1.0
    assert worst <= 2.0, worst


def test_exp_neg_tab_underflow(exe):
    got = _run(exe, [746.0, 800.0, 1e4, 1e300, float("inf")])
    assert all(v == 0.0 for v in got)
