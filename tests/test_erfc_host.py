"""The FP32 complementary error function of the face kernels (erfc_gauss in
gks_point.hpp: a fitted polynomial for exp(y^2) erfc(y) times the Gaussian
that the half-space moments compute anyway), built for the host in float from
the kernels' own header and compared with erfc in FP64 over z in [-9, 9]:
relative error a few FP32 ulp where |z| <= 4 (erfc > 1.5e-8), within 5e-6
beyond (where the rounding of z^2 in the float Gaussian dominates), and the
FP64 overload is the library erfc exactly."""
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_13821_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r'''
#include <cmath>
#include <cstdio>
#include "gks_point.hpp"
int main() {
  float z;
  while (scanf("%f", &z) == 1) {
    const float g = expf(-z * z);
    printf("%a %a\n", (double)dgk::erfc_gauss(z, g), dgk::erfc_gauss((double)z, 0.0));
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def values(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("erfc")
    src, exe = d / "t.hip", d / "t"
    src.write_text(SRC)
    subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    z = np.linspace(-9.0, 9.0, 36001).astype(np.float32)
    out = subprocess.run([str(exe)], input="\n".join(f"{float(v):.9g}" for v in z), check=True,
                         capture_output=True, text=True).stdout.split("\n")
    f32, f64 = zip(*[(float.fromhex(a), float.fromhex(b)) for a, b in (ln.split() for ln in out if ln.strip())])
    return z.astype(np.float64), np.array(f32), np.array(f64)


def test_fp32_relative_error(values):
    z, f32, _ = values
    exact = np.array([math.erfc(v) for v in z])
    rel = np.abs(f32 / exact - 1.0)
    assert rel[np.abs(z) <= 4.0].max() < 1e-6
    assert rel.max() < 5e-6


def test_fp32_special_values(values):
    z, f32, _ = values
    assert f32[np.argmin(np.abs(z))] == pytest.approx(1.0, abs=2e-7)  # erfc(0) = 1
    assert np.all(np.diff(f32) <= 0.0)  # erfc is decreasing
    assert np.all((f32 >= 0.0) & (f32 <= 2.0))


def test_fp64_overload_is_the_library_erfc(values):
    z, _, f64 = values
    assert np.array_equal(f64, np.array([math.erfc(v) for v in z]))
