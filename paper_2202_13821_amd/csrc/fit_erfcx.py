"""Coefficients of the FP32 complementary error function of the face kernels
(gks_point.hpp, erfc_gauss): erfcx(y) = exp(y^2) erfc(y) = t h(t) with
t = 1 / (1 + y / 2), h a degree-10 polynomial in t fitted by least squares,
weighted for relative error, to erfcx(y) / t at 6000 Chebyshev nodes of
t in (0, 1].  Prints the coefficients (c_0 first) as float literals and the
largest relative error of t h(t) against erfcx on y in [0, 12] in FP64.

    python -m paper_2202_13821_amd.csrc.fit_erfcx
"""
import numpy as np
from scipy.special import erfcx

P = 0.5
DEGREE = 10
NODES = 6000


def fit():
    k = np.arange(NODES)
    t = 0.5 * (1.0 - np.cos(np.pi * (k + 0.5) / NODES))
    t = t[t > 1e-7]
    y = (1.0 / t - 1.0) / P
    h = erfcx(y) / t
    V = np.vander(t, DEGREE + 1, increasing=True)
    w = 1.0 / h
    c, *_ = np.linalg.lstsq(V * w[:, None], h * w, rcond=None)
    return c


def max_rel_error(c):
    y = np.linspace(0.0, 12.0, 200001)
    t = 1.0 / (1.0 + P * y)
    return float(np.max(np.abs(t * np.polyval(c[::-1], t) / erfcx(y) - 1.0)))


if __name__ == "__main__":
    c = fit()
    print(", ".join(f"{float(np.float32(x)):.9e}f" for x in c))
    print(f"max relative error (FP64 evaluation): {max_rel_error(c):.2e}")
