"""Exact rewritings inside the device point fluxes, built for the host in FP64
from the kernels' own header and checked against the forms they replace:

- m5_acc (the m5 moment vector without its three moment matrices) against
  <u^2 psi psi^T> x + <u v psi psi^T> y + <u w psi psi^T> z built from
  mat_H<2>, mat_Gv and mat_Gw;
- hmat_mv_acc<p> (<u^p psi psi^T> x without the matrix, p = 0, 1) against
  mat_H<p> applied by sym_mv_acc;
- prim_grad_dt (primitive gradients and the Euler time derivative in one
  pass) against prim_grad and euler_dt;
- the Solver5 closed form of <a psi> = b against the Maxwellian moment
  matrix H = <psi psi^T> assembled by mat_H<0> from the full-line moments (the
  sum of the two half lines): H S(b) must return b.

Random Maxwellians (both half lines), transverse moments and vectors; the
forms must agree to a few units of FP64 rounding."""
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
#include <random>
#include "gks_point.hpp"
using namespace dgk;

static double rel(const double* a, const double* b, int n) {
  double e = 0, s = 0;
  for (int i = 0; i < n; ++i) { e += (a[i] - b[i]) * (a[i] - b[i]); s += a[i] * a[i]; }
  return std::sqrt(e / (s > 0 ? s : 1));
}

int main() {
  std::mt19937_64 g(11);
  std::uniform_real_distribution<double> U(-1.5, 1.5), Th(0.2, 3.0), R(0.5, 2.0);
  const double K = 2.0, gm1 = 0.4;
  for (int it = 0; it < 4000; ++it) {
    const double Uu = U(g), V = U(g), W = U(g), th = Th(g);
    double M[7];
    mom_half(Uu, th, it % 2 ? 1.0 : -1.0, M);
    const Transverse<double> t(V, W, th, K);
    double x[5], y[5], z[5];
    for (int k = 0; k < 5; ++k) { x[k] = U(g); y[k] = U(g); z[k] = U(g); }
    // m5
    double a[5] = {0}, b[5] = {0}, H[15];
    mat_H<2>(M, t, H); sym_mv_acc(H, x, a);
    mat_Gv(M, t, H); sym_mv_acc(H, y, a);
    mat_Gw(M, t, H); sym_mv_acc(H, z, a);
    m5_acc(M, t, x, y, z, b);
    printf("m5 %.3e\n", rel(a, b, 5));
    // <u^p psi psi^T> x matrix-free (p = 0, 1) against mat_H<p> times x
    for (int p = 0; p < 2; ++p) {
      double c[5] = {0}, d[5] = {0};
      if (p) mat_H<1>(M, t, H); else mat_H<0>(M, t, H);
      sym_mv_acc(H, y, c);
      const double hR1 = 0.5 * t.R1, q4 = 0.25 * (t.R2 - t.R1 * t.R1);
      if (p) hmat_mv_acc<1>(M, t, th, hR1, q4, y, d); else hmat_mv_acc<0>(M, t, th, hR1, q4, y, d);
      printf("hmv %.3e\n", rel(c, d, 5));
    }
    // prim_grad_dt
    const double rho = R(g);
    double Q[5] = {rho, rho * Uu, rho * V, rho * W, 0.0}, dq[3][5];
    Q[4] = th * rho / gm1 + 0.5 * rho * (Uu * Uu + V * V + W * W);
    for (int e = 0; e < 3; ++e) for (int k = 0; k < 5; ++k) dq[e][k] = U(g);
    const Prim<double> s = primitive(Q, gm1);
    double d1[5], d2[5];
    euler_dt(s, Q, gm1, dq, d1);
    const Grad<double> g1 = prim_grad(s, dq, gm1);
    const Grad<double> g2 = prim_grad_dt(s, Q, dq, gm1, d2);
    double ga[15], gb[15];
    for (int e = 0; e < 3; ++e) {
      for (int j = 0; j < 3; ++j) { ga[3 * e + j] = g1.dU[e][j]; gb[3 * e + j] = g2.dU[e][j]; }
      ga[9 + e] = g1.dp[e]; gb[9 + e] = g2.dp[e];
      ga[12 + e] = g1.dT[e]; gb[12 + e] = g2.dT[e];
    }
    printf("dt %.3e\n", rel(d1, d2, 5));
    printf("grad %.3e\n", rel(ga, gb, 15));
    // Solver5 against the full-line moment matrix <psi psi^T> (M_n of the
    // full Maxwellian = sum of the two half lines)
    double Mp[7], Mm[7], Mf[7], Hf[15];
    mom_half(Uu, th, 1.0, Mp);
    mom_half(Uu, th, -1.0, Mm);
    for (int n = 0; n < 7; ++n) Mf[n] = Mp[n] + Mm[n];
    mat_H<0>(Mf, t, Hf);
    double sol[5], back[5] = {0};
    const Prim<double> s1{1.0, 1.0, Uu, V, W, th, th};
    const Solver5<double> S(s1, K, 1.0 / (K + 3.0));
    S(x, sol);
    sym_mv_acc(Hf, sol, back);
    printf("solve %.3e\n", rel(x, back, 5));
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("ident")
    src, exe = d / "t.hip", d / "t"
    src.write_text(SRC)
    subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    res = {}
    for ln in out:
        if ln.strip():
            k, v = ln.split()
            res.setdefault(k, []).append(float(v))
    return {k: np.array(v) for k, v in res.items()}


@pytest.mark.parametrize("name,tol,n", [("m5", 1e-13, 4000), ("hmv", 1e-13, 8000), ("dt", 1e-13, 4000),
                                        ("grad", 1e-14, 4000), ("solve", 1e-12, 4000)])
def test_rewritten_forms_agree(results, name, tol, n):
    r = results[name]
    assert len(r) == n
    assert r.max() < tol, (name, r.max())
