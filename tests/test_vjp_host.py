"""The hand-written reverse of the point fluxes (gks_point_adj.hpp: the volume
flux, face_side and face_finish of the face flux), built for the host in FP64
from the kernels' own headers and checked against central differences of the
forward point functions: for random physical states and slopes, random
cotangents (F, Ft) and random directions in (Q, dQ, mu), <VJP, direction> must
match the fourth-order central difference of <cotangent, flux> along the
direction.  The matrix-free reverse of m5 that the FP32 kernels run
(m5_acc_bwd) is checked the same way on its own inputs.  Cases cover mu = 0
(tau = 0), a moderate and a large mu, Pr = 0.72 and 1, two time steps, nearly
equal left and right states, and low-Mach states (large internal energy, where
the difference quotient itself is less accurate)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_13821_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r'''
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "gks_point_adj.hpp"
using namespace dgk;

static Phys make_phys(double mu, double pr, double dt) {
  Phys ph{};
  const double g = 1.4;
  ph.K = (5 - 3 * g) / (g - 1);
  ph.gm1 = g - 1;
  ph.mu = mu;
  ph.inv_pr_m1 = 1 / pr - 1;
  ph.dt = dt;
  ph.inv_k3 = 1 / (ph.K + 3);
  ph.cp = 0.5 * (ph.K + 5);
  ph.half_dt_over_mu = mu > 0 ? 0.5 * dt / mu : 0;
  ph.inv_dt = 1 / dt;
  return ph;
}

static std::mt19937_64 rng(20220228);
static double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }
static double nrm() { return std::normal_distribution<double>(0, 1)(rng); }

// conservative state with rho in [0.5, 2], |U_i| < 1.5 and internal energy
// rho e in [0.75, 7.5] (or [170, 190]: Mach about 0.1)
static void state(double* q, bool low_mach) {
  const double r = uni(0.5, 2), u = uni(-1.5, 1.5), v = uni(-1.5, 1.5), w = uni(-1.5, 1.5);
  const double e = low_mach ? uni(170, 190) : uni(0.75, 7.5);
  q[0] = r; q[1] = r * u; q[2] = r * v; q[3] = r * w;
  q[4] = e + 0.5 * r * (u * u + v * v + w * w);
}

template <bool NF>
static double vol_obj(const Phys& ph, const double* x, const double* Fb, const double* Ftb) {
  double q[5], dq[3][5], F[3][5], Ft[3][5];
  int bad = 0;
  for (int i = 0; i < 5; ++i) q[i] = x[i];
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < 5; ++i) dq[e][i] = x[5 + 5 * e + i];
  volume_flux<double, NF>(ph, q, dq, F, Ft, bad);
  double s = 0;
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < 5; ++i) s += (NF ? Fb[5 * e + i] * F[e][i] : 0) + Ftb[5 * e + i] * Ft[e][i];
  return s;
}

template <bool NF>
static double face_obj(const Phys& ph, const double* x, const double* Fb, const double* Ftb) {
  double qL[5], qR[5], dqL[3][5], dqR[3][5], F[5], Ft[5];
  int bad = 0;
  for (int i = 0; i < 5; ++i) { qL[i] = x[i]; qR[i] = x[20 + i]; }
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < 5; ++i) { dqL[e][i] = x[5 + 5 * e + i]; dqR[e][i] = x[25 + 5 * e + i]; }
  face_flux_local<double, NF>(ph, qL, dqL, qR, dqR, F, Ft, bad);
  double s = 0;
  for (int i = 0; i < 5; ++i) s += (NF ? Fb[i] * F[i] : 0) + Ftb[i] * Ft[i];
  return s;
}

// derivative at 0 by the fourth-order central stencil, h = 1e-3 (truncation
// ~h^4, rounding ~1e-16 / h of the objective's terms)
template <class F>
static double central4(F f) {
  const double h = 1e-3;
  return (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h);
}

int main() {
  for (int trial = 0; trial < 24; ++trial) {
    const bool lm = trial % 2;
    const double mu = (trial % 3 == 0) ? 0.0 : (trial % 3 == 1 ? 1.0 / 1600 : 0.03);
    const double pr = (trial % 4 < 2) ? 0.72 : 1.0, dt = (trial % 5 == 0) ? 1e-2 : 6.7e-4;
    const Phys ph = make_phys(mu, pr, dt);
    const double dmu = mu > 0 ? 0.3 * mu : 0.0;
    double x[40], d[40], Fb[15], Ftb[15];
    // volume flux
    state(x, lm);
    for (int i = 5; i < 20; ++i) x[i] = 0.5 * nrm();
    for (int i = 0; i < 20; ++i) d[i] = nrm() * (i < 5 ? 0.01 * std::fabs(x[i]) + 1e-3 : 0.05);
    for (int i = 0; i < 15; ++i) { Fb[i] = nrm(); Ftb[i] = nrm(); }
    for (int nf = 0; nf < 2; ++nf) {
      double q[5], dq[3][5], qb[5] = {0}, dqb[3][5] = {{0}}, Fa[3][5], Fta[3][5], mub = 0;
      for (int i = 0; i < 5; ++i) q[i] = x[i];
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < 5; ++i) { dq[e][i] = x[5 + 5 * e + i]; Fa[e][i] = Fb[5 * e + i]; Fta[e][i] = Ftb[5 * e + i]; }
      if (nf) volume_flux_vjp<double, true>(ph, q, dq, Fa, Fta, qb, dqb, mub);
      else volume_flux_vjp<double, false>(ph, q, dq, Fa, Fta, qb, dqb, mub);
      double lin = mub * dmu;
      for (int i = 0; i < 5; ++i) lin += qb[i] * d[i];
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < 5; ++i) lin += dqb[e][i] * d[5 + 5 * e + i];
      auto fv = [&](double s) {
        double xs[20];
        for (int i = 0; i < 20; ++i) xs[i] = x[i] + s * d[i];
        const Phys ps = make_phys(mu + s * dmu, pr, dt);
        return nf ? vol_obj<true>(ps, xs, Fb, Ftb) : vol_obj<false>(ps, xs, Fb, Ftb);
      };
      const double fd = central4(fv);
      printf("volume %d %d %d %.3e\n", trial, nf, int(lm), std::fabs(lin - fd) / std::max(std::fabs(fd), 1e-8));
    }
    // face flux: both sides, then the finish
    state(x, lm);
    state(x + 20, lm);
    if (trial % 3 == 0)
      for (int i = 0; i < 5; ++i) x[20 + i] = x[i] * (1 + 0.02 * nrm());
    for (int i = 5; i < 20; ++i) { x[i] = 0.5 * nrm(); x[20 + i] = 0.5 * nrm(); }
    for (int i = 0; i < 40; ++i) d[i] = nrm() * ((i % 20) < 5 ? 0.01 * std::fabs(x[i]) + 1e-3 : 0.05);
    for (int i = 0; i < 5; ++i) { Fb[i] = nrm(); Ftb[i] = nrm(); }
    for (int nf = 0; nf < 2; ++nf) {
      double qL[5], qR[5], dqL[3][5], dqR[3][5];
      for (int i = 0; i < 5; ++i) { qL[i] = x[i]; qR[i] = x[20 + i]; }
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < 5; ++i) { dqL[e][i] = x[5 + 5 * e + i]; dqR[e][i] = x[25 + 5 * e + i]; }
      FaceAcc<double> acc, accb;
      face_acc_zero(acc);
      face_acc_zero(accb);
      int bad = 0;
      face_side(ph, qL, dqL, acc, bad, 1.0);
      face_side(ph, qR, dqR, acc, bad, -1.0);
      double mub = 0;
      if (nf) face_finish_vjp<double, true>(ph, acc, Fb, Ftb, accb, mub);
      else face_finish_vjp<double, false>(ph, acc, nullptr, Ftb, accb, mub);
      double qLb[5] = {0}, qRb[5] = {0}, dqLb[3][5] = {{0}}, dqRb[3][5] = {{0}};
      face_side_vjp(ph, qL, dqL, accb, qLb, dqLb, 1.0);
      face_side_vjp(ph, qR, dqR, accb, qRb, dqRb, -1.0);
      double lin = mub * dmu;
      for (int i = 0; i < 5; ++i) lin += qLb[i] * d[i] + qRb[i] * d[20 + i];
      for (int e = 0; e < 3; ++e)
        for (int i = 0; i < 5; ++i) lin += dqLb[e][i] * d[5 + 5 * e + i] + dqRb[e][i] * d[25 + 5 * e + i];
      auto ff = [&](double s) {
        double xs[40];
        for (int i = 0; i < 40; ++i) xs[i] = x[i] + s * d[i];
        const Phys ps = make_phys(mu + s * dmu, pr, dt);
        return nf ? face_obj<true>(ps, xs, Fb, Ftb) : face_obj<false>(ps, xs, Fb, Ftb);
      };
      const double fd = central4(ff);
      printf("face %d %d %d %.3e\n", trial, nf, int(lm), std::fabs(lin - fd) / std::max(std::fabs(fd), 1e-8));
    }
  }
  // m5_acc_bwd (the matrix-free reverse of m5 that the FP32 kernels run)
  // against central differences of <ob, m5_acc> in every input: M, the fifteen
  // transverse moments taken as independent inputs, and x, y, z
  for (int trial = 0; trial < 48; ++trial) {
    double M[7], x[15], ob[5], dM[7], dx[15];
    mom_half(uni(-1.5, 1.5), uni(0.2, 3.0), trial % 2 ? 1.0 : -1.0, M);
    const Transverse<double> t0(uni(-1.5, 1.5), uni(-1.5, 1.5), uni(0.2, 3.0), 2.0);
    for (int i = 0; i < 15; ++i) { x[i] = nrm(); dx[i] = nrm(); }
    for (int i = 0; i < 7; ++i) dM[i] = nrm();
    for (int k = 0; k < 5; ++k) ob[k] = nrm();
    double dt[15];
    for (int i = 0; i < 15; ++i) dt[i] = nrm();
    auto members = [](Transverse<double>& t) {
      double* m[15] = {&t.V, &t.W, &t.v2, &t.w2, &t.v3, &t.w3, &t.R1, &t.R2, &t.vr, &t.wr,
                       &t.v2r, &t.w2r, &t.vwr, &t.vr2, &t.wr2};
      return std::vector<double*>(m, m + 15);
    };
    auto f = [&](double s) {
      double Ms[7], xs[15], m5[5] = {0, 0, 0, 0, 0};
      for (int i = 0; i < 7; ++i) Ms[i] = M[i] + s * dM[i];
      for (int i = 0; i < 15; ++i) xs[i] = x[i] + s * dx[i];
      Transverse<double> ts = t0;
      std::vector<double*> mm = members(ts);
      for (int i = 0; i < 15; ++i) *mm[i] += s * dt[i];
      m5_acc(Ms, ts, xs, xs + 5, xs + 10, m5);
      double r = 0;
      for (int k = 0; k < 5; ++k) r += ob[k] * m5[k];
      return r;
    };
    double Mb[7] = {0, 0, 0, 0, 0, 0, 0}, xb[15] = {0};
    TransverseBar<double> tb = transverse_bar_zero<double>();
    m5_acc_bwd(M, t0, x, x + 5, x + 10, ob, Mb, tb, xb, xb + 5, xb + 10);
    const double tbv[15] = {tb.V, tb.W, tb.v2, tb.w2, tb.v3, tb.w3, tb.R1, tb.R2, tb.vr, tb.wr,
                            tb.v2r, tb.w2r, tb.vwr, tb.vr2, tb.wr2};
    double lin = 0;
    for (int i = 0; i < 7; ++i) lin += Mb[i] * dM[i];
    for (int i = 0; i < 15; ++i) lin += xb[i] * dx[i] + tbv[i] * dt[i];
    const double fd = central4(f);
    printf("m5bwd %d 0 0 %.3e\n", trial, std::fabs(lin - fd) / std::max(std::fabs(fd), 1e-8));
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("vjp")
    src, exe = d / "t.hip", d / "t"
    src.write_text(SRC)
    subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    rows = [ln.split() for ln in out if ln.strip()]
    return [(k, int(t), int(nf), int(lm), float(rel)) for k, t, nf, lm, rel in rows]


def test_every_case_ran(results):
    kinds = [k for k, *_ in results]
    assert kinds.count("volume") == kinds.count("face") == 24 * 2 and kinds.count("m5bwd") == 48


@pytest.mark.parametrize("kind", ["volume", "face", "m5bwd"])
def test_vjp_matches_central_differences(results, kind):
    # the stencil leaves below 1e-10 relative, up to a few 1e-9 where the low-Mach
    # objectives are small differences of large moments (its rounding part)
    bad = [(t, nf, lm, rel) for k, t, nf, lm, rel in results if k == kind and rel > 1e-7]
    assert not bad, bad
