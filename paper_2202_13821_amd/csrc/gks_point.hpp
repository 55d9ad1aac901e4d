// gks_point.hpp -- gas-kinetic point fluxes on the device (HIP, gfx950).
//
// Everything here acts on one quadrature point and is templated on the bulk
// precision T (float or double).  Notation follows the paper: conservative
// Q = (rho, rho U, rho V, rho W, rho E), Maxwellian g with lambda = rho/(2p)
// (here carried as th = 1/(2 lambda) = p/rho), K internal degrees of freedom,
// psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2), <.> moments of g divided by rho,
// collision time tau = mu/p.
//
//  * face_flux   : Section 2, Eq. (flux) with its slope systems, in the local
//                  frame of the face (normal velocity first), followed by the
//                  linear-in-time fit of Eq. (expansion-1) over [0, dt] and
//                  [0, dt/2].  The exp(-t/tau) time-integral coefficients and
//                  their combination with the flux moments are FP64.
//  * volume_flux : Section 3, Eq. (flux-2), f = g0 (1 - tau (a.u + A) + A t).
//
// Moments are formed from products of one-dimensional Maxwellian moment
// tables; 5x5 slope systems <a psi> = b use their closed-form inverse (the
// moment matrix of a Maxwellian has an explicit inverse, see slope_solve).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "dg_tables.hpp"

namespace dgk {

// ---- compile-time loop ----------------------------------------------------
template <int... I, class F>
DGK_HD void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
DGK_HD void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, static_cast<F&&>(f));
}

// ---- precision-dispatched math ---------------------------------------------
DGK_HD float d_erfc(float x) { return erfcf(x); }
DGK_HD double d_erfc(double x) { return erfc(x); }
DGK_HD float d_exp(float x) { return expf(x); }
DGK_HD double d_exp(double x) { return exp(x); }
DGK_HD float d_sqrt(float x) { return sqrtf(x); }
DGK_HD double d_sqrt(double x) { return sqrt(x); }
// x - x is 0 for every finite x and NaN for +-inf and NaN
DGK_HD bool d_finite(float x) { return (x - x) == 0.0f; }
DGK_HD bool d_finite(double x) { return (x - x) == 0.0; }

// Physical parameters of one launch.
struct Phys {
  double K;          // internal degrees of freedom (5 - 3 gamma)/(gamma - 1)
  double gm1;        // gamma - 1
  double mu;         // dynamic viscosity; tau = mu / p
  double inv_pr_m1;  // 1/Pr - 1 (Prandtl correction of the heat flux)
  double dt;         // time step (window of the time fit)
};

template <class T>
struct Prim {
  T rho, U, V, W, th, p;  // th = p / rho = 1 / (2 lambda)
};

template <class T>
DGK_HD Prim<T> primitive(const T Q[5], T gm1) {
  Prim<T> s;
  s.rho = Q[0];
  const T ir = T(1) / Q[0];
  s.U = Q[1] * ir;
  s.V = Q[2] * ir;
  s.W = Q[3] * ir;
  s.p = gm1 * (Q[4] - T(0.5) * (Q[1] * s.U + Q[2] * s.V + Q[3] * s.W));
  s.th = s.p * ir;
  return s;
}

template <class T>
DGK_HD bool unphysical(const Prim<T>& s) {
  return !(s.rho > T(0)) || !(s.p > T(0)) || !d_finite(s.U + s.V + s.W + s.p);
}

// Normalised one-dimensional moments <c^0..c^6> plus <xi^2>, <xi^4>.
template <class T>
struct Mom {
  T u[7], v[7], w[7], x2, x4;
};

// <c^{n+2}> = U <c^{n+1}> + (n+1) th <c^n>  (Gaussian integration by parts)
template <class T>
DGK_HD void mom_full(T U, T th, T* m) {
  m[0] = T(1);
  m[1] = U;
#pragma unroll
  for (int n = 0; n < 5; ++n) m[n + 2] = U * m[n + 1] + T(n + 1) * th * m[n];
}

// Half line u > 0 (side > 0) or u < 0: first two moments from erfc and the
// Gaussian at u = 0, then the same recurrence.
template <class T>
DGK_HD void mom_half(T U, T th, int side, T* m) {
  const T r = T(1) / d_sqrt(T(2) * th);  // sqrt(lambda)
  const T a = U * r;
  const T e = d_exp(-a * a) * d_sqrt(th * T(0.15915494309189533577));  // sqrt(th / (2 pi))
  if (side > 0) {
    m[0] = T(0.5) * d_erfc(-a);
    m[1] = U * m[0] + e;
  } else {
    m[0] = T(0.5) * d_erfc(a);
    m[1] = U * m[0] - e;
  }
#pragma unroll
  for (int n = 0; n < 5; ++n) m[n + 2] = U * m[n + 1] + T(n + 1) * th * m[n];
}

template <class T>
DGK_HD void mom_xi(T K, T th, Mom<T>& t) {
  t.x2 = K * th;
  t.x4 = K * (K + T(2)) * th * th;
}

template <class T>
DGK_HD Mom<T> moments_full(const Prim<T>& s, T K) {
  Mom<T> t;
  mom_full(s.U, s.th, t.u);
  mom_full(s.V, s.th, t.v);
  mom_full(s.W, s.th, t.w);
  mom_xi(K, s.th, t);
  return t;
}

// Tangential tables of a half-space set are the full ones; only u differs.
template <class T>
DGK_HD Mom<T> moments_half(const Prim<T>& s, const Mom<T>& full, int side) {
  Mom<T> t = full;
  mom_half(s.U, s.th, side, t.u);
  return t;
}

// <u^a v^b w^c (xi^2)^d>
template <int a, int b, int c, int d, class T>
DGK_HD T Mo(const Mom<T>& t) {
  static_assert(a <= 6 && b <= 6 && c <= 6 && d <= 2, "moment order");
  T r = t.u[a];
  if constexpr (b > 0) r *= t.v[b];
  if constexpr (c > 0) r *= t.w[c];
  if constexpr (d == 1) r *= t.x2;
  if constexpr (d == 2) r *= t.x4;
  return r;
}

// <u^a v^b w^c (xi^2)^d  s>, s = sum_j s_j psi_j
template <int a, int b, int c, int d, class T>
DGK_HD T Gs(const Mom<T>& t, const T s[5]) {
  return s[0] * Mo<a, b, c, d>(t) + s[1] * Mo<a + 1, b, c, d>(t) + s[2] * Mo<a, b + 1, c, d>(t) +
         s[3] * Mo<a, b, c + 1, d>(t) +
         T(0.5) * s[4] * (Mo<a + 2, b, c, d>(t) + Mo<a, b + 2, c, d>(t) + Mo<a, b, c + 2, d>(t) + Mo<a, b, c, d + 1>(t));
}

// out_k = <u^a v^b w^c s psi_k>
template <int a, int b, int c, class T>
DGK_HD void Gpsi(const Mom<T>& t, const T s[5], T out[5]) {
  out[0] = Gs<a, b, c, 0>(t, s);
  out[1] = Gs<a + 1, b, c, 0>(t, s);
  out[2] = Gs<a, b + 1, c, 0>(t, s);
  out[3] = Gs<a, b, c + 1, 0>(t, s);
  out[4] = T(0.5) * (Gs<a + 2, b, c, 0>(t, s) + Gs<a, b + 2, c, 0>(t, s) + Gs<a, b, c + 2, 0>(t, s) +
                     Gs<a, b, c, 1>(t, s));
}

// out_k = <u^a v^b w^c psi_k>
template <int a, int b, int c, class T>
DGK_HD void psim(const Mom<T>& t, T out[5]) {
  out[0] = Mo<a, b, c, 0>(t);
  out[1] = Mo<a + 1, b, c, 0>(t);
  out[2] = Mo<a, b + 1, c, 0>(t);
  out[3] = Mo<a, b, c + 1, 0>(t);
  out[4] = T(0.5) * (Mo<a + 2, b, c, 0>(t) + Mo<a, b + 2, c, 0>(t) + Mo<a, b, c + 2, 0>(t) + Mo<a, b, c, 1>(t));
}

// Closed-form solution of <a psi> = b for the Maxwellian (U, V, W, th):
// with E' = <psi_5> = (U^2+V^2+W^2)/2 + (K+3) th/2 and R_i = b_{i+1} - U_i b_0,
//   a_4 = 2/((K+3) th^2) (b_4 - E' b_0 - U R_1 - V R_2 - W R_3)
//   a_i = R_i / th - U_i a_4      (i = 1, 2, 3)
//   a_0 = b_0 - U a_1 - V a_2 - W a_3 - E' a_4
template <class T>
struct Solver5 {
  T U, V, W, ith, E, c4;
  DGK_HD Solver5(const Prim<T>& s, T K) {
    U = s.U;
    V = s.V;
    W = s.W;
    ith = T(1) / s.th;
    E = T(0.5) * (U * U + V * V + W * W) + T(0.5) * (K + T(3)) * s.th;
    c4 = T(2) * ith * ith / (K + T(3));
  }
  DGK_HD void operator()(const T b[5], T a[5]) const {
    const T R1 = b[1] - U * b[0], R2 = b[2] - V * b[0], R3 = b[3] - W * b[0];
    a[4] = c4 * (b[4] - E * b[0] - U * R1 - V * R2 - W * R3);
    a[1] = R1 * ith - U * a[4];
    a[2] = R2 * ith - V * a[4];
    a[3] = R3 * ith - W * a[4];
    a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - E * a[4];
  }
};

// Time-integral coefficients (FP64).  With e(t) = exp(-t/tau), the time
// factors of Eq. (flux) integrate over [0, delta] to
//   c1 = delta - tau (1 - e),          c2 = 2 tau^2 - tau delta - tau (2 tau + delta) e,
//   c3 = delta^2/2 - tau delta + tau^2 (1 - e),  c4 = tau (1 - e),
//   c5 = 2 tau^2 - tau (2 tau + delta) e,        c6 = tau^2 (1 - e),
// (c5, c6 enter with a minus sign).  The fit F dt + Ft dt^2/2 = FF(dt),
// F dt/2 + Ft dt^2/8 = FF(dt/2) gives F = sum alpha_i m_i, Ft = sum beta_i m_i.
// tau = 0 is the inviscid limit (e = 0): F = m1, Ft = m3.
DGK_HD void time_coefficients(double tau, double dt, double alpha[6], double beta[6]) {
  const double e2 = tau > 0.0 ? exp(-0.5 * dt / tau) : 0.0;
  const double e1 = e2 * e2;
  double c[2][6];
  const double dl[2] = {dt, 0.5 * dt};
  const double ee[2] = {e1, e2};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double d = dl[j], e = ee[j], om = 1.0 - e;
    c[j][0] = d - tau * om;
    c[j][1] = 2.0 * tau * tau - tau * d - tau * (2.0 * tau + d) * e;
    c[j][2] = 0.5 * d * d - tau * d + tau * tau * om;
    c[j][3] = tau * om;
    c[j][4] = -(2.0 * tau * tau - tau * (2.0 * tau + d) * e);
    c[j][5] = -(tau * tau * om);
  }
  const double idt = 1.0 / dt, idt2 = 4.0 * idt * idt;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    alpha[i] = (4.0 * c[1][i] - c[0][i]) * idt;
    beta[i] = (c[0][i] - 2.0 * c[1][i]) * idt2;
  }
}

// --------------------------------------------------------------------------
// Face flux in the local frame: qL, dqL (trace of the lower cell, u > 0 half
// space) and qR, dqR (upper cell, u < 0), dq*[i] = derivative along local
// direction i (0 normal, 1 and 2 tangential).  Outputs F, Ft in the local frame.
// NEED_F = false computes only Ft (second stage of S2O4).
// --------------------------------------------------------------------------
template <class T, bool NEED_F>
DGK_HD void face_flux_local(const Phys& ph, const T qL[5], const T dqL[3][5], const T qR[5], const T dqR[3][5],
                            T F[5], T Ft[5], int& bad) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> sL = primitive(qL, gm1), sR = primitive(qR, gm1);
  bad |= int(unphysical(sL)) | int(unphysical(sR));
  const Mom<T> fL = moments_full(sL, K), fR = moments_full(sR, K);
  const Mom<T> hL = moments_half(sL, fL, +1), hR = moments_half(sR, fR, -1);

  // microscopic slopes of the two sides and their time slopes (compatibility)
  T aL[3][5], aR[3][5], AL[5], AR[5];
  {
    const Solver5<T> SL(sL, K), SR(sR, K);
    T bL[5], bR[5];
    const T irL = T(1) / sL.rho, irR = T(1) / sR.rho;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        bL[k] = dqL[i][k] * irL;
        bR[k] = dqR[i][k] * irR;
      }
      SL(bL, aL[i]);
      SR(bR, aR[i]);
    }
    T y0[5], y1[5], y2[5];
    Gpsi<1, 0, 0>(fL, aL[0], y0);
    Gpsi<0, 1, 0>(fL, aL[1], y1);
    Gpsi<0, 0, 1>(fL, aL[2], y2);
#pragma unroll
    for (int k = 0; k < 5; ++k) bL[k] = -(y0[k] + y1[k] + y2[k]);
    SL(bL, AL);
    Gpsi<1, 0, 0>(fR, aR[0], y0);
    Gpsi<0, 1, 0>(fR, aR[1], y1);
    Gpsi<0, 0, 1>(fR, aR[2], y2);
#pragma unroll
    for (int k = 0; k < 5; ++k) bR[k] = -(y0[k] + y1[k] + y2[k]);
    SR(bR, AR);
  }

  // equilibrium state at the interface and its directional derivatives
  T Q0[5], dQ0[3][5];
  {
    T pL[5], pR[5];
    psim<0, 0, 0>(hL, pL);
    psim<0, 0, 0>(hR, pR);
#pragma unroll
    for (int k = 0; k < 5; ++k) Q0[k] = sL.rho * pL[k] + sR.rho * pR[k];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Gpsi<0, 0, 0>(hL, aL[i], pL);
      Gpsi<0, 0, 0>(hR, aR[i], pR);
#pragma unroll
      for (int k = 0; k < 5; ++k) dQ0[i][k] = sL.rho * pL[k] + sR.rho * pR[k];
    }
  }
  const Prim<T> s0 = primitive(Q0, gm1);
  bad |= unphysical(s0);
  const Mom<T> f0 = moments_full(s0, K);
  T ab[3][5], Ab[5];
  {
    const Solver5<T> S0(s0, K);
    const T ir0 = T(1) / s0.rho;
    T b[5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = dQ0[i][k] * ir0;
      S0(b, ab[i]);
    }
    T y0[5], y1[5], y2[5];
    Gpsi<1, 0, 0>(f0, ab[0], y0);
    Gpsi<0, 1, 0>(f0, ab[1], y1);
    Gpsi<0, 0, 1>(f0, ab[2], y2);
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = -(y0[k] + y1[k] + y2[k]);
    S0(b, Ab);
  }

  // flux moments of the six parts of Eq. (flux)
  T m[6][5];
  {
    T y0[5], y1[5], y2[5];
    psim<1, 0, 0>(f0, m[0]);
    Gpsi<2, 0, 0>(f0, ab[0], y0);
    Gpsi<1, 1, 0>(f0, ab[1], y1);
    Gpsi<1, 0, 1>(f0, ab[2], y2);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      m[0][k] *= s0.rho;
      m[1][k] = s0.rho * (y0[k] + y1[k] + y2[k]);
    }
    Gpsi<1, 0, 0>(f0, Ab, y0);
#pragma unroll
    for (int k = 0; k < 5; ++k) m[2][k] = s0.rho * y0[k];

    T zL[5], zR[5];
    psim<1, 0, 0>(hL, zL);
    psim<1, 0, 0>(hR, zR);
#pragma unroll
    for (int k = 0; k < 5; ++k) m[3][k] = sL.rho * zL[k] + sR.rho * zR[k];
    Gpsi<2, 0, 0>(hL, aL[0], y0);
    Gpsi<1, 1, 0>(hL, aL[1], y1);
    Gpsi<1, 0, 1>(hL, aL[2], y2);
    Gpsi<2, 0, 0>(hR, aR[0], zL);
#pragma unroll
    for (int k = 0; k < 5; ++k) m[4][k] = sL.rho * (y0[k] + y1[k] + y2[k]) + sR.rho * zL[k];
    Gpsi<1, 1, 0>(hR, aR[1], y0);
    Gpsi<1, 0, 1>(hR, aR[2], y1);
#pragma unroll
    for (int k = 0; k < 5; ++k) m[4][k] += sR.rho * (y0[k] + y1[k]);
    Gpsi<1, 0, 0>(hL, AL, y0);
    Gpsi<1, 0, 0>(hR, AR, y1);
#pragma unroll
    for (int k = 0; k < 5; ++k) m[5][k] = sL.rho * y0[k] + sR.rho * y1[k];
  }

  const double tau = ph.mu / double(s0.p);
  double al[6], be[6];
  time_coefficients(tau, ph.dt, al, be);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double ft = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) ft += be[j] * double(m[j][k]);
    Ft[k] = T(ft);
  }
  if constexpr (NEED_F) {
    double f[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 6; ++j) s += al[j] * double(m[j][k]);
      f[k] = s;
    }
    // Heat flux of the non-equilibrium part -tau g0 (abar.u + Abar):
    // q = -tau rho0 <(u - U0) (|u - U0|^2 + xi^2)/2 X>.  Writing
    // (|u-U0|^2 + xi^2)/2 = c.psi with c = (|U0|^2/2, -U0, -V0, -W0, 1) and using
    // <X psi> = 0 (compatibility), q = -tau c.(m2 + m3).
    const double U0 = s0.U, V0 = s0.V, W0 = s0.W;
    const double cc[5] = {0.5 * (U0 * U0 + V0 * V0 + W0 * W0), -U0, -V0, -W0, 1.0};
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) q += cc[k] * (double(m[1][k]) + double(m[2][k]));
    f[4] += ph.inv_pr_m1 * (-tau * q);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = T(f[k]);
  }
}

// --------------------------------------------------------------------------
// Volume flux (global frame).  q, dq[e] = dQ/dx_e; F[d], Ft[d] for d = x,y,z.
// F_d = rho [<u_d psi> - tau (sum_e <u_d u_e a_e psi> + <u_d A psi>)] + Pr term,
// Ft_d = rho <u_d A psi>.
// --------------------------------------------------------------------------
template <int D, int E>
struct UDE {
  static constexpr int a = (D == 0) + (E == 0), b = (D == 1) + (E == 1), c = (D == 2) + (E == 2);
};

template <class T, bool NEED_F>
DGK_HD void volume_flux(const Phys& ph, const T q[5], const T dq[3][5], T F[3][5], T Ft[3][5], int& bad) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> s = primitive(q, gm1);
  bad |= unphysical(s);
  const Mom<T> t = moments_full(s, K);
  const Solver5<T> S(s, K);
  T a[3][5], A[5];
  {
    const T ir = T(1) / s.rho;
    T b[5];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = dq[e][k] * ir;
      S(b, a[e]);
    }
    T y0[5], y1[5], y2[5];
    Gpsi<1, 0, 0>(t, a[0], y0);
    Gpsi<0, 1, 0>(t, a[1], y1);
    Gpsi<0, 0, 1>(t, a[2], y2);
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = -(y0[k] + y1[k] + y2[k]);
    S(b, A);
  }
  T uA[3][5];
  Gpsi<1, 0, 0>(t, A, uA[0]);
  Gpsi<0, 1, 0>(t, A, uA[1]);
  Gpsi<0, 0, 1>(t, A, uA[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < 5; ++k) Ft[d][k] = s.rho * uA[d][k];
  if constexpr (NEED_F) {
    const T tau = T(ph.mu) / s.p;
    const T cc[5] = {T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W), -s.U, -s.V, -s.W, T(1)};
    const T prf = T(ph.inv_pr_m1);
    static_for<3>([&](auto dc) {
      constexpr int d = decltype(dc)::value;
      T visc[5], y0[5], y1[5], y2[5], e0[5];
      Gpsi<UDE<d, 0>::a, UDE<d, 0>::b, UDE<d, 0>::c>(t, a[0], y0);
      Gpsi<UDE<d, 1>::a, UDE<d, 1>::b, UDE<d, 1>::c>(t, a[1], y1);
      Gpsi<UDE<d, 2>::a, UDE<d, 2>::b, UDE<d, 2>::c>(t, a[2], y2);
      psim<d == 0, d == 1, d == 2>(t, e0);
      T qh = T(0);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        visc[k] = uA[d][k] + y0[k] + y1[k] + y2[k];
        qh += cc[k] * visc[k];
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) F[d][k] = s.rho * (e0[k] - tau * visc[k]);
      // heat flux of -tau g (a.u + A), same reduction as on the faces
      F[d][4] += prf * (-tau * s.rho * qh);
    });
  }
}

}  // namespace dgk
