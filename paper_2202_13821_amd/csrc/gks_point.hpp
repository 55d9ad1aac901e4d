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
//                  [0, dt/2].  The exp(-t/tau) time-integral coefficients are
//                  FP64; their combination with the flux moments runs in T.
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
DGK_HD float d_exp(float x) { return expf(x); }
DGK_HD double d_exp(double x) { return exp(x); }
DGK_HD float d_sqrt(float x) { return sqrtf(x); }
DGK_HD double d_sqrt(double x) { return sqrt(x); }
// Reciprocal, reciprocal square root and exp: FP32-bulk uses the hardware
// instructions (v_rcp_f32, v_rsq_f32: 1 ulp; v_exp_f32: ~1-2 ulp).  FP64
// refines the hardware v_rcp_f64 / v_rsq_f64 estimates by two Newton-Raphson
// steps each (the relative error squares at every step), which leaves at most
// about 1 ulp for the positive, normal arguments these are used on (densities,
// temperatures, pressures); the FP64 path keeps the library exp.
#ifdef __HIP_DEVICE_COMPILE__
DGK_HD float d_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
DGK_HD float d_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
DGK_HD float d_expf_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f); }
DGK_HD double d_rcp(double x) {
  // r <- r + r (1 - x r)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
DGK_HD double d_rsqrt(double x) {
  // r <- r + r (1/2 - (x/2) r^2)
  const double h = 0.5 * x;
  double r = __builtin_amdgcn_rsq(x);
  double e = __builtin_fma(-h * r, r, 0.5);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-h * r, r, 0.5);
  return __builtin_fma(r, e, r);
}
#else
DGK_HD float d_rcp(float x) { return 1.0f / x; }
DGK_HD float d_rsqrt(float x) { return 1.0f / sqrtf(x); }
DGK_HD float d_expf_fast(float x) { return expf(x); }
DGK_HD double d_rcp(double x) { return 1.0 / x; }
DGK_HD double d_rsqrt(double x) { return 1.0 / sqrt(x); }
#endif
DGK_HD float d_exp_bulk(float x) { return d_expf_fast(x); }
DGK_HD double d_exp_bulk(double x) { return exp(x); }

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
  // derived on the host
  double inv_k3;     // 1 / (K + 3)
  double cp;         // (K + 5) / 2, heat capacity at constant pressure (R = 1)
  double half_dt_over_mu;  // dt / (2 mu), 0 when mu = 0 (tau = 0)
  double inv_dt;     // 1 / dt
};

template <class T>
struct Prim {
  T rho, ir, U, V, W, th, p;  // ir = 1/rho, th = p / rho = 1 / (2 lambda)
};

template <class T>
DGK_HD Prim<T> primitive(const T Q[5], T gm1) {
  Prim<T> s;
  s.rho = Q[0];
  const T ir = d_rcp(Q[0]);
  s.ir = ir;
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

// erfc(z) given g = exp(-z^2).  FP32: erfc(|z|) = g t h(t) with t = 1/(1 + |z|/2)
// and h a degree-10 polynomial fitted to exp(y^2) erfc(y) / t (fit_erfcx.py:
// relative error 1.2e-8 in exact arithmetic, a few FP32 ulp as evaluated),
// reflected by erfc(z) = 2 - erfc(-z) for z < 0; the Gaussian is the one the
// half-space moments need anyway.  FP64: the library erfc.
DGK_HD float erfc_gauss(float z, float g) {
#ifdef DGK_FLOPCOUNT
  (void)g;
  return erfcf(z);  // counted as one transcendental, like the FP64 library call
#else
  constexpr float c[11] = {2.820948064e-01f, 2.820937634e-01f, 2.468845993e-01f, 1.753157228e-01f,
                           9.346391261e-02f, -5.921645835e-02f, 1.321880221e-01f, -4.549888372e-01f,
                           4.937071800e-01f, -2.347392291e-01f, 4.319654033e-02f};
  const float y = fabsf(z);
  const float t = d_rcp(1.0f + 0.5f * y);
  float h = c[10];
#pragma unroll
  for (int i = 9; i >= 0; --i) h = h * t + c[i];
  const float r = g * (t * h);
  return z < 0.0f ? 2.0f - r : r;
#endif
}
DGK_HD double erfc_gauss(double z, double) { return erfc(z); }

// Moments <u^n>, n = 0..6, of the normalised Maxwellian in u over the half
// line sg u > 0 (sg = +1: u > 0, sg = -1: u < 0): the first two from erfc and
// the Gaussian at u = 0, then <u^{n+2}> = U <u^{n+1}> + (n+1) th <u^n>
// (integration by parts).
template <class T>
DGK_HD void mom_half(T U, T th, T sg, T* m) {
  const T r = d_rsqrt(T(2) * th);  // sqrt(lambda)
  const T a = U * r;
  // exp(-lambda U^2) / (2 sqrt(pi lambda)) = exp(-a^2) th r / sqrt(pi)
  const T ga = d_exp_bulk(-a * a);
  const T e = ga * (th * r * T(0.56418958354775628695));
  m[0] = T(0.5) * erfc_gauss(-sg * a, ga);
  m[1] = U * m[0] + sg * e;
#pragma unroll
  for (int n = 0; n < 5; ++n) m[n + 2] = U * m[n + 1] + T(n + 1) * th * m[n];
}

// Closed-form solution of <a psi> = b for the Maxwellian (U, V, W, th):
// with E' = <psi_5> = (U^2+V^2+W^2)/2 + (K+3) th/2 and R_i = b_{i+1} - U_i b_0,
//   a_4 = 2/((K+3) th^2) (b_4 - E' b_0 - U R_1 - V R_2 - W R_3)
//   a_i = R_i / th - U_i a_4      (i = 1, 2, 3)
//   a_0 = b_0 - U a_1 - V a_2 - W a_3 - E' a_4
template <class T>
struct Solver5 {
  T U, V, W, ith, E, c4;
  DGK_HD Solver5(const Prim<T>& s, T K, T inv_k3) {
    U = s.U;
    V = s.V;
    W = s.W;
    ith = d_rcp(s.th);
    E = T(0.5) * (U * U + V * V + W * W) + T(0.5) * (K + T(3)) * s.th;
    c4 = T(2) * ith * ith * inv_k3;
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

// exp(-x) for x >= 0 in FP64 from a table ec of 15 constants that the caller
// keeps where uniform loads are cheap (LDS in the face kernel): Cody-Waite
// reduction x = k ln 2 + r with ln 2 split into a high part with 21 trailing
// zero bits (k ln2_hi is exact for k < 2^21) and a low part, |r| <= ln2 / 2,
// then exp(-r) by its Taylor polynomial of degree 13 (truncation below 5e-18
// relative) and the exact scaling by 2^-k.  ec = (log2 e, ln2_hi, ln2_lo,
// 1/2!, ..., 1/13!).
struct ExpTab {
  double c[15];
};
template <int = 0>
struct ExpTabHolder {
  static constexpr ExpTab t{{0x1.71547652b82fep+0, 0x1.62e42fee00000p-1, 0x1.a39ef35793c76p-33, 1.0 / 2.0,
                             1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
                             1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
                             1.0 / 6227020800.0}};
};
DGK_HD double exp_neg_tab(double x, const double* ec) {
#ifdef DGK_FLOPCOUNT
  (void)ec;
  return exp(-x);  // counted as one transcendental, like the other exp calls
#else
  x = fmin(x, 800.0);  // exp(-800) already underflows to 0
  const double k = rint(x * ec[0]);
  const double s = -fma(-k, ec[2], fma(-k, ec[1], x));  // -(x - k ln 2)
  double p = ec[14];
#pragma unroll
  for (int i = 13; i >= 3; --i) p = fma(p, s, ec[i]);
  p = fma(p, s, 1.0);
  p = fma(p, s, 1.0);
  return ldexp(p, -int(k));
#endif
}

// Time-integral coefficients (FP64).  With e(t) = exp(-t/tau), the time
// factors of Eq. (flux) integrate over [0, delta] to
//   c1 = delta - tau (1 - e),          c2 = 2 tau^2 - tau delta - tau (2 tau + delta) e,
//   c3 = delta^2/2 - tau delta + tau^2 (1 - e),  c4 = tau (1 - e),
//   c5 = 2 tau^2 - tau (2 tau + delta) e,        c6 = tau^2 (1 - e),
// (c5, c6 enter with a minus sign).  The fit F dt + Ft dt^2/2 = FF(dt),
// F dt/2 + Ft dt^2/8 = FF(dt/2) gives F = sum alpha_i m_i, Ft = sum beta_i m_i.
// With e = exp(-dt/(2 tau)) (so exp(-dt/tau) = e^2), x = tau/dt,
// A = 4(1 - e) - (1 - e^2) = (1 - e)(3 - e) and B = 2(1 - e) - (1 - e^2) = (1 - e)^2
// these are, without cancellation,
//   alpha = (1 - x A, 2 x tau A + tau (e^2 - 2e - 1), tau (x A - 1), x A,
//            -2 x tau A - tau (e^2 - 2e), -x tau A),
//   beta  = (4 x B/dt, 4 x (1 - e)(e - 2 x (1 - e)), 1 - 4 x^2 B, -beta_1,
//            -beta_2, 4 x^2 B)                        (beta_4 = -beta_1 etc.),
// so that the finish can combine differences of the equilibrium and
// non-equilibrium moments.
// tau = 0 is the inviscid limit (e = 0): F = m1, Ft = m3.
// x_half = dt / (2 tau) (0 when tau = 0), inv_dt = 1 / dt; ec: the table of
// exp_neg_tab.
DGK_HD void time_coefficients(double tau, double x_half, double dt, double inv_dt, double alpha[6], double beta[6],
                              const double* ec) {
  // exp(-x) < 2^-54 for x > 37.5: then 1 - e, 3 - e and e^2 - 2e - 1 round to
  // 1, 3 and -1 in FP64, and dropping e elsewhere changes beta_1 by at most
  // x e^-x relative (2e-15), so e is taken as 0 there (the branch is uniform
  // across a wavefront in a smooth flow)
  const double e = (tau > 0.0 && x_half < 37.5) ? exp_neg_tab(x_half, ec) : 0.0;
  const double x = tau * inv_dt;
  const double om = 1.0 - e;
  const double A = om * (3.0 - e), B = om * om;
  const double xA = x * A, x2B = x * x * B;
  alpha[0] = 1.0 - xA;
  alpha[1] = 2.0 * tau * xA + tau * (e * e - 2.0 * e - 1.0);
  alpha[2] = tau * (xA - 1.0);
  alpha[3] = xA;
  alpha[4] = -2.0 * tau * xA - tau * (e * e - 2.0 * e);
  alpha[5] = -tau * xA;
  beta[0] = 4.0 * x * B * inv_dt;
  beta[1] = 4.0 * x * om * (e - 2.0 * x * om);
  beta[2] = 1.0 - 4.0 * x2B;
  beta[3] = -beta[0];
  beta[4] = -beta[1];
  beta[5] = 4.0 * x2B;
}

// --------------------------------------------------------------------------
// Identities of Maxwellian moments used below (exact; with F_d(Q) =
// rho <u_d psi> the Euler flux, J_d = dF_d/dQ):
//  (i)   rho <u_d a psi> = J_d(Q) rho <a psi> for any slope a (first variation
//        of the Maxwellian), hence the compatibility condition gives
//        rho <A psi> = -sum_e J_e(Q) dQ/dx_e (the Euler time derivative) and
//        rho <u_d A psi> = J_d(Q) rho <A psi>;
//  (ii)  rho <u_d X psi> with X = sum_e u_e a_e + A equals
//        p (0, D_d1, D_d2, D_d3, U.D_d + c_p dT/dx_d), where
//        D_dj = dU_j/dx_d + dU_d/dx_j - 2/(K+3) delta_dj div U, c_p = (K+5)/2,
//        T = p/rho (the Chapman-Enskog Navier-Stokes flux of BGK).
// --------------------------------------------------------------------------
template <class T>
struct Grad {
  T dU[3][3];  // dU[e][j] = dU_j/dx_e
  T dp[3], dT[3];
};

template <class T>
DGK_HD Grad<T> prim_grad(const Prim<T>& s, const T dq[3][5], T gm1) {
  Grad<T> g;
  const T ir = s.ir;
  const T U[3] = {s.U, s.V, s.W};
  const T ke = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    T um = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      g.dU[e][j] = (dq[e][1 + j] - U[j] * dq[e][0]) * ir;
      um += U[j] * dq[e][1 + j];
    }
    g.dp[e] = gm1 * (dq[e][4] - um + ke * dq[e][0]);
    g.dT[e] = (g.dp[e] - s.th * dq[e][0]) * ir;
  }
  return g;
}

// Euler flux along axis D of the (local or global) frame.
template <int D, class T>
DGK_HD void euler_flux(const Prim<T>& s, const T Q[5], T F[5]) {
  const T U[3] = {s.U, s.V, s.W};
  const T Ud = U[D];
  F[0] = Q[1 + D];
#pragma unroll
  for (int j = 0; j < 3; ++j) F[1 + j] = Q[1 + j] * Ud;
  F[1 + D] += s.p;
  F[4] = (Q[4] + s.p) * Ud;
}

// J_D(Q) v, the directional derivative of the Euler flux along axis D.
template <int D, class T>
DGK_HD void euler_jvp(const Prim<T>& s, const T Q[5], T gm1, const T v[5], T out[5]) {
  const T U[3] = {s.U, s.V, s.W};
  const T ir = s.ir;
  T dU[3], um = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dU[j] = (v[1 + j] - U[j] * v[0]) * ir;
    um += U[j] * v[1 + j];
  }
  const T dp = gm1 * (v[4] - um + T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W) * v[0]);
  const T Ud = U[D];
  out[0] = v[1 + D];
#pragma unroll
  for (int j = 0; j < 3; ++j) out[1 + j] = v[1 + D] * U[j] + Ud * (v[1 + j] - U[j] * v[0]);
  out[1 + D] += dp;
  out[4] = (v[4] + dp) * Ud + (Q[4] + s.p) * dU[D];
}

// out (-)= J_e(Q) dQ_e written out as in euler_jvp, each product subtracted
// from out as it is formed (assigned when first):
//   J_e dQ_e = (m, m U_j + U_e t_j + delta_je dp, (dQ_e[4] + dp) U_e + (rho E + p) t_e / rho)
// with m = dQ_e[1+e], t_j = dQ_e[1+j] - U_j dQ_e[0] and dp the pressure
// derivative; hi = (rho E + p) / rho.
template <class T>
DGK_HD void sub_euler_jvp(int e, bool first, const T U[3], T m, const T t[3], T dp, T dq4, T hi, T out[5]) {
  if (first) {
    out[0] = -m;
#pragma unroll
    for (int j = 0; j < 3; ++j) out[1 + j] = -(m * U[j]) - U[e] * t[j];
    out[4] = -((dq4 + dp) * U[e]) - hi * t[e];
  } else {
    out[0] -= m;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      out[1 + j] -= m * U[j];
      out[1 + j] -= U[e] * t[j];
    }
    out[4] -= (dq4 + dp) * U[e];
    out[4] -= hi * t[e];
  }
  out[1 + e] -= dp;
}

// The same as the sum of three euler_jvp: the form of the stage-2 volume flux,
// whose FP64 P3 kernel spills far less with it.
template <class T>
DGK_HD void euler_dt_sum(const Prim<T>& s, const T Q[5], T gm1, const T dq[3][5], T out[5]) {
  T j0[5], j1[5], j2[5];
  euler_jvp<0>(s, Q, gm1, dq[0], j0);
  euler_jvp<1>(s, Q, gm1, dq[1], j1);
  euler_jvp<2>(s, Q, gm1, dq[2], j2);
#pragma unroll
  for (int k = 0; k < 5; ++k) out[k] = -(j0[k] + j1[k] + j2[k]);
}

// rho <A psi> = -sum_e J_e(Q) dQ/dx_e
template <class T>
DGK_HD void euler_dt(const Prim<T>& s, const T Q[5], T gm1, const T dq[3][5], T out[5]) {
  const T U[3] = {s.U, s.V, s.W};
  const T ke = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
  const T hi = (Q[4] + s.p) * s.ir;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    T um = T(0), t[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      t[j] = dq[e][1 + j] - U[j] * dq[e][0];
      um += U[j] * dq[e][1 + j];
    }
    const T dp = gm1 * (dq[e][4] - um + ke * dq[e][0]);
    sub_euler_jvp(e, e == 0, U, dq[e][1 + e], t, dp, dq[e][4], hi, out);
  }
}

// prim_grad and euler_dt of the same (Q, dQ) in one pass, sharing the velocity
// and pressure derivatives: with t_ej = dQ_e[1+j] - U_j dQ_e[0] = rho dU_j/dx_e,
//   J_e dQ_e = (dQ_e[1+e],  dQ_e[1+e] U_j + U_e t_ej + delta_je dp/dx_e,
//               (dQ_e[4] + dp/dx_e) U_e + (rho E + p) dU_e/dx_e),
// and out = -sum_e J_e dQ_e.
template <class T>
DGK_HD Grad<T> prim_grad_dt(const Prim<T>& s, const T Q[5], const T dq[3][5], T gm1, T out[5]) {
  Grad<T> g;
  const T ir = s.ir;
  const T U[3] = {s.U, s.V, s.W};
  const T ke = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
  const T hi = (Q[4] + s.p) * ir;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    T um = T(0), t[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      t[j] = dq[e][1 + j] - U[j] * dq[e][0];
      g.dU[e][j] = t[j] * ir;
      um += U[j] * dq[e][1 + j];
    }
    g.dp[e] = gm1 * (dq[e][4] - um + ke * dq[e][0]);
    g.dT[e] = (g.dp[e] - s.th * dq[e][0]) * ir;
    sub_euler_jvp(e, e == 0, U, dq[e][1 + e], t, g.dp[e], dq[e][4], hi, out);
  }
  return g;
}

// Identity (ii) along axis D, without the factor p.
template <int D, class T>
DGK_HD void ns_moment(const Prim<T>& s, const Grad<T>& g, T two_k3, T cp, T out[5]) {
  const T U[3] = {s.U, s.V, s.W};
  const T div = g.dU[0][0] + g.dU[1][1] + g.dU[2][2];
  T ud = T(0);
  out[0] = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T Dj = g.dU[D][j] + g.dU[j][D];
    if (j == D) Dj -= two_k3 * div;
    out[1 + j] = Dj;
    ud += U[j] * Dj;
  }
  out[4] = ud + cp * g.dT[D];
}

// --------------------------------------------------------------------------
// Face flux, Eq. (flux) in the local frame of the face (normal = axis 0).
// The two sides are processed one after the other (face_side) into the
// accumulators below, then face_finish forms g0, its slopes and the fluxes.
//   Q0   = rho_l <psi>_{u>0, l} + rho_r <psi>_{u<0, r}
//   dQ0_i= rho_l <a_i^l psi>_{u>0} + rho_r <a_i^r psi>_{u<0}
//   m4 = sum rho_k <u psi>_{k}, m5 = sum rho_k <u (a^k.u) psi>_k,
//   m6 = sum rho_k <u A^k psi>_k   (half spaces of the two sides)
//   m1 = rho0 <u psi>_0, m3 = rho0 <u Abar psi>_0, m2 = rho0 <u (abar.u) psi>_0
// --------------------------------------------------------------------------
template <class T>
struct FaceAcc {
  T Q0[5], dQ0[3][5], m4[5], m5[5], m6[5];
};

template <class T>
DGK_HD void face_acc_zero(FaceAcc<T>& a) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    a.Q0[k] = a.m4[k] = a.m5[k] = a.m6[k] = T(0);
    a.dQ0[0][k] = a.dQ0[1][k] = a.dQ0[2][k] = T(0);
  }
}

// Moment matrices of one side.  With the normal velocity u on the side's half
// line (moments M_n = <u^n>, n = 0..6) and the tangential velocities v, w and
// xi^2 Gaussian (independent of u), every entry of
//   H^p_kj = <u^p psi_k psi_j>,  Gv_kj = <u v psi_k psi_j>,  Gw_kj = <u w psi_k psi_j>
// is a closed form in M_n and the transverse moments below (psi_4 = (u^2 + r)/2
// with r = v^2 + w^2 + xi^2).  Matrices are symmetric, stored as the upper
// triangle in row order (00 01 02 03 04 11 12 13 14 22 23 24 33 34 44).
template <class T>
struct Transverse {
  T V, W, v2, w2, v3, w3, R1, R2, vr, wr, v2r, w2r, vwr, vr2, wr2;
  DGK_HD Transverse(T V_, T W_, T th, T K) : V(V_), W(W_) {
    const T t2 = th * th;
    v2 = V * V + th;
    w2 = W * W + th;
    v3 = V * (V * V + T(3) * th);
    w3 = W * (W * W + T(3) * th);
    const T v4 = V * V * (V * V + T(6) * th) + T(3) * t2;
    const T w4 = W * W * (W * W + T(6) * th) + T(3) * t2;
    const T v5 = V * (V * V * (V * V + T(10) * th) + T(15) * t2);
    const T w5 = W * (W * W * (W * W + T(10) * th) + T(15) * t2);
    const T s1 = K * th, s2 = K * (K + T(2)) * t2;
    R1 = v2 + w2 + s1;                                           // <r>
    R2 = v4 + w4 + s2 + T(2) * (v2 * w2 + (v2 + w2) * s1);      // <r^2>
    vr = v3 + V * (w2 + s1);                                     // <v r>
    wr = w3 + W * (v2 + s1);                                     // <w r>
    v2r = v4 + v2 * (w2 + s1);                                   // <v^2 r>
    w2r = w4 + w2 * (v2 + s1);                                   // <w^2 r>
    vwr = v3 * W + V * w3 + V * W * s1;                          // <v w r>
    vr2 = v5 + T(2) * v3 * (w2 + s1) + V * (w4 + s2 + T(2) * w2 * s1);  // <v r^2>
    wr2 = w5 + T(2) * w3 * (v2 + s1) + W * (v4 + s2 + T(2) * v2 * s1);  // <w r^2>
  }
};

template <int P, class T>
DGK_HD void mat_H(const T* M, const Transverse<T>& t, T H[15]) {
  const T h = T(0.5);
  H[0] = M[P];
  H[1] = M[P + 1];
  H[2] = t.V * M[P];
  H[3] = t.W * M[P];
  H[4] = h * (M[P + 2] + t.R1 * M[P]);
  H[5] = M[P + 2];
  H[6] = t.V * M[P + 1];
  H[7] = t.W * M[P + 1];
  H[8] = h * (M[P + 3] + t.R1 * M[P + 1]);
  H[9] = t.v2 * M[P];
  H[10] = t.V * t.W * M[P];
  H[11] = h * (t.V * M[P + 2] + t.vr * M[P]);
  H[12] = t.w2 * M[P];
  H[13] = h * (t.W * M[P + 2] + t.wr * M[P]);
  H[14] = T(0.25) * (M[P + 4] + T(2) * t.R1 * M[P + 2] + t.R2 * M[P]);
}

template <class T>
DGK_HD void mat_Gv(const T* M, const Transverse<T>& t, T G[15]) {
  const T h = T(0.5), VW = t.V * t.W;
  G[0] = t.V * M[1];
  G[1] = t.V * M[2];
  G[2] = t.v2 * M[1];
  G[3] = VW * M[1];
  G[4] = h * (t.V * M[3] + t.vr * M[1]);
  G[5] = t.V * M[3];
  G[6] = t.v2 * M[2];
  G[7] = VW * M[2];
  G[8] = h * (t.V * M[4] + t.vr * M[2]);
  G[9] = t.v3 * M[1];
  G[10] = t.v2 * t.W * M[1];
  G[11] = h * (t.v2 * M[3] + t.v2r * M[1]);
  G[12] = t.V * t.w2 * M[1];
  G[13] = h * (VW * M[3] + t.vwr * M[1]);
  G[14] = T(0.25) * (t.V * M[5] + T(2) * t.vr * M[3] + t.vr2 * M[1]);
}

template <class T>
DGK_HD void mat_Gw(const T* M, const Transverse<T>& t, T G[15]) {
  const T h = T(0.5), VW = t.V * t.W;
  G[0] = t.W * M[1];
  G[1] = t.W * M[2];
  G[2] = VW * M[1];
  G[3] = t.w2 * M[1];
  G[4] = h * (t.W * M[3] + t.wr * M[1]);
  G[5] = t.W * M[3];
  G[6] = VW * M[2];
  G[7] = t.w2 * M[2];
  G[8] = h * (t.W * M[4] + t.wr * M[2]);
  G[9] = t.W * t.v2 * M[1];
  G[10] = t.V * t.w2 * M[1];
  G[11] = h * (VW * M[3] + t.vwr * M[1]);
  G[12] = t.w3 * M[1];
  G[13] = h * (t.w2 * M[3] + t.w2r * M[1]);
  G[14] = T(0.25) * (t.W * M[5] + T(2) * t.wr * M[3] + t.wr2 * M[1]);
}

// y += S x for a symmetric S stored as above, accumulated onto y one product
// at a time (one FMA per entry)
template <class T>
DGK_HD void sym_mv_acc(const T S[15], const T x[5], T y[5]) {
  constexpr int e[5][5] = {{0, 1, 2, 3, 4}, {1, 5, 6, 7, 8}, {2, 6, 9, 10, 11}, {3, 7, 10, 12, 13}, {4, 8, 11, 13, 14}};
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int j = 0; j < 5; ++j) y[k] += S[e[k][j]] * x[j];
}

// y += <u^P psi psi^T> x (P = 0, 1) without forming the matrix.  With
// phi = x.psi = x0 + x1 u + x2 v + x3 w + x4 (u^2 + r)/2 and a = x0 + V x2 + W x3
// + R1 x4 / 2 (the transverse mean part), u and (v, w, xi) independent and
// E[(v - V) r] = 2 V th, E[(w - W) r] = 2 W th, E[(r - R1) r] = R2 - R1^2:
//   e_j = <u^(P+j) phi> = M_{P+j} a + M_{P+j+1} x1 + M_{P+j+2} x4 / 2
//   y0 += e_0,  y1 += e_1,  y2 += V e_0 + M_P th (x2 + V x4),  y3 likewise with W,
//   y4 += e_2 / 2 + R1 e_0 / 2 + M_P th (V x2 + W x3) + M_P (R2 - R1^2) x4 / 4.
// hR1 = R1 / 2 and q4 = (R2 - R1^2) / 4 come from the caller (shared by the
// side's products); each term is added onto y with one FMA.
template <int P, class T>
DGK_HD void hmat_mv_acc(const T* M, const Transverse<T>& t, T th, T hR1, T q4, const T x[5], T y[5]) {
  const T hx4 = T(0.5) * x[4];
  T a = x[0];
  a += t.V * x[2];
  a += t.W * x[3];
  a += hR1 * x[4];
  T e0 = M[P] * a;
  e0 += M[P + 1] * x[1];
  e0 += M[P + 2] * hx4;
  T e2 = M[P + 2] * a;
  e2 += M[P + 3] * x[1];
  e2 += M[P + 4] * hx4;
  const T c = M[P] * th;
  y[0] += e0;
  y[1] += M[P + 1] * a;
  y[1] += M[P + 2] * x[1];
  y[1] += M[P + 3] * hx4;
  y[2] += t.V * e0;
  y[2] += c * (x[2] + t.V * x[4]);
  y[3] += t.W * e0;
  y[3] += c * (x[3] + t.W * x[4]);
  y[4] += T(0.5) * e2;
  y[4] += hR1 * e0;
  y[4] += c * (t.V * x[2] + t.W * x[3]);
  y[4] += (M[P] * q4) * x[4];
}

// m5 += <u psi Phi> with Phi = u (x.psi) + v (y.psi) + w (z.psi), i.e.
// <u^2 psi psi^T> x + <u v psi psi^T> y + <u w psi psi^T> z without forming the
// matrices.  Phi = P0 + P1 u + P2 u^2 + P3 u^3 with coefficients polynomial in
// (v, w, r) (psi_4 = (u^2 + r)/2), and <u^n f(v, w, xi)> = M_n <f>, so
//   m5_0 = sum_j M_{1+j} <P_j>,      m5_1 = sum_j M_{2+j} <P_j>,
//   m5_2 = sum_j M_{1+j} <v P_j>,    m5_3 = sum_j M_{1+j} <w P_j>,
//   m5_4 = sum_j (M_{3+j} <P_j> + M_{1+j} <r P_j>) / 2.
template <class T>
DGK_HD void m5_acc(const T* M, const Transverse<T>& t, const T x[5], const T y[5], const T z[5], T m5[5]) {
  const T hx4 = T(0.5) * x[4], hy4 = T(0.5) * y[4], hz4 = T(0.5) * z[4];
  const T VW = t.V * t.W, v2W = t.v2 * t.W, Vw2 = t.V * t.w2;
  // P3 = x4 / 2
  const T p3 = hx4, vp3 = hx4 * t.V, wp3 = hx4 * t.W, rp3 = hx4 * t.R1;
  // P2 = x1 + (y4 / 2) v + (z4 / 2) w
  const T p2 = x[1] + hy4 * t.V + hz4 * t.W;
  const T vp2 = x[1] * t.V + hy4 * t.v2 + hz4 * VW;
  const T wp2 = x[1] * t.W + hy4 * VW + hz4 * t.w2;
  const T rp2 = x[1] * t.R1 + hy4 * t.vr + hz4 * t.wr;
  // P1 = x0 + (x2 + y1) v + (x3 + z1) w + (x4 / 2) r
  const T d = x[2] + y[1], e = x[3] + z[1];
  const T p1 = x[0] + d * t.V + e * t.W + hx4 * t.R1;
  const T vp1 = x[0] * t.V + d * t.v2 + e * VW + hx4 * t.vr;
  const T wp1 = x[0] * t.W + d * VW + e * t.w2 + hx4 * t.wr;
  const T rp1 = x[0] * t.R1 + d * t.vr + e * t.wr + hx4 * t.R2;
  // P0 = y0 v + z0 w + y2 v^2 + (y3 + z2) v w + z3 w^2 + (y4 / 2) v r + (z4 / 2) w r
  const T c = y[3] + z[2];
  const T p0 = y[0] * t.V + z[0] * t.W + y[2] * t.v2 + c * VW + z[3] * t.w2 + hy4 * t.vr + hz4 * t.wr;
  const T vp0 = y[0] * t.v2 + z[0] * VW + y[2] * t.v3 + c * v2W + z[3] * Vw2 + hy4 * t.v2r + hz4 * t.vwr;
  const T wp0 = y[0] * VW + z[0] * t.w2 + y[2] * v2W + c * Vw2 + z[3] * t.w3 + hy4 * t.vwr + hz4 * t.w2r;
  const T rp0 = y[0] * t.vr + z[0] * t.wr + y[2] * t.v2r + c * t.vwr + z[3] * t.w2r + hy4 * t.vr2 + hz4 * t.wr2;
  // accumulated onto m5 one product at a time
  const T P[4] = {p0, p1, p2, p3}, VP[4] = {vp0, vp1, vp2, vp3}, WP[4] = {wp0, wp1, wp2, wp3};
  const T RP[4] = {rp0, rp1, rp2, rp3};
  T s4 = M[3] * p0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    m5[0] += M[1 + j] * P[j];
    m5[1] += M[2 + j] * P[j];
    m5[2] += M[1 + j] * VP[j];
    m5[3] += M[1 + j] * WP[j];
    if (j > 0) s4 += M[3 + j] * P[j];
    s4 += M[1 + j] * RP[j];
  }
  m5[4] += T(0.5) * s4;
}

// sg = +1: lower cell (half space u > 0); sg = -1: upper cell (u < 0).
template <class T>
DGK_HD void face_side(const Phys& ph, const T q[5], const T dq[3][5], FaceAcc<T>& acc, int& bad, T sg) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> s = primitive(q, gm1);
  bad |= int(unphysical(s));
  const Solver5<T> S(s, K, T(ph.inv_k3));
  // slopes times the density: <a_i psi> = dQ/dn_i / rho and the solve is
  // linear, so ra_i = rho a_i solves <ra_i psi> = dQ/dn_i; likewise rA = rho A
  // from the compatibility condition <rA psi> = -sum_e J_e dQ/dx_e
  T ra[3][5], rA[5], b[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) S(dq[i], ra[i]);
  euler_dt(s, q, gm1, dq, b);
  S(b, rA);
  // half-space moments of the normal velocity, transverse Gaussian moments
  T M[7];
  mom_half(s.U, s.th, sg, M);
  const Transverse<T> tr(s.V, s.W, s.th, K);
  const T r = s.rho;
  if constexpr (sizeof(T) == 4) {
    // rho <psi> and rho <u psi> (the first columns of <psi psi^T>, <u psi psi^T>),
    // then <psi psi^T> ra_i and <u psi psi^T> rA matrix-free: 3% fewer VALU
    // instructions per face point and 2-4% off the FP32 face kernel.  The FP64
    // kernel (one wavefront per SIMD, latency-bound) ran 4-5% slower with it and
    // keeps the matrices.
    const T hR1 = T(0.5) * tr.R1, q4 = T(0.25) * (tr.R2 - tr.R1 * tr.R1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const T rm = r * M[p], rm1 = r * M[p + 1];
      T* o = p ? acc.m4 : acc.Q0;
      o[0] += rm;
      o[1] += rm1;
      o[2] += tr.V * rm;
      o[3] += tr.W * rm;
      o[4] += T(0.5) * (r * M[p + 2]) + hR1 * rm;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) hmat_mv_acc<0>(M, tr, s.th, hR1, q4, ra[i], acc.dQ0[i]);
    hmat_mv_acc<1>(M, tr, s.th, hR1, q4, rA, acc.m6);
  } else {
    T H[15];
    mat_H<0>(M, tr, H);  // <psi psi^T>
    acc.Q0[0] += r * H[0];
    acc.Q0[1] += r * H[1];
    acc.Q0[2] += r * H[2];
    acc.Q0[3] += r * H[3];
    acc.Q0[4] += r * H[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) sym_mv_acc(H, ra[i], acc.dQ0[i]);
    mat_H<1>(M, tr, H);  // <u psi psi^T>
    acc.m4[0] += r * H[0];
    acc.m4[1] += r * H[1];
    acc.m4[2] += r * H[2];
    acc.m4[3] += r * H[3];
    acc.m4[4] += r * H[4];
    sym_mv_acc(H, rA, acc.m6);
  }
  // <u^2 psi psi^T> ra_0 + <u v psi psi^T> ra_1 + <u w psi psi^T> ra_2
  m5_acc(M, tr, ra[0], ra[1], ra[2], acc.m5);
}

// ec: the constants of exp_neg_tab (LDS in the face kernel).
template <class T, bool NEED_F>
DGK_HD void face_finish(const Phys& ph, const FaceAcc<T>& acc, T F[5], T Ft[5], int& bad, const double* ec) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> s0 = primitive(acc.Q0, gm1);
  bad |= int(unphysical(s0));
  T m1[5], m2[5], m3[5], dt0[5];
  euler_flux<0>(s0, acc.Q0, m1);
  const Grad<T> g = prim_grad_dt(s0, acc.Q0, acc.dQ0, gm1, dt0);  // dt0 = rho0 <Abar psi>
  euler_jvp<0>(s0, acc.Q0, gm1, dt0, m3);
  T ns[5];
  ns_moment<0>(s0, g, T(2.0 * ph.inv_k3), T(ph.cp), ns);  // (m2 + m3) / p0
#pragma unroll
  for (int k = 0; k < 5; ++k) m2[k] = s0.p * ns[k] - m3[k];

  const double tau = ph.mu * d_rcp(double(s0.p));
  double al[6], be[6];
  time_coefficients(tau, ph.half_dt_over_mu * double(s0.p), ph.dt, ph.inv_dt, al, be, ec);
  // beta_3 = -beta_0, beta_4 = -beta_1, alpha_3 = 1 - alpha_0, alpha_4 = -tau - alpha_1:
  //   Ft = beta_0 (m1 - m4) + beta_1 (m2 - m5) + beta_2 m3 + beta_5 m6
  //   F  = m4 + alpha_0 (m1 - m4) + alpha_1 (m2 - m5) - tau m5 + alpha_2 m3 + alpha_5 m6
  // The combination runs in T with the FP64 coefficients rounded once: in
  // FP32-bulk, forming it in FP64 instead changed the Taylor-Green errors
  // (state and increment) by under 0.5% and cost 1.7% of the step.
  const T b0 = T(be[0]), b1 = T(be[1]), b2 = T(be[2]), b5 = T(be[5]);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const T d14 = m1[k] - acc.m4[k], d25 = m2[k] - acc.m5[k];
    Ft[k] = b0 * d14 + b1 * d25 + b2 * m3[k] + b5 * acc.m6[k];
    if constexpr (NEED_F)
      F[k] = acc.m4[k] + T(al[0]) * d14 + T(al[1]) * d25 - T(tau) * acc.m5[k] + T(al[2]) * m3[k] + T(al[5]) * acc.m6[k];
  }
  if constexpr (NEED_F) {
    // Prandtl fix: the heat flux of -tau g0 (abar.u + Abar) is
    // q = -tau p0 c_p dT0/dn = -mu c_p dT0/dn; add (1/Pr - 1) q.
    F[4] += T(-ph.inv_pr_m1 * ph.mu * ph.cp) * g.dT[0];
  }
}

template <class T, bool NEED_F>
DGK_HD void face_flux_local(const Phys& ph, const T qL[5], const T dqL[3][5], const T qR[5], const T dqR[3][5],
                            T F[5], T Ft[5], int& bad) {
  FaceAcc<T> acc;
  face_acc_zero(acc);
  face_side(ph, qL, dqL, acc, bad, T(1));
  face_side(ph, qR, dqR, acc, bad, T(-1));
  face_finish<T, NEED_F>(ph, acc, F, Ft, bad, ExpTabHolder<>::t.c);
}

// --------------------------------------------------------------------------
// Volume flux, Eq. (flux-2), global frame.  By identities (i), (ii) its
// moments are F_d = F_d^Euler(Q) - mu (0, D_d, U.D_d + c_p/Pr dT/dx_d) and
// Ft_d = J_d(Q) rho <A psi> with rho <A psi> = -sum_e J_e(Q) dQ/dx_e.
// --------------------------------------------------------------------------
template <class T, bool NEED_F>
DGK_HD void volume_flux(const Phys& ph, const T q[5], const T dq[3][5], T F[3][5], T Ft[3][5], int& bad) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> s = primitive(q, gm1);
  bad |= int(unphysical(s));
  T dt[5];
  Grad<T> g;  // stage 1 shares the gradients with the time derivative
  if constexpr (NEED_F)
    g = prim_grad_dt(s, q, dq, gm1, dt);
  else
    euler_dt_sum(s, q, gm1, dq, dt);
  euler_jvp<0>(s, q, gm1, dt, Ft[0]);
  euler_jvp<1>(s, q, gm1, dt, Ft[1]);
  euler_jvp<2>(s, q, gm1, dt, Ft[2]);
  if constexpr (NEED_F) {
    const T mu = T(ph.mu);
    const T heat = mu * T(ph.inv_pr_m1) * T(ph.cp);  // extra heat-flux factor of 1/Pr - 1
    static_for<3>([&](auto dc) {
      constexpr int d = decltype(dc)::value;
      T e[5], ns[5];
      euler_flux<d>(s, q, e);
      ns_moment<d>(s, g, T(2.0 * ph.inv_k3), T(ph.cp), ns);
#pragma unroll
      for (int k = 0; k < 5; ++k) F[d][k] = e[k] - mu * ns[k];
      F[d][4] -= heat * g.dT[d];
    });
  }
}

}  // namespace dgk
