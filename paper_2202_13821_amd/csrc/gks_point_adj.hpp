// gks_point_adj.hpp -- hand-written reverse mode (vector-Jacobian products)
// of the point fluxes in gks_point.hpp.
//
// Every forward building block f: x -> y has a companion f_bwd that, given
// the forward inputs (it recomputes what it needs) and the cotangent ybar,
// ADDS x^T-contributions into the input cotangents (accumulation semantics).
// The derivatives are those of the exact functions (erfc' = -2/sqrt(pi)
// exp(-x^2), d/dx exp = exp, ...), also where the forward evaluates them with
// a hardware approximation in FP32-bulk mode.
#pragma once

#include "gks_point.hpp"

namespace dgk {

template <class T>
DGK_HD void zero5(T a[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) a[k] = T(0);
}

// ---- primitive variables ----------------------------------------------------
template <class T>
DGK_HD Prim<T> prim_zero() {
  Prim<T> b;
  b.rho = b.ir = b.U = b.V = b.W = b.th = b.p = T(0);
  return b;
}

// rho = Q0, ir = 1/Q0, U_j = Q_{1+j} ir, p = gm1 (Q4 - (Q1 U + Q2 V + Q3 W)/2), th = p ir
template <class T>
DGK_HD void prim_bwd(const T Q[5], const Prim<T>& s, Prim<T> sb, T gm1, T Qb[5]) {
  // th = p ir
  sb.p += sb.th * s.ir;
  sb.ir += sb.th * s.p;
  // p
  const T hp = T(0.5) * gm1 * sb.p;
  Qb[4] += gm1 * sb.p;
  Qb[1] -= hp * s.U;
  Qb[2] -= hp * s.V;
  Qb[3] -= hp * s.W;
  sb.U -= hp * Q[1];
  sb.V -= hp * Q[2];
  sb.W -= hp * Q[3];
  // U_j = Q_j ir
  Qb[1] += sb.U * s.ir;
  Qb[2] += sb.V * s.ir;
  Qb[3] += sb.W * s.ir;
  sb.ir += sb.U * Q[1] + sb.V * Q[2] + sb.W * Q[3];
  // ir = 1/Q0, rho = Q0
  Qb[0] += sb.rho - sb.ir * s.ir * s.ir;
}

// ---- moment tables ------------------------------------------------------------
template <class T>
DGK_HD void mom_zero(Mom<T>& b) {
#pragma unroll
  for (int i = 0; i < 7; ++i) b.u[i] = b.v[i] = b.w[i] = T(0);
  b.x2 = b.x4 = T(0);
}

// m_{n+2} = U m_{n+1} + (n+1) th m_n, n = 0..4, from m_0, m_1.
template <class T>
DGK_HD void mom_rec_bwd(T U, T th, const T* m, T* mb, T& Ub, T& thb) {
#pragma unroll
  for (int n = 4; n >= 0; --n) {
    const T g = mb[n + 2];
    mb[n + 1] += U * g;
    Ub += m[n + 1] * g;
    mb[n] += T(n + 1) * th * g;
    thb += T(n + 1) * m[n] * g;
  }
}

template <class T>
DGK_HD void mom_full_bwd(T U, T th, const T* m, T* mb, T& Ub, T& thb) {
  mom_rec_bwd(U, th, m, mb, Ub, thb);
  Ub += mb[1];  // m_1 = U; m_0 = 1 is constant
}

template <class T>
DGK_HD void mom_half_bwd(T U, T th, int side, const T* m, T* mb, T& Ub, T& thb) {
  mom_rec_bwd(U, th, m, mb, Ub, thb);
  const T r = d_rsqrt(T(2) * th);
  const T a = U * r;
  const T E = d_exp_bulk(-a * a);
  const T c0 = T(0.56418958354775628695);  // 1/sqrt(pi)
  const T sg = side > 0 ? T(1) : T(-1);
  // m1 = U m0 + sg e
  Ub += m[0] * mb[1];
  mb[0] += U * mb[1];
  const T eb = sg * mb[1];
  // m0 = erfc(-sg a)/2, d m0/da = sg E / sqrt(pi)
  T ab = mb[0] * sg * c0 * E;
  // e = E th r c0
  const T Eb = eb * th * r * c0;
  thb += eb * E * r * c0;
  T rb = eb * E * th * c0;
  ab += Eb * E * (T(-2) * a);
  // a = U r
  Ub += ab * r;
  rb += ab * U;
  // r = (2 th)^(-1/2), dr/dth = -r^3
  thb -= rb * r * r * r;
}

template <class T>
DGK_HD void mom_xi_bwd(T K, T th, const Mom<T>& tb, T& thb) {
  thb += tb.x2 * K + tb.x4 * T(2) * K * (K + T(2)) * th;
}

// Mo<a,b,c,d> = u[a] v[b] w[c] x[d]
template <int a, int b, int c, int d, class T>
DGK_HD void Mo_bwd(const Mom<T>& t, T g, Mom<T>& tb) {
  T fv = T(1), fw = T(1), fx = T(1);
  if constexpr (b > 0) fv = t.v[b];
  if constexpr (c > 0) fw = t.w[c];
  if constexpr (d == 1) fx = t.x2;
  if constexpr (d == 2) fx = t.x4;
  const T ua = t.u[a];
  tb.u[a] += g * fv * fw * fx;
  if constexpr (b > 0) tb.v[b] += g * ua * fw * fx;
  if constexpr (c > 0) tb.w[c] += g * ua * fv * fx;
  if constexpr (d == 1) tb.x2 += g * ua * fv * fw;
  if constexpr (d == 2) tb.x4 += g * ua * fv * fw;
}

template <int a, int b, int c, int d, class T>
DGK_HD void Gs_bwd(const Mom<T>& t, const T s[5], T g, Mom<T>& tb, T sb[5]) {
  sb[0] += g * Mo<a, b, c, d>(t);
  sb[1] += g * Mo<a + 1, b, c, d>(t);
  sb[2] += g * Mo<a, b + 1, c, d>(t);
  sb[3] += g * Mo<a, b, c + 1, d>(t);
  sb[4] += g * T(0.5) * (Mo<a + 2, b, c, d>(t) + Mo<a, b + 2, c, d>(t) + Mo<a, b, c + 2, d>(t) + Mo<a, b, c, d + 1>(t));
  Mo_bwd<a, b, c, d>(t, g * s[0], tb);
  Mo_bwd<a + 1, b, c, d>(t, g * s[1], tb);
  Mo_bwd<a, b + 1, c, d>(t, g * s[2], tb);
  Mo_bwd<a, b, c + 1, d>(t, g * s[3], tb);
  const T h = T(0.5) * g * s[4];
  Mo_bwd<a + 2, b, c, d>(t, h, tb);
  Mo_bwd<a, b + 2, c, d>(t, h, tb);
  Mo_bwd<a, b, c + 2, d>(t, h, tb);
  Mo_bwd<a, b, c, d + 1>(t, h, tb);
}

template <int a, int b, int c, class T>
DGK_HD void Gpsi_bwd(const Mom<T>& t, const T s[5], const T ob[5], Mom<T>& tb, T sb[5]) {
  Gs_bwd<a, b, c, 0>(t, s, ob[0], tb, sb);
  Gs_bwd<a + 1, b, c, 0>(t, s, ob[1], tb, sb);
  Gs_bwd<a, b + 1, c, 0>(t, s, ob[2], tb, sb);
  Gs_bwd<a, b, c + 1, 0>(t, s, ob[3], tb, sb);
  const T h = T(0.5) * ob[4];
  Gs_bwd<a + 2, b, c, 0>(t, s, h, tb, sb);
  Gs_bwd<a, b + 2, c, 0>(t, s, h, tb, sb);
  Gs_bwd<a, b, c + 2, 0>(t, s, h, tb, sb);
  Gs_bwd<a, b, c, 1>(t, s, h, tb, sb);
}

template <int a, int b, int c, class T>
DGK_HD void psim_bwd(const Mom<T>& t, const T ob[5], Mom<T>& tb) {
  Mo_bwd<a, b, c, 0>(t, ob[0], tb);
  Mo_bwd<a + 1, b, c, 0>(t, ob[1], tb);
  Mo_bwd<a, b + 1, c, 0>(t, ob[2], tb);
  Mo_bwd<a, b, c + 1, 0>(t, ob[3], tb);
  const T h = T(0.5) * ob[4];
  Mo_bwd<a + 2, b, c, 0>(t, h, tb);
  Mo_bwd<a, b + 2, c, 0>(t, h, tb);
  Mo_bwd<a, b, c + 2, 0>(t, h, tb);
  Mo_bwd<a, b, c, 1>(t, h, tb);
}

// ---- closed-form 5x5 solve --------------------------------------------------------
template <class T>
struct Solver5Bar {
  T U, V, W, ith, E, c4;
  DGK_HD Solver5Bar() : U(0), V(0), W(0), ith(0), E(0), c4(0) {}
};

// a = S(b); given abar adds bbar and the solver-parameter cotangents.
template <class T>
DGK_HD void solve_bwd(const Solver5<T>& S, const T b[5], const T a[5], const T ab_in[5], T bb[5], Solver5Bar<T>& Sb) {
  T ab[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) ab[k] = ab_in[k];
  const T R1 = b[1] - S.U * b[0], R2 = b[2] - S.V * b[0], R3 = b[3] - S.W * b[0];
  // a0 = b0 - U a1 - V a2 - W a3 - E a4
  bb[0] += ab[0];
  Sb.U -= ab[0] * a[1];
  Sb.V -= ab[0] * a[2];
  Sb.W -= ab[0] * a[3];
  Sb.E -= ab[0] * a[4];
  ab[1] -= S.U * ab[0];
  ab[2] -= S.V * ab[0];
  ab[3] -= S.W * ab[0];
  ab[4] -= S.E * ab[0];
  // a_i = R_i ith - U_i a4
  T R1b = ab[1] * S.ith, R2b = ab[2] * S.ith, R3b = ab[3] * S.ith;
  Sb.ith += ab[1] * R1 + ab[2] * R2 + ab[3] * R3;
  Sb.U -= ab[1] * a[4];
  Sb.V -= ab[2] * a[4];
  Sb.W -= ab[3] * a[4];
  ab[4] -= S.U * ab[1] + S.V * ab[2] + S.W * ab[3];
  // a4 = c4 X, X = b4 - E b0 - U R1 - V R2 - W R3
  const T X = b[4] - S.E * b[0] - S.U * R1 - S.V * R2 - S.W * R3;
  Sb.c4 += ab[4] * X;
  const T Xb = ab[4] * S.c4;
  bb[4] += Xb;
  Sb.E -= Xb * b[0];
  bb[0] -= Xb * S.E;
  Sb.U -= Xb * R1;
  Sb.V -= Xb * R2;
  Sb.W -= Xb * R3;
  R1b -= Xb * S.U;
  R2b -= Xb * S.V;
  R3b -= Xb * S.W;
  // R_i = b_{i} - U_i b0
  bb[1] += R1b;
  bb[2] += R2b;
  bb[3] += R3b;
  Sb.U -= R1b * b[0];
  Sb.V -= R2b * b[0];
  Sb.W -= R3b * b[0];
  bb[0] -= R1b * S.U + R2b * S.V + R3b * S.W;
}

// Solver5 constructor: ith = 1/th, E = |U|^2/2 + (K+3) th/2, c4 = 2 ith^2 / (K+3)
template <class T>
DGK_HD void solver_ctor_bwd(const Solver5<T>& S, const Solver5Bar<T>& Sb, T K, T inv_k3, Prim<T>& sb) {
  T ithb = Sb.ith + Sb.c4 * T(4) * S.ith * inv_k3;
  sb.U += Sb.U + Sb.E * S.U;
  sb.V += Sb.V + Sb.E * S.V;
  sb.W += Sb.W + Sb.E * S.W;
  sb.th += Sb.E * T(0.5) * (K + T(3)) - ithb * S.ith * S.ith;
}

// ---- Euler flux and its derivatives ------------------------------------------------
template <int D, class T>
DGK_HD void euler_flux_bwd(const Prim<T>& s, const T Q[5], const T Fb[5], Prim<T>& sb, T Qb[5]) {
  const T U[3] = {s.U, s.V, s.W};
  const T Ud = U[D];
  Qb[1 + D] += Fb[0];
  T udb = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Qb[1 + j] += Fb[1 + j] * Ud;
    udb += Fb[1 + j] * Q[1 + j];
  }
  sb.p += Fb[1 + D] + Fb[4] * Ud;
  Qb[4] += Fb[4] * Ud;
  udb += Fb[4] * (Q[4] + s.p);
  if constexpr (D == 0) sb.U += udb;
  if constexpr (D == 1) sb.V += udb;
  if constexpr (D == 2) sb.W += udb;
}

// out = J_D(Q) v; adds vbar, and the Q-derivative through (U, ir, p, Q4).
template <int D, class T>
DGK_HD void euler_jvp_bwd(const Prim<T>& s, const T Q[5], T gm1, const T v[5], const T ob[5], T vb[5], Prim<T>& sb,
                          T Qb[5]) {
  const T U[3] = {s.U, s.V, s.W};
  T Ub[3] = {T(0), T(0), T(0)};
  const T ir = s.ir;
  const T Ud = U[D];
  const T kk = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
  T um = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) um += U[j] * v[1 + j];
  const T dp = gm1 * (v[4] - um + kk * v[0]);
  const T dUd = (v[1 + D] - Ud * v[0]) * ir;
  // out4 = (v4 + dp) U_D + (Q4 + p) dU_D
  T dpb = ob[4] * Ud;
  vb[4] += ob[4] * Ud;
  Ub[D] += ob[4] * (v[4] + dp);
  Qb[4] += ob[4] * dUd;
  sb.p += ob[4] * dUd;
  const T dUdb = ob[4] * (Q[4] + s.p);
  // out_{1+D} += dp
  dpb += ob[1 + D];
  // out_{1+j} = v_{1+D} U_j + U_D (v_{1+j} - U_j v0)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T g = ob[1 + j];
    vb[1 + D] += g * U[j];
    Ub[j] += g * v[1 + D] - g * Ud * v[0];
    Ub[D] += g * (v[1 + j] - U[j] * v[0]);
    vb[1 + j] += g * Ud;
    vb[0] -= g * Ud * U[j];
  }
  // out0 = v_{1+D}
  vb[1 + D] += ob[0];
  // dp = gm1 (v4 - um + kk v0)
  vb[4] += dpb * gm1;
  const T umb = -dpb * gm1;
  const T kkb = dpb * gm1 * v[0];
  vb[0] += dpb * gm1 * kk;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Ub[j] += kkb * U[j] + umb * v[1 + j];
    vb[1 + j] += umb * U[j];
  }
  // dU_D = (v_{1+D} - U_D v0) ir
  vb[1 + D] += dUdb * ir;
  Ub[D] -= dUdb * v[0] * ir;
  vb[0] -= dUdb * Ud * ir;
  sb.ir += dUdb * (v[1 + D] - Ud * v[0]);
  sb.U += Ub[0];
  sb.V += Ub[1];
  sb.W += Ub[2];
}

template <class T>
DGK_HD void euler_dt_bwd(const Prim<T>& s, const T Q[5], T gm1, const T dq[3][5], const T ob[5], T dqb[3][5],
                         Prim<T>& sb, T Qb[5]) {
  T m[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) m[k] = -ob[k];
  euler_jvp_bwd<0>(s, Q, gm1, dq[0], m, dqb[0], sb, Qb);
  euler_jvp_bwd<1>(s, Q, gm1, dq[1], m, dqb[1], sb, Qb);
  euler_jvp_bwd<2>(s, Q, gm1, dq[2], m, dqb[2], sb, Qb);
}

template <class T>
DGK_HD Grad<T> grad_zero() {
  Grad<T> g;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    g.dp[e] = g.dT[e] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) g.dU[e][j] = T(0);
  }
  return g;
}

template <class T>
DGK_HD void prim_grad_bwd(const Prim<T>& s, const T dq[3][5], T gm1, const Grad<T>& g, Grad<T> gb, T dqb[3][5],
                          Prim<T>& sb) {
  const T U[3] = {s.U, s.V, s.W};
  T Ub[3] = {T(0), T(0), T(0)};
  const T ir = s.ir;
  const T ke = T(0.5) * (s.U * s.U + s.V * s.V + s.W * s.W);
  T keb = T(0);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    // dT = (dp - th dq0) ir
    gb.dp[e] += gb.dT[e] * ir;
    sb.th -= gb.dT[e] * dq[e][0] * ir;
    dqb[e][0] -= gb.dT[e] * s.th * ir;
    sb.ir += gb.dT[e] * (g.dp[e] - s.th * dq[e][0]);
    // dp = gm1 (dq4 - um + ke dq0)
    dqb[e][4] += gb.dp[e] * gm1;
    const T umb = -gb.dp[e] * gm1;
    keb += gb.dp[e] * gm1 * dq[e][0];
    dqb[e][0] += gb.dp[e] * gm1 * ke;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Ub[j] += umb * dq[e][1 + j];
      dqb[e][1 + j] += umb * U[j];
      // dU = (dq_{1+j} - U_j dq0) ir
      const T gj = gb.dU[e][j];
      dqb[e][1 + j] += gj * ir;
      Ub[j] -= gj * dq[e][0] * ir;
      dqb[e][0] -= gj * U[j] * ir;
      sb.ir += gj * (dq[e][1 + j] - U[j] * dq[e][0]);
    }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) Ub[j] += keb * U[j];
  sb.U += Ub[0];
  sb.V += Ub[1];
  sb.W += Ub[2];
}

template <int D, class T>
DGK_HD void ns_moment_bwd(const Prim<T>& s, const Grad<T>& g, T two_k3, T cp, const T ob[5], Prim<T>& sb, Grad<T>& gb) {
  const T U[3] = {s.U, s.V, s.W};
  const T div = g.dU[0][0] + g.dU[1][1] + g.dU[2][2];
  T divb = T(0);
  gb.dT[D] += ob[4] * cp;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T Dj = g.dU[D][j] + g.dU[j][D];
    if (j == D) Dj -= two_k3 * div;
    const T Djb = ob[1 + j] + ob[4] * U[j];
    if (j == 0) sb.U += ob[4] * Dj;
    if (j == 1) sb.V += ob[4] * Dj;
    if (j == 2) sb.W += ob[4] * Dj;
    gb.dU[D][j] += Djb;
    gb.dU[j][D] += Djb;
    if (j == D) divb -= two_k3 * Djb;
  }
  gb.dU[0][0] += divb;
  gb.dU[1][1] += divb;
  gb.dU[2][2] += divb;
}

// ---- time-integral coefficients (FP64) ---------------------------------------------
// Given the cotangents of alpha and beta, add those of tau and x_half.
DGK_HD void time_coefficients_bwd(double tau, double x_half, double dt, double inv_dt, const double alb[6],
                                  const double beb[6], double& taub, double& xb) {
  const double e2 = tau > 0.0 ? exp(-x_half) : 0.0;
  const double e1 = e2 * e2;
  const double idt = inv_dt, idt2 = 4.0 * idt * idt;
  const double dl[2] = {dt, 0.5 * dt};
  const double ee[2] = {e1, e2};
  double eb[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double d = dl[j], e = ee[j], om = 1.0 - e;
    double cb[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) cb[i] = (j == 0) ? (-alb[i] * idt + beb[i] * idt2) : (4.0 * alb[i] * idt - 2.0 * beb[i] * idt2);
    double omb = 0.0;
    taub += -cb[0] * om;
    omb += -cb[0] * tau;
    taub += cb[1] * (4.0 * tau - d - (4.0 * tau + d) * e);
    eb[j] += -cb[1] * tau * (2.0 * tau + d);
    taub += cb[2] * (-d + 2.0 * tau * om);
    omb += cb[2] * tau * tau;
    taub += cb[3] * om;
    omb += cb[3] * tau;
    taub += cb[4] * (-4.0 * tau + (4.0 * tau + d) * e);
    eb[j] += cb[4] * tau * (2.0 * tau + d);
    taub += -cb[5] * 2.0 * tau * om;
    omb += -cb[5] * tau * tau;
    eb[j] -= omb;
  }
  if (tau > 0.0) {
    const double e2b = eb[1] + eb[0] * 2.0 * e2;
    xb += -e2b * e2;
  }
}

// ---- volume flux ------------------------------------------------------------------------
template <class T, bool NEED_F>
DGK_HD void volume_flux_vjp(const Phys& ph, const T q[5], const T dq[3][5], const T Fb[3][5], const T Ftb[3][5],
                            T qb[5], T dqb[3][5], double& mub) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const Prim<T> s = primitive(q, gm1);
  Prim<T> sb = prim_zero<T>();
  T dt[5], dtb[5];
  euler_dt(s, q, gm1, dq, dt);
  zero5(dtb);
  euler_jvp_bwd<0>(s, q, gm1, dt, Ftb[0], dtb, sb, qb);
  euler_jvp_bwd<1>(s, q, gm1, dt, Ftb[1], dtb, sb, qb);
  euler_jvp_bwd<2>(s, q, gm1, dt, Ftb[2], dtb, sb, qb);
  if constexpr (NEED_F) {
    const Grad<T> g = prim_grad(s, dq, gm1);
    Grad<T> gb = grad_zero<T>();
    const T mu = T(ph.mu);
    const T two_k3 = T(2.0 * ph.inv_k3), cp = T(ph.cp);
    const T heatc = T(ph.inv_pr_m1) * cp;
    double mb = 0.0;
    static_for<3>([&](auto dc) {
      constexpr int d = decltype(dc)::value;
      T ns[5], nsb[5];
      ns_moment<d>(s, g, two_k3, cp, ns);
      euler_flux_bwd<d>(s, q, Fb[d], sb, qb);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        nsb[k] = -mu * Fb[d][k];
        mb -= double(Fb[d][k]) * double(ns[k]);
      }
      ns_moment_bwd<d>(s, g, two_k3, cp, nsb, sb, gb);
      // F_d[4] -= mu (1/Pr - 1) cp dT_d
      gb.dT[d] -= mu * heatc * Fb[d][4];
      mb -= double(heatc) * double(g.dT[d]) * double(Fb[d][4]);
    });
    mub += mb;
    prim_grad_bwd(s, dq, gm1, g, gb, dqb, sb);
  }
  euler_dt_bwd(s, q, gm1, dq, dtb, dqb, sb, qb);
  prim_bwd(q, s, sb, gm1, qb);
  (void)K;
}

// ---- face flux ------------------------------------------------------------------------------
template <class T>
DGK_HD void face_acc_zero_bar(FaceAcc<T>& a) {
  face_acc_zero(a);
}

// Reverse of face_side: accb holds the cotangents of the accumulators.
template <int SIDE, class T>
DGK_HD void face_side_vjp(const Phys& ph, const T q[5], const T dq[3][5], const FaceAcc<T>& accb, T qb[5],
                          T dqb[3][5]) {
  const T K = T(ph.K), gm1 = T(ph.gm1), inv_k3 = T(ph.inv_k3);
  const Prim<T> s = primitive(q, gm1);
  const Solver5<T> S(s, K, inv_k3);
  const T ir = s.ir;
  T a[3][5], A[5], b[3][5], bA[5], dtq[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int k = 0; k < 5; ++k) b[i][k] = dq[i][k] * ir;
    S(b[i], a[i]);
  }
  euler_dt(s, q, gm1, dq, dtq);
#pragma unroll
  for (int k = 0; k < 5; ++k) bA[k] = dtq[k] * ir;
  S(bA, A);
  Mom<T> h;
  mom_half(s.U, s.th, SIDE, h.u);
  mom_full(s.V, s.th, h.v);
  mom_full(s.W, s.th, h.w);
  mom_xi(K, s.th, h);
  const T r = s.rho;

  Prim<T> sb = prim_zero<T>();
  Mom<T> hb;
  mom_zero(hb);
  T ab[3][5], Ab[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) zero5(ab[i]);
  zero5(Ab);
  T y[5], g[5];
  T rb = T(0);
  // Q0 += r psim<0,0,0>(h)
  psim<0, 0, 0>(h, y);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    rb += accb.Q0[k] * y[k];
    g[k] = r * accb.Q0[k];
  }
  psim_bwd<0, 0, 0>(h, g, hb);
  // dQ0[i] += r Gpsi<0,0,0>(h, a_i)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Gpsi<0, 0, 0>(h, a[i], y);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      rb += accb.dQ0[i][k] * y[k];
      g[k] = r * accb.dQ0[i][k];
    }
    Gpsi_bwd<0, 0, 0>(h, a[i], g, hb, ab[i]);
  }
  // m4 += r psim<1,0,0>(h)
  psim<1, 0, 0>(h, y);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    rb += accb.m4[k] * y[k];
    g[k] = r * accb.m4[k];
  }
  psim_bwd<1, 0, 0>(h, g, hb);
  // m5 += r (Gpsi<2,0,0>(h,a0) + Gpsi<1,1,0>(h,a1) + Gpsi<1,0,1>(h,a2))
  {
    T z0[5], z1[5], z2[5];
    Gpsi<2, 0, 0>(h, a[0], z0);
    Gpsi<1, 1, 0>(h, a[1], z1);
    Gpsi<1, 0, 1>(h, a[2], z2);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      rb += accb.m5[k] * (z0[k] + z1[k] + z2[k]);
      g[k] = r * accb.m5[k];
    }
    Gpsi_bwd<2, 0, 0>(h, a[0], g, hb, ab[0]);
    Gpsi_bwd<1, 1, 0>(h, a[1], g, hb, ab[1]);
    Gpsi_bwd<1, 0, 1>(h, a[2], g, hb, ab[2]);
  }
  // m6 += r Gpsi<1,0,0>(h, A)
  Gpsi<1, 0, 0>(h, A, y);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    rb += accb.m6[k] * y[k];
    g[k] = r * accb.m6[k];
  }
  Gpsi_bwd<1, 0, 0>(h, A, g, hb, Ab);
  sb.rho += rb;
  // moment tables
  mom_half_bwd(s.U, s.th, SIDE, h.u, hb.u, sb.U, sb.th);
  mom_full_bwd(s.V, s.th, h.v, hb.v, sb.V, sb.th);
  mom_full_bwd(s.W, s.th, h.w, hb.w, sb.W, sb.th);
  mom_xi_bwd(K, s.th, hb, sb.th);
  // time slope A = S(dt/rho), dt = -sum_e J_e dq_e
  Solver5Bar<T> Sb;
  T bAb[5], dtqb[5];
  zero5(bAb);
  solve_bwd(S, bA, A, Ab, bAb, Sb);
  T irb = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    dtqb[k] = bAb[k] * ir;
    irb += bAb[k] * dtq[k];
  }
  euler_dt_bwd(s, q, gm1, dq, dtqb, dqb, sb, qb);
  // slopes a_i = S(dq_i / rho)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T bb[5];
    zero5(bb);
    solve_bwd(S, b[i], a[i], ab[i], bb, Sb);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      dqb[i][k] += bb[k] * ir;
      irb += bb[k] * dq[i][k];
    }
  }
  sb.ir += irb;
  solver_ctor_bwd(S, Sb, K, inv_k3, sb);
  prim_bwd(q, s, sb, gm1, qb);
}

// Reverse of face_finish.  Fb may be null when NEED_F is false.
template <class T, bool NEED_F>
DGK_HD void face_finish_vjp(const Phys& ph, const FaceAcc<T>& acc, const T Fb[5], const T Ftb[5], FaceAcc<T>& accb,
                            double& mub) {
  const T K = T(ph.K), gm1 = T(ph.gm1);
  const T two_k3 = T(2.0 * ph.inv_k3), cp = T(ph.cp);
  const Prim<T> s0 = primitive(acc.Q0, gm1);
  T m1[5], m2[5], m3[5], dt0[5], ns[5];
  euler_flux<0>(s0, acc.Q0, m1);
  euler_dt(s0, acc.Q0, gm1, acc.dQ0, dt0);
  euler_jvp<0>(s0, acc.Q0, gm1, dt0, m3);
  const Grad<T> g = prim_grad(s0, acc.dQ0, gm1);
  ns_moment<0>(s0, g, two_k3, cp, ns);
#pragma unroll
  for (int k = 0; k < 5; ++k) m2[k] = s0.p * ns[k] - m3[k];
  const double p0 = double(s0.p);
  const double ip0 = 1.0 / p0;
  const double tau = ph.mu * ip0, xh = ph.half_dt_over_mu * p0;
  double al[6], be[6];
  time_coefficients(tau, xh, ph.dt, ph.inv_dt, al, be);
  const T* mm[6] = {m1, m2, m3, acc.m4, acc.m5, acc.m6};
  double alb[6], beb[6];
  T mb[6][5];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double sa = 0.0, sbv = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double f = NEED_F ? double(Fb[k]) : 0.0;
      sa += f * double(mm[j][k]);
      sbv += double(Ftb[k]) * double(mm[j][k]);
      mb[j][k] = T(be[j] * double(Ftb[k]) + al[j] * f);
    }
    alb[j] = sa;
    beb[j] = sbv;
  }
  Prim<T> sb = prim_zero<T>();
  Grad<T> gb = grad_zero<T>();
  if constexpr (NEED_F) {
    // F4 += (1/Pr - 1) (-mu cp dT0/dn)
    gb.dT[0] -= T(ph.inv_pr_m1 * ph.mu * ph.cp * double(Fb[4]));
    mub -= ph.inv_pr_m1 * ph.cp * double(g.dT[0]) * double(Fb[4]);
  }
  double taub = 0.0, xb = 0.0;
  time_coefficients_bwd(tau, xh, ph.dt, ph.inv_dt, alb, beb, taub, xb);
  double p0b = xb * ph.half_dt_over_mu - taub * ph.mu * ip0 * ip0;
  mub += taub * ip0;
  if (ph.mu > 0.0) mub -= xb * p0 * ph.half_dt_over_mu / ph.mu;
  // m2 = p0 ns - m3
  T nsb[5], m3b[5], dt0b[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    p0b += double(mb[1][k]) * double(ns[k]);
    nsb[k] = s0.p * mb[1][k];
    m3b[k] = mb[2][k] - mb[1][k];
  }
  sb.p += T(p0b);
  ns_moment_bwd<0>(s0, g, two_k3, cp, nsb, sb, gb);
  prim_grad_bwd(s0, acc.dQ0, gm1, g, gb, accb.dQ0, sb);
  zero5(dt0b);
  euler_jvp_bwd<0>(s0, acc.Q0, gm1, dt0, m3b, dt0b, sb, accb.Q0);
  euler_dt_bwd(s0, acc.Q0, gm1, acc.dQ0, dt0b, accb.dQ0, sb, accb.Q0);
  euler_flux_bwd<0>(s0, acc.Q0, mb[0], sb, accb.Q0);
  prim_bwd(acc.Q0, s0, sb, gm1, accb.Q0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    accb.m4[k] += mb[3][k];
    accb.m5[k] += mb[4][k];
    accb.m6[k] += mb[5][k];
  }
  (void)K;
}

}  // namespace dgk
