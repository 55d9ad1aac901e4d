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
  sb.ir += sb.U * Q[1];
  sb.ir += sb.V * Q[2];
  sb.ir += sb.W * Q[3];
  // ir = 1/Q0, rho = Q0
  Qb[0] += sb.rho - sb.ir * s.ir * s.ir;
}

// ---- moment tables ------------------------------------------------------------
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
DGK_HD void mom_half_bwd(T U, T th, T sg, const T* m, T* mb, T& Ub, T& thb) {
  mom_rec_bwd(U, th, m, mb, Ub, thb);
  const T r = d_rsqrt(T(2) * th);
  const T a = U * r;
  const T E = d_exp_bulk(-a * a);
  const T c0 = T(0.56418958354775628695);  // 1/sqrt(pi)
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
  Sb.ith += ab[1] * R1;
  Sb.ith += ab[2] * R2;
  Sb.ith += ab[3] * R3;
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
  sb.U += Sb.U;
  sb.U += Sb.E * S.U;
  sb.V += Sb.V;
  sb.V += Sb.E * S.V;
  sb.W += Sb.W;
  sb.W += Sb.E * S.W;
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
  sb.p += Fb[1 + D];
  sb.p += Fb[4] * Ud;
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
    Ub[j] += kkb * U[j];
    Ub[j] += umb * v[1 + j];
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
  const double e2 = tau > 0.0 ? exp_neg_tab(x_half, ExpTabHolder<>::t.c) : 0.0;
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
// ---- reverse of the moment-matrix form of face_side -------------------------
// Cotangents of the Transverse members (V, W enter the matrices directly too).
template <class T>
struct TransverseBar {
  T V, W, v2, w2, v3, w3, R1, R2, vr, wr, v2r, w2r, vwr, vr2, wr2;
};
template <class T>
DGK_HD TransverseBar<T> transverse_bar_zero() {
  TransverseBar<T> b;
  b.V = b.W = b.v2 = b.w2 = b.v3 = b.w3 = b.R1 = b.R2 = b.vr = b.wr = b.v2r = b.w2r = b.vwr = b.vr2 = b.wr2 = T(0);
  return b;
}

// Given the member cotangents, add those of V, W, th.  The one-dimensional
// Gaussian moments v_n = <v^n> obey dv_n/dV = n v_{n-1} and
// dv_n/dth = n(n-1)/2 v_{n-2}; s1 = K th, s2 = K (K + 2) th^2.
template <class T>
DGK_HD void transverse_bwd(const Transverse<T>& t, T th, T K, const TransverseBar<T>& b, T& Vb, T& Wb, T& thb) {
  const T V = t.V, W = t.W;
  const T t2 = th * th;
  const T v4 = V * V * (V * V + T(6) * th) + T(3) * t2;
  const T w4 = W * W * (W * W + T(6) * th) + T(3) * t2;
  const T s1 = K * th, s2 = K * (K + T(2)) * t2;
  const T v2 = t.v2, w2 = t.w2, v3 = t.v3, w3 = t.w3;
  T bv2 = b.v2, bw2 = b.w2, bv3 = b.v3, bw3 = b.w3, bv4 = T(0), bw4 = T(0), bv5 = T(0), bw5 = T(0);
  T bs1 = T(0), bs2 = T(0);
  T bV = b.V, bW = b.W;
  // wr2 = w5 + 2 w3 (v2 + s1) + W (v4 + s2 + 2 v2 s1)
  {
    const T g = b.wr2;
    bw5 += g;
    bw3 += T(2) * (v2 + s1) * g;
    bv2 += (T(2) * w3 + T(2) * W * s1) * g;
    bs1 += (T(2) * w3 + T(2) * W * v2) * g;
    bW += (v4 + s2 + T(2) * v2 * s1) * g;
    bv4 += W * g;
    bs2 += W * g;
  }
  // vr2 = v5 + 2 v3 (w2 + s1) + V (w4 + s2 + 2 w2 s1)
  {
    const T g = b.vr2;
    bv5 += g;
    bv3 += T(2) * (w2 + s1) * g;
    bw2 += (T(2) * v3 + T(2) * V * s1) * g;
    bs1 += (T(2) * v3 + T(2) * V * w2) * g;
    bV += (w4 + s2 + T(2) * w2 * s1) * g;
    bw4 += V * g;
    bs2 += V * g;
  }
  // vwr = v3 W + V w3 + V W s1
  {
    const T g = b.vwr;
    bv3 += W * g;
    bW += (v3 + V * s1) * g;
    bV += (w3 + W * s1) * g;
    bw3 += V * g;
    bs1 += V * W * g;
  }
  // w2r = w4 + w2 (v2 + s1), v2r = v4 + v2 (w2 + s1)
  bw4 += b.w2r;
  bw2 += (v2 + s1) * b.w2r;
  bv2 += w2 * b.w2r;
  bs1 += w2 * b.w2r;
  bv4 += b.v2r;
  bv2 += (w2 + s1) * b.v2r;
  bw2 += v2 * b.v2r;
  bs1 += v2 * b.v2r;
  // wr = w3 + W (v2 + s1), vr = v3 + V (w2 + s1)
  bw3 += b.wr;
  bW += (v2 + s1) * b.wr;
  bv2 += W * b.wr;
  bs1 += W * b.wr;
  bv3 += b.vr;
  bV += (w2 + s1) * b.vr;
  bw2 += V * b.vr;
  bs1 += V * b.vr;
  // R2 = v4 + w4 + s2 + 2 v2 w2 + 2 (v2 + w2) s1, R1 = v2 + w2 + s1
  bv4 += b.R2;
  bw4 += b.R2;
  bs2 += b.R2;
  bv2 += (T(2) * w2 + T(2) * s1) * b.R2;
  bv2 += b.R1;
  bw2 += (T(2) * v2 + T(2) * s1) * b.R2;
  bw2 += b.R1;
  bs1 += T(2) * (v2 + w2) * b.R2;
  bs1 += b.R1;
  // the one-dimensional moments
  Vb += bV;
  Vb += T(2) * V * bv2;
  Vb += T(3) * v2 * bv3;
  Vb += T(4) * v3 * bv4;
  Vb += T(5) * v4 * bv5;
  Wb += bW;
  Wb += T(2) * W * bw2;
  Wb += T(3) * w2 * bw3;
  Wb += T(4) * w3 * bw4;
  Wb += T(5) * w4 * bw5;
  thb += bv2;
  thb += T(3) * V * bv3;
  thb += T(6) * v2 * bv4;
  thb += T(10) * v3 * bv5;
  thb += bw2;
  thb += T(3) * W * bw3;
  thb += T(6) * w2 * bw4;
  thb += T(10) * w3 * bw5;
  thb += K * bs1;
  thb += T(2) * K * (K + T(2)) * th * bs2;
}

// Reverse of mat_H<P>: add the cotangents of M[P..P+4] and of the members.
template <int P, class T>
DGK_HD void mat_H_bwd(const T* M, const Transverse<T>& t, const T Hb[15], T* Mb, TransverseBar<T>& tb) {
  const T h = T(0.5), q = T(0.25);
  Mb[P] += Hb[0];
  Mb[P] += t.V * Hb[2];
  Mb[P] += t.W * Hb[3];
  Mb[P] += h * t.R1 * Hb[4];
  Mb[P] += t.v2 * Hb[9];
  Mb[P] += t.V * t.W * Hb[10];
  Mb[P] += h * t.vr * Hb[11];
  Mb[P] += t.w2 * Hb[12];
  Mb[P] += h * t.wr * Hb[13];
  Mb[P] += q * t.R2 * Hb[14];
  Mb[P + 1] += Hb[1];
  Mb[P + 1] += t.V * Hb[6];
  Mb[P + 1] += t.W * Hb[7];
  Mb[P + 1] += h * t.R1 * Hb[8];
  Mb[P + 2] += h * Hb[4];
  Mb[P + 2] += Hb[5];
  Mb[P + 2] += h * t.V * Hb[11];
  Mb[P + 2] += h * t.W * Hb[13];
  Mb[P + 2] += h * t.R1 * Hb[14];
  Mb[P + 3] += h * Hb[8];
  Mb[P + 4] += q * Hb[14];
  tb.V += M[P] * Hb[2];
  tb.V += M[P + 1] * Hb[6];
  tb.V += t.W * M[P] * Hb[10];
  tb.V += h * M[P + 2] * Hb[11];
  tb.W += M[P] * Hb[3];
  tb.W += M[P + 1] * Hb[7];
  tb.W += t.V * M[P] * Hb[10];
  tb.W += h * M[P + 2] * Hb[13];
  tb.R1 += h * (M[P] * Hb[4] + M[P + 1] * Hb[8] + M[P + 2] * Hb[14]);
  tb.v2 += M[P] * Hb[9];
  tb.w2 += M[P] * Hb[12];
  tb.vr += h * M[P] * Hb[11];
  tb.wr += h * M[P] * Hb[13];
  tb.R2 += q * M[P] * Hb[14];
}

template <class T>
DGK_HD void mat_Gv_bwd(const T* M, const Transverse<T>& t, const T Gb[15], T* Mb, TransverseBar<T>& tb) {
  const T h = T(0.5), q = T(0.25), VW = t.V * t.W;
  Mb[1] += t.V * Gb[0];
  Mb[1] += t.v2 * Gb[2];
  Mb[1] += VW * Gb[3];
  Mb[1] += h * t.vr * Gb[4];
  Mb[1] += t.v3 * Gb[9];
  Mb[1] += t.v2 * t.W * Gb[10];
  Mb[1] += h * t.v2r * Gb[11];
  Mb[1] += t.V * t.w2 * Gb[12];
  Mb[1] += h * t.vwr * Gb[13];
  Mb[1] += q * t.vr2 * Gb[14];
  Mb[2] += t.V * Gb[1];
  Mb[2] += t.v2 * Gb[6];
  Mb[2] += VW * Gb[7];
  Mb[2] += h * t.vr * Gb[8];
  Mb[3] += h * t.V * Gb[4];
  Mb[3] += t.V * Gb[5];
  Mb[3] += h * t.v2 * Gb[11];
  Mb[3] += h * VW * Gb[13];
  Mb[3] += h * t.vr * Gb[14];
  Mb[4] += h * t.V * Gb[8];
  Mb[5] += q * t.V * Gb[14];
  tb.V += M[1] * Gb[0];
  tb.V += M[2] * Gb[1];
  tb.V += t.W * M[1] * Gb[3];
  tb.V += h * M[3] * Gb[4];
  tb.V += M[3] * Gb[5];
  tb.V += t.W * M[2] * Gb[7];
  tb.V += h * M[4] * Gb[8];
  tb.V += t.w2 * M[1] * Gb[12];
  tb.V += h * t.W * M[3] * Gb[13];
  tb.V += q * M[5] * Gb[14];
  tb.W += t.V * M[1] * Gb[3];
  tb.W += t.V * M[2] * Gb[7];
  tb.W += t.v2 * M[1] * Gb[10];
  tb.W += h * t.V * M[3] * Gb[13];
  tb.v2 += M[1] * Gb[2];
  tb.v2 += M[2] * Gb[6];
  tb.v2 += t.W * M[1] * Gb[10];
  tb.v2 += h * M[3] * Gb[11];
  tb.vr += h * (M[1] * Gb[4] + M[2] * Gb[8] + M[3] * Gb[14]);
  tb.v3 += M[1] * Gb[9];
  tb.v2r += h * M[1] * Gb[11];
  tb.w2 += t.V * M[1] * Gb[12];
  tb.vwr += h * M[1] * Gb[13];
  tb.vr2 += q * M[1] * Gb[14];
}

template <class T>
DGK_HD void mat_Gw_bwd(const T* M, const Transverse<T>& t, const T Gb[15], T* Mb, TransverseBar<T>& tb) {
  const T h = T(0.5), q = T(0.25), VW = t.V * t.W;
  Mb[1] += t.W * Gb[0];
  Mb[1] += VW * Gb[2];
  Mb[1] += t.w2 * Gb[3];
  Mb[1] += h * t.wr * Gb[4];
  Mb[1] += t.W * t.v2 * Gb[9];
  Mb[1] += t.V * t.w2 * Gb[10];
  Mb[1] += h * t.vwr * Gb[11];
  Mb[1] += t.w3 * Gb[12];
  Mb[1] += h * t.w2r * Gb[13];
  Mb[1] += q * t.wr2 * Gb[14];
  Mb[2] += t.W * Gb[1];
  Mb[2] += VW * Gb[6];
  Mb[2] += t.w2 * Gb[7];
  Mb[2] += h * t.wr * Gb[8];
  Mb[3] += h * t.W * Gb[4];
  Mb[3] += t.W * Gb[5];
  Mb[3] += h * VW * Gb[11];
  Mb[3] += h * t.w2 * Gb[13];
  Mb[3] += h * t.wr * Gb[14];
  Mb[4] += h * t.W * Gb[8];
  Mb[5] += q * t.W * Gb[14];
  tb.W += M[1] * Gb[0];
  tb.W += M[2] * Gb[1];
  tb.W += t.V * M[1] * Gb[2];
  tb.W += h * M[3] * Gb[4];
  tb.W += M[3] * Gb[5];
  tb.W += t.V * M[2] * Gb[6];
  tb.W += h * M[4] * Gb[8];
  tb.W += t.v2 * M[1] * Gb[9];
  tb.W += h * t.V * M[3] * Gb[11];
  tb.W += q * M[5] * Gb[14];
  tb.V += t.W * M[1] * Gb[2];
  tb.V += t.W * M[2] * Gb[6];
  tb.V += t.w2 * M[1] * Gb[10];
  tb.V += h * t.W * M[3] * Gb[11];
  tb.w2 += M[1] * Gb[3];
  tb.w2 += M[2] * Gb[7];
  tb.w2 += t.V * M[1] * Gb[10];
  tb.w2 += h * M[3] * Gb[13];
  tb.wr += h * (M[1] * Gb[4] + M[2] * Gb[8] + M[3] * Gb[14]);
  tb.v2 += t.W * M[1] * Gb[9];
  tb.vwr += h * M[1] * Gb[11];
  tb.w3 += M[1] * Gb[12];
  tb.w2r += h * M[1] * Gb[13];
  tb.wr2 += q * M[1] * Gb[14];
}

// Reverse of y += S x (S symmetric, upper triangle in row order): adds the
// cotangents of S and x.  xbar += S ybar, Sbar_kj += ybar_k x_j + ybar_j x_k
// (k < j), Sbar_kk += ybar_k x_k.
template <class T>
DGK_HD void sym_mv_bwd(const T S[15], const T x[5], const T yb[5], T Sb[15], T xb[5]) {
  // accumulated one product at a time (one FMA each)
  constexpr int e[5][5] = {{0, 1, 2, 3, 4}, {1, 5, 6, 7, 8}, {2, 6, 9, 10, 11}, {3, 7, 10, 12, 13}, {4, 8, 11, 13, 14}};
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int j = 0; j < 5; ++j) xb[k] += S[e[k][j]] * yb[j];
  int i = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int j = k; j < 5; ++j, ++i) {
      Sb[i] += yb[k] * x[j];
      if (j != k) Sb[i] += yb[j] * x[k];
    }
}

// Reverse of m5_acc (gks_point.hpp): given the cotangent ob of m5, adds the
// cotangents of M[1..6], of the transverse moments and of x, y, z.  Each line
// reverses one product of the forward, in the forward's grouping P3, P2, P1, P0.
template <class T>
DGK_HD void m5_acc_bwd(const T* M, const Transverse<T>& t, const T x[5], const T y[5], const T z[5], const T ob[5],
                       T* Mb, TransverseBar<T>& tb, T xb[5], T yb[5], T zb[5]) {
  // forward values
  const T hx4 = T(0.5) * x[4], hy4 = T(0.5) * y[4], hz4 = T(0.5) * z[4];
  const T VW = t.V * t.W, v2W = t.v2 * t.W, Vw2 = t.V * t.w2;
  const T d = x[2] + y[1], e = x[3] + z[1], c = y[3] + z[2];
  const T P[4] = {y[0] * t.V + z[0] * t.W + y[2] * t.v2 + c * VW + z[3] * t.w2 + hy4 * t.vr + hz4 * t.wr,
                  x[0] + d * t.V + e * t.W + hx4 * t.R1, x[1] + hy4 * t.V + hz4 * t.W, hx4};
  const T VP[4] = {y[0] * t.v2 + z[0] * VW + y[2] * t.v3 + c * v2W + z[3] * Vw2 + hy4 * t.v2r + hz4 * t.vwr,
                   x[0] * t.V + d * t.v2 + e * VW + hx4 * t.vr, x[1] * t.V + hy4 * t.v2 + hz4 * VW, hx4 * t.V};
  const T WP[4] = {y[0] * VW + z[0] * t.w2 + y[2] * v2W + c * Vw2 + z[3] * t.w3 + hy4 * t.vwr + hz4 * t.w2r,
                   x[0] * t.W + d * VW + e * t.w2 + hx4 * t.wr, x[1] * t.W + hy4 * VW + hz4 * t.w2, hx4 * t.W};
  const T RP[4] = {y[0] * t.vr + z[0] * t.wr + y[2] * t.v2r + c * t.vwr + z[3] * t.w2r + hy4 * t.vr2 + hz4 * t.wr2,
                   x[0] * t.R1 + d * t.vr + e * t.wr + hx4 * t.R2, x[1] * t.R1 + hy4 * t.vr + hz4 * t.wr, hx4 * t.R1};
  // the moment sums
  const T h4 = T(0.5) * ob[4];
  T Pb[4], VPb[4], WPb[4], RPb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    Pb[j] = M[1 + j] * ob[0];
    Pb[j] += M[2 + j] * ob[1];
    Pb[j] += M[3 + j] * h4;
    VPb[j] = M[1 + j] * ob[2];
    WPb[j] = M[1 + j] * ob[3];
    RPb[j] = M[1 + j] * h4;
    Mb[1 + j] += ob[0] * P[j];
    Mb[1 + j] += ob[2] * VP[j];
    Mb[1 + j] += ob[3] * WP[j];
    Mb[1 + j] += h4 * RP[j];
    Mb[2 + j] += ob[1] * P[j];
    Mb[3 + j] += h4 * P[j];
  }
  T hx4b = T(0), hy4b = T(0), hz4b = T(0), db = T(0), eb = T(0), cb = T(0), VWb = T(0), v2Wb = T(0), Vw2b = T(0);
  // P3 = hx4, vP3 = hx4 V, wP3 = hx4 W, rP3 = hx4 R1
  hx4b += Pb[3];
  hx4b += VPb[3] * t.V;
  tb.V += VPb[3] * hx4;
  hx4b += WPb[3] * t.W;
  tb.W += WPb[3] * hx4;
  hx4b += RPb[3] * t.R1;
  tb.R1 += RPb[3] * hx4;
  // P2 = x1 + hy4 V + hz4 W and its v, w, r moments
  xb[1] += Pb[2];
  hy4b += Pb[2] * t.V;
  tb.V += Pb[2] * hy4;
  hz4b += Pb[2] * t.W;
  tb.W += Pb[2] * hz4;
  xb[1] += VPb[2] * t.V;
  tb.V += VPb[2] * x[1];
  hy4b += VPb[2] * t.v2;
  tb.v2 += VPb[2] * hy4;
  hz4b += VPb[2] * VW;
  VWb += VPb[2] * hz4;
  xb[1] += WPb[2] * t.W;
  tb.W += WPb[2] * x[1];
  hy4b += WPb[2] * VW;
  VWb += WPb[2] * hy4;
  hz4b += WPb[2] * t.w2;
  tb.w2 += WPb[2] * hz4;
  xb[1] += RPb[2] * t.R1;
  tb.R1 += RPb[2] * x[1];
  hy4b += RPb[2] * t.vr;
  tb.vr += RPb[2] * hy4;
  hz4b += RPb[2] * t.wr;
  tb.wr += RPb[2] * hz4;
  // P1 = x0 + d V + e W + hx4 R1 and its v, w, r moments
  xb[0] += Pb[1];
  db += Pb[1] * t.V;
  tb.V += Pb[1] * d;
  eb += Pb[1] * t.W;
  tb.W += Pb[1] * e;
  hx4b += Pb[1] * t.R1;
  tb.R1 += Pb[1] * hx4;
  xb[0] += VPb[1] * t.V;
  tb.V += VPb[1] * x[0];
  db += VPb[1] * t.v2;
  tb.v2 += VPb[1] * d;
  eb += VPb[1] * VW;
  VWb += VPb[1] * e;
  hx4b += VPb[1] * t.vr;
  tb.vr += VPb[1] * hx4;
  xb[0] += WPb[1] * t.W;
  tb.W += WPb[1] * x[0];
  db += WPb[1] * VW;
  VWb += WPb[1] * d;
  eb += WPb[1] * t.w2;
  tb.w2 += WPb[1] * e;
  hx4b += WPb[1] * t.wr;
  tb.wr += WPb[1] * hx4;
  xb[0] += RPb[1] * t.R1;
  tb.R1 += RPb[1] * x[0];
  db += RPb[1] * t.vr;
  tb.vr += RPb[1] * d;
  eb += RPb[1] * t.wr;
  tb.wr += RPb[1] * e;
  hx4b += RPb[1] * t.R2;
  tb.R2 += RPb[1] * hx4;
  // P0 = y0 V + z0 W + y2 v^2 + c VW + z3 w^2 + hy4 v r + hz4 w r and its v, w, r moments
  yb[0] += Pb[0] * t.V;
  tb.V += Pb[0] * y[0];
  zb[0] += Pb[0] * t.W;
  tb.W += Pb[0] * z[0];
  yb[2] += Pb[0] * t.v2;
  tb.v2 += Pb[0] * y[2];
  cb += Pb[0] * VW;
  VWb += Pb[0] * c;
  zb[3] += Pb[0] * t.w2;
  tb.w2 += Pb[0] * z[3];
  hy4b += Pb[0] * t.vr;
  tb.vr += Pb[0] * hy4;
  hz4b += Pb[0] * t.wr;
  tb.wr += Pb[0] * hz4;
  yb[0] += VPb[0] * t.v2;
  tb.v2 += VPb[0] * y[0];
  zb[0] += VPb[0] * VW;
  VWb += VPb[0] * z[0];
  yb[2] += VPb[0] * t.v3;
  tb.v3 += VPb[0] * y[2];
  cb += VPb[0] * v2W;
  v2Wb += VPb[0] * c;
  zb[3] += VPb[0] * Vw2;
  Vw2b += VPb[0] * z[3];
  hy4b += VPb[0] * t.v2r;
  tb.v2r += VPb[0] * hy4;
  hz4b += VPb[0] * t.vwr;
  tb.vwr += VPb[0] * hz4;
  yb[0] += WPb[0] * VW;
  VWb += WPb[0] * y[0];
  zb[0] += WPb[0] * t.w2;
  tb.w2 += WPb[0] * z[0];
  yb[2] += WPb[0] * v2W;
  v2Wb += WPb[0] * y[2];
  cb += WPb[0] * Vw2;
  Vw2b += WPb[0] * c;
  zb[3] += WPb[0] * t.w3;
  tb.w3 += WPb[0] * z[3];
  hy4b += WPb[0] * t.vwr;
  tb.vwr += WPb[0] * hy4;
  hz4b += WPb[0] * t.w2r;
  tb.w2r += WPb[0] * hz4;
  yb[0] += RPb[0] * t.vr;
  tb.vr += RPb[0] * y[0];
  zb[0] += RPb[0] * t.wr;
  tb.wr += RPb[0] * z[0];
  yb[2] += RPb[0] * t.v2r;
  tb.v2r += RPb[0] * y[2];
  cb += RPb[0] * t.vwr;
  tb.vwr += RPb[0] * c;
  zb[3] += RPb[0] * t.w2r;
  tb.w2r += RPb[0] * z[3];
  hy4b += RPb[0] * t.vr2;
  tb.vr2 += RPb[0] * hy4;
  hz4b += RPb[0] * t.wr2;
  tb.wr2 += RPb[0] * hz4;
  // d = x2 + y1, e = x3 + z1, c = y3 + z2, the halves and the products of members
  xb[2] += db;
  yb[1] += db;
  xb[3] += eb;
  zb[1] += eb;
  yb[3] += cb;
  zb[2] += cb;
  xb[4] += T(0.5) * hx4b;
  yb[4] += T(0.5) * hy4b;
  zb[4] += T(0.5) * hz4b;
  tb.V += VWb * t.W;
  tb.W += VWb * t.V;
  tb.v2 += v2Wb * t.W;
  tb.W += v2Wb * t.v2;
  tb.V += Vw2b * t.w2;
  tb.w2 += Vw2b * t.V;
}

// Reverse of face_side (moment-matrix form, slopes times the density).  Adds
// the cotangents of the side's trace (q, dq) given those of its accumulator
// contributions.
template <class T>
DGK_HD void face_side_vjp(const Phys& ph, const T q[5], const T dq[3][5], const FaceAcc<T>& accb, T qb[5],
                          T dqb[3][5], T sg) {
  const T K = T(ph.K), gm1 = T(ph.gm1), inv_k3 = T(ph.inv_k3);
  const Prim<T> s = primitive(q, gm1);
  const Solver5<T> S(s, K, inv_k3);
  T ra[3][5], rA[5], dtq[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) S(dq[i], ra[i]);
  euler_dt(s, q, gm1, dq, dtq);
  S(dtq, rA);
  T M[7];
  mom_half(s.U, s.th, sg, M);
  const Transverse<T> tr(s.V, s.W, s.th, K);
  const T r = s.rho;

  T Mb[7];
#pragma unroll
  for (int n = 0; n < 7; ++n) Mb[n] = T(0);
  TransverseBar<T> trb = transverse_bar_zero<T>();
  T rab[3][5], rAb[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) zero5(rab[i]);
  zero5(rAb);
  T rb = T(0);
  T H[15], Hb[15];
  // <psi psi^T>: Q0 (r times its first column) and dQ0_i
  mat_H<0>(M, tr, H);
#pragma unroll
  for (int k = 0; k < 15; ++k) Hb[k] = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    rb += accb.Q0[k] * H[k];
    Hb[k] += r * accb.Q0[k];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) sym_mv_bwd(H, ra[i], accb.dQ0[i], Hb, rab[i]);
  mat_H_bwd<0>(M, tr, Hb, Mb, trb);
  // <u psi psi^T>: m4 (r times its first column) and m6
  mat_H<1>(M, tr, H);
#pragma unroll
  for (int k = 0; k < 15; ++k) Hb[k] = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    rb += accb.m4[k] * H[k];
    Hb[k] += r * accb.m4[k];
  }
  sym_mv_bwd(H, rA, accb.m6, Hb, rAb);
  mat_H_bwd<1>(M, tr, Hb, Mb, trb);
  // m5 = <u^2 psi psi^T> ra_0 + <u v psi psi^T> ra_1 + <u w psi psi^T> ra_2: the
  // matrix-free reverse in FP32; the FP64 lanes, which spill, run faster with
  // the matrices (5.8% on the FP64 P2 adjoint)
  if constexpr (sizeof(T) == 4) {
    m5_acc_bwd(M, tr, ra[0], ra[1], ra[2], accb.m5, Mb, trb, rab[0], rab[1], rab[2]);
  } else {
    mat_H<2>(M, tr, H);
#pragma unroll
    for (int k = 0; k < 15; ++k) Hb[k] = T(0);
    sym_mv_bwd(H, ra[0], accb.m5, Hb, rab[0]);
    mat_H_bwd<2>(M, tr, Hb, Mb, trb);
    mat_Gv(M, tr, H);
#pragma unroll
    for (int k = 0; k < 15; ++k) Hb[k] = T(0);
    sym_mv_bwd(H, ra[1], accb.m5, Hb, rab[1]);
    mat_Gv_bwd(M, tr, Hb, Mb, trb);
    mat_Gw(M, tr, H);
#pragma unroll
    for (int k = 0; k < 15; ++k) Hb[k] = T(0);
    sym_mv_bwd(H, ra[2], accb.m5, Hb, rab[2]);
    mat_Gw_bwd(M, tr, Hb, Mb, trb);
  }

  Prim<T> sb = prim_zero<T>();
  sb.rho += rb;
  transverse_bwd(tr, s.th, K, trb, sb.V, sb.W, sb.th);
  mom_half_bwd(s.U, s.th, sg, M, Mb, sb.U, sb.th);
  // rA = S(dt), dt = -sum_e J_e dq_e
  Solver5Bar<T> Sb;
  T dtqb[5];
  zero5(dtqb);
  solve_bwd(S, dtq, rA, rAb, dtqb, Sb);
  euler_dt_bwd(s, q, gm1, dq, dtqb, dqb, sb, qb);
  // ra_i = S(dq_i)
#pragma unroll
  for (int i = 0; i < 3; ++i) solve_bwd(S, dq[i], ra[i], rab[i], dqb[i], Sb);
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
  time_coefficients(tau, xh, ph.dt, ph.inv_dt, al, be, ExpTabHolder<>::t.c);
  // Reverse of the combination as face_finish computes it, in T with the FP64
  // coefficients rounded once:
  //   Ft = b0 d14 + b1 d25 + b2 m3 + b5 m6,
  //   F  = m4 + a0 d14 + a1 d25 - tau m5 + a2 m3 + a5 m6,  d14 = m1 - m4, d25 = m2 - m5.
  // With alpha_3 = 1 - alpha_0, alpha_4 = -tau - alpha_1, beta_3 = -beta_0,
  // beta_4 = -beta_1, the cotangents of the independent coefficients are the
  // dot products with d14, d25, m3, m6, and -tau m5 adds -Fb.m5 to that of tau.
  T d14[5], d25[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    d14[k] = m1[k] - acc.m4[k];
    d25[k] = m2[k] - acc.m5[k];
  }
  T fa0 = T(0), fa1 = T(0), fa2 = T(0), fa5 = T(0), fm5 = T(0);
  T fb0 = T(0), fb1 = T(0), fb2 = T(0), fb5 = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if constexpr (NEED_F) {
      fa0 += Fb[k] * d14[k];
      fa1 += Fb[k] * d25[k];
      fa2 += Fb[k] * m3[k];
      fa5 += Fb[k] * acc.m6[k];
      fm5 += Fb[k] * acc.m5[k];
    }
    fb0 += Ftb[k] * d14[k];
    fb1 += Ftb[k] * d25[k];
    fb2 += Ftb[k] * m3[k];
    fb5 += Ftb[k] * acc.m6[k];
  }
  const double alb[6] = {double(fa0), double(fa1), double(fa2), 0.0, 0.0, double(fa5)};
  const double beb[6] = {double(fb0), double(fb1), double(fb2), 0.0, 0.0, double(fb5)};
  const T a0 = T(al[0]), a1 = T(al[1]), a2 = T(al[2]), a5 = T(al[5]), tT = T(tau);
  const T b0 = T(be[0]), b1 = T(be[1]), b2 = T(be[2]), b5 = T(be[5]);
  T mb[6][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const T f = NEED_F ? Fb[k] : T(0);
    const T d14b = a0 * f + b0 * Ftb[k], d25b = a1 * f + b1 * Ftb[k];
    mb[0][k] = d14b;
    mb[1][k] = d25b;
    mb[2][k] = a2 * f + b2 * Ftb[k];
    mb[3][k] = f - d14b;
    mb[4][k] = -d25b - tT * f;
    mb[5][k] = a5 * f + b5 * Ftb[k];
  }
  Prim<T> sb = prim_zero<T>();
  Grad<T> gb = grad_zero<T>();
  if constexpr (NEED_F) {
    // F4 += (1/Pr - 1) (-mu cp dT0/dn)
    gb.dT[0] -= T(ph.inv_pr_m1 * ph.mu * ph.cp * double(Fb[4]));
    mub -= ph.inv_pr_m1 * ph.cp * double(g.dT[0]) * double(Fb[4]);
  }
  double taub = -double(fm5), xb = 0.0;
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
