// dg_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
//
// A plain, slow, obviously-correct FP64 CPU reference ("the oracle") for one
// two-stage fourth-order (S2O4) step of the modal discontinuous Galerkin
// gas-kinetic scheme of Wang & Pan, "Three-dimensional discontinuous Galerkin
// based high-order gas-kinetic scheme and GPU implementation" (arXiv
// 2202.13821).  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg
// of bench.py may load this library.  It shares no code, header, table or
// constant with the HIP library under paper_2202_13821_amd/.
//
// Style: every moment is evaluated by a generic monomial engine (products of
// one-dimensional Maxwellian moments, term by term), every 5x5 moment system is
// solved by dense Gaussian elimination, and every quadrature table is computed
// from its definition at run time.  The code is templated on the scalar type so
// that the same arithmetic also runs on forward-mode dual numbers (used by the
// tests as an independent gradient of the whole step).
//
// Notation follows the paper: Q = (rho, rho U, rho V, rho W, rho E), the
// Maxwellian g with lambda = rho / (2 p), K internal degrees of freedom,
// psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2), <.> the moment of g divided by
// rho, tau = mu / p the collision time.  R = 1, so T = p / rho.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace dgo {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Forward-mode dual number: value + one directional derivative.
// ---------------------------------------------------------------------------
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: implicit on purpose
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual& operator/=(Dual& a, Dual b) { a = a / b; return a; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
inline Dual erfc(Dual a) {
  // d/dx erfc(x) = -2/sqrt(pi) exp(-x^2)
  return {std::erfc(a.v), -2.0 / std::sqrt(kPi) * std::exp(-a.v * a.v) * a.d};
}
inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
using std::erfc;
using std::exp;
using std::sqrt;

// ---------------------------------------------------------------------------
// Configuration (the oracle's own definition).
// ---------------------------------------------------------------------------
struct Cfg {
  int32_t nx, ny, nz;
  int32_t k;   // polynomial degree of the P_k space
  int32_t nq;  // Gauss points per direction
  int32_t pad;
  double lo[3], hi[3];
  double gamma, mu, prandtl;
  // Optional separable mesh (Section 5.1 non-uniform meshes): nx + ny + nz
  // cell widths (x, then y, then z) summing to hi - lo per axis; NULL for
  // the uniform mesh dx = (hi - lo) / n.
  const double* widths;
};

// ---------------------------------------------------------------------------
// Section 3: Legendre polynomials on [-1,1] (Bonnet recurrence) and their
// derivatives; Gauss-Legendre rule by Newton iteration on P_n.
// ---------------------------------------------------------------------------
static void legendre(int lmax, double x, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (lmax >= 1) { P[1] = x; dP[1] = 1.0; }
  for (int l = 1; l < lmax; ++l) {
    P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1);
    dP[l + 1] = dP[l - 1] + (2 * l + 1) * P[l];
  }
}

static void gauss_legendre(int n, double* x, double* w) {
  std::vector<double> P(n + 1), dP(n + 1);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, P.data(), dP.data());
      double dz = P[n] / dP[n];
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    legendre(n, z, P.data(), dP.data());
    x[i] = -z;  // ascending order
    w[i] = 2.0 / ((1.0 - z * z) * dP[n] * dP[n]);
  }
}

// Mode order of the P_k basis B_n = P_nx(xi) P_ny(eta) P_nz(zeta),
// nx+ny+nz <= k: by total degree s, then nx descending, then ny descending.
struct Mode { int n[3]; };
static std::vector<Mode> mode_list(int k) {
  std::vector<Mode> m;
  for (int s = 0; s <= k; ++s)
    for (int nx = s; nx >= 0; --nx)
      for (int ny = s - nx; ny >= 0; --ny) m.push_back({{nx, ny, s - nx - ny}});
  return m;
}

// ---------------------------------------------------------------------------
// Section 2: moments of the Maxwellian.  For one velocity component with mean
// U and lambda, <c^0> = 1, <c^1> = U and <c^{n+2}> = U <c^{n+1}> +
// (n+1)/(2 lambda) <c^n> (integration by parts of the Gaussian).  On a half
// line (u > 0 or u < 0) the first two moments come from erfc and the Gaussian
// at u = 0, and the same recurrence holds because u^{n+1} vanishes at u = 0.
// Internal degrees of freedom: <xi^0> = 1, <xi^2> = K/(2 lambda),
// <xi^4> = K(K+2)/(4 lambda^2).
// ---------------------------------------------------------------------------
constexpr int kMomMax = 9;  // u^0 .. u^8

template <class R>
struct Tab {
  R u[kMomMax], v[kMomMax], w[kMomMax], x[3];
};

template <class R>
static void mom1d_full(R U, R lam, R* m) {
  m[0] = R(1.0);
  m[1] = U;
  for (int n = 0; n + 2 < kMomMax; ++n) m[n + 2] = U * m[n + 1] + R(double(n + 1)) / (R(2.0) * lam) * m[n];
}

// side = +1: integrate over u > 0; side = -1: over u < 0.
template <class R>
static void mom1d_half(R U, R lam, int side, R* m) {
  R sl = sqrt(lam);
  R gauss0 = exp(-lam * U * U) / (R(2.0) * sqrt(R(kPi) * lam));
  if (side > 0) {
    m[0] = R(0.5) * erfc(-sl * U);
    m[1] = U * m[0] + gauss0;
  } else {
    m[0] = R(0.5) * erfc(sl * U);
    m[1] = U * m[0] - gauss0;
  }
  for (int n = 0; n + 2 < kMomMax; ++n) m[n + 2] = U * m[n + 1] + R(double(n + 1)) / (R(2.0) * lam) * m[n];
}

template <class R>
static Tab<R> make_tab(const R U[3], R lam, R K, int half_side) {
  Tab<R> t;
  if (half_side == 0)
    mom1d_full(U[0], lam, t.u);
  else
    mom1d_half(U[0], lam, half_side, t.u);
  mom1d_full(U[1], lam, t.v);
  mom1d_full(U[2], lam, t.w);
  t.x[0] = R(1.0);
  t.x[1] = K / (R(2.0) * lam);
  t.x[2] = K * (K + R(2.0)) / (R(4.0) * lam * lam);
  return t;
}

// <u^a v^b w^c (xi^2)^d>
template <class R>
static inline R mono(const Tab<R>& t, int a, int b, int c, int d) {
  return t.u[a] * t.v[b] * t.w[c] * t.x[d];
}

// psi_k as lists of monomials c * u^a v^b w^c (xi^2)^d.
struct PsiTerm { double c; int e[4]; };
static const PsiTerm kPsi0[] = {{1.0, {0, 0, 0, 0}}};
static const PsiTerm kPsi1[] = {{1.0, {1, 0, 0, 0}}};
static const PsiTerm kPsi2[] = {{1.0, {0, 1, 0, 0}}};
static const PsiTerm kPsi3[] = {{1.0, {0, 0, 1, 0}}};
static const PsiTerm kPsi4[] = {{0.5, {2, 0, 0, 0}}, {0.5, {0, 2, 0, 0}}, {0.5, {0, 0, 2, 0}}, {0.5, {0, 0, 0, 1}}};
static const PsiTerm* const kPsi[5] = {kPsi0, kPsi1, kPsi2, kPsi3, kPsi4};
static const int kPsiN[5] = {1, 1, 1, 1, 4};

// G[k][j] = < u^a v^b w^c psi_k psi_j >
template <class R>
static void gmat(const Tab<R>& t, int a, int b, int c, R G[5][5]) {
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < 5; ++j) {
      R s = R(0.0);
      for (int p = 0; p < kPsiN[k]; ++p)
        for (int q = 0; q < kPsiN[j]; ++q) {
          const PsiTerm& A = kPsi[k][p];
          const PsiTerm& B = kPsi[j][q];
          s += R(A.c * B.c) * mono(t, a + A.e[0] + B.e[0], b + A.e[1] + B.e[1], c + A.e[2] + B.e[2], A.e[3] + B.e[3]);
        }
      G[k][j] = s;
    }
}

template <class R>
static void matvec5(const R G[5][5], const R x[5], R y[5]) {
  for (int k = 0; k < 5; ++k) {
    R s = R(0.0);
    for (int j = 0; j < 5; ++j) s += G[k][j] * x[j];
    y[k] = s;
  }
}

// Dense Gaussian elimination with partial pivoting: solve M x = b.
template <class R>
static void solve5(const R M_in[5][5], const R b_in[5], R x[5]) {
  R M[5][6];
  for (int i = 0; i < 5; ++i) {
    for (int j = 0; j < 5; ++j) M[i][j] = M_in[i][j];
    M[i][5] = b_in[i];
  }
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    for (int r = c + 1; r < 5; ++r)
      if (std::fabs(val(M[r][c])) > std::fabs(val(M[piv][c]))) piv = r;
    if (piv != c)
      for (int j = 0; j < 6; ++j) std::swap(M[c][j], M[piv][j]);
    for (int r = c + 1; r < 5; ++r) {
      R f = M[r][c] / M[c][c];
      for (int j = c; j < 6; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 4; i >= 0; --i) {
    R s = M[i][5];
    for (int j = i + 1; j < 5; ++j) s -= M[i][j] * x[j];
    x[i] = s / M[i][i];
  }
}

// Sparse polynomial in (u, v, w, xi^2), used for the heat-flux moment.
template <class R>
struct PTerm { R c; int e[4]; };
template <class R>
using SPoly = std::vector<PTerm<R>>;

template <class R>
static SPoly<R> pmul(const SPoly<R>& A, const SPoly<R>& B) {
  SPoly<R> out;
  out.reserve(A.size() * B.size());
  for (const auto& a : A)
    for (const auto& b : B)
      out.push_back({a.c * b.c, {a.e[0] + b.e[0], a.e[1] + b.e[1], a.e[2] + b.e[2], a.e[3] + b.e[3]}});
  return out;
}
template <class R>
static R pmoment(const Tab<R>& t, const SPoly<R>& P) {
  R s = R(0.0);
  for (const auto& p : P) s += p.c * mono(t, p.e[0], p.e[1], p.e[2], p.e[3]);
  return s;
}
// The polynomial sum_j a_j psi_j.
template <class R>
static SPoly<R> slope_poly(const R a[5]) {
  SPoly<R> P;
  for (int j = 0; j < 5; ++j)
    for (int p = 0; p < kPsiN[j]; ++p) {
      const PsiTerm& T = kPsi[j][p];
      P.push_back({a[j] * R(T.c), {T.e[0], T.e[1], T.e[2], T.e[3]}});
    }
  return P;
}
static inline void unit(int d, int e[3]) { e[0] = e[1] = e[2] = 0; e[d] = 1; }

// ---------------------------------------------------------------------------
// Macroscopic <-> Maxwellian parameters.  rho E = rho <psi_5> =
// rho (|U|^2 + (K+3)/(2 lambda)) / 2 gives lambda; p = rho / (2 lambda).
// ---------------------------------------------------------------------------
template <class R>
struct Prim { R rho, U[3], lam, p; };

template <class R>
static Prim<R> primitives(const R Q[5], R K) {
  Prim<R> s;
  s.rho = Q[0];
  for (int i = 0; i < 3; ++i) s.U[i] = Q[1 + i] / Q[0];
  R kin = R(0.5) * (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / Q[0];
  s.lam = (K + R(3.0)) * Q[0] / (R(4.0) * (Q[4] - kin));
  s.p = Q[0] / (R(2.0) * s.lam);
  return s;
}

// Slope a (coefficients on psi) from <a psi> = b.
template <class R>
static void slope(const Tab<R>& t, const R b[5], R a[5]) {
  R M[5][5];
  gmat(t, 0, 0, 0, M);
  solve5(M, b, a);
}

// ---------------------------------------------------------------------------
// Heat flux of the first-order non-equilibrium part -tau g (X) with
// X = sum_e u_e a_e + A, along direction d:
// q_d = -tau rho < (u_d - U_d) (|u - U|^2 + xi^2) / 2  X >.
// The Prandtl-number fix adds (1/Pr - 1) q_d to the energy flux.
// ---------------------------------------------------------------------------
template <class R>
static R heat_moment(const Tab<R>& t, const R U[3], int d, const R a[3][5], const R A[5]) {
  SPoly<R> lin = {{R(1.0), {d == 0, d == 1, d == 2, 0}}, {-U[d], {0, 0, 0, 0}}};
  SPoly<R> half_c2;
  for (int i = 0; i < 3; ++i) {
    int e2[4] = {0, 0, 0, 0}, e1[4] = {0, 0, 0, 0};
    e2[i] = 2;
    e1[i] = 1;
    half_c2.push_back({R(0.5), {e2[0], e2[1], e2[2], 0}});
    half_c2.push_back({-U[i], {e1[0], e1[1], e1[2], 0}});
    half_c2.push_back({R(0.5) * U[i] * U[i], {0, 0, 0, 0}});
  }
  half_c2.push_back({R(0.5), {0, 0, 0, 1}});
  SPoly<R> h = pmul(lin, half_c2);
  SPoly<R> X = slope_poly(A);
  for (int e = 0; e < 3; ++e) {
    SPoly<R> ue = {{R(1.0), {e == 0, e == 1, e == 2, 0}}};
    SPoly<R> t2 = pmul(ue, slope_poly(a[e]));
    X.insert(X.end(), t2.begin(), t2.end());
  }
  return pmoment(t, pmul(h, X));
}

// ---------------------------------------------------------------------------
// Volume flux, Eq. (flux-2): inside a cell the distribution is
// f = g0 (1 - tau (a_1 u + a_2 v + a_3 w + A) + A t), with <a_i> = dQ/dx_i,
// <a_1 u + a_2 v + a_3 w + A> = 0 and tau = mu / p.  F_d(t) is linear in t:
// F_d = rho [<u_d psi> - tau (sum_e <u_d u_e a_e psi> + <u_d A psi>)],
// dF_d/dt = rho <u_d A psi>.
// q[5], dq[3][5] = dQ/dx_e; outputs F[3][5], Ft[3][5] (global frame).
// ---------------------------------------------------------------------------
template <class R>
static void volume_flux(const Cfg& c, R mu, const R q[5], const R dq[3][5], R F[3][5], R Ft[3][5]) {
  const R K = R((5.0 - 3.0 * c.gamma) / (c.gamma - 1.0));
  Prim<R> s = primitives(q, K);
  Tab<R> t = make_tab(s.U, s.lam, K, 0);
  R M[5][5];
  gmat(t, 0, 0, 0, M);
  R a[3][5];
  for (int e = 0; e < 3; ++e) {
    R b[5];
    for (int k = 0; k < 5; ++k) b[k] = dq[e][k] / s.rho;
    solve5(M, b, a[e]);
  }
  R rhsA[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
  for (int e = 0; e < 3; ++e) {
    int ue[3];
    unit(e, ue);
    R G[5][5], y[5];
    gmat(t, ue[0], ue[1], ue[2], G);
    matvec5(G, a[e], y);
    for (int k = 0; k < 5; ++k) rhsA[k] -= y[k];
  }
  R A[5];
  solve5(M, rhsA, A);
  const R tau = mu / s.p;
  for (int d = 0; d < 3; ++d) {
    int ud[3];
    unit(d, ud);
    R Gd[5][5];
    gmat(t, ud[0], ud[1], ud[2], Gd);
    R uApsi[5];
    matvec5(Gd, A, uApsi);
    R visc[5];
    for (int k = 0; k < 5; ++k) visc[k] = uApsi[k];
    for (int e = 0; e < 3; ++e) {
      int ue[3];
      unit(e, ue);
      R G[5][5], y[5];
      gmat(t, ud[0] + ue[0], ud[1] + ue[1], ud[2] + ue[2], G);
      matvec5(G, a[e], y);
      for (int k = 0; k < 5; ++k) visc[k] += y[k];
    }
    for (int k = 0; k < 5; ++k) {
      F[d][k] = s.rho * (Gd[k][0] - tau * visc[k]);
      Ft[d][k] = s.rho * uApsi[k];
    }
    R qd = -tau * s.rho * heat_moment(t, s.U, d, a, A);
    F[d][4] += (R(1.0) / R(c.prandtl) - R(1.0)) * qd;
  }
}

// ---------------------------------------------------------------------------
// Time integrals over [0, delta] of the time factors of Eq. (flux):
// c1 = int (1 - e^{-t/tau}),         c2 = int ((t + tau) e^{-t/tau} - tau),
// c3 = int (t - tau + tau e^{-t/tau}), c4 = int e^{-t/tau},
// c5 = int (t + tau) e^{-t/tau},     c6 = int tau e^{-t/tau}.
// tau = 0 is the collisionless-free (inviscid) limit with e^{-delta/tau} = 0.
// ---------------------------------------------------------------------------
template <class R>
static void time_integrals(R tau, double delta, R c[6]) {
  R E = (val(tau) > 0.0) ? exp(-R(delta) / tau) : R(0.0);
  R dl = R(delta);
  c[0] = dl - tau * (R(1.0) - E);
  c[1] = R(2.0) * tau * tau - tau * dl - tau * (R(2.0) * tau + dl) * E;
  c[2] = dl * dl / R(2.0) - tau * dl + tau * tau * (R(1.0) - E);
  c[3] = tau * (R(1.0) - E);
  c[4] = R(2.0) * tau * tau - tau * (R(2.0) * tau + dl) * E;
  c[5] = tau * tau * (R(1.0) - E);
}

// ---------------------------------------------------------------------------
// Face flux, Eq. (flux) with its slope systems, in the local frame of a face
// whose normal is global axis d: local axes are (d, d+1, d+2) mod 3 for both
// velocity components and derivative directions; the output is rotated back.
// qL/dqL: trace of the lower cell, qR/dqR: trace of the upper cell (global).
// F = (4 FF(dt/2) - FF(dt)) / dt, Ft = 4 (FF(dt) - 2 FF(dt/2)) / dt^2 where
// FF(delta) is the time integral of the flux over [0, delta] (Eq.
// (expansion-1) and the two integrated equations that follow it).
// ---------------------------------------------------------------------------
template <class R>
static void face_flux(const Cfg& c, R mu, double dt, int d, const R qLg[5], const R dqLg[3][5], const R qRg[5],
                      const R dqRg[3][5], R Fg[5], R Ftg[5]) {
  const R K = R((5.0 - 3.0 * c.gamma) / (c.gamma - 1.0));
  const int ax[3] = {d, (d + 1) % 3, (d + 2) % 3};
  R qs[2][5], dqs[2][3][5];
  const R* qg[2] = {qLg, qRg};
  const R(*dqg[2])[5] = {dqLg, dqRg};
  for (int s = 0; s < 2; ++s) {
    qs[s][0] = qg[s][0];
    qs[s][4] = qg[s][4];
    for (int i = 0; i < 3; ++i) qs[s][1 + i] = qg[s][1 + ax[i]];
    for (int i = 0; i < 3; ++i) {
      dqs[s][i][0] = dqg[s][ax[i]][0];
      dqs[s][i][4] = dqg[s][ax[i]][4];
      for (int j = 0; j < 3; ++j) dqs[s][i][1 + j] = dqg[s][ax[i]][1 + ax[j]];
    }
  }
  // Side states: g_l over u > 0, g_r over u < 0.
  Prim<R> ps[2];
  Tab<R> full[2], half[2];
  R a[2][3][5], A[2][5];
  for (int s = 0; s < 2; ++s) {
    ps[s] = primitives(qs[s], K);
    full[s] = make_tab(ps[s].U, ps[s].lam, K, 0);
    half[s] = make_tab(ps[s].U, ps[s].lam, K, s == 0 ? +1 : -1);
    // <a_i^k> = dQ_k/dn_i and <a_1^k u + a_2^k v + a_3^k w + A^k> = 0.
    R M[5][5];
    gmat(full[s], 0, 0, 0, M);
    R rhsA[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
    for (int i = 0; i < 3; ++i) {
      R b[5];
      for (int k = 0; k < 5; ++k) b[k] = dqs[s][i][k] / ps[s].rho;
      solve5(M, b, a[s][i]);
      int ui[3];
      unit(i, ui);
      R G[5][5], y[5];
      gmat(full[s], ui[0], ui[1], ui[2], G);
      matvec5(G, a[s][i], y);
      for (int k = 0; k < 5; ++k) rhsA[k] -= y[k];
    }
    solve5(M, rhsA, A[s]);
  }
  // Equilibrium state at the face: Q0 = int_{u>0} psi g_l + int_{u<0} psi g_r,
  // dQ0/dn_i = int_{u>0} psi a_i^l g_l + int_{u<0} psi a_i^r g_r.
  R Q0[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
  R dQ0[3][5];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 5; ++k) dQ0[i][k] = R(0.0);
  for (int s = 0; s < 2; ++s) {
    R H[5][5];
    gmat(half[s], 0, 0, 0, H);
    for (int k = 0; k < 5; ++k) Q0[k] += ps[s].rho * H[k][0];
    for (int i = 0; i < 3; ++i) {
      R y[5];
      matvec5(H, a[s][i], y);
      for (int k = 0; k < 5; ++k) dQ0[i][k] += ps[s].rho * y[k];
    }
  }
  Prim<R> p0 = primitives(Q0, K);
  Tab<R> t0 = make_tab(p0.U, p0.lam, K, 0);
  R abar[3][5], Abar[5];
  {
    R M[5][5];
    gmat(t0, 0, 0, 0, M);
    R rhsA[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
    for (int i = 0; i < 3; ++i) {
      R b[5];
      for (int k = 0; k < 5; ++k) b[k] = dQ0[i][k] / p0.rho;
      solve5(M, b, abar[i]);
      int ui[3];
      unit(i, ui);
      R G[5][5], y[5];
      gmat(t0, ui[0], ui[1], ui[2], G);
      matvec5(G, abar[i], y);
      for (int k = 0; k < 5; ++k) rhsA[k] -= y[k];
    }
    solve5(M, rhsA, Abar);
  }
  const R tau = mu / p0.p;
  // Moments of u psi times each part of Eq. (flux).
  R m[6][5];
  {
    R Gu[5][5];
    gmat(t0, 1, 0, 0, Gu);
    R y[5];
    for (int k = 0; k < 5; ++k) m[0][k] = p0.rho * Gu[k][0];  // g0
    for (int k = 0; k < 5; ++k) m[1][k] = R(0.0);             // (abar . u) g0
    for (int i = 0; i < 3; ++i) {
      int ui[3];
      unit(i, ui);
      R G[5][5];
      gmat(t0, 1 + ui[0], ui[1], ui[2], G);
      matvec5(G, abar[i], y);
      for (int k = 0; k < 5; ++k) m[1][k] += p0.rho * y[k];
    }
    matvec5(Gu, Abar, y);  // Abar g0
    for (int k = 0; k < 5; ++k) m[2][k] = p0.rho * y[k];
  }
  for (int j = 3; j < 6; ++j)
    for (int k = 0; k < 5; ++k) m[j][k] = R(0.0);
  for (int s = 0; s < 2; ++s) {
    R Gu[5][5], y[5];
    gmat(half[s], 1, 0, 0, Gu);
    for (int k = 0; k < 5; ++k) m[3][k] += ps[s].rho * Gu[k][0];  // g_k
    for (int i = 0; i < 3; ++i) {                                 // (a^k . u) g_k
      int ui[3];
      unit(i, ui);
      R G[5][5];
      gmat(half[s], 1 + ui[0], ui[1], ui[2], G);
      matvec5(G, a[s][i], y);
      for (int k = 0; k < 5; ++k) m[4][k] += ps[s].rho * y[k];
    }
    matvec5(Gu, A[s], y);  // A^k g_k
    for (int k = 0; k < 5; ++k) m[5][k] += ps[s].rho * y[k];
  }
  R c1[6], c2[6];
  time_integrals(tau, dt, c1);
  time_integrals(tau, 0.5 * dt, c2);
  const double sgn[6] = {1.0, 1.0, 1.0, 1.0, -1.0, -1.0};
  R Fl[5], Ftl[5];
  for (int k = 0; k < 5; ++k) {
    R Ffull = R(0.0), Fhalf = R(0.0);
    for (int j = 0; j < 6; ++j) {
      Ffull += R(sgn[j]) * c1[j] * m[j][k];
      Fhalf += R(sgn[j]) * c2[j] * m[j][k];
    }
    Fl[k] = (R(4.0) * Fhalf - Ffull) / R(dt);
    Ftl[k] = R(4.0) * (Ffull - R(2.0) * Fhalf) / R(dt * dt);
  }
  R qn = -tau * p0.rho * heat_moment(t0, p0.U, 0, abar, Abar);
  Fl[4] += (R(1.0) / R(c.prandtl) - R(1.0)) * qn;
  // Back to the global frame.
  Fg[0] = Fl[0];
  Fg[4] = Fl[4];
  Ftg[0] = Ftl[0];
  Ftg[4] = Ftl[4];
  for (int i = 0; i < 3; ++i) {
    Fg[1 + ax[i]] = Fl[1 + i];
    Ftg[1 + ax[i]] = Ftl[1 + i];
  }
}

// ---------------------------------------------------------------------------
// Discretization: Section 3, Eqs. (expansion), (DG2), (operator), (surface),
// (volume).  Field layout q[var][mode][z][y][x].
// ---------------------------------------------------------------------------
struct Disc {
  Cfg c;
  std::vector<Mode> md;
  int nm = 0, nq = 0;
  std::vector<double> xg, wg;  // Gauss nodes on [-1,1], weights normalised to sum 1
  // separable mesh: width wd[e][i] and lower node xl[e][i] of cell i along axis e
  std::vector<double> wd[3], xl[3];
  std::vector<double> mass;  // M_nn / |K| by quadrature (exact), reference cell
  // basis values at volume points: [q][n], reference gradient [q][d][n]
  std::vector<double> Bv, dBv;
  // face traces: for direction d and side s (0: xi_d=+1, 1: xi_d=-1), face point
  // (a,b) over tangential axes (d+1, d+2): value [d][s][qf][n], ref grad [d][s][qf][e][n]
  std::vector<double> Bf, dBf;
  int64_t ncell = 0;

  explicit Disc(const Cfg& cfg) : c(cfg) {
    md = mode_list(c.k);
    nm = (int)md.size();
    nq = c.nq;
    xg.resize(nq);
    wg.resize(nq);
    gauss_legendre(nq, xg.data(), wg.data());
    for (auto& w : wg) w *= 0.5;
    const int n[3] = {c.nx, c.ny, c.nz};
    for (int e = 0, off = 0; e < 3; off += n[e], ++e) {
      wd[e].resize(n[e]);
      xl[e].resize(n[e]);
      double x = c.lo[e];
      for (int i = 0; i < n[e]; ++i) {
        wd[e][i] = c.widths ? c.widths[off + i] : (c.hi[e] - c.lo[e]) / n[e];
        xl[e][i] = c.widths ? x : c.lo[e] + i * wd[e][i];
        x += wd[e][i];
      }
    }
    ncell = (int64_t)c.nx * c.ny * c.nz;
    // mass matrix diagonal by an exact Gauss rule (k+1 points per direction)
    {
      int nm1 = c.k + 1;
      std::vector<double> x(nm1), w(nm1);
      gauss_legendre(nm1, x.data(), w.data());
      mass.assign(nm, 0.0);
      for (int n = 0; n < nm; ++n) {
        double s = 0;
        for (int a = 0; a < nm1; ++a)
          for (int b = 0; b < nm1; ++b)
            for (int g = 0; g < nm1; ++g) {
              double xi[3] = {x[a], x[b], x[g]};
              double B = basis(n, xi);
              s += 0.125 * w[a] * w[b] * w[g] * B * B;
            }
        mass[n] = s;
      }
    }
    const int nqv = nq * nq * nq;
    Bv.resize((size_t)nqv * nm);
    dBv.resize((size_t)nqv * 3 * nm);
    for (int g = 0; g < nq; ++g)
      for (int b = 0; b < nq; ++b)
        for (int a = 0; a < nq; ++a) {
          int qi = (g * nq + b) * nq + a;
          double xi[3] = {xg[a], xg[b], xg[g]};
          for (int n = 0; n < nm; ++n) {
            Bv[(size_t)qi * nm + n] = basis(n, xi);
            for (int e = 0; e < 3; ++e) dBv[((size_t)qi * 3 + e) * nm + n] = dbasis(n, e, xi);
          }
        }
    const int nqf = nq * nq;
    Bf.resize((size_t)3 * 2 * nqf * nm);
    dBf.resize((size_t)3 * 2 * nqf * 3 * nm);
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s)
        for (int bq = 0; bq < nq; ++bq)
          for (int aq = 0; aq < nq; ++aq) {
            int qf = bq * nq + aq;
            double xi[3];
            xi[d] = (s == 0) ? 1.0 : -1.0;
            xi[(d + 1) % 3] = xg[aq];
            xi[(d + 2) % 3] = xg[bq];
            for (int n = 0; n < nm; ++n) {
              Bf[(((size_t)d * 2 + s) * nqf + qf) * nm + n] = basis(n, xi);
              for (int e = 0; e < 3; ++e)
                dBf[((((size_t)d * 2 + s) * nqf + qf) * 3 + e) * nm + n] = dbasis(n, e, xi);
            }
          }
  }
  double basis(int n, const double xi[3]) const {
    double r = 1.0;
    for (int e = 0; e < 3; ++e) {
      double P[8], dP[8];
      legendre(md[n].n[e], xi[e], P, dP);
      r *= P[md[n].n[e]];
    }
    return r;
  }
  // reference-coordinate derivative d/dxi_e of B_n
  double dbasis(int n, int e, const double xi[3]) const {
    double r = 1.0;
    for (int f = 0; f < 3; ++f) {
      double P[8], dP[8];
      legendre(md[n].n[f], xi[f], P, dP);
      r *= (f == e) ? dP[md[n].n[f]] : P[md[n].n[f]];
    }
    return r;
  }
  int64_t cell(int i, int j, int k) const {
    i = (i % c.nx + c.nx) % c.nx;
    j = (j % c.ny + c.ny) % c.ny;
    k = (k % c.nz + c.nz) % c.nz;
    return ((int64_t)k * c.ny + j) * c.nx + i;
  }
  void ijk(int64_t cc, int& i, int& j, int& k) const {
    i = (int)(cc % c.nx);
    j = (int)((cc / c.nx) % c.ny);
    k = (int)(cc / ((int64_t)c.nx * c.ny));
  }
  size_t idx(int v, int n, int64_t cc) const { return ((size_t)v * nm + n) * (size_t)ncell + (size_t)cc; }
  // width of cell cc along axis e, its volume |K| and the area |Gamma_d| of its d-faces
  double width(int e, int64_t cc) const {
    int p[3];
    ijk(cc, p[0], p[1], p[2]);
    return wd[e][p[e]];
  }
  double cvol(int64_t cc) const { return width(0, cc) * width(1, cc) * width(2, cc); }
  double carea(int d, int64_t cc) const { return cvol(cc) / width(d, cc); }
  // physical coordinate of the reference point xi in cell cc
  void xphys(int64_t cc, const double xi[3], double x[3]) const {
    int p[3];
    ijk(cc, p[0], p[1], p[2]);
    for (int e = 0; e < 3; ++e) x[e] = xl[e][p[e]] + (0.5 + 0.5 * xi[e]) * wd[e][p[e]];
  }
  int64_t neighbor(int64_t cc, int d, int off) const {
    int i, j, k;
    ijk(cc, i, j, k);
    int p[3] = {i, j, k};
    p[d] += off;
    return cell(p[0], p[1], p[2]);
  }
};

// Point values Q and physical gradients dQ/dx_e from the modal coefficients.
template <class R>
static void eval_point(const Disc& D, const R* q, int64_t cc, const double* B, const double* dB, R Q[5], R dQ[3][5]) {
  for (int v = 0; v < 5; ++v) {
    R s = R(0.0), g[3] = {R(0.0), R(0.0), R(0.0)};
    for (int n = 0; n < D.nm; ++n) {
      R qn = q[D.idx(v, n, cc)];
      s += qn * R(B[n]);
      for (int e = 0; e < 3; ++e) g[e] += qn * R(dB[e * D.nm + n]);
    }
    Q[v] = s;
    for (int e = 0; e < 3; ++e) dQ[e][v] = g[e] * R(2.0 / D.width(e, cc));
  }
}

// Face flux at the upper face of cell cc in direction d, at all face points.
// out: F[qf][5], Ft[qf][5].
template <class R>
static void face_fluxes(const Disc& D, R mu, double dt, const R* q, int64_t cc, int d, R* F, R* Ft) {
  const int nqf = D.nq * D.nq;
  int64_t cr = D.neighbor(cc, d, +1);
  for (int qf = 0; qf < nqf; ++qf) {
    R QL[5], dQL[3][5], QR[5], dQR[3][5];
    eval_point(D, q, cc, &D.Bf[(((size_t)d * 2 + 0) * nqf + qf) * D.nm],
               &D.dBf[((((size_t)d * 2 + 0) * nqf + qf) * 3) * D.nm], QL, dQL);
    eval_point(D, q, cr, &D.Bf[(((size_t)d * 2 + 1) * nqf + qf) * D.nm],
               &D.dBf[((((size_t)d * 2 + 1) * nqf + qf) * 3) * D.nm], QR, dQR);
    face_flux(D.c, mu, dt, d, QL, dQL, QR, dQR, &F[qf * 5], &Ft[qf * 5]);
  }
}

// R_n = -sum_faces |Gamma| sum_q w_q F_b.n B_n + |K| sum_q w_q F_v . grad B_n,
// then L = M^{-1} R (diagonal M).  Fup/Ftup: fluxes of the upper faces of the
// cell (one block per direction), Flo/Ftlo: of its lower faces.
template <class R>
static void assemble_cell(const Disc& D, R mu, const R* q, int64_t cc, const R* const Fup[3], const R* const Ftup[3],
                          const R* const Flo[3], const R* const Ftlo[3], R* Lc, R* Ltc) {
  const int nm = D.nm, nq = D.nq, nqf = nq * nq, nqv = nq * nq * nq;
  const double vol = D.cvol(cc);
  std::vector<R> Rr(5 * nm, R(0.0)), Rt(5 * nm, R(0.0));
  for (int g = 0; g < nq; ++g)
    for (int b = 0; b < nq; ++b)
      for (int a = 0; a < nq; ++a) {
        int qi = (g * nq + b) * nq + a;
        double w = D.wg[a] * D.wg[b] * D.wg[g];
        R Q[5], dQ[3][5], F[3][5], Ft[3][5];
        eval_point(D, q, cc, &D.Bv[(size_t)qi * nm], &D.dBv[(size_t)qi * 3 * nm], Q, dQ);
        volume_flux(D.c, mu, Q, dQ, F, Ft);
        for (int n = 0; n < nm; ++n)
          for (int e = 0; e < 3; ++e) {
            double gB = D.dBv[((size_t)qi * 3 + e) * nm + n] * 2.0 / D.width(e, cc);
            for (int v = 0; v < 5; ++v) {
              Rr[v * nm + n] += R(vol * w * gB) * F[e][v];
              Rt[v * nm + n] += R(vol * w * gB) * Ft[e][v];
            }
          }
      }
  (void)nqv;
  for (int d = 0; d < 3; ++d)
    for (int bq = 0; bq < nq; ++bq)
      for (int aq = 0; aq < nq; ++aq) {
        int qf = bq * nq + aq;
        double w = D.wg[aq] * D.wg[bq];
        const double area = D.carea(d, cc);
        for (int n = 0; n < nm; ++n) {
          double Bup = D.Bf[(((size_t)d * 2 + 0) * nqf + qf) * nm + n];
          double Blo = D.Bf[(((size_t)d * 2 + 1) * nqf + qf) * nm + n];
          for (int v = 0; v < 5; ++v) {
            Rr[v * nm + n] -= R(area * w * Bup) * Fup[d][qf * 5 + v];
            Rr[v * nm + n] += R(area * w * Blo) * Flo[d][qf * 5 + v];
            Rt[v * nm + n] -= R(area * w * Bup) * Ftup[d][qf * 5 + v];
            Rt[v * nm + n] += R(area * w * Blo) * Ftlo[d][qf * 5 + v];
          }
        }
      }
  for (int v = 0; v < 5; ++v)
    for (int n = 0; n < nm; ++n) {
      Lc[v * nm + n] = Rr[v * nm + n] / R(D.mass[n] * vol);
      Ltc[v * nm + n] = Rt[v * nm + n] / R(D.mass[n] * vol);
    }
}

// L(Q), L_t(Q) on every cell: each face flux is computed once (upper face of
// each cell) and used with opposite signs by its two cells.
template <class R>
static void residual(const Disc& D, R mu, double dt, const R* q, R* L, R* Lt) {
  const int nqf = D.nq * D.nq, nm = D.nm;
  const int64_t N = D.ncell;
  std::vector<R> Fb((size_t)3 * N * nqf * 5), Ftb((size_t)3 * N * nqf * 5);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < 3 * N; ++t) {
    int d = (int)(t / N);
    int64_t cc = t % N;
    face_fluxes(D, mu, dt, q, cc, d, &Fb[(size_t)t * nqf * 5], &Ftb[(size_t)t * nqf * 5]);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t cc = 0; cc < N; ++cc) {
    const R* Fup[3];
    const R* Ftup[3];
    const R* Flo[3];
    const R* Ftlo[3];
    for (int d = 0; d < 3; ++d) {
      int64_t lo = D.neighbor(cc, d, -1);
      Fup[d] = &Fb[((size_t)d * N + cc) * nqf * 5];
      Ftup[d] = &Ftb[((size_t)d * N + cc) * nqf * 5];
      Flo[d] = &Fb[((size_t)d * N + lo) * nqf * 5];
      Ftlo[d] = &Ftb[((size_t)d * N + lo) * nqf * 5];
    }
    std::vector<R> Lc(5 * nm), Ltc(5 * nm);
    assemble_cell(D, mu, q, cc, Fup, Ftup, Flo, Ftlo, Lc.data(), Ltc.data());
    for (int v = 0; v < 5; ++v)
      for (int n = 0; n < nm; ++n) {
        L[D.idx(v, n, cc)] = Lc[v * nm + n];
        Lt[D.idx(v, n, cc)] = Ltc[v * nm + n];
      }
  }
}

// L, L_t for a list of cells only; each cell computes its own six faces.
// Output layout: [cell_in_list][var][mode].
template <class R>
static void residual_cells(const Disc& D, R mu, double dt, const R* q, const int64_t* cells, int64_t ncells, R* L,
                           R* Lt) {
  const int nqf = D.nq * D.nq, nm = D.nm;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < ncells; ++t) {
    int64_t cc = cells[t];
    std::vector<R> up(3 * nqf * 5), tup(3 * nqf * 5), lo(3 * nqf * 5), tlo(3 * nqf * 5);
    const R* Fup[3];
    const R* Ftup[3];
    const R* Flo[3];
    const R* Ftlo[3];
    for (int d = 0; d < 3; ++d) {
      face_fluxes(D, mu, dt, q, cc, d, &up[d * nqf * 5], &tup[d * nqf * 5]);
      face_fluxes(D, mu, dt, q, D.neighbor(cc, d, -1), d, &lo[d * nqf * 5], &tlo[d * nqf * 5]);
      Fup[d] = &up[d * nqf * 5];
      Ftup[d] = &tup[d * nqf * 5];
      Flo[d] = &lo[d * nqf * 5];
      Ftlo[d] = &tlo[d * nqf * 5];
    }
    assemble_cell(D, mu, q, cc, Fup, Ftup, Flo, Ftlo, &L[(size_t)t * 5 * nm], &Lt[(size_t)t * 5 * nm]);
  }
}

// Residual of the cells whose z index lies in [k0, k1): every face touching
// those cells is computed once.  Used only to time a bounded sample.
static void residual_slab(const Disc& D, double mu, double dt, const double* q, int k0, int k1, double* L,
                          double* Lt) {
  const int nqf = D.nq * D.nq, nm = D.nm;
  const int64_t plane = (int64_t)D.c.nx * D.c.ny;
  const int64_t nsl = plane * (k1 - k0);
  // faces: x and y upper faces of slab cells, z upper faces of cells in [k0-1, k1)
  std::vector<double> Fb((size_t)(3 * nsl + plane) * nqf * 5), Ftb(Fb.size());
  auto fidx = [&](int d, int64_t cc) -> int64_t {
    int i, j, k;
    D.ijk(cc, i, j, k);
    int64_t p = (int64_t)j * D.c.nx + i;
    if (d < 2) return d * nsl + (k - k0) * plane + p;
    int kk = (k - (k0 - 1) + D.c.nz) % D.c.nz;  // 0 .. nslab
    return 2 * nsl + kk * plane + p;
  };
  const int64_t nf = 3 * nsl + plane;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nf; ++t) {
    int d;
    int64_t cc;
    if (t < 2 * nsl) {
      d = (int)(t / nsl);
      cc = (int64_t)k0 * plane + t % nsl;
    } else {
      d = 2;
      int64_t r = t - 2 * nsl;
      int k = (int)((k0 - 1 + r / plane + D.c.nz) % D.c.nz);
      cc = (int64_t)k * plane + r % plane;
    }
    face_fluxes(D, mu, dt, q, cc, d, &Fb[(size_t)fidx(d, cc) * nqf * 5], &Ftb[(size_t)fidx(d, cc) * nqf * 5]);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nsl; ++t) {
    int64_t cc = (int64_t)k0 * plane + t;
    const double* Fup[3];
    const double* Ftup[3];
    const double* Flo[3];
    const double* Ftlo[3];
    for (int d = 0; d < 3; ++d) {
      int64_t lo = D.neighbor(cc, d, -1);
      if (d < 2) {  // lower x/y face of a slab cell is the upper face of a slab cell
        Fup[d] = &Fb[(size_t)fidx(d, cc) * nqf * 5];
        Ftup[d] = &Ftb[(size_t)fidx(d, cc) * nqf * 5];
        Flo[d] = &Fb[(size_t)fidx(d, lo) * nqf * 5];
        Ftlo[d] = &Ftb[(size_t)fidx(d, lo) * nqf * 5];
      } else {
        Fup[d] = &Fb[(size_t)fidx(2, cc) * nqf * 5];
        Ftup[d] = &Ftb[(size_t)fidx(2, cc) * nqf * 5];
        Flo[d] = &Fb[(size_t)fidx(2, lo) * nqf * 5];
        Ftlo[d] = &Ftb[(size_t)fidx(2, lo) * nqf * 5];
      }
    }
    assemble_cell(D, mu, q, cc, Fup, Ftup, Flo, Ftlo, &L[(size_t)t * 5 * nm], &Lt[(size_t)t * 5 * nm]);
  }
}

// Eq. (two-stage): Q* = Q^n + dt/2 L(Q^n) + dt^2/8 L_t(Q^n),
// Q^{n+1} = Q^n + dt L(Q^n) + dt^2/6 (L_t(Q^n) + 2 L_t(Q*)).  `op(Q, L, Lt)`
// evaluates the operator; the stage at t* = t_n + dt/2 uses the same time
// windows [0, dt] and [0, dt/2] measured from t*.
template <class R>
static inline R stage_star(R qn, R L, R Lt, double dt) {
  return qn + R(0.5 * dt) * L + R(dt * dt / 8.0) * Lt;
}
template <class R>
static inline R stage_final(R qn, R L, R Lt, R Lt_star, double dt) {
  return qn + R(dt) * L + R(dt * dt / 6.0) * (Lt + R(2.0) * Lt_star);
}

template <class R, class Op>
static void s2o4_update(size_t n, double dt, R* q, Op op) {
  std::vector<R> L(n), Lt(n), Qs(n), L2(n), Lt2(n);
  op(q, L.data(), Lt.data());
  for (size_t i = 0; i < n; ++i) Qs[i] = stage_star(q[i], L[i], Lt[i], dt);
  op(Qs.data(), L2.data(), Lt2.data());
  for (size_t i = 0; i < n; ++i) q[i] = stage_final(q[i], L[i], Lt[i], Lt2[i], dt);
}

template <class R>
static void s2o4_step(const Disc& D, R mu, double dt, R* q) {
  const size_t n = (size_t)5 * D.nm * D.ncell;
  s2o4_update(n, dt, q, [&](const R* x, R* L, R* Lt) { residual(D, mu, dt, x, L, Lt); });
}

// One S2O4 step evaluated only where it is needed to return Q^{n+1} at the
// listed cells: stage 1 on the cells and their six face neighbours, stage 2
// on the listed cells.  Output layout [cell_in_list][var][mode].
static void step_cells(const Disc& D, double mu, double dt, const double* q, const int64_t* cells, int64_t ncells,
                       double* out) {
  const int nm = D.nm;
  std::vector<int64_t> s1;
  for (int64_t t = 0; t < ncells; ++t) {
    s1.push_back(cells[t]);
    for (int d = 0; d < 3; ++d) {
      s1.push_back(D.neighbor(cells[t], d, -1));
      s1.push_back(D.neighbor(cells[t], d, +1));
    }
  }
  std::sort(s1.begin(), s1.end());
  s1.erase(std::unique(s1.begin(), s1.end()), s1.end());
  const int64_t n1 = (int64_t)s1.size();
  std::vector<double> L(n1 * 5 * nm), Lt(n1 * 5 * nm);
  residual_cells(D, mu, dt, q, s1.data(), n1, L.data(), Lt.data());
  std::vector<double> qs(q, q + (size_t)5 * nm * D.ncell);
  for (int64_t t = 0; t < n1; ++t)
    for (int v = 0; v < 5; ++v)
      for (int n = 0; n < nm; ++n) {
        size_t gi = D.idx(v, n, s1[t]);
        qs[gi] = stage_star(q[gi], L[(t * 5 + v) * nm + n], Lt[(t * 5 + v) * nm + n], dt);
      }
  std::vector<double> L2(ncells * 5 * nm), Lt2(ncells * 5 * nm);
  residual_cells(D, mu, dt, qs.data(), cells, ncells, L2.data(), Lt2.data());
  for (int64_t t = 0; t < ncells; ++t) {
    int64_t r = std::lower_bound(s1.begin(), s1.end(), cells[t]) - s1.begin();
    for (int v = 0; v < 5; ++v)
      for (int n = 0; n < nm; ++n) {
        size_t gi = D.idx(v, n, cells[t]);
        out[(t * 5 + v) * nm + n] = stage_final(q[gi], L[(r * 5 + v) * nm + n], Lt[(r * 5 + v) * nm + n],
                                                Lt2[(t * 5 + v) * nm + n], dt);
      }
  }
}

// L^2 projection of a pointwise state onto the P_k basis (6-point rule).
typedef void (*StateFn)(const double x[3], const Cfg& c, int which, double Q[5]);

static void exact_state(const double x[3], const Cfg& c, int which, double Q[5]) {
  double rho, U[3], p;
  if (which == 0) {
    // Section 5.1: 3-D density advection on [0,2]^3, U=V=W=1, p=1.
    rho = 1.0 + 0.2 * std::sin(kPi * (x[0] + x[1] + x[2]));
    U[0] = U[1] = U[2] = 1.0;
    p = 1.0;
  } else if (which == 1) {
    // Section 5.3: Taylor-Green vortex, L = V0 = rho0 = 1, Mach 0.1.
    const double Ma = 0.1;
    rho = 1.0;
    U[0] = std::sin(x[0]) * std::cos(x[1]) * std::cos(x[2]);
    U[1] = -std::cos(x[0]) * std::sin(x[1]) * std::cos(x[2]);
    U[2] = 0.0;
    p = 1.0 / (c.gamma * Ma * Ma) + (std::cos(2 * x[0]) + std::cos(2 * x[1])) * (std::cos(2 * x[2]) + 2.0) / 16.0;
  } else {
    // one-dimensional advection along x: rho = 1 + 0.2 sin(pi x), U=1, V=W=0, p=1
    int ax = which - 2;  // 2,3,4 -> along x,y,z
    rho = 1.0 + 0.2 * std::sin(kPi * x[ax]);
    U[0] = U[1] = U[2] = 0.0;
    U[ax] = 1.0;
    p = 1.0;
  }
  Q[0] = rho;
  for (int i = 0; i < 3; ++i) Q[1 + i] = rho * U[i];
  Q[4] = p / (c.gamma - 1.0) + 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
}

static void project(const Disc& D, int which, double* q) {
  const int ng = 6;
  double xg[ng], wg[ng];
  gauss_legendre(ng, xg, wg);
  for (auto& w : wg) w *= 0.5;
#pragma omp parallel for schedule(static)
  for (int64_t cc = 0; cc < D.ncell; ++cc) {
    std::vector<double> acc(5 * D.nm, 0.0);
    for (int g = 0; g < ng; ++g)
      for (int b = 0; b < ng; ++b)
        for (int a = 0; a < ng; ++a) {
          double xi[3] = {xg[a], xg[b], xg[g]};
          double x[3];
          D.xphys(cc, xi, x);
          double Q[5];
          exact_state(x, D.c, which, Q);
          double w = wg[a] * wg[b] * wg[g] * D.cvol(cc);
          for (int n = 0; n < D.nm; ++n) {
            double B = D.basis(n, xi);
            for (int v = 0; v < 5; ++v) acc[v * D.nm + n] += w * Q[v] * B;
          }
        }
    for (int v = 0; v < 5; ++v)
      for (int n = 0; n < D.nm; ++n) q[D.idx(v, n, cc)] = acc[v * D.nm + n] / (D.mass[n] * D.cvol(cc));
  }
}

// Domain-integrated kinetic energy J = sum_K |K| sum_q w_q |rho U|^2 / (2 rho)
// on the scheme's own volume rule.
template <class R>
static R kinetic_energy(const Disc& D, const R* q) {
  const int nq = D.nq, nm = D.nm;
  std::vector<R> part(D.ncell);
#pragma omp parallel for schedule(static)
  for (int64_t cc = 0; cc < D.ncell; ++cc) {
    R s = R(0.0);
    for (int qi = 0; qi < nq * nq * nq; ++qi) {
      int a = qi % nq, b = (qi / nq) % nq, g = qi / (nq * nq);
      double w = D.wg[a] * D.wg[b] * D.wg[g];
      R Q[5];
      for (int v = 0; v < 4; ++v) {
        R t = R(0.0);
        for (int n = 0; n < nm; ++n) t += q[D.idx(v, n, cc)] * R(D.Bv[(size_t)qi * nm + n]);
        Q[v] = t;
      }
      s += R(w) * (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / (R(2.0) * Q[0]);
    }
    part[cc] = s * R(D.cvol(cc));
  }
  R J = R(0.0);
  for (int64_t cc = 0; cc < D.ncell; ++cc) J += part[cc];
  return J;
}

// Enstrophy, sum_K |K| sum_q w_q |omega|^2 / 2 with omega = curl U, U = rho U / rho
// (the Taylor-Green diagnostic of Section 5.3), from the DG point values and
// gradients at the volume Gauss points.
static double enstrophy(const Disc& D, const double* q) {
  const int nq = D.nq, nm = D.nm;
  std::vector<double> part(D.ncell);
#pragma omp parallel for schedule(static)
  for (int64_t cc = 0; cc < D.ncell; ++cc) {
    double s = 0.0;
    for (int qi = 0; qi < nq * nq * nq; ++qi) {
      int a = qi % nq, b = (qi / nq) % nq, g = qi / (nq * nq);
      double w = D.wg[a] * D.wg[b] * D.wg[g];
      double Q[4] = {0, 0, 0, 0}, G[4][3] = {{0}};  // G[v][e] = dQ_v/dx_e
      for (int v = 0; v < 4; ++v)
        for (int n = 0; n < nm; ++n) {
          const double c = q[D.idx(v, n, cc)];
          Q[v] += c * D.Bv[(size_t)qi * nm + n];
          for (int e = 0; e < 3; ++e) G[v][e] += c * D.dBv[((size_t)qi * 3 + e) * nm + n] * 2.0 / D.width(e, cc);
        }
      // dU_j/dx_e = (d(rho U_j)/dx_e - U_j drho/dx_e) / rho
      double dU[3][3];
      for (int j = 0; j < 3; ++j)
        for (int e = 0; e < 3; ++e) dU[j][e] = (G[1 + j][e] - Q[1 + j] / Q[0] * G[0][e]) / Q[0];
      const double ox = dU[2][1] - dU[1][2], oy = dU[0][2] - dU[2][0], oz = dU[1][0] - dU[0][1];
      s += w * 0.5 * (ox * ox + oy * oy + oz * oz);
    }
    part[cc] = s * D.cvol(cc);
  }
  double E = 0.0;
  for (int64_t cc = 0; cc < D.ncell; ++cc) E += part[cc];
  return E;
}

// L^2 error of the density against the exact advection solution at time t
// (Section 5.1 error norm, Gaussian quadrature with nqe points per direction).
static double advection_l2_error(const Disc& D, const double* q, double t, int which, int nqe) {
  std::vector<double> xg(nqe), wg(nqe);
  gauss_legendre(nqe, xg.data(), wg.data());
  for (auto& w : wg) w *= 0.5;
  double err = 0.0;
#pragma omp parallel for reduction(+ : err) schedule(static)
  for (int64_t cc = 0; cc < D.ncell; ++cc) {
    for (int g = 0; g < nqe; ++g)
      for (int b = 0; b < nqe; ++b)
        for (int a = 0; a < nqe; ++a) {
          double xi[3] = {xg[a], xg[b], xg[g]};
          double x[3];
          D.xphys(cc, xi, x);
          double rho_h = 0.0;
          for (int n = 0; n < D.nm; ++n) rho_h += q[D.idx(0, n, cc)] * D.basis(n, xi);
          double rho_e;
          if (which == 0)
            rho_e = 1.0 + 0.2 * std::sin(kPi * (x[0] + x[1] + x[2] - 3.0 * t));
          else
            rho_e = 1.0 + 0.2 * std::sin(kPi * (x[which - 2] - t));
          double dr = rho_h - rho_e;
          err += wg[a] * wg[b] * wg[g] * D.cvol(cc) * dr * dr;
        }
  }
  return std::sqrt(err);
}

}  // namespace dgo

// ===========================================================================
// C entry points for the Python test harness (ctypes).
// ===========================================================================
using namespace dgo;

extern "C" {

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_gauss(int n, double* x, double* w) { gauss_legendre(n, x, w); }

void orc_legendre(int lmax, double x, double* P, double* dP) { legendre(lmax, x, P, dP); }

int orc_nmodes(int k) { return (int)mode_list(k).size(); }

void orc_modes(int k, int* out) {
  auto m = mode_list(k);
  for (size_t i = 0; i < m.size(); ++i)
    for (int e = 0; e < 3; ++e) out[3 * i + e] = m[i].n[e];
}

// Moment tables: out_u[9] for the normal component (full/half), out_x[3].
void orc_moments(double U, double lam, double K, int half_side, double* out_u, double* out_x) {
  double Uv[3] = {U, 0.0, 0.0};
  Tab<double> t = make_tab(Uv, lam, K, half_side);
  for (int i = 0; i < kMomMax; ++i) out_u[i] = t.u[i];
  for (int i = 0; i < 3; ++i) out_x[i] = t.x[i];
}

// 5x5 moment matrix <psi_k psi_j> and the slope solve for a state (rho unused).
void orc_slope(const double U[3], double lam, double K, const double b[5], double* a, double* M) {
  Tab<double> t = make_tab(U, lam, K, 0);
  double G[5][5];
  gmat(t, 0, 0, 0, G);
  for (int i = 0; i < 25; ++i) M[i] = G[i / 5][i % 5];
  solve5(G, b, a);
}

void orc_time_integrals(double tau, double delta, double* c) { time_integrals(tau, delta, c); }

void orc_volume_flux(const Cfg* c, const double* q, const double* dq, double* F, double* Ft) {
  double dqa[3][5], Fa[3][5], Fta[3][5];
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) dqa[e][v] = dq[e * 5 + v];
  volume_flux(*c, c->mu, q, dqa, Fa, Fta);
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) {
      F[e * 5 + v] = Fa[e][v];
      Ft[e * 5 + v] = Fta[e][v];
    }
}

void orc_face_flux(const Cfg* c, double dt, int d, const double* qL, const double* dqL, const double* qR,
                   const double* dqR, double* F, double* Ft) {
  double a[3][5], b[3][5];
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) {
      a[e][v] = dqL[e * 5 + v];
      b[e][v] = dqR[e * 5 + v];
    }
  face_flux(*c, c->mu, dt, d, qL, a, qR, b, F, Ft);
}

// Mass matrix entry M_{n1 n2} / |K| by an exact Gauss rule (for pins).
double orc_mass_entry(int k, int n1, int n2) {
  Cfg c{};
  c.nx = c.ny = c.nz = 1;
  c.k = k;
  c.nq = k + 1;
  for (int e = 0; e < 3; ++e) { c.lo[e] = 0; c.hi[e] = 1; }
  c.gamma = 1.4;
  c.prandtl = 1;
  Disc D(c);
  int nm1 = k + 1;
  std::vector<double> x(nm1), w(nm1);
  gauss_legendre(nm1, x.data(), w.data());
  double s = 0;
  for (int a = 0; a < nm1; ++a)
    for (int b = 0; b < nm1; ++b)
      for (int g = 0; g < nm1; ++g) {
        double xi[3] = {x[a], x[b], x[g]};
        s += 0.125 * w[a] * w[b] * w[g] * D.basis(n1, xi) * D.basis(n2, xi);
      }
  return s;
}

void orc_residual(const Cfg* c, const double* q, double dt, double* L, double* Lt) {
  Disc D(*c);
  residual(D, c->mu, dt, q, L, Lt);
}

void orc_residual_cells(const Cfg* c, const double* q, double dt, const int64_t* cells, int64_t n, double* L,
                        double* Lt) {
  Disc D(*c);
  residual_cells(D, c->mu, dt, q, cells, n, L, Lt);
}

void orc_residual_slab(const Cfg* c, const double* q, double dt, int k0, int k1, double* L, double* Lt) {
  Disc D(*c);
  residual_slab(D, c->mu, dt, q, k0, k1, L, Lt);
}

void orc_step_cells(const Cfg* c, const double* q, double dt, const int64_t* cells, int64_t n, double* out) {
  Disc D(*c);
  step_cells(D, c->mu, dt, q, cells, n, out);
}

void orc_step(const Cfg* c, double* q, double dt, int nsteps) {
  Disc D(*c);
  for (int s = 0; s < nsteps; ++s) s2o4_step(D, c->mu, dt, q);
}

void orc_project(const Cfg* c, int which, double* q) {
  Disc D(*c);
  project(D, which, q);
}

double orc_kinetic_energy(const Cfg* c, const double* q) {
  Disc D(*c);
  return kinetic_energy(D, q);
}

double orc_enstrophy(const Cfg* c, const double* q) {
  Disc D(*c);
  return enstrophy(D, q);
}

double orc_advection_error(const Cfg* c, const double* q, double t, int which, int nqe) {
  Disc D(*c);
  return advection_l2_error(D, q, t, which, nqe);
}

// Forward-mode derivative of nsteps S2O4 steps: (q, dq, dmu) -> (q_out, dq_out).
void orc_step_jvp(const Cfg* c, const double* q, const double* dq, double dmu, double dt, int nsteps, double* q_out,
                  double* dq_out) {
  Disc D(*c);
  const size_t n = (size_t)5 * D.nm * D.ncell;
  std::vector<Dual> Q(n);
  for (size_t i = 0; i < n; ++i) Q[i] = Dual(q[i], dq[i]);
  Dual mu(c->mu, dmu);
  for (int s = 0; s < nsteps; ++s) s2o4_step(D, mu, dt, Q.data());
  for (size_t i = 0; i < n; ++i) {
    q_out[i] = Q[i].v;
    dq_out[i] = Q[i].d;
  }
}

// J(q) and its directional derivative along dq.
void orc_ke_jvp(const Cfg* c, const double* q, const double* dq, double* J, double* dJ) {
  Disc D(*c);
  const size_t n = (size_t)5 * D.nm * D.ncell;
  std::vector<Dual> Q(n);
  for (size_t i = 0; i < n; ++i) Q[i] = Dual(q[i], dq[i]);
  Dual r = kinetic_energy(D, Q.data());
  *J = r.v;
  *dJ = r.d;
}

// Directional derivative of the point fluxes (for pins of the dual type).
void orc_volume_flux_jvp(const Cfg* c, const double* q, const double* dq, const double* tq, const double* tdq,
                         double tmu, double* F, double* dF, double* Ft, double* dFt) {
  Dual Q[5], dQ[3][5], Fa[3][5], Fta[3][5];
  for (int v = 0; v < 5; ++v) Q[v] = Dual(q[v], tq[v]);
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) dQ[e][v] = Dual(dq[e * 5 + v], tdq[e * 5 + v]);
  volume_flux(*c, Dual(c->mu, tmu), Q, dQ, Fa, Fta);
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) {
      F[e * 5 + v] = Fa[e][v].v;
      dF[e * 5 + v] = Fa[e][v].d;
      Ft[e * 5 + v] = Fta[e][v].v;
      dFt[e * 5 + v] = Fta[e][v].d;
    }
}

void orc_face_flux_jvp(const Cfg* c, double dt, int d, const double* x, const double* tx, double tmu, double* F,
                       double* dF, double* Ft, double* dFt) {
  // x = [qL(5), dqL(15), qR(5), dqR(15)], tx = tangent of the same layout
  Dual qL[5], qR[5], dqL[3][5], dqR[3][5], Fo[5], Fto[5];
  for (int v = 0; v < 5; ++v) {
    qL[v] = Dual(x[v], tx[v]);
    qR[v] = Dual(x[20 + v], tx[20 + v]);
  }
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) {
      dqL[e][v] = Dual(x[5 + e * 5 + v], tx[5 + e * 5 + v]);
      dqR[e][v] = Dual(x[25 + e * 5 + v], tx[25 + e * 5 + v]);
    }
  face_flux(*c, Dual(c->mu, tmu), dt, d, qL, dqL, qR, dqR, Fo, Fto);
  for (int v = 0; v < 5; ++v) {
    F[v] = Fo[v].v;
    dF[v] = Fo[v].d;
    Ft[v] = Fto[v].v;
    dFt[v] = Fto[v].d;
  }
}

// S2O4 applied to the scalar linear ODE dQ/dt = z Q (L = z Q, L_t = z^2 Q),
// through the same stage update as the grid step.
double orc_s2o4_linear(double z, double dt, int nsteps) {
  double q = 1.0;
  for (int s = 0; s < nsteps; ++s)
    s2o4_update(1, dt, &q, [&](const double* x, double* L, double* Lt) {
      L[0] = z * x[0];
      Lt[0] = z * z * x[0];
    });
  return q;
}

}  // extern "C"
