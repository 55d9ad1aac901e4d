// dg_tables.hpp -- compile-time tables of the modal DG discretisation.
//
// Basis (Section 3, Eq. (expansion)): B_n = P_nx(xi) P_ny(eta) P_nz(zeta)
// with Legendre polynomials P_l on [-1,1] and nx+ny+nz <= k (the P_k space,
// (k+1)(k+2)(k+3)/6 modes).  Mode order: by total degree s = 0..k, then nx
// from s down to 0, then ny from s-nx down to 0.  This order is part of the
// C-ABI layout of the coefficient arrays.
//
// Gauss-Legendre nodes on [-1,1] with weights normalised to sum 1 (the
// textbook weights divided by 2), used for Eq. (surface) and Eq. (volume).
#pragma once

#include <hip/hip_runtime.h>

namespace dgk {

#define DGK_HD __host__ __device__ __forceinline__

template <int NQ>
struct Gauss;
template <>
struct Gauss<1> {
  static constexpr double x[1] = {0.0};
  static constexpr double w[1] = {1.0};
};
template <>
struct Gauss<2> {
  static constexpr double x[2] = {-0.57735026918962576451, 0.57735026918962576451};
  static constexpr double w[2] = {0.5, 0.5};
};
template <>
struct Gauss<3> {
  static constexpr double x[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
  static constexpr double w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
};
template <>
struct Gauss<4> {
  static constexpr double x[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                                  0.86113631159405257522};
  static constexpr double w[4] = {0.17392742256872692869, 0.32607257743127307131, 0.32607257743127307131,
                                  0.17392742256872692869};
};

// Legendre polynomials P_0..P_3 and derivatives.
DGK_HD constexpr double leg(int l, double x) {
  return l == 0 ? 1.0 : l == 1 ? x : l == 2 ? 0.5 * (3.0 * x * x - 1.0) : 0.5 * (5.0 * x * x * x - 3.0 * x);
}
DGK_HD constexpr double dleg(int l, double x) {
  return l == 0 ? 0.0 : l == 1 ? 1.0 : l == 2 ? 3.0 * x : 0.5 * (15.0 * x * x - 3.0);
}

DGK_HD constexpr int nmodes(int k) { return (k + 1) * (k + 2) * (k + 3) / 6; }
DGK_HD constexpr int ntan(int k) { return (k + 1) * (k + 2) / 2; }

// Multi-index of mode n of P_k.
template <int K>
struct Modes {
  static constexpr int N = nmodes(K);
  int e[N][3];
  constexpr Modes() : e{} {
    int n = 0;
    for (int s = 0; s <= K; ++s)
      for (int a = s; a >= 0; --a)
        for (int b = s - a; b >= 0; --b) {
          e[n][0] = a;
          e[n][1] = b;
          e[n][2] = s - a - b;
          ++n;
        }
  }
};

// Two-dimensional (tangential) modes of degree <= K, same ordering rule:
// (a, b) with a from s down to 0 and b = s - a.
template <int K>
struct TanModes {
  static constexpr int N = ntan(K);
  int e[N][2];
  constexpr TanModes() : e{} {
    int n = 0;
    for (int s = 0; s <= K; ++s)
      for (int a = s; a >= 0; --a) {
        e[n][0] = a;
        e[n][1] = s - a;
        ++n;
      }
  }
};

template <int K>
DGK_HD constexpr int mode_e(int n, int axis) {
  return Modes<K>().e[n][axis];
}
template <int K>
DGK_HD constexpr int tan_e(int m, int i) {
  return TanModes<K>().e[m][i];
}
// Index of the tangential mode (a, b) in TanModes<K>.
template <int K>
DGK_HD constexpr int tan_index(int a, int b) {
  int s = a + b;
  return s * (s + 1) / 2 + (s - a);
}
// For a face with normal axis d, the tangential axes are (d+1)%3, (d+2)%3.
template <int K>
DGK_HD constexpr int face_tan_of_mode(int n, int d) {
  return tan_index<K>(mode_e<K>(n, (d + 1) % 3), mode_e<K>(n, (d + 2) % 3));
}
// 1 / (mass matrix diagonal / |K|) = (2nx+1)(2ny+1)(2nz+1)
template <int K>
DGK_HD constexpr double inv_mass(int n) {
  return double((2 * mode_e<K>(n, 0) + 1) * (2 * mode_e<K>(n, 1) + 1) * (2 * mode_e<K>(n, 2) + 1));
}

}  // namespace dgk
