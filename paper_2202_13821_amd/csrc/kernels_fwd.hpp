// kernels_fwd.hpp -- forward kernels of one S2O4 stage (HIP, gfx950).
//
// Data layout in HBM (structure of arrays, x fastest):
//   coefficients  q[var][mode][z][y][x]             (FP64 at the C-ABI; T copy inside)
//   face records  rec[dir][cell][var][F|Ft][tmode]   one record per upper face
//                 of each cell: the face flux projected on the tangential
//                 Legendre modes of the face, Phi_m = sum_q w_q F(x_q) phi_m(x_q)
//
// One stage is two launches:
//   face_kernel   -- every face of the grid once: traces of both cells at the
//                    face Gauss points (coefficients staged through LDS), the
//                    gas-kinetic face flux per point, then the projection on
//                    the tangential modes.  One lane per face point.
//   volume_kernel -- per cell: point values and gradients at the volume Gauss
//                    points, the volume flux per point, the projection
//                    sum_q w_q F_d dB_n/dx_d as a dense contraction on MFMA
//                    (v_mfma_*_16x16x4), the surface terms from the six face
//                    records, M^{-1}, and the fused stage update with FP64
//                    accumulation of the modal coefficients.
#pragma once

#include "gks_point.hpp"

namespace dgk {

#define DGK_D __device__ __forceinline__

struct Geo {
  int nx, ny, nz, pad;
  long long ncell;
  double two_inv_dx[3];  // 2 / dx_d  (reference -> physical derivative)
  double inv_dx[3];      // |Gamma_d| / |K| = 1 / dx_d
};

// Neighbour of cell c across its upper (+1) or lower (-1) face along axis d,
// periodic, in 32-bit arithmetic (the cell count is below 2^31).
DGK_D unsigned nb32(unsigned c, int d, int off, const Geo& g) {
  const unsigned nx = unsigned(g.nx), ny = unsigned(g.ny), nz = unsigned(g.nz);
  const unsigned i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
  if (d == 0) return (off > 0) ? (i + 1 == nx ? c - i : c + 1) : (i == 0 ? c + nx - 1 : c - 1);
  if (d == 1) return (off > 0) ? (j + 1 == ny ? c - j * nx : c + nx) : (j == 0 ? c + (ny - 1) * nx : c - nx);
  const unsigned pl = nx * ny;
  return (off > 0) ? (k + 1 == nz ? c - k * pl : c + pl) : (k == 0 ? c + (nz - 1) * pl : c - pl);
}

// Runtime-indexed node value of the NQ-point rule.
template <int NQ>
DGK_D double gauss_x(int i) {
  double r = Gauss<NQ>::x[0];
#pragma unroll
  for (int j = 1; j < NQ; ++j)
    if (i == j) r = Gauss<NQ>::x[j];
  return r;
}
template <int NQ>
DGK_D double gauss_w(int i) {
  double r = Gauss<NQ>::w[0];
#pragma unroll
  for (int j = 1; j < NQ; ++j)
    if (i == j) r = Gauss<NQ>::w[j];
  return r;
}

// Tables of the volume projection: B[kk][n] = w_q dB_n/dxi_d (x_q) with
// kk = 3 q + d, q = (qz NQ + qy) NQ + qx; rows padded to a multiple of 4 and
// columns to 16 with zeros (MFMA operand B of a 16x16x4 tile).
template <class T, int K, int NQ>
struct VolTab {
  static constexpr int NM = nmodes(K);
  static constexpr int KK = NQ * NQ * NQ * 3;
  static constexpr int KS = (KK + 3) / 4;
  T B[KS * 4][16];
  constexpr VolTab() : B{} {
    constexpr Modes<K> md{};
    for (int q = 0; q < NQ * NQ * NQ; ++q) {
      int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
      double x[3] = {Gauss<NQ>::x[qx], Gauss<NQ>::x[qy], Gauss<NQ>::x[qz]};
      double w = Gauss<NQ>::w[qx] * Gauss<NQ>::w[qy] * Gauss<NQ>::w[qz];
      for (int d = 0; d < 3; ++d)
        for (int n = 0; n < NM; ++n) {
          double v = w;
          for (int e = 0; e < 3; ++e) v *= (e == d) ? dleg(md.e[n][e], x[e]) : leg(md.e[n][e], x[e]);
          B[3 * q + d][n] = T(v);
        }
    }
  }
};
template <class T, int K, int NQ>
struct VolTabHolder {
  static constexpr VolTab<T, K, NQ> t{};
};

// Per-mode constants for the surface terms and the mass matrix.
template <int K>
struct ModeTab {
  static constexpr int NM = nmodes(K);
  int nd[NM][3];      // n_d
  int tm[NM][3];      // tangential mode index on a face with normal d
  double minv[NM];    // (2nx+1)(2ny+1)(2nz+1)
  constexpr ModeTab() : nd{}, tm{}, minv{} {
    constexpr Modes<K> md{};
    for (int n = 0; n < NM; ++n) {
      for (int d = 0; d < 3; ++d) {
        nd[n][d] = md.e[n][d];
        int a = md.e[n][(d + 1) % 3], b = md.e[n][(d + 2) % 3], s = a + b;
        tm[n][d] = s * (s + 1) / 2 + (s - a);
      }
      minv[n] = double((2 * md.e[n][0] + 1) * (2 * md.e[n][1] + 1) * (2 * md.e[n][2] + 1));
    }
  }
};
template <int K>
struct ModeTabHolder {
  static constexpr ModeTab<K> t{};
};

// Tangential basis at the face points: phi[m][qf] = w_a w_b P_ma(x_a) P_mb(x_b),
// qf = b NQ + a.
template <class T, int K, int NQ>
struct FaceTab {
  static constexpr int NT = ntan(K);
  T phi[NT][NQ * NQ];
  constexpr FaceTab() : phi{} {
    constexpr TanModes<K> tm{};
    for (int m = 0; m < NT; ++m)
      for (int b = 0; b < NQ; ++b)
        for (int a = 0; a < NQ; ++a)
          phi[m][b * NQ + a] = T(Gauss<NQ>::w[a] * Gauss<NQ>::w[b] * leg(tm.e[m][0], Gauss<NQ>::x[a]) *
                                 leg(tm.e[m][1], Gauss<NQ>::x[b]));
  }
};
template <class T, int K, int NQ>
struct FaceTabHolder {
  static constexpr FaceTab<T, K, NQ> t{};
};

// --------------------------------------------------------------------------
// Face kernel.  Block = 4 wavefronts; each wavefront takes FPW = 64/NQ^2
// faces, one lane per face point.  gridDim.y = face normal direction.
// --------------------------------------------------------------------------
template <int K, int NQ>
struct FaceCfg {
  static constexpr int NM = nmodes(K), NT = ntan(K), NQ2 = NQ * NQ;
  static constexpr int FPW = 64 / NQ2, FPB = 4 * FPW;
  static constexpr int CS = 5 * NM + 1;  // LDS stride of one cell's coefficients
};

template <class T, int K, int NQ, bool NEED_F, int D>
DGK_D void face_block(const T* __restrict__ q, T* __restrict__ rec, const Geo& g, const Phys& ph, int* flag,
                      long long f0, T (*sq)[FaceCfg<K, NQ>::FPB][FaceCfg<K, NQ>::CS],
                      T (*sF)[FaceCfg<K, NQ>::NQ2][10]) {
  using C = FaceCfg<K, NQ>;
  constexpr int NM = C::NM, NT = C::NT, NQ2 = C::NQ2, FPW = C::FPW, FPB = C::FPB;
  constexpr int NF = NEED_F ? 2 : 1;
  constexpr int RECN = 5 * NF * NT;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int tid = threadIdx.x;
  const long long N = g.ncell;

  // upper neighbours of the block's faces, then the coefficients of the lower
  // (side 0) and upper (side 1) cells
  __shared__ unsigned snb[FPB];
  if (tid < FPB && f0 + tid < N) snb[tid] = nb32(unsigned(f0 + tid), D, +1, g);
  __syncthreads();
  for (int idx = tid; idx < 2 * FPB * 5 * NM; idx += 256) {
    const int side = idx / (FPB * 5 * NM);
    const int r = idx - side * (FPB * 5 * NM);
    const int vm = r / FPB, j = r - vm * FPB;
    const long long f = f0 + j;
    if (f < N) {
      const long long c = side ? (long long)snb[j] : f;
      sq[side][j][vm] = q[(long long)vm * N + c];
    }
  }
  __syncthreads();

  const int w = tid >> 6, l = tid & 63;
  const int fl = w * FPW + l / NQ2, qp = l % NQ2;
  const bool active = (l < FPW * NQ2) && (f0 + fl < N);
  if (active) {
    const int qa = qp % NQ, qb = qp / NQ;
    const double xa = gauss_x<NQ>(qa), xb = gauss_x<NQ>(qb);
    T Pa[K + 1], dPa[K + 1], Pb[K + 1], dPb[K + 1];
#pragma unroll
    for (int i = 0; i <= K; ++i) {
      Pa[i] = T(leg(i, xa));
      dPa[i] = T(dleg(i, xa));
      Pb[i] = T(leg(i, xb));
      dPb[i] = T(dleg(i, xb));
    }
    const T sn = T(g.two_inv_dx[D]), s1 = T(g.two_inv_dx[T1]), s2 = T(g.two_inv_dx[T2]);
    // local frame: velocity (normal, t1, t2) = global (D, T1, T2)
    constexpr int vmap[5] = {0, 1 + D, 1 + T1, 1 + T2, 4};
    // trace of one side at the point: Q and its derivatives along (n, t1, t2)
    auto trace = [&](auto side_c, T qs[5], T dqs[3][5]) {
      constexpr int side = decltype(side_c)::value;
#pragma unroll
      for (int vl = 0; vl < 5; ++vl) {
        const T* c = &sq[side][fl][vmap[vl] * NM];
        T v0 = T(0), vn = T(0), v1 = T(0), v2 = T(0);
        static_for<NM>([&](auto nc) {
          constexpr int n = decltype(nc)::value;
          constexpr Modes<K> md{};
          constexpr int ed = md.e[n][D], e1 = md.e[n][T1], e2 = md.e[n][T2];
          // P_ed(+1) = 1, P_ed(-1) = (-1)^ed; P'_ed(+1) = ed(ed+1)/2, P'_ed(-1) = (-1)^(ed+1) ed(ed+1)/2
          constexpr double pv = (side == 0) ? 1.0 : ((ed % 2) ? -1.0 : 1.0);
          constexpr double dv = ((side == 0) ? 1.0 : ((ed % 2) ? 1.0 : -1.0)) * 0.5 * ed * (ed + 1);
          const T cn = c[n];
          const T t12 = Pa[e1] * Pb[e2];
          v0 += cn * (T(pv) * t12);
          if constexpr (ed > 0) vn += cn * (T(dv) * t12);
          if constexpr (e1 > 0) v1 += cn * (T(pv) * dPa[e1] * Pb[e2]);
          if constexpr (e2 > 0) v2 += cn * (T(pv) * Pa[e1] * dPb[e2]);
        });
        qs[vl] = v0;
        dqs[0][vl] = vn * sn;
        dqs[1][vl] = v1 * s1;
        dqs[2][vl] = v2 * s2;
      }
    };
    T F[5], Ft[5];
    int bad = 0;
    FaceAcc<T> acc;
    face_acc_zero(acc);
    {
      T qs[5], dqs[3][5];
      trace(std::integral_constant<int, 0>{}, qs, dqs);
      face_side<+1>(ph, qs, dqs, acc, bad);
    }
    {
      T qs[5], dqs[3][5];
      trace(std::integral_constant<int, 1>{}, qs, dqs);
      face_side<-1>(ph, qs, dqs, acc, bad);
    }
    face_finish<T, NEED_F>(ph, acc, F, Ft, bad);
    if (bad) atomicOr(flag, 1);
    // back to global variable order
#pragma unroll
    for (int vl = 0; vl < 5; ++vl) {
      if constexpr (NEED_F) {
        sF[fl][qp][vmap[vl]] = F[vl];
        sF[fl][qp][5 + vmap[vl]] = Ft[vl];
      } else {
        sF[fl][qp][vmap[vl]] = Ft[vl];
      }
    }
  }
  __syncthreads();
  // projection on the tangential modes: rec = sum_qf phi[m][qf] F(qf)
  const auto& ft = FaceTabHolder<T, K, NQ>::t;
  for (int o = l; o < FPW * RECN; o += 64) {
    const int fo = w * FPW + o / RECN;
    const int r = o % RECN;
    const int comp = r / NT, m = r - comp * NT;  // comp = F|Ft * 5 + var  (NF = 2) or var
    const long long f = f0 + fo;
    if (f < N) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < NQ2; ++k) s += ft.phi[m][k] * sF[fo][k][comp];
      rec[((long long)D * N + f) * RECN + r] = s;
    }
  }
}

// Minimum waves per SIMD requested for the face kernel (register budget).
#ifndef DGK_FACE_WAVES_F32
#define DGK_FACE_WAVES_F32 3
#endif
#ifndef DGK_FACE_WAVES_F64
#define DGK_FACE_WAVES_F64 1
#endif
template <class T>
struct FaceWaves {
  static constexpr int value = sizeof(T) == 4 ? DGK_FACE_WAVES_F32 : DGK_FACE_WAVES_F64;
};

template <class T, int K, int NQ, bool NEED_F>
__global__ __launch_bounds__(256, FaceWaves<T>::value) void face_kernel(const T* __restrict__ q, T* __restrict__ rec, Geo g, Phys ph,
                                                   int* flag) {
  using C = FaceCfg<K, NQ>;
  __shared__ T sq[2][C::FPB][C::CS];
  __shared__ T sF[C::FPB][C::NQ2][10];
  const long long f0 = (long long)blockIdx.x * C::FPB;
  switch (blockIdx.y) {
    case 0: face_block<T, K, NQ, NEED_F, 0>(q, rec, g, ph, flag, f0, sq, sF); break;
    case 1: face_block<T, K, NQ, NEED_F, 1>(q, rec, g, ph, flag, f0, sq, sF); break;
    default: face_block<T, K, NQ, NEED_F, 2>(q, rec, g, ph, flag, f0, sq, sF); break;
  }
}

// --------------------------------------------------------------------------
// MFMA 16x16x4: D = A B + C with lane l holding A[l%16][l/16], B[l/16][l%16];
// the four accumulator entries of lane l are rows 4 (l/16) + i (f32) or
// l/16 + 4 i (f64) of column l%16, i = 0..3 (measured on gfx950).
// --------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
template <class T>
struct Acc;
template <>
struct Acc<float> {
  using type = v4f;
};
template <>
struct Acc<double> {
  using type = v4d;
};
DGK_D v4f mfma16x16x4(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
DGK_D v4d mfma16x16x4(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <class T>
DGK_D int mfma_row(int lk, int i) {
  return sizeof(T) == 4 ? 4 * lk + i : lk + 4 * i;
}

// --------------------------------------------------------------------------
// Volume kernel.  Block = NQ wavefronts and CPB = 64/NQ^2 cells; wavefront w
// evaluates the points with z-index w, one lane per point.
// MODE 0: stage 1 (F and Ft)   -> Q* (T) and P = Q^n + dt L + dt^2/6 L_t (FP64)
// MODE 1: stage 2 (Ft only)    -> Q^{n+1} = P + dt^2/3 L_t(Q*) (FP64, + T copy)
// MODE 2: operator only        -> L, L_t (FP64)
// --------------------------------------------------------------------------
template <class T>
struct VolOut {
  const double* qn;  // MODE 0: Q^n (FP64)
  double* P;         // MODE 0 out / MODE 1 in
  T* qstar;          // MODE 0 out
  double* qnew;      // MODE 1 out (may alias qn of the next step)
  T* qshadow;        // MODE 1 out: T copy of Q^{n+1} (nullptr when T = double)
  double* L;         // MODE 2
  double* Lt;        // MODE 2
  double dt;
};

template <int K, int NQ>
struct VolCfg {
  static constexpr int NM = nmodes(K), NT = ntan(K), NQ2 = NQ * NQ, NQ3 = NQ * NQ * NQ;
  static constexpr int CPB = 64 / NQ2, NW = NQ, NTH = 64 * NQ;
  static constexpr int KK = NQ3 * 3, KS = (KK + 3) / 4;
  static constexpr int CS = 5 * NM + 1;
};

template <class T, int K, int NQ, int MODE>
__global__ __launch_bounds__(64 * NQ) void volume_kernel(const T* __restrict__ q, const T* __restrict__ rec, Geo g,
                                                        Phys ph, VolOut<T> out, int* flag) {
  using C = VolCfg<K, NQ>;
  constexpr int NM = C::NM, NT = C::NT, NQ2 = C::NQ2, CPB = C::CPB, NW = C::NW, NTH = C::NTH;
  constexpr int KK = C::KK, KS = C::KS;
  constexpr bool NEED_F = (MODE != 1);
  constexpr int NF = NEED_F ? 2 : 1;
  constexpr int NR = CPB * 5 * NF;  // rows of the projection: (cell, var, F|Ft)
  constexpr int NRT = (NR + 15) / 16;
  constexpr int RECN = 5 * NF * NT;
  // sA holds the MFMA operand, then the block's face records
  constexpr int NRA = (NR * KK >= 6 * CPB * RECN) ? NR : (6 * CPB * RECN + KK - 1) / KK;
  __shared__ T sq[CPB][C::CS];
  __shared__ T sA[NRA][KK];
  __shared__ T sR[NR][NM];
  const int tid = threadIdx.x;
  const long long N = g.ncell;
  const long long c0 = (long long)blockIdx.x * CPB;

  for (int idx = tid; idx < CPB * 5 * NM; idx += NTH) {
    const int vm = idx / CPB, j = idx - vm * CPB;
    if (c0 + j < N) sq[j][vm] = q[(long long)vm * N + c0 + j];
  }
  __syncthreads();

  const int w = tid >> 6, l = tid & 63;
  const int cl = l / NQ2, qxy = l % NQ2;
  if (cl < CPB) {
    const int qx = qxy % NQ, qy = qxy / NQ, qz = w;
    const int qi = (qz * NQ + qy) * NQ + qx;
    T F[3][5], Ft[3][5];
    if (c0 + cl < N) {
      const double x[3] = {gauss_x<NQ>(qx), gauss_x<NQ>(qy), gauss_x<NQ>(qz)};
      T P[3][K + 1], dP[3][K + 1];
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int i = 0; i <= K; ++i) {
          P[e][i] = T(leg(i, x[e]));
          dP[e][i] = T(dleg(i, x[e]));
        }
      T Q[5], dQ[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T* c = &sq[cl][v * NM];
        T v0 = T(0), vx = T(0), vy = T(0), vz = T(0);
        static_for<NM>([&](auto nc) {
          constexpr int n = decltype(nc)::value;
          constexpr Modes<K> md{};
          constexpr int a = md.e[n][0], b = md.e[n][1], e = md.e[n][2];
          const T cn = c[n];
          v0 += cn * (P[0][a] * P[1][b] * P[2][e]);
          if constexpr (a > 0) vx += cn * (dP[0][a] * P[1][b] * P[2][e]);
          if constexpr (b > 0) vy += cn * (P[0][a] * dP[1][b] * P[2][e]);
          if constexpr (e > 0) vz += cn * (P[0][a] * P[1][b] * dP[2][e]);
        });
        Q[v] = v0;
        dQ[0][v] = vx * T(g.two_inv_dx[0]);
        dQ[1][v] = vy * T(g.two_inv_dx[1]);
        dQ[2][v] = vz * T(g.two_inv_dx[2]);
      }
      int bad = 0;
      volume_flux<T, NEED_F>(ph, Q, dQ, F, Ft, bad);
      if (bad) atomicOr(flag, 1);
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < 5; ++v) F[d][v] = Ft[d][v] = T(0);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T s = T(g.two_inv_dx[d]);
        if constexpr (NEED_F) {
          sA[(cl * 5 + v) * 2 + 0][3 * qi + d] = F[d][v] * s;
          sA[(cl * 5 + v) * 2 + 1][3 * qi + d] = Ft[d][v] * s;
        } else {
          sA[cl * 5 + v][3 * qi + d] = Ft[d][v] * s;
        }
      }
  }
  __syncthreads();

  // volume projection on MFMA: sR[row][n] = sum_kk sA[row][kk] B[kk][n]
  {
    const auto& bt = VolTabHolder<T, K, NQ>::t;
    const int lr = l & 15, lk = l >> 4;
    for (int tile = w; tile < NRT; tile += NW) {
      typename Acc<T>::type acc = {0, 0, 0, 0};
      const int row = tile * 16 + lr;
#pragma unroll 4
      for (int s = 0; s < KS; ++s) {
        const int kk = 4 * s + lk;
        const T a = (row < NR && kk < KK) ? sA[row][kk] : T(0);
        const T b = bt.B[kk][lr];
        acc = mfma16x16x4(a, b, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = tile * 16 + mfma_row<T>(lk, i);
        if (r < NR && lr < NM) sR[r][lr] = acc[i];
      }
    }
  }
  __syncthreads();

  // face records of the block's cells, staged through LDS with coalesced
  // loads (the MFMA operand space is free now): sRec[d][0][j] = upper face of
  // cell j, sRec[d][1][j] = its lower face (upper face of the cell below).
  static_assert(6 * CPB * RECN <= NRA * KK, "face records must fit in sA");
  T(*sRec)[2][CPB][RECN] = reinterpret_cast<T(*)[2][CPB][RECN]>(&sA[0][0]);
  __shared__ unsigned sdn[3][CPB];
  if (tid < 3 * CPB) {
    const int d = tid / CPB, j = tid % CPB;
    if (c0 + j < N) sdn[d][j] = nb32(unsigned(c0 + j), d, -1, g);
  }
  __syncthreads();
  for (int idx = tid; idx < 6 * CPB * RECN; idx += NTH) {
    const int r = idx % RECN, t = idx / RECN;
    const int j = t % CPB, ds = t / CPB;  // ds = d * 2 + side
    const int d = ds >> 1, side = ds & 1;
    const long long c = c0 + j;
    if (c < N) {
      const long long cf = side ? (long long)sdn[d][j] : c;
      sRec[d][side][j][r] = rec[((long long)d * N + cf) * RECN + r];
    }
  }
  __syncthreads();

  // surface terms, M^{-1} and the stage update; item = (var, mode, cell), cell fastest
  const auto& mt = ModeTabHolder<K>::t;
  for (int it = tid; it < CPB * 5 * NM; it += NTH) {
    const int j = it % CPB, vm = it / CPB;
    const int v = vm / NM, n = vm - v * NM;
    const long long c = c0 + j;
    if (c >= N) continue;
    double Lt = double(sR[(j * 5 + v) * NF + NF - 1][n]);
    double L = NEED_F ? double(sR[(j * 5 + v) * NF][n]) : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int m = mt.tm[n][d];
      const double sg = (mt.nd[n][d] & 1) ? -1.0 : 1.0;
      const T* ru = sRec[d][0][j];
      const T* rl = sRec[d][1][j];
      if constexpr (NEED_F) {
        const int of = v * NT + m;
        const int oft = (5 + v) * NT + m;
        L += g.inv_dx[d] * (sg * double(rl[of]) - double(ru[of]));
        Lt += g.inv_dx[d] * (sg * double(rl[oft]) - double(ru[oft]));
      } else {
        const int ot = v * NT + m;
        Lt += g.inv_dx[d] * (sg * double(rl[ot]) - double(ru[ot]));
      }
    }
    L *= mt.minv[n];
    Lt *= mt.minv[n];
    const long long gi = (long long)vm * N + c;
    const double dt = out.dt;
    if constexpr (MODE == 0) {
      const double qn = out.qn[gi];
      out.qstar[gi] = T(qn + 0.5 * dt * L + 0.125 * dt * dt * Lt);
      out.P[gi] = qn + dt * L + (dt * dt / 6.0) * Lt;
    } else if constexpr (MODE == 1) {
      const double qnew = out.P[gi] + (dt * dt / 3.0) * Lt;
      out.qnew[gi] = qnew;
      if (out.qshadow) out.qshadow[gi] = T(qnew);
    } else {
      out.L[gi] = L;
      out.Lt[gi] = Lt;
    }
  }
}

// FP64 -> T copy of the coefficients (stage-1 input of the bulk-precision path).
template <class T>
__global__ __launch_bounds__(256) void convert_kernel(const double* __restrict__ a, T* __restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) b[i] = T(a[i]);
}

// Point fluxes for diagnostics: x[i] = (qL 5, dqL 15, qR 5, dqR 15) in the
// global frame, face normal d; out F[i][5], Ft[i][5] (global frame).
template <class T>
__global__ __launch_bounds__(64) void point_face_kernel(const double* __restrict__ x, double* __restrict__ F,
                                                        double* __restrict__ Ft, long long n, int d, Phys ph,
                                                        int* flag) {
  const long long i = (long long)blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const double* xi = x + 40 * i;
  const int ax[3] = {d, (d + 1) % 3, (d + 2) % 3};
  T qs[2][5], dqs[2][3][5];
  for (int s = 0; s < 2; ++s) {
    const double* q = xi + 20 * s;
    const double* dq = q + 5;
    qs[s][0] = T(q[0]);
    qs[s][4] = T(q[4]);
    for (int a = 0; a < 3; ++a) qs[s][1 + a] = T(q[1 + ax[a]]);
    for (int a = 0; a < 3; ++a) {
      dqs[s][a][0] = T(dq[5 * ax[a] + 0]);
      dqs[s][a][4] = T(dq[5 * ax[a] + 4]);
      for (int b = 0; b < 3; ++b) dqs[s][a][1 + b] = T(dq[5 * ax[a] + 1 + ax[b]]);
    }
  }
  T Fl[5], Ftl[5];
  int bad = 0;
  face_flux_local<T, true>(ph, qs[0], dqs[0], qs[1], dqs[1], Fl, Ftl, bad);
  if (bad) atomicOr(flag, 1);
  F[5 * i + 0] = double(Fl[0]);
  F[5 * i + 4] = double(Fl[4]);
  Ft[5 * i + 0] = double(Ftl[0]);
  Ft[5 * i + 4] = double(Ftl[4]);
  for (int a = 0; a < 3; ++a) {
    F[5 * i + 1 + ax[a]] = double(Fl[1 + a]);
    Ft[5 * i + 1 + ax[a]] = double(Ftl[1 + a]);
  }
}

// x[i] = (q 5, dq 15); out F[i][3][5], Ft[i][3][5].
template <class T>
__global__ __launch_bounds__(64) void point_volume_kernel(const double* __restrict__ x, double* __restrict__ F,
                                                          double* __restrict__ Ft, long long n, Phys ph, int* flag) {
  const long long i = (long long)blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  T q[5], dq[3][5], Fo[3][5], Fto[3][5];
  for (int v = 0; v < 5; ++v) q[v] = T(x[20 * i + v]);
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) dq[e][v] = T(x[20 * i + 5 + 5 * e + v]);
  int bad = 0;
  volume_flux<T, true>(ph, q, dq, Fo, Fto, bad);
  if (bad) atomicOr(flag, 1);
  for (int e = 0; e < 3; ++e)
    for (int v = 0; v < 5; ++v) {
      F[15 * i + 5 * e + v] = double(Fo[e][v]);
      Ft[15 * i + 5 * e + v] = double(Fto[e][v]);
    }
}

}  // namespace dgk
