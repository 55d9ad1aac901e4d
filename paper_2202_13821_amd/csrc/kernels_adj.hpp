// kernels_adj.hpp -- reverse-mode (adjoint) kernels of one S2O4 stage.
//
// Forward stage:  L = M^{-1} R(Q), L_t = M^{-1} R_t(Q) with
//   R = sum_q w_q sum_d F_d(q) dB_n/dx_d  - sum_faces |Gamma| sum_q w_q F_b B_n.
// Given the cotangents Lbar, Ltbar (formed on the fly from the step-level
// cotangents, see AdjIn), the adjoint of one stage is two launches, the mirror
// of the forward pass:
//   adj_face_kernel   -- per face point: Fbar_b = sum_m phi_m (projection
//                        transposed), the forward traces are recomputed, the
//                        hand-written VJP of the face flux gives the trace
//                        cotangents, and their transposed evaluation is summed
//                        over the face points into one record per face and side
//                        (FP64): the cotangent of each cell's coefficients.
//   adj_volume_kernel -- per volume point: Fbar_d(q) = sum_n w_q dB_n/dx_d Rbar_n,
//                        VJP of the volume flux, transposed evaluation summed
//                        over the points of the cell, plus the face records of
//                        the cell's six faces, combined with the step-level
//                        cotangents (FP64).
// d/dmu is summed per block into a slot of its own (deterministic order).
#pragma once

#include "gks_point_adj.hpp"
#include "kernels_fwd.hpp"

namespace dgk {

// Number of per-block partial sums of dJ/dmu kept in the workspace.
inline size_t adj_mu_slots(size_t ncell) { return 3 * ncell + 64; }

// Step-level cotangents.  With qbar = cotangent of Q^{n+1} and qsbar = that
// of Q* (output of stage 2):
//   stage 2 (at Q*):  Lbar = 0,  Ltbar = dt^2/3 qbar
//   stage 1 (at Q^n): Lbar = dt qbar + dt/2 qsbar, Ltbar = dt^2/6 qbar + dt^2/8 qsbar
template <int STAGE>
struct AdjIn {
  const double* qbar;
  const double* qsbar;
  double dt;
  DGK_D void coef(long long gi, double& lb, double& ltb) const {
    const double a = qbar[gi];
    if constexpr (STAGE == 2) {
      lb = 0.0;
      ltb = dt * dt / 3.0 * a;
    } else {
      const double b = qsbar[gi];
      lb = dt * a + 0.5 * dt * b;
      ltb = dt * dt / 6.0 * a + dt * dt / 8.0 * b;
    }
  }
};

// Volume basis values and reference gradients at the volume points.
template <class T, int K, int NQ>
struct VolBasis {
  static constexpr int NM = nmodes(K), NQ3 = NQ * NQ * NQ;
  T B[NQ3][NM], G[NQ3][3][NM];
  constexpr VolBasis() : B{}, G{} {
    constexpr Modes<K> md{};
    for (int q = 0; q < NQ3; ++q) {
      const double x[3] = {Gauss<NQ>::x[q % NQ], Gauss<NQ>::x[(q / NQ) % NQ], Gauss<NQ>::x[q / (NQ * NQ)]};
      for (int n = 0; n < NM; ++n) {
        B[q][n] = T(leg(md.e[n][0], x[0]) * leg(md.e[n][1], x[1]) * leg(md.e[n][2], x[2]));
        for (int e = 0; e < 3; ++e) {
          double v = 1.0;
          for (int f = 0; f < 3; ++f) v *= (f == e) ? dleg(md.e[n][f], x[f]) : leg(md.e[n][f], x[f]);
          G[q][e][n] = T(v);
        }
      }
    }
  }
};
template <class T, int K, int NQ>
struct VolBasisHolder {
  static constexpr VolBasis<T, K, NQ> t{};
};

// Sum of a double over the block; thread 0 adds it to slot[slot].
template <int NTH>
DGK_D void block_add_mu(double v, double* mu_part, long long slot, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NTH / 64; ++i) s += red[i];
    mu_part[slot] += s;
  }
}

// --------------------------------------------------------------------------
// Adjoint face kernel (same blocking as face_kernel).  LDS: coefficients of
// both cells (dead once the traces are formed, then reused for the trace
// cotangents) and Phibar, the cotangent of the face record.
// --------------------------------------------------------------------------
template <class T, int K, int NQ>
struct AdjFaceCfg {
  using C = FaceCfg<K, NQ>;
  static constexpr int NT = ntan(K);
  static constexpr size_t SQ = sizeof(T) * 2 * C::FPB * C::CS;
  static constexpr size_t ST = sizeof(T) * C::FPB * C::NQ2 * 20;
  static constexpr size_t SA = (SQ > ST ? SQ : ST);
  static constexpr size_t SP = sizeof(T) * C::FPB * 10 * NT;
  static constexpr size_t BYTES = (SA + SP + 15) / 16 * 16;
};

template <class T, int K, int NQ, int STAGE, int D>
DGK_D void adj_face_block(const T* __restrict__ q, const AdjIn<STAGE>& in, double* __restrict__ frec, const Geo& g,
                          const Phys& ph, double* mu_part, long long f0, unsigned char* smem, double* red) {
  using C = FaceCfg<K, NQ>;
  using A = AdjFaceCfg<T, K, NQ>;
  constexpr int NM = C::NM, NT = C::NT, NQ2 = C::NQ2, FPW = C::FPW, FPB = C::FPB, CS = C::CS;
  constexpr bool NEED_F = (STAGE == 1);
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  auto sq = reinterpret_cast<T(*)[FPB][CS]>(smem);
  auto sT = reinterpret_cast<T(*)[NQ2][20]>(smem);
  auto sP = reinterpret_cast<T(*)[10 * NT]>(smem + A::SA);
  const int tid = threadIdx.x;
  const long long N = g.ncell;
  const auto& mt = ModeTabHolder<K>::t;

  // upper neighbours, then the coefficients of the lower (side 0) and upper (side 1) cells
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
  // Phibar[comp][m] = 1/dx sum_{n: tm(n) = m} (sg_n Rbar_R[n] - Rbar_L[n]), Rbar = M^{-1} Lbar,
  // comp = F|Ft * 5 + var (the face record layout of the forward pass)
  for (int idx = tid; idx < FPB * 10 * NT; idx += 256) {
    const int j = idx % FPB, r = idx / FPB;
    const int comp = r / NT, m = r - comp * NT;
    const int v = comp % 5;
    const bool isF = comp < 5;
    const long long f = f0 + j;
    double acc = 0.0;
    if (f < N && (!isF || NEED_F)) {
      const long long cr = (long long)snb[j];
#pragma unroll
      for (int n = 0; n < NM; ++n) {
        if (mt.tm[n][D] != m) continue;
        const double sg = (mt.nd[n][D] & 1) ? -1.0 : 1.0;
        double lbL, ltbL, lbR, ltbR;
        in.coef((long long)(v * NM + n) * N + f, lbL, ltbL);
        in.coef((long long)(v * NM + n) * N + cr, lbR, ltbR);
        acc += mt.minv[n] * (isF ? (sg * lbR - lbL) : (sg * ltbR - ltbL));
      }
      acc *= g.inv_dx[D];
    }
    sP[j][r] = T(acc);
  }
  __syncthreads();

  const int w = tid >> 6, l = tid & 63;
  const int fl = w * FPW + l / NQ2, qp = l % NQ2;
  const bool active = (l < FPW * NQ2) && (f0 + fl < N);
  double mub = 0.0;
  constexpr int vmap[5] = {0, 1 + D, 1 + T1, 1 + T2, 4};
  T qbL[5], dqbL[3][5], qbR[5], dqbR[3][5];
  T qL[5], dqL[3][5], qR[5], dqR[3][5];
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
    trace(std::integral_constant<int, 0>{}, qL, dqL);
    trace(std::integral_constant<int, 1>{}, qR, dqR);
  }
  __syncthreads();  // sq is dead from here on (its space holds sT below)
  if (active) {
    // Fbar_b at this point = sum_m phi_m(qf) Phibar[m], in the local frame
    const auto& ft = FaceTabHolder<T, K, NQ>::t;
    T Fbl[5], Ftbl[5];
#pragma unroll
    for (int vl = 0; vl < 5; ++vl) {
      T sf = T(0), st = T(0);
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const T p_ = ft.phi[m][qp];
        if constexpr (NEED_F) sf += p_ * sP[fl][vmap[vl] * NT + m];
        st += p_ * sP[fl][(5 + vmap[vl]) * NT + m];
      }
      Fbl[vl] = sf;
      Ftbl[vl] = st;
    }
    FaceAcc<T> acc, accb;
    face_acc_zero(acc);
    face_acc_zero(accb);
    int bad = 0;
    face_side<+1>(ph, qL, dqL, acc, bad);
    face_side<-1>(ph, qR, dqR, acc, bad);
    face_finish_vjp<T, NEED_F>(ph, acc, Fbl, Ftbl, accb, mub);
    zero5(qbL);
    zero5(qbR);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      zero5(dqbL[i]);
      zero5(dqbR[i]);
    }
    face_side_vjp<+1>(ph, qL, dqL, accb, qbL, dqbL);
    face_side_vjp<-1>(ph, qR, dqR, accb, qbR, dqbR);
  }
  // transposed trace evaluation, side by side, summed over the face points
  const auto& tt = TraceTabHolder<T, K, NQ, D>::t;
  const T sdir[3] = {T(g.two_inv_dx[D]), T(g.two_inv_dx[T1]), T(g.two_inv_dx[T2])};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (side) __syncthreads();
    if (active) {
#pragma unroll
      for (int vl = 0; vl < 5; ++vl) {
        sT[fl][qp][vmap[vl]] = side ? qbR[vl] : qbL[vl];
#pragma unroll
        for (int i = 0; i < 3; ++i) sT[fl][qp][5 + 5 * i + vmap[vl]] = (side ? dqbR[i][vl] : dqbL[i][vl]) * sdir[i];
      }
    }
    __syncthreads();
    for (int o = l; o < FPW * 5 * NM; o += 64) {
      const int fo = w * FPW + o / (5 * NM);
      const int r = o % (5 * NM);
      const int v = r / NM, n = r - v * NM;
      const long long f = f0 + fo;
      if (f < N) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NQ2; ++k) {
          const T* c = sT[fo][k];
          s += double(c[v] * tt.B[side][n][k] + c[5 + v] * tt.Dn[side][n][k] + c[10 + v] * tt.D1[side][n][k] +
                      c[15 + v] * tt.D2[side][n][k]);
        }
        frec[(((long long)D * N + f) * 2 + side) * 5 * NM + r] = s;
      }
    }
  }
  block_add_mu<256>(mub, mu_part, (long long)blockIdx.y * gridDim.x + blockIdx.x, red);
}

template <class T, int K, int NQ, int STAGE>
__global__ __launch_bounds__(256) void adj_face_kernel(const T* __restrict__ q, AdjIn<STAGE> in,
                                                       double* __restrict__ frec, Geo g, Phys ph, double* mu_part) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[AdjFaceCfg<T, K, NQ>::BYTES];
  __shared__ double red[4];
  const long long f0 = (long long)blockIdx.x * FaceCfg<K, NQ>::FPB;
  switch (blockIdx.y) {
    case 0: adj_face_block<T, K, NQ, STAGE, 0>(q, in, frec, g, ph, mu_part, f0, smem, red); break;
    case 1: adj_face_block<T, K, NQ, STAGE, 1>(q, in, frec, g, ph, mu_part, f0, smem, red); break;
    default: adj_face_block<T, K, NQ, STAGE, 2>(q, in, frec, g, ph, mu_part, f0, smem, red); break;
  }
}

// --------------------------------------------------------------------------
// Adjoint volume kernel (same blocking as volume_kernel).
// STAGE 2 writes qsbar = cotangent of Q*; STAGE 1 writes
// qbar <- qbar + qsbar + (cotangent of Q^n through L, L_t).
// --------------------------------------------------------------------------
template <class T, int K, int NQ, int STAGE>
__global__ __launch_bounds__(64 * NQ) void adj_volume_kernel(const T* __restrict__ q, AdjIn<STAGE> in,
                                                            const double* __restrict__ frec, double* out,
                                                            Geo g, Phys ph, double* mu_part, long long slot0) {
  using C = VolCfg<K, NQ>;
  constexpr int NM = C::NM, NQ2 = C::NQ2, NQ3 = C::NQ3, CPB = C::CPB, NTH = C::NTH;
  constexpr bool NEED_F = (STAGE == 1);
  __shared__ T sq[CPB][C::CS];
  __shared__ T sr[CPB][10 * NM];
  __shared__ T sT[CPB][NQ3][20];
  __shared__ double red[NTH / 64];
  const int tid = threadIdx.x;
  const long long N = g.ncell;
  const long long c0 = (long long)blockIdx.x * CPB;
  const auto& mt = ModeTabHolder<K>::t;

  for (int idx = tid; idx < CPB * 5 * NM; idx += NTH) {
    const int vm = idx / CPB, j = idx - vm * CPB;
    if (c0 + j < N) {
      const long long gi = (long long)vm * N + c0 + j;
      sq[j][vm] = q[gi];
      double lb, ltb;
      in.coef(gi, lb, ltb);
      const double mi = mt.minv[vm % NM];
      sr[j][vm] = T(mi * lb);
      sr[j][5 * NM + vm] = T(mi * ltb);
    }
  }
  __syncthreads();

  const int w = tid >> 6, l = tid & 63;
  const int cl = l / NQ2, qxy = l % NQ2;
  double mub = 0.0;
  if (cl < CPB) {
    const int qx = qxy % NQ, qy = qxy / NQ, qz = w;
    const int qi = (qz * NQ + qy) * NQ + qx;
    T qb[5], dqb[3][5];
    zero5(qb);
#pragma unroll
    for (int e = 0; e < 3; ++e) zero5(dqb[e]);
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
      T Q[5], dQ[3][5], Fb[3][5], Ftb[3][5];
      const auto& vt = VolTabHolder<T, K, NQ>::t;
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
        // Fbar_d(q)[v] = sum_n w_q (2/dx_d) dB_n/dxi_d (q) Rbar_n[v]
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          T sf = T(0), st = T(0);
#pragma unroll
          for (int n = 0; n < NM; ++n) {
            const T wb = vt.B[3 * qi + d][n];
            if constexpr (NEED_F) sf += wb * sr[cl][v * NM + n];
            st += wb * sr[cl][5 * NM + v * NM + n];
          }
          Fb[d][v] = sf * T(g.two_inv_dx[d]);
          Ftb[d][v] = st * T(g.two_inv_dx[d]);
        }
      }
      volume_flux_vjp<T, NEED_F>(ph, Q, dQ, Fb, Ftb, qb, dqb, mub);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      sT[cl][qi][v] = qb[v];
#pragma unroll
      for (int e = 0; e < 3; ++e) sT[cl][qi][5 + 5 * e + v] = dqb[e][v] * T(g.two_inv_dx[e]);
    }
  }
  __syncthreads();
  // transposed evaluation, surface records, step-level combination
  __shared__ unsigned sdn[3][CPB];
  if (tid < 3 * CPB) {
    const int d = tid / CPB, j = tid % CPB;
    if (c0 + j < N) sdn[d][j] = nb32(unsigned(c0 + j), d, -1, g);
  }
  __syncthreads();
  const auto& vb = VolBasisHolder<T, K, NQ>::t;
  for (int it = tid; it < CPB * 5 * NM; it += NTH) {
    const int j = it % CPB, vm = it / CPB;
    const int v = vm / NM, n = vm - v * NM;
    const long long c = c0 + j;
    if (c >= N) continue;
    double s = 0.0;
#pragma unroll 9
    for (int k = 0; k < NQ3; ++k) {
      const T* t = sT[j][k];
      s += double(t[v] * vb.B[k][n] + t[5 + v] * vb.G[k][0][n] + t[10 + v] * vb.G[k][1][n] + t[15 + v] * vb.G[k][2][n]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long long cm = (long long)sdn[d][j];
      s += frec[(((long long)d * N + c) * 2 + 0) * 5 * NM + vm];
      s += frec[(((long long)d * N + cm) * 2 + 1) * 5 * NM + vm];
    }
    const long long gi = (long long)vm * N + c;
    if constexpr (STAGE == 2) {
      out[gi] = s;
    } else {
      out[gi] = in.qbar[gi] + in.qsbar[gi] + s;
    }
  }
  block_add_mu<NTH>(mub, mu_part, slot0 + blockIdx.x, red);
}

static __global__ __launch_bounds__(256) void zero_kernel(double* a, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) a[i] = 0.0;
}

// Fixed-order sum of the dJ/dmu slots into out[0] (one block).
static __global__ __launch_bounds__(256) void reduce_mu_kernel(const double* a, long long n, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) s += a[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace dgk
