// kernels_adj.hpp -- reverse-mode (adjoint) kernels of one S2O4 stage.
//
// Forward stage:  L = M^{-1} R(Q), L_t = M^{-1} R_t(Q) with
//   R = sum_q w_q sum_d F_d(q) dB_n/dx_d  - sum_faces |Gamma| sum_q w_q F_b B_n.
// Given the cotangents Lbar, Ltbar (formed on the fly from the step-level
// cotangents, see AdjIn), the adjoint of one stage is two launches, the mirror
// of the forward pass:
//   adj_face_kernel   -- one lane per face side (the two sides of a face in
//                        neighbouring lanes): the cotangent of the face record,
//                        then per face point the forward traces and side
//                        contributions (summed across the lane pair), the
//                        reverse of the face flux, and the transposed trace
//                        evaluation, accumulated per lane into the cotangent of
//                        its cell's coefficients from this face (FP64 record).
//   adj_volume_kernel -- one lane per cell: per volume point the transposed
//                        projection, the reverse of the volume flux and the
//                        transposed evaluation; plus the face records of the
//                        cell's six faces, combined with the step-level
//                        cotangents (FP64).
// d/dmu is summed per block into a slot of its own (deterministic order).
#pragma once

#include "gks_point_adj.hpp"
#include "kernels_fwd.hpp"

namespace dgk {

// Number of per-block partial sums of dJ/dmu kept in the workspace: one slot
// per block of the two adjoint launches of a stage (3 nb face blocks of
// kAdjFaceThreads / 2 faces each, then the volume blocks of kCellThreads
// cells), reused by every stage and step.  Lanes per adjoint face block:
// 128 faces x 2 sides.
constexpr int kAdjFaceThreads = 256;
inline size_t adj_face_blocks(size_t ncell) { return (ncell + kAdjFaceThreads / 2 - 1) / (kAdjFaceThreads / 2); }
inline size_t adj_mu_slots(size_t ncell) {
  return 3 * adj_face_blocks(ncell) + (ncell + kCellThreads - 1) / kCellThreads;
}
// Slots summed by one block of the first pass of the dJ/dmu reduction.
constexpr int kMuChunk = 2048;

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

// Exchange with the neighbouring lane of the pair (lanes 2j <-> 2j+1): DPP
// quad permutation [1, 0, 3, 2]; every lane of the wavefront is active.
DGK_D float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
DGK_D double pair_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <class T>
DGK_D void pair_sum(T* x, int n) {
#pragma unroll
  for (int i = 0; i < n; ++i) x[i] += pair_swap(x[i]);
}

// Face cotangent records: frec[dir][side][tile][vm][64] (tile = face / 64),
// the cotangent of the coefficients of the lower (side 0) or upper (side 1)
// cell of a face, from that face.
DGK_D long long frec_index(int d, int side, long long face, int vm, int nvm, long long ntile) {
  return ((((long long)d * 2 + side) * ntile + (face >> 6)) * nvm + vm) * 64 + (face & 63);
}

// FP64 up to P2: the lane's face-restricted coefficients and record cotangent
// live in its LDS column (read where used) instead of registers.  The FP64
// kernel runs one wavefront per SIMD either way; the 150 VGPRs this frees cut
// its spills to scratch.  FP32 keeps them in registers (its working set fits).
template <class T, int K>
struct AdjFaceLds {
  static constexpr bool use = sizeof(T) == 8 && K <= 2;
  static constexpr int NT = ntan(K), NT1 = ntan(K - 1);
  T ct[5 * NT][kAdjFaceThreads];
  T cn[5 * NT1][kAdjFaceThreads];
  T ph[5 * NT][kAdjFaceThreads];
};
struct NoAdjFaceLds {};
template <class T, int K>
using AdjFaceSmem = std::conditional_t<AdjFaceLds<T, K>::use, AdjFaceLds<T, K>, NoAdjFaceLds>;

// --------------------------------------------------------------------------
// Adjoint face kernel.  Lane 2j + s of a block handles side s of face
// f0 + j (s = 0: the lower cell, half space u > 0; s = 1: the upper cell).
// --------------------------------------------------------------------------
template <class T, int K, int NQ, int STAGE, int D>
DGK_D void adj_face_lane(const T* __restrict__ q, const AdjIn<STAGE>& in, double* __restrict__ frec, const Geo& g,
                         const Phys& ph, long long f, int side, double& mub, AdjFaceSmem<T, K>& sm) {
  constexpr int NM = nmodes(K), NT = ntan(K), NT1 = ntan(K - 1), NQ2 = NQ * NQ;
  constexpr bool NEED_F = (STAGE == 1);
  constexpr int NF = NEED_F ? 2 : 1;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr Modes<K> md{};
  constexpr int vmap[5] = {0, 1 + D, 1 + T1, 1 + T2, 4};
  using MT = ModeTabHolder<K>;
  const long long N = g.ncell;
  const bool act = f < N;
  const long long fl = act ? f : N - 1;
  const long long cell = side ? (long long)nb32(unsigned(fl), D, +1, g) : fl;
  const T sg = side ? T(-1) : T(1);  // half-space orientation of this side

  // face-restricted coefficients of this side (see face_lane): pv_n = P_{e_D}(+-1),
  // dv_n = P'_{e_D}(+-1); and this cell's share of the record cotangent,
  // Phibar[f][v][m] = 1/dx_D sum_{n: t(n) = m} minv_n (sg_n Lbar_upper[n] - Lbar_lower[n])
  // with sg_n = (-1)^{e_D(n)}, completed by the pair sum.
  T ct[5][NT], cn[5][NT1], pb[NF][5][NT];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ct[v][t] = T(0);
#pragma unroll
      for (int k = 0; k < NF; ++k) pb[k][v][t] = T(0);
    }
#pragma unroll
    for (int t = 0; t < NT1; ++t) cn[v][t] = T(0);
  }
  // this side's cell: index along each axis (tangential ones shared by the pair)
  unsigned ci[3];
  cell_ijk(unsigned(cell), g, ci);
  const double ixd = 1.0 / g.w[D][ci[D]];
#pragma unroll
  for (int v = 0; v < 5; ++v)
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      constexpr int ed = md.e[n][D], t = face_tan_of_mode<K>(n, D);
      const long long gi = (long long)(v * NM + n) * N + cell;
      const T c = q[gi];
      // P_e(+1) = 1, P_e(-1) = (-1)^e; P'_e(+1) = e(e+1)/2, P'_e(-1) = (-1)^(e+1) e(e+1)/2
      const T pv = (ed % 2) ? sg : T(1);
      ct[v][t] += pv * c;
      if constexpr (ed > 0) cn[v][t] += ((ed % 2) ? T(1) : sg) * T(0.5 * ed * (ed + 1)) * c;
      double lb, ltb;
      in.coef(gi, lb, ltb);
      // lower cell: -minv Lbar; upper cell: +minv (-1)^{e_D} Lbar
      const double w = ixd * MT::t.minv[n] * (side ? ((ed % 2) ? -1.0 : 1.0) : -1.0);
      if constexpr (NEED_F) pb[0][v][t] += T(w * lb);
      pb[NF - 1][v][t] += T(w * ltb);
    });
  // Record cotangent summed over the pair.  Stage 1: lane 0 keeps the F part
  // and lane 1 the Ft part (each point's Fbar and Ftbar are then exchanged);
  // stage 2 has the Ft part only and both lanes keep it.
  T ph_[5][NT];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if constexpr (NEED_F) {
        const T send = side ? pb[0][v][t] : pb[1][v][t];
        const T keep = side ? pb[1][v][t] : pb[0][v][t];
        ph_[v][t] = keep + pair_swap(send);
      } else {
        ph_[v][t] = pb[0][v][t] + pair_swap(pb[0][v][t]);
      }
    }

  // the coefficients and record cotangent as used in the point loop
  constexpr bool LDS = AdjFaceLds<T, K>::use;
  const int tid = threadIdx.x;
  if constexpr (LDS) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        sm.ct[v * NT + t][tid] = ct[v][t];
        sm.ph[v * NT + t][tid] = ph_[v][t];
      }
#pragma unroll
      for (int t = 0; t < NT1; ++t) sm.cn[v * NT1 + t][tid] = cn[v][t];
    }
  }
  auto CT = [&](int v, int t) -> T {
    if constexpr (LDS) return sm.ct[v * NT + t][tid]; else return ct[v][t];
  };
  auto CN = [&](int v, int t) -> T {
    if constexpr (LDS) return sm.cn[v * NT1 + t][tid]; else return cn[v][t];
  };
  auto PH = [&](int v, int m) -> T {
    if constexpr (LDS) return sm.ph[v * NT + m][tid]; else return ph_[v][m];
  };

  // cotangents of ct, cn
  T ctb[5][NT], cnb[5][NT1];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int t = 0; t < NT; ++t) ctb[v][t] = T(0);
#pragma unroll
    for (int t = 0; t < NT1; ++t) cnb[v][t] = T(0);
  }
  const T sn = T(2.0 * ixd), s1 = T(2.0 / g.w[T1][ci[T1]]), s2 = T(2.0 / g.w[T2][ci[T2]]);
  using TB = TanBasisHolder<T, K, NQ>;
  using FT = FaceTabHolder<T, K, NQ>;
  constexpr TanModes<K> tmd{};
  double mb = 0.0;
#pragma unroll 1
  for (int qf = 0; qf < NQ2; ++qf) {
    // keeps the LDS columns in LDS: no load moves across this point
    __asm__ __volatile__("" ::: "memory");
    // this side's trace (local frame)
    T qs[5], dqs[3][5];
#pragma unroll
    for (int vl = 0; vl < 5; ++vl) {
      T v0 = T(0), vn = T(0), v1 = T(0), v2 = T(0);
      static_for<NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        const T c = CT(vmap[vl], t);
        v0 += c * TB::t.val[qf][t];
        if constexpr (tmd.e[t][0] > 0) v1 += c * TB::t.d1[qf][t];
        if constexpr (tmd.e[t][1] > 0) v2 += c * TB::t.d2[qf][t];
        if constexpr (t < NT1) vn += CN(vmap[vl], t) * TB::t.val[qf][t];
      });
      qs[vl] = v0;
      dqs[0][vl] = vn * sn;
      dqs[1][vl] = v1 * s1;
      dqs[2][vl] = v2 * s2;
    }
    // accumulators of both sides
    FaceAcc<T> acc;
    face_acc_zero(acc);
    int bad = 0;
    face_side(ph, qs, dqs, acc, bad, sg);
    pair_sum(&acc.Q0[0], 5);
    pair_sum(&acc.dQ0[0][0], 15);
    pair_sum(&acc.m4[0], 5);
    pair_sum(&acc.m5[0], 5);
    pair_sum(&acc.m6[0], 5);
    // Fbar_b at this point = sum_m phi_m(qf) Phibar[m], local frame
    T Fb[5], Ftb[5];
#pragma unroll
    for (int vl = 0; vl < 5; ++vl) {
      T sp = T(0);
#pragma unroll
      for (int m = 0; m < NT; ++m) sp += FT::t.phi[m][qf] * PH(vmap[vl], m);
      if constexpr (NEED_F) {
        const T other = pair_swap(sp);
        Fb[vl] = side ? other : sp;
        Ftb[vl] = side ? sp : other;
      } else {
        Fb[vl] = T(0);
        Ftb[vl] = sp;
      }
    }
    FaceAcc<T> accb;
    face_acc_zero(accb);
    double mbp = 0.0;
    face_finish_vjp<T, NEED_F>(ph, acc, Fb, Ftb, accb, mbp);
    mb += mbp;
    T qb[5], dqb[3][5];
    zero5(qb);
#pragma unroll
    for (int i = 0; i < 3; ++i) zero5(dqb[i]);
    face_side_vjp(ph, qs, dqs, accb, qb, dqb, sg);
    // transposed trace evaluation
#pragma unroll
    for (int vl = 0; vl < 5; ++vl) {
      const T bn = dqb[0][vl] * sn, b1 = dqb[1][vl] * s1, b2 = dqb[2][vl] * s2;
      static_for<NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        T a = qb[vl] * TB::t.val[qf][t];
        if constexpr (tmd.e[t][0] > 0) a += b1 * TB::t.d1[qf][t];
        if constexpr (tmd.e[t][1] > 0) a += b2 * TB::t.d2[qf][t];
        ctb[vmap[vl]][t] += a;
        if constexpr (t < NT1) cnb[vmap[vl]][t] += bn * TB::t.val[qf][t];
      });
    }
  }
  // the face-finish reverse is computed by both lanes of the pair: count it once
  if (side == 0 && act) mub += mb;
  if (!act) return;
  // back to the cell's coefficients; FP64 record
  const long long ntile = (N + 63) >> 6;
  double* out = frec + frec_index(D, side, f, 0, 5 * NM, ntile);
#pragma unroll
  for (int v = 0; v < 5; ++v)
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      constexpr int ed = md.e[n][D], t = face_tan_of_mode<K>(n, D);
      const T pv = (ed % 2) ? sg : T(1);
      T r = pv * ctb[v][t];
      if constexpr (ed > 0) r += ((ed % 2) ? T(1) : sg) * T(0.5 * ed * (ed + 1)) * cnb[v][t];
      out[(v * NM + n) * 64] = double(r);
    });
}

// Grid: 3 nb blocks of kAdjFaceThreads lanes, nb = ceil(N / (kAdjFaceThreads / 2)),
// ordered for the XCDs like face_kernel; block b owns mu slot b.
template <class T, int K, int NQ, int STAGE>
__global__ __launch_bounds__(kAdjFaceThreads) void adj_face_kernel(const T* __restrict__ q, AdjIn<STAGE> in,
                                                                   double* __restrict__ frec, Geo g, Phys ph,
                                                                   double* mu_part) {
  __shared__ double red[kAdjFaceThreads / 64];
  constexpr int FPB = kAdjFaceThreads / 2;
  const unsigned nb = gridDim.x / 3;
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
  const unsigned d = lb / nb;
  const long long f = (long long)(lb - d * nb) * FPB + (threadIdx.x >> 1);
  const int side = threadIdx.x & 1;
  double mub = 0.0;
  __shared__ AdjFaceSmem<T, K> sm;
  switch (d) {
    case 0: adj_face_lane<T, K, NQ, STAGE, 0>(q, in, frec, g, ph, f, side, mub, sm); break;
    case 1: adj_face_lane<T, K, NQ, STAGE, 1>(q, in, frec, g, ph, f, side, mub, sm); break;
    default: adj_face_lane<T, K, NQ, STAGE, 2>(q, in, frec, g, ph, f, side, mub, sm); break;
  }
  block_add_mu<kAdjFaceThreads>(mub, mu_part, lb, red);
}

// --------------------------------------------------------------------------
// Adjoint volume kernel: one lane per cell (blocking and block order of
// volume_kernel).  STAGE 2 writes qsbar = cotangent of Q*; STAGE 1 writes
// qbar <- qbar + qsbar + (cotangent of Q^n through L, L_t).
// --------------------------------------------------------------------------
template <class T, int K, int NQ, int STAGE>
__global__ __launch_bounds__(kCellThreads) void adj_volume_kernel(const T* __restrict__ q, AdjIn<STAGE> in,
                                                                 const double* __restrict__ frec, double* out,
                                                                 Geo g, Phys ph, double* mu_part, long long slot0) {
  constexpr int NM = nmodes(K), NQ3 = NQ * NQ * NQ;
  constexpr bool NEED_F = (STAGE == 1);
  constexpr int NF = NEED_F ? 2 : 1;
  constexpr Modes<K> md{};
  __shared__ double red[kCellThreads / 64];
  const auto& mt = ModeTabHolder<K>::t;
  const long long N = g.ncell;
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
  const long long c = (long long)lb * kCellThreads + threadIdx.x;
  const bool act = c < N;
  const long long cc = act ? c : N - 1;

  // Rbar = M^{-T} Lbar for the modes with a non-zero gradient (F and Ft)
  T rb[NF][5][NM];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int n = 0; n < NM; ++n) {
      double lbv, ltb;
      in.coef((long long)(v * NM + n) * N + cc, lbv, ltb);
      if constexpr (NEED_F) rb[0][v][n] = T(mt.minv[n] * lbv);
      rb[NF - 1][v][n] = T(mt.minv[n] * ltb);
    }
  T cf[5][NM], sb[5][NM];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int n = 0; n < NM; ++n) {
      cf[v][n] = q[(long long)(v * NM + n) * N + cc];
      sb[v][n] = T(0);
    }
  unsigned ci[3];
  cell_ijk(unsigned(cc), g, ci);
  const T sc[3] = {T(2.0 / g.w[0][ci[0]]), T(2.0 / g.w[1][ci[1]]), T(2.0 / g.w[2][ci[2]])};
  using PB = PointBasisHolder<T, K, NQ>;
  // The point's basis values (scalar loads) are read one point ahead in FP32
  // up to P2, as in the forward volume kernel, and issued at the top of the
  // previous point (scheduling barrier; here, unlike the forward kernel, that
  // measured faster: -16% of the kernel at 32^3, -2.5% at 128^3).
  constexpr bool PF = sizeof(T) == 4 && K <= 2;
  struct PtBasis {
    T phi[NM], dphi[3][NM], w;
  };
  auto load_basis = [&](int qi, PtBasis& b) {
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      b.phi[n] = PB::t.phi[qi][n];
#pragma unroll
      for (int d = 0; d < 3; ++d) b.dphi[d][n] = (md.e[n][d] > 0) ? PB::t.dphi[qi][d][n] : T(0);
    });
    b.w = PB::t.w[qi];
  };
  PtBasis nxt;
  if constexpr (PF) load_basis(0, nxt);
  double mub = 0.0;
#pragma unroll 1
  for (int qi = 0; qi < NQ3; ++qi) {
    PtBasis cur;
    if constexpr (PF) {
      cur = nxt;
      load_basis(qi + 1 < NQ3 ? qi + 1 : qi, nxt);
      __builtin_amdgcn_sched_barrier(0);  // issue the next point's loads here
    }
    auto PHI = [&](int n) -> T {
      if constexpr (PF) return cur.phi[n]; else return PB::t.phi[qi][n];
    };
    T ds[3][NM];
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        T dp;
        if constexpr (PF) dp = cur.dphi[d][n]; else dp = PB::t.dphi[qi][d][n];
        ds[d][n] = (md.e[n][d] > 0) ? dp * sc[d] : T(0);
      }
    });
    T Q[5], dQ[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T v0 = T(0), vx = T(0), vy = T(0), vz = T(0);
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        const T cn = cf[v][n];
        v0 += cn * PHI(n);
        if constexpr (md.e[n][0] > 0) vx += cn * ds[0][n];
        if constexpr (md.e[n][1] > 0) vy += cn * ds[1][n];
        if constexpr (md.e[n][2] > 0) vz += cn * ds[2][n];
      });
      Q[v] = v0;
      dQ[0][v] = vx;
      dQ[1][v] = vy;
      dQ[2][v] = vz;
    }
    // Fbar_d(q)[v] = w_q sum_n (2/dx_d) dB_n/dxi_d Rbar_n[v]
    T wq;
    if constexpr (PF) wq = cur.w; else wq = PB::t.w[qi];
    T Fb[3][5], Ftb[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        T sf = T(0), st = T(0);
        static_for<NM>([&](auto nc) {
          constexpr int n = decltype(nc)::value;
          if (md.e[n][d] > 0) {
            if constexpr (NEED_F) sf += ds[d][n] * rb[0][v][n];
            st += ds[d][n] * rb[NF - 1][v][n];
          }
        });
        Fb[d][v] = sf * wq;
        Ftb[d][v] = st * wq;
      }
    T qb[5], dqb[3][5];
    zero5(qb);
#pragma unroll
    for (int e = 0; e < 3; ++e) zero5(dqb[e]);
    volume_flux_vjp<T, NEED_F>(ph, Q, dQ, Fb, Ftb, qb, dqb, mub);
    // transposed evaluation
#pragma unroll
    for (int v = 0; v < 5; ++v)
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        T a = qb[v] * PHI(n);
        if constexpr (md.e[n][0] > 0) a += dqb[0][v] * ds[0][n];
        if constexpr (md.e[n][1] > 0) a += dqb[1][v] * ds[1][n];
        if constexpr (md.e[n][2] > 0) a += dqb[2][v] * ds[2][n];
        sb[v][n] += a;
      });
  }
  if (!act) mub = 0.0;
  block_add_mu<kCellThreads>(mub, mu_part, slot0 + lb, red);
  if (!act) return;
  // face records: upper face of the cell (side 0) and lower face (side 1 of the face below)
  const long long ntile = (N + 63) >> 6;
  const double* fu[3];
  const double* fd[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    fu[d] = frec + frec_index(d, 0, c, 0, 5 * NM, ntile);
    fd[d] = frec + frec_index(d, 1, (long long)nb32(unsigned(c), d, -1, g), 0, 5 * NM, ntile);
  }
  // Up to P2 all 5 NM sums are formed before the first store: a load placed
  // after a store that may alias it (the compiler cannot tell) waits for that
  // store, one memory latency per coefficient.  At P3 the lane has no
  // registers to spare for them, and each coefficient is stored as it is
  // summed.
  constexpr int VB = NM <= 10 ? 5 : 1;
  constexpr int NG = NM <= 10 ? NM : 1;
#pragma unroll
  for (int v0 = 0; v0 < 5; v0 += VB)
#pragma unroll
    for (int n0 = 0; n0 < NM; n0 += NG) {
      double s[VB][NG];
#pragma unroll
      for (int j = 0; j < VB; ++j)
#pragma unroll
        for (int i = 0; i < NG; ++i) {
          const int vm = (v0 + j) * NM + n0 + i;
          double a = double(sb[v0 + j][n0 + i]);
#pragma unroll
          for (int d = 0; d < 3; ++d) a += fu[d][vm * 64] + fd[d][vm * 64];
          if constexpr (STAGE != 2) {
            const long long gi = (long long)vm * N + c;
            a = in.qbar[gi] + in.qsbar[gi] + a;
          }
          s[j][i] = a;
        }
#pragma unroll
      for (int j = 0; j < VB; ++j)
#pragma unroll
        for (int i = 0; i < NG; ++i) out[(long long)((v0 + j) * NM + n0 + i) * N + c] = s[j][i];
    }
}

static __global__ __launch_bounds__(256) void zero_kernel(double* a, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) a[i] = 0.0;
}

// Fixed-order sum of the dJ/dmu slots, two passes: block b sums slots
// [b chunk, (b + 1) chunk) into out[b] (first pass: chunk = kMuChunk, one block
// per chunk; second pass: one block, chunk = the number of parts).  Both
// passes sum in the same order on every call.
static __global__ __launch_bounds__(256) void reduce_mu_kernel(const double* a, long long n, long long chunk,
                                                              double* out) {
  __shared__ double sh[256];
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += 256) s += a[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

}  // namespace dgk
