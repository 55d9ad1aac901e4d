// kernels_fwd.hpp -- forward kernels of one S2O4 stage (HIP, gfx950).
//
// Data layout in HBM (structure of arrays, x fastest):
//   coefficients  q[var][mode][z][y][x]             (FP64 at the C-ABI; T copy inside)
//   face records  rec[dir][tile][F|Ft][var][tmode][64]  one record per upper
//                 face of each cell (tile = cell / 64, then cell % 64): the
//                 face flux projected on the tangential Legendre modes of the
//                 face, Phi_m = sum_q w_q F(x_q) phi_m(x_q).  A wavefront of the
//                 volume kernel (64 cells) reads each record component as one
//                 contiguous row, the rows of a tile at fixed offsets.
//
// One stage is two launches:
//   face_kernel   -- one lane per face, every face of the grid once: traces
//                    of both cells at the face Gauss points, the gas-kinetic
//                    face flux per point, and its projection on the
//                    tangential modes of the face.
//   volume_kernel -- one lane per cell: point values and gradients at the
//                    volume Gauss points, the volume flux per point, the
//                    projection sum_q w_q F_d dB_n/dx_d in registers, the
//                    surface terms from the six face records, M^{-1}, and the
//                    fused stage update with FP64 accumulation of the modal
//                    coefficients.
#pragma once

#include "gks_point.hpp"

namespace dgk {

#define DGK_D __device__ __forceinline__

struct Geo {
  int nx, ny, nz;
  int uniform;  // 1: every cell has the widths 2 / two_inv_h[d]
  long long ncell;
  // Separable mesh: w[d][i] is the width of the cells with index i along axis
  // d (device, FP64).  2 / w maps reference to physical derivatives and
  // 1 / w = |Gamma_d| / |K| scales a cell's d-face terms.
  const double* w[3];
  double two_inv_h[3];  // 2 / width on a uniform mesh (kernel argument, wave-uniform)
};

// Index of cell c along each axis.
DGK_D void cell_ijk(unsigned c, const Geo& g, unsigned ijk[3]) {
  const unsigned nx = unsigned(g.nx), ny = unsigned(g.ny);
  ijk[0] = c % nx;
  ijk[1] = (c / nx) % ny;
  ijk[2] = c / (nx * ny);
}

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

// Element index of component r of the record of cell `cell` along axis d
// (rec_len components per record, ntile = ceil(N / 64) tiles per axis).
DGK_D long long rec_index(int d, long long cell, int r, int rec_len, long long ntile) {
  return (((long long)d * ntile + (cell >> 6)) * rec_len + r) * 64 + (cell & 63);
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

// Unweighted tangential basis and its reference derivatives at the face
// points: val[qf][m] = P_ma(x_a) P_mb(x_b), d1 = P'_ma P_mb, d2 = P_ma P'_mb.
template <class T, int K, int NQ>
struct TanBasis {
  static constexpr int NT = ntan(K);
  T val[NQ * NQ][NT], d1[NQ * NQ][NT], d2[NQ * NQ][NT];
  constexpr TanBasis() : val{}, d1{}, d2{} {
    constexpr TanModes<K> tm{};
    for (int b = 0; b < NQ; ++b)
      for (int a = 0; a < NQ; ++a)
        for (int m = 0; m < NT; ++m) {
          const double xa = Gauss<NQ>::x[a], xb = Gauss<NQ>::x[b];
          val[b * NQ + a][m] = T(leg(tm.e[m][0], xa) * leg(tm.e[m][1], xb));
          d1[b * NQ + a][m] = T(dleg(tm.e[m][0], xa) * leg(tm.e[m][1], xb));
          d2[b * NQ + a][m] = T(leg(tm.e[m][0], xa) * dleg(tm.e[m][1], xb));
        }
  }
};
template <class T, int K, int NQ>
struct TanBasisHolder {
  static constexpr TanBasis<T, K, NQ> t{};
};

// Cell-per-lane kernels: 4 wavefronts per block.
constexpr int kCellThreads = 256;

// Block order for the 8 XCDs: the hardware hands consecutive block indices to
// the XCDs in turn; this bijection of [0, nb) gives XCD x (= b mod 8) one
// contiguous range of logical blocks, so that neighbouring cells (and the face
// records they share) stay in one XCD's L2.
DGK_D unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// --------------------------------------------------------------------------
// Face kernel.  One lane per face: the face between cell f (lower side) and
// its upper neighbour along D, 64 faces (one tile of lower cells) per
// wavefront.  The lane reduces the coefficients of both cells to their
// face-restricted coefficients (its own LDS column, except the lower cell's
// normal-derivative coefficients, kept in registers) and visits the face
// points in a loop that is uniform across the wavefront (trace basis and
// projection weights by scalar loads); per point the traces of both sides,
// the gas-kinetic face flux, and its projection on the tangential modes
// accumulated in registers.  Each record component is then stored as one row
// of the tile.
// --------------------------------------------------------------------------
// LDS of one face block (each lane uses only its own column, so no barrier
// is needed): the upper cell's face-restricted coefficients, the lower cell's
// trace coefficients, and the cell-width scales of the face.  At 2 x 256
// lanes per CU this is 79 floats per lane (of 80).
template <class T, int K, bool NEED_F, int NTH>
struct FaceLds {
  static constexpr int NT = ntan(K), NT1 = ntan(K - 1);
  static constexpr int NC = 5 * (NT + NT1);
  T c1[NC][NTH];
  T x[5 * NT][NTH];  // the lower cell's trace coefficients
  T st[4][NTH];  // 2 / width along the normal (lower, upper cell) and the two tangents
};

// Lanes per face block: 256, or 128 where the LDS columns of 256 lanes would
// exceed the 160 KB of a CU (FP64 at P3).
template <class T, int K>
constexpr int face_threads() {
  return sizeof(FaceLds<T, K, true, kCellThreads>) <= 160 * 1024 ? kCellThreads : kCellThreads / 2;
}

// Whether the face lane scales the normal-derivative trace coefficients by
// 2 / width once at set-up (fewer multiplications per point) instead of the
// traced derivative at every point.  Off for FP64 P3, whose face lanes already
// spill and where the longer-lived scaled values cost more than they save.
template <class T, int K>
constexpr bool kPrescaleCn = !(sizeof(T) == 8 && K == 3);

template <class T, int K, int NQ, bool NEED_F, int D, bool UNI>
DGK_D void face_lane(const T* __restrict__ q, T* __restrict__ rec, const Geo& g, const Phys& ph, int* flag,
                     long long f, FaceLds<T, K, NEED_F, face_threads<T, K>()>& sm, const double* ec) {
  constexpr int NM = nmodes(K), NT = ntan(K), NT1 = ntan(K - 1), NQ2 = NQ * NQ;
  constexpr int NF = NEED_F ? 2 : 1;
  constexpr int RECN = 5 * NF * NT;
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  constexpr Modes<K> md{};
  // local frame: velocity (normal, t1, t2) = global (D, T1, T2)
  constexpr int vmap[5] = {0, 1 + D, 1 + T1, 1 + T2, 4};
  using FT = FaceTabHolder<T, K, NQ>;
  const int tid = threadIdx.x;
  const long long N = g.ncell;
  const bool act = f < N;
  const long long fl = act ? f : N - 1;  // lanes past the end recompute the last face, store nothing
  const long long fu = (long long)nb32(unsigned(fl), D, +1, g);
  // 2 / width along the normal for each side and along the tangents (shared
  // by the sides): per lane through LDS on a non-uniform mesh (read where
  // used, to spare registers), wave-uniform kernel arguments on a uniform one
  if constexpr (!UNI) {
    unsigned ci[3];
    cell_ijk(unsigned(fl), g, ci);
    const unsigned nD = unsigned(D == 0 ? g.nx : (D == 1 ? g.ny : g.nz));
    sm.st[0][tid] = T(2.0 / g.w[D][ci[D]]);
    sm.st[1][tid] = T(2.0 / g.w[D][ci[D] + 1 == nD ? 0 : ci[D] + 1]);
    sm.st[2][tid] = T(2.0 / g.w[T1][ci[T1]]);
    sm.st[3][tid] = T(2.0 / g.w[T2][ci[T2]]);
  }

  // The traces on this face depend on a cell's modes only through their
  // values at xi_D = +-1: per side s and variable, the tangential-mode
  // coefficients of the trace, ct[v][t] = sum_{e_D} c[v][n(e_D, t)] P_{e_D}(+-1),
  // and of its normal derivative, cn[v][t] = (2 / h) sum_{e_D} c[v][n] P'_{e_D}(+-1)
  // with h the side's width along D (tangential degree <= K - 1), with
  // P_e(+1) = 1, P_e(-1) = (-1)^e,
  // P'_e(+1) = e(e+1)/2, P'_e(-1) = (-1)^(e+1) e(e+1)/2.
  // Side 1 (upper cell) goes to LDS; side 0 (lower cell) keeps its normal-
  // derivative coefficients cn in registers and its trace coefficients ct in
  // LDS (read-only in the point loop).
  T cn0[5][NT1];
  static_for<2>([&](auto sc) {
    constexpr int side = decltype(sc)::value;
    const long long cell = side ? fu : fl;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T ct[NT], cn[NT1];
#pragma unroll
      for (int t = 0; t < NT; ++t) ct[t] = T(0);
#pragma unroll
      for (int t = 0; t < NT1; ++t) cn[t] = T(0);
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        constexpr int ed = md.e[n][D], t = face_tan_of_mode<K>(n, D);
        constexpr double pv = (side == 0 || ed % 2 == 0) ? 1.0 : -1.0;
        constexpr double dv = (side == 0 || ed % 2 == 1 ? 1.0 : -1.0) * 0.5 * ed * (ed + 1);
        if constexpr (ed > 0) {
          const T c = q[(long long)(v * NM + n) * N + cell];
          ct[t] += T(pv) * c;
          cn[t] += T(dv) * c;
        }
      });
      // the modes constant along the normal last: among them the cell mean,
      // the largest term of the trace, is then added with a single rounding
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        constexpr int ed = md.e[n][D], t = face_tan_of_mode<K>(n, D);
        if constexpr (ed == 0) ct[t] += q[(long long)(v * NM + n) * N + cell];
      });
      // the normal derivative in physical units: 2 / (the side's width) once here
      // rather than at every point
      if constexpr (kPrescaleCn<T, K>) {
        T sn;
        if constexpr (UNI)
          sn = T(g.two_inv_h[D]);
        else
          sn = sm.st[side][tid];
#pragma unroll
        for (int t = 0; t < NT1; ++t) cn[t] *= sn;
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (side == 1)
          sm.c1[v * NT + t][tid] = ct[t];
        else
          sm.x[v * NT + t][tid] = ct[t];
      }
#pragma unroll
      for (int t = 0; t < NT1; ++t) {
        if constexpr (side == 0)
          cn0[v][t] = cn[t];
        else
          sm.c1[5 * NT + v * NT1 + t][tid] = cn[t];
      }
    }
  });
  // record accumulators (registers): Ft, and F in stage 1
  T acc[5][NT], accF[NEED_F ? 5 : 1][NT];
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int m = 0; m < NT; ++m) {
      acc[r][m] = T(0);
      if constexpr (NEED_F) accF[r][m] = T(0);
    }
  using TB = TanBasisHolder<T, K, NQ>;
  constexpr TanModes<K> tmd{};
  int bad = 0;
#pragma unroll 1
  for (int qf = 0; qf < NQ2; ++qf) {
    // keeps the LDS data in LDS: no load or store moves across this point
    __asm__ __volatile__("" ::: "memory");
    FaceAcc<T> fa;
    face_acc_zero(fa);
    static_for<2>([&](auto sc) {
      constexpr int side = decltype(sc)::value;
      // trace of this side at the point: Q and its derivatives along (n, t1, t2)
      T qs[5], dqs[3][5];
#pragma unroll
      for (int vl = 0; vl < 5; ++vl) {
        T v0 = T(0), vn = T(0), v1 = T(0), v2 = T(0), c00 = T(0);
        static_for<NT>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          T c;
          if constexpr (side == 1)
            c = sm.c1[vmap[vl] * NT + t][tid];
          else
            c = sm.x[vmap[vl] * NT + t][tid];
          // tangential mode 0 (value 1 at every point) is added last
          if constexpr (t > 0)
            v0 += c * TB::t.val[qf][t];
          else
            c00 = c;
          if constexpr (tmd.e[t][0] > 0) v1 += c * TB::t.d1[qf][t];
          if constexpr (tmd.e[t][1] > 0) v2 += c * TB::t.d2[qf][t];
          if constexpr (t < NT1) {
            T cnv;
            if constexpr (side == 0)
              cnv = cn0[vmap[vl]][t];
            else
              cnv = sm.c1[5 * NT + vmap[vl] * NT1 + t][tid];
            vn += cnv * TB::t.val[qf][t];
          }
        });
        qs[vl] = v0 + c00;
        if constexpr (UNI) {
          dqs[0][vl] = kPrescaleCn<T, K> ? vn : vn * T(g.two_inv_h[D]);
          dqs[1][vl] = v1 * T(g.two_inv_h[T1]);
          dqs[2][vl] = v2 * T(g.two_inv_h[T2]);
        } else {
          dqs[0][vl] = kPrescaleCn<T, K> ? vn : vn * sm.st[side][tid];
          dqs[1][vl] = v1 * sm.st[2][tid];
          dqs[2][vl] = v2 * sm.st[3][tid];
        }
      }
      face_side(ph, qs, dqs, fa, bad, T(side == 0 ? 1 : -1));
    });
    T F[5], Ft[5];
    face_finish<T, NEED_F>(ph, fa, F, Ft, bad, ec);
    // record component order: (F|Ft, global variable, tangential mode)
    static_for<NT>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      const T p = FT::t.phi[m][qf];
#pragma unroll
      for (int vl = 0; vl < 5; ++vl) {
        if constexpr (NEED_F) accF[vmap[vl]][m] += p * F[vl];
        acc[vmap[vl]][m] += p * Ft[vl];
      }
    });
  }
  __asm__ __volatile__("" ::: "memory");
  if (!act) return;
  if (bad) atomicOr(flag, 1);
  T* out = rec + rec_index(D, f, 0, RECN, (N + 63) >> 6);
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int m = 0; m < NT; ++m) {
      if constexpr (NEED_F) out[(r * NT + m) * 64] = accF[r][m];
      out[(((NF - 1) * 5 + r) * NT + m) * 64] = acc[r][m];
    }
}

// Minimum waves per SIMD requested for the face kernel (register budget):
// two for FP32 up to P2 (the LDS columns then take 79 floats per lane), one
// otherwise.
template <class T, int K>
struct FaceWaves {
  static constexpr int value = (sizeof(T) == 4 && K <= 2) ? 2 : 1;
};

// Grid: 3 nb blocks of face_threads<T, K>() lanes, nb = ceil(N / lanes);
// the logical block (after the XCD reordering) picks the normal axis and the
// range of faces.
template <class T, int K, int NQ, bool NEED_F, bool UNI>
__global__ __launch_bounds__((face_threads<T, K>()), (FaceWaves<T, K>::value)) void face_kernel(
    const T* __restrict__ q, T* __restrict__ rec, Geo g, Phys ph, int* flag) {
  constexpr int FT = face_threads<T, K>();
  const unsigned nb = gridDim.x / 3;
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
  const unsigned d = lb / nb;
  const long long f = (long long)(lb - d * nb) * FT + threadIdx.x;
  __shared__ FaceLds<T, K, NEED_F, FT> sm;
  // the constants of the FP64 exp of the time coefficients: read from LDS at
  // every point rather than kept in (and spilled from) registers
  __shared__ double ec[15];
  if (threadIdx.x < 15) ec[threadIdx.x] = ExpTabHolder<>::t.c[threadIdx.x];
  __syncthreads();
  switch (d) {
    case 0: face_lane<T, K, NQ, NEED_F, 0, UNI>(q, rec, g, ph, flag, f, sm, ec); break;
    case 1: face_lane<T, K, NQ, NEED_F, 1, UNI>(q, rec, g, ph, flag, f, sm, ec); break;
    default: face_lane<T, K, NQ, NEED_F, 2, UNI>(q, rec, g, ph, flag, f, sm, ec); break;
  }
}

// --------------------------------------------------------------------------
// Volume kernel.  One lane per cell, 256 cells per block; every lane of a
// wavefront visits the same volume point at the same time, so the basis
// values of the point are wavefront-uniform (scalar loads).  First the six
// face records of the cell (record tiles: one coalesced row per component),
// then per point the trace Q, dQ from the cell's coefficients, the volume
// flux, and its projection sum_q w_q F_d dB_n/dx_d accumulated in registers
// over the non-zero entries of dB_n/dxi_d; then M^{-1} and the stage update
// in FP64.
// MODE 0: stage 1 (F and Ft)   -> Q* (T) and P = Q^n + dt L + dt^2/6 L_t (FP64)
// MODE 1: stage 2 (Ft only)    -> Q^{n+1} = P + dt^2/3 L_t(Q*) (FP64, + T copy)
// MODE 2: operator only        -> L, L_t (FP64)
// PART (MODE 0 and 2): 0 both fluxes in one pass; 2 the Ft pass alone, writing
// L_t to out.Lt; 1 the F pass alone, then (MODE 0) the update with the L_t of
// the Ft pass read back from out.Lt.  Two passes halve the accumulators a
// lane holds, for the configurations whose single pass would spill them.
// --------------------------------------------------------------------------
template <class T>
struct VolOut {
  const double* qn;  // MODE 0: Q^n (FP64)
  double* P;         // MODE 0 out / MODE 1 in
  T* qstar;          // MODE 0 out
  double* qnew;      // MODE 1 out (may alias qn of the next step)
  T* qshadow;        // MODE 1 out: T copy of Q^{n+1} (nullptr when T = double)
  double* L;         // MODE 2
  double* Lt;        // MODE 2; MODE 0 with PART 2 (out) and PART 1 (in)
  double dt;
};

// Whether the stage-1 and operator volume passes run as an Ft pass and an F
// pass: FP64 at P3, where one pass would hold 2 x 5 x 20 FP64 accumulators
// and 5 x 20 FP64 coefficients per lane (more than the 512 registers of a
// lane at one wavefront per SIMD).
template <class T, int K>
constexpr bool kSplitVolume = sizeof(T) == 8 && K == 3;

// Minimum waves per SIMD requested from the register allocator for the
// volume kernel (FP32: two resident wavefronts per SIMD hide the memory
// phases, three for stage 2, whose 50 accumulators fit in 168 VGPRs: 6% off
// its time; FP64 needs twice the registers).
template <class T, int K, int MODE = 0>
struct CellWaves {
  static constexpr int value = (sizeof(T) == 4 && K <= 2) ? (MODE == 1 ? 3 : 2) : 1;
};

// Basis at the volume points, q = (qz NQ + qy) NQ + qx: phi[q][n] = B_n(x_q),
// dphi[q][d][n] = dB_n/dxi_d (x_q) (reference coordinates), w[q] = product
// of the Gauss weights (summing to 1).
template <class T, int K, int NQ>
struct PointBasis {
  static constexpr int NM = nmodes(K), NQ3 = NQ * NQ * NQ;
  T phi[NQ3][NM];
  T dphi[NQ3][3][NM];
  T w[NQ3];
  constexpr PointBasis() : phi{}, dphi{}, w{} {
    constexpr Modes<K> md{};
    for (int q = 0; q < NQ3; ++q) {
      const int ix[3] = {q % NQ, (q / NQ) % NQ, q / (NQ * NQ)};
      const double x[3] = {Gauss<NQ>::x[ix[0]], Gauss<NQ>::x[ix[1]], Gauss<NQ>::x[ix[2]]};
      w[q] = T(Gauss<NQ>::w[ix[0]] * Gauss<NQ>::w[ix[1]] * Gauss<NQ>::w[ix[2]]);
      for (int n = 0; n < NM; ++n) {
        phi[q][n] = T(leg(md.e[n][0], x[0]) * leg(md.e[n][1], x[1]) * leg(md.e[n][2], x[2]));
        for (int d = 0; d < 3; ++d) {
          double v = 1.0;
          for (int e = 0; e < 3; ++e) v *= (e == d) ? dleg(md.e[n][e], x[e]) : leg(md.e[n][e], x[e]);
          dphi[q][d][n] = T(v);
        }
      }
    }
  }
};
template <class T, int K, int NQ>
struct PointBasisHolder {
  static constexpr PointBasis<T, K, NQ> t{};
};

template <class T, int K, int NQ, int MODE, bool UNI, int PART = 0>
__global__ __launch_bounds__(kCellThreads, (CellWaves<T, K, MODE>::value)) void volume_kernel(
    const T* __restrict__ q, const T* __restrict__ rec, Geo g, Phys ph, VolOut<T> out, int* flag) {
  constexpr int NM = nmodes(K), NT = ntan(K), NQ3 = NQ * NQ * NQ;
  static_assert(PART == 0 || MODE != 1, "stage 2 has the Ft pass only");
  constexpr bool NEED_F = (MODE != 1) && PART != 2;  // accumulate F
  constexpr bool NEED_FT = PART != 1;                // accumulate Ft
  constexpr int NA = int(NEED_F) + int(NEED_FT);     // accumulator sets
  constexpr int NF = (MODE != 1) ? 2 : 1;            // record sets: stage-1 records hold F and Ft
  constexpr int RECN = 5 * NF * NT;
  constexpr Modes<K> md{};
  const long long N = g.ncell;
  const long long c = (long long)xcd_block(blockIdx.x, gridDim.x) * kCellThreads + threadIdx.x;
  const bool act = c < N;
  const long long cc = act ? c : N - 1;  // lanes past the end recompute the last cell, store nothing

  // 2 / width of this cell per axis: on a non-uniform mesh kept in LDS (read
  // where used, to spare registers), on a uniform one the kernel arguments
  __shared__ T sc[3][UNI ? 1 : kCellThreads];
  if constexpr (!UNI) {
    unsigned ci[3];
    cell_ijk(unsigned(cc), g, ci);
#pragma unroll
    for (int d = 0; d < 3; ++d) sc[d][threadIdx.x] = T(2.0 / g.w[d][ci[d]]);
  }
  auto scale = [&](int d) -> T { return UNI ? T(g.two_inv_h[d]) : sc[d][UNI ? 0 : threadIdx.x]; };
  // acc[a][v][n] = sum_q w_q sum_d F^a_d[v](x_q) (2/w_d) dB_n/dxi_d (x_q), a = F | Ft
  T acc[NA][5][NM];
#pragma unroll
  for (int f = 0; f < NA; ++f)
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int n = 0; n < NM; ++n) acc[f][v][n] = T(0);
  // Surface terms first: the upper face of the cell (its own record) minus
  // the lower face (record of the neighbour below) with the parity sign of B_n
  // at xi_d = -1, summed in T (a difference of two nearby records is exact in
  // T).
  const auto& mt = ModeTabHolder<K>::t;
  const long long ntile = (N + 63) >> 6;
  // Reference flux of the cell in FP32-bulk: the Euler flux of its mean state,
  // Cf[d][v].  It is subtracted from every volume point flux F_d and from the
  // mean (tangential mode 0) of both face records along d before they are
  // summed.  A flux constant over the cell adds nothing to R_n (the volume
  // rule integrates dB_n/dx_d exactly, and its integral is the surface term's
  // B_n(+1) - B_n(-1)), so this changes the result only by rounding, and the
  // float sums then hold flux differences instead of p ~ 71 or (rho E + p) U.
  constexpr bool CREF = NEED_F && sizeof(T) == 4;
  // kept in the lane's LDS column (read where used) rather than 15 registers
  __shared__ T scref[CREF ? 15 : 1][kCellThreads];
  if constexpr (CREF) {
    T cm[5], cfl[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) cm[v] = q[(long long)(v * NM) * N + cc];
    const Prim<T> sm = primitive(cm, T(ph.gm1));
    euler_flux<0>(sm, cm, cfl[0]);
    euler_flux<1>(sm, cm, cfl[1]);
    euler_flux<2>(sm, cm, cfl[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) scref[d * 5 + v][threadIdx.x] = cfl[d][v];
  }
  auto Cfr = [&](int d, int v) -> T { return scref[CREF ? d * 5 + v : 0][threadIdx.x]; };
  // Record groups (axis d, record set f, variable v): the NT values of the
  // upper and of the lower face record.  RPD groups are in flight at a time
  // (loaded ahead of their use); the scheduling barrier after each group keeps
  // the compiler from hoisting more loads than that.  Left to itself it issued
  // a whole axis at once, spilled loaded values and drained the load queue a
  // dozen times (10% of the FP32 stage-1 kernel, 8% of the FP64 one).
  const T* pu[3];
  const T* pl[3];
  T ixs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pu[d] = rec + rec_index(d, cc, 0, RECN, ntile);
    pl[d] = rec + rec_index(d, (long long)nb32(unsigned(cc), d, -1, g), 0, RECN, ntile);
    ixs[d] = T(0.5) * scale(d);  // 1 / width = |Gamma_d| / |K|
  }
  constexpr int NG = 3 * NF * 5;
  constexpr int RPD = 4;
  T rbuf[RPD][2][NT];
  auto load_grp = [&](auto gc, T (&b)[2][NT]) {
    constexpr int G = decltype(gc)::value;
    constexpr int d = G / (NF * 5), f = (G / 5) % NF, v = G % 5;
    constexpr bool is_f = (NF == 2 && f == 0);
    if constexpr (is_f ? NEED_F : NEED_FT) {
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const int r = (f * 5 + v) * NT + m;
        b[0][m] = pu[d][r * 64];
        b[1][m] = pl[d][r * 64];
      }
    }
  };
  static_for<RPD - 1>([&](auto gc) {
    constexpr int G = decltype(gc)::value;
    if constexpr (G < NG) load_grp(std::integral_constant<int, G>{}, rbuf[G % RPD]);
  });
  static_for<NG>([&](auto gc) {
    constexpr int G = decltype(gc)::value;
    if constexpr (G + RPD - 1 < NG)
      load_grp(std::integral_constant<int, G + RPD - 1>{}, rbuf[(G + RPD - 1) % RPD]);
    constexpr int d = G / (NF * 5), f = (G / 5) % NF, v = G % 5;
    // record set f holds F (f = 0 of stage-1 records) or Ft
    constexpr bool is_f = (NF == 2 && f == 0);
    constexpr int a = is_f ? 0 : NA - 1;
    if constexpr (is_f ? NEED_F : NEED_FT) {
      const T ix = ixs[d];
      static_for<NT>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        T ru = rbuf[G % RPD][0][m], rl = rbuf[G % RPD][1][m];
        if constexpr (CREF && is_f && m == 0) {
          const T cr = Cfr(d, v);
          ru -= cr;
          rl -= cr;
        }
        const T dm = ix * (rl - ru), dp = -ix * (rl + ru);
        static_for<NM>([&](auto nc) {
          constexpr int n = decltype(nc)::value;
          if constexpr (face_tan_of_mode<K>(n, d) == m) acc[a][v][n] += (md.e[n][d] & 1) ? dp : dm;
        });
      });
    }
    // (not after the last group: the cell's coefficient loads may start there)
    if constexpr (G + 1 < NG) __builtin_amdgcn_sched_barrier(0);
  });

  // the cell's coefficients, then the volume term
  T cf[5][NM];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int n = 0; n < NM; ++n) cf[v][n] = q[(long long)(v * NM + n) * N + cc];

  using PB = PointBasisHolder<T, K, NQ>;
  // The point's basis values (wavefront-uniform, scalar loads) are read one
  // point ahead in FP32 up to P2, so that their load latency overlaps the
  // previous point (FP64 and P3 have no SGPRs to spare for a second set).
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
  int bad = 0;
#pragma unroll 1
  for (int qi = 0; qi < NQ3; ++qi) {
    // keeps the width scales in LDS: no load moves across this point
    __asm__ __volatile__("" ::: "memory");
    PtBasis cur;
    if constexpr (PF) {
      cur = nxt;
      load_basis(qi + 1 < NQ3 ? qi + 1 : qi, nxt);
    }
    auto PHI = [&](int n) -> T {
      if constexpr (PF) return cur.phi[n]; else return PB::t.phi[qi][n];
    };
    auto DPHI = [&](int d, int n) -> T {
      if constexpr (PF) return cur.dphi[d][n]; else return PB::t.dphi[qi][d][n];
    };
    // physical-space derivative of the basis at this point (this cell's widths)
    T ds[3][NM];
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
#pragma unroll
      for (int d = 0; d < 3; ++d) ds[d][n] = (md.e[n][d] > 0) ? DPHI(d, n) * scale(d) : T(0);
    });
    T Q[5], dQ[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T v0 = T(0), vx = T(0), vy = T(0), vz = T(0);
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        const T cn = cf[v][n];
        if constexpr (n > 0) v0 += cn * PHI(n);
        if constexpr (md.e[n][0] > 0) vx += cn * ds[0][n];
        if constexpr (md.e[n][1] > 0) vy += cn * ds[1][n];
        if constexpr (md.e[n][2] > 0) vz += cn * ds[2][n];
      });
      Q[v] = v0 + cf[v][0];  // the cell mean (B_0 = 1) last
      dQ[0][v] = vx;
      dQ[1][v] = vy;
      dQ[2][v] = vz;
    }
    T F[3][5], Ft[3][5];
    volume_flux<T, NEED_F>(ph, Q, dQ, F, Ft, bad);
    T wq;
    if constexpr (PF) wq = cur.w; else wq = PB::t.w[qi];
    static_for<NM>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (md.e[n][d] > 0) {
          const T b = ds[d][n] * wq;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if constexpr (CREF)
              acc[0][v][n] += (F[d][v] - Cfr(d, v)) * b;
            else if constexpr (NEED_F)
              acc[0][v][n] += F[d][v] * b;
            if constexpr (NEED_FT) acc[NA - 1][v][n] += Ft[d][v] * b;
          }
        }
      }
    });
  }
  if (bad && act) atomicOr(flag, 1);

  // M^{-1} and the stage update in FP64.  The FP64 inputs of the update (Q^n,
  // P, or the L_t of the Ft pass) of a group of VB variables are loaded before
  // the group's first store: the compiler cannot prove that the output arrays
  // alias none of them, so a load placed after a store waits for that store and
  // then for its own data, one full memory latency per coefficient.  VB = 5 (one
  // group) where the inputs take at most 100 VGPRs, else smaller groups.
  if (!act) return;
  const double dt = out.dt;
  constexpr int NIN = (MODE == 0 && PART == 1) ? 2 : ((MODE == 0 && PART != 2) || MODE == 1) ? 1 : 0;
  constexpr int VB = NIN * NM * 5 <= 50 ? 5 : NIN * NM * 2 <= 50 ? 2 : 1;
#pragma unroll
  for (int v0 = 0; v0 < 5; v0 += VB) {
    double in[NIN > 0 ? NIN : 1][VB][NM];
    if constexpr (NIN > 0) {
#pragma unroll
      for (int j = 0; j < VB; ++j)
#pragma unroll
        for (int n = 0; n < NM; ++n) {
          if (v0 + j >= 5) break;
          const long long gi = (long long)((v0 + j) * NM + n) * N + c;
          in[0][j][n] = MODE == 1 ? out.P[gi] : out.qn[gi];
          if constexpr (NIN == 2) in[NIN - 1][j][n] = out.Lt[gi];
        }
    }
#pragma unroll
    for (int j = 0; j < VB; ++j)
#pragma unroll
      for (int n = 0; n < NM; ++n) {
        if (v0 + j >= 5) break;
        const int v = v0 + j;
        const double mi = mt.minv[n];
        const double Ln = NEED_F ? double(acc[0][v][n]) * mi : 0.0;
        const double Ltn = NEED_FT ? double(acc[NA - 1][v][n]) * mi : 0.0;
        const long long gi = (long long)(v * NM + n) * N + c;
        if constexpr (MODE == 0 && PART == 2) {
          out.Lt[gi] = Ltn;
        } else if constexpr (MODE == 0) {
          const double qn = in[0][j][n];
          const double lt = PART == 1 ? in[NIN - 1][j][n] : Ltn;
          out.qstar[gi] = T(qn + 0.5 * dt * Ln + 0.125 * dt * dt * lt);
          out.P[gi] = qn + dt * Ln + (dt * dt / 6.0) * lt;
        } else if constexpr (MODE == 1) {
          const double qnew = in[0][j][n] + (dt * dt / 3.0) * Ltn;
          out.qnew[gi] = qnew;
          if (out.qshadow) out.qshadow[gi] = T(qnew);
        } else {
          if constexpr (NEED_F) out.L[gi] = Ln;
          if constexpr (NEED_FT) out.Lt[gi] = Ltn;
        }
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
