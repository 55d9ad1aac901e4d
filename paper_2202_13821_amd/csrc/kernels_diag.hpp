// kernels_diag.hpp -- Taylor-Green diagnostics of a state (Section 5.3):
// the domain integrals of the kinetic energy |rho U|^2 / (2 rho) and of the
// enstrophy |curl U|^2 / 2 on the volume Gauss rule, and the gradient of the
// kinetic energy with respect to the modal coefficients (the seed of the
// adjoint for the final-kinetic-energy objective).  FP64, one lane per cell,
// fixed-order reductions (deterministic).
#pragma once

#include "kernels_fwd.hpp"

namespace dgk {

// part[2 b + 0/1] = block b's kinetic energy / enstrophy; grad (if not null)
// = dE_k/dq in the layout of q.
template <int K, int NQ>
__global__ __launch_bounds__(kCellThreads) void diag_kernel(const double* __restrict__ q, Geo g,
                                                           double* __restrict__ part, double* __restrict__ grad) {
  constexpr int NM = nmodes(K), NQ3 = NQ * NQ * NQ;
  constexpr Modes<K> md{};
  using PB = PointBasisHolder<double, K, NQ>;
  __shared__ double red[2][kCellThreads / 64];
  const long long N = g.ncell;
  const long long c = (long long)blockIdx.x * kCellThreads + threadIdx.x;
  const bool act = c < N;
  const long long cc = act ? c : N - 1;
  unsigned ci[3];
  cell_ijk(unsigned(cc), g, ci);
  const double wx = g.w[0][ci[0]], wy = g.w[1][ci[1]], wz = g.w[2][ci[2]];
  const double vol = wx * wy * wz;
  const double sx = 2.0 / wx, sy = 2.0 / wy, sz = 2.0 / wz;
  double cf[4][NM], gk[4][NM];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int n = 0; n < NM; ++n) {
      cf[v][n] = q[(long long)(v * NM + n) * N + cc];
      gk[v][n] = 0.0;
    }
  double ek = 0.0, en = 0.0;
#pragma unroll 1
  for (int qi = 0; qi < NQ3; ++qi) {
    double Q[4], G[4][3];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double v0 = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        const double a = cf[v][n];
        v0 += a * PB::t.phi[qi][n];
        if constexpr (md.e[n][0] > 0) gx += a * PB::t.dphi[qi][0][n];
        if constexpr (md.e[n][1] > 0) gy += a * PB::t.dphi[qi][1][n];
        if constexpr (md.e[n][2] > 0) gz += a * PB::t.dphi[qi][2][n];
      });
      Q[v] = v0;
      G[v][0] = gx * sx;
      G[v][1] = gy * sy;
      G[v][2] = gz * sz;
    }
    const double w = PB::t.w[qi];
    const double ir = 1.0 / Q[0];
    const double m2 = Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3];
    ek += w * 0.5 * m2 * ir;
    // dU_j/dx_e = (d(rho U_j)/dx_e - U_j drho/dx_e) / rho
    double dU[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int e = 0; e < 3; ++e) dU[j][e] = (G[1 + j][e] - Q[1 + j] * ir * G[0][e]) * ir;
    const double ox = dU[2][1] - dU[1][2], oy = dU[0][2] - dU[2][0], oz = dU[1][0] - dU[0][1];
    en += w * 0.5 * (ox * ox + oy * oy + oz * oz);
    if (grad) {
      // d(|m|^2 / (2 rho)) / drho = -|m|^2 / (2 rho^2), / dm_j = m_j / rho
      const double dq[4] = {-0.5 * m2 * ir * ir, Q[1] * ir, Q[2] * ir, Q[3] * ir};
      static_for<NM>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        const double b = w * PB::t.phi[qi][n];
#pragma unroll
        for (int v = 0; v < 4; ++v) gk[v][n] += dq[v] * b;
      });
    }
  }
  if (grad && act) {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int n = 0; n < NM; ++n) grad[(long long)(v * NM + n) * N + c] = v < 4 ? vol * gk[v][n] : 0.0;
  }
  ek = act ? vol * ek : 0.0;
  en = act ? vol * en : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ek += __shfl_xor(ek, o, 64);
    en += __shfl_xor(en, o, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = ek;
    red[1][wv] = en;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kCellThreads / 64; ++i) s += red[threadIdx.x][i];
    part[2 * (long long)blockIdx.x + threadIdx.x] = s;
  }
}

// out[k] = sum_b part[2 b + k] in a fixed order (one block of 256 lanes).
static __global__ __launch_bounds__(256) void diag_reduce_kernel(const double* part, long long nb, double* out) {
  __shared__ double sh[2][256];
  double s0 = 0.0, s1 = 0.0;
  for (long long i = threadIdx.x; i < nb; i += 256) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace dgk
