// launch.hpp -- launch sequences of one configuration (precision T, degree
// K, NQ Gauss points per axis): the S2O4 step (Eq. (two-stage)), the operator
// evaluation, and the reverse sweep of the adjoint with segment
// recomputation.  Instantiated in instantiate.hip.
//
// Launch sequence of one step, all on the caller's stream:
//   stage 1: face_kernel<F and Ft>   volume_kernel<MODE 0>  -> Q*, P
//   stage 2: face_kernel<Ft only>    volume_kernel<MODE 1>  -> Q^{n+1}
// In FP32-bulk mode the kernels read a float copy of the coefficients (written
// by the stage-2 update for the next step) while Q^n, P and Q^{n+1} stay FP64.
#pragma once

#include <algorithm>

#include "kernels_adj.hpp"
#include "kernels_fwd.hpp"
#include "runtime.hpp"

namespace dgrt {

using namespace dgk;

template <class T>
int launch_convert(dg_hgks_ctx* c, const double* a, T* b, long long n) {
  const long long nb = std::min<long long>((n + 255) / 256, 65536);
  DG_LAUNCH(c, 2, (convert_kernel<T><<<dim3((unsigned)nb), 256, 0, c->stream>>>(a, b, n)));
  return DG_HGKS_OK;
}

// One operator evaluation: face pass, then volume pass.  The two passes are
// separate functions so that each can be instantiated in its own object
// (instantiate.hip).
template <class T, int K, int NQ, int MODE>
int launch_face_pass(dg_hgks_ctx* c, const T* qin, const Geo& g, const Phys& ph) {
  T* rec = (T*)(c->ws + c->lay.rec);
  int* flag = (int*)(c->ws + c->lay.flag);
  constexpr int FT = face_threads<T, K>();
  const unsigned nfb = (unsigned)((g.ncell + FT - 1) / FT);
  // uniform meshes take the cell widths from the kernel arguments
  auto run = [&](auto uc) {
    constexpr bool UNI = decltype(uc)::value;
    if constexpr (MODE == 1) {
      DG_LAUNCH(c, 0, (face_kernel<T, K, NQ, false, UNI><<<dim3(3 * nfb), FT, 0, c->stream>>>(qin, rec, g, ph, flag)));
    } else {
      DG_LAUNCH(c, 0, (face_kernel<T, K, NQ, true, UNI><<<dim3(3 * nfb), FT, 0, c->stream>>>(qin, rec, g, ph, flag)));
    }
    return DG_HGKS_OK;
  };
  return g.uniform ? run(std::true_type{}) : run(std::false_type{});
}

template <class T, int K, int NQ, int MODE>
int launch_volume_pass(dg_hgks_ctx* c, const T* qin, const VolOut<T>& o, const Geo& g, const Phys& ph) {
  const T* rec = (const T*)(c->ws + c->lay.rec);
  int* flag = (int*)(c->ws + c->lay.flag);
  const unsigned nvb = (unsigned)((g.ncell + kCellThreads - 1) / kCellThreads);
  auto run = [&](auto uc) {
    constexpr bool UNI = decltype(uc)::value;
    if constexpr (MODE != 1 && kSplitVolume<T, K>) {
      // Ft pass (L_t to the workspace in stage 1), then F pass and update
      VolOut<T> ot = o;
      if constexpr (MODE == 0) ot.Lt = (double*)(c->ws + c->lay.lt_tmp);
      DG_LAUNCH(c, 1, (volume_kernel<T, K, NQ, MODE, UNI, 2><<<dim3(nvb), kCellThreads, 0, c->stream>>>(
                          qin, rec, g, ph, ot, flag)));
      DG_LAUNCH(c, 1, (volume_kernel<T, K, NQ, MODE, UNI, 1><<<dim3(nvb), kCellThreads, 0, c->stream>>>(
                          qin, rec, g, ph, ot, flag)));
    } else {
      DG_LAUNCH(c, 1, (volume_kernel<T, K, NQ, MODE, UNI><<<dim3(nvb), kCellThreads, 0, c->stream>>>(qin, rec, g, ph,
                                                                                                     o, flag)));
    }
    return DG_HGKS_OK;
  };
  return g.uniform ? run(std::true_type{}) : run(std::false_type{});
}

template <class T, int K, int NQ, int MODE>
int launch_stage(dg_hgks_ctx* c, const T* qin, const VolOut<T>& o, const Geo& g, const Phys& ph) {
  const int rc = launch_face_pass<T, K, NQ, MODE>(c, qin, g, ph);
  if (rc) return rc;
  return launch_volume_pass<T, K, NQ, MODE>(c, qin, o, g, ph);
}

template <class T, int K, int NQ>
int run_step(dg_hgks_ctx* c, double* q, double dt, int nsteps, double* ckpt, int stride) {
  const Geo g = make_geo(c);
  const Phys ph = make_phys(c, dt);
  const long long n = 5LL * c->nm * g.ncell;
  constexpr bool bulk = sizeof(T) == 4;
  T* qs = bulk ? (T*)(c->ws + c->lay.qs) : nullptr;
  T* qstar = (T*)(c->ws + c->lay.qstar);
  double* P = (double*)(c->ws + c->lay.P);
  int rc = ensure_ready(c);
  if (rc) return rc;
  if (bulk && nsteps > 0) {
    rc = launch_convert<T>(c, q, qs, n);
    if (rc) return rc;
  }
  for (int s = 0; s < nsteps; ++s) {
    if (ckpt && s % stride == 0)
      DG_HIP(c, hipMemcpyAsync(ckpt + (size_t)(s / stride) * n, q, n * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    const T* qin = bulk ? qs : (const T*)q;
    VolOut<T> o1{};
    o1.qn = q;
    o1.P = P;
    o1.qstar = qstar;
    o1.dt = dt;
    rc = launch_stage<T, K, NQ, 0>(c, qin, o1, g, ph);
    if (rc) return rc;
    VolOut<T> o2{};
    o2.P = P;
    o2.qnew = q;
    o2.qshadow = qs;
    o2.dt = dt;
    rc = launch_stage<T, K, NQ, 1>(c, qstar, o2, g, ph);
    if (rc) return rc;
  }
  return DG_HGKS_OK;
}

template <class T, int K, int NQ>
int run_residual(dg_hgks_ctx* c, const double* q, double dt, double* L, double* Lt) {
  const Geo g = make_geo(c);
  const Phys ph = make_phys(c, dt);
  const long long n = 5LL * c->nm * g.ncell;
  int rc = ensure_ready(c);
  if (rc) return rc;
  const T* qin;
  if constexpr (sizeof(T) == 4) {
    T* qs = (T*)(c->ws + c->lay.qs);
    rc = launch_convert<T>(c, q, qs, n);
    if (rc) return rc;
    qin = qs;
  } else {
    qin = q;
  }
  VolOut<T> o{};
  o.L = L;
  o.Lt = Lt;
  o.dt = dt;
  return launch_stage<T, K, NQ, 2>(c, qin, o, g, ph);
}

// Adjoint of one stage: face pass then volume pass (kernels_adj.hpp).  The
// two passes are separate functions so that each can be instantiated in its
// own object (instantiate.hip).
template <class T, int K, int NQ, int STAGE>
int launch_adj_face(dg_hgks_ctx* c, const T* qin, const AdjIn<STAGE>& in, const Geo& g, const Phys& ph) {
  const unsigned nbf = (unsigned)adj_face_blocks((size_t)g.ncell);
  double* frec = (double*)(c->ws + c->lay.adj_frec);
  double* mu = (double*)(c->ws + c->lay.adj_mu);
  DG_LAUNCH(c, 3, (adj_face_kernel<T, K, NQ, STAGE><<<dim3(3 * nbf), kAdjFaceThreads, 0, c->stream>>>(qin, in, frec, g, ph, mu)));
  return DG_HGKS_OK;
}

template <class T, int K, int NQ, int STAGE>
int launch_adj_volume(dg_hgks_ctx* c, const T* qin, const AdjIn<STAGE>& in, double* out, const Geo& g,
                      const Phys& ph) {
  const long long N = g.ncell;
  const unsigned nbf = (unsigned)adj_face_blocks((size_t)N);
  const unsigned nbv = (unsigned)((N + kCellThreads - 1) / kCellThreads);
  double* frec = (double*)(c->ws + c->lay.adj_frec);
  double* mu = (double*)(c->ws + c->lay.adj_mu);
  DG_LAUNCH(c, 4, (adj_volume_kernel<T, K, NQ, STAGE><<<dim3(nbv), kCellThreads, 0, c->stream>>>(
                      qin, in, frec, out, g, ph, mu, 3LL * nbf)));
  return DG_HGKS_OK;
}

template <class T, int K, int NQ, int STAGE>
int launch_adj_stage(dg_hgks_ctx* c, const T* qin, const AdjIn<STAGE>& in, double* out, const Geo& g,
                     const Phys& ph) {
  const int rc = launch_adj_face<T, K, NQ, STAGE>(c, qin, in, g, ph);
  if (rc) return rc;
  return launch_adj_volume<T, K, NQ, STAGE>(c, qin, in, out, g, ph);
}

// Reverse sweep over the steps.  Segment s covers steps [s*stride,
// min((s+1)*stride, nsteps)); it is recomputed from its checkpoint, keeping
// Q^n (FP64) and Q* (bulk precision) of every step, then reversed step by step:
//   stage 2: qsbar = (dL_t/dQ at Q*)^T (dt^2/3 qbar)
//   stage 1: qbar <- qbar + qsbar + (d(L, L_t)/dQ at Q^n)^T (dt qbar + dt/2 qsbar,
//                                                          dt^2/6 qbar + dt^2/8 qsbar)
template <class T, int K, int NQ>
int run_adjoint(dg_hgks_ctx* c, const double* ckpt, int stride, double dt, int nsteps, const double* qN_bar,
                double* q0_bar, double* mu_bar_host) {
  const Geo g = make_geo(c);
  const Phys ph = make_phys(c, dt);
  const long long n = 5LL * c->nm * g.ncell;
  constexpr bool bulk = sizeof(T) == 4;
  T* qs = bulk ? (T*)(c->ws + c->lay.qs) : nullptr;
  double* P = (double*)(c->ws + c->lay.P);
  double* states = (double*)(c->ws + c->lay.adj_states);
  T* stars = (T*)(c->ws + c->lay.adj_stars);
  double* qbar = (double*)(c->ws + c->lay.adj_qbar);
  double* qsbar = (double*)(c->ws + c->lay.adj_qsbar);
  double* mu = (double*)(c->ws + c->lay.adj_mu);
  double* mu_part2 = (double*)(c->ws + c->lay.adj_tmp);
  const long long nslots = (long long)adj_mu_slots((size_t)g.ncell);
  const unsigned nparts = (unsigned)((nslots + kMuChunk - 1) / kMuChunk);
  int rc = ensure_ready(c);
  if (rc) return rc;
  DG_HIP(c, hipMemcpyAsync(qbar, qN_bar, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  DG_LAUNCH(c, 2, (zero_kernel<<<dim3(256), 256, 0, c->stream>>>(mu, nslots)));
  const int nseg = (nsteps + stride - 1) / stride;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int n0 = seg * stride;
    const int len = std::min(stride, nsteps - n0);
    DG_HIP(c, hipMemcpyAsync(states, ckpt + (size_t)seg * n, n * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    // forward recomputation of the segment
    for (int j = 0; j < len; ++j) {
      double* Sj = states + (size_t)j * n;
      T* Qs = stars + (size_t)j * n;
      const T* qin;
      if constexpr (bulk) {
        rc = launch_convert<T>(c, Sj, qs, n);
        if (rc) return rc;
        qin = qs;
      } else {
        qin = (const T*)Sj;
      }
      VolOut<T> o1{};
      o1.qn = Sj;
      o1.P = P;
      o1.qstar = Qs;
      o1.dt = dt;
      rc = launch_stage<T, K, NQ, 0>(c, qin, o1, g, ph);
      if (rc) return rc;
      if (j + 1 < len) {
        VolOut<T> o2{};
        o2.P = P;
        o2.qnew = states + (size_t)(j + 1) * n;
        o2.qshadow = nullptr;
        o2.dt = dt;
        rc = launch_stage<T, K, NQ, 1>(c, Qs, o2, g, ph);
        if (rc) return rc;
      }
    }
    // reverse
    for (int j = len - 1; j >= 0; --j) {
      double* Sj = states + (size_t)j * n;
      const T* Qs = stars + (size_t)j * n;
      AdjIn<2> in2{qbar, qsbar, dt};
      rc = launch_adj_stage<T, K, NQ, 2>(c, Qs, in2, qsbar, g, ph);
      if (rc) return rc;
      const T* qin;
      if constexpr (bulk) {
        rc = launch_convert<T>(c, Sj, qs, n);
        if (rc) return rc;
        qin = qs;
      } else {
        qin = (const T*)Sj;
      }
      AdjIn<1> in1{qbar, qsbar, dt};
      rc = launch_adj_stage<T, K, NQ, 1>(c, qin, in1, qbar, g, ph);
      if (rc) return rc;
    }
  }
  DG_HIP(c, hipMemcpyAsync(q0_bar, qbar, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  DG_LAUNCH(c, 2, (reduce_mu_kernel<<<nparts, 256, 0, c->stream>>>(mu, nslots, kMuChunk, mu_part2)));
  DG_LAUNCH(c, 2, (reduce_mu_kernel<<<1, 256, 0, c->stream>>>(mu_part2, nparts, nparts, mu_part2 + nparts)));
  double h = 0.0;
  DG_HIP(c, hipMemcpyAsync(&h, mu_part2 + nparts, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  DG_HIP(c, hipStreamSynchronize(c->stream));
  *mu_bar_host = h;
  return dg_hgks_check(c);
}

}  // namespace dgrt
