// runtime.hpp -- host-side state shared by the C-ABI (dg_hgks.hip) and the
// per-configuration launch code (launch.hpp, instantiated once per
// precision x degree x quadrature in instantiate.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dg_hgks.h"
#include "kernels_fwd.hpp"

namespace dgrt {

// Byte offsets of the workspace regions (256-byte aligned).
struct Layout {
  size_t flag = 0, geo = 0, qs = 0, qstar = 0, P = 0, rec = 0, diag = 0, lt_tmp = 0;
  size_t adj_states = 0, adj_stars = 0, adj_qbar = 0, adj_qsbar = 0, adj_frec = 0,
         adj_mu = 0, adj_tmp = 0;
  size_t total = 0;
};

struct TimingRec {
  int cls;
  hipEvent_t a, b;
};

}  // namespace dgrt

struct dg_hgks_ctx {
  dg_hgks_params p{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int max_stride = 0;
  dgrt::Layout lay;
  long long ncell = 0;
  int nm = 0, nt = 0;
  double mu = 0.0;
  bool ready = false;          // flag cleared and cell widths uploaded
  std::vector<double> widths;  // nx + ny + nz cell widths (x, y, z)
  bool uniform = true;         // every axis has equal widths
  double w0[3] = {0, 0, 0};    // width of the first cell of each axis (of every cell on a uniform mesh)
  std::string err;
  bool timing = false;
  std::vector<dgrt::TimingRec> trecs;
  double t_ms[5] = {0, 0, 0, 0, 0};
  long long t_n[5] = {0, 0, 0, 0, 0};
};

namespace dgrt {

// Record msg as the context's (or, for c == nullptr, the thread's init) error.
int fail(dg_hgks_ctx* c, int code, const std::string& msg);
dgk::Geo make_geo(const dg_hgks_ctx* c);
dgk::Phys make_phys(const dg_hgks_ctx* c, double dt);
// HIP events around one launch of timing class cls (when timing is on).
int t_begin(dg_hgks_ctx* c, int cls);
int t_end(dg_hgks_ctx* c);
// Once per context, on its stream: clear the non-physical-state flag (a
// kernel, not a memset) and upload the cell widths to the workspace.
int ensure_ready(dg_hgks_ctx* c);

// Entry points of one compiled configuration (launch.hpp).
template <class T, int K, int NQ>
int run_step(dg_hgks_ctx* c, double* q, double dt, int nsteps, double* ckpt, int stride);
template <class T, int K, int NQ>
int run_residual(dg_hgks_ctx* c, const double* q, double dt, double* L, double* Lt);
template <class T, int K, int NQ>
int run_adjoint(dg_hgks_ctx* c, const double* ckpt, int stride, double dt, int nsteps, const double* qN_bar,
                double* q0_bar, double* mu_bar_host);

}  // namespace dgrt

#define DG_HIP(ctx, call)                                                                                    \
  do {                                                                                                       \
    hipError_t e_ = (call);                                                                                  \
    if (e_ != hipSuccess) return dgrt::fail(ctx, DG_HGKS_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

#define DG_LAUNCH(ctx, cls, ...)       \
  do {                                 \
    int rc_ = dgrt::t_begin(ctx, cls); \
    if (rc_) return rc_;               \
    __VA_ARGS__;                       \
    DG_HIP(ctx, hipGetLastError());    \
    rc_ = dgrt::t_end(ctx);            \
    if (rc_) return rc_;               \
  } while (0)
