// dg_hgks.hip -- host side of the C-ABI in include/dg_hgks.h: parameter
// validation, workspace carving, dispatch to the compiled configurations,
// per-kernel event timing, error reporting and the point-flux diagnostics.
// The launch sequences of the step and of its adjoint are in launch.hpp,
// compiled once per configuration (instantiate.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dg_hgks.h"
#include "kernels_adj.hpp"
#include "kernels_diag.hpp"
#include "kernels_fwd.hpp"
#include "runtime.hpp"

using namespace dgk;

namespace {

thread_local std::string g_init_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

namespace dgrt {

int fail(dg_hgks_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_init_error = msg;
  return code;
}

}  // namespace dgrt

namespace {

using dgrt::fail;
using dgrt::Layout;

bool supported(int k, int nq) {
  return (k == 1 && nq == 2) || (k == 2 && nq == 3) || (k == 2 && nq == 2) || (k == 3 && nq == 4) || (k == 3 && nq == 3);
}

int validate(const dg_hgks_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return DG_HGKS_EINVAL; }
  if (p->struct_size != sizeof(dg_hgks_params)) { why = "params.struct_size != sizeof(dg_hgks_params)"; return DG_HGKS_EINVAL; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "grid sizes must be >= 1"; return DG_HGKS_EINVAL; }
  if ((long long)p->nx * p->ny * p->nz > (1LL << 31)) { why = "too many cells"; return DG_HGKS_EINVAL; }
  for (int e = 0; e < 3; ++e)
    if (!(p->hi[e] > p->lo[e]) || !std::isfinite(p->hi[e] - p->lo[e])) { why = "need hi > lo on every axis"; return DG_HGKS_EINVAL; }
  if (p->degree < 1 || p->degree > 3) { why = "degree must be 1, 2 or 3"; return DG_HGKS_EINVAL; }
  const int nq = p->nq ? p->nq : p->degree + 1;
  if (nq < 1 || nq > 4) { why = "nq must be in [1, 4]"; return DG_HGKS_EINVAL; }
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) { why = "gamma must be > 1"; return DG_HGKS_EINVAL; }
  if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) { why = "mu must be >= 0"; return DG_HGKS_EINVAL; }
  if (!(p->prandtl > 0.0) || !std::isfinite(p->prandtl)) { why = "prandtl must be > 0"; return DG_HGKS_EINVAL; }
  if (p->precision != DG_HGKS_FP64 && p->precision != DG_HGKS_FP32_BULK) { why = "unknown precision"; return DG_HGKS_EINVAL; }
  if (p->cell_widths) {
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int e = 0, off = 0; e < 3; off += n[e], ++e) {
      double sum = 0.0;
      for (int i = 0; i < n[e]; ++i) {
        const double w = p->cell_widths[off + i];
        if (!(w > 0.0) || !std::isfinite(w)) { why = "cell_widths must be finite and > 0"; return DG_HGKS_EINVAL; }
        sum += w;
      }
      const double len = p->hi[e] - p->lo[e];
      if (!(std::fabs(sum - len) <= 1e-10 * len)) { why = "cell_widths must sum to hi - lo on every axis"; return DG_HGKS_EINVAL; }
    }
  }
  if (!supported(p->degree, nq)) { why = "(degree, nq) combination not compiled"; return DG_HGKS_EUNSUPPORTED; }
  return DG_HGKS_OK;
}

Layout make_layout(const dg_hgks_params& p, int max_stride) {
  Layout L;
  const int nq = p.nq ? p.nq : p.degree + 1;
  (void)nq;
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  const size_t nm = (size_t)dgk::nmodes(p.degree), nt = (size_t)dgk::ntan(p.degree);
  const size_t Ts = p.precision == DG_HGKS_FP32_BULK ? 4 : 8;
  const size_t state = 5 * nm * N;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.flag = take(kAlign);
  L.geo = take((size_t)(p.nx + p.ny + p.nz) * 8);  // cell widths per axis
  L.qs = (Ts == 4) ? take(state * Ts) : 0;
  L.qstar = take(state * Ts);
  L.P = take(state * 8);
  L.rec = take(3 * ((N + 63) / 64 * 64) * 10 * nt * Ts);  // records padded to whole 64-cell tiles
  L.diag = take((2 * ((N + dgk::kCellThreads - 1) / dgk::kCellThreads) + 2) * 8);  // diagnostics partial sums
  // L_t of the stage-1 Ft pass where the volume pass is split (FP64 at P3)
  if (Ts == 8 && p.degree == 3) L.lt_tmp = take(state * 8);
  if (max_stride > 0) {
    L.adj_states = take((size_t)max_stride * state * 8);  // Q^n of each step of a segment
    L.adj_stars = take((size_t)max_stride * state * Ts);  // Q* of each step
    L.adj_qbar = take(state * 8);
    L.adj_qsbar = take(state * 8);
    L.adj_frec = take(3 * 2 * ((N + 63) / 64 * 64) * 5 * nm * 8);  // per face: cotangents of both cells' coefficients
    L.adj_mu = take(adj_mu_slots(N) * 8);  // per-block partial sums of dJ/dmu
    L.adj_tmp = take(((adj_mu_slots(N) + dgk::kMuChunk - 1) / dgk::kMuChunk + 1) * 8);  // second pass + result
  }
  L.total = off;
  return L;
}

template <class T_, int K_, int NQ_>
struct Tag {
  using T = T_;
  static constexpr int K = K_, NQ = NQ_;
};

template <class F>
int dispatch(const dg_hgks_params& p, F&& f) {
  const bool f32 = p.precision == DG_HGKS_FP32_BULK;
  const int k = p.degree, nq = p.nq ? p.nq : p.degree + 1;
  if (k == 1 && nq == 2) return f32 ? f(Tag<float, 1, 2>{}) : f(Tag<double, 1, 2>{});
  if (k == 2 && nq == 3) return f32 ? f(Tag<float, 2, 3>{}) : f(Tag<double, 2, 3>{});
  if (k == 2 && nq == 2) return f32 ? f(Tag<float, 2, 2>{}) : f(Tag<double, 2, 2>{});
  if (k == 3 && nq == 4) return f32 ? f(Tag<float, 3, 4>{}) : f(Tag<double, 3, 4>{});
  if (k == 3 && nq == 3) return f32 ? f(Tag<float, 3, 3>{}) : f(Tag<double, 3, 3>{});
  return DG_HGKS_EUNSUPPORTED;
}

}  // namespace

__global__ void clear_flag_kernel(int* f) {
  if (threadIdx.x == 0) f[0] = 0;
}


namespace dgrt {

dgk::Geo make_geo(const dg_hgks_ctx* c) {
  const dg_hgks_params& p = c->p;
  dgk::Geo g{};
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.ncell = (long long)p.nx * p.ny * p.nz;
  const double* w = (const double*)(c->ws + c->lay.geo);
  g.w[0] = w;
  g.w[1] = w + p.nx;
  g.w[2] = w + p.nx + p.ny;
  g.uniform = c->uniform ? 1 : 0;
  g.two_inv_h[0] = 2.0 / c->w0[0];
  g.two_inv_h[1] = 2.0 / c->w0[1];
  g.two_inv_h[2] = 2.0 / c->w0[2];
  return g;
}

dgk::Phys make_phys(const dg_hgks_ctx* c, double dt) {
  dgk::Phys ph{};
  ph.K = (5.0 - 3.0 * c->p.gamma) / (c->p.gamma - 1.0);
  ph.gm1 = c->p.gamma - 1.0;
  ph.mu = c->mu;
  ph.inv_pr_m1 = 1.0 / c->p.prandtl - 1.0;
  ph.dt = dt;
  ph.inv_k3 = 1.0 / (ph.K + 3.0);
  ph.cp = 0.5 * (ph.K + 5.0);
  ph.half_dt_over_mu = c->mu > 0.0 ? 0.5 * dt / c->mu : 0.0;
  ph.inv_dt = 1.0 / dt;
  return ph;
}

// ---- event timing -----------------------------------------------------------
int t_begin(dg_hgks_ctx* c, int cls) {
  if (!c->timing) return DG_HGKS_OK;
  TimingRec r{cls, nullptr, nullptr};
  DG_HIP(c, hipEventCreate(&r.a));
  DG_HIP(c, hipEventCreate(&r.b));
  DG_HIP(c, hipEventRecord(r.a, c->stream));
  c->trecs.push_back(r);
  return DG_HGKS_OK;
}
int t_end(dg_hgks_ctx* c) {
  if (!c->timing) return DG_HGKS_OK;
  DG_HIP(c, hipEventRecord(c->trecs.back().b, c->stream));
  return DG_HGKS_OK;
}
int ensure_ready(dg_hgks_ctx* c) {
  if (c->ready) return DG_HGKS_OK;
  clear_flag_kernel<<<1, 64, 0, c->stream>>>((int*)(c->ws + c->lay.flag));
  DG_HIP(c, hipGetLastError());
  // the source is the context's own host copy, alive until dg_hgks_destroy
  DG_HIP(c, hipMemcpyAsync(c->ws + c->lay.geo, c->widths.data(), c->widths.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  c->ready = true;
  return DG_HGKS_OK;
}

}  // namespace dgrt

namespace {

using dgrt::ensure_ready;
using dgrt::make_geo;
using dgrt::make_phys;
using dgrt::t_begin;
using dgrt::t_end;

int t_collect(dg_hgks_ctx* c) {
  if (c->trecs.empty()) return DG_HGKS_OK;
  DG_HIP(c, hipStreamSynchronize(c->stream));
  for (auto& r : c->trecs) {
    float ms = 0.f;
    DG_HIP(c, hipEventElapsedTime(&ms, r.a, r.b));
    c->t_ms[r.cls] += ms;
    c->t_n[r.cls] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->trecs.clear();
  return DG_HGKS_OK;
}

}  // namespace

// ---- device scratch of the allocation-free step ------------------------------
// dg_hgks_step_noalloc keeps its workspace (flag word, stage copies, face
// records) in this file-scope array instead of a caller's buffer.  Every GPU
// the library runs on holds its own copy from module load until the process
// ends; host code reaches it only through the address looked up per device
// below (the array's name is not a device address on the host).
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ void copy_flag_kernel(const int* f, int32_t* out) {
  if (threadIdx.x == 0) out[0] = f[0];
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
int scratch_ptr(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, DG_HGKS_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, DG_HGKS_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, DG_HGKS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return DG_HGKS_OK;
}

}  // namespace

// ============================================================================
// C-ABI
// ============================================================================
extern "C" {

int64_t dg_hgks_nmodes(int32_t degree) {
  if (degree < 1 || degree > 3) return -1;
  return dgk::nmodes(degree);
}

size_t dg_hgks_workspace_bytes(const dg_hgks_params* p, int32_t max_stride) {
  std::string why;
  if (validate(p, why) != DG_HGKS_OK || max_stride < 0) return 0;
  return make_layout(*p, max_stride).total;
}

int dg_hgks_init(const dg_hgks_params* p, void* hip_stream, void* workspace, size_t workspace_bytes,
                 dg_hgks_ctx** out) {
  if (!out) return fail(nullptr, DG_HGKS_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (!workspace) return fail(nullptr, DG_HGKS_EINVAL, "workspace is NULL");
  if ((uintptr_t)workspace % kAlign) return fail(nullptr, DG_HGKS_EINVAL, "workspace must be 256-byte aligned");
  // max_stride is derived from the workspace: the largest stride that fits
  const Layout base = make_layout(*p, 0);
  if (workspace_bytes < base.total) return fail(nullptr, DG_HGKS_ENOMEM, "workspace smaller than dg_hgks_workspace_bytes");
  int ms = 0;
  while (ms < (1 << 20) && make_layout(*p, ms + 1).total <= workspace_bytes) ++ms;
  dg_hgks_ctx* c = new (std::nothrow) dg_hgks_ctx;
  if (!c) return fail(nullptr, DG_HGKS_ENOMEM, "host allocation failed");
  c->p = *p;
  if (c->p.nq == 0) c->p.nq = c->p.degree + 1;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = workspace_bytes;
  c->max_stride = ms;
  c->lay = make_layout(c->p, ms);
  c->ncell = (long long)p->nx * p->ny * p->nz;
  c->nm = dgk::nmodes(p->degree);
  c->nt = dgk::ntan(p->degree);
  c->mu = p->mu;
  {
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int e = 0, off = 0; e < 3; off += n[e], ++e)
      for (int i = 0; i < n[e]; ++i)
        c->widths.push_back(p->cell_widths ? p->cell_widths[off + i] : (p->hi[e] - p->lo[e]) / n[e]);
  }
  c->p.cell_widths = nullptr;  // the caller's array is not kept
  {
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int e = 0, off = 0; e < 3; off += n[e], ++e) {
      c->w0[e] = c->widths[off];
      for (int i = 1; i < n[e]; ++i) c->uniform = c->uniform && c->widths[off + i] == c->widths[off];
    }
  }
  *out = c;
  return DG_HGKS_OK;
}

int dg_hgks_step(dg_hgks_ctx* c, double* q, double dt, int32_t nsteps, double* ckpt, int32_t ckpt_stride) {
  if (!c) return DG_HGKS_EINVAL;
  if (!q) return fail(c, DG_HGKS_EINVAL, "q is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_HGKS_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, DG_HGKS_EINVAL, "nsteps must be >= 0");
  if (ckpt && ckpt_stride < 1) return fail(c, DG_HGKS_EINVAL, "ckpt_stride must be >= 1");
  return dispatch(c->p, [&](auto tag) {
    using Tg = decltype(tag);
    return dgrt::run_step<typename Tg::T, Tg::K, Tg::NQ>(c, q, dt, nsteps, ckpt, ckpt_stride);
  });
}

int dg_hgks_step_noalloc(const dg_hgks_params* p, void* hip_stream, double* q, double dt, int32_t nsteps,
                         int32_t* nonphys) {
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (p->cell_widths) return fail(nullptr, DG_HGKS_EINVAL, "the allocation-free step takes uniform meshes only");
  if (!q) return fail(nullptr, DG_HGKS_EINVAL, "q is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, DG_HGKS_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(nullptr, DG_HGKS_EINVAL, "nsteps must be >= 0");
  const Layout lay = make_layout(*p, 0);
  if (lay.total > kScratchBytes)
    return fail(nullptr, DG_HGKS_ENOMEM,
                "the allocation-free step needs " + std::to_string(lay.total) + " bytes of scratch, above its " +
                    std::to_string(kScratchBytes) + " (use dg_hgks_init with a workspace)");
  char* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  // a context on the stack: no host allocation (no widths array on a
  // uniform mesh), the scratch as workspace
  dg_hgks_ctx c;
  c.p = *p;
  if (c.p.nq == 0) c.p.nq = c.p.degree + 1;
  c.stream = (hipStream_t)hip_stream;
  c.ws = ws;
  c.ws_bytes = kScratchBytes;
  c.lay = lay;
  c.ncell = (long long)p->nx * p->ny * p->nz;
  c.nm = dgk::nmodes(p->degree);
  c.nt = dgk::ntan(p->degree);
  c.mu = p->mu;
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int e = 0; e < 3; ++e) c.w0[e] = (p->hi[e] - p->lo[e]) / n[e];
  // the flag word keeps the previous call's value: clear it (a kernel)
  clear_flag_kernel<<<1, 64, 0, c.stream>>>((int*)(ws + lay.flag));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, DG_HGKS_EHIP, std::string("clear_flag_kernel: ") + hipGetErrorString(e));
  c.ready = true;
  rc = dispatch(c.p, [&](auto tag) {
    using Tg = decltype(tag);
    return dgrt::run_step<typename Tg::T, Tg::K, Tg::NQ>(&c, q, dt, nsteps, nullptr, 0);
  });
  if (rc) return fail(nullptr, rc, c.err);
  if (nonphys) {
    copy_flag_kernel<<<1, 64, 0, c.stream>>>((const int*)(ws + lay.flag), nonphys);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, DG_HGKS_EHIP, std::string("copy_flag_kernel: ") + hipGetErrorString(e));
  }
  return DG_HGKS_OK;
}

int dg_hgks_residual(dg_hgks_ctx* c, const double* q, double dt, double* L, double* Lt) {
  if (!c) return DG_HGKS_EINVAL;
  if (!q || !L || !Lt) return fail(c, DG_HGKS_EINVAL, "NULL pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_HGKS_EINVAL, "dt must be finite and > 0");
  return dispatch(c->p, [&](auto tag) {
    using Tg = decltype(tag);
    return dgrt::run_residual<typename Tg::T, Tg::K, Tg::NQ>(c, q, dt, L, Lt);
  });
}

int dg_hgks_adjoint(dg_hgks_ctx* c, const double* ckpt, int32_t ckpt_stride, double dt, int32_t nsteps,
                    const double* qN_bar, double* q0_bar, double* mu_bar_host) {
  if (!c) return DG_HGKS_EINVAL;
  if (!ckpt || !qN_bar || !q0_bar || !mu_bar_host) return fail(c, DG_HGKS_EINVAL, "NULL pointer");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, DG_HGKS_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(c, DG_HGKS_EINVAL, "nsteps must be >= 0");
  if (ckpt_stride < 1) return fail(c, DG_HGKS_EINVAL, "ckpt_stride must be >= 1");
  if (ckpt_stride > c->max_stride)
    return fail(c, DG_HGKS_ENOMEM, "ckpt_stride exceeds the adjoint room of the workspace");
  return dispatch(c->p, [&](auto tag) {
    using Tg = decltype(tag);
    return dgrt::run_adjoint<typename Tg::T, Tg::K, Tg::NQ>(c, ckpt, ckpt_stride, dt, nsteps, qN_bar, q0_bar,
                                                       mu_bar_host);
  });
}

int dg_hgks_set_mu(dg_hgks_ctx* c, double mu) {
  if (!c) return DG_HGKS_EINVAL;
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(c, DG_HGKS_EINVAL, "mu must be >= 0");
  c->mu = mu;
  return DG_HGKS_OK;
}

int dg_hgks_set_stream(dg_hgks_ctx* c, void* hip_stream) {
  if (!c) return DG_HGKS_EINVAL;
  c->stream = (hipStream_t)hip_stream;
  return DG_HGKS_OK;
}

int dg_hgks_check(dg_hgks_ctx* c) {
  if (!c) return DG_HGKS_EINVAL;
  int rc = ensure_ready(c);
  if (rc) return rc;
  int h = 0;
  int* f = (int*)(c->ws + c->lay.flag);
  DG_HIP(c, hipMemcpyAsync(&h, f, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DG_HIP(c, hipStreamSynchronize(c->stream));
  if (h) {
    clear_flag_kernel<<<1, 64, 0, c->stream>>>(f);
    DG_HIP(c, hipGetLastError());
    return fail(c, DG_HGKS_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or non-finite) met");
  }
  return DG_HGKS_OK;
}

int dg_hgks_point_face_flux(dg_hgks_ctx* c, const double* x, int64_t n, int32_t axis, double dt, double* F,
                            double* Ft) {
  if (!c) return DG_HGKS_EINVAL;
  if (!x || !F || !Ft || n < 0 || axis < 0 || axis > 2 || !(dt > 0.0)) return fail(c, DG_HGKS_EINVAL, "bad argument");
  if (n == 0) return DG_HGKS_OK;
  int rc = ensure_ready(c);
  if (rc) return rc;
  const Phys ph = make_phys(c, dt);
  int* flag = (int*)(c->ws + c->lay.flag);
  const unsigned nb = (unsigned)((n + 63) / 64);
  if (c->p.precision == DG_HGKS_FP32_BULK)
    DG_LAUNCH(c, 0, (point_face_kernel<float><<<nb, 64, 0, c->stream>>>(x, F, Ft, n, axis, ph, flag)));
  else
    DG_LAUNCH(c, 0, (point_face_kernel<double><<<nb, 64, 0, c->stream>>>(x, F, Ft, n, axis, ph, flag)));
  return DG_HGKS_OK;
}

int dg_hgks_point_volume_flux(dg_hgks_ctx* c, const double* x, int64_t n, double* F, double* Ft) {
  if (!c) return DG_HGKS_EINVAL;
  if (!x || !F || !Ft || n < 0) return fail(c, DG_HGKS_EINVAL, "bad argument");
  if (n == 0) return DG_HGKS_OK;
  int rc = ensure_ready(c);
  if (rc) return rc;
  const Phys ph = make_phys(c, 1.0);
  int* flag = (int*)(c->ws + c->lay.flag);
  const unsigned nb = (unsigned)((n + 63) / 64);
  if (c->p.precision == DG_HGKS_FP32_BULK)
    DG_LAUNCH(c, 1, (point_volume_kernel<float><<<nb, 64, 0, c->stream>>>(x, F, Ft, n, ph, flag)));
  else
    DG_LAUNCH(c, 1, (point_volume_kernel<double><<<nb, 64, 0, c->stream>>>(x, F, Ft, n, ph, flag)));
  return DG_HGKS_OK;
}

int dg_hgks_diagnostics(dg_hgks_ctx* c, const double* q, double* out_host, double* grad_ke) {
  if (!c) return DG_HGKS_EINVAL;
  if (!q || !out_host) return fail(c, DG_HGKS_EINVAL, "NULL pointer");
  int rc = ensure_ready(c);
  if (rc) return rc;
  const Geo g = make_geo(c);
  const long long nb = (g.ncell + kCellThreads - 1) / kCellThreads;
  double* part = (double*)(c->ws + c->lay.diag);
  double* sums = part + 2 * nb;
  const int k = c->p.degree, nq = c->p.nq;
  auto launch = [&](auto kc, auto nqc) {
    constexpr int K = decltype(kc)::value, NQ = decltype(nqc)::value;
    diag_kernel<K, NQ><<<dim3((unsigned)nb), kCellThreads, 0, c->stream>>>(q, g, part, grad_ke);
  };
  if (k == 1 && nq == 2)
    launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
  else if (k == 2 && nq == 3)
    launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
  else if (k == 2 && nq == 2)
    launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
  else if (k == 3 && nq == 4)
    launch(std::integral_constant<int, 3>{}, std::integral_constant<int, 4>{});
  else if (k == 3 && nq == 3)
    launch(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{});
  else
    return fail(c, DG_HGKS_EUNSUPPORTED, "(degree, nq) combination not compiled");
  DG_HIP(c, hipGetLastError());
  diag_reduce_kernel<<<1, 256, 0, c->stream>>>(part, nb, sums);
  DG_HIP(c, hipGetLastError());
  DG_HIP(c, hipMemcpyAsync(out_host, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  DG_HIP(c, hipStreamSynchronize(c->stream));
  return DG_HGKS_OK;
}

int dg_hgks_set_timing(dg_hgks_ctx* c, int32_t enable) {
  if (!c) return DG_HGKS_EINVAL;
  int rc = t_collect(c);
  if (rc) return rc;
  for (int i = 0; i < 5; ++i) {
    c->t_ms[i] = 0;
    c->t_n[i] = 0;
  }
  c->timing = enable != 0;
  return DG_HGKS_OK;
}

int dg_hgks_get_timing(dg_hgks_ctx* c, double* ms, int64_t* counts, int32_t n) {
  if (!c) return DG_HGKS_EINVAL;
  int rc = t_collect(c);
  if (rc) return rc;
  for (int i = 0; i < n && i < 5; ++i) {
    if (ms) ms[i] = c->t_ms[i];
    if (counts) counts[i] = c->t_n[i];
  }
  return 5;
}

const char* dg_hgks_last_error(const dg_hgks_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

const char* dg_hgks_strerror(int s) {
  switch (s) {
    case DG_HGKS_OK: return "ok";
    case DG_HGKS_EINVAL: return "invalid argument";
    case DG_HGKS_ENOMEM: return "workspace too small";
    case DG_HGKS_EHIP: return "HIP runtime error";
    case DG_HGKS_ENONPHYS: return "non-physical state";
    case DG_HGKS_EUNSUPPORTED: return "unsupported (degree, nq)";
    default: return "unknown status";
  }
}

int dg_hgks_destroy(dg_hgks_ctx* c) {
  if (!c) return DG_HGKS_EINVAL;
  for (auto& r : c->trecs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete c;
  return DG_HGKS_OK;
}

}  // extern "C"
