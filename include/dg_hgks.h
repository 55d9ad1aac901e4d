/*
 * dg_hgks.h -- C-ABI of the MI355X (gfx950) implementation of one two-stage
 * fourth-order (S2O4) time step of the modal discontinuous Galerkin
 * gas-kinetic scheme (DG-HGKS) of Wang & Pan, "Three-dimensional
 * discontinuous Galerkin based high-order gas-kinetic scheme and GPU
 * implementation", arXiv 2202.13821.
 *
 * Problem (Section 3): on a periodic Cartesian box [lo, hi]^3 split into
 * nx*ny*nz cells (equal, or a separable non-uniform mesh given by per-axis
 * cell widths, as in the mapped meshes of Section 5.1), the conservative variables Q = (rho, rho U, rho V,
 * rho W, rho E) are expanded per cell in the P_k Legendre basis (Eq.
 * (expansion)); the ODE system dQ/dt = M^{-1} R(Q) = L(Q) of Eqs. (DG2) and
 * (operator) is integrated with Eq. (two-stage).  Face fluxes follow Eq.
 * (flux) (second-order BGK solution with equilibrium state g0, microscopic
 * slopes a, A from the compatibility conditions), volume fluxes Eq. (flux-2),
 * collision time tau = mu / p, and both are evaluated at Gauss points (Eqs.
 * (surface), (volume)) and fitted linearly in time over [0, dt] and
 * [0, dt/2] (Eq. (expansion-1)).  Pr != 1 adds (1/Pr - 1) times the heat flux
 * of the first-order non-equilibrium part to the energy flux.
 *
 * Layout of every coefficient array (device memory, float64, C order):
 *     q[var][mode][z][y][x],  var = 0..4, mode = 0..nmodes(degree)-1,
 * modes ordered by total degree s = 0..k, then nx from s down to 0, then ny
 * from s - nx down to 0 (P1: 000 100 010 001; P2 adds 200 110 101 020 011 002).
 * Mode 0 is the cell average.  Cell (i, j, k) covers
 * [lo + i dx, lo + (i+1) dx] x ... with dx = (hi - lo) / n per axis, or on a
 * non-uniform mesh [lo + w_0 + ... + w_{i-1}, ... + w_i] x ... with the
 * widths w of dg_hgks_params.cell_widths.
 *
 * Ownership: the caller owns every device buffer (coefficients, checkpoints,
 * adjoint seeds and outputs, workspace); the library never allocates or frees
 * device memory (dg_hgks_step_noalloc works in a fixed device array that the
 * library's code object holds on each GPU).  The context owns only host state.  Calls are asynchronous on
 * the stream given to dg_hgks_init unless stated otherwise; they are not
 * thread-safe per context.  No C++ exception crosses this boundary: every call
 * returns a status code (0 on success, negative on error) and
 * dg_hgks_last_error() holds the message of the last failure.
 */
#ifndef DG_HGKS_H
#define DG_HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define DG_HGKS_OK 0
#define DG_HGKS_EINVAL (-1)       /* invalid argument (value or NULL pointer) */
#define DG_HGKS_ENOMEM (-2)       /* workspace smaller than dg_hgks_workspace_bytes */
#define DG_HGKS_EHIP (-3)         /* HIP runtime error; message in dg_hgks_last_error */
#define DG_HGKS_ENONPHYS (-4)     /* rho <= 0, p <= 0 or a non-finite value was met */
#define DG_HGKS_EUNSUPPORTED (-5) /* (degree, nq) combination not compiled */

#define DG_HGKS_FP64 0      /* every flux and projection in float64 */
#define DG_HGKS_FP32_BULK 1 /* fluxes (including the combination of the
                               face-flux moments with the time-integral
                               coefficients) and projections in float32; stage
                               accumulation of the coefficients and the
                               exp(-dt/tau) time-integral coefficients in float64 */

typedef struct dg_hgks_params {
  uint32_t struct_size; /* sizeof(dg_hgks_params) */
  int32_t nx, ny, nz;   /* cells per axis, >= 1 */
  double lo[3], hi[3];  /* periodic box, hi > lo */
  int32_t degree;       /* k of the P_k space: 1, 2 or 3 */
  int32_t nq;           /* Gauss points per direction; 0 -> degree + 1.
                           Compiled pairs (degree, nq): (1,2) (2,3) (2,2)
                           (3,4) (3,3); nq = degree is the paper's rule */
  double gamma;         /* specific heat ratio > 1; K = (5 - 3 gamma)/(gamma - 1) */
  double mu;            /* dynamic viscosity >= 0, tau = mu / p */
  double prandtl;       /* Prandtl number > 0 */
  int32_t precision;    /* DG_HGKS_FP64 or DG_HGKS_FP32_BULK */
  int32_t reserved;
  const double* cell_widths; /* NULL: uniform cells (hi - lo) / n.  Otherwise a
                           host array of nx + ny + nz cell widths (the x widths,
                           then y, then z) of a separable non-uniform mesh, as
                           in Section 5.1's mapped meshes: every width finite and
                           > 0, each axis summing to hi - lo within 1e-10
                           relative.  Copied by dg_hgks_init (the caller may free
                           it afterwards) and uploaded to the workspace with the
                           first launch. */
} dg_hgks_params;

typedef struct dg_hgks_ctx dg_hgks_ctx;

/* Number of modes of P_k, (k+1)(k+2)(k+3)/6; -1 if degree is not 1, 2 or 3. */
int64_t dg_hgks_nmodes(int32_t degree);

/* Bytes of device workspace for these parameters.  max_stride > 0 adds room
 * for adjoint segments of up to max_stride steps (dg_hgks_adjoint); 0 for a
 * forward-only context.  Returns 0 for invalid parameters. */
size_t dg_hgks_workspace_bytes(const dg_hgks_params* p, int32_t max_stride);

/* Validate p, record the HIP stream (hipStream_t, NULL = default stream) and
 * the caller's device workspace (256-byte aligned, >= workspace_bytes).  No
 * kernel is launched and no memory is allocated.  On success *out receives a
 * new context.  Errors: EINVAL, ENOMEM, EUNSUPPORTED. */
int dg_hgks_init(const dg_hgks_params* p, void* hip_stream, void* workspace, size_t workspace_bytes,
                 dg_hgks_ctx** out);

/* Advance q (device, float64, layout above, in/out) by nsteps S2O4 steps of
 * size dt (Eq. (two-stage); the second stage at t* uses the windows [0, dt]
 * and [0, dt/2] from t*).  If ckpt != NULL, before every step s with
 * s % ckpt_stride == 0 the state Q^s is copied to slot s / ckpt_stride of
 * ckpt (device, ceil(nsteps/ckpt_stride) states of the same layout).
 * Asynchronous.  Errors: EINVAL (dt <= 0 or non-finite, nsteps < 0, NULL q,
 * ckpt_stride < 1 with ckpt), EHIP. */
int dg_hgks_step(dg_hgks_ctx* ctx, double* q, double dt, int32_t nsteps, double* ckpt, int32_t ckpt_stride);

/* dg_hgks_step without a context or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): advances q (device, float64, layout above,
 * in/out) by nsteps steps of size dt with the parameters p (uniform meshes
 * only: p->cell_widths must be NULL) on the HIP stream hip_stream, using the
 * same kernels as dg_hgks_step.  Its buffers live in a static device array of
 * 96 MiB that the library holds on each GPU it runs on until the process
 * ends (enough for 32^3 cells at P2 in both precisions); parameters that
 * need more (dg_hgks_workspace_bytes(p, 0) > 96 MiB) fail with ENOMEM.
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (two streams, two threads) race and give undefined results.  The
 * device must be current.  If nonphys is not NULL (device int32), it
 * receives 1 if the call met rho <= 0, p <= 0 or a non-finite state, else 0.
 * Asynchronous; allocates nothing, host or device (errors excepted).  Errors
 * (message in dg_hgks_last_error(NULL)): EINVAL, ENOMEM, EUNSUPPORTED, EHIP. */
int dg_hgks_step_noalloc(const dg_hgks_params* p, void* hip_stream, double* q, double dt, int32_t nsteps,
                         int32_t* nonphys);

/* The operator of Eqs. (operator), (surface), (volume) at q: L = M^{-1} R(Q)
 * and L_t = M^{-1} R_t(Q) (the time derivative from the linear-in-time
 * fit over [0, dt], [0, dt/2]).  q, L, Lt: device float64, layout above.
 * Asynchronous.  Same kernels as one stage of dg_hgks_step. */
int dg_hgks_residual(dg_hgks_ctx* ctx, const double* q, double dt, double* L, double* Lt);

/* Reverse-mode derivative of nsteps steps (hand-written adjoint of the S2O4
 * step, not in the paper): given the cotangent qN_bar = dJ/dQ^N (device) of
 * a scalar J(Q^N), writes q0_bar = dJ/dQ^0 (device, may alias qN_bar) and
 * *mu_bar_host = dJ/dmu (host).  ckpt holds the states written by
 * dg_hgks_step(..., ckpt, ckpt_stride) from the same Q^0, dt and mu; each
 * segment of ckpt_stride steps is recomputed from its checkpoint (needs
 * max_stride >= ckpt_stride at init).  Synchronises the stream.
 * Errors: EINVAL, ENOMEM (stride above max_stride), EHIP, ENONPHYS. */
int dg_hgks_adjoint(dg_hgks_ctx* ctx, const double* ckpt, int32_t ckpt_stride, double dt, int32_t nsteps,
                    const double* qN_bar, double* q0_bar, double* mu_bar_host);

/* Change mu (>= 0) for later calls.  Errors: EINVAL. */
int dg_hgks_set_mu(dg_hgks_ctx* ctx, double mu);

/* Change the HIP stream used by later calls. */
int dg_hgks_set_stream(dg_hgks_ctx* ctx, void* hip_stream);

/* Synchronise the stream; return ENONPHYS if any flux evaluation since the
 * last check met rho <= 0, p <= 0 or a non-finite state (the flag is then
 * cleared), else OK.  Errors: EHIP. */
int dg_hgks_check(dg_hgks_ctx* ctx);

/* Point-flux diagnostics (same device functions as the step kernels, in the
 * context's precision).  face: x[n][40] = (Q_L, dQ_L/dx_e (3x5), Q_R,
 * dQ_R/dx_e (3x5)) in the global frame, face normal axis `axis` (0..2),
 * out F[n][5], Ft[n][5] (Eq. (flux) + time fit with the context's mu and the
 * given dt).  volume: x[n][20] = (Q, dQ/dx_e), out F[n][3][5], Ft[n][3][5]
 * (Eq. (flux-2)).  All pointers are device float64.  Asynchronous. */
int dg_hgks_point_face_flux(dg_hgks_ctx* ctx, const double* x, int64_t n, int32_t axis, double dt, double* F,
                            double* Ft);
int dg_hgks_point_volume_flux(dg_hgks_ctx* ctx, const double* x, int64_t n, double* F, double* Ft);

/* Diagnostics of a state q (device float64, layout above) on the volume Gauss
 * rule, the Taylor-Green quantities of Section 5.3 (FP64 in both precision
 * modes): out_host[0] = kinetic energy sum_K |K| sum_q w_q |rho U|^2/(2 rho),
 * out_host[1] = enstrophy sum_K |K| sum_q w_q |curl U|^2/2 (U = rho U / rho,
 * w_q the Gauss weights normalised to sum 1 per cell).  If grad_ke is not
 * NULL it receives dE_k/dq (device float64, layout of q; zero for rho E), the
 * seed of dg_hgks_adjoint for the final-kinetic-energy objective.  The sums
 * are reduced in a fixed order (deterministic).  Synchronises the stream.
 * Errors: EINVAL (NULL q or out_host), EHIP. */
int dg_hgks_diagnostics(dg_hgks_ctx* ctx, const double* q, double* out_host, double* grad_ke);

/* Per-kernel timing with HIP events on the context's stream.  enable != 0
 * starts recording (clearing earlier records); get_timing synchronises and
 * writes, for up to n kernel classes, the summed milliseconds and launch
 * counts: class 0 face, 1 volume + update, 2 precision copy, 3 adjoint face,
 * 4 adjoint volume.  Returns the number of classes. */
int dg_hgks_set_timing(dg_hgks_ctx* ctx, int32_t enable);
int dg_hgks_get_timing(dg_hgks_ctx* ctx, double* ms, int64_t* counts, int32_t n);

/* Message of the last failed call on ctx (or of the last failed init when
 * ctx is NULL); static text for a status code. */
const char* dg_hgks_last_error(const dg_hgks_ctx* ctx);
const char* dg_hgks_strerror(int status);

/* Free the host state of ctx (no device memory is touched). */
int dg_hgks_destroy(dg_hgks_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DG_HGKS_H */
