/*
 * libsfrde -- one ETDRK4 step of a space-fractional reaction-diffusion system
 * on an AMD MI355X (gfx950), behind a plain C ABI.
 *
 * The problem (Section 1, eq. 1):  u_t = -kappa (-Delta)^(alpha/2) u + f(u, t)
 * on a box in 2D or 3D with periodic, homogeneous Dirichlet or homogeneous
 * Neumann boundary conditions, for S coupled species.
 *
 * Space (Section 3): the compact fourth-order Laplacian A^-1 B raised to
 * alpha/2 by the matrix transfer technique (eq. MTT). It is diagonal in the
 * basis of the boundary condition's transform (discrete Hartley for periodic,
 * DST-I for Dirichlet, weighted DCT-I for Neumann), with eigenvalues
 * lambda_k = 4 s^2 / (h^2 (1 - s^2/3)) per axis, summed over the axes
 * (Sections 3.1-3.3, E16-E18, E22).
 *
 * Time (Section 4, eq. ETDRK4P13 and Alg. 1): four stages per step, each a
 * forward transform of the reaction, a diagonal multiply-and-combine with six
 * coefficient arrays of L = kappa dt Lambda^(alpha/2), an inverse transform
 * and a pointwise reaction. Two coefficient schemes: the paper's Pade-based
 * ETDRK4-P13 (default) and the exact-exponential ETDRK4 of Cox and Matthews.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Fields are device arrays [S][nz][ny][nx] (2D: [S][ny][nx], 1D: [S][nx])
 *   of the plan's dtype, x contiguous; ensemble plans (sfrde_plan_batch) put
 *   the member first, [B][S][...]. Sizes are *unknowns* per axis: N = n
 *   (periodic), n + 1 (Dirichlet), n - 1 (Neumann) intervals with spacing h.
 * - Every transform runs in hand-written kernels: axes of up to 256 points
 *   (255 periodic) on the matrix cores, periodic axes of 256, 512 and 1024
 *   points as radix-8/4 FFTs in LDS, any other axis (up to 1024 points) as a
 *   dense product in LDS; each fused with the same pointwise stages.
 * - n[0] is the x (fastest) extent, n[1] y, n[2] z; h[] in the same order.
 * - The caller owns every buffer passed in (state, checkpoints, gradients)
 *   and the stream; the library never frees caller memory. The plan owns its
 *   tables and workspace; sfrde_destroy frees them.
 * - All work is enqueued on the plan's stream. sfrde_integrate synchronizes
 *   once at its end (to report non-finite values); sfrde_backward
 *   synchronizes at its end (host scalar outputs).
 * - Return codes are SFRDE_OK (0) or a negative sfrde_status; the message
 *   for the last failure on the calling thread is sfrde_last_error().
 * - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef SFRDE_H
#define SFRDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFRDE_MAX_SPECIES 4
#define SFRDE_MAX_PARAMS 16
#define SFRDE_CKPT_HEADER_BYTES 256

typedef struct sfrde_plan_s* sfrde_plan_t;

enum sfrde_status {
  SFRDE_OK = 0,
  SFRDE_EINVAL = -1,       /* bad argument; detected before any device call */
  SFRDE_ENOMEM = -2,       /* device or host allocation failed */
  SFRDE_EDEVICE = -3,      /* a HIP runtime call failed */
  SFRDE_ENONFINITE = -4,   /* a stage value or reaction became NaN/Inf */
  SFRDE_EUNSUPPORTED = -5, /* valid request the library does not support */
  SFRDE_ESTATE = -6        /* checkpoint incompatible with the request */
};

enum sfrde_bc { SFRDE_BC_PERIODIC = 0, SFRDE_BC_DIRICHLET = 1, SFRDE_BC_NEUMANN = 2 };
enum sfrde_dtype { SFRDE_F32 = 0, SFRDE_F64 = 1 };
enum sfrde_scheme { SFRDE_SCHEME_P13 = 0, SFRDE_SCHEME_EXP = 1 };

/* Reaction terms (Section 5.2) and their parameter vectors p[]:
 *   LINEAR            p = (g_0..g_{S-1})         f_s = g_s u_s   (any S <= 4)
 *   FHN               p = (mu, eps, beta, gamma, delta)
 *                     f_u = u(1-u)(u-mu) - v,  f_v = eps(beta u - gamma v - delta)
 *   GRAY_SCOTT        p = (F, K)
 *                     f_u = -u v^2 + F(1-u),   f_v = u v^2 - (F+K) v
 *   SCHNAKENBERG      p = (gamma, a, b)
 *                     f_u = gamma(a - u + u^2 v),  f_v = gamma(b - u^2 v)
 *   GIERER_MEINHARDT  p = (rho, mu_u, sigma_u, sigma_v, mu_v)
 *                     f_u = rho - mu_u u + sigma_u u^2/v,  f_v = sigma_v u^2 - mu_v v
 * FHN .. GIERER_MEINHARDT need S = 2.
 * Manufactured-solution problems of Section 5.1 (S = 1, no parameters: the
 * source is built from the plan's kappa and alpha; x_j is the node position
 * on [0, 1], x_j = j h for periodic and Neumann, (j + 1) h for Dirichlet):
 *   HUXLEY_MMS   Example 2, 2D, periodic or Neumann:
 *                f = u(1-u)(u-1) + s(x, y, t), with s making
 *                u = t^alpha cos^3(2 pi x) cos^3(2 pi y) the exact solution
 *   FISHER_MMS   Example 1, 1D, Dirichlet:
 *                f = u - u^2 + s(x, t), with s making
 *                u = e^-t sin^3(2 pi x) the exact solution
 * The sources are evaluated in FP64 at each stage's time. sfrde_backward
 * returns u0 gradients for them; kappa, alpha and parameter gradients are
 * SFRDE_EUNSUPPORTED (the sources depend on kappa and alpha). */
enum sfrde_reaction {
  SFRDE_RXN_LINEAR = 0,
  SFRDE_RXN_FHN = 1,
  SFRDE_RXN_GRAY_SCOTT = 2,
  SFRDE_RXN_SCHNAKENBERG = 3,
  SFRDE_RXN_GIERER_MEINHARDT = 4,
  SFRDE_RXN_HUXLEY_MMS = 5,
  SFRDE_RXN_FISHER_MMS = 6
};

/* Create a plan (Sections 3-4; Alg. 1 precompute).
 *   out       receives the plan handle (host pointer, required)
 *   ndim      1, 2 or 3 (a 1D plan runs as a 2D one whose second axis has
 *             one point, eigenvalue 0 and the identity transform)
 *   n[ndim]   unknowns per axis, x first; each >= 2, each <= 1024
 *   bc        enum sfrde_bc, the same on every axis
 *   h[ndim]   mesh width per axis (> 0)
 *   nspecies  S, 1..4
 *   alpha[S]  fractional order per species, 0 < alpha <= 2 (paper: 1 < alpha <= 2)
 *   kappa[S]  diffusion coefficient per species, >= 0
 *   dt        time step tau > 0
 *   reaction  enum sfrde_reaction; nparams must match it, params[nparams]
 *   dtype     SFRDE_F32 or SFRDE_F64: the type of fields and of the
 *             transforms; eigenvalues and coefficients are always computed
 *             in FP64 and stored in dtype
 *   scheme    SFRDE_SCHEME_P13 (the paper's) or SFRDE_SCHEME_EXP
 *   hip_stream  hipStream_t to enqueue on (NULL: the default stream)
 * Errors: EINVAL for any argument outside the ranges above (no device call is
 * made), ENOMEM/EDEVICE from the device. */
int sfrde_plan(sfrde_plan_t* out, int32_t ndim, const int64_t* n, int32_t bc,
               const double* h, int32_t nspecies, const double* alpha,
               const double* kappa, double dt, int32_t reaction, int32_t nparams,
               const double* params, int32_t dtype, int32_t scheme, void* hip_stream);

/* Ensemble plan: `batch` members (1..65535) of one grid, boundary
 * condition, species count, time step, reaction kind, dtype and scheme, each
 * with its own orders, diffusion coefficients and reaction parameters, all
 * advanced by the same launches (the paper's parameter sweeps, Section 5.2).
 *   alpha, kappa  [batch][nspecies]      params  [batch][nparams]
 * Every other argument as in sfrde_plan, which is this call with batch = 1.
 * With such a plan, state (and grad_uT, grad_u0) are [batch][S][...] device
 * arrays; checkpoints hold every member; sfrde_backward's grad_kappa and
 * grad_alpha are [batch][S] and grad_params [batch][nparams]. Members are
 * independent: each computes what a plan of its own computes. */
int sfrde_plan_batch(sfrde_plan_t* out, int32_t batch, int32_t ndim, const int64_t* n,
                     int32_t bc, const double* h, int32_t nspecies, const double* alpha,
                     const double* kappa, double dt, int32_t reaction, int32_t nparams,
                     const double* params, int32_t dtype, int32_t scheme, void* hip_stream);

/* One step from time t (eq. ETDRK4P13): state <- u(t + dt), in place.
 * state: device [S][...] of the plan's dtype. Same as sfrde_integrate with
 * nsteps = 1 and no checkpoints. */
int sfrde_step(sfrde_plan_t plan, void* state, double t);

/* nsteps steps from t0, in place on state (Alg. 1 time loop). If ckpt_every
 * > 0 and ckpt != NULL, the spectral state before steps 0, K, 2K, ...
 * (K = ckpt_every) is stored in ckpt (device, sfrde_ckpt_bytes() bytes),
 * which sfrde_backward and sfrde_resume read. nsteps = 0 leaves state
 * untouched. Returns SFRDE_ENONFINITE (state then holds the non-finite
 * result) if any stage produced NaN/Inf. */
int sfrde_integrate(sfrde_plan_t plan, void* state, int64_t nsteps, double t0,
                    int64_t ckpt_every, void* ckpt);

/* Bytes of the checkpoint buffer for (nsteps, ckpt_every): a
 * SFRDE_CKPT_HEADER_BYTES header plus ceil(nsteps/ckpt_every) spectral
 * states. Negative sfrde_status on bad arguments. */
int64_t sfrde_ckpt_bytes(sfrde_plan_t plan, int64_t nsteps, int64_t ckpt_every);

/* Continue from checkpoint slot `slot` (the spectral state before step
 * slot*K of the run that wrote ckpt): runs nsteps steps from t0 into state.
 * Bitwise identical to the original run's continuation. ckpt_out as in
 * sfrde_integrate (may be NULL). The checkpoint header records the writer's
 * species count, dtype, dimension, boundary condition, ensemble size and
 * unknowns per axis; ESTATE if any differs from this plan's (another shape
 * or boundary condition is another spectral basis) or slot is past the last
 * stored state. */
int sfrde_resume(sfrde_plan_t plan, const void* ckpt, int64_t slot, void* state,
                 int64_t nsteps, double t0, int64_t ckpt_every, void* ckpt_out);

/* Discrete adjoint of nsteps steps (the reverse sweep of eq. ETDRK4P13 with
 * transposed transforms, the same diagonal coefficients and the reaction
 * Jacobian transposed). ckpt must come from sfrde_integrate(nsteps, t0,
 * ckpt_every) with this plan's shape, dtype and species count. Segments of
 * ckpt_every steps are recomputed from their checkpoint (memory: about
 * 9 * ckpt_every fields of workspace when kappa or alpha gradients are asked,
 * 4 * ckpt_every when not).
 *   grad_uT     device [S][...] dtype: dLoss/du(T)
 *   grad_u0     device [S][...] dtype: receives dLoss/du(0) (NULL: skip)
 *   grad_kappa  host double[S] (NULL: skip)   dLoss/dkappa_s
 *   grad_alpha  host double[S] (NULL: skip)   dLoss/dalpha_s
 *   grad_params host double[nparams] (NULL: skip)
 * Errors: ESTATE if the checkpoint does not match (header fields as for
 * sfrde_resume, or another ckpt_every, or fewer than nsteps steps). */
int sfrde_backward(sfrde_plan_t plan, const void* ckpt, int64_t nsteps,
                   int64_t ckpt_every, double t0, const void* grad_uT, void* grad_u0,
                   double* grad_kappa, double* grad_alpha, double* grad_params);

/* Allocation-free variant of sfrde_backward, for callers that cannot
 * allocate device memory at call time (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). Same arguments, results
 * and errors as sfrde_backward, computed by the same kernels; the backward
 * buffers (adjoint fields, the segment store of ckpt_every steps, gradient
 * partials) live in one static device array of SFRDE_NOALLOC_SCRATCH_BYTES
 * per GPU, which the library holds from its first plan on that GPU until the
 * process ends, instead of plan memory allocated on first use. The call
 * makes no device allocation and frees nothing.
 * Limits: the buffers need about (5 + 9 * min(ckpt_every, nsteps)) fields
 * of [B][S][...] dtype (plus one FP64 field and six dtype fields when the
 * kappa/alpha gradients take the per-point path); a request that does not
 * fit returns SFRDE_EINVAL before any device work. Every call on one GPU uses
 * the same array: calls that overlap in time on one GPU (other threads,
 * other streams) race and must be serialized by the caller. Nothing is
 * carried over between calls (each call initializes what it reads). */
#define SFRDE_NOALLOC_SCRATCH_BYTES (128LL * 1024 * 1024)
int sfrde_backward_noalloc(sfrde_plan_t plan, const void* ckpt, int64_t nsteps,
                           int64_t ckpt_every, double t0, const void* grad_uT, void* grad_u0,
                           double* grad_kappa, double* grad_alpha, double* grad_params);

/* Free the plan and everything it owns (waits for its stream first). */
int sfrde_destroy(sfrde_plan_t plan);

/* Message for the last non-OK return on this thread ("" if none). */
const char* sfrde_last_error(void);

/* Device bytes owned by the plan (tables and workspace) right now. */
int64_t sfrde_workspace_bytes(sfrde_plan_t plan);

/* Measurement. sfrde_profile(plan, k) with k >= 1 clears the record, makes
 * events for k launches up front, and brackets every later kernel launch of
 * the plan with HIP events on its stream (more are made if needed);
 * sfrde_profile(plan, 0) stops recording. sfrde_profile_read synchronizes
 * the stream and returns, per kernel class, the summed event time in ms and
 * the launch count (arrays of SFRDE_K_COUNT entries). */
enum sfrde_kernel_class {
  SFRDE_K_X = 0,     /* inverse-x, reaction, forward-x */
  SFRDE_K_Y = 1,     /* single-axis transform passes */
  SFRDE_K_Z = 2,     /* forward, stage combine, inverse along the last axis */
  SFRDE_K_XADJ = 3,  /* adjoint X */
  SFRDE_K_ZADJ = 4,  /* adjoint Z */
  SFRDE_K_OTHER = 5,
  SFRDE_K_COUNT = 6
};
int sfrde_profile(sfrde_plan_t plan, int32_t enable);
int sfrde_profile_read(sfrde_plan_t plan, double* ms, int64_t* launches);

/* Host-only helpers (no device needed), for checks of the plan's tables:
 * the per-axis eigenvalues (Section 3.1) in the library's spectral order, and
 * the six coefficients (R, Q, phi, phi1, phi2, phi3) at one L >= 0 or their
 * derivatives d/dL (deriv != 0). */
int sfrde_axis_eigenvalues(int32_t bc, int64_t n, double h, double* out);
int sfrde_eval_coefficients(int32_t scheme, double L, double dt, int32_t deriv,
                            double* out6);

/* Linear stability (Section 4.2.2, eq. Eq41). The test equation
 * u' + c u = gamma u, with y = -c tau (real, <= 0) and x = gamma tau
 * (complex), is advanced one step by the scheme's four stages, with its
 * coefficients at L = -y; the ratio u^{k+1}/u^k is the amplification factor
 * r(x, y), a quartic in x. Both calls run one GPU thread per point in FP64,
 * are enqueued on hip_stream (NULL: the default stream) and return without
 * waiting for it. Points with y > 0 or non-finite inputs give NaN.
 * Errors: EINVAL for an unknown scheme, sizes out of range, or NULL arrays
 * with a non-zero size; EDEVICE if the launch fails.
 *
 * sfrde_amplification: r(x_i, y_i) for i < count.
 *   x  device double[count][2] (real, imaginary)
 *   y  device double[count]
 *   r  device double[count][2], written
 *
 * sfrde_stability_boundary: points of the |r| = 1 contours. For each y_i
 * (i < ny) and theta_k = 2 pi k / ntheta (k < ntheta), the four complex x
 * with r(x, y_i) = e^{i theta_k} (Durand-Kerner iteration on the quartic).
 *   y      device double[ny]
 *   roots  device double[ny][ntheta][4][2], written; the four roots of one
 *          (i, k) come in no particular order
 *   poly   device double[ny][5], written with c_0..c_4 of
 *          r(x, y_i) = sum_k c_k x^k; may be NULL */
int sfrde_amplification(int32_t scheme, int64_t count, const double* x, const double* y,
                        double* r, void* hip_stream);
int sfrde_stability_boundary(int32_t scheme, int64_t ny, const double* y, int64_t ntheta,
                             double* roots, double* poly, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
