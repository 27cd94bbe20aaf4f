/*
 * tt.h -- C ABI of the MI355X tensor-train S_N step-then-truncate library.
 *
 * The library advances the gray specific intensity of the time-dependent
 * thermal radiation transport equation stored as a three-core tensor train
 *     I_{i l p} = X_i Theta_l Phi_p                  (paper Sec. 4.1,
 *                                                     eq. tensor_decomp)
 * X: N_s x r1 (all spatial cells grouped into one mode), Theta:
 * r1 x N_theta x r2, Phi: r2 x N_phi.  One step (tt_step) applies the
 * explicit transport operator in TT form with the upwind or the Rusanov
 * flux (Sec. 3.1 eqs. lhs, upwind, rusanov_flux_toro; Sec. 4.3), the
 * backward-Euler absorption/emission/scattering split (Sec. 3.2 eqs.
 * couple_a/couple_b, Sec. 4.4), sums all terms by core concatenation
 * (Sec. 4.1 Addition) and rounds the sum with Gram-SVD (Sec. 4.2, App. A
 * Algorithm 1 with the truncate step of App. A.2).
 *
 * Conventions for every entry point
 *  - Return value: TT_OK (0) or a negative tt_status; nothing throws across
 *    the ABI.  tt_last_error(ctx) returns a message owned by ctx (by the
 *    calling thread when ctx is NULL); it stays valid until the next call.
 *  - Pointers documented "host" are read (or written) during the call only;
 *    the library copies what it keeps.  Pointers documented "device" are
 *    caller-owned device memory that must stay valid as stated.
 *  - All device work is ordered on the caller's HIP stream given to
 *    tt_create; each call returns after its work is complete (one stream
 *    synchronisation), except where stated.
 *  - All arrays are row-major float64.  Host core layouts:
 *      X  [N_s][r1],  Th [r1][N_theta][r2],  Ph [r2][N_phi],
 *    with spatial index i = ix + nx*(iy + ny*iz).
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - After TT_ERR_NUMERIC (non-finite values, Newton or eigensolver
 *    failure) the context is poisoned: stepping returns TT_ERR_STATE until
 *    tt_set_cores installs a new state.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TT_OK = 0,
  TT_ERR_INVALID_ARG = -1, /* bad config, size or pointer                    */
  TT_ERR_DEVICE = -2,      /* a HIP call failed                              */
  TT_ERR_OOM = -3,         /* workspace smaller than tt_workspace_bytes()    */
  TT_ERR_NUMERIC = -4,     /* non-finite state, Newton/eigensolver failure   */
  TT_ERR_STATE = -5        /* context poisoned, or call out of order         */
} tt_status;

/* Boundary condition per face (Sec. 4.5): vacuum = zero ghost cells;
 * periodic = wrapped ghost cells (must be set on both faces of an axis);
 * inflow = Dirichlet ghost values given as rank-1 terms (tt_inflow);
 * outflow = the ghost cell copies the adjacent interior cell. */
enum { TT_BC_VACUUM = 0, TT_BC_PERIODIC = 1, TT_BC_INFLOW = 2, TT_BC_OUTFLOW = 3 };
/* Interface flux of the transport operator (Sec. 3.1, Sec. 4.3).
 * UPWIND: eq. upwind, one stencil block per axis and direction sign.
 * RUSANOV: eq. rusanov_flux_toro with the wavespeed S+ = s_plus * c: a
 * central-difference block and a diffusion block per axis (the latter
 * omitted when s_plus == 0, the thick-medium choice of Sec. 5.3); a
 * Dirichlet face then adds two rank-1 terms per tt_inflow entry.
 * HLL: eq. hll with the asymptotic wavespeeds of Sec. 3.1 and the local
 * optical depth of eq. tauc (tau_c at face i+1/2 = 2 hll_beta dx /
 * (1/(rho k)_i + 1/(rho k)_{i+1}), k = kappa + kappa_s; a non-periodic
 * boundary face takes the interior cell's rho k on both sides; the series
 * forms below hll_tau_threshold).  With piecewise-constant states the face
 * flux is c n (alpha U_L + beta U_R), alpha + beta = 1, per sign of n: one
 * variable-weight stencil block per axis and sign (B = 1 + 2 dim) and two
 * rank-1 terms per tt_inflow entry.  The weights are formed on the device
 * at tt_create and again by tt_set_kappa and tt_set_scattering. */
enum { TT_FLUX_UPWIND = 0, TT_FLUX_RUSANOV = 1, TT_FLUX_HLL = 2 };
/* Arithmetic of the N_s-long contractions and Gram formation. */
enum { TT_FP64 = 0, TT_FP32_MIXED = 1 };
/* ONCE: one rounding per step, after the transport and source terms are
 * summed.  TWICE: the schedule of Sec. 4.2 Rounding -- the transport sum is
 * rounded, the source update is applied to that rounded state, and the
 * result is rounded again (two roundings per step, both with tol/rmax; in
 * TT_RANK_REPLAY mode each rounding takes the next schedule entry). */
enum { TT_ROUND_ONCE = 0, TT_ROUND_TWICE = 1 };
/* FROZEN: temperature fixed (constant emission); COUPLED: backward-Euler
 * material temperature with energy-conserving update (Sec. 3.2). */
enum { TT_MAT_FROZEN = 0, TT_MAT_COUPLED = 1 };
/* AUTO: ranks from the tolerance rule; REPLAY: ranks taken from the
 * schedule set by tt_set_rank_schedule (for finite differences / adjoint). */
enum { TT_RANK_AUTO = 0, TT_RANK_REPLAY = 1 };

typedef struct {
  int32_t dim;                 /* 2 or 3                                      */
  int32_t nx, ny, nz;          /* cells per axis; nz = 1 when dim == 2        */
  int32_t ntheta, nphi;        /* ordinates: ntheta even, nphi % 4 == 0       */
  double lx, ly, lz;           /* domain extents; cell size = l / n           */
  double c, a_r;               /* speed of light, radiation constant          */
  double cfl;                  /* dt = cfl * min cell size / c when dt <= 0   */
  double dt;                   /* explicit time step if > 0                   */
  double tol;                  /* relative Frobenius rounding tolerance       */
  int32_t rmax;                /* rank cap; <= 0: none (mode sizes bound)     */
  int32_t bc_lo[3], bc_hi[3];  /* TT_BC_* per axis (index 2 unused in 2-D)    */
  int32_t precision;           /* TT_FP64 / TT_FP32_MIXED                     */
  int32_t schedule;            /* TT_ROUND_ONCE / TT_ROUND_TWICE              */
  int32_t material;            /* TT_MAT_FROZEN / TT_MAT_COUPLED              */
  int32_t rank_mode;           /* TT_RANK_AUTO / TT_RANK_REPLAY               */
  int32_t ckpt_every;          /* > 0: tt_step records a tape for tt_grad     */
  int32_t max_steps;           /* capacity of the rank history and the tape   */
  int32_t r1_cap, r2_cap;      /* 0: derived from rmax and the mode sizes     */
  int32_t flux;                /* TT_FLUX_UPWIND / _RUSANOV / _HLL            */
  double s_plus;               /* Rusanov wavespeed S+ in units of c (>= 0)   */
  double hll_beta;             /* HLL: optical-depth factor beta (> 0)        */
  double hll_tau_threshold;    /* HLL: series threshold of tau_c (>= 0)       */
} tt_config;

/* One Dirichlet inflow term: the ghost value on `face` is
 * face_w[q] * theta_w[l] * phi_w[p] (host arrays, copied at tt_create).
 * face: 0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi, 4 z-lo, 5 z-hi.  face_w is indexed
 * by the face's own cell index: iy + ny*iz (x faces), ix + nx*iz (y faces),
 * ix + nx*iy (z faces).  The face's bc must be TT_BC_INFLOW. */
typedef struct {
  int32_t face;
  const double *face_w, *theta_w, *phi_w;
} tt_inflow;

typedef struct tt_ctx tt_ctx;

/* Bytes of device workspace a context needs for `cfg` with `n_inflow`
 * inflow terms (0 if cfg is invalid; see tt_last_error(NULL)).  The
 * concatenated rank capacity max(B r1_cap, B r2_cap) + n_bc + 1 must not
 * exceed 1024, where B is the number of transport blocks (1 + 2 dim; 1 + dim
 * for Rusanov with s_plus == 0) and n_bc the number of rank-1 inflow terms
 * (n_inflow, or 2 n_inflow for Rusanov with s_plus > 0).
 * The tape (ckpt_every > 0) covers the upwind flux with vacuum, periodic or
 * inflow faces, frozen material, no scattering and TT_ROUND_ONCE; other
 * combinations are rejected with TT_ERR_INVALID_ARG. */
size_t tt_workspace_bytes(const tt_config* cfg, int32_t n_inflow);

/* Create a context.
 *  kappa, rho, cv, T0: host, N_s each (absorption opacity kappa_a, density,
 *      specific heat, initial temperature); rho, cv may be NULL (-> 1).
 *  inflow[n_inflow]: host inflow terms (may be NULL when n_inflow == 0).
 *  X0, Th0, Ph0: host initial cores with ranks r1, r2 (<= the rank caps).
 *  dev_workspace: device, >= tt_workspace_bytes(cfg, n_inflow) bytes,
 *      caller-owned, must outlive the context; the library allocates no
 *      other device memory.
 *  hip_stream: a hipStream_t (NULL = default stream), caller-owned.
 *  out: receives the context.
 * Host inputs are validated before any device work: every value finite,
 * kappa >= 0, rho > 0, cv > 0, T0 >= 0; inflow weights finite.
 * Errors: TT_ERR_INVALID_ARG (config, ranks, non-finite or out-of-range
 * input), TT_ERR_OOM (ws_bytes too small), TT_ERR_DEVICE. */
tt_status tt_create(const tt_config* cfg, const double* kappa, const double* rho,
                    const double* cv, const double* T0, const tt_inflow* inflow,
                    int32_t n_inflow, const double* X0, const double* Th0,
                    const double* Ph0, int32_t r1, int32_t r2, void* dev_workspace,
                    size_t ws_bytes, void* hip_stream, tt_ctx** out);

/* Advance nsteps time steps (Sec. 3-4; one step = transport operator apply,
 * absorption/emission/scattering, TT sum, Gram-SVD rounding (twice with
 * TT_ROUND_TWICE), material update).  Ranks stay on the device; the call
 * synchronises once at the end, then checks that the cores (X, Theta, Phi
 * at their live ranks) and the temperature are finite.  With ckpt_every > 0
 * the steps are recorded for tt_grad (at most max_steps).
 * Errors: TT_ERR_STATE (poisoned / tape full), TT_ERR_NUMERIC (non-finite
 * state, Newton failure, eigensolver failure, or a grid barrier of the
 * large-order eigensolvers that timed out). */
tt_status tt_step(tt_ctx* ctx, int32_t nsteps);

/* Round the stored state once (App. A Algorithm 1, Gram-SVD truncate of
 * App. A.2) with tolerance `tol` and cap `rmax` (<= 0: the context's cap
 * capacity).  ranks_out (host, 2 ints, may be NULL) receives (r1, r2).
 * A rounding is not a recorded step: on a context with recorded steps the
 * tape no longer describes the state, and tt_grad returns TT_ERR_STATE
 * until tt_set_cores. */
tt_status tt_round(tt_ctx* ctx, double tol, int32_t rmax, int32_t ranks_out[2]);

/* Randomized rounding of the stored state to the fixed target ranks
 * (k1, k2) (App. A.3, eqs. randfinal and randprojection), bond 1 then
 * bond 2.  omega1: device, (N_theta N_phi) x k1 row-major, row l N_phi + p
 * for ordinate (l, p); omega2: device, N_phi x k2 row-major.  They are the
 * Gaussian test matrices the caller draws (read only, caller-owned); their
 * column counts are the target ranks.  Each bond sketches its right factor
 * (W = B^T Omega), takes an orthonormal basis Q of A W (shifted
 * CholeskyQR3: k x k Grams and tall products on the FP64 MFMA kernels) and
 * carries Q^T A into the next core; X' and Theta' come out with
 * orthonormal columns.  TT_FP64 contexts only; needs
 * 1 <= k1 <= min(r1, N_theta N_phi) and 1 <= k2 <= min(r2, N_phi, k1 N_theta)
 * at the current ranks (r1, r2), and two 8-column-aligned sketch slots in
 * the concatenation buffers (round_up(k1, 8) + k1 <= the X_cat capacity,
 * round_up(k2, 8) + k2 <= the Theta_cat capacity).  ranks_out (host, may be NULL)
 * receives (k1, k2).  Like tt_round it is not a recorded step.
 * Errors: TT_ERR_INVALID_ARG (sizes, null pointers, FP32-mixed context),
 * TT_ERR_NUMERIC (a sketch Gram not positive definite after its shift:
 * the context is then poisoned). */
tt_status tt_round_randomized(tt_ctx* ctx, const double* omega1, int32_t k1, const double* omega2,
                              int32_t k2, int32_t ranks_out[2]);

/* Radiation energy density E_i = (1/c) X_i (sum_l Theta_l w_l)(sum_p Phi_p v_p)
 * (Sec. 4.1 eq. tt_energy_density).  E_dev: device N_s doubles or NULL.
 * rad_total / mat_total (host, may be NULL): sum_i E_i dV and
 * sum_i rho_i c_v,i T_i dV. */
tt_status tt_energy(tt_ctx* ctx, double* E_dev, double* rad_total, double* mat_total);

/* Detector loss L = dV sum_i w_i E_i of the current state, with E the
 * energy density of tt_energy (Sec. 4.1 eq. tt_energy_density) and dV the
 * cell volume.  detector_w: host N_s weights (finite).  loss_out: host. */
tt_status tt_detector_loss(tt_ctx* ctx, const double* detector_w, double* loss_out);

/* Gradient of L = loss_w . E(final) dV with respect to the per-cell
 * absorption opacity, by reverse mode over the steps recorded since the
 * last tt_set_cores (ckpt_every > 0, frozen material).  detector_w: host
 * N_s weights.  loss_out: host, may be NULL.  dkappa_dev: device N_s,
 * receives loss_bar * dL/dkappa.  Errors: TT_ERR_STATE if nothing taped,
 * or if the tape is stale (tt_set_kappa or tt_round after the steps). */
tt_status tt_grad(tt_ctx* ctx, const double* detector_w, double loss_bar,
                  double* loss_out, double* dkappa_dev);

/* Replace the absorption opacity (device N_s doubles, copied). */
tt_status tt_set_kappa(tt_ctx* ctx, const double* kappa_dev);

/* Isotropic scattering opacity kappa_s (host N_s doubles, finite, >= 0;
 * copied), Sec. 3.2 eq. couple_a with implicit J^{m+1}.  All zero turns
 * scattering off.  Rejected (TT_ERR_INVALID_ARG) on a context with a tape. */
tt_status tt_set_scattering(tt_ctx* ctx, const double* kappa_s);

/* Copy the current cores to host buffers sized at least N_s*r1,
 * r1*N_theta*r2 and r2*N_phi (any may be NULL); r (host, 2 ints) receives
 * the ranks.  Call with all buffers NULL to query the ranks. */
tt_status tt_get_cores(tt_ctx* ctx, double* X, double* Th, double* Ph, int32_t r[2]);

/* Install new cores (host, finite) with ranks r[0], r[1]; clears the poison
 * flag, the rank history and the tape. */
tt_status tt_set_cores(tt_ctx* ctx, const double* X, const double* Th, const double* Ph,
                       const int32_t r[2]);

/* Per-cell temperature (host N_s). */
tt_status tt_get_temperature(tt_ctx* ctx, double* T);

/* Ranks after each recorded step, (r1, r2) pairs, oldest first.  buf: host,
 * 2*cap ints; n (host) receives the number of pairs available. */
tt_status tt_get_rank_history(tt_ctx* ctx, int32_t* buf, int32_t cap, int32_t* n);

/* Ranks to use in TT_RANK_REPLAY mode: r1r2[2*k], r1r2[2*k+1] for the k-th
 * rounding after this call (host, copied). */
tt_status tt_set_rank_schedule(tt_ctx* ctx, const int32_t* r1r2, int32_t nroundings);

/* Diagnostics of the last rounding (host, 16 doubles): [0] ||T||^2,
 * [1] delta^2, [2..3] kept Gram eigenpairs bond 1 (A, B), [4..5] bond 2,
 * [6] r1', [7] r2', [8] tail(r1')/delta^2, [9] tail(r2')/delta^2,
 * [10] sigma_1 bond 1, [11] sigma_{r1'}, [12] sigma_{r1'+1},
 * [13] sigma_{r2'}, [14] sigma_{r2'+1}, [15] R1 (pre-rounding rank). */
tt_status tt_get_round_info(tt_ctx* ctx, double out[16]);

/* Kernel timing with HIP events on the context's stream.  enable != 0
 * starts recording (resets counters): 1 records every class, any other
 * value records the classes k whose bit k + 1 is set (one event pair per
 * timed region of those classes only).  tt_profile_read fills, for up to
 * `cap` kernel classes, the total milliseconds, the launch count and a
 * static name; returns the number of classes in *n. */
tt_status tt_profile_enable(tt_ctx* ctx, int32_t enable);
tt_status tt_profile_read(tt_ctx* ctx, double* ms, int32_t* count, const char** names,
                          int32_t cap, int32_t* n);

/* Slices of the FP32-mixed Gram (TT_FP32_MIXED only; no effect in TT_FP64).
 * Each FP32 entry is split on its column's exponent grid into `slices`
 * 11-bit integer slices and the slice pairs (a, b) with a + b < slices are
 * multiplied exactly on FP32 MFMA and accumulated in FP64, so the Gram is
 * exact to about 2^(-11 slices) of each column's largest entry (1 slice: 11
 * bits, below FP32's own 24; 3 or more cover all 24) at slices (slices + 1)
 * / 2 MFMA passes.  Default 4.  A speed/accuracy knob beside the paper's
 * method (its Gram is FP64), kept for measuring that trade-off.  Drops the
 * captured step graphs and synchronises the context's stream.
 * Errors: TT_ERR_INVALID_ARG unless 1 <= slices <= 6. */
tt_status tt_set_gram_slices(tt_ctx* ctx, int32_t slices);

/* Caps the sweeps of the one-sided Jacobi SVD of M (used when the short side
 * of M is at most 64) at jacobi_max_sweeps (0, the default: its own limit of
 * 40).  For exercising the failure path: with a cap too low for the matrix
 * the solver stops unconverged (its rotations keep every value finite), the
 * next tt_step or tt_round returns TT_ERR_NUMERIC ("the Jacobi SVD did not
 * converge") and the context is poisoned.  Synchronises the context's
 * stream; captured step graphs stay valid (the kernels read the cap from the
 * device at run time).
 * Errors: TT_ERR_INVALID_ARG if jacobi_max_sweeps < 0. */
tt_status tt_set_solver_limits(tt_ctx* ctx, int32_t jacobi_max_sweeps);

/* Step execution mode.  enable != 0 (the default): tt_step replays the
 * step's launch sequence as a HIP graph, captured on first use once per
 * state buffer (the step alternates two) on a private non-blocking stream
 * of the context and launched on the context's stream; steps taken while
 * event timing is on or while the gradient tape records run eagerly, and
 * so does every step after a capture the runtime refuses.  enable == 0:
 * every step launches its kernels one by one.  Both modes compute the same
 * bits.  Captured graphs are dropped when this is called, when the
 * scattering field or the rank schedule changes, and by tt_destroy.
 * Synchronises the context's stream. */
tt_status tt_use_graphs(tt_ctx* ctx, int32_t enable);

const char* tt_last_error(const tt_ctx* ctx);

/* Destroy a context (NULL is accepted); the workspace is not freed. */
void tt_destroy(tt_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TT_H */
