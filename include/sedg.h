/*
 * libsedg - sub-element adaptive blended DG/FV right-hand side on MI355X (gfx950).
 *
 * Method: Markert, Gassner & Walch, "A Sub-Element Adaptive Shock Capturing
 * Approach for Discontinuous Galerkin Methods", arXiv:2011.03338.
 *
 * Each Cartesian element carries K^dim subcell mean values of the compressible
 * Euler state (Sec. 2, eq. subcell-grid; App. 3D extension).  The library
 * evaluates the semi-discrete right-hand side of the multi-level blending
 * scheme (Sec. 2.6, eq. multilevel-blending-scheme and
 * multilevel-blending-discretizations; App. eq. dgfv-scheme-3d): per element it
 * reconstructs the hierarchy O(K) .. O(2) from the mean values (eq. reco-*),
 * squeezes non-permissible reconstructions (eq. positivity-limiter), computes
 * the sub-element blending factors (Sec. 2.7, eq. calc-blending-factor) with the
 * level pruning of the multi-level algorithm (App. sketch of the algorithm),
 * evaluates unique common interface fluxes (Sec. 2.6; App. eq.
 * 3D-blend-interface-fluxes) and blends the level right-hand sides with the
 * weights of eq. blending-weights.  Time stepping is the three-stage SSP
 * Runge-Kutta scheme with the CFL step of eq. cfl-condition.
 *
 * Conventions
 *   K      mean values per direction per element (the paper's N): 4 or 8.
 *   dim    2 or 3; nvar = dim + 2, conserved (rho, rho*v, E).
 *   State  device array of nvar * DOF doubles, structure of arrays on the
 *          global subcell grid: u[var][gz][gy][gx], gx fastest, extents
 *          G_a = nelem_a * K.  Elements are numbered ex fastest, then ey, ez.
 *   Alpha  per element A = sum over DG levels n = top, top/2, ..., 2 of (K/n)^dim
 *          values, level top first; inside a level the sub-element index is
 *          sx + (K/n) * (sy + (K/n) * sz).  The same layout holds for beta.
 *
 * Ownership and errors
 *   The caller owns every device pointer passed in (contiguous FP64 on the
 *   current device); the library only borrows them for the call and enqueues
 *   all work asynchronously on the given stream (a hipStream_t passed as
 *   void*, NULL = default stream).  A context owns its operator tables,
 *   interface buffers, blending-factor arrays and stage buffers.  Use one
 *   context per stream; calls on one context are not thread-safe.
 *   Functions return SEDG_OK (0) or a negative code; no exception or abort
 *   crosses the interface.  Arguments are validated before anything is
 *   enqueued (SEDG_EINVAL).  A mean value that is not permissible (rho <= 0,
 *   p <= 0 or not finite) is detected on the device and reported by
 *   sedg_check (SEDG_ESTATE); the kernels never index memory with data values,
 *   so such a state yields garbage, never a fault.
 */
#ifndef SEDG_H
#define SEDG_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SEDG_OK = 0,
    SEDG_EINVAL = -1,      /* bad argument */
    SEDG_EHIP = -2,        /* HIP runtime error */
    SEDG_ENOMEM = -3,      /* device allocation failed */
    SEDG_ESTATE = -4,      /* non-permissible or non-finite mean value detected */
    SEDG_EUNSUPPORTED = -5,/* configuration not compiled (dim, K) */
    SEDG_ESCRATCH = -6     /* problem larger than the static work space of sedg_rhs_noalloc */
};

/* Largest mesh a context takes: 2^28 - 1 elements (a 2-D K=8 mesh of that size would hold
 * 2 TB of state, a 3-D one 5 TB), and at most INT_MAX subcells along an axis; larger
 * requests give SEDG_EINVAL from sedg_create, sedg_batch_create (per member) and
 * sedg_rhs_noalloc before any device work. */
#define SEDG_MAX_ELEMENTS 268435455

enum { SEDG_PERIODIC = 0, SEDG_OUTFLOW = 1 };
enum { SEDG_SSPRK3 = 0, SEDG_SSPRK54 = 1 };
enum { SEDG_GAUSS = 0, SEDG_LGL = 1 };
enum { SEDG_ADAPTIVE = 0, SEDG_FORCE_DG = 1, SEDG_FORCE_FV = 2, SEDG_EXTERNAL = 3, SEDG_RANDOM = 4 };

typedef struct sedg_mesh {
    int dim;            /* 2 or 3 */
    int K;              /* 4 or 8 */
    int nelem[3];       /* elements per axis (1 on unused axes) */
    double lo[3], hi[3];/* domain box */
    int bc[3];          /* SEDG_PERIODIC or SEDG_OUTFLOW per axis; outflow = zero gradient of the
                           subcell means: a boundary face sees the boundary subcell's mean outside,
                           with the same blending weights */
    double gamma;       /* ratio of specific heats (eq. equation-of-state) */
    int family;         /* collocation nodes: SEDG_GAUSS (the paper's, Sec. 2.2) or SEDG_LGL */
} sedg_mesh;

typedef struct sedg_params {
    double tau_A, tau_S;     /* indicator amplification / sensitivity (Sec. 2.7): 100, 0.05 */
    double alpha_H, alpha_L; /* level snapping thresholds (Sec. 2.8): 0.99, 0.01 */
    double beta_L;           /* squeeze rejection threshold (Sec. 2.8): 0.95 */
    double cfl;              /* CFL number of eq. cfl-condition */
    int top_level;           /* highest DG order used (DGFVn, Sec. 3.5); 0 = K */
    unsigned level_mask;     /* bit log2(n) enables DG level n; 0 = all levels */
    int mode;                /* SEDG_ADAPTIVE, SEDG_FORCE_DG (alpha_top = 1),
                                SEDG_FORCE_FV (all alpha = 0), SEDG_EXTERNAL (alpha given),
                                SEDG_RANDOM (alpha drawn afresh for every right-hand side) */
    unsigned long long seed; /* SEDG_RANDOM: seed of the generator */
    double sigma_floor;      /* floor of the denominator max(sigma_n/2, sigma_n, floor) of
                                eq. calc-blending-factor; 0 = the paper's 1 (a smaller floor
                                is a variant, not the paper's scheme) */
    int integrator;          /* SEDG_SSPRK3 (three-stage SSP-RK, Shu-Osher form) or SEDG_SSPRK54
                                (the five-stage fourth-order SSP-RK of Spiteri and Ruuth, which
                                the paper uses, Sec. 3) for sedg_rk_step; the step-tape, frozen
                                and adjoint steps are SSP-RK3 only */
} sedg_params;

typedef struct sedg_ctx sedg_ctx;

/* Create a context for one mesh and parameter set on the current HIP device.
 * Builds the operator tables of Sec. 2.2-2.4 and 2.6 (nodes, weights, D, Dhat,
 * Bhat, P, R, interface interpolation) and allocates the context's device
 * buffers.  *out receives the context.  Returns SEDG_EINVAL for a bad mesh,
 * SEDG_EUNSUPPORTED for (dim, K) not compiled, SEDG_ENOMEM, SEDG_EHIP. */
int sedg_create(const sedg_mesh *mesh, const sedg_params *params, sedg_ctx **out);

/* Release a context (synchronises the device first).  NULL is allowed. */
int sedg_destroy(sedg_ctx *ctx);

/* Doubles in one state array (nvar * DOF) and in one blending-factor array
 * (A * number of elements); negative on a NULL context. */
long sedg_state_len(const sedg_ctx *ctx);
long sedg_alpha_len(const sedg_ctx *ctx);

/* Replace the parameters of an existing context (same mesh).  Restarts the
 * SEDG_RANDOM draw counter at 0. */
int sedg_set_params(sedg_ctx *ctx, const sedg_params *params);

/* Copy a host state into the device array u_dev (nvar * DOF doubles, layout above)
 * and check every mean value: SEDG_ESTATE with *bad_elem (optional) = the smallest
 * index of an element holding a non-permissible (rho <= 0 or p <= 0) or non-finite
 * mean value, else SEDG_OK and *bad_elem = -1.  Synchronous (the whole device); the
 * host array is only read during the call.  Clears the context's state-error flag. */
int sedg_init_state(sedg_ctx *ctx, double *u_dev, const double *u_host, long *bad_elem);

/* One evaluation of the blended right-hand side d(u)/dt (eq.
 * multilevel-blending-scheme blended by eq. blending-weights).
 * In SEDG_RANDOM mode (the conservation stress test of Sec. 3.3) every factor of
 * every level and sub-element is uniform in [0, 1), drawn afresh for each
 * right-hand side the context evaluates (sedg_rhs, every stage of the step
 * functions, sedg_diagnose): factor q of element e in draw d is the k-th output of
 * SplitMix64 (Steele, Lea & Flood 2014) seeded with params.seed, k = (d * nel + e)
 * * A + q, as a double from its top 53 bits; d counts the draws since sedg_create
 * or sedg_set_params.  Squeezing parameters are computed on every level, as in
 * SEDG_EXTERNAL mode.
 *   u         device, state (read only)
 *   dudt      device, output state-shaped array (must not alias u)
 *   alpha_out device, optional (NULL): blending factors used, A per element
 *   beta_out  device, optional (NULL): squeezing parameters, A per element
 *   alpha_in  device, required in SEDG_EXTERNAL mode (ignored otherwise)
 *   stream    hipStream_t or NULL
 * Asynchronous; state errors are reported by sedg_check. */
int sedg_rhs(sedg_ctx *ctx, const double *u, double *dudt, double *alpha_out, double *beta_out,
             const double *alpha_in, void *stream);

/* CFL step of the state u (eq. cfl-condition with eq. euler-max-eigenvalue),
 * written to the device scalar *dt_dev. */
int sedg_max_dt(sedg_ctx *ctx, const double *u, double *dt_dev, void *stream);

/* Advance u in place by nsteps steps of params.integrator: three-stage SSP-RK
 * (Shu-Osher form) or SSP-RK(5,4) (five stages; alpha_log then holds 5 arrays per step).
 *   dt_fixed > 0: that step size; otherwise the CFL step of each step's
 *   initial state, computed on the device.
 *   dt_log_dev: device, optional, receives the nsteps step sizes (fixed or CFL).
 *   alpha_log_dev: device, optional, receives the blending factors of every stage,
 *   3 * nsteps arrays of sedg_alpha_len doubles, step-major ([step][stage][...]).
 * The step sequence is captured once into a HIP graph per (u, dt_log, alpha_log,
 * fixed step) and replayed.  EXTERNAL mode is rejected (SEDG_EINVAL). */
int sedg_rk_step(sedg_ctx *ctx, double *u, int nsteps, double dt_fixed, double *dt_log_dev, double *alpha_log_dev,
                 void *stream);

/* Diagnostics of one right-hand side at u (computed as sedg_rhs computes it, into
 * dudt, device): the change of bulk of eq. change-of-bulk (Sec. 3.3), read as the
 * sum over elements of |Omega_q| times the element mean of d(u)/dt, with the same
 * sum of |d(u)/dt| as its scale; the weighted blending factor of eq. order-estimate
 * per subcell (alpha_bar: device, optional, state-shaped for one variable) and its
 * minimum, mean and maximum; the elements by the lowest order carrying weight
 * anywhere in them (index 0: FV, 1: O(2), 2: O(4), 3: O(8)); the sub-elements
 * squeezed (beta < 1) and rejected (beta < beta_L) on the levels evaluated; and the
 * interface-safety fallbacks taken (an FV flux input replaced by the subcell mean,
 * or a DG candidate handing its weight to FV, counted per face subcell).
 * Synchronises the stream; *out is host memory.  Not in SEDG_EXTERNAL mode. */
typedef struct sedg_diag {
    double bulk_change[5], bulk_abs[5];
    double alpha_bar_min, alpha_bar_mean, alpha_bar_max;
    long elems_by_lowest_order[4];
    long squeezed, beta_rejected, fallbacks;
} sedg_diag;
int sedg_diagnose(sedg_ctx *ctx, const double *u, double *dudt, double *alpha_bar, sedg_diag *out, void *stream);

/* Synchronise the context's last stream and report device-side state errors:
 * SEDG_ESTATE with *bad_elem = index of an element holding a non-permissible
 * or non-finite mean value, else SEDG_OK and *bad_elem = -1.  Clears the flag. */
int sedg_check(sedg_ctx *ctx, long *bad_elem);

/* Per-kernel timing with HIP events, for benchmarking.  After sedg_profile(ctx, 1)
 * sedg_rk_step enqueues its kernels directly (no graph replay) and records an event
 * on the caller's stream before its first launch and after every launch, so that a
 * launch is timed from the end of the one before it (within the call) to its own
 * end, one event marker per launch; sedg_profile_read synchronises
 * that stream and returns, for the analyse, residual, step-size and element-face
 * flux kernels (arrays of 4, in that order), the summed milliseconds and the launch
 * counts, then clears them.  sedg_profile(ctx, 0) returns to graph replay. */
int sedg_profile(sedg_ctx *ctx, int on);
int sedg_profile_read(sedg_ctx *ctx, double *ms, long *count);

/* ---- frozen map and its adjoint --------------------------------------------
 * The paper defines the forward scheme only; differentiation is an extension.
 * The frozen map is the right-hand side with the blending factors alpha and the
 * squeezing parameters beta of eq. calc-squeezing-parameter held fixed (weights
 * of eq. blending-weights from alpha), every other step as in sedg_rhs.  Its
 * adjoint is the exact transposed Jacobian of that map at u: the interface-safety
 * decisions (non-admissible flux inputs) are taken at u and held, and the
 * min/max of the HLL-Einfeldt wave speeds are differentiated on the branch the
 * evaluation at u takes.  alpha and beta are device arrays of sedg_alpha_len
 * doubles in the layout above (e.g. sedg_rhs's alpha_out / beta_out). */

/* dudt = frozen right-hand side at u.  Any dim and K the context supports. */
int sedg_rhs_frozen(sedg_ctx *ctx, const double *u, const double *alpha, const double *beta, double *dudt,
                    void *stream);

/* lam_out = (dL/du)^T lam for the frozen map L at u (vector-Jacobian product).
 *   u, lam    device, state-shaped (read only)
 *   lam_out   device, state-shaped output; must alias neither u nor lam
 * SEDG_EUNSUPPORTED at dim 3 with K = 8 (one element's adjoint data exceed the
 * on-chip memory of a workgroup).  Allocates the context's adjoint buffers on
 * first use (SEDG_ENOMEM).  State errors are reported by sedg_check. */
int sedg_adjoint_rhs(sedg_ctx *ctx, const double *u, const double *alpha, const double *beta, const double *lam,
                     double *lam_out, void *stream);

/* Doubles in one step tape: the three stage states of one SSP-RK3 step and, for
 * each stage, its blending factors, squeezing parameters, element-face states,
 * sub-element means and element data scales,
 * [u^n | u^(1) | u^(2) | alpha x 3 | beta x 3 | face states x 3 | means x 3 | scales x 3]
 * (alpha and beta in the layout above). */
long sedg_tape_len(const sedg_ctx *ctx);

/* nsteps SSP-RK3 steps of u in place, step j with the step size dt_dev[j] (device),
 * recording step j's tape at tapes + j * sedg_tape_len (device, caller-owned).  The
 * arithmetic is that of sedg_rk_step, so steps replayed from a checkpoint with the
 * logged step sizes reproduce the original steps bit for bit. */
int sedg_rk_step_tape(sedg_ctx *ctx, double *u, int nsteps, const double *dt_dev, double *tapes, void *stream);

/* The frozen forward map over nsteps SSP-RK3 steps, u in place: step j with step size
 * dt_dev[j] and, in each stage k, the blending factors and squeezing parameters held at
 * factors + j * 6 * A_len + k * A_len and + (3 + k) * A_len (A_len = sedg_alpha_len:
 * exactly the factor block of a step tape, [alpha x 3 | beta x 3]); every other step
 * of the right-hand side as in sedg_rhs_frozen.  The map the adjoint steps transpose. */
int sedg_rk_step_frozen(sedg_ctx *ctx, double *u, int nsteps, const double *dt_dev, const double *factors,
                        void *stream);

/* Transposed SSP-RK3 steps: on entry lam holds dJ/du after the nsteps steps recorded in
 * tapes (step j at tapes + j * sedg_tape_len, step size dt_dev[j]); on return dJ/du
 * before them, with alpha, beta and the step sizes frozen.  Same support and
 * allocation rules as sedg_adjoint_rhs. */
int sedg_adjoint_rk_step(sedg_ctx *ctx, const double *tapes, int nsteps, const double *dt_dev, double *lam,
                         void *stream);

/* ---- batched ensembles -------------------------------------------------------
 * Many independent 2-D problems of the scheme above, each with its own mesh
 * (element counts, box, boundary conditions, K = 4 or 8) and its own CFL step,
 * sharing the scheme parameters (params->top_level must be 0; EXTERNAL mode is
 * not available), the ratio of specific heats and the node family.  Their states
 * sit back to back in one device array: problem p occupies
 * [sedg_batch_state_offset(p), + 4 * its DOF) in the single-problem layout.
 * One step advances every problem by one step of params->integrator (SSP-RK3 or
 * SSP-RK(5,4)) with one launch each of the analyse, element-face flux and
 * residual kernels per stage for the whole ensemble (plus a per-problem
 * step-size kernel), captured once per (u, dt_log, fixed) into a HIP graph and
 * replayed; each problem's result equals, bit for bit, that of a single-problem
 * context with the same mesh and parameters. */
typedef struct sedg_batch sedg_batch;

/* Launch shape of the batched kernels (chosen by an autotuner):
 *   epb4, epb8     elements per workgroup for K = 4 and K = 8: (4, 1) or (8, 2)
 *                  (64 or 128 threads)
 *   blocks_per_cu  0: one workgroup per tile; n > 0: a persistent grid of n
 *                  workgroups per compute unit, each taking a contiguous run of
 *                  tiles (at most 64)
 *   xcd_map        1: workgroups remapped so that each XCD takes a contiguous
 *                  range of tiles (neighbour face data stay in its L2); 0: none
 *   waves_analyse  register budget of the analyse kernel, as the number of
 *                  wavefronts per SIMD it must leave room for: 3 (<= 168
 *                  VGPRs) or 4 (<= 128 VGPRs, values may spill to scratch);
 *                  0 selects 3
 *   waves_residual the same for the residual kernel: 3 (or 0); 4 is not built
 *                  and returns SEDG_EUNSUPPORTED
 * Every shape computes bit-identical results (the same arithmetic in the same order). */
typedef struct sedg_batch_tuning {
    int epb4, epb8, blocks_per_cu, xcd_map;
    int waves_analyse, waves_residual;
} sedg_batch_tuning;

/* Create an ensemble of count problems (meshes[0..count-1], dim 2).  Returns
 * SEDG_EUNSUPPORTED for dim != 2 or K not in {4, 8}, SEDG_EINVAL for mixed gamma
 * or node family, a bad mesh, top_level != 0 or EXTERNAL mode; SEDG_ENOMEM. */
int sedg_batch_create(const sedg_mesh *meshes, int count, const sedg_params *params, sedg_batch **out);
int sedg_batch_destroy(sedg_batch *batch);

/* Doubles in the ensemble state; offset of problem p's state (negative on error). */
long sedg_batch_state_len(const sedg_batch *batch);
long sedg_batch_state_offset(const sedg_batch *batch, int p);

/* Set / read the launch shape (synchronises the device; drops captured graphs). */
int sedg_batch_set_tuning(sedg_batch *batch, const sedg_batch_tuning *tuning);
int sedg_batch_get_tuning(const sedg_batch *batch, sedg_batch_tuning *tuning);

/* Advance every problem by nsteps steps of params->integrator in place.  dt_fixed > 0:
 * that step for all problems; otherwise each problem's own CFL step of each step's
 * initial state.  dt_log_dev (device, optional, CFL steps only) receives
 * nsteps * count step sizes, step-major.  SSP-RK(5,4) allocates one more
 * ensemble-sized state on its first call (SEDG_ENOMEM if that fails). */
int sedg_batch_rk_step(sedg_batch *batch, double *u, int nsteps, double dt_fixed, double *dt_log_dev, void *stream);

/* Synchronise and report a non-permissible or non-finite mean value: SEDG_ESTATE
 * with the problem index and its element index, else SEDG_OK and -1, -1. */
int sedg_batch_check(sedg_batch *batch, int *bad_problem, long *bad_elem);

/* ---- refinement and coarsening (App., non-conforming interfaces) ----------------
 * Blended refinement of every element of the context's mesh into 2^dim children
 * (eq. 3D-refinement) and its reverse, the blended coarsening of every family of
 * 2^dim children (eq. 3D-coarsening), as the building blocks of 4:1 non-conforming
 * meshes.  The fine mesh has twice the elements of the context's mesh along every axis
 * and the same K: its state (2^dim * sedg_state_len doubles, same layout) is the state
 * on the doubled global subcell grid.  Written for the multi-level weights of eq.
 * blending-weights: a fine subcell receives theta_FV times its parent cell's mean (the
 * expansion E = I (x) 1_2) plus, per DG level n, theta^(n) times the mean over the fine
 * subcell of the level-n sub-element's nodal polynomial (Z = P^(n->2n) along every
 * axis); coarsening compresses each child with its own weights (C = 1/2 I (x) 1_2^T,
 * Q = P^(n->n/2)) and glues the children.  With single-level factors (level mask
 * {1, K}) these are the paper's formulas.  Both conserve every element's integral for
 * any factors.
 *   u, u_fine     device states of the context's mesh and of the fine mesh
 *   alpha         device, the factors of the context's elements (refine) or of the
 *                 fine elements (coarsen), A per element in the layout above
 * Asynchronous; in and out must not alias.  Allocates the context's tables on first
 * use (SEDG_ENOMEM). */
int sedg_refine(sedg_ctx *ctx, const double *u, const double *alpha, double *u_fine, void *stream);
int sedg_coarsen(sedg_ctx *ctx, const double *u_fine, const double *alpha_fine, double *u, void *stream);

/* Host-only: the refinement, coarsening and mortar tables of level n (2, 4, 8) for
 * node family fam, in the order Z = P^(n->2n) [2n*n], Q = P^(n->n/2) [(n/2)*n],
 * L_- [n*n], L_+ [n*n] (row-major; (L_+-)_ij = l_i(xi_j/2 +- 1/4) w_j / (2 w_i), the
 * L2 projection of a fine face's flux onto the coarse face, App. non-conforming
 * interfaces).  Returns the count written or SEDG_EINVAL. */
int sedg_nc_tables(int n, int family, double *out, int cap);

/* Host-only: the library's own operator tables of level n (2, 4, 8) for node
 * family fam, in the order xi[n], w[n], Dcal[n*n], D[n*n], bm[n], bp[n],
 * P[n*n], R[n*n], Dhat[n*n], Bhat_left[n], Bhat_right[n], Iplus[n*n],
 * Iminus[n*n] (row-major).  Returns the count written or SEDG_EINVAL. */
int sedg_tables(int n, int family, double *out, int cap);

/* ---- right-hand side without device allocation ------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Computes what sedg_rhs
 * computes (same kernels, same results bit for bit) for the given mesh and
 * parameters, with no context: every work array (blending factors, squeezing
 * parameters, sub-element means, face states, element-face fluxes, data scales,
 * the error flag) and the operator tables live in one static device array of
 * 64 MiB per device, held from the first call until the process ends.
 *   mesh, params  host; modes SEDG_ADAPTIVE, SEDG_FORCE_DG and SEDG_FORCE_FV
 *                 (SEDG_EINVAL otherwise)
 *   u             device, state (read only)
 *   dudt          device, output state-shaped array (must not alias u)
 *   bad_dev       device int, optional (NULL): receives the index of an element
 *                 holding a non-permissible or non-finite mean value, INT_MAX if none
 *   stream        hipStream_t or NULL
 * Returns SEDG_ESCRATCH when the work arrays of the mesh exceed the static space
 * (per element 8 * ((2 + nvar) * A + 4 * dim * nvar * K^(dim-1) + 2) bytes: 2-D
 * K = 8 about 21 800 elements, 3-D K = 8 about 1 900).  It calls no hipMalloc or
 * hipFree.  The first call on a device locates that device's array and copies the
 * operator tables into it synchronously, so it must not be made under stream
 * capture; later calls only enqueue kernels.  All calls on one device share its
 * array and leave the last call's contents there: calls that overlap in time on
 * one device (different streams or threads) race and must be serialised by the
 * caller. */
int sedg_rhs_noalloc(const sedg_mesh *mesh, const sedg_params *params, const double *u, double *dudt, int *bad_dev,
                     void *stream);

/* Text of a return code. */
const char *sedg_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
