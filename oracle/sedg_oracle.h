/*
 * Oracle for the sub-element adaptive blended DG/FV scheme of
 * Markert, Gassner & Walch, "A Sub-Element Adaptive Shock Capturing Approach
 * for Discontinuous Galerkin Methods" (arXiv:2011.03338).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU definition of the
 * right-hand side that the HIP library computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header or table generator with the library: it builds its own
 * operator tables in long double.
 *
 * Notation: K = number of subcell mean values per direction per element (the
 * paper's N, a power of two); levels are written by their order n in
 * {1 (FV), 2, 4, ..., K}.  Conserved state (rho, rho*v, E), nvar = dim + 2.
 *
 * State layout (global subcell grid, structure of arrays):
 *   u[var][gz][gy][gx], gx fastest, extents G_a = nelem_a * K (1 for unused axes).
 * Element order: ex fastest, then ey, then ez.
 * Blending factor layout per element (A values): level K first (one value),
 * then K/2 ((2)^dim values), ..., down to level 2; within a level the
 * sub-element index is sx + (K/n)*(sy + (K/n)*sz).
 */
#ifndef SEDG_ORACLE_H
#define SEDG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_EINVAL = -1, OR_ESTATE = -4 };
enum { OR_PERIODIC = 0, OR_OUTFLOW = 1 };
enum { OR_GAUSS = 0, OR_LGL = 1 };
enum { OR_ADAPTIVE = 0, OR_FORCE_DG = 1, OR_FORCE_FV = 2, OR_EXTERNAL = 3, OR_RANDOM = 4, OR_FROZEN = 9 };

typedef struct or_mesh {
    int dim;            /* 1, 2 or 3 */
    int K;              /* mean values per direction per element: 2, 4 or 8 */
    int nelem[3];       /* elements per axis (1 for unused axes) */
    double lo[3], hi[3];
    int bc[3];          /* OR_PERIODIC or OR_OUTFLOW per axis */
    double gamma;
    int family;         /* OR_GAUSS (default) or OR_LGL collocation nodes */
} or_mesh;

typedef struct or_params {
    double tau_A, tau_S;        /* indicator amplification / sensitivity */
    double alpha_H, alpha_L;    /* level snapping thresholds */
    double beta_L;              /* squeeze rejection threshold */
    double cfl;
    int top_level;              /* highest DG order used (DGFVn); <= K */
    unsigned level_mask;        /* bit log2(n) enables DG level n; 0 = all */
    int mode;                   /* OR_ADAPTIVE, OR_FORCE_DG, OR_FORCE_FV, OR_EXTERNAL, OR_RANDOM */
    unsigned long long seed;    /* OR_RANDOM: generator seed */
    long long draw;             /* OR_RANDOM: index of the (first) draw of factors */
    double sigma_floor;         /* floor in the indicator's denominator; <= 0: the paper's 1 */
    int integrator;             /* or_rk3: 0 SSP-RK3, 1 SSP-RK(5,4) */
} or_params;

/* Number of blending factors per element. */
int or_alpha_len(const or_mesh *m, const or_params *p);

/* Operator tables of level n (2..8) for node family fam.  Writes, in order:
 * xi[n], w[n], Dcal[n*n], D[n*n], bm[n], bp[n], P[n*n], R[n*n], Dhat[n*n],
 * Bhat_left[n], Bhat_right[n], Iplus[n*n], Iminus[n*n]  (row-major).
 * Returns the number of doubles written, or OR_EINVAL. */
int or_tables(int n, int fam, double *out, int cap);

/* One right-hand-side evaluation.
 *   u        : state (nvar * DOF doubles), read only
 *   dudt     : output, same shape
 *   alpha    : output (nelem_total * A) blending factors actually used, may be NULL
 *   beta     : output (nelem_total * A) squeezing parameters, may be NULL
 *   alpha_in : input for OR_EXTERNAL mode, else ignored
 *   xraw     : output (nelem_total * A) pre-clamp indicator value max_phi tau_A(r - tau_S)
 *              (NaN where not computed), may be NULL
 *   araw     : output (nelem_total * A) blending factors before level snapping, may be NULL
 *   nfallback: output count of interface-safety fallbacks, may be NULL
 * Returns OR_OK, OR_EINVAL, or OR_ESTATE if a mean value is not permissible. */
int or_rhs(const or_mesh *m, const or_params *p, const double *u, double *dudt,
           double *alpha, double *beta, const double *alpha_in,
           double *xraw, double *araw, long *nfallback);

/* CFL time step of the state u; returns a negative value on a bad state. */
double or_max_dt(const or_mesh *m, const or_params *p, const double *u);

/* nsteps steps in place of SSP-RK3 or (p->integrator = 1) SSP-RK(5,4).  dt_fixed > 0
 * uses that step, else the CFL step of each step's initial state.  dt_log (nsteps)
 * may be NULL. */
int or_rk3(const or_mesh *m, const or_params *p, double *u, int nsteps,
           double dt_fixed, double *dt_log);

/* Right-hand side with frozen blending factors and squeezing parameters
 * (alpha, beta: nel * A each): the map whose derivative the adjoint transposes. */
int or_rhs_frozen(const or_mesh *m, const or_params *p, const double *u, const double *alpha,
                  const double *beta, double *dudt);

/* Adjoint of the frozen right-hand side at u: lam_out = (dL/du)^T lam, with alpha
 * and beta held fixed, the interface-safety decisions and the HLLE wave-speed
 * branches taken at u. */
int or_adjoint_rhs(const or_mesh *m, const or_params *p, const double *u, const double *alpha,
                   const double *beta, const double *lam, double *lam_out);

/* Weighted blending factor of every subcell (eq. order-estimate) from the blending
 * factors alpha (nel * A): abar[dof] in the state layout of one variable. */
int or_alpha_bar(const or_mesh *m, const or_params *p, const double *alpha, double *abar);

/* Tables of the non-conforming appendix for level n: Z = P^(n->2n) [2n*n],
 * Q = P^(n->n/2) [(n/2)*n], L_- [n*n], L_+ [n*n].  Returns the count or OR_EINVAL. */
int or_nc_tables(int n, int fam, double *out, int cap);

/* Blended refinement (eq. 3D-refinement) of every element of mesh m into 2^dim
 * children, and the blended coarsening (eq. 3D-coarsening) of the mesh with twice the
 * elements per axis back onto m; alpha: factors of the input mesh's elements. */
int or_refine(const or_mesh *m, const or_params *p, const double *u, const double *alpha, double *u_fine);
int or_coarsen(const or_mesh *m, const or_params *p, const double *u_fine, const double *alpha_fine, double *u);

/* Number of OpenMP threads the oracle runs with. */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
