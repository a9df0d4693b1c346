/*
 * mlb_batch.h - many independent 2D static analyses in one set of launches.
 *
 * A batch holds up to 64 independent Q4 problems of different sizes (the
 * same material, each with its own grid, clamp, load and density).  Each is
 * the static step of the analysis (Alg. 1: solve K[x] u = f with the SIMP
 * stiffness of eq. interpolationSIMP2-SIMP), followed by the compliance
 * J = f^T u and its gradient (Sec. 3).  Every instance gets its own geometric
 * multigrid hierarchy (Galerkin coarse levels, damped Jacobi, dense coarsest
 * inverse), and its own FP64 CG with its own scalars and convergence test.
 *
 * All instances advance together: each step of a CG iteration (operator
 * apply, vector updates, every level of the V-cycle) is ONE kernel launch
 * over a work list of (instance, level, 256-node chunk) items, dispatched
 * one block per item or drained by a persistent grid through atomic work
 * queues (one per XCD, with stealing).  Converged instances
 * drop out of the queue's work (their items are skipped) while the others
 * continue.  With graphs enabled, one whole iteration is captured once and
 * replayed.
 *
 * Layout.  Instance i has nel_i = (nx_i, ny_i) elements, n_i = 2 (nx_i+1)
 * (ny_i+1) DOFs (interleaved, node x fastest, as in mlb.h) and m_i = nx_i
 * ny_i elements.  Batched vectors are the instances' vectors concatenated in
 * instance order: DOF offsets dof_off[i] = sum_{k<i} n_k, element offsets
 * elem_off[i] = sum_{k<i} m_k (mlb_batch_layout).
 *
 * Coarsening: instance i is coarsened by 2 per axis at least once, then
 * while both element counts are even and its current level has more than
 * max_coarse_dofs DOFs; the last level is solved by its dense inverse, which
 * may have at most 1024 DOFs (else mlb_batch_create returns MLB_EINVAL).
 *
 * Ownership, errors and streams follow mlb.h: the caller owns all pointers,
 * every call returns MLB_OK or a negative MLB_E* code, mlb_batch_last_error
 * explains the last failure.  Solve calls synchronise their stream.
 */
#ifndef MLB_BATCH_H
#define MLB_BATCH_H

#include <stdint.h>

#include "mlb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlb_batch mlb_batch;

typedef struct {
    int ninst;            /* number of instances, 1..64 */
    int nel[128];         /* (nx, ny) of instance i at nel[2i], nel[2i+1]; even, >= 2 */
    double E1;            /* solid Young's modulus */
    double E0;            /* void Young's modulus, 0 <= E0 < E1 */
    double nu;            /* Poisson ratio */
    double penal;         /* SIMP exponent p >= 1 */
    int precision;        /* MLB_FP64 or MLB_MIXED (FP32 V-cycle) */
    int device;           /* HIP device ordinal */
    int max_coarse_dofs;  /* coarsening threshold; 0 selects 256 */
} mlb_batch_desc;

typedef struct {
    int smooth_steps;     /* V(nu, nu) Jacobi sweeps, default 2 */
    double jacobi_omega;  /* omega_j = jacobi_omega / (1.05 rho(D^-1 A_j)), default 4/3 */
    int queue;            /* 0: one block per work item, the hardware dispatcher
                             is the queue (default); 1: persistent grid draining
                             8 XCD-local atomic queues with stealing (same
                             results bit for bit, slower for these uniform
                             256-node items: every block pays one round trip
                             per ticket on contended counters) */
    int graphs;           /* 1: capture one CG iteration as a HIP graph (default) */
    int check_every;      /* iterations between host convergence reads, default 4 */
    int refine_steps;     /* iterative-refinement steps after the solve, 0..16, default 10 (0: none);
                             see mlb_batch_solve_dev */
} mlb_batch_opts;

typedef struct {
    int max_iterations;       /* largest CG iteration count over the instances */
    int total_iterations;     /* sum over the instances */
    int batch_iterations;     /* batched iterations launched */
    int converged;            /* instances whose CG met the tolerance (recursive residual) */
    double worst_true_rel_res;/* max_i ||f_i - K_i u_i|| / ||f_i|| (free DOFs) of the returned FP64 u,
                                 evaluated in double-double */
    double setup_s;           /* wall time of the last mlb_batch_set_problem_dev */
    double solve_s;           /* wall time of the last solve */
    int refine_steps;         /* refinement steps taken */
    int misses;               /* instances whose true residual stays above tol */
    double worst_floor;       /* largest FP64 floor eps ||(|K_i||u_i|)|| / ||f_i|| among the misses */
    double worst_refined_rel_res; /* the same for the double-double solution the returned u rounds */
} mlb_batch_info;

/* Creates a batch for the grids in desc; allocates all device memory. */
int mlb_batch_create(const mlb_batch_desc* desc, mlb_batch** out);
void mlb_batch_destroy(mlb_batch* b);
const char* mlb_batch_last_error(const mlb_batch* b);
int mlb_batch_set_opts(mlb_batch* b, const mlb_batch_opts* o);
int mlb_batch_get_opts(const mlb_batch* b, mlb_batch_opts* o);

/* dof_off[ninst+1], elem_off[ninst+1] (prefix sums as above) and the number
   of multigrid levels of every instance, levels[ninst]; any may be NULL. */
int mlb_batch_layout(const mlb_batch* b, int64_t* dof_off, int64_t* elem_off, int* levels);

/* Sets every instance's problem at once from device arrays in the batched
   layout: fixed[dof_off[ninst]] (1 = clamped DOF), F[dof_off[ninst]] (one
   load case each), x[elem_off[ninst]] (densities in [0, 1]).  Builds the
   SIMP moduli, all hierarchies and Jacobi weights, and the coarsest
   inverses.  MLB_EINVAL for densities outside [0, 1] or NaN. */
int mlb_batch_set_problem_dev(mlb_batch* b, const uint8_t* fixed, const double* F, const double* x, void* stream);

/* Solves K_i u_i = f_i for every instance by FP64 CG preconditioned with one
   V-cycle per iteration, each to ||f_i - K_i u_i|| <= tol ||f_i|| (free
   DOFs, recursive residual).  Then up to refine_steps steps of iterative
   refinement of a double-double solution u_hi + u_lo: its true residual in
   double-double (error-free products and sums), a batched correction solve
   to 1e-4 relative, u += correction in double-double; an instance is done at
   a residual below tol / 100, and the steps stop when all are done or none
   of the others lowers its residual by 10 % in a step.  The returned u is
   fl(u_hi + u_lo), the double nearest to the refined solution.
   Near-singular designs (tiny moduli over large regions, displacements
   orders of magnitude above their strain parts) can have an FP64 floor
   above tol: rounding u to doubles alone moves the residual by about
   eps ||(|K||u|)|| / ||f||, so no FP64 u meets tol there, even the rounded
   exact solution; such instances are counted in info->misses, and every
   instance's residuals (returned u, refined solution) and floor come from
   mlb_batch_residuals.
   U: device [dof_off[ninst]] (output; zero start).  J: host [ninst]
   compliances f_i^T u_i, iters: host [ninst] iteration counts of all CG
   passes (either may be NULL).  MLB_ENOTCONV if an instance needs more than
   max_it iterations, MLB_EBREAKDOWN on p^T K p <= 0. */
int mlb_batch_solve_dev(mlb_batch* b, double tol, int max_it, double* U, double* J, int* iters,
                        mlb_batch_info* info, void* stream);

/* Per-instance results of the last solve (host arrays of ninst, any may be
   NULL): res[i] = ||f_i - K_i u_i|| / ||f_i|| of the returned u, evaluated
   in double-double; floor[i] = eps ||(|K_i||u_i|)|| / ||f_i|| (free DOFs),
   the residual that rounding u_i to doubles alone can cause; res_refined[i]
   the residual of the double-double solution u_i rounds.  MLB_ESTATE before
   a solve. */
int mlb_batch_residuals(const mlb_batch* b, double* res, double* floor, double* res_refined);

/* Compliance sensitivities dJ_i/dx_e = -p x_e^(p-1) (E1 - E0) u_e^T K0 u_e of
   the last solve, device [elem_off[ninst]]. */
int mlb_batch_compliance_sens_dev(mlb_batch* b, double* dJ, void* stream);

#ifdef __cplusplus
}
#endif

#endif
