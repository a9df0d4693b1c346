/* Optimisation layer of the multilevel buckling library: the pieces that
 * turn the analysis of mlb.h into the paper's design problems
 *   P1 (Sec. 3): minimum compliance s.t. lowest buckling factors >= lambda_bar
 *                and volume fraction <= f_bar;
 *   P2 (Sec. 6): minimum volume s.t. lowest buckling factors >= lambda_bar and
 *                compliance <= J_max.
 * Continuation of the SIMP exponent and of the projection sharpness, the bound
 * formulation of the buckling constraint (Sec. 3) and the method of moving
 * asymptotes (MMA, Svanberg 1987), whose per-element work runs on the GPU.
 *
 * Conventions as in mlb.h: status codes MLB_*, device pointers are HIP device
 * memory owned by the caller, `stream` is a hipStream_t (NULL: the default
 * stream).  Every *_dev call here synchronises its stream before returning
 * (each reads a few reductions back to the host). */
#ifndef MLB_OPT_H
#define MLB_OPT_H

#include <stdint.h>

#include "mlb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- continuation (Secs. 3 and 6) --------------------------------------- */

/* SIMP exponent and projection sharpness at design step `step` (0, 1, ...):
 *   p = min(p0 + dp floor(step / p_every), p_max);
 *   k_p = first step with p = p_max;  beta = beta0 before k_p + beta_every,
 *   then doubled every beta_every steps, at most beta_max
 *   (beta_every = 0: beta stays beta0).
 * Sec. 3 uses (1, 0.25, 25, 6, 6, 0, -); Sec. 6 uses (3, 0.25, 25, 6, 1, 50, 32).
 * Host only.  MLB_EINVAL for step < 0, dp <= 0, p_every < 1, p_max < p0,
 * beta0 <= 0, beta_every < 0, or beta_max < beta0 when beta_every > 0. */
int mlb_continuation(int step, double p0, double dp, int p_every, double p_max, double beta0, int beta_every,
                     double beta_max, double* p, double* beta);

/* ---- problem functions in MMA form (Secs. 3 and 6) ---------------------- */

/* Bound formulation of the buckling constraint (Sec. 3), read as the lower
 * bounds lambda_i >= lambda_bar alpha^-i (the printed form flips the sign;
 * this reading keeps the stated gap between bounds and makes the section's
 * coalescence measure vanish on the bounds):
 *   g_i = 1 - alpha^i lambda_i / lambda_bar,  i = 1 .. nb.
 *
 * mlb_p1_functions_dev (P1): f0 = J / J0;
 *   fval = [mean(x) / f_bar - 1, g_1 .. g_nb];
 *   grad columns (device, (2 + nb) x m, column c at c m):
 *     [dJ / J0, 1 / (m f_bar), -(alpha^i / lambda_bar) dlam_i].
 * mlb_p2_functions_dev (P2): f0 = mean(x);
 *   fval = [J / J_max - 1, g_1 .. g_nb];
 *   grad columns: [1 / m, dJ / J_max, -(alpha^i / lambda_bar) dlam_i].
 * x, dJ: device, m doubles; dlam: device, nb columns of m at stride ld (the
 * layout mlb_sensitivities_dev writes, ld = m); lam: host, nb doubles; f0,
 * fval: host outputs (1, 1 + nb).  1 <= nb <= 30.  Synchronises `stream`
 * (the volume is a device reduction). */
int mlb_p1_functions_dev(int64_t m, int nb, const double* x, double J, const double* dJ, const double* lam,
                         const double* dlam, int64_t ld, double J0, double lam_bar, double f_bar, double alpha,
                         double* f0, double* fval, double* grad, void* stream);
int mlb_p2_functions_dev(int64_t m, int nb, const double* x, double J, const double* dJ, const double* lam,
                         const double* dlam, int64_t ld, double J_max, double lam_bar, double alpha, double* f0,
                         double* fval, double* grad, void* stream);

/* ---- method of moving asymptotes ---------------------------------------- */

/* Options (zero fields take the defaults in brackets). */
typedef struct {
    double xmin;      /* lower bound of every variable [0] (used only when xmax > xmin) */
    double xmax;      /* upper bound [1] */
    double move;      /* move limit as a fraction of xmax - xmin [0.2] */
    double asyinit;   /* initial asymptote distance [0.5] */
    double asyincr;   /* asymptote widening where a variable keeps its direction [1.2] */
    double asydecr;   /* narrowing where it reverses [0.7] */
    double c;         /* linear cost of the elastic variables y_i [1000] */
    double d;         /* quadratic cost of y_i [1] */
} mlb_mma_opts;

typedef struct {
    int dual_iterations;   /* Newton steps of the dual subproblem solve */
    int dual_evaluations;  /* dual function evaluations (one device pass each) */
    double proj_grad;      /* final projected dual gradient (max norm) */
    double dual_value;     /* final dual value */
    double lam[32];        /* subproblem multipliers (first m used) */
    double y[32];          /* elastic variables (first m used) */
    double seconds;        /* wall time of the update */
} mlb_mma_info;

typedef struct mlb_mma mlb_mma;

/* One MMA instance for n variables and m <= 32 constraints on HIP device
 * `device` (the device current at the update calls must be this one).  It
 * owns the iteration history (x^(k-1), x^(k-2)), the asymptotes and device
 * work space of about (m + 7) n doubles. */
int mlb_mma_create(int64_t n, int m, const mlb_mma_opts* opts, int device, mlb_mma** out);
void mlb_mma_destroy(mlb_mma* h);
const char* mlb_mma_last_error(const mlb_mma* h);

/* One design update (Svanberg 1987): min f_0(x) s.t. f_i(x) <= 0 (i = 1..m),
 * xmin <= x <= xmax, from the current point x^k.
 *   x:    device, n doubles: x^k in, x^(k+1) out;
 *   f0:   objective value; df0: device, n doubles, its gradient;
 *   fval: host, m constraint values; dfdx: device, m rows of n at stride ldg
 *         (row i at i ldg, ldg >= n), their gradients.
 * Convex separable approximations around x^k (the regularised coefficients
 * of Svanberg's later notes, exact value and gradient at x^k), asymptotes
 * from the last two steps, move limits, and the subproblem with elastic
 * variables solved exactly through its dual: damped projected Newton steps
 * on the m multipliers, the per-variable minimisers and the dual sums on the
 * device (the dual Hessian as a tall-skinny Gram product).  info may be
 * NULL.  The dual solve stops at a projected gradient below
 * 1e-13 (1 + max |r_i|) (r_i the approximations' constants), or when no
 * damped step raises the dual value (its sums' rounding floor) with the
 * projected gradient below 1e-9 (1 + max |r_i|).  MLB_EINVAL for sizes or
 * non-finite inputs, MLB_ENOTCONV if it stalls above that (x then holds the
 * last dual iterate's minimiser, still inside the move limits). */
int mlb_mma_update_dev(mlb_mma* h, double* x, double f0, const double* df0, const double* fval, const double* dfdx,
                       int64_t ldg, mlb_mma_info* info, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MLB_OPT_H */
