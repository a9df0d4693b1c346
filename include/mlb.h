/*
 * mlb.h - C ABI of the MI355X multilevel linearized-buckling engine.
 *
 * The calls follow the analysis the paper performs for every design
 * (Ferrari & Sigmund, "Towards solving large-scale topology optimization
 * problems with buckling constraints at the cost of linear analyses"):
 *   Alg. 1       set a reference load, solve K[x] u = f, set up G[x, u],
 *                compute the lowest buckling pairs (K + lambda G) phi = 0;
 *   Sec. 2.1     multilevel approximation of those pairs: Galerkin coarse
 *                eigenproblem, interpolation of the coarse modes to the fine
 *                grid, one fine block solve K Phi~ = G Psi, Rayleigh-Ritz;
 *   Sec. 2       SIMP interpolations E_kappa = E0 + x^p (E1 - E0),
 *                E_sigma = x^p E1 (eq. interpolationSIMP2-SIMP), modes
 *                normalised phi_i^T K phi_j = delta_ij;
 *   eqs. SensitivityLambda, AdjointSystem
 *                buckling-factor sensitivities with one adjoint solve per
 *                mode; compliance J = f^T u (Sec. 3) and its gradient.
 *
 * Discretisation: regular grid of unit Q4 (dim 2, plane stress, unit
 * thickness) or H8 (dim 3) elements, nel = (nx, ny[, nz]).
 *   node index  node = i + (nx+1)*(j + (ny+1)*k)        (x fastest)
 *   DOF index   dof  = dim*node + c                     (interleaved)
 *   element     e    = i + nx*(j + ny*k)
 *   blocks      column-major, leading dimension n (DOFs) or m (elements).
 * Vectors are full length, Dirichlet DOFs included (they hold zero in every
 * solution and mode).  Level 1 is the fine grid; level j has nel / 2^(j-1)
 * elements per axis, so every nel[i] must be divisible by 2^(levels-1).
 *
 * Ownership: the caller owns every pointer it passes.  The library copies
 * inputs before returning (host calls) or before the enqueued work completes
 * (device calls) and never keeps a caller pointer.  Device work memory is
 * owned by the context and freed by mlb_destroy.
 *
 * Errors: every call returns an int status, MLB_OK (0) or a negative code;
 * mlb_last_error() gives a message for the last failure on that context.
 * A context is used by one host thread at a time.
 *
 * Streams: *_dev calls take device pointers and a hipStream_t passed as
 * void* (NULL = the context's own stream).  Kernel-level *_dev calls only
 * enqueue work.  Solver calls (static, buckling, sensitivities) synchronise
 * the stream they run on, because convergence is decided on the host.
 */
#ifndef MLB_H
#define MLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MLB_OK          0
#define MLB_EINVAL     -1   /* bad argument: sizes, NaN/Inf, density outside [0,1] */
#define MLB_ESTATE     -2   /* call order: e.g. buckling before a static solve */
#define MLB_ENOMEM     -3   /* device allocation failed */
#define MLB_EDEVICE    -4   /* HIP runtime error */
#define MLB_ENOTCONV   -5   /* iteration limit reached; outputs hold the last iterate */
#define MLB_ENOPOS     -6   /* fewer than k positive buckling factors */
#define MLB_EBREAKDOWN -7   /* CG breakdown (p^T K p <= 0) or singular Gram matrix */

/* element of mlb_desc */
#define MLB_ELEM_CONFORMING   0
#define MLB_ELEM_INCOMPATIBLE 1

/* precision of the preconditioner (the outer Krylov solvers are FP64) */
#define MLB_FP64   0
#define MLB_MIXED  1        /* FP32 V-cycle; FP64 outer CG, coarsest solve, Rayleigh-Ritz */

/* warm-start kinds for mlb_set_warm_start */
#define MLB_WARM_NONE    0
#define MLB_WARM_COARSE  1  /* start block for the coarse eigensolve */
#define MLB_WARM_STATIC  2  /* initial guess for the static solve */

typedef struct mlb_ctx mlb_ctx;

/* Result of mlb_autotune: the chosen tile parameters and the mean time (ms)
   of a Jacobi sweep for each candidate (z chunk 4, 6, 8, 10, 12; stencil
   columns per thread 2, 3, 4, 6, 12; 3D fine-apply variant 0 = register tiles
   of 8 x 8 element columns per wave prefetching the next node plane, 1 =
   16 x 16 tiles staged in LDS, 2 = register tiles without prefetch, 3 = the
   register tiles of variant 0 with each node plane transformed once, plane
   contributions summed in the transformed basis and range-checked buffer
   accesses; levels whose vectors exceed 1 GiB run variant 0 instead).  The
   first fields describe the apply in the precision of the multigrid cycle,
   the wht64_* fields the FP64 apply of the outer solvers (tuned separately
   in mixed precision on plain products K x, the only FP64 use of the fine
   apply there; equal to the first ones otherwise). */
typedef struct {
    int wht_zchunk;
    int stencil_cols;
    float wht_ms[5];
    float stencil_ms[5];
    int wht_variant;
    float wht_lds_ms[5];
    float wht_nopf_ms[5];
    int wht64_zchunk;
    int wht64_variant;
    float wht64_ms[5];
    float wht64_lds_ms[5];
    float wht64_nopf_ms[5];
    float wht_v3_ms[5];
    float wht64_v3_ms[5];
    /* score of candidate (variant v, z chunk i) at [5 v + i]: one
       ncols-column plus one single-column sweep (ms); the chosen tile has
       the smallest (3D: 4 variants; 2D: variant 0 only) */
    float wht_score_ms[20];
    float wht64_score_ms[20];
} mlb_tune_info;

/* Problem description (copied by mlb_create). */
typedef struct {
    int dim;            /* 2 (Q4) or 3 (H8) */
    int nel[3];         /* elements per axis; nel[2] ignored when dim == 2 */
    double E1;          /* solid Young modulus (Sec. 2) */
    double E0;          /* void modulus in E_kappa only; E_sigma has no floor */
    double nu;          /* Poisson ratio */
    double penal;       /* SIMP exponent p */
    int mg_levels;      /* geometric multigrid levels, >= 1 (1: Jacobi-PCG) */
    int eig_level;      /* level l of the coarse eigenproblem, 1..mg_levels */
    int precision;      /* MLB_FP64 or MLB_MIXED */
    int device;         /* HIP device ordinal */
    int element;        /* MLB_ELEM_CONFORMING (bilinear Q4 / trilinear H8, the default) or
                           MLB_ELEM_INCOMPATIBLE (the paper's Q6 / H11, Sec. 2: one mode
                           4 x_m (1 - x_m) per axis and component, condensed out of K_e0;
                           G_e0 and the centroid stress keep the nodal interpolation) */
} mlb_desc;

/* Solver options (mlb_set_opts); zero fields keep their defaults. */
typedef struct {
    int smooth_steps;     /* Jacobi sweeps before and after the coarse correction (default 2) */
    double jacobi_omega;  /* damping factor times rho(D^-1 A); default 4/3 (omega = 4/(3 rho)) */
    int eig_guard;        /* extra vectors in the coarse eigensolver block (default max(4, k/2)) */
    int eig_max_it;       /* coarse eigensolver iteration limit (default 400) */
    int check_every;      /* CG iterations between host reads of the device convergence flags (default 8;
                             results do not depend on it) */
    uint64_t seed;        /* seed of the coarse eigensolver start block (default 1) */
    int cycle;            /* coarse-grid visits per level: 1 = V-cycle, 2 = W-cycle (default 1) */
    int block_cg;         /* multi-column solves: 1 = block CG (default), 2 = column-wise CG */
    int eig_sweeps;       /* multigrid sweeps per coarse-eigensolver preconditioner application (default 3) */
    int graphs;           /* 1 = replay each multigrid cycle as a captured HIP graph (default), 2 = launch eagerly */
    int pinvit_steps;     /* preconditioned inverse iteration steps on the fine modes after their
                             Rayleigh-Ritz (App. A, eq. PInvIt-GeneralInteration): each Ritz vector
                             takes phi_i <- phi_i - M^-1 (K + lam~_i G) phi_i with M^-1 one multigrid
                             cycle of the static solves and lam~_i its Ritz value, then the block is
                             replaced by its Ritz vectors again.  > 0 sets the count (at most 64),
                             < 0 sets none (the default), 0 keeps the current value */
    int refine_sweeps;    /* intermediate-level refinement of Alg. 2: on every level l-1 .. 2 the
                             prolonged modes take this many Kaczmarz sweeps on
                             (K^j + sigma_j G^j) psi = 0, sigma_j the smallest Ritz value of the
                             coarser level, and are replaced by their level-j Ritz vectors.  Rows
                             are visited by colour (i mod 3) + 3 (j mod 3) + 9 (k mod 3), then by
                             component.  > 0 sets the count (at most 16), < 0 sets none (the
                             default: the main text's method), 0 keeps the current value */
    int coarse_sweeps;    /* Jacobi sweeps before and after the coarse correction on levels >= 3,
                             where sweeps are cheap (> 0 sets it, at most 64; default: smooth_steps) */
    int pinvit_shift;     /* shift of the inverse iteration steps: 1 = each Ritz vector's own Ritz value
                             (the default: the gradient step of its Rayleigh quotient), 2 = lam~_1 for
                             every vector (the step as printed in App. A); 0 keeps the current value */
    int refine_fine;      /* with refine_sweeps: 1 = the refinement loop also visits the fine grid (Alg. 2's
                             loop is printed down to it): the prolonged modes take the sweeps on
                             (K + sigma G) psi = 0 with assembled fine stencils of K and G (about
                             (dim 3^dim)^2 + 3^dim doubles per node, allocated on first use) and a fine
                             Ritz step before the block solve; < 0 = not (the default); 0 keeps */
} mlb_opts;

/* Per-call solver report; for blocks, the worst column is reported. */
typedef struct {
    int iterations;             /* CG iterations of the last solve */
    int converged;              /* 1 if every column met the tolerance */
    double rel_residual;        /* recursive ||r|| / ||b|| at exit */
    double true_rel_residual;   /* ||b - K x|| / ||b|| recomputed at exit */
    double seconds;             /* wall time of the call */
} mlb_solve_info;

typedef struct {
    int coarse_iterations;      /* coarse eigensolver iterations */
    double coarse_residual;     /* max relative residual of the coarse pairs */
    double coarse_gap;          /* (mu_k - mu_{k+1}) / mu_k at the coarse level */
    int fine_iterations;        /* CG iterations of the fine block solve K Phi~ = G Psi */
    double fine_true_residual;  /* worst true relative residual of that solve */
    double seconds_coarse;      /* Galerkin operators + coarse eigensolve */
    double seconds_fine;        /* interpolation + fine block solve */
    double seconds_ritz;        /* Rayleigh-Ritz + residuals */
    int coarse_warm_used;       /* 1 if a MLB_WARM_COARSE block started the coarse eigensolve
                                   (it is dropped for the plain start when its initial Ritz
                                   residual is worse or the block is rank deficient) */
    int pinvit_steps;           /* preconditioned inverse iteration steps taken (mlb_opts) */
    double lambda1_before_pinvit; /* lam~_1 of the first Rayleigh-Ritz, before those steps */
    double seconds_pinvit;      /* wall time of those steps */
    int refine_levels;          /* intermediate levels refined (mlb_opts.refine_sweeps) */
    double refine_lambda1[8];   /* smallest Ritz value on each of them, level l-1 first */
    double seconds_refine;      /* wall time of the sweeps and Ritz steps */
    int coarse_guard_fired;     /* 1 if the coarse eigensolver stopped above tol_eig because its
                                   residual had stalled (accepted only below sqrt(tol_eig));
                                   coarse_residual then holds the residual reached */
} mlb_eig_info;

/* ---- lifetime --------------------------------------------------------- */

/* Creates a context on desc->device: element tables, grid hierarchy and
 * device work buffers.  EINVAL for bad sizes or levels; ENOMEM/EDEVICE. */
int mlb_create(const mlb_desc* desc, mlb_ctx** out);
void mlb_destroy(mlb_ctx* ctx);
const char* mlb_last_error(const mlb_ctx* ctx);
int mlb_set_opts(mlb_ctx* ctx, const mlb_opts* opts);
/* Sizes: DOFs and elements of level `level` (1 = fine). */
int mlb_level_size(const mlb_ctx* ctx, int level, int64_t* n_dofs, int64_t* n_elems);

/* ---- problem data (Alg. 1, reference load; Sec. 2) ------------------------------ */

/* Dirichlet mask, one byte per DOF (nonzero = fixed).  The fixed set must be
 * nested: every fixed fine DOF may interpolate only from fixed coarse DOFs
 * (true for clamped faces/edges); otherwise EINVAL. */
int mlb_set_bc(mlb_ctx* ctx, const uint8_t* fixed);
int mlb_set_bc_dev(mlb_ctx* ctx, const uint8_t* fixed, void* stream);
/* Load cases F (n x ncases, column-major).  Entries at fixed DOFs are ignored. */
int mlb_set_loads(mlb_ctx* ctx, int ncases, const double* F);
int mlb_set_loads_dev(mlb_ctx* ctx, int ncases, const double* F, void* stream);
/* Physical densities x (m), each in [0, 1] (EINVAL otherwise, or NaN).
 * Builds the multigrid hierarchy for K[x]; invalidates previous solutions. */
int mlb_set_density(mlb_ctx* ctx, const double* x);
int mlb_set_density_dev(mlb_ctx* ctx, const double* x, void* stream);

/* ---- analysis -------------------------------------------------------- */

/* LA (Alg. 1, static solve): U = K^-1 F for every load case by multigrid-
 * preconditioned CG to ||F - K U|| <= tol ||F|| per column; J = f^T u.
 * U (n x ncases) and J (ncases) may be NULL.  ENOTCONV after max_it. */
int mlb_solve_static(mlb_ctx* ctx, double tol, int max_it, double* U, double* J,
                     mlb_solve_info* info);
int mlb_solve_static_dev(mlb_ctx* ctx, double tol, int max_it, double* U, double* J_host,
                         mlb_solve_info* info, void* stream);

/* EA by the multilevel procedure (Sec. 2.1 steps 1-4) for load case
 * ref_case: G[x, u] from that case, Galerkin K^l, G^l, lowest k positive
 * coarse pairs to relative residual tol_eig, interpolation to the fine
 * grid, K Phi~ = G Psi to relative residual `tol_solve` (set by
 * mlb_solve_static's tol), Rayleigh-Ritz.  lambda (k, ascending) and Phi
 * (n x k, K-normalised, largest-magnitude entry positive) may be NULL.
 * With eig_level == 1 the eigensolve runs on the fine grid (exact pairs).
 * ESTATE without a converged static solve; ENOPOS if fewer than k
 * positive factors exist; ENOTCONV if the coarse eigensolver stalls above
 * sqrt(tol_eig) or reaches its iteration limit above tol_eig; EBREAKDOWN if a
 * Gram matrix of the eigensolver is not finite or not positive. */
int mlb_buckling(mlb_ctx* ctx, int ref_case, int k, double tol_eig, double* lambda,
                 double* Phi, mlb_eig_info* info);
int mlb_buckling_dev(mlb_ctx* ctx, int ref_case, int k, double tol_eig, double* lambda_host,
                     double* Phi, mlb_eig_info* info, void* stream);

/* Residual norms ||(K + lambda_i G) phi_i||_inf of the last buckling call
 * (eq. eigResidual); res_inf has k entries (host). */
int mlb_eig_residuals(mlb_ctx* ctx, double* res_inf);
/* The same norms into device memory res_inf (k doubles), enqueued on `stream`
 * (they stay valid until the next mlb_buckling*). */
int mlb_eig_residuals_dev(mlb_ctx* ctx, double* res_inf, void* stream);

/* Sensitivities w.r.t. the physical densities (no filter/projection):
 * dJ (m x ncases) = -p x^(p-1) (E1-E0) u_e^T K_e0 u_e; dlam (m x k) for the
 * pairs of the last buckling call:
 *   dlam_i/dx_e = lam_i [phi_i^T K'_e phi_i + lam_i (phi_i^T G'_e phi_i - z_i^T K'_e u)]
 * with K z_i = grad_u(phi_i^T G phi_i) solved as one block (eq. AdjointSystem).
 * (eq. SensitivityLambda times lam_i, the factor the normalisation
 * phi^T K phi = 1 implies.)  Either output may be NULL; ESTATE if dlam is
 * requested before mlb_buckling. */
int mlb_sensitivities(mlb_ctx* ctx, double* dJ, double* dlam, mlb_solve_info* info);
int mlb_sensitivities_dev(mlb_ctx* ctx, double* dJ, double* dlam, mlb_solve_info* info,
                          void* stream);

/* Consistent sensitivities of the multilevel factors (appendix on numerical
 * procedures, eq. consistentSensitivity, with the residual y_i = (K +
 * lam~_i G) phi~_i of eq. eigResidual).  Printed literally, that formula's
 * adjoint -2 (K + lam~ G)^-1 y equals -2 phi~ and the formula reduces to the
 * plain one; here it is the derivative of what the method computes:
 * lam~_i(x) = i-th Ritz value of span(K^-1 G[x, u(x)] Psi) with the
 * interpolated coarse modes Psi held fixed:
 *   dlam_i/dx_e = lam [phi^T K'_e phi + lam (phi^T G'_e phi - zt^T K'_e u)]
 *                 + 2 lam (w^T G'_e psi - w^T K'_e phi),
 *   w = K^-1 y_i,  K zt = grad_u(phi^T G phi) + (2 / lam) grad_u(w^T G psi),
 * psi = the combination of Psi with K phi = G psi.  Two block solves of k
 * columns (tolerance of mlb_solve_static).  dlam: m x k (host / device).
 * ESTATE before mlb_buckling or after one with inverse-iteration steps
 * (mlb_opts.pinvit_steps), whose modes are not of that form.  Afterwards
 * mlb_adjoints_dev returns zt. */
int mlb_sensitivities_consistent(mlb_ctx* ctx, double* dlam, mlb_solve_info* info);
int mlb_sensitivities_consistent_dev(mlb_ctx* ctx, double* dlam, mlb_solve_info* info, void* stream);

/* Tile parameters of the fine apply (pencil length in node planes, 1..64;
   3D variant 0..3 as in mlb_tune_info, -1 keeps it) and of the stencil
   applies (columns per thread, 1..12); 0 keeps a value; both precisions are
   set.  For a given variant the operator applies give bitwise the same
   results for every pencil length and column count; variants 0 and 2 agree
   bitwise, variants 1 and 3 sum a node's element contributions in other
   orders (results agree to rounding).  Dot products fused into the fine apply group their partial
   sums by tile, so solver iterates may differ in the last bits. */
int mlb_set_tiles(mlb_ctx* ctx, int wht_zchunk, int stencil_cols, int wht_variant);
/* Jacobi weights omega_j of the multigrid smoother on levels 1 .. nlevels
   (nlevels <= the number of levels - 1; the coarsest level is solved
   exactly).  mlb_set_density* estimates them as jacobi_omega / (1.05 rho_j)
   with rho_j from 12 power iterations on D_j^-1 A_j; mlb_set_omegas replaces
   them (each in (0, 2 / rho_j) for a convergent smoother) until the next
   mlb_set_density*, so that a cycle can be reproduced exactly elsewhere.
   MLB_ESTATE before the densities are set, MLB_EINVAL for a weight that is
   not positive and finite. */
int mlb_set_omegas(mlb_ctx* ctx, int nlevels, const double* omega);
int mlb_get_omegas(const mlb_ctx* ctx, int nlevels, double* omega);
/* Times Jacobi sweeps of ncols (<= 32) columns on the current hierarchy for
   each candidate tile and keeps the fastest (needs mask and densities); a
   fine-apply candidate is scored by one ncols-column sweep plus one
   single-column sweep (the solvers run both about equally often), and the
   times reported are the ncols-column ones. */
int mlb_autotune(mlb_ctx* ctx, int ncols, mlb_tune_info* info, void* stream);

/* Warm starts.  kind MLB_WARM_COARSE: `data` holds ncols start vectors of
 * the eigen level (n_l x ncols, column-major, host); MLB_WARM_STATIC: one
 * fine initial guess per load case (n x ncases, host), scaled per column
 * by alpha = f^T u0 / u0^T K u0 before the solve.  MLB_WARM_NONE clears both.
 * A warm start only changes iteration counts, never the tolerance the
 * solvers reach.  A coarse block is used only if the worst initial Ritz
 * residual of the wanted pairs is no larger than that of the random start
 * block.  The context keeps its warm-start buffers between calls and
 * reallocates only to grow them (MLB_WARM_NONE frees them). */
int mlb_set_warm_start(mlb_ctx* ctx, int kind, int ncols, const double* data);
/* The same from device memory: `data` is copied on `stream` into the
 * context's buffers (no host round trip), so a prediction computed on the
 * device can start the solvers directly.  At most 64 coarse or 32 static
 * columns. */
int mlb_set_warm_start_dev(mlb_ctx* ctx, int kind, int ncols, const double* data, void* stream);

/* ---- kernel-level entry points (device pointers, enqueue only) -------- */

/* y = A x on level `level` for ncols columns (leading dimension n_level),
 * A = K (identity rows/columns at fixed DOFs).  Level 1 is matrix-free;
 * levels > 1 use the Galerkin element matrices built by mlb_set_density. */
int mlb_apply_K_dev(mlb_ctx* ctx, int level, int ncols, const double* x, double* y, void* stream);
/* y = G x (zero rows/columns at fixed DOFs) for the stress state of the
 * last mlb_set_state_dev / static solve; levels > 1 after mlb_buckling. */
int mlb_apply_G_dev(mlb_ctx* ctx, int level, int ncols, const double* x, double* y, void* stream);
/* Sets the reference displacement u (n, device) used for G[x, u]; computes
 * element stresses E_sigma(x_e) D0 B_c u_e (centroid), stored SoA (m x nv)
 * into `stress_out` when non-NULL. */
int mlb_set_state_dev(mlb_ctx* ctx, const double* u, double* stress_out, void* stream);
/* Interpolation from level+1 to level (y = P x) and restriction (y = P^T x)
 * of ncols columns, masked at fixed DOFs of both levels. */
int mlb_prolong_dev(mlb_ctx* ctx, int level, int ncols, const double* xc, double* yf, void* stream);
int mlb_restrict_dev(mlb_ctx* ctx, int level, int ncols, const double* xf, double* yc, void* stream);
/* The K^l-orthonormal coarse modes Psi^l (n_l x k, column-major) of the last
   mlb_buckling (Sec. 2.1 step 1), e.g. as training targets of a warm start. */
int mlb_coarse_modes_dev(mlb_ctx* ctx, int k, double* Psi, void* stream);
/* The adjoint solutions z_i of K z_i = grad_u(phi_i^T G phi_i) (eq. AdjointSystem),
   n x k column-major, from the last mlb_sensitivities with dlam requested. */
int mlb_adjoints_dev(mlb_ctx* ctx, int k, double* Z, void* stream);
/* The adjoint right-hand sides b_i = grad_u(phi_i^T G phi_i) (n x k) of the
   last mlb_sensitivities with dlam requested. */
int mlb_adjoint_rhs_dev(mlb_ctx* ctx, int k, double* B, void* stream);

/* K X = B for ncols <= 32 arbitrary right-hand sides (n x ncols, device) on the
   current density, as one block CG (App. B, block mgPCG) from X = 0, to the
   relative residual tol per column.  B is masked at Dirichlet DOFs; X receives
   zeros there.  Invalidates the adjoint accessors. */
int mlb_solve_block_dev(mlb_ctx* ctx, int ncols, const double* B, double* X, double tol, int max_it,
                        mlb_solve_info* info, void* stream);

/* `reps` damped-Jacobi sweeps x <- x + omega_j D^-1 (r - A x) of the multigrid
 * cycle on level `level` (1 .. levels - 1) for ncols <= 32 columns, in the
 * cycle's precision (FP32 in MLB_MIXED), on the level's own work blocks
 * (zeroed on first use): the smoother kernel exactly as a cycle launches it,
 * for timing it on `stream`.  Enqueue only. */
int mlb_sweep_dev(mlb_ctx* ctx, int level, int ncols, int reps, void* stream);

/* One multigrid V-cycle z = M^-1 r starting at `level` (ncols columns). */
int mlb_vcycle_dev(mlb_ctx* ctx, int level, int ncols, const double* r, double* z, void* stream);

/* ---- post-processing measures of local buckling (Sec. 5) -------------- */

/* Energy-weighted modal correlation (eq. macCorrelationIndex):
 *   C[j + qa r] = a_j^T K b_r,  j < qa, r < qb
 * with K the fine stiffness of the current densities, identity rows/columns
 * at fixed DOFs (the operator of mlb_apply_K_dev).  For modes normalised to
 * a^T K a = b^T K b = 1 (as mlb_buckling returns them) |C| <= 1, 1 for equal
 * modes, 0 for K-orthogonal ones; the sign follows the modes' signs.
 * A (n x qa), B (n x qb): device, column-major, read only.  W: device
 * workspace n x qb, caller-owned, overwritten with K B; it must not overlap
 * B.  C_host: host, qa x qb column-major.  Synchronises the stream.
 * MLB_EINVAL if qa + qb > 192 or qa qb > 96 x 192, MLB_ESTATE before the
 * mask and the densities are set. */
int mlb_mac_dev(mlb_ctx* ctx, int qa, const double* A, int qb, const double* B, double* W, double* C_host,
                void* stream);

/* Strain energy density, its gradient and total variation (eq. TVsed) of q
 * modes Phi (n x q, device, column-major):
 *   sed[i m + e]   = E_kappa(x_e) phi_{i|e}^T K_e0 phi_{i|e}
 *   gradn[i m + e] = |grad sed_i| at element e on the solid set
 *                    {x_e >= xbar}, 0 elsewhere
 *   tv_host[i]     = sum of gradn[i m + e] over the solid set (unit cells)
 * The gradient of the element-constant density uses differences between
 * neighbouring solid elements only, per axis central when both neighbours
 * are solid, one-sided when one is, none when neither is; so a density
 * constant on the solid set has zero variation.  x is the density of the
 * last mlb_set_density*, K_e0 the context's element.  sed, gradn: device
 * q x m, caller-owned.  tv_host: host q doubles, or NULL (then nothing
 * synchronises).  MLB_ESTATE before the densities are set. */
int mlb_sed_tv_dev(mlb_ctx* ctx, int q, const double* Phi, double xbar, double* sed, double* gradn,
                   double* tv_host, void* stream);

/* Local dilation of densities (eq. postProcessingDilation):
 *   xout_e = max(x_e, max { x_k : |c_k - c_e| <= r_th, k flagged })
 * with c the element centroids (unit cells) and k flagged when, for some
 * selected mode s < nsel, gradn[s m + k] >= rel_thr * max_e gradn[s m + e]
 * (and that maximum is positive).  gradn: device nsel x m, non-negative
 * (rows of mlb_sed_tv_dev's gradn); x, xout: device m, distinct; r_th in
 * [0, 8], rel_thr >= 0.  Enqueue only. */
int mlb_dilate_dev(mlb_ctx* ctx, int nsel, const double* gradn, double rel_thr, double r_th, const double* x,
                   double* xout, void* stream);

/* mlb_dilate_dev for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, with the partial maxima in
 * a fixed per-GPU scratch array of the library (525 KiB, held until the
 * process ends) instead of the context's growable buffers.  It calls no
 * allocating routine.  nsel <= 64 (MLB_EINVAL above).  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other contexts, other threads) race; calls ordered on one stream do not.
 * Enqueue only. */
int mlb_dilate_noalloc_dev(mlb_ctx* ctx, int nsel, const double* gradn, double rel_thr, double r_th,
                           const double* x, double* xout, void* stream);

/* SIMP exponent p of eq. interpolationSIMP2-SIMP for the following
 * mlb_set_density* calls (continuation of p, Secs. 3 and 6).  The moduli of
 * the current densities are stale afterwards, so every later solve returns
 * MLB_ESTATE until the densities are set again.  MLB_EINVAL unless p >= 1. */
int mlb_set_penal(mlb_ctx* ctx, double penal);

/* ---- three-field design variables (Sec. 2) ------------------------------ */

/* Density filter and relaxed Heaviside projection (eq. projectionOperator):
 *   xtilde_e = sum_k w_ek xhat_k / sum_k w_ek,  w_ek = max(0, rmin - |c_e - c_k|)
 *   x_e = (tanh(beta eta) + tanh(beta (xtilde_e - eta)))
 *         / (tanh(beta eta) + tanh(beta (1 - eta)))
 * with c the element centroids on the grid of unit cells and k over the
 * elements inside the grid (rows renormalised at the boundary).  xhat,
 * xtilde, x: device, m doubles each, distinct.  rmin in (0, 16], eta in
 * [0, 1], beta > 0.  The first call with a new rmin uploads its weight
 * table (synchronising the stream); later calls enqueue only.  The result
 * does not depend on the launch: each sum runs in one fixed order. */
int mlb_filter_project_dev(mlb_ctx* ctx, const double* xhat, double rmin, double eta, double beta,
                           double* xtilde, double* x, void* stream);

/* Chain rule from physical to design variables for ncols fields
 * (Sec. 2, after eq. AdjointSystem):
 *   dfdxhat[c m + k] = sum_e w_ek dfdx[c m + e] (dx/dxtilde)_e / W_e,
 *   (dx/dxtilde)_e = beta (1 - tanh^2(beta (xtilde_e - eta)))
 *                    / (tanh(beta eta) + tanh(beta (1 - eta))),
 *   W_e = sum_j w_ej,
 * with xtilde from mlb_filter_project_dev for the same rmin, eta, beta.
 * dfdx, dfdxhat: device ncols x m (column c at c m); work: device
 * workspace ncols x m, caller-owned, overwritten, distinct from both. */
int mlb_filter_chain_dev(mlb_ctx* ctx, int ncols, const double* xtilde, double rmin, double eta, double beta,
                         const double* dfdx, double* work, double* dfdxhat, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MLB_H */
