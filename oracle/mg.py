"""Multigrid V-cycle and preconditioned inverse iteration on the fine modes (oracle).

Test infrastructure: only tests/, the package's smoke check and the
benchmark's CPU baseline may import this module.

App. A (eq. PInvIt-GeneralInteration) improves the fine-scale modes after the
Ritz step by preconditioned inverse iteration: every vector of the block takes
steps

    phi_i <- phi_i - P^-1 (K + lambda~_i G) phi_i

with P the multigrid preconditioner of the static solves and lambda~_i the
current Rayleigh quotient of phi_i; eq. errorEstimate states that the
Rayleigh quotients then decrease monotonically towards the eigenvalues.

Readings (the paper names the ingredients, not their arrangement):
  * P^-1 is one V(nu, nu)-cycle on the hierarchy of the static solves:
    level 1 is K, coarser levels are Galerkin products P^T A P (Dirichlet DOFs
    excluded, as in levels.py); damped Jacobi with weights omega_j (inputs);
    the first pre-smoothing sweep starts from zero, nu - 1 more follow, then
    one coarse-grid correction (restriction = interpolation^T) and nu
    post-smoothing sweeps; the coarsest level is solved exactly.
  * The printed step shifts every vector by lambda~_1, but the text calls it
    the gradient step of R_i, whose shift is R_i itself, and states the
    convergence estimate for every R_i.  A common shift lambda~_1 drives the
    whole block towards the first mode and raises the higher Ritz values;
    the shift is taken as each vector's own Ritz value lambda~_i.
  * After each step the block is replaced by its Ritz vectors on its span
    (the Rayleigh-Ritz of Sec. 2.1 step 4), so lambda~_i is the i-th Ritz
    value of the current block.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import levels as lv
from .lba import generalized_lowest_positive, rayleigh_ritz


def _free(mask):
    return np.flatnonzero(np.asarray(mask) == 0)


def free_hierarchy(K, fixed, nel, nlevels):
    """Level operators on free DOFs: A_1 = K_ff, A_{j+1} = P_j^T A_j P_j, and
    the interpolations P_j (free coarse DOFs -> free fine DOFs)."""
    grids, masks, Ps = lv.hierarchy(nel, fixed, nlevels)
    f0 = _free(masks[0])
    As = [K[f0][:, f0].tocsr()]
    Pf = []
    A_full = K
    for j in range(nlevels - 1):
        A_full = lv.galerkin(A_full, Ps[j], masks[j + 1], 1.0)
        ff, fc = _free(masks[j]), _free(masks[j + 1])
        Pf.append(Ps[j][ff][:, fc].tocsr())
        As.append(A_full[fc][:, fc].tocsr())
    return As, Pf


def spectral_radius_dinv_a(A):
    """rho(D^-1 A) of an SPD level operator (dense; small levels only)."""
    d = A.diagonal()
    s = 1.0 / np.sqrt(d)
    M = (A.toarray() * s[:, None]) * s[None, :]
    return float(sla.eigvalsh(M)[-1])


class VCycle:
    """z = P^-1 r for blocks r (n_1 x k) on free DOFs (nu = 0: the coarse-grid
    correction alone, P A_c^-1 P^T on two levels)."""

    def __init__(self, As, Ps, omegas, nu=2):
        if len(omegas) < len(As) - 1:
            raise ValueError("one Jacobi weight per level above the coarsest")
        self.As, self.Ps, self.omegas, self.nu = As, Ps, list(omegas), nu
        self.d = [A.diagonal() for A in As]
        self.coarse = sla.cho_factor(As[-1].toarray())

    def _cycle(self, j, r):
        A = self.As[j]
        if j == len(self.As) - 1:
            return sla.cho_solve(self.coarse, r)
        w, d = self.omegas[j], self.d[j][:, None]
        z = w * r / d if self.nu > 0 else np.zeros_like(r)
        for _ in range(self.nu - 1):
            z = z + w * (r - A @ z) / d
        zc = self._cycle(j + 1, self.Ps[j].T @ (r - A @ z))
        z = z + self.Ps[j] @ zc
        for _ in range(self.nu):
            z = z + w * (r - A @ z) / d
        return z

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64)
        vec = r.ndim == 1
        z = self._cycle(0, r[:, None] if vec else r)
        return z[:, 0] if vec else z


def pinvit(Kff, Gff, Phi, lam, apply_P, steps, shift="own"):
    """``steps`` preconditioned inverse iteration steps on the Ritz block Phi
    (free DOFs, columns paired with the Ritz values lam), each followed by
    Rayleigh-Ritz.  ``shift``: "own" shifts each vector by its Ritz value (the
    gradient step of its Rayleigh quotient, the reading taken), "first" by
    lambda~_1 for every vector (the step as printed).  Returns the final Ritz
    values and vectors and the Ritz values before and after every step."""
    if shift not in ("own", "first"):
        raise ValueError("shift must be 'own' or 'first'")
    hist = [np.array(lam, dtype=np.float64)]
    q = Phi.shape[1]
    for _ in range(steps):
        sh = np.asarray(lam) if shift == "own" else np.full(q, lam[0])
        R = Kff @ Phi + (Gff @ Phi) * sh[None, :]
        Phi = Phi - apply_P(R)
        lam, Phi = rayleigh_ritz(Kff, Gff, Phi)
        if len(lam) < q:
            raise ValueError("fewer than q positive Ritz values after a step")
        hist.append(np.array(lam))
    return lam, Phi, hist


# ---------------------------------------------------------------------------
# Alg. 2, intermediate levels: on each level j = l-1 .. 2 the prolonged modes
# are smoothed by Kaczmarz sweeps on (K^j + sigma_j G^j) psi = 0, sigma_j the
# smallest Ritz value of the coarser level, and replaced by the Ritz vectors
# of the level-j pencil on their span (App. A; Kaczmarz as in the paper: row
# projections, i.e. Gauss-Seidel on A A^T).
#
# Readings:
#   * The loop of Alg. 2 is printed as j = l-1, ..., 0 with the fine grid
#     called Omega_1; it is read as the intermediate levels l-1 .. 2, the
#     fine level being handled by the block solve and Ritz step that follow.
#   * The row order of a sweep is fixed by colour: node (i, j, k) has colour
#     (i mod 3) + 3 (j mod 3) + 9 (k mod 3); colours are visited in
#     increasing order, the nodes of a colour in any order (their rows touch
#     disjoint columns, as every row couples a node to its 3^d neighbours
#     only), and the components of a node in increasing order.  Each free row
#     r replaces psi by its projection onto a_r . psi = 0 (no damping); rows of
#     Dirichlet DOFs are skipped.
#   * The number of sweeps is an input (the paper does not give it).


def node_colors(nel):
    """Colour (i mod 3) + 3 (j mod 3) [+ 9 (k mod 3)] of every node of a grid."""
    nn = [v + 1 for v in nel]
    idx = np.indices(nn[::-1]).reshape(len(nn), -1)[::-1]   # (i, j[, k]) with i fastest
    col = idx[0] % 3 + 3 * (idx[1] % 3)
    if len(nn) == 3:
        col = col + 9 * (idx[2] % 3)
    return col


def kaczmarz_sweep(A, X, nel, fixed):
    """One Kaczmarz sweep for A x = 0 on every column of X (full-length
    vectors of a level with Dirichlet mask ``fixed``)."""
    A = A.tocsr()
    dim = len(nel)
    X = np.array(X, dtype=np.float64, copy=True)
    col = node_colors(nel)
    fixed = np.asarray(fixed)
    for cidx in range(3 ** dim):
        nodes = np.flatnonzero(col == cidx)
        for c in range(dim):
            rows = nodes * dim + c
            rows = rows[fixed[rows] == 0]
            if rows.size == 0:
                continue
            Ar = A[rows]
            nrm = np.asarray(Ar.multiply(Ar).sum(axis=1)).ravel()
            keep = nrm > 0
            Ar, nrm = Ar[keep], nrm[keep]
            res = Ar @ X
            X -= Ar.T @ (res / nrm[:, None])
    return X


def kaczmarz_sweep_rowwise(A, X, nel, fixed):
    """The same sweep one row at a time (definition; for small grids)."""
    A = A.tocsr()
    dim = len(nel)
    X = np.array(X, dtype=np.float64, copy=True)
    col = node_colors(nel)
    for cidx in range(3 ** dim):
        for node in np.flatnonzero(col == cidx):
            for c in range(dim):
                r = node * dim + c
                if fixed[r]:
                    continue
                lo, hi = A.indptr[r], A.indptr[r + 1]
                cols, a = A.indices[lo:hi], A.data[lo:hi]
                nrm = float(a @ a)
                if nrm > 0:
                    X[cols] -= np.outer(a, (a @ X[cols]) / nrm)
    return X


def multilevel_buckling_refined(nel, K, G, fixed, ell, q, sweeps, dense_limit=6000, fine_step=False):
    """Sec. 2.1 steps 1-4 with the intermediate-level smoothing and Ritz steps
    of Alg. 2 (``sweeps`` Kaczmarz sweeps per level).  K, G: constrained fine
    operators.  With ``fine_step`` the loop also visits the fine grid (the
    printed loop runs down to it): the prolonged modes take the same sweeps
    on (K + sigma G) psi = 0 and a fine Ritz step before the block solve.
    Returns the fine Ritz values and vectors and, per refined level (l-1
    first, the fine grid last when ``fine_step``), its Ritz values."""
    grids, masks, Ps = lv.hierarchy(nel, fixed, ell)
    Ks, Gs = [K], [G]
    for j in range(ell - 1):
        Ks.append(lv.galerkin(Ks[-1], Ps[j], masks[j + 1], 1.0))
        Gs.append(lv.galerkin(Gs[-1], Ps[j], masks[j + 1], 0.0))
    fl = _free(masks[ell - 1])
    lam_l, V, _ = generalized_lowest_positive(Ks[-1][fl][:, fl], Gs[-1][fl][:, fl], q, dense_limit=dense_limit)
    Psi = np.zeros((Ks[-1].shape[0], q))
    Psi[fl] = V
    sigma = float(lam_l[0])
    per_level = []
    for j in range(ell - 2, 0, -1):           # 0-based index of levels l-1 .. 2
        Psi = Ps[j] @ Psi
        A = (Ks[j] + sigma * Gs[j]).tocsr()
        for _ in range(sweeps):
            Psi = kaczmarz_sweep(A, Psi, grids[j], masks[j])
        fj = _free(masks[j])
        lam_j, Vj = rayleigh_ritz(Ks[j][fj][:, fj], Gs[j][fj][:, fj], Psi[fj])
        if len(lam_j) < q:
            raise ValueError("fewer than q positive Ritz values on an intermediate level")
        Psi = np.zeros((Ks[j].shape[0], q))
        Psi[fj] = Vj
        sigma = float(lam_j[0])
        per_level.append(lam_j)
    Psi = Ps[0] @ Psi if ell > 1 else Psi
    f0 = _free(fixed)
    if fine_step and ell > 1:
        A = (K + sigma * G).tocsr()
        for _ in range(sweeps):
            Psi = kaczmarz_sweep(A, Psi, nel, fixed)
        lam_1, V1 = rayleigh_ritz(K[f0][:, f0], G[f0][:, f0], Psi[f0])
        if len(lam_1) < q:
            raise ValueError("fewer than q positive Ritz values on the fine grid")
        Psi = np.zeros((K.shape[0], q))
        Psi[f0] = V1
        per_level.append(lam_1)
    Kff = K[f0][:, f0].tocsc()
    import scipy.sparse.linalg as spla
    Phi_t = spla.splu(Kff).solve(np.ascontiguousarray((G @ Psi)[f0]))
    lam, Vf = rayleigh_ritz(K[f0][:, f0], G[f0][:, f0], Phi_t)
    return lam, Vf, lam_l, per_level
