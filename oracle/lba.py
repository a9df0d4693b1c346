"""Linearized buckling analysis, direct and multilevel (oracle).

Follows Alg. 1 (LA then EA) and the four steps of Sec. 2.1:
  1. coarse eigenproblem (K^l + lambda^l G^l) psi = 0 with Galerkin K^l, G^l;
  2. the q lowest coarse modes interpolated level by level to the fine grid;
  3. one fine linear solve  K Phi~ = G Psi;
  4. buckling factors from the Rayleigh quotient of Phi~.

Readings:
  * "Lowest" buckling factors are the lowest POSITIVE lambda (negative ones
    belong to the reversed load).  They are computed as the largest positive
    mu = 1/lambda of (-G) psi = mu K psi, K symmetric positive definite.
  * Eq. FineScaleRQ is printed as a ratio of matrices; it is read as the
    Rayleigh-Ritz values of span(Phi~) (Alg. 2 calls it a Ritz projection):
    A = Phi~^T K Phi~, B = -Phi~^T G Phi~, B y = mu A y, lambda~ = 1/mu.
  * The main text (no intermediate-level smoothing) is followed, not the
    Kaczmarz smoothing of Alg. 2.
  * Modes are K-normalised (phi_i^T K phi_j = delta_ij, Sec. 2) and signed so
    that the entry of largest magnitude is positive (ties: lowest index).
  * Loads: the reference load is one column of F; Dirichlet rows of F are
    ignored (the solution is zero there).

Direct solves use SuperLU (scipy.sparse.linalg.splu) on the free DOFs; dense
generalized eigenproblems use LAPACK (scipy.linalg.eigh), larger ones ARPACK
(scipy.sparse.linalg.eigsh) in generalized mode with an exact K^-1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, levels


def _free(fixed):
    return np.flatnonzero(np.asarray(fixed) == 0)


class FreeSolver:
    """Sparse direct solver for K_ff (K restricted to free DOFs)."""

    def __init__(self, K, fixed):
        self.free = _free(fixed)
        self.n = K.shape[0]
        Kff = K[self.free][:, self.free].tocsc()
        self.lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def solve(self, B):
        B = np.asarray(B, dtype=np.float64)
        one = B.ndim == 1
        Bm = B[:, None] if one else B
        X = np.zeros_like(Bm)
        X[self.free] = self.lu.solve(np.ascontiguousarray(Bm[self.free]))
        return X[:, 0] if one else X


def static_solve(K, F, fixed, solver=None):
    """Alg. 1 / Alg. 2, linear analysis: u = K^-1 f for every column of F;
    compliance J = f^T u (Sec. 3, problem P1 objective)."""
    solver = solver or FreeSolver(K, fixed)
    F = np.asarray(F, dtype=np.float64)
    Fm = F[:, None] if F.ndim == 1 else F
    Fm = Fm * (np.asarray(fixed) == 0)[:, None]
    U = solver.solve(Fm)
    J = np.einsum("ij,ij->j", Fm, U)
    return U, J, solver


def static_solve_refined(nel, x, F, fixed, mat, steps=40, rtol=1e-13):
    """The direct solve of ``static_solve`` followed by iterative refinement
    of an extended-precision solution (numpy longdouble): residual
    r = f - K u by fem.residual_extended, correction K d = r by the same
    factorisation, u += d, while the residual shrinks and is above
    rtol ||f||.  For nearly singular designs the direct solve's backward
    error, eps |K||u|, is far above the residual of the exact solution, and
    two double-precision solutions at that level can differ visibly; the
    refined solution rounded to doubles is the double nearest to it.
    Returns (u rounded to float64, J = f^T u, history of ||r|| / ||f|| of
    the extended-precision iterates)."""
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    f = np.asarray(F, dtype=np.float64).reshape(-1) * (np.asarray(fixed) == 0)
    U, _, solver = static_solve(K, f[:, None], fixed)
    u = U[:, 0].astype(np.longdouble)
    nf = np.linalg.norm(f)
    r, _ = fem.residual_extended(nel, x, u, f, fixed, mat)
    hist = [np.linalg.norm(r) / nf]
    for _ in range(steps):
        if hist[-1] <= rtol:
            break
        un = u + solver.solve(r).astype(np.longdouble)
        rn, _ = fem.residual_extended(nel, x, un, f, fixed, mat)
        if not np.linalg.norm(rn) < np.linalg.norm(r):
            break
        u, r = un, rn
        hist.append(np.linalg.norm(r) / nf)
    u64 = u.astype(np.float64)
    return u64, float(f @ u64), hist


def _sign_fix(V):
    V = V.copy()
    for j in range(V.shape[1]):
        a = np.abs(V[:, j])
        i = int(np.flatnonzero(a == a.max())[0])
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def generalized_lowest_positive(Kff, Gff, q, dense_limit=6000, tol=1e-13):
    """Lowest q positive lambda of (K + lambda G) psi = 0 on the free DOFs.

    Returns (lambda ascending (q,), Psi (nf, q) K-normalised, mu_next) where
    mu_next = 1/lambda_{q+1} (for gap reporting; 0 if unavailable)."""
    nf = Kff.shape[0]
    if nf <= dense_limit:
        Kd = Kff.toarray() if sp.issparse(Kff) else np.asarray(Kff)
        Gd = Gff.toarray() if sp.issparse(Gff) else np.asarray(Gff)
        lo = max(nf - q - 1, 0)
        mu, V = sla.eigh(-Gd, Kd, subset_by_index=[lo, nf - 1])
        order = np.argsort(-mu)
        mu, V = mu[order], V[:, order]
    else:
        lu = spla.splu(Kff.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        Minv = spla.LinearOperator(Kff.shape, matvec=lu.solve, dtype=np.float64)
        mu, V = spla.eigsh(-Gff, k=q + 1, M=Kff, Minv=Minv, which="LA", tol=tol,
                           ncv=max(3 * (q + 1), 40))
        order = np.argsort(-mu)
        mu, V = mu[order], V[:, order]
    pos = mu > 0
    if pos[:q].sum() < q:
        raise ValueError("fewer than q positive buckling factors")
    mu_next = float(mu[q]) if len(mu) > q else 0.0
    mu, V = mu[:q], V[:, :q]
    # K-normalise (eigh/eigsh already do up to rounding; do it explicitly)
    KV = Kff @ V
    V = V / np.sqrt(np.einsum("ij,ij->j", V, KV))[None, :]
    return 1.0 / mu, V, mu_next


def rayleigh_ritz(Kff, Gff, Phi):
    """Sec. 2.1 step 4 read as Rayleigh-Ritz on span(Phi):
    B y = mu A y, A = Phi^T K Phi, B = -Phi^T G Phi; lambda = 1/mu for mu > 0."""
    A = Phi.T @ (Kff @ Phi)
    B = -(Phi.T @ (Gff @ Phi))
    A = 0.5 * (A + A.T)
    B = 0.5 * (B + B.T)
    mu, Y = sla.eigh(B, A)
    order = np.argsort(-mu)
    mu, Y = mu[order], Y[:, order]
    keep = mu > 0
    mu, Y = mu[keep], Y[:, keep]
    V = Phi @ Y
    return 1.0 / mu, V


@dataclass
class BucklingResult:
    lam: np.ndarray                 # (q,) ascending
    phi: np.ndarray                 # (n, q) full length, K-normalised
    coarse_lam: np.ndarray = None   # (q,) coarse-level factors
    coarse_psi: np.ndarray = None   # (n_l, q) full-length coarse modes
    gap: float = 0.0                # (mu_q - mu_{q+1}) / mu_q at the eigen level
    residual_inf: np.ndarray = None  # ||(K + lam G) phi||_inf per mode
    extra: dict = field(default_factory=dict)


def operators(nel, x, u, fixed, mat):
    """Constrained fine K (identity at Dirichlet DOFs) and G (zero there)."""
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    s = fem.element_stresses(nel, x, u, mat)
    G = fem.constrain(fem.assemble_G(nel, s), fixed, 0.0)
    return K, G, s


def exact_buckling(K, G, fixed, q, dense_limit=6000):
    """Alg. 1 eigenproblem on the fine grid (l = 1): exact lowest q positive pairs."""
    free = _free(fixed)
    Kff = K[free][:, free]
    Gff = G[free][:, free]
    lam, V, mu_next = generalized_lowest_positive(Kff, Gff, q, dense_limit=dense_limit)
    n = K.shape[0]
    phi = np.zeros((n, q))
    phi[free] = V
    phi = _sign_fix(phi)
    gap = (1.0 / lam[-1] - mu_next) * lam[-1]
    res = np.abs(K @ phi + (G @ phi) * lam[None, :]).max(axis=0)
    return BucklingResult(lam=lam, phi=phi, coarse_lam=lam, coarse_psi=phi, gap=gap,
                          residual_inf=res)


def multilevel_buckling(nel, x, u, fixed, mat, ell, q, mg_levels=None, K=None, G=None,
                        solver=None, dense_limit=6000, psi_mix=None):
    """Sec. 2.1 steps 1-4 with eigen level ``ell`` (1 = fine).

    ``psi_mix`` (q x q, optional) right-multiplies the coarse modes before
    prolongation; span and hence the result are unchanged (used by tests)."""
    mg_levels = max(mg_levels or ell, ell)
    if K is None or G is None:
        K, G, _ = operators(nel, x, u, fixed, mat)
    grids, masks, Ps = levels.hierarchy(nel, fixed, mg_levels)
    if ell == 1:
        Kl, Gl, fl = K, G, masks[0]
    else:
        Kl, Gl = K, G
        for j in range(ell - 1):
            Kl = levels.galerkin(Kl, Ps[j], masks[j + 1], 1.0)
            Gl = levels.galerkin(Gl, Ps[j], masks[j + 1], 0.0)
        fl = masks[ell - 1]
    free_l = _free(fl)
    lam_l, V, mu_next = generalized_lowest_positive(Kl[free_l][:, free_l], Gl[free_l][:, free_l],
                                                    q, dense_limit=dense_limit)
    psi = np.zeros((Kl.shape[0], q))
    psi[free_l] = V
    gap = (1.0 / lam_l[-1] - mu_next) * lam_l[-1]
    Psi = psi if psi_mix is None else psi @ psi_mix
    for j in reversed(range(ell - 1)):        # step 2: Psi^j = I^j_{j+1} Psi^{j+1}
        Psi = Ps[j] @ Psi
    solver = solver or FreeSolver(K, fixed)
    Phi_t = solver.solve(G @ Psi)              # step 3: K Phi~ = G Psi
    free = _free(fixed)
    lam, Vf = rayleigh_ritz(K[free][:, free], G[free][:, free], Phi_t[free])   # step 4
    phi = np.zeros((K.shape[0], len(lam)))
    phi[free] = Vf
    phi = _sign_fix(phi)
    res = np.abs(K @ phi + (G @ phi) * lam[None, :]).max(axis=0)
    return BucklingResult(lam=lam, phi=phi, coarse_lam=lam_l, coarse_psi=_sign_fix(psi),
                          gap=gap, residual_inf=res, extra=dict(Phi_tilde=Phi_t, Psi=Psi))


def analysis(nel, x, F, fixed, mat, ell, q, ref_case=0, dense_limit=6000):
    """Static solve followed by the (multilevel) buckling analysis."""
    K0 = fem.assemble_K(nel, x, mat)
    K = fem.constrain(K0, fixed, 1.0)
    U, J, solver = static_solve(K, F, fixed)
    u = U[:, ref_case]
    s = fem.element_stresses(nel, x, u, mat)
    G = fem.constrain(fem.assemble_G(nel, s), fixed, 0.0)
    if ell == 1:
        res = exact_buckling(K, G, fixed, q, dense_limit=dense_limit)
    else:
        res = multilevel_buckling(nel, x, u, fixed, mat, ell, q, K=K, G=G, solver=solver,
                                  dense_limit=dense_limit)
    return dict(U=U, J=J, u=u, s=s, K=K, G=G, solver=solver, buck=res)
