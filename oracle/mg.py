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
from .lba import rayleigh_ritz


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


def pinvit(Kff, Gff, Phi, lam, apply_P, steps):
    """``steps`` preconditioned inverse iteration steps on the Ritz block Phi
    (free DOFs, columns paired with the Ritz values lam), each followed by
    Rayleigh-Ritz.  Returns the final Ritz values and vectors and the Ritz
    values before and after every step."""
    hist = [np.array(lam, dtype=np.float64)]
    q = Phi.shape[1]
    for _ in range(steps):
        R = Kff @ Phi + (Gff @ Phi) * np.asarray(lam)[None, :]
        Phi = Phi - apply_P(R)
        lam, Phi = rayleigh_ritz(Kff, Gff, Phi)
        if len(lam) < q:
            raise ValueError("fewer than q positive Ritz values after a step")
        hist.append(np.array(lam))
    return lam, Phi, hist
