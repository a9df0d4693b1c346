"""Nested grids, transfer operators and Galerkin coarse operators (oracle).

Follows Sec. 2.1 step 1 (coarse operators by Galerkin projection of the fine
ones) and Alg. 2 (nested discretizations Omega_1 > ... >
Omega_l, restriction of K and G, interpolation of modes).

Readings:
  * Coarsening halves the element count per axis per level (level 1 = fine).
    This matches the DOF counts the paper quotes for its coarse levels.
  * Interpolation I^j_{j+1} is bilinear/trilinear nodal interpolation applied
    to each displacement component; restriction is its transpose.
  * A coarse DOF is a Dirichlet DOF iff the fine DOF at the coincident node
    is one.  Interpolation is masked on both sides: P_hat = M_f P M_c.
  * Coarse operators: K^c = P_hat^T K_hat P_hat + (I - M_c) and
    G^c = P_hat^T G_hat P_hat, i.e. identity (K) / zero (G) at coarse
    Dirichlet DOFs, as on the fine level.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def coarsen(nel):
    for v in nel:
        if v % 2:
            raise ValueError(f"grid {nel} cannot be halved")
    return tuple(v // 2 for v in nel)


def level_grids(nel, levels):
    grids = [tuple(nel)]
    for _ in range(levels - 1):
        grids.append(coarsen(grids[-1]))
    return grids


def _interp_1d(nc):
    """(2nc+1) x (nc+1) linear interpolation from coarse to fine nodes."""
    rows, cols, vals = [], [], []
    for i in range(2 * nc + 1):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [i // 2, i // 2 + 1]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc + 1, nc + 1))


def prolongation(nel_fine):
    """Unmasked DOF interpolation P (n_fine x n_coarse) from grid nel_fine/2."""
    dim = len(nel_fine)
    ncs = coarsen(nel_fine)
    Pn = _interp_1d(ncs[0])
    for ax in range(1, dim):
        Pn = sp.kron(_interp_1d(ncs[ax]), Pn)  # x is the fastest node index
    return sp.kron(Pn, sp.eye(dim)).tocsr()


def coarse_fixed(nel_fine, fixed_fine):
    """Dirichlet mask on the coarse grid: the coincident fine DOF's flag."""
    dim = len(nel_fine)
    ncs = coarsen(nel_fine)
    nnf = [v + 1 for v in nel_fine]
    nnc = [v + 1 for v in ncs]
    grids = np.meshgrid(*[np.arange(v) for v in reversed(nnc)], indexing="ij")
    idx = [g.ravel() for g in reversed(grids)]  # idx[0] = I (x), ...
    fine_node = 2 * idx[0]
    stride = 1
    for ax in range(1, dim):
        stride *= nnf[ax - 1]
        fine_node = fine_node + stride * 2 * idx[ax]
    out = np.zeros(dim * len(fine_node), dtype=np.uint8)
    for c in range(dim):
        out[dim * np.arange(len(fine_node)) + c] = np.asarray(fixed_fine)[dim * fine_node + c]
    return out


def masked_prolongation(nel_fine, fixed_fine):
    fixed_c = coarse_fixed(nel_fine, fixed_fine)
    P = prolongation(nel_fine)
    Mf = sp.diags((np.asarray(fixed_fine) == 0).astype(np.float64))
    Mc = sp.diags((fixed_c == 0).astype(np.float64))
    return (Mf @ P @ Mc).tocsr(), fixed_c


def hierarchy(nel, fixed, levels):
    """Masked prolongations P_hat_j (level j+1 -> j) and masks for every level."""
    grids = level_grids(nel, levels)
    masks = [np.asarray(fixed, dtype=np.uint8)]
    Ps = []
    for j in range(levels - 1):
        P, fc = masked_prolongation(grids[j], masks[j])
        Ps.append(P)
        masks.append(fc)
    return grids, masks, Ps


def composite_prolongation(Ps, ell):
    """P_{1<-ell} = P_hat_1 P_hat_2 ... P_hat_{ell-1} (the level-by-level prolongation of Alg. 2, repeated)."""
    n = Ps[0].shape[0] if Ps else None
    P = sp.eye(n).tocsr() if ell > 1 else None
    for j in range(ell - 1):
        P = P @ Ps[j]
    return P


def galerkin(A_hat, P_hat, fixed_coarse, diag_value):
    """P_hat^T A_hat P_hat plus diag_value at coarse Dirichlet DOFs."""
    Ac = (P_hat.T @ A_hat @ P_hat).tocsr()
    free_c = (np.asarray(fixed_coarse) == 0).astype(np.float64)
    return (Ac + sp.diags(diag_value * (1.0 - free_c))).tocsr()


def nested_fixed_set_ok(nel_fine, fixed_fine):
    """True iff every fine Dirichlet DOF interpolates only from coarse
    Dirichlet DOFs, i.e. M_f P M_c == P M_c."""
    P = prolongation(nel_fine)
    fc = coarse_fixed(nel_fine, fixed_fine)
    Mc = sp.diags((fc == 0).astype(np.float64))
    Fix = sp.diags((np.asarray(fixed_fine) != 0).astype(np.float64))
    return (Fix @ P @ Mc).count_nonzero() == 0
