"""Shared helpers of the GPU parity tests (oracle side and device plumbing)."""
import numpy as np
import scipy.sparse as sp

from oracle import fem, levels
import workloads as W

MAT = fem.Material()


def torch_dev():
    import torch
    return torch


def to_dev(a):
    """numpy (n,) or (n, k) column block -> torch (k, n) contiguous float64 on cuda."""
    torch = torch_dev()
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda()


def from_dev(t):
    a = t.detach().cpu().numpy()
    return a if a.ndim == 1 else a.T.copy()


def oracle_levels(nel, x, fixed, L, mat=MAT):
    """Constrained K on every level (fine assembled, coarse by Galerkin)."""
    grids, masks, Ps = levels.hierarchy(nel, fixed, L)
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    Ks = [K]
    for j in range(L - 1):
        Ks.append(levels.galerkin(Ks[-1], Ps[j], masks[j + 1], 1.0))
    return grids, masks, Ps, Ks


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
