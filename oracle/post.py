"""Post-processing measures of local buckling (oracle; test infrastructure only).

Sec. 5 of the paper inspects an optimized design with four quantities:
  * the energy-weighted modal correlation, eq. macCorrelationIndex:
        c_jr = a_j^T K[x] b_r
    for two mode sets normalised to a^T K a = 1 (values in [0, 1] for such
    modes; 1 when the modes coincide);
  * the strain energy density of mode j in element e,
        pi_{j|e} = phi_{j|e}^T K_e[x_e] phi_{j|e} = E_kappa(x_e) phi_{j|e}^T K_e0 phi_{j|e};
  * its total variation over the solid part of the design, eq. TVsed:
        L_j = int over {x_e >= xbar} of |grad pi_j|;
  * a local dilation of the densities, eq. postProcessingDilation, around the
    elements where the gradient of a selected mode's density is large.

Readings (the paper does not fix the discretisation):
  * pi_j is constant per element on a grid of unit cells.  Its gradient is
    taken with differences between neighbouring elements of the solid set
    Omega_>= only (the integration domain of eq. TVsed): per axis the central
    difference (pi_{e+1} - pi_{e-1}) / 2 when both neighbours are solid, the
    one-sided difference when one is, 0 when none is.  Outside Omega_>= the
    gradient is 0.  So pi constant on Omega_>= gives L_j = 0, as the paper
    states, and on a full grid this is numpy.gradient's first-order scheme.
  * The integral is the sum over solid elements (unit cell volume).
  * Dilation: element e takes the largest density among the elements k whose
    centroid lies within r_th of its own and that are flagged, i.e. where the
    gradient magnitude of some selected mode reaches rel_thr times that mode's
    largest value; e keeps its density when no such k exists (or when its own
    is larger).  The flag is read on the neighbour k, the element that sits in
    the buckling bar, so that the void around such a bar is filled to width
    r_th ("local thickening").
The element numbering is e = i + nx (j + ny k).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import fem


def mac(K, A, B):
    """C = A^T K B (eq. macCorrelationIndex) for column blocks A (n x qa), B (n x qb)."""
    return np.asarray(A).T @ (K @ np.asarray(B))


def strain_energy_density(nel, x, Phi, mat, elements=None):
    """pi[j, e] = E_kappa(x_e) phi_{j|e}^T K_e0 phi_{j|e} for the columns of Phi (n x q)
    (for the listed elements only, in that order, when ``elements`` is given)."""
    dim = len(nel)
    Ke0 = fem.material_stiffness(dim, mat)
    Ek, _ = fem.moduli(np.asarray(x, dtype=np.float64), mat)
    ed = fem.element_dofs(nel)
    elems = np.arange(len(Ek)) if elements is None else np.asarray(elements)
    Phi = np.asarray(Phi)
    Phi = Phi[:, None] if Phi.ndim == 1 else Phi
    out = np.empty((Phi.shape[1], len(elems)))
    for j in range(Phi.shape[1]):
        for t, e in enumerate(elems):
            pe = Phi[ed[e], j]
            out[j, t] = Ek[e] * (pe @ Ke0 @ pe)
    return out


def _grid(nel, v):
    """Element vector -> array indexed [k, j, i] (or [j, i] in 2D)."""
    return np.asarray(v).reshape(tuple(reversed(nel)))


def gradient_magnitude(nel, pi, solid):
    """|grad pi| per element, differences restricted to the solid set (reading above)."""
    P = _grid(nel, pi)
    S = _grid(nel, solid).astype(bool)
    shape = P.shape
    out = np.zeros(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        if not S[idx]:
            continue
        g2 = 0.0
        for ax in range(len(shape)):
            lo = list(idx)
            hi = list(idx)
            lo[ax] -= 1
            hi[ax] += 1
            has_lo = lo[ax] >= 0 and S[tuple(lo)]
            has_hi = hi[ax] < shape[ax] and S[tuple(hi)]
            if has_lo and has_hi:
                d = (P[tuple(hi)] - P[tuple(lo)]) / 2.0
            elif has_hi:
                d = P[tuple(hi)] - P[idx]
            elif has_lo:
                d = P[idx] - P[tuple(lo)]
            else:
                d = 0.0
            g2 += d * d
        out[idx] = np.sqrt(g2)
    return out.ravel()


def total_variation(nel, pi, x, xbar):
    """L = sum over {x_e >= xbar} of |grad pi|_e (eq. TVsed, unit cells); also returns |grad pi|."""
    solid = np.asarray(x) >= xbar
    g = gradient_magnitude(nel, pi, solid)
    return float(g[solid].sum()), g


def dilation_flags(gradn, rel_thr):
    """Elements where some selected mode's |grad pi| reaches rel_thr times its largest value."""
    gradn = np.atleast_2d(gradn)
    flags = np.zeros(gradn.shape[1], dtype=bool)
    for g in gradn:
        gm = g.max()
        if gm > 0.0:
            flags |= g >= rel_thr * gm
    return flags


def dilate(nel, x, flags, r_th):
    """Eq. postProcessingDilation with the reading above, by brute force over element pairs."""
    X = _grid(nel, x)
    Fl = _grid(nel, flags).astype(bool)
    shape = X.shape
    out = X.copy()
    r = int(np.floor(r_th))
    offs = [o for o in itertools.product(range(-r, r + 1), repeat=len(shape)) if sum(t * t for t in o) <= r_th * r_th]
    for idx in itertools.product(*[range(s) for s in shape]):
        best = X[idx]
        for o in offs:
            k = tuple(a + b for a, b in zip(idx, o))
            if all(0 <= k[a] < shape[a] for a in range(len(shape))) and Fl[k]:
                best = max(best, X[k])
        out[idx] = best
    return out.ravel()
