"""Compliance and buckling-factor sensitivities (oracle).

Follows eq. SensitivityLambda with the adjoint system eq. AdjointSystem, applied
to the multilevel pairs (lambda~, phi~) as the paper does (Sec. 2.1, residual
eq. eigResidual ignored).  Sensitivities are with respect to the physical
densities x (the filter/projection chain rule is left to the caller).

Readings:
  * eq. SensitivityLambda holds for the normalisation -phi^T G phi = 1.  With
    the normalisation the paper states (phi^T K phi = 1) the derivative of
    lambda = -phi^T K phi / phi^T G phi carries one more factor lambda:
        dlambda/dx_e = lambda [ phi^T K'_e phi
                               + lambda (phi^T G'_e phi - z^T K'_e u) ]
    (scalar check: K = k, G = g gives dlambda = (lambda/k)(k' + lambda g')).
  * K'_e = p x_e^(p-1) (E1 - E0) K_e0 and G'_e = p x_e^(p-1) E1 G_e0[u_e]
    (derivatives of eq. interpolationSIMP2-SIMP, u held fixed).
  * The adjoint right-hand side b = grad_u (phi^T G[x, u] phi) is formed by
    brute-force linearity: G is linear in u, so its a-th entry is
    phi^T G[x, e_a] phi for the unit displacement e_a (element by element).
  * Compliance J = f^T u has dJ/dx_e = -u_e^T K'_e u_e.
"""
from __future__ import annotations

import numpy as np

from . import fem


def compliance_sensitivity(nel, x, U, mat, elements=None):
    """dJ/dx_e = -p x^(p-1) (E1 - E0) u_e^T K_e0 u_e for each load case column
    (for the listed elements only when ``elements`` is given)."""
    dim = len(nel)
    Ke0 = fem.material_stiffness(dim, mat)
    ed = fem.element_dofs(nel)
    xs = np.asarray(x, dtype=np.float64)
    if elements is not None:
        ed, xs = ed[elements], xs[elements]
    U = np.asarray(U)
    Um = U[:, None] if U.ndim == 1 else U
    dE = mat.p * np.power(xs, mat.p - 1.0) * (mat.E1 - mat.E0)
    out = np.empty((len(xs), Um.shape[1]))
    for c in range(Um.shape[1]):
        ue = Um[ed, c]
        out[:, c] = -dE * np.einsum("ei,ij,ej->e", ue, Ke0, ue)
    return out


def _unit_stress_stiffness(dim, nu):
    """G_e0[e_a] for every local unit displacement e_a: (nde, nde, nde)."""
    D = fem.constitutive(dim, nu)
    Bc = fem.strain_matrix(dim, np.full(dim, 0.5))
    nde = Bc.shape[1]
    out = np.empty((nde, nde, nde))
    for a in range(nde):
        ea = np.zeros(nde)
        ea[a] = 1.0
        out[a] = fem.stress_stiffness_local(dim, D @ Bc @ ea)
    return out


def adjoint_rhs(nel, x, phi, fixed, mat):
    """b = grad_u (phi^T G phi), entries phi^T G[x, e_a] phi (fixed rows 0)."""
    dim = len(nel)
    Gunit = _unit_stress_stiffness(dim, mat.nu)
    _, Es = fem.moduli(np.asarray(x, dtype=np.float64), mat)
    ed = fem.element_dofs(nel)
    nde = Gunit.shape[0]
    # loc[e, a] = phi_e^T G_e0[e_a] phi_e = sum_ij phi_ei phi_ej G_e0[e_a]_ij,
    # evaluated as (phi_e outer phi_e) . G_e0[e_a] over blocks of elements
    Gmat = Gunit.transpose(1, 2, 0).reshape(nde * nde, nde)
    loc = np.empty((len(ed), nde))
    for lo in range(0, len(ed), 65536):
        pe = np.asarray(phi)[ed[lo:lo + 65536]]
        loc[lo:lo + 65536] = (pe[:, :, None] * pe[:, None, :]).reshape(-1, nde * nde) @ Gmat
    loc *= Es[:, None]
    b = np.bincount(ed.ravel(), weights=loc.ravel(), minlength=fem.n_dofs(nel))
    b[np.asarray(fixed) != 0] = 0.0
    return b


def buckling_sensitivity(nel, x, u, lam, phi, fixed, mat, solver):
    """dlambda_i/dx_e for each column of phi (K-normalised), with adjoints z_i
    from K z_i = b_i (eq. AdjointSystem).  Returns (dlam (m, q), Z (n, q))."""
    q = phi.shape[1]
    B = np.stack([adjoint_rhs(nel, x, phi[:, i], fixed, mat) for i in range(q)], axis=1)
    Z = solver.solve(B)
    return buckling_sensitivity_from_adjoints(nel, x, u, lam, phi, Z, mat), Z


def buckling_sensitivity_from_adjoints(nel, x, u, lam, phi, Z, mat, elements=None):
    """eq. SensitivityLambda (times lambda, see the module notes) given the
    adjoint solutions Z; for the listed elements only when ``elements`` is given."""
    dim = len(nel)
    Ke0 = fem.material_stiffness(dim, mat)
    D = fem.constitutive(dim, mat.nu)
    Bc = fem.strain_matrix(dim, np.full(dim, 0.5))
    ed = fem.element_dofs(nel)
    xs = np.asarray(x, dtype=np.float64)
    if elements is not None:
        ed, xs = ed[elements], xs[elements]
    q = phi.shape[1]
    ue = np.asarray(u)[ed]
    s0 = ue @ (D @ Bc).T                                   # unit-modulus stress
    xp1 = mat.p * np.power(xs, mat.p - 1.0)
    dEk = xp1 * (mat.E1 - mat.E0)
    dEs = xp1 * mat.E1
    H = fem.gradient_products(dim)
    nn = 2 ** dim
    g0 = np.zeros((len(xs), nn, nn))
    for k, (i, j) in enumerate(fem.voigt_pairs(dim)):
        Hk = H[i, i] if i == j else H[i, j] + H[j, i]
        g0 += s0[:, k, None, None] * Hk[None]
    dlam = np.empty((len(xs), q))
    for i in range(q):
        pe = phi[ed, i]
        ze = Z[ed, i]
        pK = np.einsum("ei,ij,ej->e", pe, Ke0, pe)
        pr = pe.reshape(-1, nn, dim)
        pG = np.einsum("eac,eab,ebc->e", pr, g0, pr)
        zKu = np.einsum("ei,ij,ej->e", ze, Ke0, ue)
        dlam[:, i] = lam[i] * (dEk * pK + lam[i] * (dEs * pG - dEk * zKu))
    return dlam


def rayleigh_quotient(K, G, v):
    """R(x, v) = -v^T K v / v^T G v (eq. minBLFcharRayleigh)."""
    return -(v @ (K @ v)) / (v @ (G @ v))
