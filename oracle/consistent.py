"""Consistent buckling-factor sensitivities of the multilevel pairs (oracle;
appendix on numerical procedures, eq. consistentSensitivity with the residual
of eq. eigResidual).  Test infrastructure: only the tests, the smoke check
and the benchmark's CPU leg use this package.

The multilevel factor lambda~_i is not an eigenvalue of (K + lambda G) phi = 0;
its residual y_i = (K + lambda~_i G) phi~_i (eq. eigResidual) is not zero, so
eq. SensitivityLambda (which assumes an eigenpair) is not its derivative.

Reading.  Printed literally, the appendix's adjoint p_i = -2 (K + lambda~_i
G)^-1 y_i equals -2 phi~_i (y_i is (K + lambda~_i G) phi~_i), and with it the
appendix formula reduces to eq. SensitivityLambda; the remaining term, the
derivative of y_i, is left undefined there.  What the formula expresses is
the chain rule through the way phi~ depends on x: lambda~_i = R(x, phi~_i(x))
with grad_phi R = 2 lambda~ y (for phi^T K phi = 1), so the residual term is
2 lambda~ y_i^T dphi~_i/dx.  In the method of Sec. 2.1 phi~ comes from the
fine solve K Phi~ = G Psi (step 3) followed by Rayleigh-Ritz (step 4), hence:

  quantity differentiated: lambda~_i(x) = i-th Ritz value of
      span(K[x]^-1 G[x, u(x)] Psi),  u(x) = K[x]^-1 f,
  with the interpolated coarse modes Psi held fixed (the coarse eigenpairs
  are the method's only exact ones; their own dependence on x is not part
  of this derivative);

  derivative (phi~ K-normalised, psi_i = Psi c_i with phi~_i = Phi~ c_i, so
  K phi~_i = G psi_i; primes are partial derivatives at fixed u):
      dlambda~_i/dx_e = lambda~ phi~^T K'_e phi~ + lambda~^2 phi~^T G'_e phi~
                        - lambda~^2 zt^T K'_e u
                        + 2 lambda~ (w^T G'_e psi - w^T K'_e phi~),
      w  = K^-1 y_i                                   (residual adjoint),
      zt = K^-1 (b_i + (2 / lambda~) d_i),
      b_i = grad_u (phi~^T G[x, u] phi~)              (eq. AdjointSystem),
      d_i = grad_u (w^T G[x, u] psi_i).
  With y_i = 0 (exact pairs, eigen level 1) w = 0, d = 0 and this is
  eq. SensitivityLambda times lambda~ (the plain sensitivities).

Both adjoint right-hand sides are formed by brute-force linearity (entry a is
the form with G[x, e_a] for the unit displacement e_a), as in sens.py.
"""
from __future__ import annotations

import numpy as np

from . import fem, lba
from .sens import _unit_stress_stiffness


def bilinear_adjoint_rhs(nel, x, w, psi, fixed, mat):
    """d = grad_u (w^T G[x, u] psi): entries w^T G[x, e_a] psi (fixed rows 0)."""
    dim = len(nel)
    Gunit = _unit_stress_stiffness(dim, mat.nu)
    _, Es = fem.moduli(np.asarray(x, dtype=np.float64), mat)
    ed = fem.element_dofs(nel)
    we, pe = np.asarray(w)[ed], np.asarray(psi)[ed]
    loc = Es[:, None] * np.einsum("ei,aij,ej->ea", we, Gunit, pe)
    d = np.bincount(ed.ravel(), weights=loc.ravel(), minlength=fem.n_dofs(nel))
    d[np.asarray(fixed) != 0] = 0.0
    return d


def ritz_coefficients(Phi_tilde, phi):
    """c with phi = Phi_tilde c for vectors of span(Phi_tilde) (least squares)."""
    c, *_ = np.linalg.lstsq(Phi_tilde, phi, rcond=None)
    return c


def consistent_sensitivity(nel, x, u, lam, phi, psi, K, G, fixed, mat, solver):
    """dlambda~_i/dx_e (m, q) by the formula in the module notes.
    phi: (n, q) K-normalised Ritz vectors; psi: (n, q) with K phi = G psi;
    K, G: constrained operators; solver: K^-1 on the free DOFs."""
    from .sens import adjoint_rhs
    q = phi.shape[1]
    Y = K @ phi + (G @ phi) * lam[None, :]
    Y[np.asarray(fixed) != 0] = 0.0
    Wv = solver.solve(Y)
    rhs = np.empty_like(phi)
    for i in range(q):
        rhs[:, i] = adjoint_rhs(nel, x, phi[:, i], fixed, mat) \
            + (2.0 / lam[i]) * bilinear_adjoint_rhs(nel, x, Wv[:, i], psi[:, i], fixed, mat)
    Zt = solver.solve(rhs)
    dim = len(nel)
    Ke0 = fem.material_stiffness(dim, mat)
    D = fem.constitutive(dim, mat.nu)
    Bc = fem.strain_matrix(dim, np.full(dim, 0.5))
    ed = fem.element_dofs(nel)
    xs = np.asarray(x, dtype=np.float64)
    ue = np.asarray(u)[ed]
    s0 = ue @ (D @ Bc).T                                  # unit-modulus centroid stress
    xp1 = mat.p * np.power(xs, mat.p - 1.0)
    dEk, dEs = xp1 * (mat.E1 - mat.E0), xp1 * mat.E1
    H = fem.gradient_products(dim)
    nn = 2 ** dim
    g0 = np.zeros((len(xs), nn, nn))                       # G_e0[u_e] scalar part
    for k, (a, b) in enumerate(fem.voigt_pairs(dim)):
        Hk = H[a, a] if a == b else H[a, b] + H[b, a]
        g0 += s0[:, k, None, None] * Hk[None]
    out = np.empty((len(xs), q))
    for i in range(q):
        pe = phi[ed, i]
        we, se, ze = Wv[ed, i], psi[ed, i], Zt[ed, i]
        pr, wr, sr = (v.reshape(-1, nn, dim) for v in (pe, we, se))
        pKp = np.einsum("ei,ij,ej->e", pe, Ke0, pe)
        pGp = np.einsum("eac,eab,ebc->e", pr, g0, pr)
        zKu = np.einsum("ei,ij,ej->e", ze, Ke0, ue)
        wGs = np.einsum("eac,eab,ebc->e", wr, g0, sr)
        wKp = np.einsum("ei,ij,ej->e", we, Ke0, pe)
        L = lam[i]
        out[:, i] = L * dEk * pKp + L * L * dEs * pGp - L * L * dEk * zKu + 2.0 * L * (dEs * wGs - dEk * wKp)
    return out, Wv, Zt


def frozen_ritz_values(nel, x, F, fixed, mat, Psi, ref_case=0):
    """The quantity differentiated: Ritz values of span(K[x]^-1 G[x, u(x)] Psi)
    for fixed Psi (n, q), ascending positive (for central differences)."""
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    U, _, solver = lba.static_solve(K, F, fixed)
    u = U[:, ref_case]
    s = fem.element_stresses(nel, x, u, mat)
    G = fem.constrain(fem.assemble_G(nel, s), fixed, 0.0)
    Phi_t = solver.solve(G @ Psi)
    free = np.flatnonzero(np.asarray(fixed) == 0)
    lam, _ = lba.rayleigh_ritz(K[free][:, free], G[free][:, free], Phi_t[free])
    return lam
