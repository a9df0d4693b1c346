"""Pins of the consistent sensitivity oracle (appendix on numerical
procedures, eq. consistentSensitivity with the residual of eq. eigResidual),
against facts that do not come from its own formula:

* printed literally, the appendix adjoint -2 (K + lambda~ G)^-1 y equals
  -2 phi~ (a dense indefinite solve), which is why the literal formula
  collapses to eq. SensitivityLambda;
* exact pairs (eigen level 1): the residual vanishes and the consistent
  sensitivity equals the plain one;
* central finite differences of the quantity it differentiates, the Ritz
  values of span(K^-1 G[u] Psi) with Psi fixed, recomputed from scratch at
  x +- h e_e (the plain formula misses them by orders of magnitude more);
* Euler homogeneity for E0 = 0: K has degree p in x, G degree 0 (E_sigma
  ~ x^p, u ~ x^-p), so lambda~(c x) = c^p lambda~(x) and
  sum_e x_e dlambda~/dx_e = p lambda~.
"""
import numpy as np
import pytest

import workloads as W
from oracle import consistent, fem, lba, sens


def _ml(nel, x, F, fixed, mat, ell, q):
    ref = lba.analysis(nel, x, F, fixed, mat, ell=ell, q=q)
    b = ref["buck"]
    free = np.flatnonzero(fixed == 0)
    c = consistent.ritz_coefficients(b.extra["Phi_tilde"][free], b.phi[free])
    psi = b.extra["Psi"] @ c
    return ref, b, psi


def _case(seed=7, nel=(24, 12), E0=1e-6, lo=None):
    mat = fem.Material(E0=E0) if E0 != 1e-6 else fem.Material()
    x = W.density_uniform_noise(nel, seed, mean=0.6, amp=0.3)
    if lo is not None:
        x = np.clip(x, lo, 1.0)
    return mat, x, W.clamp_mask(nel), W.axial_load(nel)[:, None]


def test_literal_appendix_adjoint_is_minus_two_phi():
    nel, q = (24, 12), 4
    mat, x, fixed, F = _case()
    ref, b, _ = _ml(nel, x, F, fixed, mat, 2, q)
    K, G = ref["K"].toarray(), ref["G"].toarray()
    free = np.flatnonzero(fixed == 0)
    for i in range(q):
        A = (K + b.lam[i] * G)[np.ix_(free, free)]
        y = (K @ b.phi[:, i] + b.lam[i] * (G @ b.phi[:, i]))[free]
        assert np.linalg.norm(y) > 1e-6 * np.linalg.norm((K @ b.phi[:, i])[free])   # a true residual
        p = -2.0 * np.linalg.solve(A, y)
        assert np.abs(p + 2.0 * b.phi[free, i]).max() < 1e-8 * np.abs(b.phi[free, i]).max()


def test_exact_pairs_give_the_plain_sensitivity():
    nel, q = (24, 12), 4
    mat, x, fixed, F = _case()
    ref = lba.analysis(nel, x, F, fixed, mat, ell=1, q=q)
    b = ref["buck"]
    # at level 1 the interpolated modes are the exact ones: phi = K^-1 G psi
    # with psi = -lambda phi
    psi = -b.phi * b.lam[None, :]
    dl, _, _ = consistent.consistent_sensitivity(nel, x, ref["u"], b.lam, b.phi, psi, ref["K"], ref["G"], fixed,
                                                 mat, ref["solver"])
    dp, _ = sens.buckling_sensitivity(nel, x, ref["u"], b.lam, b.phi, fixed, mat, ref["solver"])
    assert np.abs(dl - dp).max() <= 1e-8 * np.abs(dp).max()


def test_central_differences_of_the_frozen_ritz_values():
    nel, q, ell = (24, 12), 4, 2
    mat, x, fixed, F = _case()
    ref, b, psi = _ml(nel, x, F, fixed, mat, ell, q)
    Psi = b.extra["Psi"]
    lam0 = consistent.frozen_ritz_values(nel, x, F, fixed, mat, Psi)
    assert np.abs(lam0 / b.lam - 1).max() < 1e-12
    dl, _, _ = consistent.consistent_sensitivity(nel, x, ref["u"], b.lam, b.phi, psi, ref["K"], ref["G"], fixed,
                                                 mat, ref["solver"])
    dp, _ = sens.buckling_sensitivity(nel, x, ref["u"], b.lam, b.phi, fixed, mat, ref["solver"])
    rng = np.random.default_rng(5)
    es = rng.choice(x.size, size=16, replace=False)
    h = 1e-5
    fd = np.empty((len(es), q))
    for r, e in enumerate(es):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd[r] = (consistent.frozen_ritz_values(nel, xp, F, fixed, mat, Psi)
                 - consistent.frozen_ritz_values(nel, xm, F, fixed, mat, Psi)) / (2 * h)
    for i in range(q):
        scale = np.abs(fd[:, i]).max()
        err_c = np.abs(dl[es, i] - fd[:, i]).max() / scale
        err_p = np.abs(dp[es, i] - fd[:, i]).max() / scale
        assert err_c < 1e-6, (i, err_c)
        assert err_p > 100 * max(err_c, 1e-9), (i, err_p, err_c)


def test_euler_homogeneity():
    nel, q = (24, 12), 4
    mat, x, fixed, F = _case(E0=0.0, lo=0.2)
    ref, b, psi = _ml(nel, x, F, fixed, mat, 2, q)
    dl, _, _ = consistent.consistent_sensitivity(nel, x, ref["u"], b.lam, b.phi, psi, ref["K"], ref["G"], fixed,
                                                 mat, ref["solver"])
    lhs = x @ dl
    assert np.abs(lhs / (mat.p * b.lam) - 1).max() < 1e-9, (lhs, mat.p * b.lam)
