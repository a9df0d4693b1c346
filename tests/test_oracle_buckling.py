"""Pins of the oracle's buckling analysis and sensitivities (CPU only).

  * Euler column: clamped-free column, L/H = 20, conforming Q4: the lowest
    buckling factor converges from above to the Timoshenko-corrected Euler
    load P_E / (1 + P_E / (kappa G A)), P_E = pi^2 E I / (4 L^2).
  * Scale laws lambda(cE) = c lambda, lambda(s f) = lambda / s.
  * Courant-Fischer: multilevel factors bound the exact ones from above.
  * l = 1: the multilevel steps reproduce the exact pairs
    (Phi~ = -Psi Lambda^-1).
  * Ritz values do not depend on the basis of the coarse subspace.
  * Central finite differences of compliance, of the exact lambda_1 and of
    the frozen-vector Rayleigh quotient with u re-solved (the quantity whose
    exact derivative the multilevel sensitivity formula is).
  * Homogeneity (E0 = 0): sum_e x_e dJ/dx_e = -p J, sum_e x_e dlam/dx_e = p lam.
"""
import numpy as np
import pytest

from oracle import fem, levels, lba, sens
import workloads as W

MAT = fem.Material()


def _euler_ratio(ny):
    nel = (20 * ny, ny)
    x = np.ones(W.n_elems(nel))
    r = lba.analysis(nel, x, W.axial_load(nel), W.clamp_mask(nel), MAT, ell=1, q=1, dense_limit=2000)
    L, H = nel
    I = H ** 3 / 12.0
    PE = np.pi ** 2 * I / (4.0 * L * L)
    kGA = (5.0 / 6.0) * (1.0 / (2.0 * (1.0 + MAT.nu))) * H
    return r["buck"].lam[0] / (PE / (1.0 + PE / kGA))


def test_euler_column_converges_from_above():
    ratios = [_euler_ratio(ny) for ny in (4, 8, 16)]
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] - 1.0 < 5e-3
    # second-order convergence of the conforming element: error ratio ~4
    e = [r - 1.0 for r in ratios]
    assert 3.0 < e[0] / e[1] < 5.0 and 3.0 < e[1] / e[2] < 5.0


@pytest.fixture(scope="module")
def small2d():
    nel = (24, 8)
    x = W.density_uniform_noise(nel, 11, sigma=1.0)
    return dict(nel=nel, x=x, fixed=W.clamp_mask(nel), F=W.axial_load(nel)[:, None])


def test_scale_laws(small2d):
    p = small2d
    r = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=1, q=3)
    mat5 = fem.Material(E1=5.0, E0=5e-6)
    r5 = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], mat5, ell=1, q=3)
    assert np.allclose(r5["buck"].lam, 5.0 * r["buck"].lam, rtol=1e-10)
    r2 = lba.analysis(p["nel"], p["x"], 2.0 * p["F"], p["fixed"], MAT, ell=1, q=3)
    assert np.allclose(r2["buck"].lam, r["buck"].lam / 2.0, rtol=1e-10)


@pytest.mark.parametrize("ell", [2, 3])
def test_courant_fischer_and_coarse_bound(small2d, ell):
    p = small2d
    ex = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=1, q=4)
    ml = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=ell, q=4)
    lam, lt = ex["buck"].lam, ml["buck"].lam
    assert np.all(lt >= lam * (1 - 1e-12))
    # coarse Galerkin factors bound from above too (subspace of the fine space)
    assert np.all(ml["buck"].coarse_lam >= lam * (1 - 1e-12))
    # and the fine solve improves on them
    assert np.all(lt <= ml["buck"].coarse_lam * (1 + 1e-12))


def test_ell1_is_exact(small2d):
    p = small2d
    r = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=1, q=4)
    K, G, fixed = r["K"], r["G"], p["fixed"]
    res = lba.multilevel_buckling(p["nel"], p["x"], r["u"], fixed, MAT, 1, 4, K=K, G=G,
                                  solver=r["solver"])
    lam = r["buck"].lam
    assert np.allclose(res.lam, lam, rtol=1e-11)
    Psi = res.extra["Psi"]
    Phi_t = res.extra["Phi_tilde"]
    assert np.abs(Phi_t + Psi / lam[None, :]).max() < 1e-9 * np.abs(Phi_t).max()
    assert res.residual_inf.max() < 1e-9


def test_ritz_basis_invariance(small2d):
    p = small2d
    r = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=2, q=4)
    mix = np.random.default_rng(7).standard_normal((4, 4)) + 4 * np.eye(4)
    res = lba.multilevel_buckling(p["nel"], p["x"], r["u"], p["fixed"], MAT, 2, 4, K=r["K"], G=r["G"],
                                  solver=r["solver"], psi_mix=mix)
    assert np.allclose(res.lam, r["buck"].lam, rtol=1e-11)


def test_modes_k_normalised(small2d):
    p = small2d
    r = lba.analysis(p["nel"], p["x"], p["F"], p["fixed"], MAT, ell=2, q=4)
    phi = r["buck"].phi
    M = phi.T @ (r["K"] @ phi)
    assert np.abs(M - np.eye(4)).max() < 1e-10
    # Rayleigh quotient of each Ritz vector equals its Ritz value
    for i in range(4):
        assert abs(sens.rayleigh_quotient(r["K"], r["G"], phi[:, i]) / r["buck"].lam[i] - 1) < 1e-10


def _solve_J(nel, x, F, fixed, mat):
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    U, J, _ = lba.static_solve(K, F, fixed)
    return U, J


@pytest.mark.parametrize("nel", [(8, 4), (4, 2, 2)])
def test_fd_compliance(nel):
    x = W.random_small(len(nel), nel, 21, 0.3, 1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    U, J = _solve_J(nel, x, F, fixed, MAT)
    dJ = sens.compliance_sensitivity(nel, x, U, MAT)[:, 0]
    h = 1e-5
    for e in range(len(x)):
        xp, xm = x.copy(), x.copy()
        xp[e] += h; xm[e] -= h
        fd = (_solve_J(nel, xp, F, fixed, MAT)[1][0] - _solve_J(nel, xm, F, fixed, MAT)[1][0]) / (2 * h)
        assert abs(fd - dJ[e]) <= 1e-6 * np.abs(dJ).max()


def _lam_exact(nel, x, F, fixed, q):
    r = lba.analysis(nel, x, F, fixed, MAT, ell=1, q=q)
    return r


@pytest.mark.parametrize("nel", [(10, 4), (4, 2, 2)])
def test_fd_exact_buckling_factor(nel):
    x = W.random_small(len(nel), nel, 22, 0.3, 1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    r = _lam_exact(nel, x, F, fixed, 2)
    lam = r["buck"].lam
    assert (lam[1] - lam[0]) / lam[0] > 1e-3          # simple eigenvalue
    dlam, _ = sens.buckling_sensitivity(nel, x, r["u"], lam, r["buck"].phi, fixed, MAT, r["solver"])
    h = 1e-5
    rng = np.random.default_rng(3)
    for e in rng.choice(len(x), size=min(len(x), 12), replace=False):
        xp, xm = x.copy(), x.copy()
        xp[e] += h; xm[e] -= h
        fd = (_lam_exact(nel, xp, F, fixed, 2)["buck"].lam[0] -
              _lam_exact(nel, xm, F, fixed, 2)["buck"].lam[0]) / (2 * h)
        assert abs(fd - dlam[e, 0]) <= 1e-6 * np.abs(dlam[:, 0]).max()


def test_fd_multilevel_frozen_rayleigh_quotient():
    nel = (16, 8)
    x = W.random_small(2, nel, 23, 0.3, 1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    r = lba.analysis(nel, x, F, fixed, MAT, ell=2, q=3)
    lam, phi = r["buck"].lam, r["buck"].phi
    dlam, _ = sens.buckling_sensitivity(nel, x, r["u"], lam, phi, fixed, MAT, r["solver"])

    def R(xx, v):
        K = fem.constrain(fem.assemble_K(nel, xx, MAT), fixed, 1.0)
        U, _, _ = lba.static_solve(K, F, fixed)
        G = fem.constrain(fem.assemble_G(nel, fem.element_stresses(nel, xx, U[:, 0], MAT)), fixed, 0.0)
        return sens.rayleigh_quotient(K, G, v)
    h = 1e-5
    for i in range(3):
        for e in np.random.default_rng(4 + i).choice(len(x), size=8, replace=False):
            xp, xm = x.copy(), x.copy()
            xp[e] += h; xm[e] -= h
            fd = (R(xp, phi[:, i]) - R(xm, phi[:, i])) / (2 * h)
            assert abs(fd - dlam[e, i]) <= 1e-6 * np.abs(dlam[:, i]).max()


@pytest.mark.parametrize("nel,ell", [((16, 8), 1), ((16, 8), 2), ((4, 4, 2), 2)])
def test_homogeneity(nel, ell):
    mat = fem.Material(E0=0.0)
    x = W.random_small(len(nel), nel, 24, 0.2, 1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    r = lba.analysis(nel, x, F, fixed, mat, ell=ell, q=2)
    dJ = sens.compliance_sensitivity(nel, x, r["U"], mat)[:, 0]
    assert abs(x @ dJ + mat.p * r["J"][0]) < 1e-10 * abs(r["J"][0])
    lam = r["buck"].lam
    dlam, _ = sens.buckling_sensitivity(nel, x, r["u"], lam, r["buck"].phi, fixed, mat, r["solver"])
    for i in range(2):
        assert abs(x @ dlam[:, i] - mat.p * lam[i]) < 1e-10 * lam[i]


def test_adjoint_rhs_directional_derivative():
    # b = grad_u (phi^T G[x, u] phi); G is linear in u, so for any v the
    # difference quotient with any step is exact.
    nel = (6, 4)
    x = W.random_small(2, nel, 25)
    fixed = W.clamp_mask(nel)
    rng = np.random.default_rng(8)
    n = W.n_dofs(nel)
    free = (fixed == 0)
    phi = rng.standard_normal(n) * free
    u = rng.standard_normal(n) * free
    v = rng.standard_normal(n) * free
    b = sens.adjoint_rhs(nel, x, phi, fixed, MAT)

    def q(uu):
        G = fem.assemble_G(nel, fem.element_stresses(nel, x, uu, MAT))
        return phi @ (G @ phi)
    assert abs((q(u + 0.7 * v) - q(u)) / 0.7 - b @ v) < 1e-12 * max(1.0, abs(b @ v))


@pytest.mark.parametrize("nel,q", [((40, 12), 6), ((12, 4, 4), 12)])
def test_arpack_branch_matches_dense_eigh(nel, q):
    """The two branches of generalized_lowest_positive (dense LAPACK eigh
    below the size limit, ARPACK shift-invert above it) on the same free-DOF
    matrices: factors to 1e-11, K-normalised modes equal up to sign
    (|psi_a^T K psi_d| = 1 to 1e-9) for separated factors, same next gap."""
    import workloads as W
    from oracle import fem, lba
    x = W.random_small(len(nel), nel, 9, 0.2, 1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    mat = fem.Material()
    an = lba.analysis(nel, x, F, fixed, mat, 1, 1)
    free = np.flatnonzero(fixed == 0)
    Kff = an["K"][free][:, free]
    Gff = an["G"][free][:, free]
    assert Kff.shape[0] < 6000
    lam_d, V_d, mu_d = lba.generalized_lowest_positive(Kff, Gff, q, dense_limit=10 ** 9)
    lam_a, V_a, mu_a = lba.generalized_lowest_positive(Kff, Gff, q, dense_limit=0)
    assert np.max(np.abs(lam_a / lam_d - 1)) < 1e-11
    assert abs(mu_a / mu_d - 1) < 1e-9
    KV = Kff @ V_d
    for i in range(q):
        gaps = [abs(lam_d[i] - lam_d[j]) / lam_d[i] for j in range(q) if j != i]
        if min(gaps) > 1e-6:
            assert abs(abs(V_a[:, i] @ KV[:, i]) - 1) < 1e-9, i
