"""Pins of the oracle's intermediate-level refinement of Alg. 2 (Kaczmarz
smoothing of the prolonged modes on (K^j + sigma G^j) psi = 0 and a Ritz step
on every level between the eigen level and the fine grid).

  * The coloured sweep equals the row-by-row Kaczmarz sweep in the same
    order (its rows of one colour touch disjoint columns).
  * A Kaczmarz sweep for A x = 0 is a product of orthogonal projections onto
    hyperplanes through 0: it never increases the norm, and it leaves an
    exact null vector of A (an eigenvector with sigma its eigenvalue) alone.
  * With no sweep the pipeline is the plain multilevel method: the Ritz
    values of span(P Psi^{j+1}) on level j equal those of level j + 1
    (Galerkin operators), and the fine factors are unchanged.
  * Courant-Fischer: every Ritz value, on every level and on the fine grid,
    bounds the exact fine eigenvalue of its index from above.
"""
import numpy as np
import pytest

from oracle import fem, lba, levels, mg
import workloads as W

MAT = fem.Material()


def _problem(nel, seed):
    x = W.density_uniform_noise(nel, seed, sigma=1.0)
    fixed = W.clamp_mask(nel)
    K = fem.constrain(fem.assemble_K(nel, x, MAT), fixed, 1.0)
    U, _, _ = lba.static_solve(K, W.axial_load(nel)[:, None], fixed)
    K, G, _ = lba.operators(nel, x, U[:, 0], fixed, MAT)
    return K, G, fixed


CASES = {"col2d": ((24, 8), 41), "box3d": ((8, 4, 4), 42)}


@pytest.mark.parametrize("case", list(CASES))
def test_coloured_sweep_is_the_rowwise_sweep_and_contracts(case):
    nel, seed = CASES[case]
    K, G, fixed = _problem(nel, seed)
    free = np.flatnonzero(fixed == 0)
    lam = lba.generalized_lowest_positive(K[free][:, free], G[free][:, free], 2)[0]
    A = (K + 1.3 * lam[0] * G).tocsr()          # indefinite
    X = np.random.default_rng(seed).standard_normal((K.shape[0], 3))
    X[fixed != 0] = 0.0
    Y = mg.kaczmarz_sweep(A, X, nel, fixed)
    Z = mg.kaczmarz_sweep_rowwise(A, X, nel, fixed)
    assert np.abs(Y - Z).max() <= 1e-12 * np.abs(Z).max()
    assert np.all(np.linalg.norm(Y, axis=0) < np.linalg.norm(X, axis=0))
    assert np.all(Y[fixed != 0] == 0.0)


def test_exact_null_vector_is_a_fixed_point():
    nel, seed = CASES["box3d"]
    K, G, fixed = _problem(nel, seed)
    free = np.flatnonzero(fixed == 0)
    lam, V, _ = lba.generalized_lowest_positive(K[free][:, free], G[free][:, free], 1)
    v = np.zeros((K.shape[0], 1))
    v[free] = V
    A = (K + lam[0] * G).tocsr()
    w = mg.kaczmarz_sweep(A, v, nel, fixed)
    assert np.abs(w - v).max() <= 1e-9 * np.abs(v).max()


@pytest.mark.parametrize("nel,ell,seed", [((32, 8), 3, 43), ((16, 8, 8), 3, 44)])
def test_refinement_without_sweeps_is_the_plain_method_and_bounds_hold(nel, ell, seed):
    K, G, fixed = _problem(nel, seed)
    q = 4
    plain = lba.multilevel_buckling(nel, None, None, fixed, MAT, ell, q, K=K, G=G)
    lam0, _, lam_l, per0 = mg.multilevel_buckling_refined(nel, K, G, fixed, ell, q, 0)
    assert np.allclose(lam0, plain.lam, rtol=1e-10, atol=0)
    for lj in per0:
        assert np.allclose(lj, lam_l, rtol=1e-10, atol=0)
    free = np.flatnonzero(fixed == 0)
    exact = lba.generalized_lowest_positive(K[free][:, free], G[free][:, free], q)[0]
    for sweeps in (1, 3):
        lam, _, _, per = mg.multilevel_buckling_refined(nel, K, G, fixed, ell, q, sweeps)
        assert np.all(lam >= exact * (1 - 1e-12))
        for lj in per:
            assert np.all(lj >= exact * (1 - 1e-12))


@pytest.mark.parametrize("nel,ell,seed", [((32, 8), 3, 43), ((16, 8, 8), 3, 44)])
def test_fine_level_step_bounds(nel, ell, seed):
    """The loop run down to the fine grid: the fine-grid Ritz values of the
    smoothed modes and the final Ritz values stay above the exact ones
    (Courant-Fischer), the fine-grid Ritz step is reported last, and with no
    sweeps the fine Ritz step leaves the final values unchanged (the block
    solve's span is that of G Psi, whatever basis of span Psi is used)."""
    K, G, fixed = _problem(nel, seed)
    q = 4
    free = np.flatnonzero(fixed == 0)
    exact = lba.generalized_lowest_positive(K[free][:, free], G[free][:, free], q)[0]
    lam_plain, _, _, per_plain = mg.multilevel_buckling_refined(nel, K, G, fixed, ell, q, 0)
    lam0, _, _, per0 = mg.multilevel_buckling_refined(nel, K, G, fixed, ell, q, 0, fine_step=True)
    assert len(per0) == len(per_plain) + 1
    assert np.allclose(lam0, lam_plain, rtol=1e-10, atol=0)
    for sweeps in (1, 3):
        lam, _, _, per = mg.multilevel_buckling_refined(nel, K, G, fixed, ell, q, sweeps, fine_step=True)
        assert len(per) == ell - 1
        assert np.all(per[-1] >= exact * (1 - 1e-12))
        assert np.all(lam >= exact * (1 - 1e-12))
