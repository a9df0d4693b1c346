"""Pins of the oracle's post-processing measures (Sec. 5: eqs.
macCorrelationIndex, TVsed and postProcessingDilation).

  * Strain energy density: its sum over the elements is the assembled
    quadratic form phi^T K phi (element loop against the sparse assembly);
    rigid motions store none.
  * Correlation: for K-normalised modes c = 1 - ||a - b||_K^2 / 2, with the
    energy of the difference taken from the element densities; fine
    eigenvectors of the buckling problem are K-orthonormal (c = I); the
    Cauchy-Schwarz bound |c| <= 1.
  * Gradient: on a full grid it is numpy.gradient's first-order scheme; a
    linear density has |grad| = |a| everywhere; a density constant on the
    solid set has zero total variation whatever it is on the void.
  * Dilation: with every element flagged it is the grey dilation of
    scipy.ndimage with a ball footprint; with none it is the identity; one
    flagged solid element in void grows into the lattice ball of radius r_th
    (7, 19, 27, 33 cells for r_th = 1, sqrt 2, sqrt 3, 2 in 3D).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.ndimage as ndi

from oracle import fem, post
import workloads as W

MAT = fem.Material()


@pytest.mark.parametrize("nel", [(6, 4), (4, 3, 3)])
def test_sed_sums_to_the_quadratic_form(nel):
    rng = np.random.default_rng(1)
    x = rng.uniform(0.1, 1.0, W.n_elems(nel))
    K = fem.assemble_K(nel, x, MAT)
    Phi = rng.standard_normal((fem.n_dofs(nel), 3))
    pi = post.strain_energy_density(nel, x, Phi, MAT)
    for j in range(3):
        q = Phi[:, j] @ (K @ Phi[:, j])
        assert abs(pi[j].sum() - q) <= 1e-12 * abs(q)
    assert np.all(pi >= -1e-14)
    dim = len(nel)
    t = np.zeros((fem.n_dofs(nel) // dim, dim))
    t[:, 0] = 1.0
    assert np.abs(post.strain_energy_density(nel, x, t.ravel(), MAT)).max() < 1e-13


def _fine_modes(nel, q):
    x = W.density_uniform_noise(nel, 11)
    fixed = W.clamp_mask(nel)
    K = fem.constrain(fem.assemble_K(nel, x, MAT), fixed, 1.0).toarray()
    F = W.axial_load(nel)
    u = np.linalg.solve(K, F)
    s = fem.element_stresses(nel, x, u, MAT)
    G = fem.constrain(fem.assemble_G(nel, s), fixed, 0.0).toarray()
    free = fixed == 0
    # K phi = -lambda G phi  <=>  (-G) phi = (1/lambda) K phi: largest 1/lambda first
    mu, V = sla.eigh(-G[np.ix_(free, free)], K[np.ix_(free, free)])
    Phi = np.zeros((fem.n_dofs(nel), q))
    Phi[free] = V[:, ::-1][:, :q]
    return x, fixed, K, Phi


def test_mac_of_fine_eigenvectors_is_identity_and_matches_the_energy_of_differences():
    nel = (30, 10)
    x, fixed, K, Phi = _fine_modes(nel, 4)
    C = post.mac(K, Phi, Phi)
    assert np.abs(C - np.eye(4)).max() < 1e-10
    rng = np.random.default_rng(4)
    b = Phi[:, 0] + 0.05 * rng.standard_normal(len(Phi)) * (fixed == 0)
    b /= np.sqrt(b @ K @ b)
    c = post.mac(K, Phi[:, :1], b[:, None])[0, 0]
    dist2 = post.strain_energy_density(nel, x, Phi[:, 0] - b, MAT).sum()
    assert abs(c - (1.0 - dist2 / 2.0)) < 1e-10
    assert abs(c) <= 1.0


@pytest.mark.parametrize("nel", [(7, 5), (5, 4, 3)])
def test_gradient_full_grid_is_numpy_gradient(nel):
    pi = np.random.default_rng(2).standard_normal(W.n_elems(nel))
    g = post.gradient_magnitude(nel, pi, np.ones(len(pi), bool))
    P = pi.reshape(tuple(reversed(nel)))
    ref = np.sqrt(sum(d * d for d in np.gradient(P, edge_order=1)))
    assert np.abs(g - ref.ravel()).max() < 1e-14


@pytest.mark.parametrize("nel", [(7, 5), (5, 4, 3)])
def test_linear_density_and_constant_on_solid(nel):
    dim = len(nel)
    a = np.array([0.3, -1.2, 0.7][:dim])
    idx = np.indices(tuple(reversed(nel))).reshape(dim, -1)[::-1]   # i, j, (k) per element
    pi = a @ idx
    tv, g = post.total_variation(nel, pi, np.ones(len(pi)), 1.0)
    assert np.abs(g - np.linalg.norm(a)).max() < 1e-13
    assert abs(tv - np.linalg.norm(a) * len(pi)) < 1e-11
    rng = np.random.default_rng(3)
    x = np.where(rng.uniform(size=len(pi)) < 0.6, 1.0, 1e-3)
    pi2 = np.where(x >= 1.0, 2.5, rng.uniform(size=len(pi)))
    tv2, g2 = post.total_variation(nel, pi2, x, 1.0)
    assert tv2 == 0.0 and np.all(g2 == 0.0)


def _ball(dim, r):
    R = int(np.floor(r))
    o = np.indices((2 * R + 1,) * dim) - R
    return (o ** 2).sum(0) <= r * r


@pytest.mark.parametrize("nel,r", [((9, 7), 1.0), ((9, 7), 2.3), ((6, 5, 4), 1.5), ((6, 5, 4), 2.0)])
def test_dilation_all_flagged_is_grey_dilation(nel, r):
    x = np.random.default_rng(5).uniform(size=W.n_elems(nel))
    out = post.dilate(nel, x, np.ones(len(x), bool), r)
    X = x.reshape(tuple(reversed(nel)))
    ref = ndi.grey_dilation(X, footprint=_ball(len(nel), r), mode="constant", cval=-np.inf)
    assert np.array_equal(out, ref.ravel())
    assert np.array_equal(post.dilate(nel, x, np.zeros(len(x), bool), r), x)


@pytest.mark.parametrize("r,count", [(1.0, 7), (np.sqrt(2.0), 19), (np.sqrt(3.0), 27), (2.0, 33)])
def test_dilation_single_flag_grows_a_lattice_ball(r, count):
    nel = (7, 7, 7)
    x = np.full(343, 1e-3)
    c = 3 + 7 * (3 + 7 * 3)
    x[c] = 1.0
    flags = np.zeros(343, bool)
    flags[c] = True
    out = post.dilate(nel, x, flags, r + 1e-12)
    assert int((out == 1.0).sum()) == count


def test_flags_threshold():
    g = np.array([[0.0, 1.0, 0.5, 0.099], [0.0, 0.0, 0.0, 0.0], [4.0, 0.0, 0.0, 0.4]])
    f = post.dilation_flags(g, 0.1)
    assert f.tolist() == [True, True, True, True]
    f = post.dilation_flags(g[:2], 0.5)
    assert f.tolist() == [False, True, True, False]
