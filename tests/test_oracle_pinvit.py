"""Pins of the oracle's V-cycle and of the preconditioned inverse iteration
on the fine modes (App. A, eqs. PInvIt-GeneralInteration and errorEstimate).

  * The V-cycle is symmetric and positive definite, and its error propagator
    I - V K is a contraction (eigenvalues of V K in (0, 2)).
  * With no smoothing on two levels the V-cycle is the coarse-grid
    correction P A_c^-1 P^T, so it reproduces any coarse-representable
    vector exactly: V (K P y) = P y.
  * With the exact preconditioner P = K, one step is one step of block
    inverse iteration: phi_i - K^-1 (K + s_i G) phi_i = -s_i K^-1 G phi_i, so
    the Ritz values equal those of span(K^-1 G Phi) computed directly.
  * With the V-cycle, no Ritz value increases from step to step (eq.
    errorEstimate), each stays above the exact eigenvalue of the same index
    (Courant-Fischer), and every error shrinks.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, lba, mg
import workloads as W

MAT = fem.Material()


def _setup(nel, seed, levels, ell, q):
    x = W.density_uniform_noise(nel, seed, sigma=1.0)
    fixed = W.clamp_mask(nel)
    r = lba.analysis(nel, x, W.axial_load(nel)[:, None], fixed, MAT, ell=ell, q=q)
    free = np.flatnonzero(fixed == 0)
    Kff = r["K"][free][:, free].tocsr()
    Gff = r["G"][free][:, free].tocsr()
    As, Ps = mg.free_hierarchy(r["K"], fixed, nel, levels)
    omegas = [(4.0 / 3.0) / (1.05 * mg.spectral_radius_dinv_a(A)) for A in As[:-1]]
    return dict(r=r, free=free, Kff=Kff, Gff=Gff, As=As, Ps=Ps, omegas=omegas, nel=nel, fixed=fixed)


@pytest.fixture(scope="module")
def col2d():
    return _setup((32, 8), 21, levels=3, ell=2, q=4)


@pytest.fixture(scope="module")
def box3d():
    return _setup((8, 4, 4), 22, levels=2, ell=2, q=4)


@pytest.mark.parametrize("case", ["col2d", "box3d"])
def test_vcycle_symmetric_positive_and_contracting(case, request):
    p = request.getfixturevalue(case)
    V = mg.VCycle(p["As"], p["Ps"], p["omegas"], nu=2)
    n = p["Kff"].shape[0]
    Vm = V(np.eye(n))
    assert np.abs(Vm - Vm.T).max() <= 1e-12 * np.abs(Vm).max()
    assert np.linalg.eigvalsh(0.5 * (Vm + Vm.T))[0] > 0
    ev = np.linalg.eigvals(Vm @ p["Kff"].toarray()).real
    assert ev.min() > 0 and ev.max() < 2
    # the cycle converges as an iteration: rho(I - V K) < 1
    assert np.abs(1.0 - ev).max() < 0.9


def test_coarse_correction_alone_reproduces_coarse_vectors(col2d):
    p = col2d
    As2, Ps2 = p["As"][:2], p["Ps"][:1]
    V = mg.VCycle(As2, Ps2, p["omegas"][:1], nu=0)
    y = np.random.default_rng(5).standard_normal((As2[1].shape[0], 3))
    Py = Ps2[0] @ y
    z = V(p["Kff"] @ Py)
    assert np.abs(z - Py).max() <= 1e-10 * np.abs(Py).max()


def test_exact_preconditioner_step_is_block_inverse_iteration(col2d):
    p = col2d
    Kff, Gff = p["Kff"], p["Gff"]
    b = p["r"]["buck"]
    Phi = b.phi[p["free"]]
    lu = spla.splu(Kff.tocsc())
    lam1, Phi1, hist = mg.pinvit(Kff, Gff, Phi, b.lam, lu.solve, 1)
    lam_ref, _ = lba.rayleigh_ritz(Kff, Gff, lu.solve(Gff @ Phi))
    assert np.allclose(lam1, lam_ref, rtol=1e-10, atol=0)
    assert np.array_equal(hist[0], b.lam) and np.array_equal(hist[1], lam1)


@pytest.mark.parametrize("case", ["col2d", "box3d"])
def test_vcycle_pinvit_is_monotone_and_bounded(case, request):
    p = request.getfixturevalue(case)
    Kff, Gff = p["Kff"], p["Gff"]
    b = p["r"]["buck"]
    q = len(b.lam)
    exact = lba.generalized_lowest_positive(Kff, Gff, q)[0]
    V = mg.VCycle(p["As"], p["Ps"], p["omegas"], nu=2)
    lam, Phi, hist = mg.pinvit(Kff, Gff, b.phi[p["free"]], b.lam, V, 6)
    h = np.asarray(hist)                      # (steps + 1) x q
    assert np.all(np.diff(h, axis=0) <= 1e-12 * h[0]), h
    assert np.all(h >= exact[None, :] * (1 - 1e-12)), (h, exact)
    assert np.all(lam >= exact * (1 - 1e-12)), (lam, exact)
    assert np.all(h[-1] - exact < 0.5 * (h[0] - exact)), (h, exact)


@pytest.mark.parametrize("case", ["col2d", "box3d"])
def test_printed_shift_variant(case, request):
    """The printed step (every vector shifted by lambda~_1): the fundamental
    Ritz value still never grows and stays above the exact one, every Ritz
    value stays above its exact counterpart (Courant-Fischer), and on the
    first step the two variants give the same fundamental value update only
    if q = 1; with q > 1 the higher Ritz values move differently."""
    p = request.getfixturevalue(case)
    Kff, Gff = p["Kff"], p["Gff"]
    b = p["r"]["buck"]
    q = len(b.lam)
    exact = lba.generalized_lowest_positive(Kff, Gff, q)[0]
    V = mg.VCycle(p["As"], p["Ps"], p["omegas"], nu=2)
    lam_f, _, hist_f = mg.pinvit(Kff, Gff, b.phi[p["free"]], b.lam, V, 3, shift="first")
    lam_o, _, hist_o = mg.pinvit(Kff, Gff, b.phi[p["free"]], b.lam, V, 3, shift="own")
    h = np.asarray(hist_f)
    assert np.all(np.diff(h[:, 0]) <= 1e-12 * h[0, 0])
    assert np.all(h >= exact[None, :] * (1 - 1e-12))
    assert not np.allclose(lam_f[1:], lam_o[1:], rtol=1e-6)
    # a single vector: both shifts are its own Ritz value
    l1f, _, _ = mg.pinvit(Kff, Gff, b.phi[p["free"]][:, :1], b.lam[:1], V, 2, shift="first")
    l1o, _, _ = mg.pinvit(Kff, Gff, b.phi[p["free"]][:, :1], b.lam[:1], V, 2, shift="own")
    assert np.array_equal(l1f, l1o)
    with pytest.raises(ValueError):
        mg.pinvit(Kff, Gff, b.phi[p["free"]], b.lam, V, 1, shift="mean")
