"""Pins of the oracle's incompatible-mode elements (Q6/H11, Sec. 2: the
paper's element), condensed to the nodal DOFs.

  * K_e0 is symmetric positive semidefinite and its null space is exactly
    the rigid motions (3 in 2D, 6 in 3D).
  * Patch test: on every linear displacement field the incompatible and the
    bilinear/trilinear element give the same nodal forces (the modes'
    strains average to zero over the element, so constant strain does not
    excite them).
  * Pure bending: the exact plane-stress (2D) and 3D pure-bending fields lie
    in the enlarged space and are stationary for it, so the condensed element
    stores exactly their energy E kappa^2 / 24 on the unit cell, while the
    conforming element locks in shear and stores more.
  * The clamped-free Euler column (L/H = 20) converges to the
    Timoshenko-corrected Euler load from above, far faster than with Q4.
"""
import numpy as np
import pytest

from oracle import fem, lba
import workloads as W


def _rigid_modes(dim):
    nodes = fem.Q4_NODES if dim == 2 else fem.H8_NODES
    modes = []
    for c in range(dim):
        t = np.zeros((len(nodes), dim))
        t[:, c] = 1.0
        modes.append(t.ravel())
    axes = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in axes:
        r = np.zeros((len(nodes), dim))
        r[:, i] = -nodes[:, j]
        r[:, j] = nodes[:, i]
        modes.append(r.ravel())
    return np.array(modes).T


@pytest.mark.parametrize("dim", [2, 3])
def test_null_space_is_the_rigid_motions(dim):
    K = fem.element_stiffness(dim, 0.3, incompatible=True)
    assert np.abs(K - K.T).max() == 0.0
    ev = np.linalg.eigvalsh(K)
    nr = 3 if dim == 2 else 6
    assert np.all(ev[:nr] > -1e-12) and np.all(np.abs(ev[:nr]) < 1e-12) and ev[nr] > 1e-2
    R = _rigid_modes(dim)
    assert np.abs(K @ R).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_linear_fields(dim):
    nodes = fem.Q4_NODES if dim == 2 else fem.H8_NODES
    Ki = fem.element_stiffness(dim, 0.3, incompatible=True)
    Kc = fem.element_stiffness(dim, 0.3)
    rng = np.random.default_rng(7)
    for _ in range(5):
        Aff = rng.standard_normal((dim, dim))
        b = rng.standard_normal(dim)
        u = (nodes @ Aff.T + b).ravel()
        assert np.abs(Ki @ u - Kc @ u).max() < 1e-13


def _pure_bending(dim, nu, kappa):
    nodes = fem.Q4_NODES if dim == 2 else fem.H8_NODES
    u = []
    for p in nodes:
        x, y = float(p[0]), p[1] - 0.5
        if dim == 2:
            u += [kappa * x * y, -kappa * x * x / 2 - nu * kappa * y * y / 2]
        else:
            z = p[2] - 0.5
            u += [kappa * x * y, -kappa * x * x / 2 - nu * kappa * (y * y - z * z) / 2, -nu * kappa * y * z]
    return np.array(u)


@pytest.mark.parametrize("dim", [2, 3])
def test_pure_bending_energy_is_exact(dim):
    nu, kappa = 0.3, 0.7
    u = _pure_bending(dim, nu, kappa)
    exact = kappa ** 2 / 24.0              # 1/2 int E kappa^2 (y - 1/2)^2, E = 1
    Ki = fem.element_stiffness(dim, nu, incompatible=True)
    Kc = fem.element_stiffness(dim, nu)
    assert abs(0.5 * u @ Ki @ u - exact) <= 1e-14
    assert 0.5 * u @ Kc @ u > 1.4 * exact


def test_euler_column_converges_much_faster():
    def ratio(ny, element):
        nel = (20 * ny, ny)
        mat = fem.Material(element=element)
        x = np.ones(W.n_elems(nel))
        r = lba.analysis(nel, x, W.axial_load(nel), W.clamp_mask(nel), mat, ell=1, q=1, dense_limit=2000)
        L, H = nel
        PE = np.pi ** 2 * (H ** 3 / 12.0) / (4.0 * L * L)
        kGA = (5.0 / 6.0) * (1.0 / (2.0 * (1.0 + mat.nu))) * H
        return r["buck"].lam[0] / (PE / (1.0 + PE / kGA)) - 1.0
    e4, e8 = ratio(4, "incompatible"), ratio(8, "incompatible")
    c4 = ratio(4, "conforming")
    assert 0 < e8 < e4 < 1e-3
    assert e4 < c4 / 20
