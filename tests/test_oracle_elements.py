"""Pins of the oracle's element matrices and assembled operators (CPU only).

Each test checks the oracle against something other than itself: a published
closed form, an exact property of the finite-element space, or an exact
solution the element must reproduce.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, levels, lba
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
MAT = fem.Material()


def test_q4_stiffness_closed_form():
    # Published closed form of the unit-square bilinear plane-stress element
    # (E = 1, thickness 1), nodes counter-clockwise from (0,0).
    nu = 0.3
    k = [1 / 2 - nu / 6, 1 / 8 + nu / 8, -1 / 4 - nu / 12, -1 / 8 + 3 * nu / 8,
         -1 / 4 + nu / 12, -1 / 8 - nu / 8, nu / 6, 1 / 8 - 3 * nu / 8]
    idx = [[0, 1, 2, 3, 4, 5, 6, 7], [1, 0, 7, 6, 5, 4, 3, 2], [2, 7, 0, 5, 6, 3, 4, 1],
           [3, 6, 5, 0, 7, 2, 1, 4], [4, 5, 6, 7, 0, 1, 2, 3], [5, 4, 3, 2, 1, 0, 7, 6],
           [6, 3, 4, 1, 2, 7, 0, 5], [7, 2, 1, 4, 3, 6, 5, 0]]
    KE = np.array([[k[j] for j in row] for row in idx]) / (1 - nu * nu)
    assert np.abs(fem.element_stiffness(2, nu) - KE).max() < 1e-15


def test_q4_gradient_product_closed_form():
    Hxx = np.array([[2, -2, -1, 1], [-2, 2, 1, -1], [-1, 1, 2, -2], [1, -1, -2, 2]]) / 6.0
    H = fem.gradient_products(2)
    assert np.abs(H[0, 0] - Hxx).max() < 1e-15
    # y-derivative product is the same matrix with x and y swapped
    perm = [0, 3, 2, 1]  # reflect across the diagonal x <-> y
    assert np.abs(H[1, 1] - Hxx[np.ix_(perm, perm)]).max() < 1e-15


def _rigid_modes(dim):
    nodes = fem.local_nodes(dim).astype(float)
    nn = len(nodes)
    modes = []
    for c in range(dim):
        v = np.zeros((nn, dim)); v[:, c] = 1.0; modes.append(v.ravel())
    rots = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, b in rots:
        v = np.zeros((nn, dim)); v[:, a] = -nodes[:, b]; v[:, b] = nodes[:, a]; modes.append(v.ravel())
    return np.array(modes).T


@pytest.mark.parametrize("dim", [2, 3])
def test_element_symmetric_psd_rigid_nullspace(dim):
    K = fem.element_stiffness(dim, 0.3)
    assert np.abs(K - K.T).max() < 1e-15
    ev = np.linalg.eigvalsh(K)
    nrig = 3 if dim == 2 else 6
    assert np.all(np.abs(ev[:nrig]) < 1e-14)
    assert ev[nrig] > 1e-2
    R = _rigid_modes(dim)
    assert np.abs(K @ R).max() < 1e-14
    # stress stiffness annihilates translations (component-wise constants)
    s = np.random.default_rng(0).standard_normal(3 if dim == 2 else 6)
    G = fem.stress_stiffness_local(dim, s)
    assert np.abs(G @ R[:, :dim]).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_stress_stiffness_linear_field_closed_form(dim):
    # For a displacement field with constant gradient A (v_c = A_ci x_i),
    # v^T G_e v = sum_c sum_ij sigma_ij A_ci A_cj * volume (volume 1).
    rng = np.random.default_rng(1)
    A = rng.standard_normal((dim, dim))
    s = rng.standard_normal(3 if dim == 2 else 6)
    sig = np.zeros((dim, dim))
    for k, (i, j) in enumerate(fem.voigt_pairs(dim)):
        sig[i, j] = sig[j, i] = s[k]
    v = (fem.local_nodes(dim).astype(float) @ A.T).ravel()
    G = fem.stress_stiffness_local(dim, s)
    expect = np.einsum("ij,ci,cj->", sig, A, A)
    assert abs(v @ G @ v - expect) < 1e-13


@pytest.mark.parametrize("nel", [(6, 4), (4, 3, 3)])
def test_assembled_symmetry_and_nullity(nel):
    x = W.random_small(len(nel), nel, 3)
    K = fem.assemble_K(nel, x, MAT).toarray()
    assert np.abs(K - K.T).max() < 1e-15 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    nrig = 3 if len(nel) == 2 else 6
    assert np.all(np.abs(ev[:nrig]) < 1e-12 * ev[-1])
    assert ev[nrig] > 1e-9 * ev[-1]


@pytest.mark.parametrize("nel", [(5, 4), (3, 4, 2)])
def test_patch_test(nel):
    # Uniform material; prescribe an affine displacement at all boundary
    # nodes; the interior solution must reproduce it and the stress must be
    # the constant D0 * strain in every element.
    dim = len(nel)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((dim, dim)) * 1e-2
    b = rng.standard_normal(dim) * 1e-2
    nn = [v + 1 for v in nel]
    coords = np.stack([g.ravel() for g in reversed(np.meshgrid(*[np.arange(v) for v in reversed(nn)],
                                                              indexing="ij"))], axis=1).astype(float)
    uex = (coords @ A.T + b).ravel()
    onb = np.zeros(len(coords), dtype=bool)
    for ax in range(dim):
        onb |= (coords[:, ax] == 0) | (coords[:, ax] == nel[ax])
    fixed = np.repeat(onb, dim).astype(np.uint8)
    x = np.ones(W.n_elems(nel))
    K = fem.assemble_K(nel, x, MAT)
    free = np.flatnonzero(fixed == 0)
    fx = np.flatnonzero(fixed)
    rhs = -(K[free][:, fx] @ uex[fx])
    u = uex.copy()
    u[free] = spla.spsolve(K[free][:, free].tocsc(), rhs)
    assert np.abs(u - uex).max() < 1e-12
    s = fem.element_stresses(nel, x, u, MAT)
    eps = 0.5 * (A + A.T)
    if dim == 2:
        ev = np.array([eps[0, 0], eps[1, 1], 2 * eps[0, 1]])
    else:
        ev = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[0, 1], 2 * eps[1, 2], 2 * eps[0, 2]])
    sig = fem.constitutive(dim, MAT.nu) @ ev
    assert np.abs(s - sig[None]).max() < 1e-12


def test_uniaxial_bar_3d_exact():
    # Bar with roller supports on x = 0 (u_x = 0) plus two pins removing the
    # remaining rigid motions; a uniform unit traction on x = nx gives
    # u_x = x / (E A), lateral strain -nu/(E A): exact for H8.
    nel = (4, 2, 3)
    nx, ny, nz = nel
    mat = fem.Material(E0=0.0)
    x = np.ones(W.n_elems(nel))
    K = fem.constrain(fem.assemble_K(nel, x, mat), np.zeros(W.n_dofs(nel), np.uint8), 1.0)
    f = -W.axial_load(nel)          # tension +x, total 1
    fixed = np.zeros(W.n_dofs(nel), dtype=np.uint8)
    node = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    for j in range(ny + 1):
        for k in range(nz + 1):
            fixed[3 * node(0, j, k)] = 1
    fixed[3 * node(0, 0, 0) + 1] = fixed[3 * node(0, 0, 0) + 2] = 1
    fixed[3 * node(0, ny, 0) + 2] = 1
    fixed[3 * node(0, 0, nz) + 1] = 1
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    U, J, _ = lba.static_solve(K, f, fixed)
    u = U[:, 0]
    area = ny * nz
    for i in range(nx + 1):
        for j in range(ny + 1):
            for k in range(nz + 1):
                n = node(i, j, k)
                assert abs(u[3 * n] - i / area) < 1e-12
                assert abs(u[3 * n + 1] - (-mat.nu * j / area)) < 1e-12
                assert abs(u[3 * n + 2] - (-mat.nu * k / area)) < 1e-12


def test_energy_identity_and_scaling():
    nel = (12, 6)
    x = W.random_small(2, nel, 4)
    fixed = W.clamp_mask(nel)
    f = W.axial_load(nel)
    K = fem.constrain(fem.assemble_K(nel, x, MAT), fixed, 1.0)
    U, J, _ = lba.static_solve(K, f, fixed)
    u = U[:, 0]
    assert abs(J[0] - u @ (K @ u)) < 1e-12 * abs(J[0])
    U2, J2, _ = lba.static_solve(K, 3.0 * f, fixed)
    assert np.abs(U2[:, 0] - 3.0 * u).max() < 1e-12 * np.abs(u).max()
    mat2 = fem.Material(E1=5.0, E0=5e-6)
    K5 = fem.constrain(fem.assemble_K(nel, x, mat2), fixed, 1.0)
    U5, _, _ = lba.static_solve(K5, f, fixed)
    assert np.abs(U5[:, 0] - u / 5.0).max() < 1e-12 * np.abs(u).max()


def test_paper_size_pins():
    with open(os.path.join(HERE, "golden", "paper_sizes.json")) as fh:
        g = json.load(fh)
    assert W.n_dofs(tuple(g["frame_2d_coarse"]["nel"])) == g["frame_2d_coarse"]["dofs"]
    assert W.n_dofs(tuple(g["frame_2d_fine"]["nel"])) == g["frame_2d_fine"]["dofs"]
    c3 = g["cantilever_3d"]
    nel = tuple(c3["nel"])
    assert W.n_elems(nel) == c3["design_variables"]
    assert W.n_dofs(nel) == c3["dofs"]
    grids = levels.level_grids(nel, c3["coarse_level"])
    assert W.n_dofs(grids[-1]) == c3["coarse_dofs"]
    for ell, cut in g["dof_cut_2d"]["levels"].items():
        gr = levels.level_grids((840, 360), int(ell))
        ratio = W.n_dofs((840, 360)) / W.n_dofs(gr[-1])
        # the paper quotes the asymptotic factor 4^(l-1); node counts of the
        # (nx/2^(l-1) + 1)(ny/2^(l-1) + 1) grid sit a few percent below it
        assert cut == 4 ** (int(ell) - 1)
        assert 0.95 < ratio / cut <= 1.0


@pytest.mark.parametrize("nel", [(8, 4), (4, 4, 2)])
def test_prolongation_affine_exact(nel):
    dim = len(nel)
    P = levels.prolongation(nel)
    # rows sum to one per component
    rs = np.asarray(P.sum(axis=1)).ravel()
    assert np.abs(rs - 1.0).max() < 1e-15
    nc = levels.coarsen(nel)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((dim, dim)); b = rng.standard_normal(dim)

    def affine(g, h):
        nn = [v + 1 for v in g]
        co = np.stack([c.ravel() for c in reversed(np.meshgrid(*[np.arange(v) for v in reversed(nn)],
                                                               indexing="ij"))], axis=1) * h
        return (co @ A.T + b).ravel()
    assert np.abs(P @ affine(nc, 2.0) - affine(nel, 1.0)).max() < 1e-13


@pytest.mark.parametrize("nel,scale", [((8, 4), 1.0), ((4, 4, 2), 2.0)])
def test_galerkin_uniform_equals_coarse_assembly(nel, scale):
    # Nested conforming spaces: for uniform E the Galerkin operator equals the
    # matrix assembled directly on the coarse grid (element size h = 2):
    # h-independent in 2D, times h in 3D.  Same for G with uniform stress.
    dim = len(nel)
    nc = levels.coarsen(nel)
    P = levels.prolongation(nel)
    Kf = fem.assemble_K(nel, np.ones(W.n_elems(nel)), MAT)
    Kc = fem.assemble_K(nc, np.ones(W.n_elems(nc)), MAT)
    assert np.abs((P.T @ Kf @ P - scale * Kc).toarray()).max() < 1e-13
    s = np.random.default_rng(6).standard_normal(3 if dim == 2 else 6)
    Gf = fem.assemble_G(nel, np.tile(s, (W.n_elems(nel), 1)))
    Gc = fem.assemble_G(nc, np.tile(s, (W.n_elems(nc), 1)))
    assert np.abs((P.T @ Gf @ P - scale * Gc).toarray()).max() < 1e-13


def test_nested_fixed_set_check():
    nel = (8, 4)
    assert levels.nested_fixed_set_ok(nel, W.clamp_mask(nel))
    bad = np.zeros(W.n_dofs(nel), dtype=np.uint8)
    bad[2 * (1 + 9 * 2)] = 1      # fixed DOF at odd x node, sources free
    assert not levels.nested_fixed_set_ok(nel, bad)


def test_residual_extended_against_exact_rationals():
    """fem.residual_extended on a 3x2 Q4 grid with random densities and a
    random u of large amplitude (a rigid shift 1e6 plus a small field):
    against the exact residual in rational arithmetic (Fractions from the
    same float64 data), to a few units of its own rounding (far below the
    FP64 evaluation's error eps |K||u|)."""
    from fractions import Fraction
    import workloads as W
    from oracle import fem
    nel = (3, 2)
    mat = fem.Material()
    rng = np.random.default_rng(4)
    x = rng.uniform(0.01, 1.0, 6)
    fixed = W.clamp_mask(nel)
    n = fem.n_dofs(nel)
    u = 1e6 + rng.normal(size=n)
    u[fixed == 1] = 0.0
    f = rng.normal(size=n)
    r, absK = fem.residual_extended(nel, x, u, f, fixed, mat)
    Ke0 = fem.material_stiffness(2, mat)
    Ek, _ = fem.moduli(x, mat)
    ed = fem.element_dofs(nel)
    exact = [Fraction(v) for v in f]
    for e in range(6):
        for a in range(8):
            acc = Fraction(0)
            for b in range(8):
                acc += Fraction(Ke0[a, b]) * Fraction(u[ed[e, b]])
            exact[ed[e, a]] -= Fraction(Ek[e]) * acc
    ex = np.array([float(v) for v in exact])
    ex[fixed == 1] = 0.0
    # the FP64 evaluation misses by about eps |K||u|; the extended one by
    # about 2^-64 |K||u|
    fp64 = f - fem.apply_K_matfree(nel, x, u, mat)
    fp64[fixed == 1] = 0.0
    err_ext = np.abs(r - ex).max()
    err_64 = np.abs(fp64 - ex).max()
    assert err_ext <= 64 * 2.0 ** -64 * absK.max() + 2 * np.finfo(float).eps * np.abs(ex).max()
    assert err_ext * 100 < err_64


def test_refined_solve_reaches_the_extended_residual_floor():
    """On a nearly singular design (a solid bar in void, E0 = 1e-6) the
    refined solve's extended-precision solution has a residual far below
    the FP64 representation floor eps ||(|K||u|)|| / ||f||, and its rounding
    to doubles a residual at about that floor."""
    import workloads as W
    from oracle import fem, lba
    nel = (48, 16)
    x = np.full(48 * 16, 1e-6)
    x.reshape(16, 48)[6:10, :] = 1.0
    fixed = W.clamp_mask(nel)
    F = W.shear_load(nel, 1)
    mat = fem.Material()
    u, J, hist = lba.static_solve_refined(nel, x, F, fixed, mat)
    f = F * (fixed == 0)
    r, absK = fem.residual_extended(nel, x, u, f, fixed, mat)
    floor = np.finfo(float).eps * np.linalg.norm(absK) / np.linalg.norm(f)
    assert hist[-1] <= 1e-3 * floor and hist[-1] < hist[0]
    assert np.linalg.norm(r) / np.linalg.norm(f) <= floor
