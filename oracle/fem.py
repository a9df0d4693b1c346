"""Element matrices and assembled operators (oracle; test infrastructure only).

Follows Sec. 2 of the paper: K = K[x] assembled from K_e = E_kappa(x_e) K_e0,
G = G[x, u] assembled from G_e = E_sigma(x_e) G_e0[u_e], with the two SIMP
interpolations of eq. interpolationSIMP2-SIMP.

Readings (the paper is silent or chooses otherwise):
  * Elements: bilinear Q4 (2D, plane stress, unit thickness) and trilinear H8
    (3D) on unit squares/cubes by default.  The paper's own incompatible
    elements (Q6/H11, Sec. 2) are the option ``Material.element =
    "incompatible"``: every displacement component gets one extra mode
    4 x_m (1 - x_m) per axis m (zero at the nodes), condensed out element by
    element (K_e0 = K_cc - K_ci K_ii^-1 K_ic).  On rectangles these modes pass
    the patch test without correction.
  * K_e0 = integral of B^T D0 B with 2 Gauss points per axis (exact on a
    rectangle, also with the incompatible modes); D0 is the unit-modulus
    constitutive matrix.
  * With the incompatible element, G_e0 keeps the bilinear/trilinear
    interpolation (the condensed modes do not enter the stress stiffness),
    and the centroid stress is unchanged: the modes' gradients vanish there.
  * G_e0[u_e] uses ONE stress per element, evaluated at the element centroid:
    sigma0 = D0 B_c u_e, and G_e0 = (sum_ij sigma0_ij H^ij) kron I_d with
    H^ij = integral of dN/dx_i dN/dx_j^T.  The stress entering G is therefore
    E_sigma(x_e) * D0 B_c u_e.
  * Dirichlet DOFs: identity rows/columns in K, zero rows/columns in G.

Local node order here is counter-clockwise (Q4) and bottom-face then top-face
(H8); global vectors use node = i + (nx+1)(j + (ny+1)k), dof = d*node + c.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

Q4_NODES = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.int64)
H8_NODES = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


@dataclass(frozen=True)
class Material:
    """SIMP data of eq. interpolationSIMP2-SIMP: E1, E0, Poisson ratio, penalty;
    element "conforming" (Q4/H8) or "incompatible" (Q6/H11)."""
    E1: float = 1.0
    E0: float = 1e-6
    nu: float = 0.3
    p: float = 3.0
    element: str = "conforming"


def local_nodes(dim):
    return Q4_NODES if dim == 2 else H8_NODES


def constitutive(dim, nu):
    """Unit-modulus D0: plane stress (2D, Voigt xx,yy,xy) or isotropic 3D
    (Voigt xx,yy,zz,xy,yz,xz) with engineering shear strains."""
    if dim == 2:
        return np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, (1.0 - nu) / 2.0]]) / (1.0 - nu * nu)
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def shape_gradients(dim, pt):
    """dN_a/dx_i at reference point ``pt`` in [0,1]^dim for the unit element.
    Returns array (nn, dim)."""
    nodes = local_nodes(dim)
    nn = len(nodes)
    grads = np.zeros((nn, dim))
    for a in range(nn):
        for i in range(dim):
            g = 1.0
            for k in range(dim):
                if k == i:
                    g *= 1.0 if nodes[a, k] == 1 else -1.0
                else:
                    g *= pt[k] if nodes[a, k] == 1 else 1.0 - pt[k]
            grads[a, i] = g
    return grads


def gauss_points(dim):
    """2-point Gauss-Legendre per axis on [0,1]: points and weights."""
    g = 0.5 / np.sqrt(3.0)
    pts1 = [0.5 - g, 0.5 + g]
    if dim == 2:
        pts = [np.array([a, b]) for b in pts1 for a in pts1]
    else:
        pts = [np.array([a, b, c]) for c in pts1 for b in pts1 for a in pts1]
    w = 1.0 / len(pts)
    return pts, [w] * len(pts)


def strain_matrix(dim, pt):
    """B (nv x nde) at ``pt``: strains (Voigt, engineering shear) from nodal
    displacements ordered (node a, component c) -> row-index d*a + c."""
    G = shape_gradients(dim, pt)
    nn = G.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * nn))
        for a in range(nn):
            gx, gy = G[a]
            B[0, 2 * a] = gx
            B[1, 2 * a + 1] = gy
            B[2, 2 * a] = gy
            B[2, 2 * a + 1] = gx
        return B
    B = np.zeros((6, 3 * nn))
    for a in range(nn):
        gx, gy, gz = G[a]
        B[0, 3 * a] = gx
        B[1, 3 * a + 1] = gy
        B[2, 3 * a + 2] = gz
        B[3, 3 * a] = gy
        B[3, 3 * a + 1] = gx
        B[4, 3 * a + 1] = gz
        B[4, 3 * a + 2] = gy
        B[5, 3 * a] = gz
        B[5, 3 * a + 2] = gx
    return B


def bubble_strain_matrix(dim, pt):
    """Strains (nv x dim^2) of the incompatible modes: column d*c + m is the
    field u_c = 4 x_m (1 - x_m) (component c, axis m)."""
    pairs = voigt_pairs(dim)
    Bt = np.zeros((len(pairs), dim * dim))
    for c in range(dim):
        for m in range(dim):
            grad = np.zeros(dim)            # d u_c / d x_k
            grad[m] = 4.0 - 8.0 * pt[m]
            for k, (i, j) in enumerate(pairs):
                if i == j:
                    Bt[k, dim * c + m] = grad[i] if c == i else 0.0
                else:
                    Bt[k, dim * c + m] = (grad[j] if c == i else 0.0) + (grad[i] if c == j else 0.0)
    return Bt


def element_stiffness(dim, nu, incompatible=False):
    """K_e0 = sum over Gauss points of w B^T D0 B (unit modulus, unit element);
    with ``incompatible``, the incompatible modes are added and condensed."""
    D = constitutive(dim, nu)
    pts, ws = gauss_points(dim)
    nde = dim * (2 ** dim)
    K = np.zeros((nde, nde))
    Kci = np.zeros((nde, dim * dim))
    Kii = np.zeros((dim * dim, dim * dim))
    for pt, w in zip(pts, ws):
        B = strain_matrix(dim, pt)
        K += w * B.T @ D @ B
        if incompatible:
            Bt = bubble_strain_matrix(dim, pt)
            Kci += w * B.T @ D @ Bt
            Kii += w * Bt.T @ D @ Bt
    if incompatible:
        K = K - Kci @ np.linalg.solve(Kii, Kci.T)
        K = 0.5 * (K + K.T)
    return K


def material_stiffness(dim, mat):
    """K_e0 of the element the material selects."""
    return element_stiffness(dim, mat.nu, incompatible=(mat.element == "incompatible"))


def gradient_products(dim):
    """H[i][j] = integral over the unit element of dN/dx_i dN/dx_j^T (nn x nn)."""
    pts, ws = gauss_points(dim)
    nn = 2 ** dim
    H = np.zeros((dim, dim, nn, nn))
    for pt, w in zip(pts, ws):
        G = shape_gradients(dim, pt)
        for i in range(dim):
            for j in range(dim):
                H[i, j] += w * np.outer(G[:, i], G[:, j])
    return H


def voigt_pairs(dim):
    """(i, j) index pair of each Voigt stress component."""
    if dim == 2:
        return [(0, 0), (1, 1), (0, 1)]
    return [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]


def stress_stiffness_local(dim, s):
    """G_e for one element from its Voigt stress ``s``:
    (sum_ij sigma_ij H^ij) kron I_d, both (i,j) and (j,i) for shear terms."""
    H = gradient_products(dim)
    nn = 2 ** dim
    g = np.zeros((nn, nn))
    for k, (i, j) in enumerate(voigt_pairs(dim)):
        if i == j:
            g += s[k] * H[i, i]
        else:
            g += s[k] * (H[i, j] + H[j, i])
    return np.kron(g, np.eye(dim))


def element_dofs(nel):
    """(m, nde) global DOF numbers of every element in this module's local order."""
    dim = len(nel)
    nodes = local_nodes(dim)
    nx, ny = nel[0], nel[1]
    nz = nel[2] if dim == 3 else 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    cols = []
    for a in range(len(nodes)):
        if dim == 2:
            node = (i + nodes[a, 0]) + (nx + 1) * (j + nodes[a, 1])
        else:
            node = (i + nodes[a, 0]) + (nx + 1) * ((j + nodes[a, 1]) + (ny + 1) * (k + nodes[a, 2]))
        for c in range(dim):
            cols.append(dim * node + c)
    return np.stack(cols, axis=1).astype(np.int64)


def n_dofs(nel):
    n = len(nel)
    for v in nel:
        n *= v + 1
    return n


def moduli(x, mat):
    """E_kappa and E_sigma of eq. interpolationSIMP2-SIMP."""
    xp = np.power(x, mat.p)
    return mat.E0 + xp * (mat.E1 - mat.E0), xp * mat.E1


def assemble(nel, elem_mats):
    """Sparse sum_e P_e^T A_e P_e from per-element dense matrices (m, nde, nde)."""
    ed = element_dofs(nel)
    n = n_dofs(nel)
    nde = ed.shape[1]
    rows = np.repeat(ed, nde, axis=1).ravel()
    cols = np.tile(ed, (1, nde)).ravel()
    return sp.csr_matrix((elem_mats.ravel(), (rows, cols)), shape=(n, n))


def assemble_K(nel, x, mat):
    """Unconstrained K[x] = sum_e E_kappa(x_e) K_e0 (Sec. 2)."""
    dim = len(nel)
    Ke0 = material_stiffness(dim, mat)
    Ek, _ = moduli(np.asarray(x, dtype=np.float64), mat)
    ed = element_dofs(nel)
    n = n_dofs(nel)
    nde = ed.shape[1]
    rows = np.repeat(ed, nde, axis=1).ravel()
    cols = np.tile(ed, (1, nde)).ravel()
    data = (Ek[:, None, None] * Ke0[None]).ravel()
    return sp.csr_matrix((data, (rows, cols)), shape=(n, n))


def element_stresses(nel, x, u, mat):
    """Voigt stress per element E_sigma(x_e) D0 B_c u_e at the centroid (m, nv)."""
    dim = len(nel)
    D = constitutive(dim, mat.nu)
    Bc = strain_matrix(dim, np.full(dim, 0.5))
    _, Es = moduli(np.asarray(x, dtype=np.float64), mat)
    ue = np.asarray(u)[element_dofs(nel)]
    return Es[:, None] * (ue @ (D @ Bc).T)


def assemble_G(nel, s):
    """Unconstrained G = sum_e G_e from per-element stresses ``s`` (m, nv)."""
    dim = len(nel)
    H = gradient_products(dim)
    nn = 2 ** dim
    pairs = voigt_pairs(dim)
    g = np.zeros((s.shape[0], nn, nn))
    for k, (i, j) in enumerate(pairs):
        Hk = H[i, i] if i == j else H[i, j] + H[j, i]
        g += s[:, k, None, None] * Hk[None]
    Ge = np.einsum("eab,cd->eacbd", g, np.eye(dim)).reshape(s.shape[0], nn * dim, nn * dim)
    return assemble(nel, Ge)


def constrain(A, fixed, diag_value):
    """M A M + diag_value (I - M), M = diag(free): identity (K) or zero (G)
    rows and columns at Dirichlet DOFs."""
    free = (np.asarray(fixed) == 0).astype(np.float64)
    M = sp.diags(free)
    return (M @ A @ M + sp.diags(diag_value * (1.0 - free))).tocsr()


def apply_K_matfree(nel, x, v, mat):
    """y = K[x] v by an element loop (no assembly); for large-size checks."""
    dim = len(nel)
    Ke0 = material_stiffness(dim, mat)
    Ek, _ = moduli(np.asarray(x, dtype=np.float64), mat)
    ed = element_dofs(nel)
    contrib = Ek[:, None] * (np.asarray(v)[ed] @ Ke0.T)
    return np.bincount(ed.ravel(), weights=contrib.ravel(), minlength=n_dofs(nel))


def residual_extended(nel, x, u, f, fixed, mat):
    """r = f - K[x] u on the free DOFs (zero at fixed ones), evaluated in the
    platform's extended precision (numpy longdouble: a 64-bit significand on
    x86-64) by an element loop, then rounded to float64; u may be float64 or
    longdouble.  On x86-64 it is
    about 2000 times closer to the exact residual of the stored u than an
    FP64 evaluation, whose own rounding (eps |K||u|) hides the residual of
    nearly singular designs.  Also returns |K||u| (free DOFs, float64)."""
    ld = np.longdouble
    dim = len(nel)
    Ke0 = material_stiffness(dim, mat).astype(ld)
    Ek, _ = moduli(np.asarray(x, dtype=np.float64), mat)
    ed = element_dofs(nel)
    uu = np.asarray(u)
    ue = (uu if uu.dtype == ld else uu.astype(np.float64))[ed].astype(ld)
    contrib = Ek.astype(ld)[:, None] * (ue @ Ke0.T)
    Ku = np.zeros(n_dofs(nel), dtype=ld)
    np.add.at(Ku, ed.ravel(), contrib.ravel())
    # |K||u| entrywise: sum over the row's terms of |E_e K0_ab u_b|
    acontrib = Ek[:, None] * (np.abs(uu.astype(np.float64)[ed]) @ np.abs(material_stiffness(dim, mat)).T)
    absK = np.bincount(ed.ravel(), weights=acontrib.ravel(), minlength=n_dofs(nel))
    free = np.asarray(fixed) == 0
    r = (np.asarray(f, dtype=np.float64).astype(ld) - Ku).astype(np.float64)
    r[~free] = 0.0
    absK[~free] = 0.0
    return r, absK


def apply_G_matfree(nel, s, v):
    """y = G v by an element loop from per-element stresses ``s``."""
    dim = len(nel)
    H = gradient_products(dim)
    nn = 2 ** dim
    g = np.zeros((s.shape[0], nn, nn))
    for k, (i, j) in enumerate(voigt_pairs(dim)):
        Hk = H[i, i] if i == j else H[i, j] + H[j, i]
        g += s[:, k, None, None] * Hk[None]
    ed = element_dofs(nel)
    ve = np.asarray(v)[ed].reshape(-1, nn, dim)
    contrib = np.einsum("eab,ebc->eac", g, ve).reshape(s.shape[0], nn * dim)
    return np.bincount(ed.ravel(), weights=contrib.ravel(), minlength=n_dofs(nel))
