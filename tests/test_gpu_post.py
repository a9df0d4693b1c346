"""Post-processing measures of local buckling (Sec. 5) through the C-ABI
against the oracle: energy-weighted modal correlation (eq.
macCorrelationIndex), strain energy density and its total variation (eq.
TVsed), local dilation (eq. postProcessingDilation).

Bars: correlations within twice the forward error bound of the product
A^T (K B) in FP64, (n + 81) eps |A|^T |K| |B| (81 = entries of a row of K;
both sides round); each density within twice the bound of its element
quadratic form, 2 nde eps E_e |phi_e|^T |K_e0| |phi_e|; the gradient within
the error that differencing such densities carries; total variations within
that per element plus the rounding of the sum.  The
dilation flags are a floating-point decision, so the oracle takes it on the
library's gradient; the dilated densities must then agree bit for bit.
Full size (192x64x64 H8, 12 modes): densities at sampled elements against
the oracle, the gradient on a full solid set against numpy.gradient of the
library's densities, and the dilation with every element flagged against
scipy's grey dilation with a ball footprint.
"""
import time

import numpy as np
import pytest
import scipy.ndimage as ndi

import workloads as W
from oracle import fem, post

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _step(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _ctx(nel, x, element, levels=2, ell=2):
    import paper_1909_13585_amd as mlb
    c = mlb.Context(nel, mg_levels=levels, eig_level=ell, element=element)
    c.set_bc(W.clamp_mask(nel))
    c.set_loads(W.axial_load(nel)[:, None])
    c.set_density(x)
    return c


def _check_mac(C, K, A, B):
    """C against A^T K B (A, B: n x q numpy) within the product's rounding bound."""
    ref = post.mac(K, A, B)
    bound = 2.0 * (A.shape[0] + 81) * np.finfo(np.float64).eps * (np.abs(A).T @ (abs(K) @ np.abs(B)))
    assert C.shape == ref.shape
    assert np.all(np.abs(C - ref) <= bound), np.max(np.abs(C - ref) / bound)


def _sed_bound(nel, x, Phi_cols, mat, elements=None):
    """Rounding bound of each element density: 2 (2 nde) eps E_e |phi_e|^T |K_e0| |phi_e|."""
    dim = len(nel)
    K0 = np.abs(fem.material_stiffness(dim, mat))
    Ek, _ = fem.moduli(np.asarray(x, dtype=np.float64), mat)
    ed = fem.element_dofs(nel)
    if elements is not None:
        ed, Ek = ed[elements], Ek[elements]
    nde = ed.shape[1]
    out = []
    for j in range(Phi_cols.shape[1]):
        P = np.abs(Phi_cols[ed, j])
        out.append(2.0 * 2 * nde * np.finfo(np.float64).eps * Ek * np.einsum("ei,ij,ej->e", P, K0, P))
    return np.array(out)


def _check_sed_tv(torch, c, nel, x, Phi, mat, xbar):
    q = Phi.shape[0]
    sed = torch.empty((q, c.m), dtype=torch.float64, device="cuda")
    gradn = torch.empty_like(sed)
    tv = c.sed_tv_dev(Phi, xbar, sed, gradn)
    torch.cuda.synchronize()
    sed_h, g_h = sed.cpu().numpy(), gradn.cpu().numpy()
    Ph = Phi.cpu().numpy().T
    ref = post.strain_energy_density(nel, x, Ph, mat)
    bnd = _sed_bound(nel, x, Ph, mat)
    assert np.all(np.abs(sed_h - ref) <= bnd), np.max(np.abs(sed_h - ref) / bnd)
    solid = x >= xbar
    eps = np.finfo(np.float64).eps
    for i in range(q):
        tv_o, g_o = post.total_variation(nel, ref[i], x, xbar)
        # a difference of two densities carries both their errors; sqrt(dim) axes
        tol_g = 2.0 * np.sqrt(len(nel)) * bnd[i].max() + 8 * eps * g_o.max()
        assert np.abs(g_h[i] - g_o).max() <= tol_g, i
        assert abs(tv[i] - tv_o) <= solid.sum() * tol_g + 2 * len(x) * eps * tv_o, (i, tv[i], tv_o)
        assert np.all(g_h[i][~solid] == 0.0)
    return sed_h, g_h, tv


@pytest.mark.parametrize("nel,element", [((60, 20), 0), ((60, 20), 1), ((20, 12, 12), 0), ((20, 12, 12), 1)])
def test_measures_of_buckling_modes(torch_mod, nel, element):
    """Modes of a buckling analysis (m = 1200 / 2880: several blocks and a ragged tail)."""
    torch = torch_mod
    _step(f"post-processing of modes nel={nel} element={element}")
    x = W.density_uniform_noise(nel, 21, sigma=1.0)
    mat = fem.Material(element="incompatible" if element else "conforming")
    c = _ctx(nel, x, element)
    U = torch.empty((1, c.n), dtype=torch.float64, device="cuda")
    c.solve_static_dev(U, tol=1e-10, max_it=3000)
    q = 6
    Phi = torch.empty((q, c.n), dtype=torch.float64, device="cuda")
    c.buckling_dev(q, Phi, tol_eig=1e-10)
    # correlation of the modes with themselves and with a perturbed copy
    fixed = W.clamp_mask(nel)
    K = fem.constrain(fem.assemble_K(nel, x, mat), fixed, 1.0)
    B = Phi.clone()
    B[:3] += 0.05 * torch.randn((3, c.n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(2))
    Wk = torch.empty_like(B)
    C = c.mac_dev(Phi, B, Wk)
    _check_mac(C, K, Phi.cpu().numpy().T, B.cpu().numpy().T)
    assert np.abs(np.diag(C)[3:] - 1.0).max() < 1e-8
    # densities, gradients and total variations on the solid set, two thresholds
    for xbar in (0.5, 0.0):
        _, g_h, tv = _check_sed_tv(torch, c, nel, x, Phi, mat, xbar)
    # dilation around the two modes with the largest normalised variation
    sel = np.argsort(tv / tv[0])[-2:]
    gsel = torch.from_numpy(np.ascontiguousarray(g_h[sel])).cuda()
    xd = torch.from_numpy(x).cuda()
    for rel_thr, r_th in ((1e-2, 1.5), (0.3, 2.0), (0.9, 1.0)):
        xo = torch.empty_like(xd)
        c.dilate_dev(gsel, rel_thr, r_th, xd, xo)
        torch.cuda.synchronize()
        ref = post.dilate(nel, x, post.dilation_flags(g_h[sel], rel_thr), r_th)
        assert np.array_equal(xo.cpu().numpy(), ref), (rel_thr, r_th)
    c.close()


@pytest.mark.parametrize("nel", [(52, 20), (20, 12, 10)])
def test_measures_of_random_blocks_ragged(torch_mod, nel):
    """Random blocks (not zero at fixed DOFs), a mostly solid design, one level
    (m = 1040 / 2400: a ragged last block)."""
    torch = torch_mod
    _step(f"post-processing of random blocks nel={nel}")
    rng = np.random.default_rng(8)
    x = np.where(rng.uniform(size=W.n_elems(nel)) < 0.7, 1.0, 1e-3) * rng.uniform(0.8, 1.0, W.n_elems(nel))
    c = _ctx(nel, x, 0, levels=1, ell=1)
    mat = fem.Material()
    A = torch.from_numpy(rng.standard_normal((5, c.n))).cuda()
    B = torch.from_numpy(rng.standard_normal((3, c.n))).cuda()
    Wk = torch.empty_like(B)
    C = c.mac_dev(A, B, Wk)
    K = fem.constrain(fem.assemble_K(nel, x, mat), W.clamp_mask(nel), 1.0)
    assert C.shape == (5, 3)
    _check_mac(C, K, A.cpu().numpy().T, B.cpu().numpy().T)
    _, g_h, _ = _check_sed_tv(torch, c, nel, x, A, mat, 0.8)
    xd = torch.from_numpy(x).cuda()
    xo = torch.empty_like(xd)
    c.dilate_dev(torch.from_numpy(np.ascontiguousarray(g_h[1:4])).cuda(), 0.05, 2.5, xd, xo)
    torch.cuda.synchronize()
    assert np.array_equal(xo.cpu().numpy(), post.dilate(nel, x, post.dilation_flags(g_h[1:4], 0.05), 2.5))
    # nothing flagged (all-zero gradients): identity
    c.dilate_dev(torch.zeros((1, c.m), dtype=torch.float64, device="cuda"), 0.5, 3.0, xd, xo)
    torch.cuda.synchronize()
    assert np.array_equal(xo.cpu().numpy(), x)
    c.close()


def test_argument_errors(torch_mod):
    torch = torch_mod
    import paper_1909_13585_amd as mlb
    nel = (8, 4)
    c = _ctx(nel, np.full(32, 0.5), 0, levels=1, ell=1)
    g = torch.zeros((1, c.m), dtype=torch.float64, device="cuda")
    xd = torch.full((c.m,), 0.5, dtype=torch.float64, device="cuda")
    xo = torch.empty_like(xd)
    for r_th, thr in ((9.0, 0.1), (-1.0, 0.1), (1.0, -0.5), (1.0, float("nan"))):
        with pytest.raises(mlb.MlbError):
            c.dilate_dev(g, thr, r_th, xd, xo)
    with pytest.raises(mlb.MlbError):
        c.dilate_dev(g, 0.1, 1.0, xd, xd)
    A = torch.zeros((100, c.n), dtype=torch.float64, device="cuda")
    with pytest.raises(mlb.MlbError):
        c.mac_dev(A, A, torch.empty_like(A))
    c.close()


def test_full_size_box(torch_mod):
    torch = torch_mod
    import paper_1909_13585_amd as mlb
    nel = (192, 64, 64)
    _step(f"post-processing full size nel={nel}, 12 random columns")
    p = W.box_3d(nel=nel)
    x = p["x"]
    c = mlb.Context(nel, mg_levels=1, eig_level=1)      # one level: no multigrid hierarchy needed
    c.set_bc(p["fixed"])
    c.set_loads(p["F"])
    c.set_density(x)
    q = 12
    Phi = torch.randn((q, c.n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    sed = torch.empty((q, c.m), dtype=torch.float64, device="cuda")
    gradn = torch.empty_like(sed)
    xbar = float(x.min()) - 1.0        # every element solid
    tv = c.sed_tv_dev(Phi, xbar, sed, gradn)
    torch.cuda.synchronize()
    sed_h, g_h = sed.cpu().numpy(), gradn.cpu().numpy()
    rng = np.random.default_rng(6)
    els = np.concatenate([[0, c.m - 1, 191, 192 * 64 - 1], rng.integers(0, c.m, 60)])
    Phi_h = Phi.cpu().numpy().T
    ref = post.strain_energy_density(nel, x, Phi_h, fem.Material(), elements=els)
    bnd = _sed_bound(nel, x, Phi_h, fem.Material(), elements=els)
    assert np.all(np.abs(sed_h[:, els] - ref) <= bnd)
    for i in (0, 7, 11):
        G = np.gradient(sed_h[i].reshape(64, 64, 192), edge_order=1)
        gn = np.sqrt(G[0] ** 2 + G[1] ** 2 + G[2] ** 2).ravel()
        assert np.abs(g_h[i] - gn).max() <= 1e-13 * np.abs(sed_h[i]).max()
        assert abs(tv[i] - gn.sum()) <= 2 * c.m * np.finfo(np.float64).eps * gn.sum()
    xd = torch.from_numpy(x).cuda()
    xo = torch.empty_like(xd)
    c.dilate_dev(gradn[:2], 0.0, 2.0, xd, xo)      # rel_thr 0: every element flagged
    torch.cuda.synchronize()
    o = np.indices((5, 5, 5)) - 2
    fp = (o ** 2).sum(0) <= 4
    ref = ndi.grey_dilation(x.reshape(64, 64, 192), footprint=fp, mode="constant", cval=-np.inf).ravel()
    assert np.array_equal(xo.cpu().numpy(), ref)
    c.close()
