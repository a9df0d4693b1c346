"""The paper's incompatible-mode elements (Q6/H11, Sec. 2; MLB_ELEM_INCOMPATIBLE)
through the whole analysis against the oracle built with the same element:
static solve, multilevel buckling factors and modes, compliance and
buckling-factor sensitivities, to the bars of test_gpu_analysis; plus every
level's K apply element-wise and the element's effect on an Euler column.
"""
import numpy as np
import pytest

from gpu_util import rel_inf
from oracle import fem, lba, sens
import workloads as W
import test_gpu_analysis as TA

pytestmark = pytest.mark.gpu
MAT_I = fem.Material(element="incompatible")


def _run(nel, x, F, fixed, L, ell, k, precision=0):
    import paper_1909_13585_amd as mlb
    c = mlb.Context(nel, mg_levels=L, eig_level=ell, precision=precision, element=mlb.MLB_ELEM_INCOMPATIBLE)
    c.set_bc(fixed)
    c.set_loads(F)
    c.set_density(x)
    U, J, si = c.solve_static(tol=1e-10, max_it=2000)
    lam, Phi, ei = c.buckling(k, tol_eig=1e-11)
    res = c.eig_residuals()
    dJ, dl, ai = c.sensitivities()
    c.close()
    return dict(U=U, J=J, si=si, lam=lam, Phi=Phi, ei=ei, res=res, dJ=dJ, dl=dl, ai=ai)


def _oracle(nel, x, F, fixed, ell, k, L):
    ref = lba.analysis(nel, x, F, fixed, MAT_I, ell=ell, q=k)
    if ell > 1:
        ref["buck"] = lba.multilevel_buckling(nel, x, ref["u"], fixed, MAT_I, ell, k, mg_levels=L, K=ref["K"],
                                              G=ref["G"], solver=ref["solver"])
    ref["dJ"] = sens.compliance_sensitivity(nel, x, ref["U"], MAT_I)
    ref["dl"], _ = sens.buckling_sensitivity(nel, x, ref["u"], ref["buck"].lam, ref["buck"].phi, fixed, MAT_I,
                                             ref["solver"])
    return ref


@pytest.mark.parametrize("ell,precision", [(1, 0), (2, 0), (2, 1)])
def test_column_2d(ell, precision):
    p = W.column_2d_small()
    nel, k, L = p["nel"], 6, 3
    print(f"case incompatible column_2d_small ell={ell} precision={precision}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, ell, k, precision)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], ell, k, L)
    print("lam", g["lam"], "oracle", ref["buck"].lam)
    TA._check(g, ref, p["fixed"], p["F"], k)


def test_box_3d():
    nel = (32, 8, 8)
    p = W.box_3d(nel=nel, seed=5, sigma=2.0)
    k, L, ell = 4, 3, 2
    print(f"case incompatible box_3d nel={nel}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, ell, k)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], ell, k, L)
    print("lam", g["lam"], "oracle", ref["buck"].lam)
    TA._check(g, ref, p["fixed"], p["F"], k)


@pytest.mark.parametrize("nel", [(24, 8), (16, 8, 8)])
def test_fine_apply_matches_element_loop(nel):
    """The public fine apply (every variant in 3D) against the oracle's element
    loop with the condensed element, input not zero at Dirichlet DOFs."""
    import torch
    import paper_1909_13585_amd as mlb
    x = W.random_small(len(nel), nel, 9, lo=0.1, hi=1.0)
    fixed = W.clamp_mask(nel)
    c = mlb.Context(nel, mg_levels=2, eig_level=2, element=mlb.MLB_ELEM_INCOMPATIBLE)
    c.set_bc(fixed)
    c.set_loads(W.axial_load(nel)[:, None])
    c.set_density(x)
    v = np.random.default_rng(3).standard_normal(c.n)
    xin = v.copy()
    xin[fixed != 0] = 0.0
    ref = fem.apply_K_matfree(nel, x, xin, MAT_I)
    ref[fixed != 0] = v[fixed != 0]
    for var in ((0, 1, 2, 3) if len(nel) == 3 else (-1,)):
        if var >= 0:
            c.set_tiles(0, 0, var)
        y = torch.empty(c.n, dtype=torch.float64, device="cuda")
        c.apply_K_dev(1, torch.from_numpy(v).cuda(), y)
        torch.cuda.synchronize()
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (var, err)
    c.close()


def test_euler_column_is_closer_with_the_incompatible_element():
    import paper_1909_13585_amd as mlb
    ny = 4
    nel = (20 * ny, ny)
    x = np.ones(W.n_elems(nel))
    L, H = nel
    PE = np.pi ** 2 * (H ** 3 / 12.0) / (4.0 * L * L)
    kGA = (5.0 / 6.0) * (1.0 / (2.0 * 1.3)) * H
    target = PE / (1.0 + PE / kGA)
    errs = {}
    for el in (mlb.MLB_ELEM_CONFORMING, mlb.MLB_ELEM_INCOMPATIBLE):
        c = mlb.Context(nel, mg_levels=2, eig_level=1, element=el)
        c.set_bc(W.clamp_mask(nel))
        c.set_loads(W.axial_load(nel)[:, None])
        c.set_density(x)
        c.solve_static(tol=1e-12, max_it=4000)
        lam, _, _ = c.buckling(1, tol_eig=1e-12, want_modes=False)
        c.close()
        errs[el] = lam[0] / target - 1
    print(errs)
    assert 0 < errs[mlb.MLB_ELEM_INCOMPATIBLE] < errs[mlb.MLB_ELEM_CONFORMING] / 20
