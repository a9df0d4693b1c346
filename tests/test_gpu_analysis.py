"""GPU parity of the full analysis (static solve, multilevel buckling,
sensitivities) against the CPU oracle, through the C ABI.

Tolerances (normwise readings of the stated targets):
  * static solve: true relative residual <= 1e-8 measured with the oracle's K;
  * buckling factors (coarse and fine): relative error <= 1e-6 each;
  * modes: |phi_gpu^T K phi_oracle| >= 1 - 1e-6 for modes separated by >1e-3;
  * sensitivities: ||s_gpu - s_oracle||_inf <= 1e-5 ||s_oracle||_inf.
"""
import numpy as np
import pytest

from gpu_util import MAT, rel_inf
from oracle import fem, lba, sens
import workloads as W

pytestmark = pytest.mark.gpu


def _run(nel, x, F, fixed, L, ell, k, precision=0, tol=1e-10, tol_eig=1e-11):
    import paper_1909_13585_amd as mlb
    c = mlb.Context(nel, mg_levels=L, eig_level=ell, precision=precision)
    c.set_bc(fixed)
    c.set_loads(F)
    c.set_density(x)
    U, J, si = c.solve_static(tol=tol, max_it=2000)
    lam, Phi, ei = c.buckling(k, tol_eig=tol_eig)
    res = c.eig_residuals()
    dJ, dl, ai = c.sensitivities()
    c.close()
    return dict(U=U, J=J, si=si, lam=lam, Phi=Phi, ei=ei, res=res, dJ=dJ, dl=dl, ai=ai)


def _oracle(nel, x, F, fixed, ell, k, L):
    ref = lba.analysis(nel, x, F, fixed, MAT, ell=ell, q=k)
    if ell > 1:
        ref["buck"] = lba.multilevel_buckling(nel, x, ref["u"], fixed, MAT, ell, k, mg_levels=L, K=ref["K"],
                                              G=ref["G"], solver=ref["solver"])
    dJ = sens.compliance_sensitivity(nel, x, ref["U"], MAT)
    dl, _ = sens.buckling_sensitivity(nel, x, ref["u"], ref["buck"].lam, ref["buck"].phi, fixed, MAT,
                                      ref["solver"])
    ref["dJ"], ref["dl"] = dJ, dl
    return ref


def _check(g, ref, fixed, F, k, lam_tol=1e-6):
    K = ref["K"]
    # static: true residual with the oracle operator.  1e-8 relative, or 4x
    # the FP64 floor eps*|| |K||u| ||/||f|| where that floor is higher (3D
    # fields with large void fractions: even the oracle's direct solve sits
    # at ~half the floor there).
    absK = abs(K)
    for cse in range(g["U"].shape[1]):
        f = K @ ref["U"][:, cse]
        u = g["U"][:, cse]
        r = f - K @ u
        floor = 2.2e-16 * np.linalg.norm(absK @ np.abs(u))
        assert np.linalg.norm(r) <= max(1e-8 * np.linalg.norm(f), 4 * floor)
    # compliance: with f = K u_o (the load u_o solves exactly) and the true
    # load F = f + r_o, J_gpu - J_oracle = F^T (u_g - u_o)
    #   = -u_o^T (f - K u_g) + r_o^T (u_g - u_o), hence the bound below.
    for cse in range(g["U"].shape[1]):
        uo, ug = ref["U"][:, cse], g["U"][:, cse]
        Fc = F[:, cse] * (fixed == 0)
        f = K @ uo
        bound = (1e-12 * abs(ref["J"][cse]) + np.linalg.norm(uo) * np.linalg.norm(f - K @ ug)
                 + np.linalg.norm(Fc - f) * np.linalg.norm(ug - uo))
        assert abs(g["J"][cse] - ref["J"][cse]) <= bound
    b = ref["buck"]
    assert np.all(np.abs(g["lam"] / b.lam - 1) < lam_tol), (g["lam"], b.lam)
    # modes: K-inner product with the oracle's modes, separated ones only
    lam = b.lam
    for i in range(k):
        gaps = [abs(lam[i] - lam[j]) / lam[i] for j in range(k) if j != i]
        if min(gaps) > 1e-3:
            mac = abs(g["Phi"][:, i] @ (K @ b.phi[:, i]))
            assert mac > 1 - 1e-6, (i, mac)
    assert rel_inf(g["dJ"], ref["dJ"]) < 1e-5
    for i in range(k):
        gaps = [abs(lam[i] - lam[j]) / lam[i] for j in range(k) if j != i]
        if min(gaps) > 1e-3:
            assert rel_inf(g["dl"][:, i], ref["dl"][:, i]) < 1e-5, i


@pytest.mark.parametrize("ell", [1, 2, 3])
def test_column_2d_small(ell):
    p = W.column_2d_small()
    nel, k, L = p["nel"], 6, 3
    print(f"case column_2d_small ell={ell}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, ell, k)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], ell, k, L)
    assert np.all(np.abs(g["lam"] / ref["buck"].lam - 1) < 1e-6)
    _check(g, ref, p["fixed"], p["F"], k)


def test_box_3d_small():
    nel = (32, 8, 8)
    p = W.box_3d(nel=nel, seed=5, sigma=2.0)
    k, L, ell = 4, 3, 2
    print(f"case box_3d nel={nel}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, ell, k)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], ell, k, L)
    _check(g, ref, p["fixed"], p["F"], k)


def test_four_load_cases_3d():
    nel = (16, 8, 8)
    p = W.box_3d_four_cases(nel=nel)
    print(f"case four cases nel={nel}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], 3, 2, 3)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], 2, 3, 3)
    _check(g, ref, p["fixed"], p["F"], 3)


def test_mixed_precision_matches_fp64_oracle():
    p = W.column_2d_small()
    nel, k, L = p["nel"], 6, 3
    print("case mixed precision column_2d_small", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, 2, k, precision=1)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], 2, k, L)
    _check(g, ref, p["fixed"], p["F"], k)


def test_error_paths():
    import paper_1909_13585_amd as mlb
    nel = (16, 8)
    p = dict(x=W.random_small(2, nel, 3), fixed=W.clamp_mask(nel), F=W.axial_load(nel))
    c = mlb.Context(nel, mg_levels=2, eig_level=2)
    with pytest.raises(mlb.MlbError) as e:
        c.buckling(2)
    assert e.value.status == -2
    bad = np.zeros(W.n_dofs(nel), dtype=np.uint8)
    bad[2 * 1] = 1                      # odd node on the bottom edge, sources free
    with pytest.raises(mlb.MlbError) as e:
        c.set_bc(bad)
    assert e.value.status == -1
    c.set_bc(p["fixed"])
    xb = p["x"].copy()
    xb[3] = np.nan
    with pytest.raises(mlb.MlbError) as e:
        c.set_density(xb)
    assert e.value.status == -1
    c.set_density(p["x"])
    c.set_loads(p["F"])
    with pytest.raises(mlb.MlbError) as e:
        c.solve_static(tol=1e-14, max_it=1)
    assert e.value.status == -5
    c.set_loads(-p["F"])                # tension: no positive buckling factor
    c.solve_static(tol=1e-10, max_it=500)
    with pytest.raises(mlb.MlbError) as e:
        c.buckling(2)
    assert e.value.status in (-6, -5)
    c.close()
    with pytest.raises(mlb.MlbError):
        mlb.Context((15, 8), mg_levels=2, eig_level=1)


def test_24_modes_2d():
    """24 modes (the count Secs. 3 and 6 compute): the coarse eigensolver's
    block is 32 columns wide, so its Gram products take two passes.  Factors,
    modes and sensitivities against the oracle."""
    p = W.column_2d_small()
    nel, k, L, ell = p["nel"], 24, 3, 2
    print(f"case column_2d_small k={k} ell={ell}", flush=True)
    g = _run(nel, p["x"], p["F"], p["fixed"], L, ell, k)
    ref = _oracle(nel, p["x"], p["F"], p["fixed"], ell, k, L)
    _check(g, ref, p["fixed"], p["F"], k)
