"""Preconditioned inverse iteration on the fine modes (App. A, eq.
PInvIt-GeneralInteration) against the oracle.

The oracle computes the Jacobi weights of every level from its own exact
spectral radii and hands them to the library (mlb_set_omegas), so both run
the same V-cycle.  Both then take the same steps
phi_i <- phi_i - M^-1 (K + lam~_i G) phi_i, each followed by Rayleigh-Ritz,
from the multilevel Ritz block; the Ritz values must agree, and none may grow.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import fem, lba, mg

pytestmark = pytest.mark.gpu
MAT = fem.Material()


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _step(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


CASES = {
    "column_2d": dict(nel=(64, 16), levels=3, ell=2, q=4, seed=31),
    "box_3d": dict(nel=(16, 8, 8), levels=3, ell=2, q=4, seed=32),
}


def _oracle(c, steps, shift="own"):
    nel = c["nel"]
    x = W.density_uniform_noise(nel, c["seed"], sigma=1.0)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    r = lba.analysis(nel, x, F, fixed, MAT, ell=c["ell"], q=c["q"])
    free = np.flatnonzero(fixed == 0)
    Kff = r["K"][free][:, free].tocsr()
    Gff = r["G"][free][:, free].tocsr()
    As, Ps = mg.free_hierarchy(r["K"], fixed, nel, c["levels"])
    omegas = [(4.0 / 3.0) / (1.05 * mg.spectral_radius_dinv_a(A)) for A in As[:-1]]
    V = mg.VCycle(As, Ps, omegas, nu=2)
    out = {}
    for s in steps:
        lam, _, hist = mg.pinvit(Kff, Gff, r["buck"].phi[free], r["buck"].lam, V, s, shift=shift)
        out[s] = (lam, hist)
    return dict(x=x, fixed=fixed, F=F, omegas=omegas, ml=r["buck"].lam, pinvit=out)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("shift", ["own", "first"])
def test_pinvit_matches_oracle(torch_mod, case, precision, shift):
    """Both shifts: each vector's own Ritz value (the default) and the
    printed common lam~_1 (pinvit_shift = 2)."""
    torch = torch_mod
    import paper_1909_13585_amd as mlb
    c = CASES[case]
    steps = (1, 3)
    ref = _oracle(c, steps, shift)
    tol = 1e-9 if precision == mlb.MLB_FP64 else 1e-6
    for s in steps:
        _step(f"{case} precision {precision} shift {shift}: {s} step(s)")
        ctx = mlb.Context(c["nel"], mg_levels=c["levels"], eig_level=c["ell"], precision=precision)
        ctx.set_bc(ref["fixed"])
        ctx.set_loads(ref["F"])
        ctx.set_density_dev(torch.from_numpy(ref["x"]).cuda())
        ctx.set_omegas(ref["omegas"])
        assert np.allclose(ctx.get_omegas(c["levels"] - 1), ref["omegas"], rtol=0, atol=0)
        ctx.set_opts(pinvit_steps=s, pinvit_shift=1 if shift == "own" else 2)
        U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
        ctx.solve_static_dev(U, tol=1e-10, max_it=3000)
        lam, _, info = ctx.buckling(c["q"], tol_eig=1e-12, want_modes=False)
        ctx.close()
        lam_o, hist = ref["pinvit"][s]
        err = np.abs(lam / lam_o - 1).max()
        err0 = abs(info["lambda1_before_pinvit"] / hist[0][0] - 1)
        print(f"  lam {lam} oracle {lam_o} rel err {err:.2e}; lam1 before {info['lambda1_before_pinvit']:.12g} "
              f"({err0:.1e}); {info['seconds_pinvit']*1e3:.1f} ms")
        assert info["pinvit_steps"] == s
        assert err <= tol, (s, lam, lam_o)
        assert err0 <= tol
        assert lam[0] <= info["lambda1_before_pinvit"] * (1 + 1e-12)
        if shift == "own":   # the printed shift can raise the higher Ritz values
            assert np.all(lam <= ref["ml"] * (1 + 1e-9))


def test_pinvit_option_and_weights_are_checked(torch_mod):
    torch = torch_mod
    import paper_1909_13585_amd as mlb
    from paper_1909_13585_amd import MlbError
    c = CASES["column_2d"]
    ctx = mlb.Context(c["nel"], mg_levels=c["levels"], eig_level=c["ell"])
    with pytest.raises(MlbError):   # before the densities
        ctx.set_omegas([0.5, 0.5])
    nel = c["nel"]
    ctx.set_bc(W.clamp_mask(nel))
    ctx.set_loads(W.axial_load(nel)[:, None])
    ctx.set_density_dev(torch.from_numpy(W.density_uniform_noise(nel, 3, sigma=1.0)).cuda())
    est = ctx.get_omegas(2)
    assert np.all(est > 0)
    for bad in ([0.5, -1.0], [0.5, float("nan")], [0.5, 0.5, 0.5]):
        with pytest.raises(MlbError):
            ctx.set_omegas(bad)
    assert np.array_equal(ctx.get_omegas(2), est)
    U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
    ctx.solve_static_dev(U, tol=1e-10, max_it=3000)
    lam0, _, i0 = ctx.buckling(c["q"], want_modes=False)
    ctx.set_opts(pinvit_steps=2)
    lam2, _, i2 = ctx.buckling(c["q"], want_modes=False)
    ctx.set_opts(pinvit_steps=-1)
    lam0b, _, i0b = ctx.buckling(c["q"], want_modes=False)
    ctx.close()
    assert i0["pinvit_steps"] == 0 and i2["pinvit_steps"] == 2 and i0b["pinvit_steps"] == 0
    assert np.allclose(lam0b, lam0, rtol=1e-12)
    assert np.all(lam2 <= lam0) and i2["lambda1_before_pinvit"] == pytest.approx(lam0[0], rel=1e-12)
