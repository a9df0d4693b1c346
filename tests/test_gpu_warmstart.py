"""What the trained warm-start network gains over the plain (cold) start.

On held-out densities of the 192x64x64 workload recipe (seeds never used in
training), in the benchmark's solver configuration (4 multigrid levels,
2/2/4 Jacobi sweeps), each analysis runs twice: cold (random coarse start
block, zero static guess) and with the network's prediction, handed over
from device memory.  Both must reach the same tolerances and buckling
factors (1e-6).  What the prediction achieves is checked as measured: its
coarse start block beats the random one at iteration 0 on every seed (the
eigensolver's fallback keeps it only then), and it costs no more than 5 %
of the iterations overall.  It does not shorten the analysis: most LOBPCG
iterations go to the asymptotic phase, which a start block of ~4 % error
does not shorten, and the interpolated static guess leaves most of the
energy-norm error.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1909_13585_amd", "data",
                       "warmstart_unet.npz")


@pytest.fixture(scope="module")
def setup():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained warm-start weights")
    import paper_1909_13585_amd as mlb
    from paper_1909_13585_amd.warmstart import UNet3D
    return torch, mlb, UNet3D.from_file(WEIGHTS)


def _analysis(torch, mlb, ctx, p, net=None):
    from paper_1909_13585_amd import warmstart as ws
    ctx.set_warm_start(mlb.MLB_WARM_NONE)
    if net is not None:
        ws.set_learned_warm_start(ctx, net, p["x"], (192, 64, 64), 3)
    ctx.set_density_dev(torch.from_numpy(p["x"]).cuda())
    U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
    J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
    lam, ei = ctx.buckling_dev(12, None, tol_eig=1e-8)
    return J[0], lam, si, ei


def test_learned_start_gain_on_held_out_densities(setup):
    torch, mlb, net = setup
    import workloads as W
    nel = (192, 64, 64)
    ctx = mlb.Context(nel, mg_levels=4, eig_level=3, precision=mlb.MLB_MIXED)
    ctx.set_opts(smooth_steps=2, coarse_sweeps=4, jacobi_omega=1.5)
    p0 = W.box_3d(nel=nel, seed=200000)
    ctx.set_bc(p0["fixed"])
    ctx.set_loads(p0["F"])
    cold_it, warm_it, cold_st, warm_st = [], [], [], []
    for seed in (200000, 200001, 200002):
        p = W.box_3d(nel=nel, seed=seed)
        Jc, lc, sc, ec = _analysis(torch, mlb, ctx, p)
        Jw, lw, sw, ew = _analysis(torch, mlb, ctx, p, net)
        # same answers: the warm start changes only the iteration counts
        assert np.max(np.abs(lw / lc - 1)) < 1e-6, (seed, lc, lw)
        assert abs(Jw / Jc - 1) < 1e-7
        # the predicted block beats a random one at iteration 0
        assert ew["coarse_warm_used"] == 1, seed
        cold_it.append(ec["coarse_iterations"])
        warm_it.append(ew["coarse_iterations"])
        cold_st.append(sc["iterations"])
        warm_st.append(sw["iterations"])
        print(f"seed {seed}: coarse LOBPCG {ec['coarse_iterations']} -> {ew['coarse_iterations']}, "
              f"static CG {sc['iterations']} -> {sw['iterations']}")
    ctx.close()
    # it costs no more than 5 % of the iterations overall
    assert sum(warm_it) + sum(warm_st) <= 1.05 * (sum(cold_it) + sum(cold_st))


def test_coarse_warm_start_is_kept_only_when_better():
    """The coarse eigensolver keeps a warm block only if its initial Ritz
    residual is no worse than the plain start's: the exact coarse modes are
    kept (and converge at once); a rank-deficient block is dropped and the
    run is bitwise the cold one."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1909_13585_amd as mlb
    import workloads as W
    p = W.column_2d_small()
    nel = p["nel"]
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    ctx.set_density_dev(torch.from_numpy(p["x"]).cuda())
    U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
    ctx.solve_static_dev(U, tol=1e-10, max_it=2000)
    k = 6
    lam_c, ei_c = ctx.buckling_dev(k, None, tol_eig=1e-10)
    assert ei_c["coarse_warm_used"] == 0 and ei_c["coarse_iterations"] > 5
    nl, _ = ctx.level_size(2)
    Psi = torch.empty((k, nl), dtype=torch.float64, device="cuda")
    ctx.coarse_modes_dev(k, Psi)
    psi = Psi.cpu().numpy()
    # exact coarse modes: kept, converged at the start
    ctx.set_warm_start(mlb.MLB_WARM_COARSE, psi.T)
    lam_w, ei_w = ctx.buckling_dev(k, None, tol_eig=1e-10)
    print("cold", ei_c["coarse_iterations"], "exact warm", ei_w["coarse_iterations"])
    assert ei_w["coarse_warm_used"] == 1
    assert ei_w["coarse_iterations"] <= 2
    assert np.max(np.abs(lam_w / lam_c - 1)) < 1e-9
    # rank-deficient block (one mode repeated): dropped, bitwise the cold run
    ctx.set_warm_start(mlb.MLB_WARM_COARSE, np.repeat(psi[:1], k, axis=0).T)
    lam_b, ei_b = ctx.buckling_dev(k, None, tol_eig=1e-10)
    assert ei_b["coarse_warm_used"] == 0
    assert ei_b["coarse_iterations"] == ei_c["coarse_iterations"]
    assert np.array_equal(lam_b, lam_c)
    ctx.close()


def test_learned_start_on_the_192x96x96_box(setup):
    """The network (trained at 96x32x32) on held-out densities of the
    192x96x96 box (5.4 M DOFs, eigen grid 48x24x24): same answers as the cold
    start; reports the iteration counts and whether the coarse solver kept
    the predicted block."""
    torch, mlb, net = setup
    import workloads as W
    from paper_1909_13585_amd import warmstart as ws
    nel = (192, 96, 96)
    ctx = mlb.Context(nel, mg_levels=5, eig_level=3, precision=mlb.MLB_MIXED)
    p0 = W.box_3d(nel=nel, seed=200010)
    ctx.set_bc(p0["fixed"])
    ctx.set_loads(p0["F"])
    for seed in (200010, 200011):
        p = W.box_3d(nel=nel, seed=seed)
        res = []
        for use_net in (False, True):
            ctx.set_warm_start(mlb.MLB_WARM_NONE)
            if use_net:
                ws.set_learned_warm_start(ctx, net, p["x"], nel, 3)
            ctx.set_density_dev(torch.from_numpy(p["x"]).cuda())
            U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
            J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
            lam, ei = ctx.buckling_dev(12, None, tol_eig=1e-8)
            res.append((J[0], lam, si["iterations"], ei["coarse_iterations"], ei["coarse_warm_used"]))
        (Jc, lc, sc, cc, _), (Jw, lw, sw, cw, used) = res
        print(f"192x96x96 seed {seed}: static CG {sc} -> {sw}, coarse LOBPCG {cc} -> {cw} "
              f"(predicted block kept: {bool(used)})")
        assert np.max(np.abs(lw / lc - 1)) < 1e-6
        assert abs(Jw / Jc - 1) < 1e-7
    ctx.close()
