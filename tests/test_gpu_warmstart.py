"""What the trained warm-start network gains over the plain (cold) start.

On held-out densities of the 192x64x64 workload recipe (seeds never used in
training), each analysis is run twice: cold (random coarse start block, zero
static guess) and with the network's prediction.  Both must reach the same
tolerances and the same buckling factors (1e-6); the test reports and checks
the iteration counts of the coarse eigensolve and of the static solve.
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
    ctx = mlb.Context(nel, mg_levels=5, eig_level=3, precision=mlb.MLB_MIXED)
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
        cold_it.append(ec["coarse_iterations"])
        warm_it.append(ew["coarse_iterations"])
        cold_st.append(sc["iterations"])
        warm_st.append(sw["iterations"])
        print(f"seed {seed}: coarse LOBPCG {ec['coarse_iterations']} -> {ew['coarse_iterations']}, "
              f"static CG {sc['iterations']} -> {sw['iterations']}")
    ctx.close()
    # the learned start must not cost iterations overall
    assert sum(warm_it) + sum(warm_st) <= sum(cold_it) + sum(cold_st)
