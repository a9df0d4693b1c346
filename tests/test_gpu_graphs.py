"""Captured multigrid cycles (HIP graphs) give bit-identical results to eager
launches: every solve replays its cycle graph many times, with the solver's
own eager kernels and host synchronisations between the replays, and a new
density must invalidate the graphs (they hold the Jacobi weights)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _analysis(torch, mlb, nel, p, x, graphs, precision):
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2, precision=precision)
    ctx.set_opts(graphs=graphs)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    n, m = ctx.level_size(1)
    out = []
    for xi in x:   # two densities in a row on one context
        ctx.set_density_dev(torch.from_numpy(xi).cuda())
        U = torch.empty((1, n), dtype=torch.float64, device="cuda")
        J, si = ctx.solve_static_dev(U, tol=1e-10, max_it=2000)
        Phi = torch.empty((4, n), dtype=torch.float64, device="cuda")
        lam, ei = ctx.buckling_dev(4, Phi, tol_eig=1e-9)
        dl = torch.empty((4, m), dtype=torch.float64, device="cuda")
        ctx.sensitivities_dev(None, dl)
        torch.cuda.synchronize()
        out.append((U.cpu().numpy(), np.asarray(lam), Phi.cpu().numpy(), dl.cpu().numpy(),
                    si["iterations"], ei["coarse_iterations"]))
    ctx.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_bitwise_equals_eager(precision):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1909_13585_amd as mlb
    nel = (32, 16, 8)
    p = W.box_3d(nel=nel, seed=5, sigma=1.0)
    x2 = W.density_volume_fraction(nel, 6, 0.35, 1.0)
    eager = _analysis(torch, mlb, nel, p, [p["x"], x2], 2, precision)
    graph = _analysis(torch, mlb, nel, p, [p["x"], x2], 1, precision)
    for a, b in zip(eager, graph):
        for u, v in zip(a[:4], b[:4]):
            assert np.array_equal(u, v)
        assert a[4:] == b[4:]
