"""Tile parameters and the autotuner: operator applies are bitwise independent
of the tiles, and the autotuner picks one of its candidates."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_tiles_do_not_change_applies_and_autotune_picks_a_candidate():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1909_13585_amd as mlb
    nel = (48, 24, 40)
    p = W.box_3d(nel=nel, seed=8, sigma=1.5)
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2, precision=mlb.MLB_MIXED)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    ctx.set_density_dev(torch.from_numpy(p["x"]).cuda())
    n1, _ = ctx.level_size(1)
    n2, _ = ctx.level_size(2)
    g = torch.Generator(device="cuda").manual_seed(3)
    x1 = torch.randn((5, n1), dtype=torch.float64, device="cuda", generator=g)
    x2 = torch.randn((7, n2), dtype=torch.float64, device="cuda", generator=g)
    outs = []
    for zc, cb in [(4, 2), (8, 6), (16, 3), (12, 8)]:
        ctx.set_tiles(zc, cb)
        y1 = torch.empty_like(x1)
        y2 = torch.empty_like(x2)
        ctx.apply_K_dev(1, x1, y1)
        ctx.apply_K_dev(2, x2, y2)
        torch.cuda.synchronize()
        outs.append((y1.cpu().numpy(), y2.cpu().numpy()))
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])
    info = ctx.autotune(12)
    assert info["wht_zchunk"] in (4, 6, 8, 12, 16)
    assert info["stencil_cols"] in (2, 3, 4, 6, 8)
    assert all(t > 0 for t in info["wht_ms"]) and all(t > 0 for t in info["stencil_ms"])
    U = torch.empty((1, n1), dtype=torch.float64, device="cuda")
    J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=2000)
    assert si["converged"] == 1
    print("autotune", info)
    ctx.close()
