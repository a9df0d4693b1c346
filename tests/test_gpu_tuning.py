"""Tile parameters and the autotuner: for each fine-apply variant the operator
applies are bitwise independent of the tiles, every variant matches the
oracle's element loop, and the autotuner picks one of its candidates."""
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
    outs = {0: [], 1: [], 2: [], 3: []}
    for zc, cb, var in [(4, 2, 0), (8, 6, 0), (16, 3, 0), (12, 8, 0), (4, 2, 1), (6, 6, 1), (16, 3, 1), (12, 8, 1),
                        (4, 2, 2), (12, 6, 2), (4, 2, 3), (5, 6, 3), (10, 3, 3), (41, 8, 3)]:
        ctx.set_tiles(zc, cb, var)
        y1 = torch.empty_like(x1)
        y2 = torch.empty_like(x2)
        ctx.apply_K_dev(1, x1, y1)
        ctx.apply_K_dev(2, x2, y2)
        torch.cuda.synchronize()
        outs[var].append((y1.cpu().numpy(), y2.cpu().numpy()))
    # within a variant: bitwise the same for every tile choice
    for var in (0, 1, 2, 3):
        for a, b in outs[var][1:]:
            assert np.array_equal(a, outs[var][0][0]) and np.array_equal(b, outs[var][0][1]), var
    # the stencil levels do not depend on the fine variant; the register
    # tiles with and without prefetch sum in the same order
    assert np.array_equal(outs[0][0][1], outs[1][0][1])
    assert np.array_equal(outs[0][0][1], outs[3][0][1])
    assert np.array_equal(outs[0][0][0], outs[2][0][0])
    # both fine variants against the oracle's element loop (input not zero at
    # Dirichlet DOFs: masked columns, identity rows)
    from oracle import fem
    mat = fem.Material()
    xh = x1.cpu().numpy()
    fixed = p["fixed"].astype(bool)
    for var in (0, 1, 2, 3):
        yv = outs[var][0][0]
        for j in range(xh.shape[0]):
            xin = xh[j].copy()
            xin[fixed] = 0.0
            ref = fem.apply_K_matfree(nel, p["x"], xin, mat)
            ref[fixed] = xh[j][fixed]
            err = np.abs(yv[j] - ref).max() / np.abs(ref).max()
            assert err < 1e-13, (var, j, err)
    info = ctx.autotune(12)
    assert info["wht_zchunk"] in (4, 6, 8, 10, 12) and info["wht64_zchunk"] in (4, 6, 8, 10, 12)
    assert info["wht_variant"] in (0, 1, 2, 3) and info["wht64_variant"] in (0, 1, 2, 3)
    assert info["stencil_cols"] in (2, 3, 4, 6, 12)
    assert all(t > 0 for k in ("wht_ms", "wht_lds_ms", "wht_nopf_ms", "wht_v3_ms", "wht64_ms", "wht64_lds_ms",
                               "wht64_nopf_ms", "wht64_v3_ms") for t in info[k])
    assert all(t > 0 for t in info["stencil_ms"])
    # the chosen tile has the smallest score (a 12-column plus a one-column
    # sweep), and every score covers at least its 12-column sweep
    zs = (4, 6, 8, 10, 12)
    for pre in ("wht", "wht64"):
        tabs = {0: info[f"{pre}_ms"], 1: info[f"{pre}_lds_ms"], 2: info[f"{pre}_nopf_ms"], 3: info[f"{pre}_v3_ms"]}
        score = info[f"{pre}_score_ms"]
        v, z = info[f"{pre}_variant"], info[f"{pre}_zchunk"]
        assert score[5 * v + zs.index(z)] == min(score), (pre, info)
        for vv in range(4):
            for i in range(5):
                assert score[5 * vv + i] >= tabs[vv][i], (pre, vv, i)
    U = torch.empty((1, n1), dtype=torch.float64, device="cuda")
    J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=2000)
    assert si["converged"] == 1
    print("autotune", info)
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_static_solve_agrees_across_fine_variants(precision):
    """The solvers run the clean-input instances of the fine apply (with fused
    dot products, residual and Jacobi epilogues); the same static solve with
    variants 0 and 3 must reach the same displacements."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1909_13585_amd as mlb
    nel = (40, 24, 20)
    p = W.box_3d(nel=nel, seed=12, sigma=1.5)
    res = {}
    for var in (0, 3):
        ctx = mlb.Context(nel, mg_levels=3, eig_level=2, precision=precision)
        ctx.set_bc(p["fixed"])
        ctx.set_loads(p["F"])
        ctx.set_density_dev(torch.from_numpy(p["x"]).cuda())
        ctx.set_tiles(6, 0, var)
        U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
        J, si = ctx.solve_static_dev(U, tol=1e-10, max_it=2000)
        assert si["converged"] == 1 and si["true_rel_residual"] <= 1e-9, (var, si)
        res[var] = (J[0], U.cpu().numpy()[0], si["iterations"])
        ctx.close()
    print({v: (r[0], r[2]) for v, r in res.items()})
    assert abs(res[3][0] / res[0][0] - 1) < 1e-9
    u0, u3 = res[0][1], res[3][1]
    assert np.abs(u3 - u0).max() <= 1e-8 * np.abs(u0).max()
    assert abs(res[3][2] - res[0][2]) <= 2
