"""Optimisation layer on the GPU against the oracle (oracle/opt.py): the MMA
update (closed-form optima, random instances over many tiles with a ragged
tail, consecutive updates that exercise the asymptote rule), the P1/P2
problem functions with the bound formulation, and whole P1 design steps
(filter, analysis, sensitivities, chain rule, MMA) on a small column."""
import numpy as np
import pytest

from oracle import opt as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("needs a GPU")
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_mma_cantilever_iterates_match_oracle(torch):
    from paper_1909_13585_amd.optimize import MMA
    a = np.array([61.0, 37.0, 19.0, 7.0, 1.0])
    x_star = a ** 0.25 * (a ** 0.25).sum() ** (1.0 / 3.0)
    orc = O.MMA(5, 1, xmin=1.0, xmax=10.0, move=0.5)
    gpu = MMA(5, 1, xmin=1.0, xmax=10.0, move=0.5)
    xo = np.full(5, 5.0)
    xg = _dev(torch, xo)
    for k in range(40):
        xh = xg.cpu().numpy()
        info = gpu.update_dev(xg, 0.0624 * xh.sum(), _dev(torch, np.full(5, 0.0624)), [(a / xh ** 3).sum() - 1.0],
                              _dev(torch, (-3.0 * a / xh ** 4)[None, :]))
        xo, _ = orc.update(xo, 0.0624 * xo.sum(), np.full(5, 0.0624), [(a / xo ** 3).sum() - 1.0],
                           (-3.0 * a / xo ** 4)[None, :])
        assert np.max(np.abs(xg.cpu().numpy() - xo)) < 1e-11 * (1 + k), k
    assert np.max(np.abs(xg.cpu().numpy() - x_star)) < 1e-9
    assert info["proj_grad"] < 1e-10
    gpu.close()


def _random_problem(seed, n, m):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 0.95, n)
    df0 = -rng.uniform(0.0, 1.0, n) / n
    dfdx = rng.normal(size=(m, n)) / n
    fval = rng.normal(size=m) * 0.05
    return x, df0, dfdx, fval


@pytest.mark.parametrize("n,m", [(100003, 13), (4099, 1), (2500, 30)])
def test_mma_random_updates_match_oracle(torch, n, m):
    """Three consecutive updates with fresh gradients each time (the third
    uses the asymptote rule on the history); x to 1e-10, multipliers to 1e-8."""
    from paper_1909_13585_amd.optimize import MMA
    x, _, _, _ = _random_problem(11, n, m)
    orc = O.MMA(n, m)
    gpu = MMA(n, m)
    xo = x.copy()
    xg = _dev(torch, x)
    for step in range(3):
        _, df0, dfdx, fval = _random_problem(100 + step, n, m)
        # gradients at the current point are inputs here; both sides get the same
        info = gpu.update_dev(xg, 1.0, _dev(torch, df0), fval, _dev(torch, dfdx))
        xo, oi = orc.update(xo, 1.0, df0, fval, dfdx)
        xgh = xg.cpu().numpy()
        err = np.max(np.abs(xgh - xo))
        print(f"n={n} m={m} step {step}: max|dx| {err:.2e}, dual its gpu {info['dual_iterations']} "
              f"oracle {oi['dual_iterations']}, {info['seconds'] * 1e3:.2f} ms")
        assert err < 1e-10, step
        assert np.allclose(info["lam"], oi["lam"], rtol=1e-8, atol=1e-10 * (1 + np.abs(oi["lam"]).max()))
        assert np.all(xgh >= oi["alpha"] - 1e-15) and np.all(xgh <= oi["beta"] + 1e-15)
        xg = _dev(torch, xo)   # continue both from the same point
    gpu.close()


def test_p1_p2_functions_match_oracle(torch):
    from paper_1909_13585_amd.optimize import p1_functions_dev, p2_functions_dev
    rng = np.random.default_rng(5)
    m, nb, q = 30011, 12, 14
    x = rng.uniform(0.0, 1.0, m)
    dJ = -rng.uniform(0.0, 1.0, m)
    lam = np.sort(rng.uniform(0.5, 1.5, q))
    dlam = rng.normal(size=(q, m))
    grad = torch.empty((2 + nb, m), dtype=torch.float64, device="cuda")
    f0, fval = p1_functions_dev(_dev(torch, x), 2.5, _dev(torch, dJ), lam[:nb], _dev(torch, dlam), 3.0, 0.8, 0.35,
                                grad)
    of0, odf0, ofval, odfdx = O.p1_functions(2.5, dJ, lam[:nb], dlam[:nb].T, x, 3.0, 0.8, 0.35)
    g = grad.cpu().numpy()
    assert abs(f0 - of0) < 1e-15 and np.allclose(fval, ofval, rtol=0, atol=1e-14)
    assert np.allclose(g[0], odf0, rtol=1e-15, atol=0)
    assert np.allclose(g[1:], odfdx, rtol=1e-15, atol=0)
    f0, fval = p2_functions_dev(_dev(torch, x), 2.5, _dev(torch, dJ), lam[:nb], _dev(torch, dlam), 4.0, 0.8, grad)
    of0, odf0, ofval, odfdx = O.p2_functions(2.5, dJ, lam[:nb], dlam[:nb].T, x, 4.0, 0.8)
    g = grad.cpu().numpy()
    assert abs(f0 - of0) < 1e-14 and np.allclose(fval, ofval, rtol=0, atol=1e-14)
    assert np.allclose(g[0], odf0, rtol=1e-15, atol=0)
    assert np.allclose(g[1:], odfdx, rtol=1e-15, atol=0)


def test_p1_design_steps_match_oracle(torch):
    """Three P1 steps on a 48x16 Q4 column (eigen level 2, 6 modes, 4
    constrained, filter radius 2.5, beta 6; p and beta moved on the third
    step) from the same start: the GPU's
    design variables, compliance and factors against the oracle's
    (direct solves), each side on its own trajectory."""
    import paper_1909_13585_amd as mlb
    import workloads as W
    from oracle import fem, lba
    from paper_1909_13585_amd.optimize import P1Step
    nel = (48, 16)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    m = 48 * 16
    x0 = np.full(m, 0.4)
    mat = fem.Material(p=3.0)
    an = lba.analysis(nel, x0, F, fixed, mat, 2, 6)
    J0, lam_bar = float(an["J"][0]), 1.3 * an["buck"].lam[0]
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2)
    ctx.set_bc(fixed)
    ctx.set_loads(F)
    stepper = P1Step(ctx, 6, 4, 2.5, 0.5, 6.0, J0, lam_bar, 0.4, tol=1e-11, tol_eig=1e-11)
    xg = _dev(torch, x0)
    xo = x0.copy()
    orc = O.MMA(m, 5)
    bars = [1e-8, 1e-8, 1e-8]
    # the third step moves p and beta (continuation) on both sides
    sched = [(3.0, 6.0), (3.0, 6.0), (3.25, 8.0)]
    for k in range(3):
        p, beta = sched[k]
        gi = stepper.step(xg, penal=p, beta=beta)
        xo, oi = O.p1_step(nel, xo, F, fixed, fem.Material(p=p), 2, 6, 4, 2.5, 0.5, beta, J0, lam_bar, 0.4, orc)
        err = np.max(np.abs(xg.cpu().numpy() - xo))
        print(f"step {k}: J {gi['J']:.10e} vs {oi['J']:.10e}, lam1 {gi['lam'][0]:.10f} vs {oi['lam'][0]:.10f}, "
              f"max|dxhat| {err:.2e}, dual its {gi['dual_iterations']}")
        assert abs(gi["J"] / oi["J"] - 1) < 1e-8
        assert np.max(np.abs(gi["lam"][:4] / oi["lam"][:4] - 1)) < 1e-7
        assert np.allclose(gi["fval"], oi["fval"], rtol=0, atol=1e-7)
        assert err < bars[k], k
    ctx.close()


def test_p2_design_steps_match_oracle(torch):
    """Two P2 steps (Sec. 6: minimum volume, compliance at most J_max) on a
    16x12x8 H8 box from a random start (eigen level 2, 6 modes, 4
    constrained), continuation of p on the second step, against the
    oracle's steps.  The section and the start are chosen so that the
    bounded factors are simple (gaps of 14 % or more): a repeated factor's
    individual sensitivities depend on the basis of its eigenspace, which
    two correct solvers need not share."""
    import paper_1909_13585_amd as mlb
    import workloads as W
    from oracle import fem, lba
    from paper_1909_13585_amd.optimize import P2Step
    nel = (16, 12, 8)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    m = 16 * 12 * 8
    x0 = W.random_small(3, nel, 21, 0.35, 0.65)
    an = lba.analysis(nel, x0, F, fixed, fem.Material(p=3.0), 2, 6)
    J_max, lam_bar = 1.5 * float(an["J"][0]), 1.1 * an["buck"].lam[0]
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2)
    ctx.set_bc(fixed)
    ctx.set_loads(F)
    stepper = P2Step(ctx, 6, 4, 1.8, 0.5, 2.0, J_max, lam_bar, tol=1e-11, tol_eig=1e-11)
    xg = _dev(torch, x0)
    xo = x0.copy()
    orc = O.MMA(m, 5)
    for k, p in enumerate((3.0, 3.25)):
        gi = stepper.step(xg, penal=p)
        xo, oi = O.p2_step(nel, xo, F, fixed, fem.Material(p=p), 2, 6, 4, 1.8, 0.5, 2.0, J_max, lam_bar, orc)
        err = np.max(np.abs(xg.cpu().numpy() - xo))
        print(f"P2 step {k}: volume {gi['f0']:.8f} vs {oi['f0']:.8f}, fval {np.round(gi['fval'], 5)}, "
              f"max|dxhat| {err:.2e}")
        assert abs(gi["f0"] - oi["f0"]) < 1e-12
        assert abs(gi["J"] / oi["J"] - 1) < 1e-8
        assert np.allclose(gi["fval"], oi["fval"], rtol=0, atol=1e-7)
        assert err < 1e-8, k
    ctx.close()


def test_design_steps_recycling(torch):
    """Three P2 steps that recycle the previous analysis (its coarse modes
    start the coarse eigensolve, its displacement the static CG) against the
    same steps started cold, with a move limit of 0.02 (the small steps of a
    settling design): the designs agree to the solver tolerances, and from
    the second step on the recycled block is kept and the coarse eigensolve
    needs fewer iterations."""
    import paper_1909_13585_amd as mlb
    import workloads as W
    from oracle import fem, lba
    from paper_1909_13585_amd.optimize import P2Step
    nel = (16, 12, 8)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    x0 = W.random_small(3, nel, 21, 0.35, 0.65)
    an = lba.analysis(nel, x0, F, fixed, fem.Material(p=3.0), 2, 6)
    J_max, lam_bar = 1.5 * float(an["J"][0]), 1.1 * an["buck"].lam[0]
    runs = {}
    for rec in (False, True):
        ctx = mlb.Context(nel, mg_levels=3, eig_level=2)
        ctx.set_bc(fixed)
        ctx.set_loads(F)
        stepper = P2Step(ctx, 6, 4, 1.8, 0.5, 2.0, J_max, lam_bar, tol=1e-11, tol_eig=1e-11, recycle=rec,
                         move=0.02)
        xg = _dev(torch, x0)
        infos = [stepper.step(xg, penal=3.0) for _ in range(3)]
        runs[rec] = (xg.cpu().numpy(), infos)
        ctx.close()
    (xc, ic), (xr, ir) = runs[False], runs[True]
    for k in range(3):
        print(f"step {k}: coarse its cold {ic[k]['coarse_iterations']} recycled {ir[k]['coarse_iterations']} "
              f"(kept {ir[k]['coarse_warm_used']}), static its {ic[k]['static_iterations']} / "
              f"{ir[k]['static_iterations']}, f0 {ic[k]['f0']:.12f} / {ir[k]['f0']:.12f}")
    assert np.max(np.abs(xc - xr)) < 1e-8
    assert ir[0]["coarse_warm_used"] == 0 and ir[0]["coarse_iterations"] == ic[0]["coarse_iterations"]
    for k in (1, 2):
        assert ir[k]["coarse_warm_used"] == 1
        assert ir[k]["coarse_iterations"] < ic[k]["coarse_iterations"]
        assert abs(ir[k]["f0"] - ic[k]["f0"]) < 1e-12
        assert np.allclose(ir[k]["fval"], ic[k]["fval"], rtol=0, atol=1e-8)
