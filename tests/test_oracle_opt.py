"""Pins of the optimisation oracle (oracle/opt.py): continuation schedules
against the numbers Secs. 3 and 6 state, the bound formulation against its
purpose and the coalescence measure of Sec. 3, and the MMA against closed-form
optima, first-order exactness of its approximations and the KKT conditions of
its subproblem (checked directly, not through the dual it is solved by)."""
import numpy as np
import pytest

from oracle import opt


# ------------------------------------------------------------ continuation
def test_sec6_schedule_numbers():
    """Sec. 6: start p = 3, beta = 1; p += 0.25 every 25 steps up to 6; then
    beta doubles every 50 steps up to 32, all within the 600 steps run."""
    assert opt.sec6_schedule(0) == (3.0, 1.0)
    assert opt.sec6_schedule(24) == (3.0, 1.0)
    assert opt.sec6_schedule(25) == (3.25, 1.0)
    ps = [opt.sec6_schedule(k)[0] for k in range(600)]
    assert min(k for k in range(600) if ps[k] == 6.0) == 300
    assert all(np.diff(ps) >= 0) and set(np.diff(ps)) <= {0.0, 0.25}
    bs = [opt.sec6_schedule(k)[1] for k in range(600)]
    assert bs[349] == 1.0 and bs[350] == 2.0 and bs[399] == 2.0 and bs[400] == 4.0
    assert min(k for k in range(600) if bs[k] == 32.0) == 550
    assert max(bs) == 32.0 and bs[-1] == 32.0
    # beta only moves once p has reached its maximum
    assert all(b == 1.0 for p, b in zip(ps, bs) if p < 6.0)


def test_sec3_schedule_numbers():
    """Sec. 3: p from 1 to 6 by 0.25 every 25 steps, beta fixed at 6; p is at
    6 over the last 150 of the 700 steps."""
    assert opt.sec3_schedule(0) == (1.0, 6.0)
    assert opt.sec3_schedule(25) == (1.25, 6.0)
    ps = [opt.sec3_schedule(k)[0] for k in range(700)]
    assert ps.count(1.0) == 25
    assert all(p == 6.0 for p in ps[550:])
    assert {opt.sec3_schedule(k)[1] for k in range(700)} == {6.0}
    assert len(set(ps)) == 21          # 1, 1.25, ..., 6


# ------------------------------------------------------- bound formulation
def test_bound_constraints_gap_and_coalescence_measure():
    """At the bounds lambda_i = lambda_bar alpha^-i every constraint is zero,
    the bounds rise with i (a gap of about 1 % between neighbours), and the
    coalescence measure of Sec. 3, with lambda_1 / lambda_i, vanishes there."""
    alpha, lam_bar, nb = 0.99, 1.3, 12
    i = np.arange(1, nb + 1)
    lam = lam_bar * alpha ** (-i)
    g, _ = opt.bound_constraints(lam, np.zeros((nb, 3)), lam_bar, alpha)
    assert np.max(np.abs(g)) < 1e-15
    assert np.all(np.diff(lam) > 0)
    assert np.allclose(lam[1:] / lam[:-1], 1.0 / alpha)
    delta = lam[0] / lam[1:] - alpha ** (i[1:] - 1)
    assert np.max(np.abs(delta)) < 1e-15
    # feasible above the bound, violated below; the fundamental factor's
    # bound lies above lambda_bar, so g_1 <= 0 implies lambda_1 >= lambda_bar
    g_hi, _ = opt.bound_constraints(lam * 1.01, np.zeros((nb, 3)), lam_bar, alpha)
    g_lo, _ = opt.bound_constraints(lam * 0.99, np.zeros((nb, 3)), lam_bar, alpha)
    assert np.all(g_hi < 0) and np.all(g_lo > 0)
    assert lam[0] > lam_bar


def test_bound_constraint_gradient_by_finite_differences():
    """Chain rule through lambda_i(x) for lambda_i(x) = sum_e c_ie x_e^2."""
    rng = np.random.default_rng(1)
    C = rng.uniform(0.5, 2.0, (4, 6))
    x = rng.uniform(0.2, 0.9, 6)
    lam_of = lambda x: np.sort(C @ (x * x))
    lam = lam_of(x)
    order = np.argsort(C @ (x * x))
    dlam = (2.0 * C * x[None, :])[order]
    g, dg = opt.bound_constraints(lam, dlam, 1.7, 0.99)
    h = 1e-6
    for e in range(6):
        xp, xm = x.copy(), x.copy()
        xp[e] += h
        xm[e] -= h
        fd = (opt.bound_constraints(lam_of(xp), dlam, 1.7)[0] - opt.bound_constraints(lam_of(xm), dlam, 1.7)[0]) / (2 * h)
        assert np.allclose(dg[:, e], fd, rtol=1e-7, atol=1e-9)


# --------------------------------------------------------------------- MMA
def test_mma_cantilever_closed_form():
    """min 0.0624 sum x s.t. sum a_j / x_j^3 <= 1 (Svanberg's five-segment
    cantilever).  Lagrange's conditions give x_j = a_j^(1/4) (sum_k a_k^(1/4))^(1/3);
    the optimum volume is 1.33996."""
    a = np.array([61.0, 37.0, 19.0, 7.0, 1.0])
    x_star = a ** 0.25 * (a ** 0.25).sum() ** (1.0 / 3.0)
    mma = opt.MMA(5, 1, xmin=1.0, xmax=10.0, move=0.5)
    x = np.full(5, 5.0)
    for _ in range(60):
        x, info = mma.update(x, 0.0624 * x.sum(), np.full(5, 0.0624), [(a / x ** 3).sum() - 1.0],
                             (-3.0 * a / x ** 4)[None, :])
    assert np.max(np.abs(x - x_star)) < 1e-9
    assert abs(0.0624 * x.sum() - 1.33996) < 1e-5


def test_mma_resource_allocation_closed_form():
    """min sum c_j / x_j s.t. sum x_j <= V, 0.01 <= x <= 1: x_j = V sqrt(c_j) / sum sqrt(c)."""
    rng = np.random.default_rng(0)
    n, V = 50, 10.0
    c = rng.uniform(0.5, 2.0, n)
    x_star = V * np.sqrt(c) / np.sqrt(c).sum()
    assert x_star.max() < 1.0 and x_star.min() > 0.01
    mma = opt.MMA(n, 1, xmin=0.01, xmax=1.0)
    x = np.full(n, 0.5)
    for _ in range(100):
        x, _ = mma.update(x, (c / x).sum(), -c / x ** 2, [x.sum() - V], np.ones((1, n)))
    assert np.max(np.abs(x - x_star)) < 1e-10


def _instance(seed, n=400, m=5):
    rng = np.random.default_rng(seed)
    mma = opt.MMA(n, m)
    x = rng.uniform(0.05, 0.95, n)
    df0 = -rng.uniform(0.0, 1.0, n) / n
    dfdx = rng.normal(size=(m, n)) / n
    fval = rng.normal(size=m) * 0.05
    return mma, x, 1.0, df0, fval, dfdx


def test_mma_approximations_are_first_order_exact():
    """f~_i(x^k) = f_i(x^k) and grad f~_i(x^k) = grad f_i(x^k) (central differences)."""
    mma, x, f0, df0, fval, dfdx = _instance(3, n=40, m=3)
    low, upp, _, _ = mma.asymptotes(x)
    grad = np.vstack([df0[None], dfdx])
    fv = np.concatenate(([f0], fval))
    p, q, r = opt.MMA.coefficients(x, low, upp, mma.xmax - mma.xmin, fv, grad)
    assert np.allclose(opt.MMA.approx(x, low, upp, p, q, r), fv, rtol=0, atol=1e-14)
    h = 1e-6
    for j in range(0, 40, 7):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (opt.MMA.approx(xp, low, upp, p, q, r) - opt.MMA.approx(xm, low, upp, p, q, r)) / (2 * h)
        assert np.allclose(fd, grad[:, j], rtol=1e-6, atol=1e-12)


def test_mma_asymptote_rule():
    """Asymptotes widen by 1.2 where x keeps its direction, narrow by 0.7 where
    it reverses, stay within [0.01, 10] dx of x; move limits nest inside."""
    mma = opt.MMA(3, 1, xmin=0.0, xmax=1.0)
    x0 = np.array([0.5, 0.5, 0.5])
    mma.update(x0, 0.0, np.zeros(3), [-1.0], np.zeros((1, 3)))
    x1 = np.array([0.6, 0.6, 0.5])
    mma.update(x1, 0.0, np.zeros(3), [-1.0], np.zeros((1, 3)))
    L1, U1 = mma.low.copy(), mma.upp.copy()
    assert np.allclose(L1, x1 - 0.5) and np.allclose(U1, x1 + 0.5)
    x2 = np.array([0.7, 0.5, 0.5])            # keeps, reverses, stays
    low, upp, alpha, beta = mma.asymptotes(x2)
    assert np.allclose(low, x2 - np.array([1.2, 0.7, 1.0]) * (x1 - L1))
    assert np.allclose(upp, x2 + np.array([1.2, 0.7, 1.0]) * (U1 - x1))
    assert np.all(low < alpha) and np.all(alpha <= x2) and np.all(x2 <= beta) and np.all(beta < upp)
    assert np.all(alpha >= 0.0) and np.all(beta <= 1.0)
    assert np.all(x2 - alpha <= 0.2 + 1e-15) and np.all(beta - x2 <= 0.2 + 1e-15)


def _kkt_residuals(mma, info, xn):
    """KKT conditions of the subproblem evaluated from their definitions."""
    low, upp, alpha, beta = info["low"], info["upp"], info["alpha"], info["beta"]
    p, q, r, y, lam = info["p"], info["q"], info["r"], info["y"], info["lam"]
    h = opt.MMA.approx(xn, low, upp, p, q, r)
    dh = p / (upp - xn) ** 2 - q / (xn - low) ** 2          # rows: d f~_i / d x_j
    grad_L = dh[0] + lam @ dh[1:]
    interior = (xn > alpha + 1e-12) & (xn < beta - 1e-12)
    at_lo = xn <= alpha + 1e-12
    at_hi = xn >= beta - 1e-12
    stat = max(np.abs(grad_L[interior]).max(initial=0.0),
               np.maximum(-grad_L[at_lo], 0).max(initial=0.0),       # at alpha: dL/dx >= 0
               np.maximum(grad_L[at_hi], 0).max(initial=0.0))        # at beta:  dL/dx <= 0
    feas = np.maximum(h[1:] - y, 0).max()
    comp = np.abs(lam * (h[1:] - y)).max()
    eta = mma.c + mma.d * y - lam                             # multiplier of y >= 0
    ycond = max(np.maximum(-eta, 0).max(), np.abs(eta * y).max())
    return stat, feas, comp, ycond, lam.min(), np.abs(dh).max()


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_mma_subproblem_meets_its_kkt_conditions(seed):
    mma, x, f0, df0, fval, dfdx = _instance(seed)
    xn, info = mma.update(x, f0, df0, fval, dfdx)
    stat, feas, comp, ycond, lam_min, gscale = _kkt_residuals(mma, info, xn)
    assert lam_min >= 0.0
    assert stat <= 1e-10 * gscale * (1 + np.abs(info["lam"]).max())
    lmax = 1.0 + np.abs(info["lam"]).max()
    assert feas <= 1e-12 and comp <= 1e-12 * lmax and ycond <= 1e-12 * lmax
    assert np.all(xn >= info["alpha"]) and np.all(xn <= info["beta"])


def test_mma_subproblem_brute_force_two_variables():
    """n = 2, m = 1: the subproblem optimum is no worse than any grid point of
    the box (y taken at its optimum max(0, f~_1) for each x)."""
    mma = opt.MMA(2, 1)
    x = np.array([0.4, 0.6])
    xn, info = mma.update(x, 1.0, np.array([-1.0, -0.5]), [0.02], np.array([[1.0, 1.5]]))
    low, upp, alpha, beta = info["low"], info["upp"], info["alpha"], info["beta"]
    p, q, r = info["p"], info["q"], info["r"]

    def obj(X):
        h = r[:, None] + (p[:, :, None] / (upp[None, :, None] - X[None]) + q[:, :, None]
                          / (X[None] - low[None, :, None])).sum(axis=1)
        y = np.maximum(h[1], 0.0)
        return h[0] + mma.c[0] * y + 0.5 * mma.d[0] * y * y

    g1 = np.linspace(alpha[0], beta[0], 801)
    g2 = np.linspace(alpha[1], beta[1], 801)
    G1, G2 = np.meshgrid(g1, g2)
    grid_min = obj(np.stack([G1.ravel(), G2.ravel()])).min()
    here = obj(xn[:, None])[0]
    assert here <= grid_min + 1e-12
    assert here >= grid_min - 1e-4       # and the grid's resolution reaches it


def test_p1_functions_volume_gradient():
    rng = np.random.default_rng(7)
    m, nb = 30, 4
    x = rng.uniform(0.1, 0.9, m)
    lam = np.sort(rng.uniform(1.0, 2.0, nb))
    dlam = rng.normal(size=(m, nb))
    f0, df0, fval, dfdx = opt.p1_functions(2.0, np.ones(m), lam, dlam, x, 4.0, 1.5, 0.3)
    assert f0 == 0.5 and np.allclose(df0, 0.25)
    assert np.isclose(fval[0], x.mean() / 0.3 - 1.0)
    e = 11
    xp = x.copy()
    xp[e] += 1e-7
    assert np.isclose((xp.mean() - x.mean()) / 0.3 / 1e-7, dfdx[0, e], rtol=1e-6)
    assert np.allclose(dfdx[1:], -(0.99 ** np.arange(1, nb + 1) / 1.5)[:, None] * dlam.T)


def test_p1_loop_reaches_feasibility_on_a_small_column():
    """Twelve P1 steps on a 48x16 Q4 column (eigen level 2, 6 modes, 4
    constrained, lambda_bar 1.3 times the start's fundamental factor): the
    buckling constraints start violated and end satisfied, the volume
    constraint ends active, and the compliance falls over the last steps."""
    import workloads as W
    from oracle import fem, lba
    nel = (48, 16)
    fixed = W.clamp_mask(nel)
    F = W.axial_load(nel)[:, None]
    xhat = np.full(48 * 16, 0.4)
    mat = fem.Material(p=3.0)
    an = lba.analysis(nel, xhat, F, fixed, mat, 2, 6)
    J0, lam_bar = float(an["J"][0]), 1.3 * an["buck"].lam[0]
    mma = opt.MMA(xhat.size, 1 + 4)
    hist = []
    for _ in range(12):
        xhat, info = opt.p1_step(nel, xhat, F, fixed, mat, 2, 6, 4, 2.5, 0.5, 6.0, J0, lam_bar, 0.4, mma)
        hist.append((info["f0"], info["fval"].copy()))
        assert np.all(xhat >= 0.0) and np.all(xhat <= 1.0)
    assert hist[0][1][1:].max() > 0.5
    assert hist[-1][1][1:].max() < 0.0
    assert -0.02 < hist[-1][1][0] <= 1e-3
    assert hist[-1][0] < hist[-4][0]


def test_p2_functions_values_and_gradients():
    rng = np.random.default_rng(8)
    m, nb = 20, 3
    x = rng.uniform(0.1, 0.9, m)
    lam = np.sort(rng.uniform(1.0, 2.0, nb))
    dlam = rng.normal(size=(m, nb))
    dJ = rng.normal(size=m)
    f0, df0, fval, dfdx = opt.p2_functions(3.0, dJ, lam, dlam, x, 2.0, 1.2)
    assert np.isclose(f0, x.mean()) and np.allclose(df0, 1.0 / m)
    assert np.isclose(fval[0], 0.5) and np.allclose(dfdx[0], dJ / 2.0)
    assert np.allclose(fval[1:], 1.0 - 0.99 ** np.arange(1, nb + 1) * lam / 1.2)
    assert np.allclose(dfdx[1:], -(0.99 ** np.arange(1, nb + 1) / 1.2)[:, None] * dlam.T)
