"""Three-field design variables (Sec. 2: density filter, eq.
projectionOperator, chain rule) through the C-ABI against the oracle.

Bars: the filtered field within nt eps of its value (a sum of nt positive
terms; both sides add in the same order, so it is normally bit-exact); the
projected field within that times the projection's largest slope plus
8 eps; the chain rule within 2 nt eps of the same sum taken over absolute
values plus the rounding of the projection's slope.  Full size (192x64x64,
the paper's r_min = 8): sampled elements against the oracle, a constant
field kept constant, and the chain rule's conservation
sum_k df/dxhat_k = sum_e df/dx_e dx/dxtilde_e.
"""
import time

import numpy as np
import pytest

import workloads as W
from oracle import design

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def _step(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _ctx(nel):
    import paper_1909_13585_amd as mlb
    return mlb.Context(nel, mg_levels=1, eig_level=1)


def _nt(dim, rmin):
    r = int(np.ceil(rmin))
    o = np.indices((2 * r + 1,) * dim).reshape(dim, -1) - r
    return int((rmin - np.sqrt((o ** 2).sum(0)) > 0).sum())


def _run(torch, c, xh, rmin, eta, beta, dfdx):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xt = torch.empty(c.m, dtype=torch.float64, device="cuda")
    x = torch.empty_like(xt)
    c.filter_project_dev(d(xh), rmin, eta, beta, xt, x)
    df = d(dfdx.T)
    work = torch.empty_like(df)
    out = torch.empty_like(df)
    c.filter_chain_dev(xt, rmin, eta, beta, df, work, out)
    torch.cuda.synchronize()
    return xt.cpu().numpy(), x.cpu().numpy(), out.cpu().numpy().T


# the last case has a filter ball wider than the grid
@pytest.mark.parametrize("nel,rmin,eta,beta", [((60, 20), 2.5, 0.5, 6.0), ((20, 12, 10), 2.2, 0.5, 6.0),
                                               ((52, 20), 0.7, 0.3, 16.0), ((20, 12, 10), 1.5, 0.6, 1.0),
                                               ((6, 5, 4), 8.3, 0.5, 6.0)])
def test_filter_projection_chain(torch_mod, nel, rmin, eta, beta):
    torch = torch_mod
    _step(f"design chain nel={nel} rmin={rmin} eta={eta} beta={beta}")
    m = int(np.prod(nel))
    rng = np.random.default_rng(31)
    xh = rng.uniform(size=m)
    dfdx = rng.standard_normal((m, 3))
    c = _ctx(nel)
    xt, x, g = _run(torch, c, xh, rmin, eta, beta, dfdx)
    c.close()
    nt = _nt(len(nel), rmin)
    xt_o = design.filter_density(nel, xh, rmin)
    err_t = np.abs(xt - xt_o)
    assert np.all(err_t <= nt * EPS * xt_o), err_t.max()
    den = np.tanh(beta * eta) + np.tanh(beta * (1 - eta))
    x_o = design.project(xt_o, eta, beta)
    assert np.abs(x - x_o).max() <= (beta / den) * nt * EPS + 8 * EPS
    g_o = design.chain_rule(nel, xt, rmin, eta, beta, dfdx)
    g_abs = design.chain_rule(nel, xt, rmin, eta, beta, np.abs(dfdx))
    bound = 2 * nt * EPS * g_abs + 64 * EPS * (beta / den) * np.abs(dfdx).max()
    assert np.all(np.abs(g - g_o) <= bound), np.max(np.abs(g - g_o) / bound)
    print(f"  max |dxtilde| {err_t.max():.1e}, |dx| {np.abs(x - x_o).max():.1e}, |dg| {np.abs(g - g_o).max():.1e}")


def test_argument_errors(torch_mod):
    torch = torch_mod
    import paper_1909_13585_amd as mlb
    c = _ctx((8, 4))
    a = torch.zeros(c.m, dtype=torch.float64, device="cuda")
    b, x = torch.empty_like(a), torch.empty_like(a)
    for r, eta, beta in ((0.0, 0.5, 1.0), (17.0, 0.5, 1.0), (2.0, 1.5, 1.0), (2.0, 0.5, 0.0),
                         (2.0, 0.5, float("inf"))):
        with pytest.raises(mlb.MlbError):
            c.filter_project_dev(a, r, eta, beta, b, x)
    with pytest.raises(mlb.MlbError):
        c.filter_project_dev(a, 2.0, 0.5, 1.0, b, b)
    with pytest.raises(mlb.MlbError):
        c.filter_chain_dev(b, 2.0, 0.5, 1.0, a[None], a[None], x[None])
    c.close()


def test_full_size_box(torch_mod):
    torch = torch_mod
    nel = (192, 64, 64)
    m = int(np.prod(nel))
    _step(f"design chain full size nel={nel}")
    c = _ctx(nel)
    x0 = W.box_3d(nel=nel)["x"]
    rng = np.random.default_rng(32)
    dfdx = rng.standard_normal((m, 2))
    eta, beta = 0.5, 6.0
    samples = np.concatenate([[0, m - 1, 191, 192 * 64, 192 * 64 * 32 + 96 + 192 * 31], rng.integers(0, m, 25)])
    for rmin in (8.0, 3.0):
        xt, x, g = _run(torch, c, x0, rmin, eta, beta, dfdx)
        nt = _nt(3, rmin)
        ref = design.filter_density(nel, x0, rmin, elements=samples)
        assert np.all(np.abs(xt[samples] - ref) <= nt * EPS * ref)
        den = np.tanh(beta * eta) + np.tanh(beta * (1 - eta))
        assert np.abs(x - design.project(xt, eta, beta)).max() <= 8 * EPS * (1 + beta / den)
        lhs = g.sum(0)
        rhs = (dfdx * design.project_derivative(xt, eta, beta)[:, None]).sum(0)
        scale = (np.abs(dfdx) * design.project_derivative(xt, eta, beta)[:, None]).sum(0)
        assert np.all(np.abs(lhs - rhs) <= 1e-11 * scale), (lhs, rhs)
        if rmin == 3.0:
            g_o = design.chain_rule(nel, xt, rmin, eta, beta, dfdx, elements=samples)
            g_abs = design.chain_rule(nel, xt, rmin, eta, beta, np.abs(dfdx), elements=samples)
            bound = 2 * nt * EPS * g_abs + 64 * EPS * (beta / den) * np.abs(dfdx).max()
            assert np.all(np.abs(g[samples] - g_o) <= bound)
    xt, _, _ = _run(torch, c, np.full(m, 0.3), 8.0, eta, beta, dfdx)
    assert np.abs(xt - 0.3).max() <= _nt(3, 8.0) * EPS * 0.3 * 2
    c.close()
