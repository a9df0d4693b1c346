"""Pins of the oracle's three-field design chain (Sec. 2: density filter and
eq. projectionOperator, with the chain rule back to the design variables).

  * Filter: a constant field is unchanged (rows are normalised); with
    r_min <= 1 only the element itself has weight, so it is the identity;
    the weights are symmetric; away from the boundary the weight sum equals
    the closed lattice sum; its output lies between the neighbours' extremes.
  * Projection: x(0) = 0, x(1) = 1, x(eta) = tanh(beta eta) / den; for small
    beta it tends to the identity; it is monotone and its derivative matches
    central differences.
  * Chain rule: against central finite differences of f = c^T x(xhat)
    through the whole chain, on random fields and both dimensions.
"""
import numpy as np
import pytest

from oracle import design


@pytest.mark.parametrize("nel,rmin", [((9, 7), 2.5), ((6, 5, 4), 1.8)])
def test_filter_constant_and_bounds(nel, rmin):
    m = int(np.prod(nel))
    assert np.allclose(design.filter_density(nel, np.full(m, 0.37), rmin), 0.37, rtol=0, atol=1e-15)
    xh = np.random.default_rng(1).uniform(size=m)
    xt = design.filter_density(nel, xh, rmin)
    for e in range(m):
        vals = [xh[k] for k, _ in design.neighbours(nel, e, rmin)]
        assert min(vals) - 1e-15 <= xt[e] <= max(vals) + 1e-15


@pytest.mark.parametrize("nel", [(9, 7), (6, 5, 4)])
def test_filter_small_radius_is_identity(nel):
    xh = np.random.default_rng(2).uniform(size=int(np.prod(nel)))
    assert np.array_equal(design.filter_density(nel, xh, 1.0), xh)
    assert np.allclose(design.filter_density(nel, xh, 0.6), xh, rtol=2.3e-16, atol=0)   # (0.6 x) / 0.6


def test_weights_symmetric_and_interior_sum():
    nel, rmin = (15, 15), 3.2
    w = {}
    for e in range(225):
        for k, v in design.neighbours(nel, e, rmin):
            w[(e, k)] = v
    assert all(w[(k, e)] == v for (e, k), v in w.items())
    c = 7 + 15 * 7
    ref = sum(rmin - np.hypot(i, j) for i in range(-3, 4) for j in range(-3, 4) if np.hypot(i, j) < rmin)
    assert abs(sum(v for (e, _), v in w.items() if e == c) - ref) < 1e-12


@pytest.mark.parametrize("eta,beta", [(0.5, 6.0), (0.3, 2.0), (0.7, 16.0)])
def test_projection_closed_forms(eta, beta):
    den = np.tanh(beta * eta) + np.tanh(beta * (1 - eta))
    assert abs(design.project(0.0, eta, beta)) < 1e-15
    assert abs(design.project(1.0, eta, beta) - 1.0) < 1e-15
    assert abs(design.project(eta, eta, beta) - np.tanh(beta * eta) / den) < 1e-15
    t = np.linspace(0, 1, 101)
    assert np.all(np.diff(design.project(t, eta, beta)) > 0)
    h = 1e-6
    fd = (design.project(t + h, eta, beta) - design.project(t - h, eta, beta)) / (2 * h)
    assert np.abs(fd - design.project_derivative(t, eta, beta)).max() < 1e-7 * beta
    assert np.abs(design.project(t, 0.5, 1e-4) - t).max() < 1e-8


@pytest.mark.parametrize("nel,rmin", [((8, 6), 2.2), ((5, 4, 4), 1.7)])
def test_chain_rule_against_finite_differences(nel, rmin):
    m = int(np.prod(nel))
    rng = np.random.default_rng(3)
    xh = rng.uniform(0.2, 0.8, m)
    C = rng.standard_normal((m, 2))
    eta, beta = 0.45, 4.0

    def f(v):
        return C.T @ design.project(design.filter_density(nel, v, rmin), eta, beta)

    xt = design.filter_density(nel, xh, rmin)
    g = design.chain_rule(nel, xt, rmin, eta, beta, C)
    h = 1e-6
    for k in range(m):
        d = np.zeros(m)
        d[k] = h
        fd = (f(xh + d) - f(xh - d)) / (2 * h)
        assert np.abs(fd - g[k]).max() < 1e-7, k
    sub = design.chain_rule(nel, xt, rmin, eta, beta, C, elements=[3, 0, m - 1])
    assert np.array_equal(sub, g[[3, 0, m - 1]])
