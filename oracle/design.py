"""Three-field design variables (oracle; test infrastructure only).

Sec. 2 maps the design variables xhat to physical densities in two steps:
  * a density filter of radius r_min (Bourdin's), xtilde = filter(xhat);
  * the relaxed Heaviside projection, eq. projectionOperator,
        x = (tanh(beta eta) + tanh(beta (xtilde - eta)))
            / (tanh(beta eta) + tanh(beta (1 - eta))),
and sensitivities with respect to x are taken back to xhat by the chain
rule (the paper applies it after eq. AdjointSystem).

Reading (the paper names the filter, not its weights): the standard linear
"hat" weights w_ek = max(0, r_min - |c_e - c_k|) between element centroids
on the grid of unit cells, over the elements inside the domain, each row
normalised by its sum W_e:
    xtilde_e = sum_k w_ek xhat_k / W_e.
The chain rule is then
    df/dxtilde_e = df/dx_e * dx/dxtilde_e,
    dx/dxtilde   = beta (1 - tanh^2(beta (xtilde - eta)))
                   / (tanh(beta eta) + tanh(beta (1 - eta))),
    df/dxhat_k   = sum_e w_ek df/dxtilde_e / W_e.
The element numbering is e = i + nx (j + ny k).
"""
from __future__ import annotations

import itertools

import numpy as np


def _coords(nel, e):
    c = []
    for n in nel:
        c.append(e % n)
        e //= n
    return tuple(c)


def _index(nel, c):
    e = 0
    for a in reversed(range(len(nel))):
        e = e * nel[a] + c[a]
    return e


def neighbours(nel, e, rmin):
    """(k, w_ek) for every element k with w_ek > 0, by brute force over the ball."""
    c = _coords(nel, e)
    r = int(np.ceil(rmin))
    out = []
    for o in itertools.product(range(-r, r + 1), repeat=len(nel)):
        k = tuple(a + b for a, b in zip(c, o))
        if not all(0 <= k[a] < nel[a] for a in range(len(nel))):
            continue
        w = rmin - np.sqrt(float(sum(t * t for t in o)))
        if w > 0.0:
            out.append((_index(nel, k), w))
    return out


def filter_density(nel, xhat, rmin, elements=None):
    """xtilde_e = sum_k w_ek xhat_k / W_e (for the listed elements only when given)."""
    m = int(np.prod(nel))
    elems = range(m) if elements is None else elements
    out = []
    for e in elems:
        nb = neighbours(nel, e, rmin)
        out.append(sum(w * xhat[k] for k, w in nb) / sum(w for _, w in nb))
    return np.array(out)


def project(xtilde, eta, beta):
    """Eq. projectionOperator."""
    xt = np.asarray(xtilde, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (xt - eta))) / den


def project_derivative(xtilde, eta, beta):
    """dx/dxtilde of eq. projectionOperator."""
    xt = np.asarray(xtilde, dtype=np.float64)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return beta * (1.0 - np.tanh(beta * (xt - eta)) ** 2) / den


def chain_rule(nel, xtilde, rmin, eta, beta, dfdx, elements=None):
    """df/dxhat for each column of dfdx (m, ncols), for the listed elements only when given."""
    m = int(np.prod(nel))
    dfdx = np.asarray(dfdx, dtype=np.float64)
    dfdx = dfdx[:, None] if dfdx.ndim == 1 else dfdx
    dxt = project_derivative(xtilde, eta, beta)
    elems = list(range(m)) if elements is None else list(elements)
    wsum = {}

    def W(e):
        if e not in wsum:
            wsum[e] = sum(w for _, w in neighbours(nel, e, rmin))
        return wsum[e]

    out = np.zeros((len(elems), dfdx.shape[1]))
    for t, k in enumerate(elems):
        for e, w in neighbours(nel, k, rmin):      # w_ek = w_ke
            out[t] += w * dfdx[e] * dxt[e] / W(e)
    return out
