"""Pins of the FP64 network reference (oracle/nn.py) against definitions:
brute-force loops, adjoint identities, closed forms and finite differences."""
import numpy as np
import pytest

from oracle import nn


def _rng(s):
    return np.random.default_rng(s)


def test_bf16_round_known_values():
    one = 1.0
    assert nn.bf16_round(one) == 1.0
    assert nn.bf16_round(1.0 + 2.0 ** -8) == 1.0                      # tie -> even
    assert nn.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6       # tie -> even (up)
    assert nn.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert nn.bf16_round(-3.0) == -3.0
    x = _rng(0).standard_normal(1000)
    r = nn.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-300)


def test_conv3d_matches_brute_force_loops():
    rng = _rng(1)
    x = rng.standard_normal((2, 3, 4, 3, 5))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = nn.conv3d(x, w, b)
    N, Ci, D, H, W = x.shape
    ref = np.zeros((N, 2, D, H, W))
    for n in range(N):
        for o in range(2):
            for z in range(D):
                for yy in range(H):
                    for xx in range(W):
                        s = b[o]
                        for i in range(Ci):
                            for tz in range(3):
                                for ty in range(3):
                                    for tx in range(3):
                                        zz, y2, x2 = z + tz - 1, yy + ty - 1, xx + tx - 1
                                        if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                                            s += w[o, i, tz, ty, tx] * x[n, i, zz, y2, x2]
                        ref[n, o, z, yy, xx] = s
    assert np.abs(y - ref).max() < 1e-12
    assert np.abs(nn.conv3d(x, w, b, relu=True) - np.maximum(ref, 0)).max() < 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_conv3d_adjoints(k):
    rng = _rng(2 + k)
    x = rng.standard_normal((2, 3, 4, 6, 5))
    w = rng.standard_normal((4, 3, k, k, k))
    g = rng.standard_normal((2, 4, 4, 6, 5))
    lhs = np.sum(nn.conv3d(x, w) * g)
    assert abs(lhs - np.sum(x * nn.conv3d_input_grad(g, w))) < 1e-10 * abs(lhs) + 1e-12
    dw, db = nn.conv3d_weight_grad(x, g, k)
    assert abs(lhs - np.sum(w * dw)) < 1e-10 * abs(lhs) + 1e-12
    assert np.allclose(db, g.sum(axis=(0, 2, 3, 4)))


def test_pool_upsample_cell2node():
    rng = _rng(7)
    x = rng.standard_normal((1, 2, 4, 6, 8))
    g = rng.standard_normal((1, 2, 2, 3, 4))
    assert abs(np.sum(nn.pool2(x) * g) - np.sum(x * nn.pool2_adjoint(g))) < 1e-12
    assert abs(np.sum(nn.upsample2(g) * x) - np.sum(g * nn.upsample2_adjoint(x))) < 1e-12
    c = np.full((2, 3, 4, 5), 1.5)
    assert np.allclose(nn.cell2node(c), 1.5)
    c = rng.standard_normal((2, 3, 4, 5))
    gn = rng.standard_normal((2, 4, 5, 6))
    assert abs(np.sum(nn.cell2node(c) * gn) - np.sum(c * nn.cell2node_adjoint(gn))) < 1e-12
    # interior node = mean of 8 cells, corner node = its single cell
    assert abs(nn.cell2node(c)[0, 1, 1, 1] - c[0, 0:2, 0:2, 0:2].mean()) < 1e-14
    assert nn.cell2node(c)[1, 0, 0, 0] == c[1, 0, 0, 0]


def test_adam_first_step_closed_form():
    w0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = nn.adam(w0, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w0 - 0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_unet_backward_matches_finite_differences():
    rng = _rng(11)
    c = 2
    layers = nn.unet_layers(2, 3, c)
    params = {name: (rng.standard_normal((co, ci, k, k, k)) * (1.0 / np.sqrt(ci * k ** 3)),
                     rng.standard_normal(co) * 0.1) for name, ci, co, k, _ in layers}
    x = rng.standard_normal((1, 2, 4, 8, 4))
    R = rng.standard_normal((1, 3, 5, 9, 5))

    def loss(p):
        out, _ = nn.unet_forward(p, x, c)
        return float(np.sum(out * R))

    out, A = nn.unet_forward(params, x, c)
    assert out.shape == (1, 3, 5, 9, 5)
    G = nn.unet_backward(params, A, R, c)
    h = 1e-6
    for name in ["e1a", "e2b", "b1", "d2a", "d1b", "head"]:
        w, b = params[name]
        idx = tuple(rng.integers(0, s) for s in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fd = (loss({**params, name: (wp, b)}) - loss({**params, name: (wm, b)})) / (2 * h)
        assert abs(fd - G[name][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, G[name][0][idx])
        j = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        fd = (loss({**params, name: (w, bp)}) - loss({**params, name: (w, bm)})) / (2 * h)
        assert abs(fd - G[name][1][j]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, G[name][1][j])


def test_unet_forward_with_bf16_activations():
    """act_bf16 rounds exactly the inputs of the 3x3x3 convolutions: the first
    layer's output equals conv3d of the rounded input, the head (1x1x1)
    reads its FP64 input, and the whole pass stays within BF16 rounding of
    the plain one."""
    rng = np.random.default_rng(3)
    cin, cout, c = 2, 3, 4
    params = {}
    for name, ci, co, k, _ in nn.unet_layers(cin, cout, c):
        params[name] = (nn.bf16_round(rng.standard_normal((co, ci, k, k, k)) / np.sqrt(ci * k ** 3)),
                        rng.standard_normal(co) * 0.1)
    x = rng.standard_normal((1, cin, 4, 4, 8))
    y0, A0 = nn.unet_forward(params, x, c)
    y1, A1 = nn.unet_forward(params, x, c, act_bf16=True)
    w, b = params["e1a"]
    assert np.array_equal(A1["e1a"][1], nn.conv3d(nn.bf16_round(x), w, b, relu=True))
    wh, bh = params["head"]
    assert np.array_equal(A1["head"][1], nn.conv3d(A1["head"][0], wh, bh))
    rel = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    assert 0 < rel < 2e-2
