"""FP64 reference of the warm-start network (test infrastructure only).

Every operation is written from its definition with numpy: a 3-D
convolution (zero padding, stride 1, taps ordered z, y, x with x fastest),
its adjoints with respect to the input and to the filter, ReLU, 2x2x2 mean
pooling and nearest up-sampling, the cell-to-node mean, the weighted squared
error and one Adam step.  Weights are rounded to BF16 (nearest even) before
use, as the network stores them.  Nothing here is shared with the HIP path.
"""
import numpy as np


def bf16_round(a):
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (rounded << 16).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _pad(x, r):
    if r == 0:
        return x
    return np.pad(x, ((0, 0), (0, 0), (r, r), (r, r), (r, r)))


def conv3d(x, w, b=None, relu=False):
    """y[n,o] = b[o] + sum_{i,t} w[o,i,t] x[n,i,p+off(t)];  x: (N,Ci,D,H,W), w: (Co,Ci,k,k,k)."""
    N, Ci, D, H, W = x.shape
    Co, _, k, _, _ = w.shape
    r = k // 2
    xp = _pad(np.asarray(x, dtype=np.float64), r)
    y = np.zeros((N, Co, D, H, W))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                patch = xp[:, :, tz:tz + D, ty:ty + H, tx:tx + W]
                y += np.einsum("nidhw,oi->nodhw", patch, w[:, :, tz, ty, tx])
    if b is not None:
        y += np.asarray(b, dtype=np.float64)[None, :, None, None, None]
    return np.maximum(y, 0.0) if relu else y


def conv3d_input_grad(dy, w):
    """Adjoint of conv3d in x: scatter every output gradient back to the taps it read."""
    N, Co, D, H, W = dy.shape
    _, Ci, k, _, _ = w.shape
    r = k // 2
    dxp = np.zeros((N, Ci, D + 2 * r, H + 2 * r, W + 2 * r))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                dxp[:, :, tz:tz + D, ty:ty + H, tx:tx + W] += np.einsum("nodhw,oi->nidhw", dy, w[:, :, tz, ty, tx])
    return dxp[:, :, r:r + D, r:r + H, r:r + W]


def conv3d_weight_grad(x, dy, k):
    """dw[o,i,t] = sum_{n,p} dy[n,o,p] x[n,i,p+off(t)],  db[o] = sum dy[n,o,p]."""
    N, Ci, D, H, W = x.shape
    Co = dy.shape[1]
    r = k // 2
    xp = _pad(np.asarray(x, dtype=np.float64), r)
    dw = np.zeros((Co, Ci, k, k, k))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                dw[:, :, tz, ty, tx] = np.einsum("nodhw,nidhw->oi", dy, xp[:, :, tz:tz + D, ty:ty + H, tx:tx + W])
    return dw, dy.sum(axis=(0, 2, 3, 4))


def pool2(x):
    N, C, D, H, W = x.shape
    return x.reshape(N, C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(3, 5, 7))


def upsample2(x):
    return x.repeat(2, axis=2).repeat(2, axis=3).repeat(2, axis=4)


def pool2_adjoint(g):
    return upsample2(g) / 8.0


def upsample2_adjoint(g):
    N, C, D, H, W = g.shape
    return g.reshape(N, C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(3, 5, 7))


def cell2node(c):
    """Node value = mean of the cells sharing the node; cells (.., D, H, W) -> nodes (.., D+1, H+1, W+1)."""
    lead = c.shape[:-3]
    D, H, W = c.shape[-3:]
    s = np.zeros(lead + (D + 1, H + 1, W + 1))
    cnt = np.zeros((D + 1, H + 1, W + 1))
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                s[..., oz:oz + D, oy:oy + H, ox:ox + W] += c
                cnt[oz:oz + D, oy:oy + H, ox:ox + W] += 1
    return s / cnt


def cell2node_adjoint(g):
    D, H, W = (v - 1 for v in g.shape[-3:])
    cnt = np.zeros((D + 1, H + 1, W + 1))
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                cnt[oz:oz + D, oy:oy + H, ox:ox + W] += 1
    gs = g / cnt
    out = np.zeros(g.shape[:-3] + (D, H, W))
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                out += gs[..., oz:oz + D, oy:oy + H, ox:ox + W]
    return out


def mse(pred, target, weight=None, scale=1.0):
    wgt = 1.0 if weight is None else weight
    d = pred - target
    return float(np.sum(wgt * d * d)), 2.0 * wgt * d * scale


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return w, m, v


# ---------------------------------------------------------------------------
# the 3-level U-Net (channels c, 2c, 4c; two 3x3x3 convolutions per level,
# mean pooling down, nearest up-sampling and concatenation up, a 1x1x1 head
# and the cell-to-node mean)

def unet_layers(cin, cout, c=16):
    """(name, ci, co, k, relu) of every convolution, in forward order."""
    return [("e1a", cin, c, 3, True), ("e1b", c, c, 3, True),
            ("e2a", c, 2 * c, 3, True), ("e2b", 2 * c, 2 * c, 3, True),
            ("b1", 2 * c, 4 * c, 3, True), ("b2", 4 * c, 4 * c, 3, True),
            ("d2a", 6 * c, 2 * c, 3, True), ("d2b", 2 * c, 2 * c, 3, True),
            ("d1a", 3 * c, c, 3, True), ("d1b", c, c, 3, True),
            ("head", c, cout, 1, False)]


def unet_forward(params, x, c=16, act_bf16=False):
    """params: name -> (w (BF16-rounded float64), b).  Returns node outputs and
    the cache.  act_bf16: the inputs of the 3x3x3 convolutions are rounded to
    BF16 first (the matrix-core forward pass)."""
    A = {}

    def conv(name, inp, relu):
        w, b = params[name]
        src = bf16_round(inp) if act_bf16 and w.shape[-1] == 3 else inp
        out = conv3d(src, w, b, relu)
        A[name] = (inp, out)
        return out

    e1 = conv("e1b", conv("e1a", x, True), True)
    e2 = conv("e2b", conv("e2a", pool2(e1), True), True)
    bt = conv("b2", conv("b1", pool2(e2), True), True)
    d2 = conv("d2b", conv("d2a", np.concatenate([upsample2(bt), e2], axis=1), True), True)
    d1 = conv("d1b", conv("d1a", np.concatenate([upsample2(d2), e1], axis=1), True), True)
    h = conv("head", d1, False)
    return cell2node(h), A


def unet_backward(params, A, gout, c=16):
    """Gradients of every (w, b) for the node-output gradient gout."""
    G = {}

    def back(name, g, relu):
        w, _ = params[name]
        inp, out = A[name]
        if relu:
            g = g * (out > 0)
        dw, db = conv3d_weight_grad(inp, g, w.shape[-1])
        G[name] = (dw, db)
        return conv3d_input_grad(g, w)

    g = back("head", cell2node_adjoint(gout), False)
    g = back("d1a", back("d1b", g, True), True)          # (3c channels)
    g_up1, g_e1 = g[:, :2 * c], g[:, 2 * c:]
    g = back("d2a", back("d2b", upsample2_adjoint(g_up1), True), True)   # (6c channels)
    g_up2, g_e2 = g[:, :4 * c], g[:, 4 * c:]
    g = back("b1", back("b2", upsample2_adjoint(g_up2), True), True)
    g_e2 = g_e2 + pool2_adjoint(g)
    g = back("e2a", back("e2b", g_e2, True), True)
    g_e1 = g_e1 + pool2_adjoint(g)
    back("e1a", back("e1b", g_e1, True), True)
    return G
