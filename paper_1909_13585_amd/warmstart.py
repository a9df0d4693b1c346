"""Learned warm start of the buckling analysis (3-D U-Net on the eigen level).

The network maps the density field averaged onto the eigen-level grid (plus
three fixed coordinate channels) to q = 12 start vectors of the coarse
eigensolver and to a static displacement guess, all at the eigen-level nodes
(3 components each: 39 output channels).  It is trained on coarse modes and
displacements that the plain method computes.  The solvers still converge
to their tolerances, so the network only changes iteration counts.

Every tensor operation runs in the library's kernels (include/mlb_nn.h);
this module allocates the torch tensors that hold parameters and
activations and sequences the calls.  Weights are BF16 for the convolutions
(FP32 master copies for Adam), activations and accumulation FP32.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B

NMODES = 12
COUT = 3 * NMODES + 3
CIN = 4


def _layers(cin, cout, c):
    return [("e1a", cin, c, 3, True), ("e1b", c, c, 3, True),
            ("e2a", c, 2 * c, 3, True), ("e2b", 2 * c, 2 * c, 3, True),
            ("b1", 2 * c, 4 * c, 3, True), ("b2", 4 * c, 4 * c, 3, True),
            ("d2a", 6 * c, 2 * c, 3, True), ("d2b", 2 * c, 2 * c, 3, True),
            ("d1a", 3 * c, c, 3, True), ("d1b", c, c, 3, True),
            ("head", c, cout, 1, False)]


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _st():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class UNet3D:
    """3-level U-Net (c, 2c, 4c channels), 3x3x3 convolutions, mean pooling,
    nearest up-sampling with skip concatenation, 1x1x1 head, cell-to-node mean."""

    def __init__(self, cin=CIN, cout=COUT, c=16, seed=0):
        import torch
        self.lib = B.load()
        self.cin, self.cout, self.c = cin, cout, c
        self.layers = _layers(cin, cout, c)
        rng = np.random.default_rng(seed)
        self.w, self.wb, self.b = {}, {}, {}
        self.gw, self.gb, self.m, self.v = {}, {}, {}, {}
        for name, ci, co, k, relu in self.layers:
            std = np.sqrt((2.0 if relu else 1.0) / (ci * k ** 3))
            w = torch.from_numpy((rng.standard_normal((co, ci, k, k, k)) * std).astype(np.float32)).cuda()
            self.w[name] = w
            self.wb[name] = torch.empty(w.shape, dtype=torch.int16, device="cuda")
            self.b[name] = torch.zeros(co, dtype=torch.float32, device="cuda")
            self.gw[name] = torch.zeros_like(w)
            self.gb[name] = torch.zeros_like(self.b[name])
            for d in (self.m, self.v):
                d[name] = (torch.zeros_like(w), torch.zeros_like(self.b[name]))
        self.step_no = 0
        # forward 3x3x3 convolutions on the matrix cores (BF16 activations);
        # training keeps the FP32-activation kernels
        self.mfma = False
        self.refresh_bf16()

    # -- plumbing
    def _check(self, st, what):
        if st != B.MLB_OK:
            raise B.MlbError(st, what)

    def refresh_bf16(self):
        for name in self.w:
            self._check(self.lib.mlb_nn_to_bf16(self.w[name].numel(), _p(self.w[name]), _p(self.wb[name]), _st()),
                        "to_bf16")

    def _conv(self, name, x, relu):
        import torch
        _, ci, co, k, _ = next(L for L in self.layers if L[0] == name)
        N, _, D, H, W = x.shape
        y = torch.empty((N, co, D, H, W), dtype=torch.float32, device="cuda")
        if self.mfma and k == 3 and self._cache_off():
            self._check(self.lib.mlb_nn_conv3d_mfma(N, ci, co, D, H, W, _p(x), _p(self.wb[name]), _p(self.b[name]),
                                                    _p(y), 1 if relu else 0, _st()), "conv3d_mfma " + name)
            return y
        self._check(self.lib.mlb_nn_conv3d(N, ci, co, D, H, W, k, 0, _p(x), _p(self.wb[name]), _p(self.b[name]),
                                           _p(y), 1 if relu else 0, _st()), "conv3d " + name)
        return y

    def _cache_off(self):
        # the matrix-core path serves inference only (no backward cache)
        return not getattr(self, "_keeping", False)

    def _pool(self, x, scale=1.0):
        import torch
        N, Cc, D, H, W = x.shape
        y = torch.empty((N, Cc, D // 2, H // 2, W // 2), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_pool2(N * Cc, D, H, W, scale, _p(x), _p(y), _st()), "pool2")
        return y

    def _unpool(self, g, scale):
        import torch
        N, Cc, D, H, W = g.shape
        y = torch.empty((N, Cc, 2 * D, 2 * H, 2 * W), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_unpool2(N * Cc, 2 * D, 2 * H, 2 * W, scale, _p(g), _p(y), _st()), "unpool2")
        return y

    def _cat(self, a, b):
        import torch
        N, Ca, D, H, W = a.shape
        Cb = b.shape[1]
        y = torch.empty((N, Ca + Cb, D, H, W), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_concat(N, Ca, Cb, D * H * W, _p(a), _p(b), _p(y), _st()), "concat")
        return y

    def _split(self, y, Ca):
        import torch
        N, Ct, D, H, W = y.shape
        a = torch.empty((N, Ca, D, H, W), dtype=torch.float32, device="cuda")
        b = torch.empty((N, Ct - Ca, D, H, W), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_split(N, Ca, Ct - Ca, D * H * W, _p(y), _p(a), _p(b), _st()), "split")
        return a, b

    # -- network
    def forward(self, x, keep=False):
        """x: (N, cin, D, H, W) float32 on the GPU, D, H, W divisible by 4.
        Returns (N, cout, D+1, H+1, W+1) node values."""
        import torch
        A = {}

        def conv(name, inp, relu=True):
            out = self._conv(name, inp, relu)
            if keep:
                A[name] = (inp, out)
            return out

        x = x.contiguous()
        self._keeping = keep
        e1 = conv("e1b", conv("e1a", x))
        e2 = conv("e2b", conv("e2a", self._pool(e1)))
        bt = conv("b2", conv("b1", self._pool(e2)))
        d2 = conv("d2b", conv("d2a", self._cat(self._unpool(bt, 1.0), e2)))
        d1 = conv("d1b", conv("d1a", self._cat(self._unpool(d2, 1.0), e1)))
        h = conv("head", d1, relu=False)
        N, Co, D, H, W = h.shape
        out = torch.empty((N, Co, D + 1, H + 1, W + 1), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_cell2node(N * Co, D, H, W, _p(h), _p(out), _st()), "cell2node")
        self._cache = A if keep else None
        return out

    def _back(self, name, g, relu, need_dx=True):
        import torch
        _, ci, co, k, _ = next(L for L in self.layers if L[0] == name)
        inp, out = self._cache[name]
        if relu:
            self._check(self.lib.mlb_nn_relu_mask(g.numel(), _p(out), _p(g), _st()), "relu_mask")
        N, _, D, H, W = g.shape
        self._check(self.lib.mlb_nn_conv3d_wgrad(N, ci, co, D, H, W, k, _p(inp), _p(g), _p(self.gw[name]),
                                                 _p(self.gb[name]), _st()), "wgrad " + name)
        if not need_dx:
            return None
        dx = torch.empty((N, ci, D, H, W), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_conv3d(N, co, ci, D, H, W, k, 1, _p(g), _p(self.wb[name]), None, _p(dx), 0,
                                           _st()), "dgrad " + name)
        return dx

    def backward(self, gout):
        """Parameter gradients (self.gw, self.gb) for the gradient of the node output."""
        import torch
        c = self.c
        N, Co, Dn, Hn, Wn = gout.shape
        gh = torch.empty((N, Co, Dn - 1, Hn - 1, Wn - 1), dtype=torch.float32, device="cuda")
        self._check(self.lib.mlb_nn_node2cell_grad(N * Co, Dn - 1, Hn - 1, Wn - 1, _p(gout.contiguous()), _p(gh),
                                                   _st()), "node2cell")
        g = self._back("head", gh, False)
        g = self._back("d1a", self._back("d1b", g, True), True)
        g_u1, g_e1 = self._split(g, 2 * c)
        g = self._back("d2a", self._back("d2b", self._pool(g_u1, 8.0), True), True)
        g_u2, g_e2 = self._split(g, 4 * c)
        g = self._back("b1", self._back("b2", self._pool(g_u2, 8.0), True), True)
        gp = self._unpool(g, 0.125)
        self._check(self.lib.mlb_nn_axpy(g_e2.numel(), 1.0, _p(gp), _p(g_e2), _st()), "axpy")
        g = self._back("e2a", self._back("e2b", g_e2, True), True)
        gp = self._unpool(g, 0.125)
        self._check(self.lib.mlb_nn_axpy(g_e1.numel(), 1.0, _p(gp), _p(g_e1), _st()), "axpy")
        self._back("e1a", self._back("e1b", g_e1, True), True, need_dx=False)

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step_no += 1
        for name in self.w:
            mw, mb = self.m[name]
            vw, vb = self.v[name]
            self._check(self.lib.mlb_nn_adam(self.w[name].numel(), lr, b1, b2, eps, self.step_no, _p(self.w[name]),
                                             _p(self.wb[name]), _p(self.gw[name]), _p(mw), _p(vw), _st()), "adam")
            self._check(self.lib.mlb_nn_adam(self.b[name].numel(), lr, b1, b2, eps, self.step_no, _p(self.b[name]),
                                             None, _p(self.gb[name]), _p(mb), _p(vb), _st()), "adam")

    def mse(self, pred, target, weight=None, scale=1.0):
        """(loss on the device as a 1-element float64 tensor, gradient)."""
        import torch
        n = pred.numel()
        grad = torch.empty_like(pred)
        work = torch.empty(int(self.lib.mlb_nn_mse_work(n)), dtype=torch.float64, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        self._check(self.lib.mlb_nn_mse(n, _p(pred.contiguous()), _p(target.contiguous()), _p(weight), scale,
                                        _p(grad), _p(work), _p(loss), _st()), "mse")
        return loss, grad

    # -- persistence (BF16 weights as stored by the network, FP32 biases)
    def state(self):
        out = {}
        for name in self.w:
            out[name + ".w"] = self.w[name].cpu().numpy()
            out[name + ".b"] = self.b[name].cpu().numpy()
        return out

    def save(self, path, meta=None):
        d = self.state()
        if meta:
            for k_, v_ in meta.items():
                d["meta." + k_] = np.asarray(v_)
        np.savez(path, **d)

    def load_state(self, d):
        import torch
        for name in self.w:
            self.w[name].copy_(torch.from_numpy(np.asarray(d[name + ".w"], dtype=np.float32)))
            self.b[name].copy_(torch.from_numpy(np.asarray(d[name + ".b"], dtype=np.float32)))
        self.refresh_bf16()

    @classmethod
    def from_file(cls, path):
        d = np.load(path, allow_pickle=False)
        c = int(d["meta.c"]) if "meta.c" in d else 16
        net = cls(c=c)
        net.load_state(d)
        return net


def coarse_inputs(x_fine, nel, ell):
    """Network input for a fine density field: the density averaged over the
    2^(ell-1)-cubes of the eigen-level cells (pooling kernel), concatenated
    with normalised cell-centre coordinates (concat kernel), as a
    (1, 4, D, H, W) float32 GPU tensor (NCDHW, x fastest)."""
    import torch
    lib = B.load()
    nx, ny, nz = nel
    x = torch.from_numpy(np.asarray(x_fine, dtype=np.float32).reshape(1, 1, nz, ny, nx).copy()).cuda()
    for _ in range(ell - 1):
        _, _, D, H, W = x.shape
        y = torch.empty((1, 1, D // 2, H // 2, W // 2), dtype=torch.float32, device="cuda")
        st = lib.mlb_nn_pool2(1, D, H, W, 1.0, _p(x), _p(y), _st())
        if st != B.MLB_OK:
            raise B.MlbError(st, "pool2")
        x = y
    _, _, D, H, W = x.shape
    zz, yy, xx = np.meshgrid((np.arange(D) + 0.5) / D, (np.arange(H) + 0.5) / H, (np.arange(W) + 0.5) / W,
                             indexing="ij")
    coords = torch.from_numpy(np.stack([xx, yy, zz])[None].astype(np.float32).copy()).cuda()
    out = torch.empty((1, 4, D, H, W), dtype=torch.float32, device="cuda")
    st = lib.mlb_nn_concat(1, 1, 3, D * H * W, _p(x), _p(coords), _p(out), _st())
    if st != B.MLB_OK:
        raise B.MlbError(st, "concat")
    return out


def node_channels_to_blocks(out_nodes, n_modes=NMODES):
    """Host arrays from (N, 3q+3, Dn, Hn, Wn) node channels of sample 0:
    modes (n_l, q) column-major blocks and u (n_l,), in the library's
    interleaved DOF order (dof = 3 node + c, node x fastest)."""
    o = out_nodes[0].cpu().numpy().astype(np.float64)
    nodes = o.shape[1] * o.shape[2] * o.shape[3]
    o = o.reshape(3 * n_modes + 3, nodes)
    modes = o[: 3 * n_modes].reshape(n_modes, 3, nodes).transpose(2, 1, 0).reshape(3 * nodes, n_modes)
    u = o[3 * n_modes:].reshape(3, nodes).T.reshape(3 * nodes)
    return np.asfortranarray(modes), u.copy()


def blocks_to_node_channels(modes, u, dims):
    """Inverse of node_channels_to_blocks (host): modes (n_l, q), u (n_l,) ->
    (3q+3, Dn, Hn, Wn) float32 node channels."""
    n, q = modes.shape
    nodes = n // 3
    mc = modes.reshape(nodes, 3, q).transpose(2, 1, 0).reshape(3 * q, nodes)
    uc = u.reshape(nodes, 3).T
    return np.concatenate([mc, uc], axis=0).reshape(3 * q + 3, *dims).astype(np.float32)


def normalize_modes(Psi):
    """Training targets: each mode (column) sign-fixed so that its
    largest-magnitude component is positive, and scaled to max-abs 1."""
    P = np.array(Psi, dtype=np.float64, copy=True)
    for j in range(P.shape[1]):
        i = int(np.argmax(np.abs(P[:, j])))
        s = P[i, j]
        if s != 0:
            P[:, j] /= s if abs(s) > 0 else 1.0
    return P


def coarse_nodes_of_fine(u_fine, nel, ell):
    """Injection of a fine nodal field onto the eigen-level nodes (every
    2^(ell-1)-th node per axis), interleaved DOF order."""
    nx, ny, nz = nel
    f = 2 ** (ell - 1)
    u = np.asarray(u_fine).reshape(nz + 1, ny + 1, nx + 1, 3)
    return np.ascontiguousarray(u[::f, ::f, ::f, :]).reshape(-1)


def predict(net, x_fine, nel, ell):
    """Network prediction for a fine density: (modes (n_l, 12), u_l (n_l,)) on the host."""
    inp = coarse_inputs(x_fine, nel, ell)
    out = net.forward(inp)
    return node_channels_to_blocks(out)


def predict_dev(net, x_fine, nel, ell):
    """Network prediction as device blocks: (q + 1) x n_l FP64 (q start
    vectors, then the displacement), interleaved DOF order, converted from the
    node channels by the library's kernel (no host round trip)."""
    import torch
    inp = coarse_inputs(x_fine, nel, ell)
    out = net.forward(inp)
    nfields = out.shape[1] // 3
    nodes = out.shape[2] * out.shape[3] * out.shape[4]
    blocks = torch.empty((nfields, 3 * nodes), dtype=torch.float64, device="cuda")
    st = net.lib.mlb_nn_nodes_to_dofs(nfields, nodes, _p(out), _p(blocks), _st())
    if st != B.MLB_OK:
        raise B.MlbError(st, "nodes_to_dofs")
    return blocks


def set_learned_warm_start(ctx, net, x_fine, nel, ell):
    """Predicts the coarse start block and the static guess for this density
    and hands them to the context from device memory: the q start vectors as
    MLB_WARM_COARSE, the displacement prolonged level by level to the fine
    grid in the library's transfer kernel as MLB_WARM_STATIC."""
    import torch
    from . import MLB_WARM_COARSE, MLB_WARM_STATIC
    blocks = predict_dev(net, x_fine, nel, ell)
    q = blocks.shape[0] - 1
    ctx.set_warm_start_dev(MLB_WARM_COARSE, blocks[:q].T)
    cur = blocks[q]
    for j in range(ell - 1, 0, -1):
        nj, _ = ctx.level_size(j)
        nxt = torch.empty(nj, dtype=torch.float64, device="cuda")
        ctx.prolong_dev(j, cur, nxt)
        cur = nxt
    ctx.set_warm_start_dev(MLB_WARM_STATIC, cur)
    return blocks
