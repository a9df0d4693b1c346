"""Warm-start network kernels (include/mlb_nn.h) against the FP64 reference
(oracle/nn.py) on identical BF16 weights: every kernel, then a full U-Net
forward and backward.  FP32 accumulation: normwise relative error <= 1e-4."""
import ctypes as C

import numpy as np
import pytest

from oracle import nn

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1909_13585_amd import _binding as B
    lib = B.load()
    return torch, lib


def _t(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).cuda()


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _bf16_bits(torch, w):
    r = nn.bf16_round(w).astype(np.float32)
    return torch.from_numpy((r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16).copy()).cuda(), r


@pytest.mark.parametrize("shape", [(2, 3, 5, 6, 7, 3), (1, 16, 8, 4, 12, 3), (2, 5, 3, 9, 4, 1), (1, 96, 4, 4, 4, 3)])
@pytest.mark.parametrize("co", [1, 11, 16])
def test_conv3d_forward_data_weight_grads(env, shape, co):
    torch, lib = env
    N, ci, D, H, W, k = shape
    rng = np.random.default_rng(ci * 7 + co)
    x = rng.standard_normal((N, ci, D, H, W)).astype(np.float32)
    w = rng.standard_normal((co, ci, k, k, k)) / np.sqrt(ci * k ** 3)
    b = rng.standard_normal(co).astype(np.float32)
    g = rng.standard_normal((N, co, D, H, W)).astype(np.float32)
    wbits, wr = _bf16_bits(torch, w)
    xd, bd, gd = _t(torch, x), _t(torch, b), _t(torch, g)
    y = torch.empty((N, co, D, H, W), dtype=torch.float32, device="cuda")
    for relu in (0, 1):
        assert lib.mlb_nn_conv3d(N, ci, co, D, H, W, k, 0, _p(xd), _p(wbits), _p(bd), _p(y), relu, None) == 0
        ref = nn.conv3d(x.astype(np.float64), wr.astype(np.float64), b.astype(np.float64), relu=bool(relu))
        assert _rel(y.cpu().numpy(), ref) < 1e-5
    dx = torch.empty((N, ci, D, H, W), dtype=torch.float32, device="cuda")
    assert lib.mlb_nn_conv3d(N, co, ci, D, H, W, k, 1, _p(gd), _p(wbits), None, _p(dx), 0, None) == 0
    assert _rel(dx.cpu().numpy(), nn.conv3d_input_grad(g.astype(np.float64), wr.astype(np.float64))) < 1e-5
    dw = torch.empty((co, ci, k, k, k), dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    assert lib.mlb_nn_conv3d_wgrad(N, ci, co, D, H, W, k, _p(xd), _p(gd), _p(dw), _p(db), None) == 0
    rdw, rdb = nn.conv3d_weight_grad(x.astype(np.float64), g.astype(np.float64), k)
    torch.cuda.synchronize()
    assert _rel(dw.cpu().numpy(), rdw) < 1e-5
    # bias gradient: a plain FP32 sum, bounded by the sum of the magnitudes
    bound = 1e-6 * np.abs(g.astype(np.float64)).sum(axis=(0, 2, 3, 4)) + 1e-30
    assert np.all(np.abs(db.cpu().numpy() - rdb) <= bound)


def test_elementwise_kernels(env):
    torch, lib = env
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 6, 8)).astype(np.float32)
    xd = _t(torch, x)
    y = torch.empty((2, 3, 2, 3, 4), dtype=torch.float32, device="cuda")
    assert lib.mlb_nn_pool2(6, 4, 6, 8, 1.0, _p(xd), _p(y), None) == 0
    assert _rel(y.cpu().numpy(), nn.pool2(x.astype(np.float64))) < 1e-6
    assert lib.mlb_nn_pool2(6, 4, 6, 8, 8.0, _p(xd), _p(y), None) == 0
    assert _rel(y.cpu().numpy(), nn.upsample2_adjoint(x.astype(np.float64))) < 1e-6
    up = torch.empty_like(xd)
    assert lib.mlb_nn_unpool2(6, 4, 6, 8, 1.0, _p(y), _p(up), None) == 0
    assert _rel(up.cpu().numpy(), nn.upsample2(y.cpu().numpy().astype(np.float64))) < 1e-6
    c = rng.standard_normal((5, 3, 4, 6)).astype(np.float32)
    cd = _t(torch, c)
    nd = torch.empty((5, 4, 5, 7), dtype=torch.float32, device="cuda")
    assert lib.mlb_nn_cell2node(5, 3, 4, 6, _p(cd), _p(nd), None) == 0
    assert _rel(nd.cpu().numpy(), nn.cell2node(c.astype(np.float64))) < 1e-6
    gc = torch.empty_like(cd)
    assert lib.mlb_nn_node2cell_grad(5, 3, 4, 6, _p(nd), _p(gc), None) == 0
    assert _rel(gc.cpu().numpy(), nn.cell2node_adjoint(nd.cpu().numpy().astype(np.float64))) < 1e-6
    a = rng.standard_normal((2, 3, 10)).astype(np.float32)
    b2 = rng.standard_normal((2, 2, 10)).astype(np.float32)
    cat = torch.empty((2, 5, 10), dtype=torch.float32, device="cuda")
    assert lib.mlb_nn_concat(2, 3, 2, 10, _p(_t(torch, a)), _p(_t(torch, b2)), _p(cat), None) == 0
    assert np.array_equal(cat.cpu().numpy(), np.concatenate([a, b2], axis=1))
    a2, b3 = torch.empty((2, 3, 10), device="cuda"), torch.empty((2, 2, 10), device="cuda")
    assert lib.mlb_nn_split(2, 3, 2, 10, _p(cat), _p(a2), _p(b3), None) == 0
    assert np.array_equal(a2.cpu().numpy(), a) and np.array_equal(b3.cpu().numpy(), b2)
    # relu mask, axpy, mse, adam
    yv = rng.standard_normal(1000).astype(np.float32)
    gv = rng.standard_normal(1000).astype(np.float32)
    gd = _t(torch, gv)
    assert lib.mlb_nn_relu_mask(1000, _p(_t(torch, yv)), _p(gd), None) == 0
    assert np.array_equal(gd.cpu().numpy(), gv * (yv > 0))
    t = rng.standard_normal(1000).astype(np.float32)
    wt = rng.random(1000).astype(np.float32)
    grad = torch.empty(1000, dtype=torch.float32, device="cuda")
    work = torch.empty(int(lib.mlb_nn_mse_work(1000)), dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    assert lib.mlb_nn_mse(1000, _p(_t(torch, yv)), _p(_t(torch, t)), _p(_t(torch, wt)), 0.5, _p(grad), _p(work),
                          _p(loss), None) == 0
    rl, rg = nn.mse(yv.astype(np.float64), t.astype(np.float64), wt.astype(np.float64), 0.5)
    assert abs(loss.item() - rl) < 1e-6 * rl
    assert _rel(grad.cpu().numpy(), rg) < 1e-6
    w0 = rng.standard_normal(1000).astype(np.float32)
    wd, md, vd = _t(torch, w0), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    wb = torch.empty(1000, dtype=torch.int16, device="cuda")
    rw, rm, rv = w0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in (1, 2, 3):
        gs = rng.standard_normal(1000).astype(np.float32)
        assert lib.mlb_nn_adam(1000, 1e-2, 0.9, 0.999, 1e-8, step, _p(wd), _p(wb), _p(_t(torch, gs)), _p(md), _p(vd),
                               None) == 0
        rw, rm, rv = nn.adam(rw, gs.astype(np.float64), rm, rv, step, 1e-2)
    assert _rel(wd.cpu().numpy(), rw) < 1e-5
    bits = wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(bits.view(np.float32).astype(np.float64), nn.bf16_round(wd.cpu().numpy()))


def test_unet_forward_backward_match_reference(env):
    torch, lib = env
    from paper_1909_13585_amd.warmstart import UNet3D
    c, cin, cout = 4, 4, 39
    net = UNet3D(cin=cin, cout=cout, c=c, seed=5)
    rng = np.random.default_rng(9)
    for name in net.w:   # non-zero biases so that they are exercised
        net.b[name].copy_(torch.from_numpy(rng.standard_normal(net.b[name].numel()).astype(np.float32) * 0.1))
    x = rng.standard_normal((2, cin, 8, 4, 12)).astype(np.float32)
    out = net.forward(_t(torch, x), keep=True)
    params = {}
    for name in net.w:
        params[name] = (nn.bf16_round(net.w[name].cpu().numpy()), net.b[name].cpu().numpy().astype(np.float64))
    ref, A = nn.unet_forward(params, x.astype(np.float64), c)
    assert _rel(out.cpu().numpy(), ref) < 1e-4
    R = rng.standard_normal(ref.shape).astype(np.float32)
    net.backward(_t(torch, R))
    G = nn.unet_backward(params, A, R.astype(np.float64), c)
    torch.cuda.synchronize()
    for name in net.w:
        assert _rel(net.gw[name].cpu().numpy(), G[name][0]) < 1e-4, name
        assert _rel(net.gb[name].cpu().numpy(), G[name][1]) < 1e-4, name


def test_nodes_to_dofs_matches_host_permutation():
    # device-resident prediction path: the kernel's channel -> DOF blocks
    # against the host permutation used for training targets (bit for bit)
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import ctypes as C
    from paper_1909_13585_amd import _binding as B
    from paper_1909_13585_amd import warmstart as ws
    lib = B.load()
    q, dims = 12, (5, 7, 9)
    nodes = dims[0] * dims[1] * dims[2]
    rng = np.random.default_rng(3)
    out = torch.from_numpy(rng.standard_normal((1, 3 * q + 3) + dims).astype(np.float32)).cuda()
    blocks = torch.empty((q + 1, 3 * nodes), dtype=torch.float64, device="cuda")
    st = lib.mlb_nn_nodes_to_dofs(q + 1, nodes, C.c_void_p(out.data_ptr()), C.c_void_p(blocks.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    modes, u = ws.node_channels_to_blocks(out, q)
    b = blocks.cpu().numpy()
    assert np.array_equal(b[:q].T, modes)
    assert np.array_equal(b[q], u)


@pytest.mark.parametrize("shape", [(2, 3, 5, 6, 7), (1, 16, 8, 4, 12), (1, 37, 4, 4, 4), (2, 1, 3, 9, 5)])
@pytest.mark.parametrize("co", [1, 11, 16, 40, 70])
def test_conv3d_mfma_matches_reference(env, shape, co):
    """The matrix-core forward convolution: the oracle's convolution of the
    BF16-rounded activations with the BF16 weights (products exact in FP32,
    sums in FP32 on the GPU): normwise 1e-5, maximum 1e-5 of the largest
    entry.  Shapes with voxel counts that are not multiples of 16, channel
    counts that are not multiples of 16, k ranges not a multiple of 32 and
    more than 64 output channels (two channel groups)."""
    torch, lib = env
    N, ci, D, H, W = shape
    rng = np.random.default_rng(ci * 13 + co)
    x = rng.standard_normal((N, ci, D, H, W)).astype(np.float32)
    w = rng.standard_normal((co, ci, 3, 3, 3)) / np.sqrt(ci * 27)
    b = rng.standard_normal(co).astype(np.float32)
    wbits, wr = _bf16_bits(torch, w)
    xd, bd = _t(torch, x), _t(torch, b)
    y = torch.empty((N, co, D, H, W), dtype=torch.float32, device="cuda")
    xr = nn.bf16_round(x.astype(np.float64))
    for relu in (0, 1):
        for bias in (bd, None):
            assert lib.mlb_nn_conv3d_mfma(N, ci, co, D, H, W, _p(xd), _p(wbits), _p(bias), _p(y), relu, None) == 0
            ref = nn.conv3d(xr, wr.astype(np.float64), b.astype(np.float64) if bias is not None else None,
                            relu=bool(relu))
            got = y.cpu().numpy()
            assert _rel(got, ref) < 1e-5
            assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def test_unet_forward_on_the_matrix_cores(env):
    """The U-Net forward pass with its 3x3x3 convolutions on the matrix cores
    equals the oracle's forward pass with every such convolution's input
    rounded to BF16 (1e-4 normwise), and stays within BF16 rounding of the
    FP32-activation pass (2e-2 normwise)."""
    torch, lib = env
    from paper_1909_13585_amd.warmstart import UNet3D
    net = UNet3D(cin=4, cout=3, c=8, seed=5)
    rng = np.random.default_rng(9)
    for name in net.w:
        net.b[name].copy_(torch.from_numpy(rng.standard_normal(net.b[name].numel()).astype(np.float32) * 0.1))
    x = rng.standard_normal((1, 4, 8, 8, 16)).astype(np.float32)
    xd = _t(torch, x)
    y_valu = net.forward(xd).cpu().numpy()
    net.mfma = True
    y_mfma = net.forward(xd).cpu().numpy()
    params = {name: (nn.bf16_round(net.w[name].cpu().numpy()), net.b[name].cpu().numpy().astype(np.float64))
              for name in net.w}
    ref, _ = nn.unet_forward(params, x.astype(np.float64), c=8, act_bf16=True)
    print(f"U-Net forward: MFMA vs BF16-activation oracle {_rel(y_mfma, ref):.2e}, "
          f"vs FP32-activation pass {_rel(y_mfma, y_valu):.2e}")
    assert _rel(y_mfma, ref) < 1e-4
    assert _rel(y_mfma, y_valu) < 2e-2
