"""Trains the warm-start U-Net on data the plain method generates.

    python -m paper_1909_13585_amd.train_warmstart --samples 2000 --epochs 40 --out weights.npz

Each sample is a seeded Gaussian-filtered density on a 96x32x32 H8 grid
(the 192x64x64 workload recipe at half resolution: volume fraction 0.3,
filter width 2 elements, solid end layers), analysed by the library
(mixed precision, 4 multigrid levels, eigen level 2, i.e. the same
48x16x16-element eigen-level grid as the 192x64x64 workload at level 3).

Targets are invariant to the rotations inside the 12-mode subspace: the
K-orthogonal projections Y = Psi (Psi^T K^l Q) of 12 fixed probe vectors Q
(the coarse modes of the recipe's mean density field) onto the span of the
sample's coarse modes Psi, each column scaled to max-abs 1.  Y spans the
same subspace as Psi and varies smoothly with the density, while single
modes swap order and sign where their factors cross.  Plus the static
displacement injected onto the eigen-level nodes (max-abs 1).  Inputs: the
density averaged onto the eigen-level cells plus coordinate channels.
Training: Adam, mean squared error, all in the library's kernels.
"""
import argparse
import sys
import time

import numpy as np


def generate(n_samples, seed0, nel=(96, 32, 32), ell=2, levels=4, log=print):
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W
    from paper_1909_13585_amd import warmstart as ws
    ctx = mlb.Context(nel, mg_levels=levels, eig_level=ell, precision=mlb.MLB_MIXED)
    ctx.set_opts(smooth_steps=2, coarse_sweeps=4, jacobi_omega=1.5)
    p0 = W.box_3d(nel=nel, seed=seed0, sigma=2.0)
    ctx.set_bc(p0["fixed"])
    ctx.set_loads(p0["F"])
    n_l, _ = ctx.level_size(ell)
    Psi = torch.empty((12, n_l), dtype=torch.float64, device="cuda")
    U = torch.empty((1, ctx.n), dtype=torch.float64, device="cuda")
    # probes: the coarse modes of the recipe's mean density (volume fraction
    # everywhere, the solid end layers kept)
    xm = np.where(p0["x"] >= 1.0, 1.0, 0.3)
    ctx.set_density_dev(torch.from_numpy(xm).cuda())
    ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
    ctx.buckling_dev(12, None, tol_eig=1e-8)
    Q = torch.empty((12, n_l), dtype=torch.float64, device="cuda")
    ctx.coarse_modes_dev(12, Q)
    KQ = torch.empty_like(Q)
    Dn, Hn, Wn = nel[2] // 2 ** (ell - 1) + 1, nel[1] // 2 ** (ell - 1) + 1, nel[0] // 2 ** (ell - 1) + 1
    X, Y = [], []
    t0 = time.perf_counter()
    for s in range(n_samples):
        p = W.box_3d(nel=nel, seed=seed0 + s, sigma=2.0)
        xd = torch.from_numpy(p["x"]).cuda()
        ctx.set_density_dev(xd)
        ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
        ctx.buckling_dev(12, None, tol_eig=1e-6)
        ctx.coarse_modes_dev(12, Psi)
        ctx.apply_K_dev(ell, Q, KQ)            # K^l of this density on the probes
        P = Psi.cpu().numpy()                  # (12, n_l), K^l-orthonormal rows
        Yp = (P @ KQ.cpu().numpy().T).T @ P    # rows: projections of the probes
        Yp /= np.maximum(np.abs(Yp).max(axis=1, keepdims=True), 1e-300)
        modes = np.asfortranarray(Yp.T)
        ul = ws.coarse_nodes_of_fine(U[0].cpu().numpy(), nel, ell)
        ul = ul / max(np.abs(ul).max(), 1e-300)
        X.append(ws.coarse_inputs(p["x"], nel, ell))
        Y.append(torch.from_numpy(ws.blocks_to_node_channels(modes, ul, (Dn, Hn, Wn))[None]).cuda())
        if (s + 1) % 50 == 0:
            log(f"# data {s + 1}/{n_samples} {time.perf_counter() - t0:.1f}s")
    ctx.close()
    return torch.cat(X), torch.cat(Y)


def train(X, Y, epochs, batch=8, lr=1e-3, c=16, seed=0, val_frac=0.1, log=print):
    import torch
    from paper_1909_13585_amd.warmstart import UNet3D
    n = X.shape[0]
    nval = max(1, int(round(val_frac * n)))
    idx = np.random.default_rng(seed).permutation(n)
    tr, va = idx[nval:], idx[:nval]
    net = UNet3D(c=c, seed=seed)
    steps_per_epoch = max(1, len(tr) // batch)
    total = epochs * steps_per_epoch
    hist = []
    rng = np.random.default_rng(seed + 1)
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(tr)
        acc = 0.0
        for b in range(steps_per_epoch):
            sel = torch.from_numpy(perm[b * batch:(b + 1) * batch]).cuda()
            xb = X.index_select(0, sel).contiguous()
            yb = Y.index_select(0, sel).contiguous()
            out = net.forward(xb, keep=True)
            loss, g = net.mse(out, yb, scale=1.0 / out.numel())
            net.backward(g)
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / total))   # cosine decay
            net.adam_step(lr_t)
            acc += loss.item() / out.numel()
            step += 1
        vl = 0.0
        for j in range(0, nval, batch):
            sel = torch.from_numpy(va[j:j + batch]).cuda()
            out = net.forward(X.index_select(0, sel).contiguous())
            loss, _ = net.mse(out, Y.index_select(0, sel).contiguous())
            vl += loss.item()
        vl /= nval * Y[0].numel()
        hist.append((acc / steps_per_epoch, vl))
        log(f"# epoch {ep + 1}/{epochs} train {acc / steps_per_epoch:.4e} val {vl:.4e} {time.perf_counter() - t0:.1f}s")
    return net, hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=600)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--channels", type=int, default=16)
    ap.add_argument("--seed0", type=int, default=100000)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    X, Y = generate(a.samples, a.seed0, log=log)
    net, hist = train(X, Y, a.epochs, a.batch, a.lr, a.channels, log=log)
    net.save(a.out, meta={"c": a.channels, "samples": a.samples, "epochs": a.epochs, "seed0": a.seed0,
                          "train_loss": hist[-1][0], "val_loss": hist[-1][1],
                          "grid": np.array([96, 32, 32]), "eigen_level": 2})
    log(f"# saved {a.out}")


if __name__ == "__main__":
    main()
