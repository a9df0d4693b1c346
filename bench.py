"""Benchmark: full linearized buckling analysis on the 2.4M-DOF H8 box.

One step = one complete analysis with the densities already in HBM:
SIMP moduli + multigrid hierarchy (Galerkin levels, coarsest inverse),
static MG-PCG solve to 1e-8, element stresses, Galerkin K^l/G^l, 12 coarse
modes (LOBPCG to 1e-8), interpolation, 12-column fine block solve
K Phi = G Psi to 1e-8, Rayleigh-Ritz, compliance sensitivities, 12 adjoint
solves (block, 1e-8) and buckling sensitivities.  The default precision is
mixed (FP32 multigrid cycle inside FP64 Krylov solvers, the workload's
configuration); the plain FP64 path is timed in the same run and reported
beside it.  Prints ONE JSON line (rank 0, N = 1 only).

Also reported: MG-PCG throughput of the static solve (free DOFs x iterations
/ solve time) and the roofline of the fine-level H8 stiffness apply, timed
with HIP events on the stream the library launches on.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the fine FP64 1-column apply, per 3D variant (0
# register tiles, 1 LDS tiles, 2 register tiles without prefetch, 3 register
# tiles with per-plane transforms): rocprofv3 FETCH_SIZE x (copy factor,
# 1.99977 and 1.99963 in the two runs) + WRITE_SIZE x 1.0 (factors from a
# 256 MiB calibration copy), KiB per dispatch, from
# profiles/fine_apply_h8_192x64x64_hbm_counters.md; None where the counters
# were not taken for the current kernel.
FINE_KERNELS = {0: "k_apply_wht3", 1: "k_apply_wht3_lds", 2: "k_apply_wht3 (no prefetch)", 3: "k_apply_wht3r"}
TRAFFIC_BYTES = {0: (17363 * 1.99977 + 19153) * 1024, 1: None, 2: None, 3: (17031 * 1.99963 + 19169) * 1024}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="skip timing the plain FP64 path next to the mixed one")
    ap.add_argument("--tol-eig", type=float, default=1e-8)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile parameters")
    ap.add_argument("--learned", default=os.path.join(ROOT, "paper_1909_13585_amd", "data", "warmstart_unet.npz"),
                    help="trained warm-start network; the learned leg is timed when the file exists")
    ap.add_argument("--nel", type=str, default="192,64,64")
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--eig-level", type=int, default=3)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--instances-only", action="store_true",
                    help="run only the 32 independent 2D instances and print their JSON object")
    ap.add_argument("--no-instances", action="store_true",
                    help="skip the 32 independent 2D instances (batched vs one context at a time)")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-post", action="store_true",
                    help="skip the post-processing measures (strain energy density, variation, correlation, dilation) "
                         "and the design chain (filter, projection, chain rule)")
    ap.add_argument("--no-incompatible", action="store_true",
                    help="skip the analysis with the incompatible-mode element (Q6/H11)")
    ap.add_argument("--no-pinvit", action="store_true",
                    help="skip the legs with preconditioned inverse iteration steps on the fine modes and with "
                         "the intermediate-level refinement")
    ap.add_argument("--wht-variant", type=int, default=-1,
                    help="with --roofline-only: fine-apply variant to run (0 register tiles, 1 LDS tiles, "
                         "2 register tiles without prefetch, 3 register tiles with per-plane transforms)")
    ap.add_argument("--wht-zchunk", type=int, default=0,
                    help="with --roofline-only: pencil length of the fine apply (0 keeps the default)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the dominant-kernel timing and a copy of known size (for counter runs)")
    return ap.parse_args()


CPU_SAMPLE = (64, 12, 12)


def cpu_baseline(args):
    """The oracle (sparse direct + LAPACK/ARPACK) on a bounded sample of the
    same workload recipe: 64x12x12 H8 box, eigen level 2, 12 modes."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import workloads as W
    from oracle import fem, lba, sens
    nel = CPU_SAMPLE
    p = W.box_3d(nel=nel, seed=3, sigma=1.0)
    mat = fem.Material()
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    t0 = time.perf_counter()
    r = lba.analysis(nel, p["x"], p["F"], p["fixed"], mat, ell=2, q=args.modes)
    sens.compliance_sensitivity(nel, p["x"], r["U"], mat)
    sens.buckling_sensitivity(nel, p["x"], r["u"], r["buck"].lam, r["buck"].phi, p["fixed"], mat, r["solver"])
    t = time.perf_counter() - t0
    if ctx is not None:
        ctx.__exit__(None, None, None)
    n_sample = W.n_dofs(nel)
    return t, n_sample


def run_path(args, precision, p, x_dev, steps, warmup, label, net=None, element=0):
    """Times `steps` full analyses after `warmup` untimed ones.  With `net`,
    every timed analysis first predicts its warm starts from the density."""
    import torch
    import paper_1909_13585_amd as mlb
    nel = tuple(int(v) for v in args.nel.split(","))
    ctx = mlb.Context(nel, mg_levels=args.levels, eig_level=args.eig_level, precision=precision,
                      element=element)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    n, m = ctx.level_size(1)
    k = args.modes
    U = torch.empty((ctx.ncases, n), dtype=torch.float64, device="cuda")
    Phi = torch.empty((k, n), dtype=torch.float64, device="cuda")
    dJ = torch.empty((ctx.ncases, m), dtype=torch.float64, device="cuda")
    dlam = torch.empty((k, m), dtype=torch.float64, device="cuda")
    ctx.set_density_dev(x_dev)
    ctx.tune = ctx.autotune(k) if not args.no_autotune else None   # untimed, once per context
    print(f"# {label} tiles {ctx.tune}", file=sys.stderr, flush=True)

    def step():
        if net is not None:
            from paper_1909_13585_amd import warmstart as ws
            ws.set_learned_warm_start(ctx, net, p["x"], nel, args.eig_level)
        ctx.set_density_dev(x_dev)
        J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=2000)
        lam, ei = ctx.buckling_dev(k, Phi, tol_eig=args.tol_eig)
        ai = ctx.sensitivities_dev(dJ, dlam)
        return J, si, lam, ei, ai

    for w in range(warmup):
        out = step()
        print(f"# {label} warmup {w} static_it={out[1]['iterations']} coarse_it={out[3]['coarse_iterations']} "
              f"fine_it={out[3]['fine_iterations']} adj_it={out[4]['iterations']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    out = None
    t0 = time.perf_counter()
    for s_ in range(steps):
        ts = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        print(f"# {label} step {s_} {time.perf_counter() - ts:.3f}s static_it={out[1]['iterations']} "
              f"coarse_it={out[3]['coarse_iterations']} fine_it={out[3]['fine_iterations']} "
              f"adj_it={out[4]['iterations']} lam1={out[2][0]:.9g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(steps, 1)
    return ctx, sec, out


def batched_instances(reps=3):
    """The 32 independent Q4 instances (64x32 ... 512x128, mixed precision,
    1e-8): static solve + compliance gradient of all of them as one batch
    (one launch per solver step for all instances), against the same analyses
    run one context at a time.  Both start from densities on the device."""
    import numpy as np
    import torch
    import paper_1909_13585_amd as mlb
    from paper_1909_13585_amd import batch as mlb_batch
    import workloads as W
    insts = W.small_instances_2d()
    b = mlb_batch.Batch([q["nel"] for q in insts], precision=mlb.MLB_MIXED)
    fixed = torch.from_numpy(b.concat([q["fixed"] for q in insts], np.uint8)).cuda()
    F = torch.from_numpy(b.concat([q["F"][:, 0] for q in insts], np.float64)).cuda()
    x = torch.from_numpy(b.concat([q["x"] for q in insts], np.float64)).cuda()
    U = torch.empty(b.n, dtype=torch.float64, device="cuda")
    dJ = torch.empty(b.m, dtype=torch.float64, device="cuda")

    def batched(opts):
        b.set_opts(**opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.set_problem_dev(fixed, F, x)
        J, its, info = b.solve_dev(U, tol=1e-8, max_it=3000)
        b.compliance_sens_dev(dJ)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, J, its, info

    variants = {}
    for name, opts in (("queue+graph", dict(queue=1, graphs=1)), ("queue", dict(queue=1, graphs=0)),
                       ("per-item+graph", dict(queue=0, graphs=1)), ("per-item", dict(queue=0, graphs=0))):
        batched(opts)   # warm-up (captures the graph)
        ts = [batched(opts) for _ in range(reps)]
        t = min(ts, key=lambda r: r[0])
        variants[name] = {"s": t[0], "setup_s": t[3]["setup_s"], "solve_s": t[3]["solve_s"],
                          "batch_iterations": t[3]["batch_iterations"]}
        print(f"# instances {name}: {t[0]:.4f} s (setup {t[3]['setup_s']:.4f}, solve {t[3]['solve_s']:.4f}, "
              f"{t[3]['batch_iterations']} batched iterations)", file=sys.stderr, flush=True)
    _, J, its, info = batched(dict(queue=1, graphs=1))
    levels = [int(v) for v in b.levels]
    b.close()
    ctxs = []
    for q, L in zip(insts, levels):
        c = mlb.Context(q["nel"], mg_levels=L, eig_level=1, precision=mlb.MLB_MIXED)
        c.set_bc(q["fixed"])
        c.set_loads(q["F"])
        ctxs.append((c, torch.from_numpy(q["x"]).cuda(), torch.empty((1, c.n), dtype=torch.float64, device="cuda"),
                     torch.empty((1, c.m), dtype=torch.float64, device="cuda")))

    def sequential():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Js = []
        for c, xd, Ud, dJd in ctxs:
            c.set_density_dev(xd)
            Jc, _ = c.solve_static_dev(Ud, tol=1e-8, max_it=3000)
            c.sensitivities_dev(dJd, None)
            Js.append(Jc[0])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, Js

    sequential()
    tseq, Js = min((sequential() for _ in range(reps)), key=lambda r: r[0])
    for c, *_ in ctxs:
        c.close()
    best_name = min(variants, key=lambda k: variants[k]["s"])
    best = variants[best_name]["s"]
    return {"instances": len(insts), "dofs": int(sum(int(np.prod([v + 1 for v in q["nel"]])) * 2 for q in insts)),
            "levels": levels, "precision": "mixed", "tol": 1e-8,
            "s_batched": best, "batched_variant": best_name, "variants": variants, "s_one_context_at_a_time": tseq, "speedup": tseq / best,
            "max_iterations": int(info["max_iterations"]), "total_iterations": int(info["total_iterations"]),
            "worst_true_rel_res": info["worst_true_rel_res"],
            "max_rel_J_diff_vs_contexts": float(np.max(np.abs(np.asarray(Js) / J - 1)))}


def pinvit_leg(ctx, k, n, tol_eig, lam0):
    """Buckling with 1 and 2 preconditioned inverse iteration steps on the fine
    modes after the multilevel Ritz step (same context, after the timed
    analyses); reports their cost and how far the Ritz values drop."""
    import numpy as np
    import torch
    Phi = torch.empty((k, n), dtype=torch.float64, device="cuda")
    out = {}
    for s in (1, 2):
        ctx.set_opts(pinvit_steps=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, ei = ctx.buckling_dev(k, Phi, tol_eig=tol_eig)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rel = (np.asarray(lam0) - np.asarray(lam)) / np.asarray(lam0)
        out[f"steps_{s}"] = {"buckling_s": t, "pinvit_s": ei["seconds_pinvit"],
                             "lambda": [float(v) for v in lam],
                             "rel_drop_min": float(rel.min()), "rel_drop_max": float(rel.max()),
                             "lambda1_before": ei["lambda1_before_pinvit"]}
    ctx.set_opts(pinvit_steps=-1)
    return out


def refine_leg(ctx, k, n, tol_eig, lam0):
    """Buckling with 1 and 2 Kaczmarz sweeps plus a Ritz step on every
    intermediate level (Alg. 2) on the same context, after the timed
    analyses; reports their cost and how far the fine Ritz values drop."""
    import numpy as np
    import torch
    Phi = torch.empty((k, n), dtype=torch.float64, device="cuda")
    out = {}
    for s in (1, 2):
        ctx.set_opts(refine_sweeps=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, ei = ctx.buckling_dev(k, Phi, tol_eig=tol_eig)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        rel = (np.asarray(lam0) - np.asarray(lam)) / np.asarray(lam0)
        out[f"sweeps_{s}"] = {"buckling_s": t, "refine_s": ei["seconds_refine"],
                              "levels": ei["refine_levels"],
                              "level_lambda1": [float(v) for v in ei["refine_lambda1"][:ei["refine_levels"]]],
                              "lambda": [float(v) for v in lam],
                              "rel_drop_min": float(rel.min()), "rel_drop_max": float(rel.max())}
    ctx.set_opts(refine_sweeps=-1)
    return out


def post_leg(ctx, k, n, m, x_dev, tol_eig, reps=5):
    """Post-processing measures of Sec. 5 on the fine modes of the same context
    (after the timed analyses): strain energy density, gradient and total
    variation on {x >= 0.5}, the k x k modal energy correlation, and the
    dilation (r_th = 2, threshold 1e-2 of the maximum) around the two modes of
    largest normalised variation.  Times are HIP events on the library's
    stream, per call, including the read-back of the host results."""
    import numpy as np
    import torch
    Phi = torch.empty((k, n), dtype=torch.float64, device="cuda")
    ctx.buckling_dev(k, Phi, tol_eig=tol_eig)
    sed = torch.empty((k, m), dtype=torch.float64, device="cuda")
    gradn = torch.empty_like(sed)
    Wk = torch.empty_like(Phi)
    xo = torch.empty_like(x_dev)
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    ms_tv, tv = timed(lambda: ctx.sed_tv_dev(Phi, 0.5, sed, gradn))
    ms_mac, C = timed(lambda: ctx.mac_dev(Phi, Phi, Wk))
    sel = np.argsort(tv / tv[0])[-2:]
    gsel = gradn[torch.from_numpy(sel).cuda()].contiguous()
    ms_dil, _ = timed(lambda: ctx.dilate_dev(gsel, 1e-2, 2.0, x_dev, xo))
    xs = x_dev.sum().item()
    alg_tv = k * (8 * n + 32 * m) + 8 * m   # Phi, sed write + read, x, gradn write; E_kappa
    return {"sed_tv_ms": ms_tv, "sed_tv_alg_bytes": alg_tv,
            "sed_tv_gbs": alg_tv / (ms_tv * 1e-3) / 1e9,
            "mac_ms": ms_mac, "dilate_ms": ms_dil,
            "tv_normalised": [float(v) for v in tv / tv[0]],
            "mac_offdiag_max": float(np.abs(C - np.diag(np.diag(C))).max()),
            "mac_diag_min": float(np.diag(C).min()),
            "dilated_modes": [int(v) for v in sel],
            "volume_increase_pct": float((xo.sum().item() - xs) / xs * 100.0)}


def design_leg(ctx, m, x_dev, k, reps=5, rmin=8.0, eta=0.5, beta=6.0):
    """Three-field design chain of Sec. 2 at the bench size: the density filter
    (r_min = 8, the paper's radius) with the Heaviside projection (eta 0.5,
    beta 6), and the chain rule of 1 + k sensitivity fields (compliance and k
    buckling factors) back to the design variables.  HIP events on the
    library's stream, per call."""
    import numpy as np
    import torch
    xt = torch.empty_like(x_dev)
    xp = torch.empty_like(x_dev)
    df = torch.randn((1 + k, m), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    work = torch.empty_like(df)
    out = torch.empty_like(df)
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_f = timed(lambda: ctx.filter_project_dev(x_dev, rmin, eta, beta, xt, xp))
    ms_c = timed(lambda: ctx.filter_chain_dev(xt, rmin, eta, beta, df, work, out))
    r = int(np.ceil(rmin))
    o = np.indices((2 * r + 1,) * 3).reshape(3, -1) - r
    nt = int((rmin - np.sqrt((o ** 2).sum(0)) > 0).sum())
    return {"rmin": rmin, "eta": eta, "beta": beta, "weights_per_element": nt,
            "filter_project_ms": ms_f, "chain_rule_columns": 1 + k, "chain_rule_ms": ms_c,
            "filter_gweights_per_s": m * nt / (ms_f * 1e-3) / 1e9}


def apply_roofline(ctx, n, m, reps, ncols=1):
    """Fine-level H8 apply (public entry, FP64), HIP events on the stream the
    library launches on (the caller's current stream)."""
    import torch
    xa = torch.randn((ncols, n) if ncols > 1 else (n,), dtype=torch.float64, device="cuda")
    ya = torch.empty_like(xa)
    for _ in range(5):
        ctx.apply_K_dev(1, xa, ya)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ctx.apply_K_dev(1, xa, ya)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nodes = n // 3
    alg = ncols * 16 * n + 8 * m + nodes   # x read + y write per column, E_kappa, node mask
    return ms, alg


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the analysis is built for one GPU; "
              "sharding it across GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W

    torch.cuda.set_device(0)
    if args.instances_only:
        print(json.dumps({"batched_instances": batched_instances()}), flush=True)
        return
    nel = tuple(int(v) for v in args.nel.split(","))
    p = W.box_3d(nel=nel, seed=3)
    x_dev = torch.from_numpy(p["x"]).cuda()

    if args.roofline_only:
        # counter runs: the fine apply, then a calibration copy of a buffer far
        # larger than the L2 caches, written by a fill and flushed before
        ctx = mlb.Context(nel, mg_levels=args.levels, eig_level=args.eig_level)
        ctx.set_bc(p["fixed"])
        ctx.set_loads(p["F"])
        ctx.set_density_dev(x_dev)
        if args.wht_variant >= 0 or args.wht_zchunk > 0:
            ctx.set_tiles(args.wht_zchunk, 0, args.wht_variant)
        n, m = ctx.level_size(1)
        xa = torch.randn(n, dtype=torch.float64, device="cuda")
        ya = torch.empty_like(xa)
        for _ in range(args.apply_reps):
            ctx.apply_K_dev(1, xa, ya)
        cal = 1 << 25   # 32 Mi doubles = 256 MiB
        src = torch.empty(cal, dtype=torch.float64, device="cuda").fill_(1.0)
        flush = torch.empty(cal, dtype=torch.float64, device="cuda").fill_(2.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"roofline_only": True, "n": n, "m": m, "copy_bytes": 8 * cal,
                          "flush_bytes": int(flush.numel() * 8)}), flush=True)
        ctx.close()
        return

    prec = mlb.MLB_MIXED if args.precision == "mixed" else mlb.MLB_FP64
    ctx, sec, out = run_path(args, prec, p, x_dev, args.steps, args.warmup, args.precision)
    J, si, lam, ei, ai = out
    n, m = ctx.level_size(1)
    k = args.modes
    free = int(n - p["fixed"].sum())
    gdofs = free * si["iterations"] / si["seconds"] / 1e9

    var64 = ctx.tune["wht64_variant"] if ctx.tune else 0
    apply_ms, alg_bytes = apply_roofline(ctx, n, m, args.apply_reps, 1)
    achieved = alg_bytes / (apply_ms * 1e-3) / 1e9
    pinv = None if args.no_pinvit else pinvit_leg(ctx, k, n, args.tol_eig, lam)
    refine = None if args.no_pinvit else refine_leg(ctx, k, n, args.tol_eig, lam)
    postp = None if args.no_post else post_leg(ctx, k, n, m, x_dev, args.tol_eig)
    designp = None if args.no_post else design_leg(ctx, m, x_dev, k)
    ctx.close()

    learned = None
    if os.path.exists(args.learned):
        from paper_1909_13585_amd.warmstart import UNet3D
        net = UNet3D.from_file(args.learned)
        ctxl, secl, outl = run_path(args, prec, p, x_dev, args.steps, 1, "learned", net=net)
        ctxl.close()
        learned = {"s_per_analysis": secl, "static_iterations": outl[1]["iterations"],
                   "coarse_iterations": outl[3]["coarse_iterations"],
                   "fine_block_iterations": outl[3]["fine_iterations"],
                   "adjoint_iterations": outl[4]["iterations"],
                   "max_rel_lambda_diff_vs_cold": float(np.max(np.abs(np.asarray(outl[2]) / np.asarray(lam) - 1))),
                   "weights": os.path.relpath(args.learned, ROOT)}

    incompatible = None
    if not args.no_incompatible:
        ctxi, seci, outi = run_path(args, prec, p, x_dev, 1, 1, "incompatible", element=mlb.MLB_ELEM_INCOMPATIBLE)
        ctxi.close()
        incompatible = {"s_per_analysis": seci, "static_iterations": outi[1]["iterations"],
                        "coarse_iterations": outi[3]["coarse_iterations"],
                        "fine_block_iterations": outi[3]["fine_iterations"],
                        "adjoint_iterations": outi[4]["iterations"],
                        "lambda": [float(v) for v in outi[2]],
                        "lambda_ratio_to_conforming": [float(a / b) for a, b in zip(outi[2], lam)]}

    fp64 = None
    if args.precision == "mixed" and not args.no_fp64_reference:
        ctx64, sec64, out64 = run_path(args, mlb.MLB_FP64, p, x_dev, max(1, min(args.steps, 2)), 1, "fp64")
        ctx64.close()
        fp64 = {"s_per_analysis": sec64, "static_iterations": out64[1]["iterations"],
                "coarse_iterations": out64[3]["coarse_iterations"],
                "fine_block_iterations": out64[3]["fine_iterations"],
                "adjoint_iterations": out64[4]["iterations"],
                "max_rel_lambda_diff_vs_mixed": float(np.max(np.abs(np.asarray(out64[2]) / np.asarray(lam) - 1)))}

    inst = None if args.no_instances else batched_instances()

    cpu = None
    if not args.no_cpu_baseline:
        t_cpu, n_sample = cpu_baseline(args)
        cpu = {"value": t_cpu * n / n_sample, "unit": "s/analysis", "cores": 1, "kind": "oracle",
               "sample": (f"oracle analysis (SuperLU static + adjoint solves, dense/ARPACK coarse eigen, Ritz, "
                          f"sensitivities) on the {CPU_SAMPLE[0]}x{CPU_SAMPLE[1]}x{CPU_SAMPLE[2]} H8 box of the "
                          f"same recipe ({n_sample} DOFs, eigen level 2, {k} modes, one thread): {t_cpu:.2f}s, "
                          f"scaled linearly in DOFs to {n} DOFs (a lower bound: direct solvers scale "
                          f"superlinearly)")}

    line = {
        "metric": "buckling-analysis wall time @2.4M DOF, FP64 vs mixed/learned; MG-PCG GDOF/s",
        "value": sec,
        "unit": "s/analysis",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"H8 box {nel[0]}x{nel[1]}x{nel[2]} ({n} DOFs), clamped x=0, unit axial load, "
                               f"Gaussian-filtered density vf 0.3 (seed 3), {args.levels}-level MG, eigen level "
                               f"{args.eig_level}, {k} modes, solves to 1e-8, coarse eigen to {args.tol_eig:g}",
                   "precision": args.precision},
        "tiles": {k: ctx.tune[k] for k in ("wht_zchunk", "wht_variant", "wht64_zchunk", "wht64_variant", "stencil_cols")} if ctx.tune else None,
        "mgpcg_gdof_per_s": gdofs,
        "static_iterations": si["iterations"],
        "coarse_iterations": ei["coarse_iterations"],
        "fine_block_iterations": ei["fine_iterations"],
        "adjoint_iterations": ai["iterations"],
        "lambda": [float(v) for v in lam],
        "phase_s": {"coarse": ei["seconds_coarse"], "fine": ei["seconds_fine"], "ritz": ei["seconds_ritz"],
                    "static": si["seconds"], "adjoint": ai["seconds"]},
        "fp64_reference": fp64,
        "learned_warm_start": learned,
        "pinvit_refinement": pinv,
        "intermediate_refinement": refine,
        "incompatible_element": incompatible,
        "post_processing": postp,
        "design_chain": designp,
        "batched_instances": inst,
        "roofline": {"bound": "hbm", "kernel": f"{FINE_KERNELS[var64]}<double> (fine H8 K apply, 1 column)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_BYTES.get(var64), "apply_ms": apply_ms,
                     "alg_bytes": alg_bytes, "launches_timed": args.apply_reps},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
