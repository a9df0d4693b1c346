"""Benchmark: full linearized buckling analysis on the 2.4M-DOF H8 box.

One step = one complete analysis with the densities already in HBM:
SIMP moduli + multigrid hierarchy (Galerkin levels, coarsest FP64 inverse on
the matrix cores), static MG-PCG solve to 1e-8, element stresses, Galerkin
K^l/G^l, 12 coarse modes (LOBPCG to 1e-8), interpolation, 12-column fine
block solve K Phi = G Psi to 1e-8, Rayleigh-Ritz, compliance sensitivities,
12 adjoint solves (block, 1e-8) and buckling sensitivities.  The default is
mixed precision (FP32 multigrid cycle inside FP64 Krylov solvers) on a
4-level hierarchy (2 Jacobi sweeps on levels 1-2, 4 on level 3, omega =
1.5 / (1.05 rho)), the fastest setting of the multigrid study; the 5-level
hierarchy and the plain FP64 path are timed in the same run and reported
beside it, with the achieved residuals of every solve.  Prints ONE JSON line
(rank 0, N = 1 only).

Also reported: MG-PCG throughput of the static solve, the 960x320 column in
FP64 (the oracle solves it directly), the 16-column block solve on the
96x48x48 box, the roofline of the dominant kernel (the 12-column FP32
Jacobi sweep of the fine level, timed with HIP events on the stream the
library launches on), and the oracle timed on the host on a bounded sample
of the same workload recipe, next to the GPU on that sample.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the dominant kernel (12-column FP32 Jacobi sweep of
# the fine level) by tuned (variant, z chunk): rocprofv3 FETCH_SIZE x ~2.0
# + WRITE_SIZE x 1.0 (factors from a 256 MiB calibration copy), KiB per
# dispatch, from profiles/jacobi_sweep_h8_192x64x64_12col_fp32_hbm_counters.md;
# reported only when the run tuned the same tile.
SWEEP_TRAFFIC_BYTES = {(3, 6): (167796.60 * 1.99964 + 120207.33) * 1024,
                       (0, 6): (169269.43 * 1.99976 + 118064.79) * 1024,
                       (0, 12): (160371.06 * 1.99964 + 118585.46) * 1024,
                       (3, 12): (162433.38 * 1.99978 + 125531.06) * 1024}
# wave-level VALU instructions per launch of the same sweep (rocprofv3
# SQ_INSTS_VALU, profiles/jacobi_sweep_h8_192x64x64_12col_fp32_sq_counters.md):
# at 4 cycles per FP32 wave instruction on 1,024 SIMDs at 2.4 GHz they set
# the kernel's VALU ceiling, reported beside the HBM roofline.
SWEEP_VALU_INSTS = {(3, 6): 53621856}
VALU_CYCLES_PER_INST, SIMDS, CLOCK_HZ = 4, 1024, 2.4e9


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
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--smooth", type=int, default=2, help="Jacobi sweeps per half cycle on levels 1-2")
    ap.add_argument("--coarse-sweeps", type=int, default=4, help="Jacobi sweeps per half cycle on levels >= 3")
    ap.add_argument("--omega", type=float, default=1.5, help="Jacobi weight times 1.05 rho(D^-1 A)")
    ap.add_argument("--eig-level", type=int, default=3)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--no-five-level", action="store_true", help="skip the 5-level hierarchy leg")
    ap.add_argument("--no-column", action="store_true", help="skip the 960x320 column leg")
    ap.add_argument("--no-block16", action="store_true", help="skip the 16-column block leg on 96x48x48")
    ap.add_argument("--no-opt", action="store_true", help="skip the design-step (P2, Sec. 6) leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle runs of the CPU sample (median reported)")
    ap.add_argument("--instances-only", action="store_true",
                    help="run only the 32 independent 2D instances and print their JSON object")
    ap.add_argument("--no-instances", action="store_true",
                    help="skip the 32 independent 2D instances (batched vs one context at a time)")
    ap.add_argument("--sweep-reps", type=int, default=50)
    ap.add_argument("--force-wht", type=str, default="",
                    help="with --roofline-only: variant,zchunk of the fine sweep instead of the autotuned ones")
    ap.add_argument("--no-post", action="store_true",
                    help="skip the post-processing measures (strain energy density, variation, correlation, dilation) "
                         "and the design chain (filter, projection, chain rule)")
    ap.add_argument("--no-incompatible", action="store_true",
                    help="skip the analysis with the incompatible-mode element (Q6/H11)")
    ap.add_argument("--no-pinvit", action="store_true",
                    help="skip the legs with preconditioned inverse iteration steps on the fine modes and with "
                         "the intermediate-level refinement")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the dominant-kernel sweeps and a copy of known size (for counter runs)")
    return ap.parse_args()


CPU_SAMPLE = (40, 16, 16)


def cpu_baseline(args):
    """The oracle (SuperLU, LAPACK/ARPACK, numpy) on a bounded sample of the
    same workload recipe, in a child process that imports only the oracle and
    the input generators: per-phase times, median of `cpu_reps` runs, peak
    RSS, BLAS threads, CPU model."""
    code = r"""
import json, resource, sys, time
sys.path.insert(0, %r)
import numpy as np
from threadpoolctl import threadpool_info
import workloads as W
from oracle import fem, lba, sens
nel = %r
p = W.box_3d(nel=nel, seed=3)
mat = fem.Material()
runs = []
for rep in range(%d):
    ph = {}
    t = time.perf_counter()
    K = fem.constrain(fem.assemble_K(nel, p["x"], mat), p["fixed"], 1.0); ph["assembly"] = time.perf_counter() - t
    t = time.perf_counter(); solver = lba.FreeSolver(K, p["fixed"]); ph["factorization"] = time.perf_counter() - t
    t = time.perf_counter(); U, J, _ = lba.static_solve(K, p["F"], p["fixed"], solver); ph["static"] = time.perf_counter() - t
    t = time.perf_counter()
    u = U[:, 0]
    s = fem.element_stresses(nel, p["x"], u, mat)
    G = fem.constrain(fem.assemble_G(nel, s), p["fixed"], 0.0); ph["stress_G"] = time.perf_counter() - t
    t = time.perf_counter()
    b = lba.multilevel_buckling(nel, p["x"], u, p["fixed"], mat, 2, 12, K=K, G=G, solver=solver)
    ph["multilevel_eigen"] = time.perf_counter() - t
    t = time.perf_counter()
    sens.compliance_sensitivity(nel, p["x"], U, mat)
    sens.buckling_sensitivity(nel, p["x"], u, b.lam, b.phi, p["fixed"], mat, solver)
    ph["sensitivities"] = time.perf_counter() - t
    ph["total"] = sum(ph.values())
    runs.append(ph)
tot = sorted(r["total"] for r in runs)
med = min(runs, key=lambda r: abs(r["total"] - tot[len(tot) // 2]))
blas = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas")
model = ""
try:
    for line in open("/proc/cpuinfo"):
        if line.startswith("model name"):
            model = line.split(":", 1)[1].strip(); break
except OSError:
    pass
print(json.dumps({"median": med, "totals": tot, "dofs": int(fem.n_dofs(nel)), "lambda1": float(b.lam[0]),
                  "rss_gb": resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6, "blas_threads": blas,
                  "cpu_model": model, "logical_cpus": len(__import__("os").sched_getaffinity(0))}))
""" % (ROOT, CPU_SAMPLE, args.cpu_reps)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=1200)
    if r.returncode != 0:
        raise RuntimeError("oracle sample failed: " + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def gpu_on_cpu_sample(args, reps=3):
    """The GPU analysis (same precision and settings) on the CPU sample box."""
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W
    nel = CPU_SAMPLE
    p = W.box_3d(nel=nel, seed=3)
    ctx = mlb.Context(nel, mg_levels=3, eig_level=2, precision=mlb.MLB_MIXED if args.precision == "mixed" else 0)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    n, m = ctx.level_size(1)
    xd = torch.from_numpy(p["x"]).cuda()
    U = torch.empty((1, n), dtype=torch.float64, device="cuda")
    dJ = torch.empty((1, m), dtype=torch.float64, device="cuda")
    dl = torch.empty((args.modes, m), dtype=torch.float64, device="cuda")
    ts = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_density_dev(xd)
        ctx.solve_static_dev(U, tol=1e-8, max_it=2000)
        lam, _ = ctx.buckling_dev(args.modes, None, tol_eig=args.tol_eig)
        ctx.sensitivities_dev(dJ, dl)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ctx.close()
    ts = sorted(ts[1:])
    return ts[len(ts) // 2], float(lam[0])


def set_solver_opts(ctx, args):
    ctx.set_opts(smooth_steps=args.smooth, coarse_sweeps=args.coarse_sweeps, jacobi_omega=args.omega)


def run_path(args, precision, p, x_dev, steps, warmup, label, net=None, element=0, levels=None, tuned=True):
    """Times `steps` full analyses after `warmup` untimed ones.  With `net`,
    every timed analysis first predicts its warm starts from the density.
    `tuned`: the benchmark's multigrid settings (else the library defaults)."""
    import torch
    import paper_1909_13585_amd as mlb
    nel = tuple(int(v) for v in args.nel.split(","))
    ctx = mlb.Context(nel, mg_levels=levels or args.levels, eig_level=args.eig_level, precision=precision,
                      element=element)
    if tuned:
        set_solver_opts(ctx, args)
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
    1e-8): static solve (with iterative refinement on a double-double
    residual) + compliance gradient of all of them as one batch (one launch
    per solver step for all instances), against the same analyses run one
    context at a time.  Both start from densities on the device.  Instances
    whose true residual stays above 1e-8 are listed with their FP64 floor
    eps ||(|K||u|)|| / ||f||, the residual rounding u to doubles can cause."""
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
    # the same solve without the refinement steps: the work the separate
    # contexts below do (one CG solve to 1e-8 each)
    batched(dict(queue=0, graphs=1, refine_steps=0))
    t_norefine = min(batched(dict(queue=0, graphs=1, refine_steps=0))[0] for _ in range(reps))
    b.set_opts(refine_steps=10)
    _, J, its, info = batched(dict(queue=1, graphs=1))
    res, floor, res_dd = b.residuals()
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
            "s_batched_without_refinement": t_norefine, "speedup_same_work": tseq / t_norefine,
            "max_iterations": int(info["max_iterations"]), "total_iterations": int(info["total_iterations"]),
            "worst_true_rel_res": info["worst_true_rel_res"], "refine_steps": int(info["refine_steps"]),
            "worst_refined_rel_res": info["worst_refined_rel_res"],
            "misses_above_tol": [{"instance": i, "nel": list(insts[i]["nel"]), "true_rel_res": float(res[i]),
                                  "fp64_floor": float(floor[i])} for i in range(len(insts)) if res[i] > 1e-8],
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


def sweep_timing(ctx, level, ncols, reps):
    """Mean time (ms) of one Jacobi sweep of the cycle (the smoother kernel as
    a cycle launches it), HIP events on the stream the library launches on
    (the caller's current stream)."""
    import torch
    ctx.sweep_dev(level, ncols, 5)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    ctx.sweep_dev(level, ncols, reps)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def valu_ceiling(tiles, word, sweep_ms):
    """The fine sweep's VALU ceiling (ms) from its counted instructions, and
    the fraction of it the timed sweep reaches (tuned tile with counters
    only, else None)."""
    insts = SWEEP_VALU_INSTS.get((tiles["wht_variant"], tiles["wht_zchunk"])) if tiles and word == 4 else None
    if insts is None:
        return None
    ms = insts * VALU_CYCLES_PER_INST / (SIMDS * CLOCK_HZ) * 1e3
    return {"valu_insts": insts, "ceiling_ms": ms, "frac": ms / sweep_ms}


def sweep_bytes(dim, nel, level, ncols, word):
    """Algorithmic HBM bytes of one Jacobi sweep of `ncols` columns on `level`:
    per column x and r read and y written (3 words per DOF); D^-1 read once;
    level 1 (matrix-free): one modulus per element and one mask byte per
    node; coarser levels: the node-block stencil, dim x dim words for each of
    the 3^dim neighbour blocks per node in FP64, for the (3^dim + 1) / 2
    stored ones in FP32 (the FP32 stencil is kept by half, its other blocks
    being the neighbours' transposes)."""
    f = 2 ** (level - 1)
    ne = [v // f for v in nel]
    nodes = 1
    for v in ne:
        nodes *= v + 1
    m = 1
    for v in ne:
        m *= v
    n = dim * nodes
    b = ncols * 3 * word * n + word * n
    nblk = 3 ** dim if word == 8 else (3 ** dim + 1) // 2
    b += word * m + nodes if level == 1 else nodes * nblk * dim * dim * word
    return b


def optimisation_leg(args, steps=3):
    """Design steps of problem P2 (Sec. 6) on the bench box: minimum volume
    with the lowest 12 of 24 buckling factors bounded (bound formulation,
    alpha 0.99) and the compliance at most 6 times the solid design's; filter
    radius 4 sqrt(3), eta 0.5, p = 3 and beta = 1 (the start of Sec. 6's
    continuation).  As in Sec. 6 the start is the solid design, feasible
    for lambda_bar = 0.4 lambda_1(solid) (the section's bounds are at most
    0.42 of its solid factor).  Each step: filter and projection, analysis,
    sensitivities, problem functions, chain rule, MMA update.  One untimed
    step, then the median of ``steps``; the steps recycle the previous
    analysis (coarse modes and displacement as warm starts), and the same
    steps are timed cold beside them."""
    import numpy as np
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W
    from paper_1909_13585_amd.optimize import P2Step
    nel = tuple(int(v) for v in args.nel.split(","))
    p = W.box_3d(nel=nel, seed=3)
    ctx = mlb.Context(nel, mg_levels=args.levels, eig_level=args.eig_level, precision=mlb.MLB_MIXED)
    set_solver_opts(ctx, args)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    n, m = ctx.level_size(1)
    U = torch.empty((1, n), dtype=torch.float64, device="cuda")
    ctx.set_density_dev(torch.ones(m, dtype=torch.float64, device="cuda"))
    J_solid, _ = ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
    rmin, q, nb = 4.0 * np.sqrt(3.0), 24, 12
    lam_solid, _ = ctx.buckling_dev(q, None, tol_eig=args.tol_eig)
    lam_bar = 0.4 * lam_solid[0]

    def run(recycle):
        xhat = torch.ones(m, dtype=torch.float64, device="cuda")
        stepper = P2Step(ctx, q, nb, rmin, 0.5, 1.0, 6.0 * J_solid[0], lam_bar, tol_eig=args.tol_eig,
                         recycle=recycle)
        ctx.set_warm_start(mlb.MLB_WARM_NONE)
        rows = []
        for s in range(steps + 1):
            tm = {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = stepper.step(xhat, penal=3.0, beta=1.0, timings=tm)
            torch.cuda.synchronize()
            tm["step_s"] = time.perf_counter() - t0
            tm.update(volume=info["f0"], max_constraint=float(np.max(info["fval"])),
                      dual_evaluations=info["dual_evaluations"], dual_iterations=info["dual_iterations"],
                      static_iterations=info["static_iterations"], coarse_iterations=info["coarse_iterations"],
                      coarse_warm_used=info["coarse_warm_used"], fine_iterations=info["fine_iterations"])
            rows.append(tm)
            print(f"# P2 step {s} (recycle {recycle}): {tm}", file=sys.stderr, flush=True)
        return rows

    cold = run(False)
    rows = run(True)
    ctx.close()
    timed = rows[1:]
    med = lambda key: float(np.median([r[key] for r in timed]))
    medc = lambda key: float(np.median([r[key] for r in cold[1:]]))
    mcon = 1 + nb
    ev = float(np.median([r["dual_evaluations"] for r in timed]))
    # algorithmic bytes of one MMA update: the preparation pass, the dual
    # passes (gradient rows, 5 per-variable arrays, B written and read by the
    # Gram product) and the final pass
    mma_bytes = 8 * m * ((mcon + 12) + ev * (3 * mcon + 6) + (mcon + 7))
    return {"workload": f"P2 (Sec. 6) design steps on the H8 box {nel[0]}x{nel[1]}x{nel[2]}: {q} modes, lowest "
                        f"{nb} bounded, rmin 4 sqrt(3), p 3, beta 1, mixed precision, {args.levels} levels",
            "s_per_design_step": med("step_s"), "analysis_s": med("analysis_s"),
            "recycled": {"coarse_iterations": [r["coarse_iterations"] for r in rows],
                         "coarse_block_kept": [r["coarse_warm_used"] for r in rows],
                         "static_iterations": [r["static_iterations"] for r in rows]},
            "cold": {"s_per_design_step": medc("step_s"), "analysis_s": medc("analysis_s"),
                     "coarse_iterations": [r["coarse_iterations"] for r in cold],
                     "static_iterations": [r["static_iterations"] for r in cold],
                     "max_rel_volume_diff": float(max(abs(a["volume"] / b["volume"] - 1) for a, b in zip(rows, cold)))},
            "functions_chain_s": med("functions_chain_s"), "mma_s": med("mma_s"),
            "mma_dual_evaluations": ev, "mma_alg_bytes": mma_bytes,
            "mma_gbs": mma_bytes / med("mma_s") / 1e9,
            "volume_after": [r["volume"] for r in rows], "max_constraint_after": [r["max_constraint"] for r in rows],
            "lambda_bar": float(lam_bar), "lambda1_solid": float(lam_solid[0]), "J_max": float(6.0 * J_solid[0])}


def nn_forward_leg(net, nel, ell, reps=20):
    """The warm-start network's forward pass on its input for the bench box
    (eigen-level cells), with the 3x3x3 convolutions on the VALU kernels
    (FP32 activations) and on the matrix cores (BF16 activations, FP32
    accumulation); HIP events on the current stream, mean over ``reps``.
    The flop count is that of the 3x3x3 convolutions (2 flops per
    multiply-add)."""
    import numpy as np
    import torch
    shp = [v // 2 ** (ell - 1) for v in nel]
    x = torch.randn((1, net.cin) + tuple(reversed(shp)), dtype=torch.float32, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(3))
    V = [int(np.prod(shp)), int(np.prod(shp)) // 8, int(np.prod(shp)) // 64]
    lev = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "b1": 2, "b2": 2, "d2a": 1, "d2b": 1, "d1a": 0, "d1b": 0}
    flops = sum(2.0 * V[lev[name]] * ci * co * 27 for name, ci, co, k, _ in net.layers if k == 3)
    st = torch.cuda.current_stream()
    out = {}
    for mode in (False, True):
        net.mfma = mode
        net.forward(x)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            net.forward(x)
        e1.record(st)
        torch.cuda.synchronize()
        out["mfma_ms" if mode else "valu_ms"] = e0.elapsed_time(e1) / reps
    net.mfma = False
    out.update(input=[1, net.cin] + list(reversed(shp)), conv_gflop=flops / 1e9,
               mfma_tflops=flops / (out["mfma_ms"] * 1e-3) / 1e12,
               note="whole forward pass (convolutions, pooling, concatenation, head) per call")
    return out


def column_leg(args, steps=3):
    """The 960x320 Q4 column (616,962 DOFs) in plain FP64 on 4 and 5 multigrid
    levels: static solve + 12 modes on the 240x80 eigen level + sensitivities."""
    import numpy as np
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W
    nel = (960, 320)
    p = W.column_2d_large()
    xd = torch.from_numpy(p["x"]).cuda()
    out = {}
    for L in (4, 5):
        ctx = mlb.Context(nel, mg_levels=L, eig_level=3, precision=mlb.MLB_FP64)
        ctx.set_bc(p["fixed"])
        ctx.set_loads(p["F"])
        n, m = ctx.level_size(1)
        U = torch.empty((1, n), dtype=torch.float64, device="cuda")
        dJ = torch.empty((1, m), dtype=torch.float64, device="cuda")
        dl = torch.empty((12, m), dtype=torch.float64, device="cuda")
        ts = []
        for _ in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.set_density_dev(xd)
            J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
            lam, ei = ctx.buckling_dev(12, None, tol_eig=1e-8)
            ai = ctx.sensitivities_dev(dJ, dl)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ctx.close()
        ts = sorted(ts[1:])
        out[f"levels_{L}"] = {"s_per_analysis": ts[len(ts) // 2], "static_iterations": si["iterations"],
                              "static_true_rel_res": si["true_rel_residual"],
                              "coarse_iterations": ei["coarse_iterations"], "coarse_residual": ei["coarse_residual"],
                              "coarse_guard_fired": ei["coarse_guard_fired"],
                              "fine_block_iterations": ei["fine_iterations"],
                              "fine_true_rel_res": ei["fine_true_residual"],
                              "adjoint_iterations": ai["iterations"], "adjoint_true_rel_res": ai["true_rel_residual"],
                              "lambda1": float(lam[0])}
        print(f"# column levels {L}: {out[f'levels_{L}']}", file=sys.stderr, flush=True)
    return {"workload": "Q4 column 960x320 (616962 DOFs), FP64, eigen level 3 (240x80), 12 modes, 1e-8", **out}


def block16_leg(args, reps=3):
    """16-column block CG on the 96x48x48 box (698,691 DOFs, mixed precision):
    4 static load cases (axial, shear y, shear z, torsion) and the 12 adjoint
    right-hand sides of a prior analysis of the same density, one block solve
    to 1e-8 per column, against the same 16 columns solved one at a time."""
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W
    nel = (96, 48, 48)
    p = W.box_3d_four_cases(nel=nel)
    ctx = mlb.Context(nel, mg_levels=4, eig_level=3, precision=mlb.MLB_MIXED)
    set_solver_opts(ctx, args)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    n, m = ctx.level_size(1)
    xd = torch.from_numpy(p["x"]).cuda()
    ctx.set_density_dev(xd)
    ctx.autotune(16)
    U = torch.empty((4, n), dtype=torch.float64, device="cuda")
    ctx.solve_static_dev(U, tol=1e-8, max_it=3000)
    ctx.buckling_dev(12, None, tol_eig=args.tol_eig)
    dl = torch.empty((12, m), dtype=torch.float64, device="cuda")
    ctx.sensitivities_dev(None, dl)
    Badj = torch.empty((12, n), dtype=torch.float64, device="cuda")
    ctx.adjoint_rhs_dev(12, Badj)
    B = torch.cat([torch.from_numpy(p["F"].T.copy()).cuda(), Badj]).contiguous()
    X = torch.empty_like(B)

    def timed(fn):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts = sorted(ts[1:])
        return ts[len(ts) // 2], r

    t_blk, info = timed(lambda: ctx.solve_block_dev(B, X, tol=1e-8, max_it=3000))
    Xc = torch.empty((1, n), dtype=torch.float64, device="cuda")

    def one_by_one():
        its = []
        for j in range(16):
            its.append(ctx.solve_block_dev(B[j:j + 1].contiguous(), Xc, tol=1e-8, max_it=3000)["iterations"])
        return its

    t_col, its = timed(one_by_one)
    ctx.close()
    free = int(n - p["fixed"].sum())
    return {"workload": "H8 box 96x48x48 (698691 DOFs), mixed, 4 levels: 4 load cases + 12 adjoint RHS",
            "columns": 16, "s_block": t_blk, "block_iterations": info["iterations"],
            "worst_true_rel_res": info["true_rel_residual"], "s_one_column_at_a_time": t_col,
            "column_iterations": its, "speedup": t_col / t_blk,
            "gdof_col_iter_per_s": free * 16 * info["iterations"] / t_blk / 1e9}


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
    prec = mlb.MLB_MIXED if args.precision == "mixed" else mlb.MLB_FP64
    word = 4 if args.precision == "mixed" else 8

    if args.roofline_only:
        # counter runs: the dominant kernel (12-column Jacobi sweeps of the
        # fine level, tuned tiles), then a calibration copy of a buffer far
        # larger than the L2 caches, written by a fill and flushed before
        ctx = mlb.Context(nel, mg_levels=args.levels, eig_level=args.eig_level, precision=prec)
        set_solver_opts(ctx, args)
        ctx.set_bc(p["fixed"])
        ctx.set_loads(p["F"])
        ctx.set_density_dev(x_dev)
        tune = ctx.autotune(args.modes)
        if args.force_wht:
            fv, fz = (int(v) for v in args.force_wht.split(","))
            ctx.set_tiles(wht_zchunk=fz, wht_variant=fv)
            tune = dict(tune, wht_variant=fv, wht_zchunk=fz)
        torch.cuda.synchronize()
        ctx.sweep_dev(1, args.modes, args.sweep_reps)
        cal = 1 << 25   # 32 Mi doubles = 256 MiB
        src = torch.empty(cal, dtype=torch.float64, device="cuda").fill_(1.0)
        flush = torch.empty(cal, dtype=torch.float64, device="cuda").fill_(2.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"roofline_only": True, "tiles": {k: tune[k] for k in ("wht_zchunk", "wht_variant")},
                          "sweeps": args.sweep_reps, "copy_bytes": 8 * cal,
                          "alg_bytes": sweep_bytes(3, nel, 1, args.modes, word),
                          "flush_bytes": int(flush.numel() * 8)}), flush=True)
        ctx.close()
        return

    ctx, sec, out = run_path(args, prec, p, x_dev, args.steps, args.warmup, args.precision)
    J, si, lam, ei, ai = out
    n, m = ctx.level_size(1)
    k = args.modes
    free = int(n - p["fixed"].sum())
    gdofs = free * si["iterations"] / si["seconds"] / 1e9

    # dominant kernel: the 12-column Jacobi sweep of the fine level; the
    # level-2 stencil sweep beside it
    sw1 = sweep_timing(ctx, 1, k, args.sweep_reps)
    b1 = sweep_bytes(3, nel, 1, k, word)
    sw2 = sweep_timing(ctx, 2, k, args.sweep_reps)
    b2 = sweep_bytes(3, nel, 2, k, word)
    pinv = None if args.no_pinvit else pinvit_leg(ctx, k, n, args.tol_eig, lam)
    refine = None if args.no_pinvit else refine_leg(ctx, k, n, args.tol_eig, lam)
    postp = None if args.no_post else post_leg(ctx, k, n, m, x_dev, args.tol_eig)
    designp = None if args.no_post else design_leg(ctx, m, x_dev, k)
    tiles = {q: ctx.tune[q] for q in ("wht_zchunk", "wht_variant", "wht64_zchunk", "wht64_variant",
                                      "stencil_cols")} if ctx.tune else None
    ctx.close()

    five = None
    if not args.no_five_level:
        ctx5, sec5, out5 = run_path(args, prec, p, x_dev, max(1, min(args.steps, 3)), 1, "five-level", levels=5,
                                    tuned=False)
        ctx5.close()
        five = {"s_per_analysis": sec5, "levels": 5, "settings": "library defaults (2 sweeps, omega 4/3)",
                "static_iterations": out5[1]["iterations"], "coarse_iterations": out5[3]["coarse_iterations"],
                "fine_block_iterations": out5[3]["fine_iterations"], "adjoint_iterations": out5[4]["iterations"],
                "max_rel_lambda_diff": float(np.max(np.abs(np.asarray(out5[2]) / np.asarray(lam) - 1)))}

    learned = None
    if os.path.exists(args.learned):
        from paper_1909_13585_amd.warmstart import UNet3D
        net = UNet3D.from_file(args.learned)
        ctxl, secl, outl = run_path(args, prec, p, x_dev, args.steps, 1, "learned", net=net)
        ctxl.close()
        learned = {"s_per_analysis": secl, "static_iterations": outl[1]["iterations"],
                   "coarse_iterations": outl[3]["coarse_iterations"], "coarse_warm_used": outl[3]["coarse_warm_used"],
                   "fine_block_iterations": outl[3]["fine_iterations"],
                   "adjoint_iterations": outl[4]["iterations"],
                   "max_rel_lambda_diff_vs_cold": float(np.max(np.abs(np.asarray(outl[2]) / np.asarray(lam) - 1))),
                   "weights": os.path.relpath(args.learned, ROOT),
                   "network_forward": nn_forward_leg(net, nel, args.eig_level)}

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
        ctx64, sec64, out64 = run_path(args, mlb.MLB_FP64, p, x_dev, max(1, min(args.steps, 3)), 1, "fp64")
        ctx64.close()
        fp64 = {"s_per_analysis": sec64, "static_iterations": out64[1]["iterations"],
                "coarse_iterations": out64[3]["coarse_iterations"],
                "fine_block_iterations": out64[3]["fine_iterations"],
                "adjoint_iterations": out64[4]["iterations"],
                "max_rel_lambda_diff_vs_mixed": float(np.max(np.abs(np.asarray(out64[2]) / np.asarray(lam) - 1)))}

    column = None if args.no_column else column_leg(args)
    block16 = None if args.no_block16 else block16_leg(args)
    optim = None if args.no_opt else optimisation_leg(args)
    inst = None if args.no_instances else batched_instances()

    cpu = None
    if not args.no_cpu_baseline:
        o = cpu_baseline(args)
        g_s, g_l1 = gpu_on_cpu_sample(args)
        med = o["median"]
        cpu = {"value": med["total"], "unit": "s/analysis", "cores": o["blas_threads"], "kind": "oracle",
               "sample": (f"oracle analysis (SuperLU factorization and solves, dense LAPACK eigen level, "
                          f"Rayleigh-Ritz, adjoints, sensitivities) of the {CPU_SAMPLE[0]}x{CPU_SAMPLE[1]}x"
                          f"{CPU_SAMPLE[2]} H8 box of the same recipe ({o['dofs']} DOFs, eigen level 2, {k} modes), "
                          f"median of {len(o['totals'])} runs on the host, not scaled; the SuperLU "
                          f"factorization runs on one thread, LAPACK on {o['blas_threads']}"),
               "phases_s": med, "totals_s": o["totals"], "peak_rss_gb": o["rss_gb"], "cpu_model": o["cpu_model"],
               "logical_cpus": o["logical_cpus"], "gpu_s_same_sample": g_s,
               "lambda1_oracle": o["lambda1"], "lambda1_gpu": g_l1}

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
                               f"Gaussian-filtered density vf 0.3 (seed 3), {args.levels}-level MG "
                               f"({args.smooth}/{args.smooth}/{args.coarse_sweeps} Jacobi sweeps, omega "
                               f"{args.omega:g}/(1.05 rho); the 5-level hierarchy is timed in five_level_mg), "
                               f"eigen level {args.eig_level}, {k} modes, solves to 1e-8, coarse eigen to "
                               f"{args.tol_eig:g}",
                   "precision": args.precision},
        "tiles": tiles,
        "mgpcg_gdof_per_s": gdofs,
        "static_iterations": si["iterations"],
        "coarse_iterations": ei["coarse_iterations"],
        "fine_block_iterations": ei["fine_iterations"],
        "adjoint_iterations": ai["iterations"],
        "residuals": {"static_true_rel": si["true_rel_residual"], "fine_block_true_rel": ei["fine_true_residual"],
                      "adjoint_true_rel": ai["true_rel_residual"], "coarse_eigen_rel": ei["coarse_residual"],
                      "coarse_guard_fired": ei["coarse_guard_fired"]},
        "lambda": [float(v) for v in lam],
        "phase_s": {"coarse": ei["seconds_coarse"], "fine": ei["seconds_fine"], "ritz": ei["seconds_ritz"],
                    "static": si["seconds"], "adjoint": ai["seconds"]},
        "five_level_mg": five,
        "fp64_reference": fp64,
        "learned_warm_start": learned,
        "column_960x320_fp64": column,
        "block16_96x48x48": block16,
        "optimisation_p2": optim,
        "pinvit_refinement": pinv,
        "intermediate_refinement": refine,
        "incompatible_element": incompatible,
        "post_processing": postp,
        "design_chain": designp,
        "batched_instances": inst,
        "roofline": {"bound": "hbm", "kernel": f"fine-level Jacobi sweep, {k} columns, "
                                               f"{'FP32' if word == 4 else 'FP64'} (k_apply_wht3*)",
                     "achieved": b1 / (sw1 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b1 / (sw1 * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": SWEEP_TRAFFIC_BYTES.get((tiles["wht_variant"], tiles["wht_zchunk"])) if tiles and word == 4 else None,
                     "sweep_ms": sw1, "alg_bytes": b1, "launches_timed": args.sweep_reps,
                     "valu_ceiling": valu_ceiling(tiles, word, sw1),
                     "level2_stencil_sweep": {"sweep_ms": sw2, "alg_bytes": b2,
                                              "achieved": b2 / (sw2 * 1e-3) / 1e9,
                                              "frac": b2 / (sw2 * 1e-3) / 1e9 / HBM_PEAK_GBS}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
