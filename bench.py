"""Benchmark: full linearized buckling analysis on the 2.4M-DOF H8 box.

One step = one complete analysis with the densities already in HBM:
SIMP moduli + multigrid hierarchy (Galerkin levels, coarsest inverse),
static MG-PCG solve to 1e-8, element stresses, Galerkin K^l/G^l, 12 coarse
modes (LOBPCG), interpolation, 12-column fine block solve K Phi = G Psi,
Rayleigh-Ritz, compliance sensitivities, 12 adjoint solves and buckling
sensitivities.  Prints ONE JSON line (rank 0, N = 1 only).

Also reported: MG-PCG throughput of the static solve (free DOFs x iterations
/ solve time) and the roofline of the dominant kernel (fine-level H8
stiffness apply), timed with HIP events on the library's stream.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--nel", type=str, default="192,64,64")
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--eig-level", type=int, default=3)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the dominant-kernel timing and a copy of known size (for counter runs)")
    return ap.parse_args()


def cpu_baseline(args):
    """The oracle (sparse direct + LAPACK/ARPACK) on a bounded sample of the
    same workload recipe: 48x16x16 H8 box, eigen level 2, 12 modes."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import workloads as W
    from oracle import fem, lba, sens
    nel = (48, 16, 16)
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the analysis is single-GPU by design "
              "(multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1909_13585_amd as mlb
    import workloads as W

    torch.cuda.set_device(0)
    nel = tuple(int(v) for v in args.nel.split(","))
    t_setup = time.perf_counter()
    p = W.box_3d(nel=nel, seed=3)
    prec = mlb.MLB_MIXED if args.precision == "mixed" else mlb.MLB_FP64
    ctx = mlb.Context(nel, mg_levels=args.levels, eig_level=args.eig_level, precision=prec)
    ctx.set_bc(p["fixed"])
    ctx.set_loads(p["F"])
    x_dev = torch.from_numpy(p["x"]).cuda()
    n, m = ctx.level_size(1)
    k = args.modes
    U = torch.empty((ctx.ncases, n), dtype=torch.float64, device="cuda")
    Phi = torch.empty((k, n), dtype=torch.float64, device="cuda")
    dJ = torch.empty((ctx.ncases, m), dtype=torch.float64, device="cuda")
    dlam = torch.empty((k, m), dtype=torch.float64, device="cuda")
    print(f"# setup {time.perf_counter() - t_setup:.1f}s n={n} m={m}", file=sys.stderr, flush=True)

    def step():
        ctx.set_density_dev(x_dev)
        J, si = ctx.solve_static_dev(U, tol=1e-8, max_it=2000)
        lam, ei = ctx.buckling_dev(k, Phi, tol_eig=1e-10)
        ai = ctx.sensitivities_dev(dJ, dlam)
        return J, si, lam, ei, ai

    if args.roofline_only:
        ctx.set_density_dev(x_dev)
        xa = torch.randn(n, dtype=torch.float64, device="cuda")
        ya = torch.empty_like(xa)
        for _ in range(args.apply_reps):
            ctx.apply_K_dev(1, xa, ya)
        ya.copy_(xa)   # calibration: reads and writes exactly 8 n bytes each
        torch.cuda.synchronize()
        print(json.dumps({"roofline_only": True, "n": n, "m": m, "copy_bytes": 8 * n}), flush=True)
        ctx.close()
        return

    for w in range(args.warmup):
        out = step()
        print(f"# warmup {w} static_it={out[1]['iterations']} coarse_it={out[3]['coarse_iterations']} "
              f"fine_it={out[3]['fine_iterations']} adj_it={out[4]['iterations']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times = []
    infos = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        infos.append(out)
        print(f"# step {s} {times[-1]:.3f}s static_it={out[1]['iterations']} "
              f"coarse_it={out[3]['coarse_iterations']} fine_it={out[3]['fine_iterations']} "
              f"adj_it={out[4]['iterations']} lam1={out[2][0]:.6g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    sec = total / max(args.steps, 1)
    J, si, lam, ei, ai = infos[-1]
    free = int(n - p["fixed"].sum())
    gdofs = free * si["iterations"] / si["seconds"] / 1e9

    # dominant kernel: fine-level stiffness apply, one column, timed with
    # HIP events on the library's stream (the caller's current stream).
    xa = torch.randn(n, dtype=torch.float64, device="cuda")
    ya = torch.empty_like(xa)
    for _ in range(5):
        ctx.apply_K_dev(1, xa, ya)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.apply_reps):
        ctx.apply_K_dev(1, xa, ya)
    e1.record(st)
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1) / args.apply_reps
    word = 8
    nodes = n // 3
    alg_bytes = 2 * word * n + word * m + nodes      # x read, y write, E_kappa, node mask
    achieved = alg_bytes / (apply_ms * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        t_cpu, n_sample = cpu_baseline(args)
        cpu = {"value": t_cpu * n / n_sample, "unit": "s/analysis", "cores": 1, "kind": "oracle",
               "sample": (f"oracle analysis (SuperLU static + adjoint solves, ARPACK coarse eigen, Ritz, "
                          f"sensitivities) on the 48x16x16 H8 box of the same recipe ({n_sample} DOFs, eigen "
                          f"level 2, {k} modes): {t_cpu:.2f}s, scaled linearly in DOFs to {n} DOFs "
                          f"(a lower bound: direct solvers scale superlinearly)")}

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
        "config": {"workload": f"H8 box {nel[0]}x{nel[1]}x{nel[2]} ({n} DOFs), clamped x=0, axial load, "
                               f"filtered density vf 0.3, {args.levels}-level MG, eigen level {args.eig_level}, "
                               f"{k} modes, tol 1e-8",
                   "precision": args.precision},
        "mgpcg_gdof_per_s": gdofs,
        "static_iterations": si["iterations"],
        "coarse_iterations": ei["coarse_iterations"],
        "fine_block_iterations": ei["fine_iterations"],
        "adjoint_iterations": ai["iterations"],
        "lambda": [float(v) for v in lam],
        "phase_s": {"coarse": ei["seconds_coarse"], "fine": ei["seconds_fine"], "ritz": ei["seconds_ritz"],
                    "static": si["seconds"], "adjoint": ai["seconds"]},
        "roofline": {"bound": "hbm", "kernel": "k_apply_fine<3,double> (fine H8 K apply, 1 column)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "apply_ms": apply_ms,
                     "alg_bytes": alg_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
