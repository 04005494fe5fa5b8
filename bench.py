"""Benchmark of the hpG hot path on one MI355X.

One step = one complete hpG solve (proximal-point loop, Newton, MINRES with
the block preconditioner, all on the GPU) of the 2-D obstacle workload:
unit square, 32 x 32 cells, p = 6, f = sum_{i,j<=4} c_ij sin(i pi x) sin(j pi y)
(c_ij ~ N(0,1) 20/(i^2+j^2), seed 0), phi = 0.05 + 0.3 |x - (1/2,1/2)|^2,
alpha_k = 2^k, outer tolerance 1e-10.  Inputs are resident in HBM before the
timed region; each solve writes u and psi into device buffers.

Reported: DOF * Krylov iterations per second (value), solves/s and p50/p99
solve latency, the roofline position of the dominant kernel (HIP events
around its launches inside the timed region, algorithmic bytes per launch),
and the CPU oracle's throughput on a bounded sample (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--p", type=int, default=6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-newton-sample", type=int, default=2)
    return ap.parse_args()


def algorithmic_bytes(group, mesh, b):
    """Bytes a launch of the kernel group must move (each input read once,
    each output written once)."""
    n_u, n_psi, N = mesh.n_u, mesh.n_psi, mesh.n_cells
    Pd, Qd = mesh.P ** mesh.dim, mesh.q ** mesh.dim
    if group == "prec_psi":        # Sinv blocks, r_psi in, z_psi out
        return b * (N * Pd * Pd + 2 * n_psi)
    if group == "apply_G":         # x in, omega in, y out
        return b * (2 * n_u + 2 * n_psi + N * Qd)
    if group == "apply_prec":      # r in, z out, Sinv blocks (FDM factors stay in cache)
        return b * (2 * n_u + 2 * n_psi + N * Pd * Pd)
    raise KeyError(group)


def run_solves(prob, d_u, d_psi, opts, steps, torch, group=None):
    lat = []
    kry = 0
    newton = 0
    prox = 0
    if group:
        prob.set_kernel_timing(group)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        st = prob.solve_device(d_u, d_psi, opts)
        lat.append(time.perf_counter() - ts)
        kry += st.krylov_iters
        newton += st.newton_iters
        prox += st.prox_steps
        assert st.status == 0, st.as_dict()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = None
    if group:
        kt = prob.kernel_time(group)
        prob.set_kernel_timing(None)
    return dict(seconds=t1 - t0, lat=lat, krylov=kry, newton=newton, prox=prox, ktime=kt)


def cpu_baseline(args, newton_per_solve):
    """The oracle as it stands, on a bounded sample: a few Newton steps of the
    first proximal subproblem of the same workload (sparse LU of G each step),
    one thread; extrapolated to solves/s with the Newton count of a solve."""
    from threadpoolctl import threadpool_limits
    from oracle import assemble, lvpp, mesh as OM
    import workloads as W
    f, phi = W.w2d(args.seed)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        om = OM.uniform_mesh(2, args.m, args.p)
        xo = om.quadrature_points()
        sysm = assemble.System(om, f(xo), phi(xo))
        t_asm = time.perf_counter() - t0
        res = lvpp.Result()
        res.newton = 0
        res.lu_seconds = 0.0
        k = args.cpu_newton_sample
        opts = lvpp.Options(max_newton=k)
        z = np.zeros(om.n_psi)
        t1 = time.perf_counter()
        lvpp.newton_subproblem(sysm, np.zeros(om.n_u), z, z.copy(), 2.0, opts, res)
        dt = time.perf_counter() - t1
    per_newton = dt / max(res.newton, 1)
    solve_s = t_asm + per_newton * newton_per_solve
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "%d Newton steps (sparse LU of the full saddle matrix, %d DOF) of the "
                      "first proximal subproblem, %.1f s, plus assembly %.1f s; extrapolated "
                      "with the GPU solve's %d Newton steps per solve; 1 thread"
                      % (res.newton, om.n_u + om.n_psi, dt, t_asm, newton_per_solve),
            "seconds_per_newton_step": per_newton}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hpG path here is a single-GPU build "
              "(no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_13733_amd import hpg
    import workloads as W

    torch.cuda.set_device(0)
    f, phi = W.w2d(args.seed)
    mesh = hpg.Mesh(2, [args.m, args.m], args.p)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh, device=0)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    n_dof = mesh.n_u + mesh.n_psi
    d_u = torch.zeros(mesh.n_u, dtype=torch.float64, device="cuda")
    d_psi = torch.zeros(mesh.n_psi, dtype=torch.float64, device="cuda")
    d_u64 = torch.zeros_like(d_u)

    results = {}
    group = "prec_psi"
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for prec in precs:
        opts = hpg.default_opts(precision=hpg.FP64 if prec == "fp64" else hpg.MIXED)
        if prec == "mixed":
            opts.newton_tol = 1e-10
            opts.krylov_rtol = 1e-6
        for _ in range(args.warmup):
            prob.solve_device(d_u, d_psi, opts)
        r = run_solves(prob, d_u, d_psi, opts, args.steps, torch, group=group)
        if prec == "fp64":
            d_u64.copy_(d_u)
        else:
            diff, nrm = prob.l2_diff(d_u, d_u64)
            r["rel_l2_vs_fp64"] = diff / nrm
        r["opts"] = opts
        results[prec] = r
        print("[bench] %s: %d solves in %.3f s, krylov %d, newton %d, prox %d"
              % (prec, args.steps, r["seconds"], r["krylov"], r["newton"], r["prox"]),
              file=sys.stderr, flush=True)

    def summary(r):
        return dict(dof_krylov_per_s=n_dof * r["krylov"] / r["seconds"],
                    solves_per_s=args.steps / r["seconds"],
                    ms_per_solve=1e3 * r["seconds"] / args.steps,
                    p50_ms=1e3 * float(np.percentile(r["lat"], 50)),
                    p99_ms=1e3 * float(np.percentile(r["lat"], 99)),
                    krylov_per_solve=r["krylov"] / args.steps,
                    newton_per_solve=r["newton"] / args.steps,
                    prox_per_solve=r["prox"] / args.steps)

    # the headline line: the faster path whose solution meets rel-L2 1e-8
    best = "fp64"
    if "mixed" in results and results["mixed"].get("rel_l2_vs_fp64", 1.0) <= 1e-8:
        if "fp64" not in results or results["mixed"]["seconds"] < results["fp64"]["seconds"]:
            best = "mixed"
    if "fp64" not in results:
        best = precs[0]
    rb = results[best]
    sb = summary(rb)
    b = 8 if best == "fp64" else 4
    nl, ms = rb["ktime"]
    avg = ms / max(nl, 1)
    byts = algorithmic_bytes(group, mesh, b)
    achieved = byts / (avg * 1e-3) / 1e9
    out = {
        "metric": "DOF·Krylov-iters/s",
        "value": sb["dof_krylov_per_s"],
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sb["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2-D obstacle, unit square %dx%d cells, p=%d, sine forcing seed %d, "
                               "paraboloid obstacle, alpha_k=2^k, tol 1e-10" % (args.m, args.m, args.p, args.seed),
                   "n_dof": n_dof, "n_u": mesh.n_u, "n_psi": mesh.n_psi, "path": best},
        "solves_per_s": sb["solves_per_s"],
        "p50_ms": sb["p50_ms"],
        "p99_ms": sb["p99_ms"],
        "krylov_per_solve": sb["krylov_per_solve"],
        "newton_per_solve": sb["newton_per_solve"],
        "prox_per_solve": sb["prox_per_solve"],
        "roofline": {"bound": "hbm", "kernel": group, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": byts, "avg_launch_us": avg * 1e3, "launches": nl},
    }
    for prec, r in results.items():
        s = summary(r)
        s.pop("dof_krylov_per_s")
        s["dof_krylov_per_s"] = n_dof * r["krylov"] / r["seconds"]
        if "rel_l2_vs_fp64" in r:
            s["rel_l2_vs_fp64"] = r["rel_l2_vs_fp64"]
        out["path_" + prec] = s
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, int(round(results[precs[0]]["newton"] / args.steps)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
