"""Benchmark of the hpG hot path on one MI355X.

One step = one complete hpG solve (proximal-point loop, Newton, MINRES with
the block preconditioner P_D, all on the GPU) of the 2-D obstacle workload:
unit square, 32 x 32 cells, p = 6, f = sum_{i,j<=4} c_ij sin(i pi x) sin(j pi y)
(c_ij ~ N(0,1) 20/(i^2+j^2), seed 0), phi = 0.05 + 0.3 |x - (1/2,1/2)|^2,
alpha_k = 2^k, outer tolerance 1e-10.  Inputs are resident in HBM before the
timed region; each solve writes u and psi into device buffers.

Timed regions (each bracketed by torch.cuda.synchronize()):
  1. K solves per precision path (FP64; mixed = FP32 Krylov + FP64 Newton),
     MINRES chunks replayed as HIP graphs: value, solves/s, p50/p99 latency.
  2. the same K solves of the headline path with HIP events around every
     launch of each kernel group (graphs off, so each launch can be
     bracketed): per-group average durations, from which the roofline
     position of the dominant group is computed.
  3. apply_G alone on the large low-p mesh (2-D 4096 x 4096 cells, p = 2:
     2.55 GB of algorithmic traffic per FP64 apply), HIP events per launch:
     the HBM-roofline position of the operator apply.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-probe]
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
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}


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
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--probes", default="R1,R2,R3",
                    help="roofline probes of the G apply: R1 = 2-D 4096^2 p=2, R2 = 2-D 2048^2 "
                         "p=3, R3 = 3-D 160^3 p=2 (FP64)")
    ap.add_argument("--probe-launches", type=int, default=20)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched solves and the batched apply probe B1")
    ap.add_argument("--batch-n", type=int, default=32,
                    help="slots of the batched solve of the headline mesh")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched stream: one JSON line with its section")
    ap.add_argument("--batch-requests", type=int, default=0,
                    help="requests (seeds 0..n-1) streamed through the slots (0: 3 x slots)")
    ap.add_argument("--b1-n", type=int, default=4096,
                    help="requests of 32x32 cells at p=2 in the batched apply probe B1")
    ap.add_argument("--no-3d", action="store_true",
                    help="skip the 3-D 16^3 p=5 obstacle solves")
    ap.add_argument("--3d-gradient", dest="gradient3d", action="store_true",
                    help="also solve the 3-D 16^3 p=4 gradient-constraint problem (minutes)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="prefix of the 512-request serving stream to run")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving stream: one JSON line with its section")
    ap.add_argument("--serve-paths", default="fp64x1,fp64,mixed,poisson",
                    help="serving runs: fp64x1 (one slot), fp64 and mixed (the slots, all "
                         "requests at once), poisson (mixed, the arrival times)")
    ap.add_argument("--serve-stratified", action="store_true",
                    help="serve only the stratified sample of the 512-request stream "
                         "(workloads.stratified_sample: 36 requests)")
    ap.add_argument("--serve-save", default="",
                    help="directory: u and stats of a stratified sample of the stream "
                         "(workloads.stratified_sample) per run, for the oracle check "
                         "tests/check_serving_stream.py")
    ap.add_argument("--serve-chunk", type=int, default=16,
                    help="MINRES iterations per captured chunk of a serving request")
    ap.add_argument("--no-hp", action="store_true",
                    help="skip the per-cell-degree workload (2-D 64x64, degrees 2..12)")
    ap.add_argument("--hp-steps", type=int, default=2)
    ap.add_argument("--hp-only", action="store_true",
                    help="run only the per-cell-degree workload (for profiling)")
    ap.add_argument("--counters", action="store_true",
                    help="only a few operator launches for rocprofv3 --pmc passes: the "
                         "workload's G apply and preconditioner (FP32 and FP64), the G apply of "
                         "each roofline probe, and a 1 GiB device copy to calibrate the counters")
    ap.add_argument("--hp-counters", action="store_true",
                    help="only a few operator launches of the per-cell-degree workload for "
                         "rocprofv3 --pmc passes: two setups, five G applies and five "
                         "preconditioner applies per precision, each kernel group on its own")
    return ap.parse_args()


def hp_counters_run(args, torch, hpg, W):
    """Short, fixed sequence of launches of the 64 x 64 degree-2..12 workload
    (the cell pass of G, the setup, the preconditioner parts) to read VALU
    and LDS counters against."""
    deg = np.loadtxt(HP_DEGREES, dtype=np.int32).reshape(-1)
    f, phi = W.w2d_dip(0)
    mesh = hpg.Mesh(2, [64, 64], 0, degree=deg)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh, device=0)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    n = mesh.n_u + mesh.n_psi
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    psi = 0.5 * torch.randn(mesh.n_psi, dtype=torch.float64, device="cuda", generator=g)
    prob.set_kernel_timing("all")
    for prec, dt in ((hpg.MIXED, torch.float32), (hpg.FP64, torch.float64)):
        for _ in range(2):
            prob.op_setup(psi, 4.0, 0.0, precision=prec)
        v = torch.randn(n, dtype=dt, device="cuda", generator=g)
        w = torch.empty_like(v)
        for _ in range(5):
            prob.op_apply_G(v, w)
            prob.op_apply_prec(v, w)
    torch.cuda.synchronize()
    prob.set_kernel_timing(None)
    print(json.dumps({"hp_counters_run": "done", "n_u": mesh.n_u, "n_psi": mesh.n_psi,
                      "degree_histogram": np.bincount(deg, minlength=13)[2:].tolist()}),
          flush=True)


def counters_run(args, torch, hpg, W):
    """Short, fixed sequence of launches to read HBM counters against."""
    f, phi = W.w2d(args.seed)
    mesh = hpg.Mesh(2, [args.m, args.m], args.p)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh, device=0)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    n = mesh.n_u + mesh.n_psi
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    psi = 0.5 * torch.randn(mesh.n_psi, dtype=torch.float64, device="cuda", generator=g)
    # kernel timing on: every group launched on its own, as in the timed pass
    # whose per-kernel durations the roofline uses
    prob.set_kernel_timing("all")
    for prec, dt in ((hpg.MIXED, torch.float32), (hpg.FP64, torch.float64)):
        prob.op_setup(psi, 4.0, 0.0, precision=prec)
        v = torch.randn(n, dtype=dt, device="cuda", generator=g)
        w = torch.empty_like(v)
        for _ in range(5):
            prob.op_apply_prec(v, w)
            prob.op_apply_G(v, w)
    # the fast-diagonalisation passes with the 32x32 block tile too (the tile
    # of a problem without a Krylov solve follows HPG_GEMM_TILE, else 16x16)
    keep = os.environ.get("HPG_GEMM_TILE")
    os.environ["HPG_GEMM_TILE"] = "32"
    for prec, dt in ((hpg.MIXED, torch.float32), (hpg.FP64, torch.float64)):
        prob.op_setup(psi, 4.0, 0.0, precision=prec)
        v = torch.randn(n, dtype=dt, device="cuda", generator=g)
        w = torch.empty_like(v)
        for _ in range(5):
            prob.op_apply_prec(v, w)
    if keep is None:
        del os.environ["HPG_GEMM_TILE"]
    else:
        os.environ["HPG_GEMM_TILE"] = keep
    torch.cuda.synchronize()
    prob.set_kernel_timing(None)
    del prob
    args.probe_launches = 5
    for name in [s_.strip() for s_ in args.probes.split(",") if s_.strip()]:
        dim, m, p = PROBES[name]
        apply_probe(args, torch, hpg, dim, m, p, None)
    if not args.no_batch:
        batch_probe(args, torch, hpg)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": "done", "copy_bytes": a.numel() * 8}), flush=True)


GROUPS = ["apply_G", "apply_G_u", "apply_G_psi", "fdm", "prec_psi", "prec_u", "minres_vec",
          "setup", "residual"]


def group_work(mesh, b):
    """Algorithmic work of one launch of each kernel group: bytes each input
    is read once and each output written once, or flops for the MFMA passes."""
    n_u, n_psi, N = mesh.n_u, mesh.n_psi, mesh.n_cells
    Pd, Qd = mesh.P ** mesh.dim, mesh.q ** mesh.dim
    n1 = mesh.info.ncells[0] * mesh.p - 1
    d = mesh.dim
    return {
        # fused apply: x (u and psi) and omega in, y out
        "apply_G": ("hbm", b * (2 * n_u + 2 * n_psi + N * Qd)),
        # u-side: x_u, x_psi in, y_u out
        "apply_G_u": ("hbm", b * (2 * n_u + n_psi)),
        # psi-side: x_u, x_psi, omega in, y_psi out
        "apply_G_psi": ("hbm", b * (n_u + 2 * n_psi + N * Qd)),
        # one fast-diagonalisation pass (one GEMM launch; 2d per preconditioner apply)
        "fdm": ("mfma", 2.0 * n1 ** (d + 1)),
        # inverse blocks, r_psi in, z_psi out
        "prec_psi": ("hbm", b * (N * Pd * Pd + 2 * n_psi)),
    }


TRAFFIC_LABEL = {"fdm": "fdm pass", "apply_G": "G apply", "prec_psi": "psi-block preconditioner"}


def measured_traffic(group, m, p, path):
    """HBM bytes per launch of a kernel group as read by rocprofv3 --pmc
    (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy) and recorded in
    profiles/pmc_traffic.json; None if that kernel/workload was not measured."""
    fn = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "pmc_traffic.json")
    if group not in TRAFFIC_LABEL or not os.path.exists(fn):
        return None
    key = "%s, 2-D %dx%d p=%d, %s" % (TRAFFIC_LABEL[group], m, m, p,
                                      "FP64" if path == "fp64" else "FP32")
    ent = json.load(open(fn))["kernels"].get(key)
    return ent["traffic_bytes"] if ent else None


def run_solves(prob, d_u, d_psi, opts, steps, torch, group=None, check=True):
    lat = []
    kry = newton = prox = 0
    st = None
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
        assert st.status == 0 or not check, st.as_dict()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = {}
    if group:
        for g in GROUPS:
            kt[g] = prob.kernel_time(g)
        prob.set_kernel_timing(None)
    return dict(seconds=t1 - t0, lat=lat, krylov=kry, newton=newton, prox=prox, ktime=kt, last=st)


def cpu_baseline(args, newton_per_solve):
    """The oracle as it stands, on a bounded sample: a few Newton steps of the
    first proximal subproblem of the same workload (sparse LU of the full
    saddle matrix G each step), one thread; extrapolated to solves/s with the
    Newton count of one solve of the same discrete problem."""
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
        opts = lvpp.Options(max_newton=args.cpu_newton_sample)
        z = np.zeros(om.n_psi)
        t1 = time.perf_counter()
        lvpp.newton_subproblem(sysm, np.zeros(om.n_u), z, z.copy(), 2.0, opts, res)
        dt = time.perf_counter() - t1
    per_newton = dt / max(res.newton, 1)
    solve_s = t_asm + per_newton * newton_per_solve
    out = {"value": 1.0 / solve_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": "%d Newton steps (sparse LU of the full saddle matrix, %d DOF) of the "
                     "first proximal subproblem, %.1f s, plus assembly %.1f s; extrapolated "
                     "with %d Newton steps per solve; 1 thread"
                     % (res.newton, om.n_u + om.n_psi, dt, t_asm, newton_per_solve),
           "seconds_per_newton_step": per_newton,
           "lu_share": res.lu_seconds / max(dt, 1e-300),
           "host": host_info()}
    # the whole oracle solve of this workload, timed where the stored oracle
    # solution was written (tests/golden), for comparison with the extrapolation
    fn = os.path.join(ROOT, "tests", "golden", "solve_2d_%dx%d_p%d.npz" % (args.m, args.m, args.p))
    if args.seed == 0 and os.path.exists(fn):
        z = np.load(fn)
        out["full_solve_reference"] = {
            "seconds": float(z["solve_seconds"]), "lu_seconds": float(z["lu_seconds"]),
            "newton": int(z["newton"]), "prox_steps": int(z["prox_steps"]),
            "nproc": int(z["nproc"]), "cpu_model": str(z["cpu_model"]),
            "where": "the machine that wrote the stored oracle solution, 1 thread"}
    return out


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = 0
    try:
        with open("/proc/meminfo") as fh:
            mem = int(fh.readline().split()[1]) * 1024
    except (OSError, ValueError, IndexError):
        pass
    return {"nproc": os.cpu_count() or 0, "cpu_model": model, "mem_GB": mem / 1e9}


PROBES = {"R1": (2, 4096, 2), "R2": (2, 2048, 3), "R3": (3, 160, 2)}


def copy_bandwidth(torch):
    """Device-to-device copy of a 1 GiB FP64 buffer (HIP events): bytes read
    plus bytes written per second, the bandwidth a streaming kernel can reach."""
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    out = {"bytes": 2 * a.numel() * 8, "us": sec * 1e6, "GBs": 2 * a.numel() * 8 / sec / 1e9}
    del a, b
    torch.cuda.empty_cache()
    return out


def apply_probe(args, torch, hpg, dim, m, p, copy_gbs):
    """HBM roofline of the operator apply on a large low-p mesh (FP64)."""
    mesh = hpg.Mesh(dim, [m] * dim, p)
    prob = hpg.Problem(mesh, device=0)
    n = mesh.n_u + mesh.n_psi
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    psi = 0.5 * torch.randn(mesh.n_psi, dtype=torch.float64, device="cuda", generator=gen)
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.empty_like(x)
    prob.op_setup(psi, 4.0, 0.0, precision=hpg.FP64)
    for _ in range(3):
        prob.op_apply_G(x, y)
    prob.set_kernel_timing("all")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.probe_launches):
        prob.op_apply_G(x, y)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.probe_launches
    nf, msf = prob.kernel_time("apply_G")
    nu, msu = prob.kernel_time("apply_G_u")
    npx, msp = prob.kernel_time("apply_G_psi")
    prob.set_kernel_timing(None)
    Qd = mesh.q ** dim
    alg = 8 * (2 * mesh.n_u + 2 * mesh.n_psi + mesh.n_cells * Qd)
    if nf:
        t_apply = msf / nf * 1e-3
        launches = nf
    else:
        t_apply = (msu / nu + msp / npx) * 1e-3
        launches = nu
    ach = alg / t_apply / 1e9
    fn = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "pmc_traffic.json")
    ent = None
    if os.path.exists(fn):
        ent = json.load(open(fn))["kernels"].get("G apply, %d-D %s p=%d, FP64"
                                                 % (dim, "x".join([str(m)] * dim), p))
    out = {"workload": "apply_G, %d-D %s cells, p=%d, FP64" % (dim, "x".join([str(m)] * dim), p),
           "traffic": ent["traffic_bytes"] if ent else None,
           "kernel": "fused tiled apply" if nf else "u-side + psi-side kernels",
           "algorithmic_bytes": alg, "apply_us": t_apply * 1e6,
           "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
           "frac_of_copy": ach / copy_gbs if copy_gbs else None,
           "wall_us_per_call": wall * 1e6, "launches": launches}
    del prob, mesh, x, y, psi
    torch.cuda.empty_cache()
    return out


# ---- serving: the Poisson request stream (2-D n x n cells, n in 8..64,
# p in 2..10, 25% gradient constraint) through the continuous-batching server
def serving_requests(hpg, W, n_req, only=None):
    """The first n_req requests of the 512-request stream (or the listed ones)."""
    arrivals, reqs = W.serving_stream(512, 40.0, 12345)
    idx = list(only) if only is not None else list(range(n_req))
    arrivals = arrivals[idx]
    reqs = [reqs[i] for i in idx]
    built = []
    for r in reqs:
        kind = hpg.GRADIENT if r["kind"] == "gradient" else hpg.OBSTACLE
        mesh = hpg.Mesh(2, [r["n"], r["n"]], r["p"], constraint=kind)
        x = mesh.quadrature_points()
        f, phi = W.request_data(r)
        built.append((mesh, f(x), phi(x), r))
    return arrivals, built


SERVE_KRYLOV_CHUNK = 16   # MINRES iterations per captured chunk of a serving request


def request_opts(hpg, r, precision):
    """Obstacle requests: alpha_k = 2^k to the 1e-10 proximal tolerance.
    Gradient requests: the paper's schedule for that problem class,
    alpha_1 = 2^-7, alpha_{k+1} = min(sqrt(2) alpha_k, 4), 20 steps, with up
    to 20000 MINRES iterations per Newton step (P_D is weak once the gradient
    constraint is active: a cap of 2000 stalls Newton at errors ~3e-3 on large
    high-degree requests).  A Newton stall is accepted at error 1e-8 (the
    serving accuracy target); up to 200 Newton steps per subproblem (large
    high-degree obstacle requests need over 100 in their second subproblem,
    whose linear tail cuts the error by ~e per step)."""
    kw = dict(stall_tol=1e-8, max_newton=200, krylov_chunk=SERVE_KRYLOV_CHUNK)
    if r["kind"] == "gradient":
        kw.update(alpha0=2.0 ** -7, alpha_factor=2.0 ** 0.5, alpha_max=4.0, fixed_prox_steps=20,
                  max_krylov=20000)
    if precision == hpg.MIXED:
        kw.update(precision=hpg.MIXED, newton_tol=1e-10, krylov_rtol=1e-6)
    return hpg.default_opts(**kw)


def serve(hpg, built, arrivals, slots, precision, label):
    srv = hpg.Server(device=0, max_slots=slots)
    t0 = time.perf_counter()
    tickets = []
    for i, (mesh, f, phi, r) in enumerate(built):
        if arrivals is not None:
            dt = t0 + float(arrivals[i]) - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        tickets.append(srv.submit(mesh, f, phi, request_opts(hpg, r, precision)))
    out = [None] * len(tickets)
    pending = dict(enumerate(tickets))
    while pending:
        for i, t in list(pending.items()):
            res = srv.poll(t)
            if res is None:
                continue
            u, psi, st, info = res
            out[i] = (u, st, info)
            del pending[i]
            print("[bench] serving %s: request %d done (status %d, %.2f s), %d/%d, %.1f s"
                  % (label, i, st.status, info.run_s, len(tickets) - len(pending), len(tickets),
                     time.perf_counter() - t0), file=sys.stderr, flush=True)
        time.sleep(0.01)
    stats = srv.stats().as_dict()
    srv.close()
    return out, stats


def serving_bench(args, hpg, W):
    if args.serve_stratified:
        # only the stratified sample of the whole stream, in stream order
        _, allreqs = W.serving_stream(512, 40.0, 12345)
        index = W.stratified_sample(allreqs)
        arrivals, built = serving_requests(hpg, W, 0, only=index)
        sample = list(range(len(built)))
    else:
        arrivals, built = serving_requests(hpg, W, args.serve_requests)
        index = list(range(len(built)))
        sample = W.stratified_sample([r for _, _, _, r in built])
    paths = [x.strip() for x in args.serve_paths.split(",") if x.strip()]

    def summary(res, stats):
        ok = [st.status == 0 for _, st, _ in res]
        return {"requests": len(res), "converged": int(sum(ok)),
                "solves_per_s": stats["solves_per_s"],
                "dof_krylov_per_s": stats["dof_krylov_per_s"],
                "p50_latency_s": stats["p50_latency_s"], "p99_latency_s": stats["p99_latency_s"],
                "max_running": stats["max_running"], "span_s": stats["span_s"],
                "hbm_peak_reserved_GB": stats["hbm_peak_reserved"] / 1e9,
                "fp64_fallbacks": int(sum(st.fp64_fallbacks for _, st, _ in res)),
                "fp64_recomputations": int(sum(st.fp64_recomputations for _, st, _ in res))}

    def save(label, res):
        if not args.serve_save:
            return
        os.makedirs(args.serve_save, exist_ok=True)
        for i in sample:
            u, st, info = res[i]
            np.savez(os.path.join(args.serve_save, "req%03d_%s.npz" % (index[i], label)), u=u,
                     stats=json.dumps(st.as_dict()), request=json.dumps(built[i][3]))

    runs = {}
    if "fp64x1" in paths:
        runs["fp64_sequential"] = serve(hpg, built, None, 1, hpg.FP64, "fp64 x1")
    if "fp64" in paths:
        runs["fp64_batched"] = serve(hpg, built, None, args.serve_slots, hpg.FP64,
                                     "fp64 x%d" % args.serve_slots)
        save("fp64", runs["fp64_batched"][0])
    if "mixed" in paths:
        runs["mixed_batched"] = serve(hpg, built, None, args.serve_slots, hpg.MIXED,
                                      "mixed x%d" % args.serve_slots)
        save("mixed", runs["mixed_batched"][0])
    if "poisson" in paths:
        runs["mixed_poisson"] = serve(hpg, built, arrivals, args.serve_slots, hpg.MIXED,
                                      "mixed poisson")
    kinds = [r["kind"] for _, _, _, r in built]
    out = {
        "workload": "serving stream: %s of 512 requests, Poisson arrivals 40/s (seed "
                    "12345); 2-D n x n cells, n in 8..64, p in 2..10, f sine family and "
                    "paraboloid / dip obstacle, 25%% gradient constraint with phi ~ U[0.2, 0.5]"
                    % ("the stratified sample (%d)" % len(built) if args.serve_stratified
                       else "the first %d" % len(built)),
        "gradient_requests": kinds.count("gradient"),
        "slots": args.serve_slots,
    }
    for k, (res, st) in runs.items():
        out[k] = summary(res, st)
    sps = {k: st["solves_per_s"] for k, (res, st) in runs.items()}
    # mixed x slots over FP64 x1 mixes precision and concurrency; the two
    # ratios after it separate them
    if "mixed_batched" in sps and "fp64_sequential" in sps:
        out["speedup_batched_mixed_vs_fp64"] = sps["mixed_batched"] / max(sps["fp64_sequential"], 1e-300)
    if "mixed_batched" in sps and "fp64_batched" in sps:
        out["speedup_mixed_vs_fp64_same_slots"] = sps["mixed_batched"] / max(sps["fp64_batched"], 1e-300)
    if "fp64_batched" in sps and "fp64_sequential" in sps:
        out["speedup_fp64_slots_vs_one"] = sps["fp64_batched"] / max(sps["fp64_sequential"], 1e-300)
    ref = runs.get("fp64_sequential", runs.get("fp64_batched"))
    if "mixed_batched" in runs and ref is not None:
        errs = [float(np.linalg.norm(ub - us) / max(np.linalg.norm(us), 1e-300))
                for (ub, sb, _), (us, ss, _) in zip(runs["mixed_batched"][0], ref[0])
                if sb.status == 0 and ss.status == 0]
        out["accuracy_note"] = ("relative l2 distance of the mixed-path u to the FP64-path u, over "
                                "the requests both paths converged on")
        out["max_rel_l2_mixed_vs_fp64"] = max(errs) if errs else None
        out["median_rel_l2_mixed_vs_fp64"] = float(np.median(errs)) if errs else None
    if "mixed_batched" in runs and "mixed_poisson" in runs:
        differ = [i for i, (a, b) in enumerate(zip(runs["mixed_batched"][0], runs["mixed_poisson"][0]))
                  if not np.array_equal(a[0], b[0])]
        out["poisson_equals_batched"] = not differ
        out["poisson_differs_at"] = differ
    if args.serve_save:
        out["saved_sample"] = [index[i] for i in sample]
    return out


HP_DEGREES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                          "dip_64x64_degrees.txt")


def hp_bench(args, torch, hpg, W):
    """Per-cell degrees: the 2-D 64x64 dip-obstacle workload with degrees 2..12
    graded away from the contact boundary; FP64 and mixed full solves."""
    deg = np.loadtxt(HP_DEGREES, dtype=np.int32).reshape(-1)
    f, phi = W.w2d_dip(0)
    mesh = hpg.Mesh(2, [64, 64], 0, degree=deg)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh, device=0)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    n_dof = mesh.n_u + mesh.n_psi
    d_u = torch.zeros(mesh.n_u, dtype=torch.float64, device="cuda")
    d_psi = torch.zeros(mesh.n_psi, dtype=torch.float64, device="cuda")
    d_u64 = torch.zeros_like(d_u)
    out = {"workload": "2-D obstacle 64x64 cells, per-cell degree 2..12 (2 within 0.1 of the "
                       "contact boundary of a p=2 pilot solve, 12 beyond 0.4), sine forcing seed 0, "
                       "dip obstacle phi = 0.2 - 0.15 exp(-20|x-x0|^2), alpha_k=2^k, tol 1e-10",
           "n_u": mesh.n_u, "n_psi": mesh.n_psi,
           "degree_histogram": np.bincount(deg, minlength=13)[2:].tolist()}
    for prec in ("fp64", "mixed"):
        opts = hpg.default_opts(precision=hpg.FP64 if prec == "fp64" else hpg.MIXED)
        if prec == "mixed":
            opts.newton_tol = 1e-10
            opts.krylov_rtol = 1e-6
        prob.solve_device(d_u, d_psi, opts)   # warm-up (tables, graphs)
        steps = 1 if prec == "fp64" else args.hp_steps
        r = run_solves(prob, d_u, d_psi, opts, steps, torch)
        ent = {"solves_per_s": steps / r["seconds"], "ms_per_solve": 1e3 * r["seconds"] / steps,
               "dof_krylov_per_s": n_dof * r["krylov"] / r["seconds"],
               "krylov_per_solve": r["krylov"] / steps, "newton_per_solve": r["newton"] / steps,
               "prox_per_solve": r["prox"] / steps}
        if prec == "fp64":
            d_u64.copy_(d_u)
        else:
            diff, nrm = prob.l2_diff(d_u, d_u64)
            ent["rel_l2_vs_fp64"] = diff / nrm
            rt = run_solves(prob, d_u, d_psi, opts, 1, torch, group="all")
            ent["kernel_groups"] = {g: {"launches": nl, "avg_us": 1e3 * ms / nl}
                                    for g, (nl, ms) in rt["ktime"].items() if nl}
        out["path_" + prec] = ent
        print("[bench] hp %s: %.3f s per solve, krylov %d, newton %d"
              % (prec, 1e-3 * ent["ms_per_solve"], ent["krylov_per_solve"],
                 ent["newton_per_solve"]), file=sys.stderr, flush=True)
    return out


def batch_probe(args, torch, hpg):
    """B1: the G apply of args.b1_n requests of 32 x 32 cells at p = 2 (FP64)
    in one launch (hpg_batch_op_apply_G), HIP events per launch."""
    nb = args.b1_n
    mesh = hpg.Mesh(2, [32, 32], 2)
    bt = hpg.Batch(mesh, nb)
    n = mesh.n_u + mesh.n_psi
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    psi = 0.5 * torch.randn(nb * mesh.n_psi, dtype=torch.float64, device="cuda", generator=gen)
    x = torch.randn(nb * n, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.empty_like(x)
    bt.op_setup(psi, 4.0, 0.0, precision=hpg.FP64)
    for _ in range(3):
        bt.op_apply_G(x, y)
    bt.set_kernel_timing("apply_G")
    for _ in range(args.probe_launches):
        bt.op_apply_G(x, y)
    nl, ms = bt.kernel_time("apply_G")
    bt.set_kernel_timing(None)
    alg = nb * 8 * (2 * mesh.n_u + 2 * mesh.n_psi + mesh.n_cells * mesh.q ** 2)
    t = ms / nl * 1e-3
    out = {"workload": "apply_G of %d requests of 2-D 32x32 cells, p=2, FP64, one launch" % nb,
           "algorithmic_bytes": alg, "apply_us": t * 1e6, "achieved_GBs": alg / t / 1e9,
           "frac": alg / t / 1e9 / HBM_PEAK_GBS, "launches": nl}
    del bt, x, y, psi
    torch.cuda.empty_cache()
    return out


def batch_bench(args, torch, hpg, W):
    """Batched solves of a request stream: args.batch_requests requests of the
    headline mesh (32 x 32 cells, p = 6, paraboloid obstacle), request i with
    the sine forcing of seed i, through args.batch_n slots of one
    hpg_batch_solve (a slot whose request finishes takes the next one), FP64
    and mixed; request 0's result against the single-problem path."""
    nb = args.batch_n
    nreq = args.batch_requests if args.batch_requests > 0 else 3 * nb
    mesh = hpg.Mesh(2, [args.m, args.m], args.p)
    x = mesh.quadrature_points()
    fs = np.stack([W.sine_forcing(i)[0](x) for i in range(nreq)])
    ps = np.stack([W.paraboloid_phi(x)] * nreq)
    n_dof = mesh.n_u + mesh.n_psi
    bt = hpg.Batch(mesh, nb)
    bt.set_data(fs, ps)
    out = {"workload": "stream of %d requests of the 2-D %dx%d p=%d obstacle problem (sine forcing "
                       "seeds 0..%d) through %d slots of one batched solve"
                       % (nreq, args.m, args.m, args.p, nreq - 1, nb),
           "requests": nreq, "slots": nb,
           "latency_note": "per-request service time, from taking a slot to finishing"}
    ref = {}
    for prec in ("fp64", "mixed"):
        kw = dict(precision=hpg.FP64 if prec == "fp64" else hpg.MIXED)
        if prec == "mixed":
            kw.update(newton_tol=1e-10, krylov_rtol=1e-6)
        opts = hpg.default_opts(**kw)
        t0 = time.perf_counter()
        u, psi, _, st = bt.solve(opts)
        sec = time.perf_counter() - t0
        kry = sum(s_.krylov_iters for s_ in st)
        lat = [s_.seconds for s_ in st]
        ent = {"seconds": sec, "solves_per_s": nreq / sec, "dof_krylov_per_s": n_dof * kry / sec,
               "converged": int(sum(s_.status == 0 for s_ in st)),
               "krylov_per_request": kry / nreq,
               "krylov_per_request_min_max": [min(s_.krylov_iters for s_ in st),
                                              max(s_.krylov_iters for s_ in st)],
               "newton_per_request": sum(s_.newton_iters for s_ in st) / nreq,
               "p50_service_s": float(np.percentile(lat, 50)),
               "p99_service_s": float(np.percentile(lat, 99))}
        ref[prec] = u
        out["path_" + prec] = ent
        print("[bench] batch stream of %d through %d slots, %s: %.2f s, %.2f solves/s"
              % (nreq, nb, prec, sec, nreq / sec), file=sys.stderr, flush=True)
    out["speedup_mixed_vs_fp64"] = out["path_mixed"]["solves_per_s"] / out["path_fp64"]["solves_per_s"]
    # request 0 through the single-problem path, and mixed against FP64
    prob = hpg.Problem(mesh, device=0)
    prob.set_forcing(fs[0])
    prob.set_obstacle(ps[0])
    u0, _, _, _ = prob.solve(hpg.default_opts())
    du = ref["fp64"][0] - u0
    out["request0_max_rel_vs_single_fp64"] = float(np.max(np.abs(du)) / np.max(np.abs(u0)))
    dm = ref["mixed"] - ref["fp64"]
    out["mixed_max_rel_vs_fp64"] = float(np.max(np.abs(dm)) / np.max(np.abs(ref["fp64"])))
    del bt, prob
    torch.cuda.empty_cache()
    return out


def bench_3d(args, torch, hpg, W):
    """3-D unit cube, 16^3 cells: the p = 5 obstacle problem (f = 50,
    phi = 0.05 + 0.2 |x - c|^2, alpha_k = 2^k) in FP64 and mixed, and with
    --3d-gradient the p = 4 gradient-constraint problem (|grad u| <= 0.3,
    the paper's gradient step sizes) in mixed precision.  One solve each,
    after an untimed warm-up; feasibility and complementarity diagnostics of
    each result."""
    out = {}
    cases = [("obstacle_p5", hpg.OBSTACLE, 5, W.w3d(), {})]
    if args.gradient3d:
        cases.append(("gradient_p4", hpg.GRADIENT, 4, W.w3d_gradient(),
                      dict(alpha0=2.0 ** -7, alpha_factor=2.0 ** 0.5, alpha_max=4.0,
                           fixed_prox_steps=20, max_newton=200, stall_tol=1e-8,
                           max_krylov=20000)))
    for name, kind, p, (f, phi), extra in cases:
        mesh = hpg.Mesh(3, [16, 16, 16], p, constraint=kind)
        x = mesh.quadrature_points()
        prob = hpg.Problem(mesh, device=0)
        prob.set_forcing(f(x))
        prob.set_obstacle(phi(x))
        n_dof = mesh.n_u + mesh.n_psi
        d_u = torch.zeros(mesh.n_u, dtype=torch.float64, device="cuda")
        d_psi = torch.zeros(mesh.n_psi, dtype=torch.float64, device="cuda")
        d_u64 = torch.zeros_like(d_u)
        ent = {"n_u": mesh.n_u, "n_psi": mesh.n_psi}
        precs = ("fp64", "mixed") if kind == hpg.OBSTACLE else ("mixed",)
        for prec in precs:
            kw = dict(extra)
            kw["precision"] = hpg.FP64 if prec == "fp64" else hpg.MIXED
            if prec == "mixed":
                kw.update(newton_tol=1e-10, krylov_rtol=1e-6)
            opts = hpg.default_opts(**kw)
            if kind == hpg.OBSTACLE:
                prob.solve_device(d_u, d_psi, opts)   # warm-up (tables, graphs)
            r = run_solves(prob, d_u, d_psi, opts, 1, torch, check=False)
            st = r["last"]
            e = {"seconds": r["seconds"], "status": st.status,
                 "dof_krylov_per_s": n_dof * r["krylov"] / r["seconds"],
                 "krylov": r["krylov"], "newton": r["newton"], "prox": r["prox"],
                 "complementarity_rel": st.complementarity_rel,
                 "max_violation": st.max_violation, "fp64_fallbacks": st.fp64_fallbacks}
            if prec == "fp64":
                d_u64.copy_(d_u)
            elif "fp64" in precs:
                diff, nrm = prob.l2_diff(d_u, d_u64)
                e["rel_l2_vs_fp64"] = diff / nrm
            ent["path_" + prec] = e
            print("[bench] 3-D 16^3 %s %s: %.2f s, status %d, krylov %d, newton %d"
                  % (name, prec, r["seconds"], st.status, r["krylov"], r["newton"]),
                  file=sys.stderr, flush=True)
        out[name] = ent
        del prob
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    global SERVE_KRYLOV_CHUNK
    SERVE_KRYLOV_CHUNK = args.serve_chunk
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this hpG build is single-GPU "
              "(no collectives); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_13733_amd import hpg
    import workloads as W

    torch.cuda.set_device(0)
    if args.counters:
        counters_run(args, torch, hpg, W)
        return
    if args.hp_counters:
        hp_counters_run(args, torch, hpg, W)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_bench(args, torch, hpg, W)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args, hpg, W)}), flush=True)
        return
    if args.hp_only:
        print(json.dumps({"hp_dip_64x64": hp_bench(args, torch, hpg, W)}), flush=True)
        return
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

    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precs:
        opts = hpg.default_opts(precision=hpg.FP64 if prec == "fp64" else hpg.MIXED)
        if prec == "mixed":
            opts.newton_tol = 1e-10
            opts.krylov_rtol = 1e-6
        for _ in range(args.warmup):
            prob.solve_device(d_u, d_psi, opts)
        r = run_solves(prob, d_u, d_psi, opts, args.steps, torch)
        if prec == "fp64":
            d_u64.copy_(d_u)
        elif "fp64" in precs:
            diff, nrm = prob.l2_diff(d_u, d_u64)
            r["rel_l2_vs_fp64"] = diff / nrm
        r["opts"] = opts
        results[prec] = r
        print("[bench] %s: %d solves in %.3f s, krylov %d, newton %d, prox %d"
              % (prec, args.steps, r["seconds"], r["krylov"], r["newton"], r["prox"]),
              file=sys.stderr, flush=True)

    # headline: the faster path whose solution meets rel-L2 1e-8 (vs FP64)
    best = precs[0]
    if "mixed" in results and "fp64" in results:
        if results["mixed"].get("rel_l2_vs_fp64", 1.0) <= 1e-8 and \
                results["mixed"]["seconds"] < results["fp64"]["seconds"]:
            best = "mixed"
    rb = results[best]
    # timed region 2: per-group kernel durations of the headline path
    rt = run_solves(prob, d_u, d_psi, rb["opts"], args.steps, torch, group="all")
    print("[bench] kernel timing pass (%s): %.3f s" % (best, rt["seconds"]), file=sys.stderr,
          flush=True)
    b = 8 if best == "fp64" else 4
    work = group_work(mesh, b)
    groups = {}
    for g, (nl, ms) in rt["ktime"].items():
        if nl == 0:
            continue
        ent = {"launches": nl, "total_ms": ms, "avg_us": 1e3 * ms / nl}
        if g in work:
            kind, amount = work[g]
            if kind == "hbm":
                ent["achieved_GBs"] = amount / (ms / nl * 1e-3) / 1e9
            else:
                ent["achieved_TFLOPs"] = amount / (ms / nl * 1e-3) / 1e12
        groups[g] = ent
    dom = max((g for g in groups if g in work), key=lambda g: groups[g]["total_ms"])
    kind, amount = work[dom]
    avg_s = groups[dom]["avg_us"] * 1e-6
    if kind == "hbm":
        ach = amount / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": amount}
    else:
        ach = amount / avg_s / 1e12
        pk = MFMA_PEAK_TFLOPS[best]
        roof = {"bound": "mfma", "kernel": dom, "achieved": ach, "peak": pk, "unit": "TFLOP/s",
                "frac": ach / pk, "traffic": None, "flops_per_launch": amount}
    roof["avg_launch_us"] = groups[dom]["avg_us"]
    roof["launches"] = groups[dom]["launches"]
    roof["traffic"] = measured_traffic(dom, args.m, args.p, best)

    def summary(r):
        return dict(dof_krylov_per_s=n_dof * r["krylov"] / r["seconds"],
                    solves_per_s=args.steps / r["seconds"],
                    ms_per_solve=1e3 * r["seconds"] / args.steps,
                    p50_ms=1e3 * float(np.percentile(r["lat"], 50)),
                    p99_ms=1e3 * float(np.percentile(r["lat"], 99)),
                    krylov_per_solve=r["krylov"] / args.steps,
                    newton_per_solve=r["newton"] / args.steps,
                    prox_per_solve=r["prox"] / args.steps)

    sb = summary(rb)
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
                               "paraboloid obstacle, alpha_k=2^k, tol 1e-10, one full solve per step"
                               % (args.m, args.m, args.p, args.seed),
                   "n_dof": n_dof, "n_u": mesh.n_u, "n_psi": mesh.n_psi, "path": best},
        "solves_per_s": sb["solves_per_s"],
        "p50_ms": sb["p50_ms"],
        "p99_ms": sb["p99_ms"],
        "krylov_per_solve": sb["krylov_per_solve"],
        "newton_per_solve": sb["newton_per_solve"],
        "prox_per_solve": sb["prox_per_solve"],
        "roofline": roof,
        "kernel_groups": groups,
    }
    for prec, r in results.items():
        s = summary(r)
        if "rel_l2_vs_fp64" in r:
            s["rel_l2_vs_fp64"] = r["rel_l2_vs_fp64"]
        out["path_" + prec] = s
    # the headline path again with the optional extension of full Newton steps
    # (not the paper's line search, which only backtracks; same subproblem
    # solutions): reported beside it, never as the headline
    if "mixed" in results:
        opts = results["mixed"]["opts"]
        opts.step_extension = 1
        prob.solve_device(d_u, d_psi, opts)
        r = run_solves(prob, d_u, d_psi, opts, args.steps, torch)
        s = summary(r)
        if "fp64" in results:
            diff, nrm = prob.l2_diff(d_u, d_u64)
            s["rel_l2_vs_fp64"] = diff / nrm
        out["path_mixed_step_extension"] = s
        print("[bench] mixed with step extension: %d solves in %.3f s, newton %d"
              % (args.steps, r["seconds"], r["newton"]), file=sys.stderr, flush=True)
    if not args.no_probe:
        del prob
        torch.cuda.empty_cache()
        cp = copy_bandwidth(torch)
        out["copy_bandwidth"] = cp
        print("[bench] 1 GiB device copy: %.0f GB/s" % cp["GBs"], file=sys.stderr, flush=True)
        for name in [s_.strip() for s_ in args.probes.split(",") if s_.strip()]:
            dim, m, p = PROBES[name]
            ent = apply_probe(args, torch, hpg, dim, m, p, cp["GBs"])
            out["apply_G_probe" if name == "R1" else "apply_G_probe_" + name] = ent
            print("[bench] apply_G probe %s: %.1f us, %.0f GB/s (%.1f %% of 8 TB/s, %.1f %% of "
                  "the copy)" % (name, ent["apply_us"], ent["achieved_GBs"], 100 * ent["frac"],
                                 100 * ent["frac_of_copy"]), file=sys.stderr, flush=True)
    if not args.no_batch:
        out["apply_G_probe_B1"] = batch_probe(args, torch, hpg)
        print("[bench] apply_G probe B1: %.1f us, %.0f GB/s" % (out["apply_G_probe_B1"]["apply_us"],
                                                               out["apply_G_probe_B1"]["achieved_GBs"]),
              file=sys.stderr, flush=True)
        out["batch"] = batch_bench(args, torch, hpg, W)
    if not args.no_3d:
        out["solve_3d"] = bench_3d(args, torch, hpg, W)
    if not args.no_hp:
        out["hp_dip_64x64"] = hp_bench(args, torch, hpg, W)
    if not args.no_serving:
        out["serving"] = serving_bench(args, hpg, W)
        sv = out["serving"]
        print("[bench] serving: fp64 x1 %.2f solves/s, mixed x%d %.2f solves/s, poisson p50 "
              "%.2f s p99 %.2f s" % (sv["fp64_sequential"]["solves_per_s"], sv["slots"],
                                    sv["mixed_batched"]["solves_per_s"],
                                    sv["mixed_poisson"]["p50_latency_s"],
                                    sv["mixed_poisson"]["p99_latency_s"]),
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, int(round(results[precs[0]]["newton"] / args.steps)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
