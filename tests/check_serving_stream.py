"""Oracle check of a serving-stream run (test infrastructure, not collected by
pytest): the GPU results that ``bench.py --serving-only --serve-save DIR``
saved for a stratified sample of the stream (workloads.stratified_sample: the
four smallest meshes of each constraint/obstacle kind and degree band) against
the oracle's solve of the same request with the same options (the serving
requests' options of bench.request_opts: obstacle alpha_k = 2^k to the 1e-10
proximal tolerance; gradient the paper's schedule over 20 steps; a Newton stall
accepted at 1e-8; up to 200 Newton steps).

    python tests/check_serving_stream.py DIR [OUT.md [MAX_DOF]]

Prints one line per request and path as the oracle finishes it (smallest
first); with OUT.md keeps the table there up to date; requests with more than
MAX_DOF unknowns (n_u + n_psi) are listed as not checked."""
import glob
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

from oracle import assemble, lvpp, mesh as OM  # noqa: E402
import workloads as W  # noqa: E402


def oracle_opts(req):
    kw = dict(newton_tol=1e-12, max_newton=200, stall_tol=1e-8)
    if req["kind"] == "gradient":
        kw.update(alpha0=2.0 ** -7, alpha_factor=2.0 ** 0.5, alpha_max=4.0, fixed_steps=20)
    return lvpp.Options(**kw)


def check(idx_files):
    idx, files = idx_files
    req = json.loads(str(np.load(files[0])["request"]))
    kind = OM.GRADIENT if req["kind"] == "gradient" else OM.OBSTACLE
    om = OM.uniform_mesh(2, req["n"], req["p"], kind)
    xo = om.quadrature_points()
    f, phi = W.request_data(req)
    t0 = time.time()
    sysm = assemble.System(om, f(xo), phi(xo))
    ro = lvpp.solve(sysm, oracle_opts(req))
    sec = time.time() - t0
    rows = []
    for fn in files:
        z = np.load(fn)
        st = json.loads(str(z["stats"]))
        u = z["u"]
        e = sysm.l2_norm_u(u - ro.u) / max(sysm.l2_norm_u(ro.u), 1e-300)
        path = os.path.basename(fn).split("_")[1].split(".")[0]
        rows.append(dict(index=idx, stratum="%s %s" % W.serving_strata(req), n=req["n"], p=req["p"],
                         path=path, status=st["status"], gpu_prox=st["prox_steps"],
                         oracle_prox=ro.prox_steps, oracle_converged=bool(ro.converged),
                         rel_l2=float(e), fallbacks=st["fp64_fallbacks"], oracle_s=sec))
    return rows


def _dofs(req):
    n, p = req["n"], req["p"]
    return (n * p - 1) ** 2 + n * n * (p - 1) ** 2 * (2 if req["kind"] == "gradient" else 1)


def _write(rows, out_md, skipped):
    lines = ["| request | stratum | n | p | path | GPU status | GPU / oracle prox steps | "
             "FP64 fallbacks | rel L2 vs oracle |", "|---|---|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: (r["index"], r["path"])):
        lines.append("| %d | %s | %d | %d | %s | %d | %d / %d | %d | %.2e |"
                     % (r["index"], r["stratum"], r["n"], r["p"], r["path"], r["status"],
                        r["gpu_prox"], r["oracle_prox"], r["fallbacks"], r["rel_l2"]))
    for path in sorted({r["path"] for r in rows}):
        e = [r["rel_l2"] for r in rows if r["path"] == path]
        lines.append("")
        lines.append("%s: %d requests, max rel L2 %.2e, median %.2e" % (path, len(e), max(e),
                                                                       float(np.median(e))))
    if skipped:
        lines.append("")
        lines.append("not checked (beyond the oracle's DOF budget): " + ", ".join(
            "%d (n %d, p %d)" % s_ for s_ in skipped))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    d = sys.argv[1]
    out_md = sys.argv[2] if len(sys.argv) > 2 else None
    max_dof = int(sys.argv[3]) if len(sys.argv) > 3 else 10 ** 9
    files = sorted(glob.glob(os.path.join(d, "req*_*.npz")))
    by_idx = {}
    for fn in files:
        by_idx.setdefault(int(os.path.basename(fn)[3:6]), []).append(fn)
    reqs = {i: json.loads(str(np.load(f[0])["request"])) for i, f in by_idx.items()}
    # smallest first, so that results accumulate early; the largest may be skipped
    jobs = sorted(by_idx.items(), key=lambda kv: _dofs(reqs[kv[0]]))
    skipped = [(i, reqs[i]["n"], reqs[i]["p"]) for i, _ in jobs if _dofs(reqs[i]) > max_dof]
    jobs = [j for j in jobs if _dofs(reqs[j[0]]) <= max_dof]
    rows = []
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        for rs in pool.imap_unordered(check, jobs):
            rows.extend(rs)
            for r in rs:
                print("[check] request %3d %-28s n %2d p %2d %-5s status %d prox %d/%d rel L2 %.2e "
                      "(oracle %.0f s)" % (r["index"], r["stratum"], r["n"], r["p"], r["path"],
                                          r["status"], r["gpu_prox"], r["oracle_prox"],
                                          r["rel_l2"], r["oracle_s"]), flush=True)
            if out_md:
                _write(rows, out_md, skipped)
    for path in sorted({r["path"] for r in rows}):
        e = [r["rel_l2"] for r in rows if r["path"] == path]
        print("[check] %s: %d requests, max rel L2 %.2e, median %.2e" % (path, len(e), max(e),
                                                                           float(np.median(e))))
    if skipped:
        print("[check] not checked:", skipped)


if __name__ == "__main__":
    main()
