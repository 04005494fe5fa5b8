"""Oracle check of a serving-stream run (test infrastructure, not collected by
pytest): the GPU results that ``bench.py --serving-only --serve-save DIR``
saved for a stratified sample of the stream (workloads.stratified_sample: the
four smallest meshes of each constraint/obstacle kind and degree band) against
the oracle's solve of the same request with the same options (the serving
requests' options of bench.request_opts: obstacle alpha_k = 2^k to the 1e-10
proximal tolerance; gradient the paper's schedule over 20 steps; a Newton stall
accepted at 1e-8; up to 200 Newton steps).

    python tests/check_serving_stream.py DIR [OUT.md]

Prints one line per request and path; with OUT.md writes the table there."""
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


def main():
    d = sys.argv[1]
    out_md = sys.argv[2] if len(sys.argv) > 2 else None
    files = sorted(glob.glob(os.path.join(d, "req*_*.npz")))
    by_idx = {}
    for fn in files:
        by_idx.setdefault(int(os.path.basename(fn)[3:6]), []).append(fn)
    jobs = sorted(by_idx.items(), key=lambda kv: -json.loads(str(np.load(kv[1][0])["request"]))["n"])
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        rows = [r for rs in pool.imap_unordered(check, jobs) for r in rs]
    rows.sort(key=lambda r: (r["index"], r["path"]))
    lines = ["| request | stratum | n | p | path | GPU status | GPU / oracle prox steps | "
             "FP64 fallbacks | rel L2 vs oracle |", "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        print("[check] request %3d %-28s n %2d p %2d %-5s status %d prox %d/%d rel L2 %.2e "
              "(oracle %.0f s)" % (r["index"], r["stratum"], r["n"], r["p"], r["path"], r["status"],
                                  r["gpu_prox"], r["oracle_prox"], r["rel_l2"], r["oracle_s"]),
              flush=True)
        lines.append("| %d | %s | %d | %d | %s | %d | %d / %d | %d | %.2e |"
                     % (r["index"], r["stratum"], r["n"], r["p"], r["path"], r["status"],
                        r["gpu_prox"], r["oracle_prox"], r["fallbacks"], r["rel_l2"]))
    for path in sorted({r["path"] for r in rows}):
        e = [r["rel_l2"] for r in rows if r["path"] == path]
        print("[check] %s: %d requests, max rel L2 %.2e, median %.2e" % (path, len(e), max(e),
                                                                           float(np.median(e))))
        lines.append("")
        lines.append("%s: %d requests, max rel L2 %.2e, median %.2e" % (path, len(e), max(e),
                                                                       float(np.median(e))))
    if out_md:
        with open(out_md, "w") as fh:
            fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
