"""Writes full-size oracle solutions used by the GPU parity tests:

* solve_2d_32x32_p6.npz: the 2-D unit square, 32 x 32 uniform cells, p = 6,
  sine forcing (seed 0) and paraboloid obstacle, alpha_k = 2^k, outer
  tolerance 1e-10, Newton tolerance 1e-12;
* solve_3d_16_p2.npz: the 3-D unit cube, 16^3 cells, p = 2, f = 50,
  phi = 0.05 + 0.2 |x - c|^2, same rules;
* solve_3d_4_p5.npz: the same 3-D data on 4^3 cells at p = 5;
* solve_3d_4_p3_gradient.npz: the 3-D gradient constraint |grad u| <= 0.3,
  f = 50, 4^3 cells, p = 3, with the step sizes of the paper's gradient
  example (alpha_1 = 2^-7, alpha_{k+1} = min(sqrt(2) alpha_k, 4), 20 steps).

Each file holds u, psi, lam (lambda_K of the last proximal step), the
proximal-step and Newton counts, the wall time of the oracle solve and of
its sparse LU factorisations and solves, and the host it ran on (nproc,
CPU model, memory).  The recipe calls only the oracle (assembled FP64 saddle
system, sparse LU per Newton step).

Run: python tests/golden/make_solve_goldens.py [2d|3d]
"""
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from oracle import assemble, lvpp, mesh as OM   # noqa: E402
import workloads as W   # noqa: E402


def host_info():
    model = platform.processor()
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
    return {"nproc": os.cpu_count() or 0, "cpu_model": model, "mem_bytes": mem}


GRADIENT_STEPS = dict(alpha0=2.0 ** -7, alpha_factor=2.0 ** 0.5, alpha_max=4.0, fixed_steps=20)

CASES = {
    "2d": ("solve_2d_32x32_p6.npz", 2, 32, 6, OM.OBSTACLE, lambda: W.w2d(0), {}),
    "3d": ("solve_3d_16_p2.npz", 3, 16, 2, OM.OBSTACLE, W.w3d, {}),
    "3d4p5": ("solve_3d_4_p5.npz", 3, 4, 5, OM.OBSTACLE, W.w3d, {}),
    "3d4p3g": ("solve_3d_4_p3_gradient.npz", 3, 4, 3, OM.GRADIENT, W.w3d_gradient,
               GRADIENT_STEPS),
}


def run(key):
    name, d, m, p, kind, data, opts = CASES[key]
    f, phi = data()
    mesh = OM.uniform_mesh(d, m, p, kind)
    x = mesh.quadrature_points()
    t0 = time.perf_counter()
    sysm = assemble.System(mesh, f(x), phi(x))
    t_asm = time.perf_counter() - t0
    res = lvpp.solve(sysm, lvpp.Options(**opts))
    info = host_info()
    print("%s: converged %s prox %d newton %d solve %.1f s (LU %.1f s) assembly %.1f s"
          % (name, res.converged, res.prox_steps, res.newton, res.seconds, res.lu_seconds, t_asm))
    np.savez_compressed(
        os.path.join(HERE, name), u=res.u, psi=res.psi, lam=res.lam,
        prox_steps=res.prox_steps, newton=res.newton, converged=res.converged,
        solve_seconds=res.seconds, lu_seconds=res.lu_seconds, assembly_seconds=t_asm,
        nproc=info["nproc"], cpu_model=np.array(info["cpu_model"]), mem_bytes=info["mem_bytes"])


if __name__ == "__main__":
    for k in (sys.argv[1:] or list(CASES)):
        run(k)
