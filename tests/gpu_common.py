"""Shared set-up for the GPU parity tests: builds the same discrete problem on
the HIP side (through the C ABI) and on the oracle side (its own quadrature
points, assembly and DOF map); only the input generators are shared."""
import sys

import numpy as np

from paper_2412_13733_amd import hpg
from oracle import assemble, mesh as OM

import workloads as W


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def build_pair(dim, m, p, data, breaks=None, kind=OM.OBSTACLE):
    f, phi = data
    if breaks is None:
        breaks = [W.uniform_breaks(m)] * dim
    mcells = [len(b) - 1 for b in breaks]
    mesh = hpg.Mesh(dim, mcells, p, breaks=breaks,
                    constraint=hpg.OBSTACLE if kind == OM.OBSTACLE else hpg.GRADIENT)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    om = OM.TensorMesh(breaks, p, kind)
    xo = om.quadrature_points()
    sysm = assemble.System(om, f(xo), phi(xo))
    return mesh, prob, sysm


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
