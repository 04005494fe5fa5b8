"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds only data generators: the forcing f and the obstacle phi
of each workload as plain functions of x, meshes as breakpoint vectors, and
the serving stream's request draws.  It contains none of the method's
arithmetic (no basis, quadrature, assembly or solver).

Random draws use NumPy's PCG64 (``numpy.random.default_rng(seed)``).

Workloads (sizes as in the problem class of the paper's Sec. 6: tensor
domains, smooth data, p from 2 to 12, meshes up to 64^2 and 16^3):
* ``w1d``      1-D (0,1), 16 cells, p=4, f = 10, phi = 0.1 + 0.5 (x - 1/2)^2.
* ``w2d``      2-D 32x32, p=6, f = sum_{i,j<=4} c_ij sin(i pi x) sin(j pi y),
               c_ij ~ N(0,1) * 20/(i^2+j^2); phi = 0.05 + 0.3 |x - (1/2,1/2)|^2.
* ``w2d_dip``  2-D 64x64 data family: same f, phi = 0.2 - 0.15 exp(-20|x-x0|^2),
               x0 ~ U[0.3,0.7]^2.
* ``w3d``      3-D 16^3, p=5, f = 50, phi = 0.05 + 0.2 |x - (1/2,1/2,1/2)|^2;
               gradient variant |grad u| <= 0.3 at p=4.
* ``serving``  512 requests, Poisson arrivals at 40/s (seed 12345); request i
               uses seed 10000+i: n ~ U{8..64}, p ~ U{2..10}, 25 % gradient
               with phi ~ U[0.2, 0.5], else obstacle with the paraboloid or
               the Gaussian-dip phi (50/50).
"""
import numpy as np


def sine_forcing(seed, scale=20.0):
    """f(x, y) = sum_{i,j=1..4} c_ij sin(i pi x) sin(j pi y), c_ij ~ N(0,1) scale/(i^2+j^2).

    Draw order: standard_normal((4, 4)) row-major (i outer, j inner), then the
    caller may continue drawing from the same generator (returned)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((4, 4))
    ij = np.arange(1, 5)
    c = c * scale / (ij[:, None] ** 2 + ij[None, :] ** 2)

    def f(x):
        x = np.atleast_2d(x)
        sx = np.sin(np.pi * np.outer(x[:, 0], ij))      # (n, 4)
        sy = np.sin(np.pi * np.outer(x[:, 1], ij))
        return np.einsum("ni,ij,nj->n", sx, c, sy)

    return f, rng


def w1d():
    f = lambda x: np.full(np.atleast_2d(x).shape[0], 10.0)
    phi = lambda x: 0.1 + 0.5 * (np.atleast_2d(x)[:, 0] - 0.5) ** 2
    return f, phi


def paraboloid_phi(x):
    x = np.atleast_2d(x)
    return 0.05 + 0.3 * np.sum((x - 0.5) ** 2, axis=1)


def w2d(seed=0):
    f, _ = sine_forcing(seed)
    return f, paraboloid_phi


def w2d_dip(seed=0):
    f, rng = sine_forcing(seed)
    x0 = rng.uniform(0.3, 0.7, 2)

    def phi(x):
        x = np.atleast_2d(x)
        return 0.2 - 0.15 * np.exp(-20.0 * np.sum((x - x0) ** 2, axis=1))

    return f, phi


def w3d():
    f = lambda x: np.full(np.atleast_2d(x).shape[0], 50.0)
    phi = lambda x: 0.05 + 0.2 * np.sum((np.atleast_2d(x) - 0.5) ** 2, axis=1)
    return f, phi


def w3d_gradient():
    f = lambda x: np.full(np.atleast_2d(x).shape[0], 50.0)
    phi = lambda x: np.full(np.atleast_2d(x).shape[0], 0.3)
    return f, phi


def const(c):
    return lambda x: np.full(np.atleast_2d(x).shape[0], float(c))


def uniform_breaks(m):
    return np.linspace(0.0, 1.0, m + 1)


def serving_stream(n_req=512, rate=40.0, seed=12345):
    """Arrival times (s) and per-request descriptors for the serving workload."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_req):
        r = np.random.default_rng(10000 + i)
        n = int(r.integers(8, 65))
        p = int(r.integers(2, 11))
        gradient = bool(r.uniform() < 0.25)
        if gradient:
            phic = float(r.uniform(0.2, 0.5))
            reqs.append(dict(n=n, p=p, kind="gradient", seed=10000 + i, phi_const=phic))
        else:
            dip = bool(r.uniform() < 0.5)
            reqs.append(dict(n=n, p=p, kind="obstacle", seed=10000 + i,
                             phi="dip" if dip else "paraboloid"))
    return arrivals, reqs


def request_data(req):
    """(f, phi) callables of one serving request."""
    f, _ = sine_forcing(req["seed"])
    if req["kind"] == "gradient":
        return f, const(req["phi_const"])
    if req["phi"] == "dip":
        return w2d_dip(req["seed"])
    return f, paraboloid_phi


def serving_strata(req):
    """Stratum of a serving request: (constraint and obstacle kind, degree band)."""
    kind = req["kind"] if req["kind"] == "gradient" else "obstacle-" + req["phi"]
    band = "p2-4" if req["p"] <= 4 else ("p5-7" if req["p"] <= 7 else "p8-10")
    return kind, band


def stratified_sample(reqs, per_stratum=4):
    """Indices of the per_stratum smallest-mesh requests (ties: lower index) of
    each (kind, degree band) stratum of a serving stream, sorted."""
    groups = {}
    for i, r in enumerate(reqs):
        groups.setdefault(serving_strata(r), []).append(i)
    out = []
    for key in sorted(groups):
        idx = sorted(groups[key], key=lambda i: (reqs[i]["n"], i))
        out.extend(idx[:per_stratum])
    return sorted(out)
