"""hpg_op_residual_noalloc (the residual for callers that cannot allocate)
against hpg_op_residual: the same R bit for bit and the squared norms of its
two parts, on two calls in a row with the second on a smaller problem, on the
fused tiled path, the generic and gradient paths, a 3-D mesh and a mesh with
one degree per cell; and the size limit of its fixed scratch array."""
import numpy as np
import pytest

import workloads as W

from gpu_common import build_pair, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda").contiguous()


def _hpg():
    from paper_2412_13733_amd import hpg
    return hpg


def _problem(case):
    hpg = _hpg()
    from oracle import mesh as OM
    if case == "hp":
        deg = np.random.default_rng(11).integers(2, 9, 30)
        mesh = hpg.Mesh(2, [6, 5], 0, degree=deg)
        x = mesh.quadrature_points()
        prob = hpg.Problem(mesh)
        f, phi = W.w2d(0)
        prob.set_forcing(f(x))
        prob.set_obstacle(phi(x))
        return mesh, prob
    dim, m, p, kind = case
    data = W.w1d() if dim == 1 else (W.w2d(0) if dim == 2 else W.w3d())
    if kind == "gradient":
        data = (data[0], W.const(0.3))
    mesh, prob, _ = build_pair(dim, m, p, data, kind=OM.GRADIENT if kind == "gradient" else OM.OBSTACLE)
    return mesh, prob


def _check(case, seed):
    mesh, prob = _problem(case)
    rng = np.random.default_rng(seed)
    u = _dev(0.1 * rng.standard_normal(mesh.n_u))
    psi = _dev(rng.standard_normal(mesh.n_psi))
    psi_prev = _dev(rng.standard_normal(mesh.n_psi))
    n = mesh.n_u + mesh.n_psi
    R1 = torch.zeros(n, dtype=torch.float64, device="cuda")
    R2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    prob.op_residual(u, psi, psi_prev, 8.0, R1)
    nu2, np2 = prob.op_residual_noalloc(u, psi, psi_prev, 8.0, R2)
    a, b = R1.cpu().numpy(), R2.cpu().numpy()
    assert np.array_equal(a, b)
    ru, rp = a[:mesh.n_u], a[mesh.n_u:]
    log("  case", case, "norms", nu2, np2)
    assert abs(nu2 - ru @ ru) <= 1e-12 * (ru @ ru)
    assert abs(np2 - rp @ rp) <= 1e-12 * (rp @ rp)


@pytest.mark.parametrize("first,second", [
    ((2, 32, 6, "obstacle"), (2, 5, 6, "obstacle")),
    ((2, 9, 3, "gradient"), (1, 16, 4, "obstacle")),
    ((3, 6, 5, "obstacle"), (3, 3, 2, "obstacle")),
    ("hp", (2, 4, 13, "obstacle")),
])
def test_noalloc_residual_matches_residual_twice(first, second):
    log("noalloc residual", first, "then", second)
    _check(first, 1)
    _check(second, 2)


def test_noalloc_residual_rejects_meshes_beyond_its_scratch():
    hpg = _hpg()
    mesh = hpg.Mesh(2, [150, 150], 0, degree=np.full(150 * 150, 6))   # 1.1e6 local values
    prob = hpg.Problem(mesh)
    x = mesh.quadrature_points()
    prob.set_forcing(np.ones(mesh.n_qp))
    prob.set_obstacle(np.ones(mesh.n_qp))
    n = mesh.n_u + mesh.n_psi
    R = torch.zeros(n, dtype=torch.float64, device="cuda")
    u = torch.zeros(mesh.n_u, dtype=torch.float64, device="cuda")
    p = torch.zeros(mesh.n_psi, dtype=torch.float64, device="cuda")
    with pytest.raises(hpg.HpgError) as e:
        prob.op_residual_noalloc(u, p, p, 2.0, R)
    assert e.value.status == hpg.ERR_INVALID_ARG
