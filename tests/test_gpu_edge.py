"""GPU edge cases against the oracle: single-cell meshes (no interior vertex:
u is bubbles only), gradient p = 1, the largest degrees of the tiled apply
(2-D p = 12, 3-D p = 7) and the first degree beyond it (generic kernels),
strongly graded
breakpoints (width ratio 1e3), Schur blocks too large for LDS (formed and
inverted in global memory, streamed by the preconditioner), zero inputs, and a
solve whose constraint never activates.  Tolerances as in test_gpu_parity."""
import numpy as np
import pytest

from oracle import lvpp, precond, mesh as OM
import workloads as W

from gpu_common import FP32_G, FP32_P, FP64_G, FP64_P, FP64_P_COND, FP64_RES, build_pair, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _data(dim):
    return W.w1d() if dim == 1 else (W.w2d(0) if dim == 2 else W.w3d())


GRADED = np.r_[0.0, np.cumsum(np.geomspace(1.0, 1000.0, 6))] / np.sum(np.geomspace(1.0, 1000.0, 6))

CASES = [
    (1, 1, 2, None, OM.OBSTACLE),
    (2, 1, 5, None, OM.OBSTACLE),
    (3, 1, 3, None, OM.OBSTACLE),
    (2, 2, 12, None, OM.OBSTACLE),    # largest tiled degree in 2-D
    (2, 2, 13, None, OM.OBSTACLE),    # generic kernels
    (3, 2, 7, None, OM.OBSTACLE),     # largest tiled degree in 3-D
    (3, 1, 8, None, OM.OBSTACLE),     # generic kernels in 3-D
    (2, 6, 2, [GRADED, W.uniform_breaks(3)], OM.OBSTACLE),
    (2, 6, 3, [GRADED, GRADED], OM.OBSTACLE),
    (1, 2, 1, None, OM.GRADIENT),     # p = 1: one interior vertex
    (2, 1, 2, None, OM.GRADIENT),
    (3, 1, 2, None, OM.GRADIENT),
]


@pytest.mark.parametrize("dim,m,p,breaks,kind", CASES)
def test_edge_operators(dim, m, p, breaks, kind):
    log("edge", dim, m, p, kind, "graded" if breaks is not None else "")
    data = _data(dim)
    if kind == OM.GRADIENT:
        data = (data[0], lambda x: 0.25 + 0.1 * np.sum(np.atleast_2d(x), axis=1))
    mesh, prob, sysm = build_pair(dim, m, p, data, breaks, kind=kind)
    rng = np.random.default_rng(31)
    psi = 0.6 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 4.5, 1e-3
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    for prec, dt, tol_g, tol_p in ((1, torch.float32, FP32_G, FP32_P), (0, torch.float64, FP64_G, FP64_P)):
        prob.op_setup(_dev(psi), alpha, beta, precision=prec)
        y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=dt, device="cuda")
        prob.op_apply_G(_dev(x, dt), y)
        yg = y.double().cpu().numpy()
        z = torch.zeros_like(y)
        prob.op_apply_prec(_dev(x, dt), z)
        zg = z.double().cpu().numpy()
        log("  prec", prec, "G", rel(yg[:mesh.n_u], yu), rel(yg[mesh.n_u:], yp),
            "P", rel(zg[:mesh.n_u], zu), rel(zg[mesh.n_u:], zp))
        assert rel(yg[:mesh.n_u], yu) < tol_g and rel(yg[mesh.n_u:], yp) < tol_g
        # FP64 psi-blocks of 3-D degree >= 7: the conditioning bar
        tol_pp = FP64_P_COND if prec == 0 and dim == 3 and p >= 7 else tol_p
        assert rel(zg[:mesh.n_u], zu) < tol_p and rel(zg[mesh.n_u:], zp) < tol_pp
    # zero in, zero out
    y.fill_(1.0)
    prob.op_apply_G(torch.zeros_like(y), y)
    assert float(y.abs().max()) == 0.0
    R = torch.zeros_like(y)
    u = 0.1 * rng.standard_normal(mesh.n_u)
    pp = 0.5 * rng.standard_normal(mesh.n_psi)
    prob.op_residual(_dev(u), _dev(psi), _dev(pp), alpha, R)
    Ru, Rp = sysm.residual(u, psi, pp, alpha)
    Rg = R.cpu().numpy()
    assert rel(Rg[:mesh.n_u], Ru) < FP64_RES and rel(Rg[mesh.n_u:], Rp) < FP64_RES


def test_edge_inactive_constraint_solve():
    # phi far above the unconstrained solution: the constraint never binds and
    # the solve reproduces the oracle (which here approaches the Poisson solution)
    from paper_2412_13733_amd import hpg
    f = lambda x: np.full(np.atleast_2d(x).shape[0], 1.0)
    phi = lambda x: np.full(np.atleast_2d(x).shape[0], 5.0)
    mesh, prob, sysm = build_pair(2, 4, 3, (f, phi))
    ro = lvpp.solve(sysm, lvpp.Options())
    assert ro.converged
    u, psi, lam, st = prob.solve(hpg.default_opts(fixed_prox_steps=ro.prox_steps), want_lambda=True)
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    log("inactive: gpu", st.as_dict(), "rel L2", eu)
    assert st.status == 0 and eu < 1e-10
    # no contact: the multiplier vanishes
    assert np.max(np.abs(lam - ro.lam)) < 1e-8


def test_edge_single_cell_solve():
    from paper_2412_13733_amd import hpg
    mesh, prob, sysm = build_pair(2, 1, 4, W.w2d(1))
    ro = lvpp.solve(sysm, lvpp.Options())
    assert ro.converged
    u, psi, lam, st = prob.solve(hpg.default_opts(fixed_prox_steps=ro.prox_steps))
    eu = sysm.l2_norm_u(u - ro.u) / max(sysm.l2_norm_u(ro.u), 1e-300)
    log("single cell: gpu", st.as_dict(), "rel L2", eu)
    assert st.status == 0 and eu < 1e-10
