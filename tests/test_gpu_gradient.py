"""GPU parity of the gradient-constraint path (|grad u| <= phi, eq.
(pG:gradient)) against the oracle: the Newton operator G, the preconditioner
diag(alpha A, D_psi + beta E_beta), the residual and whole solves, element by
element on seeded inputs.  The cases cover 1-D, 2-D (uniform and non-uniform
breaks) and 3-D, and psi blocks small enough for LDS as well as blocks that
are formed and inverted in HBM (2-D p = 8: block 128 x 128; 3-D p = 3: the
preconditioner streams 81 x 81 blocks).  Tolerances as for the obstacle path:
the operator bars of gpu_common (max-norm relative), FP64 solves 1e-10
relative L2."""
import numpy as np
import pytest

from oracle import lvpp, precond, mesh as OM
import workloads as W

from gpu_common import FP32_G, FP32_P, FP64_G, FP64_P, FP64_RES, build_pair, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _data(dim):
    """f from the sine family (constant in 1-D), a positive varying phi."""
    if dim == 1:
        f = lambda x: np.full(np.atleast_2d(x).shape[0], 10.0)
    else:
        f, _ = W.sine_forcing(3)
    phi = lambda x: 0.2 + 0.3 * np.sum((np.atleast_2d(x) - 0.4) ** 2, axis=1)
    return f, phi


OP_CASES = [
    (1, 12, 3, None),
    (1, 9, 1, None),
    (2, 5, 3, None),
    (2, 4, 4, [np.array([0, .15, .5, .8, 1.0]), np.array([0, .3, .45, .7, 1.0])]),
    (2, 2, 8, None),     # psi blocks of 128: formed and inverted in HBM
    (3, 3, 2, None),
    (3, 2, 3, None),     # psi blocks of 81: streamed preconditioner
]


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _pair(dim, m, p, breaks):
    return build_pair(dim, m, p, _data(dim), breaks, kind=OM.GRADIENT)


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
@pytest.mark.parametrize("beta", [0.0, 1e-3])
def test_gradient_apply_G_fp64(dim, m, p, breaks, beta):
    log("gradient apply_G fp64", dim, m, p, beta)
    mesh, prob, sysm = _pair(dim, m, p, breaks)
    rng = np.random.default_rng(17)
    psi = 0.8 * rng.standard_normal(mesh.n_psi)
    alpha = 3.1
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, beta, precision=0)
    y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_apply_G(_dev(x), y)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    yg = y.cpu().numpy()
    log("  rel", rel(yg[:mesh.n_u], yu), rel(yg[mesh.n_u:], yp))
    assert rel(yg[:mesh.n_u], yu) < FP64_G
    assert rel(yg[mesh.n_u:], yp) < FP64_G


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
def test_gradient_apply_prec_fp64(dim, m, p, breaks):
    log("gradient apply_prec fp64", dim, m, p)
    mesh, prob, sysm = _pair(dim, m, p, breaks)
    rng = np.random.default_rng(21)
    psi = 0.6 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 5.0, 1e-3
    r = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, beta, precision=0)
    z = torch.zeros_like(_dev(r))
    prob.op_apply_prec(_dev(r), z)
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, r[:mesh.n_u], r[mesh.n_u:])
    zg = z.cpu().numpy()
    log("  rel", rel(zg[:mesh.n_u], zu), rel(zg[mesh.n_u:], zp))
    assert rel(zg[:mesh.n_u], zu) < FP64_P
    assert rel(zg[mesh.n_u:], zp) < FP64_P


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
def test_gradient_operators_fp32(dim, m, p, breaks):
    log("gradient operators fp32", dim, m, p)
    mesh, prob, sysm = _pair(dim, m, p, breaks)
    rng = np.random.default_rng(23)
    psi = 0.5 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 2.0, 1e-3
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, beta, precision=1)
    y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float32, device="cuda")
    prob.op_apply_G(_dev(x, torch.float32), y)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    yg = y.double().cpu().numpy()
    assert rel(yg[:mesh.n_u], yu) < FP32_G
    assert rel(yg[mesh.n_u:], yp) < FP32_G
    z = torch.zeros_like(y)
    prob.op_apply_prec(_dev(x, torch.float32), z)
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    zg = z.double().cpu().numpy()
    log("  prec rel", rel(zg[:mesh.n_u], zu), rel(zg[mesh.n_u:], zp))
    assert rel(zg[:mesh.n_u], zu) < FP32_P
    assert rel(zg[mesh.n_u:], zp) < FP32_P


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
def test_gradient_residual_fp64(dim, m, p, breaks):
    log("gradient residual", dim, m, p)
    mesh, prob, sysm = _pair(dim, m, p, breaks)
    rng = np.random.default_rng(29)
    u = 0.1 * rng.standard_normal(mesh.n_u)
    psi = 0.9 * rng.standard_normal(mesh.n_psi)
    psi_prev = 0.9 * rng.standard_normal(mesh.n_psi)
    alpha = 6.0
    R = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_residual(_dev(u), _dev(psi), _dev(psi_prev), alpha, R)
    Ru, Rp = sysm.residual(u, psi, psi_prev, alpha)
    Rg = R.cpu().numpy()
    assert rel(Rg[:mesh.n_u], Ru) < FP64_RES
    assert rel(Rg[mesh.n_u:], Rp) < FP64_RES


SOLVE_CASES = [(1, 16, 2), (1, 10, 3), (2, 4, 2), (2, 3, 3), (3, 2, 2)]


@pytest.mark.parametrize("dim,m,p", SOLVE_CASES)
def test_gradient_solve_matches_oracle_fp64(dim, m, p):
    from paper_2412_13733_amd import hpg
    log("gradient solve fp64", dim, m, p)
    mesh, prob, sysm = _pair(dim, m, p, None)
    K = 6
    ro = lvpp.solve(sysm, lvpp.Options(fixed_steps=K, max_newton=200))
    assert ro.converged
    u, psi, lam, st = prob.solve(hpg.default_opts(fixed_prox_steps=K, max_newton=200),
                                 want_lambda=True)
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    ep = np.linalg.norm(psi - ro.psi) / np.linalg.norm(ro.psi)
    log("  oracle newton", ro.newton, "| gpu", st.as_dict(), "| rel L2 u", eu, "psi", ep)
    assert st.status == 0
    assert eu < 1e-10
    assert ep < 1e-9


@pytest.mark.parametrize("dim,m,p", SOLVE_CASES[::2])
def test_gradient_solve_mixed_precision(dim, m, p):
    from paper_2412_13733_amd import hpg
    log("gradient solve mixed", dim, m, p)
    mesh, prob, sysm = _pair(dim, m, p, None)
    K = 6
    ro = lvpp.solve(sysm, lvpp.Options(fixed_steps=K, max_newton=200))
    u, psi, lam, st = prob.solve(hpg.default_opts(fixed_prox_steps=K, max_newton=200,
                                                  precision=hpg.MIXED, newton_tol=1e-10,
                                                  krylov_rtol=1e-6))
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    log("  gpu", st.as_dict(), "rel L2 u", eu)
    assert st.status == 0
    assert eu < 1e-8
