"""GPU parity: the HIP operators and solves against the oracle, element by
element, on seeded inputs.  Sizes span several thread blocks with ragged
tails; tolerances: the operator bars of gpu_common (max-norm relative, at
most ten times the worst observed error), FP64 solves 1e-10 relative L2 (the
bar stated for the FP64 path)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import lvpp, precond, mesh as OM
import workloads as W

from gpu_common import FP32_G, FP32_P, FP64_G, FP64_P, FP64_RES, build_pair, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OP_CASES = [
    (1, 16, 4, None),
    (1, 37, 2, None),
    (2, 5, 6, None),
    (2, 9, 3, None),
    (2, 4, 5, [np.array([0, .1, .45, .7, 1.0]), np.array([0, .3, .55, .9, 1.0])]),
    (3, 3, 5, None),
    (3, 5, 2, None),
    # several tiles with a ragged tail on the dense low-degree path
    (1, 40, 3, None),
    (2, 37, 2, None),
    (2, 19, 3, None),
    (2, 21, 2, [np.sort(np.r_[0.0, np.random.default_rng(7).uniform(0.02, 0.98, 20), 1.0]),
                np.linspace(0.0, 1.0, 22) ** 1.3]),
    (3, 9, 2, None),
]


def _data(dim):
    return W.w1d() if dim == 1 else (W.w2d(0) if dim == 2 else W.w3d())


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
@pytest.mark.parametrize("beta", [0.0, 1e-3])
def test_apply_G_fp64(dim, m, p, breaks, beta):
    log("apply_G fp64", dim, m, p, beta)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim), breaks)
    rng = np.random.default_rng(7)
    psi = 0.7 * rng.standard_normal(mesh.n_psi)
    alpha = 3.7
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, beta, precision=0)
    y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_apply_G(_dev(x), y)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    yg = y.cpu().numpy()
    assert rel(yg[:mesh.n_u], yu) < FP64_G
    assert rel(yg[mesh.n_u:], yp) < FP64_G


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
def test_apply_prec_fp64(dim, m, p, breaks):
    log("apply_prec fp64", dim, m, p)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim), breaks)
    rng = np.random.default_rng(11)
    psi = 0.5 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 5.0, 1e-4
    r = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, beta, precision=0)
    z = torch.zeros_like(_dev(r))
    prob.op_apply_prec(_dev(r), z)
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, r[:mesh.n_u], r[mesh.n_u:])
    zg = z.cpu().numpy()
    assert rel(zg[:mesh.n_u], zu) < FP64_P
    assert rel(zg[mesh.n_u:], zp) < FP64_P


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES[::2])
def test_operators_fp32(dim, m, p, breaks):
    log("operators fp32", dim, m, p)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim), breaks)
    rng = np.random.default_rng(3)
    psi = 0.5 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 2.0, 0.0
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
    assert rel(zg[:mesh.n_u], zu) < FP32_P
    assert rel(zg[mesh.n_u:], zp) < FP32_P


@pytest.mark.parametrize("dim,m,p,breaks", OP_CASES)
def test_residual_fp64(dim, m, p, breaks):
    log("residual", dim, m, p)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim), breaks)
    rng = np.random.default_rng(5)
    u = 0.1 * rng.standard_normal(mesh.n_u)
    psi = 0.8 * rng.standard_normal(mesh.n_psi)
    psi_prev = 0.8 * rng.standard_normal(mesh.n_psi)
    alpha = 8.0
    R = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_residual(_dev(u), _dev(psi), _dev(psi_prev), alpha, R)
    Ru, Rp = sysm.residual(u, psi, psi_prev, alpha)
    Rg = R.cpu().numpy()
    assert rel(Rg[:mesh.n_u], Ru) < FP64_RES
    assert rel(Rg[mesh.n_u:], Rp) < FP64_RES


@pytest.mark.parametrize("dim,m,p", [(1, 16, 4), (2, 6, 4), (3, 3, 3)])
def test_minres_solves_newton_system(dim, m, p):
    log("minres", dim, m, p)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim))
    rng = np.random.default_rng(9)
    psi = 0.5 * rng.standard_normal(mesh.n_psi)
    alpha = 4.0
    b = rng.standard_normal(mesh.n_u + mesh.n_psi)
    prob.op_setup(_dev(psi), alpha, 0.0, precision=0)
    x = torch.zeros_like(_dev(b))
    its = prob.op_minres(_dev(b), x, 1e-12, 3000)
    G = sysm.jacobian(psi, alpha, 0.0)
    xr = spla.spsolve(G, b)
    xg = x.cpu().numpy()
    assert 0 < its < 3000
    assert np.linalg.norm(xg - xr) <= 1e-8 * np.linalg.norm(xr)


SOLVE_CASES = [
    (1, 16, 4, "w1d"),
    (1, 16, 2, "w1d"),
    (2, 6, 4, "w2d"),
    (2, 5, 2, "w2d"),
    (3, 3, 3, "w3d"),
]


@pytest.mark.parametrize("dim,m,p,which", SOLVE_CASES)
def test_full_solve_matches_oracle_fp64(dim, m, p, which):
    log("solve fp64", dim, m, p, which)
    data = {"w1d": W.w1d(), "w2d": W.w2d(0), "w3d": W.w3d()}[which]
    mesh, prob, sysm = build_pair(dim, m, p, data)
    ro = lvpp.solve(sysm, lvpp.Options())
    assert ro.converged
    opts = prob_opts(fixed=ro.prox_steps)
    u, psi, lam, st = prob.solve(opts, want_lambda=True)
    log("  oracle K", ro.prox_steps, "newton", ro.newton, "| gpu", st.as_dict())
    assert st.status == 0
    assert st.prox_steps == ro.prox_steps
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    ep = np.linalg.norm(psi - ro.psi) / max(np.linalg.norm(ro.psi), 1e-300)
    el = np.linalg.norm(lam - ro.lam) / max(np.linalg.norm(ro.lam), 1e-300)
    log("  rel L2 u", eu, "rel psi", ep, "rel lambda", el)
    assert eu < 1e-10
    assert ep < 1e-9
    assert el < 1e-8


def prob_opts(fixed=0, precision=0, **kw):
    from paper_2412_13733_amd import hpg
    return hpg.default_opts(fixed_prox_steps=fixed, precision=precision, **kw)


@pytest.mark.parametrize("dim,m,p,which", SOLVE_CASES)
def test_full_solve_mixed_precision(dim, m, p, which):
    # FP32 operator/preconditioner in MINRES, FP64 residual, exp and update:
    # the Newton loop refines the FP32 Krylov solutions to the FP64 answer
    log("solve mixed", dim, m, p, which)
    data = {"w1d": W.w1d(), "w2d": W.w2d(0), "w3d": W.w3d()}[which]
    mesh, prob, sysm = build_pair(dim, m, p, data)
    ro = lvpp.solve(sysm, lvpp.Options())
    opts = prob_opts(fixed=ro.prox_steps, precision=1, newton_tol=1e-10, krylov_rtol=1e-6)
    u, psi, lam, st = prob.solve(opts, want_lambda=True)
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    log("  gpu", st.as_dict(), "rel L2 u", eu)
    assert st.status == 0
    assert eu < 1e-8


@pytest.mark.parametrize("dim,m,p,which,precision", [(1, 16, 4, "w1d", 0), (2, 6, 4, "w2d", 0),
                                                     (2, 6, 4, "w2d", 1), (3, 3, 3, "w3d", 0)])
def test_step_extension_same_solution(dim, m, p, which, precision):
    # the optional extension of full Newton steps changes the Newton path, not
    # the subproblem solutions: the result still matches the oracle (whose
    # line search only backtracks)
    log("step extension", dim, m, p, which, "precision", precision)
    data = {"w1d": W.w1d(), "w2d": W.w2d(0), "w3d": W.w3d()}[which]
    mesh, prob, sysm = build_pair(dim, m, p, data)
    ro = lvpp.solve(sysm, lvpp.Options())
    kw = dict(newton_tol=1e-10, krylov_rtol=1e-6) if precision else {}
    opts = prob_opts(fixed=ro.prox_steps, precision=precision, step_extension=1, **kw)
    u, psi, lam, st = prob.solve(opts, want_lambda=True)
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    log("  gpu", st.as_dict(), "rel L2 u", eu)
    assert st.status == 0
    assert eu < (1e-8 if precision else 1e-10)


def test_step_extension_rejects_other_values():
    from paper_2412_13733_amd import hpg
    mesh, prob, sysm = build_pair(1, 4, 2, W.w1d())
    with pytest.raises(hpg.HpgError) as e:
        prob.solve(prob_opts(step_extension=2))
    assert e.value.status == hpg.ERR_INVALID_ARG
