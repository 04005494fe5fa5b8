"""GPU parity of the per-cell-degree (hp) path against the oracle's HpMesh.

Operators (G, the block preconditioner with its block-Jacobi A-block, the
Newton residual) element by element on small hp meshes in 1-D, 2-D and 3-D
(random degrees, graded breakpoints, a single cell, degrees up to 14 with the
largest Schur blocks inverted in HBM beside LDS-sized ones, a 70 x 3 grid whose
vertex solve exceeds the one-workgroup size, a 3-D cell of degree 11 whose
1000-unknown interior entity is applied alone), FP64
and FP32 (the bars of gpu_common); full LVPP solves (FP64 to 1e-10 rel-L2,
mixed to 1e-8); and the 2-D 64 x 64 workload with degrees 2..12 graded away
from the contact boundary (tests/golden/dip_64x64_degrees.txt): G and the
residual in full, the A-block in full, the psi-block on sampled cells."""
import os
import zlib

import numpy as np
import pytest

from oracle import assemble, lvpp, precond, mesh as OM
from oracle.hpmesh import HpMesh
import workloads as W

from gpu_common import FP32_G, FP32_P, FP64_G, FP64_P, FP64_P_COND, FP64_RES, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _pair(breaks, deg, data):
    from paper_2412_13733_amd import hpg
    d = len(breaks)
    mesh = hpg.Mesh(d, [len(b) - 1 for b in breaks], 0, breaks=breaks, degree=deg)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh)
    prob.set_forcing(data[0](x))
    prob.set_obstacle(data[1](x))
    om = HpMesh(breaks, deg)
    xo = om.quadrature_points()
    assert mesh.n_u == om.n_u and mesh.n_psi == om.n_psi and np.max(np.abs(x - xo)) < 1e-15
    return mesh, prob, om, assemble.System(om, data[0](xo), data[1](xo))


def _graded(m, seed):
    rng = np.random.default_rng(seed)
    return np.sort(np.r_[0.0, rng.uniform(0.03, 0.97, m - 1), 1.0])


def _data(d):
    return W.w1d() if d == 1 else (W.w2d(0) if d == 2 else W.w3d())


def _case(name):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "1d-graded":
        return [_graded(7, 1)], rng.integers(2, 8, 7)
    if name == "2d-graded":
        return [_graded(5, 2), _graded(5, 3)], rng.integers(2, 9, 25)
    if name == "2d-high":
        return [W.uniform_breaks(3)] * 2, rng.integers(8, 13, 9)
    if name == "2d-aniso":
        return [W.uniform_breaks(4), _graded(6, 4)], rng.integers(2, 7, 24)
    if name == "2d-one-cell":
        return [W.uniform_breaks(1)] * 2, np.array([5])
    if name == "2d-all-p2":
        return [W.uniform_breaks(6)] * 2, np.full(36, 2)
    if name == "2d-wide":   # 69 interior vertices in direction 0: the batched-GEMM vertex solve
        return [W.uniform_breaks(70), W.uniform_breaks(3)], rng.integers(2, 5, 210)
    if name == "2d-big":   # degrees 13, 14: Schur blocks inverted in HBM next to LDS ones
        return [W.uniform_breaks(3), W.uniform_breaks(2)], np.array([2, 13, 5, 14, 3, 12])
    if name == "3d":
        return [W.uniform_breaks(3), _graded(3, 5), W.uniform_breaks(3)], rng.integers(2, 6, 27)
    if name == "3d-high":   # a 1000-unknown interior entity: one entity per chunk
        return [W.uniform_breaks(2), W.uniform_breaks(1), W.uniform_breaks(1)], np.array([11, 3])
    raise KeyError(name)


CASES = ["1d-graded", "2d-graded", "2d-high", "2d-aniso", "2d-one-cell", "2d-all-p2", "2d-wide",
         "2d-big", "3d", "3d-high"]


@pytest.mark.parametrize("name", CASES)
def test_hp_operators(name):
    breaks, deg = _case(name)
    d = len(breaks)
    log("hp operators", name, "degrees", np.bincount(deg).nonzero()[0].tolist())
    mesh, prob, om, sysm = _pair(breaks, deg, _data(d))
    rng = np.random.default_rng(17)
    # 0.6 per Legendre mode makes psi_h swing by +-15 over a degree-11 3-D cell
    # and its Schur block's condition number 3e9 (the oracle's); 0.1 keeps
    # psi_h within +-3 there and the condition number at 1.3e4
    psi = (0.1 if name == "3d-high" else 0.6) * rng.standard_normal(mesh.n_psi)
    alpha, beta = 3.5, 1e-3
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    for prec, dt, tg, tp in ((0, torch.float64, FP64_G, FP64_P), (1, torch.float32, FP32_G, FP32_P)):
        prob.op_setup(_dev(psi), alpha, beta, precision=prec)
        y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=dt, device="cuda")
        prob.op_apply_G(_dev(x, dt), y)
        yg = y.double().cpu().numpy()
        z = torch.zeros_like(y)
        prob.op_apply_prec(_dev(x, dt), z)
        zg = z.double().cpu().numpy()
        e = (rel(yg[:mesh.n_u], yu), rel(yg[mesh.n_u:], yp), rel(zg[:mesh.n_u], zu),
             rel(zg[mesh.n_u:], zp))
        log("  prec", prec, "G u/psi %.2e %.2e  P u/psi %.2e %.2e" % e)
        # FP64 psi-blocks of degree >= 13 cells (2-D) or >= 7 (3-D): the conditioning bar
        tpp = FP64_P_COND if prec == 0 and deg.max() >= (13 if d < 3 else 7) else tp
        assert e[0] < tg and e[1] < tg and e[2] < tp and e[3] < tpp
    u = 0.1 * rng.standard_normal(mesh.n_u)
    pp = 0.5 * rng.standard_normal(mesh.n_psi)
    R = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_residual(_dev(u), _dev(psi), _dev(pp), alpha, R)
    Ru, Rp = sysm.residual(u, psi, pp, alpha)
    Rg = R.cpu().numpy()
    log("  residual %.2e %.2e" % (rel(Rg[:mesh.n_u], Ru), rel(Rg[mesh.n_u:], Rp)))
    assert rel(Rg[:mesh.n_u], Ru) < FP64_RES and rel(Rg[mesh.n_u:], Rp) < FP64_RES


@pytest.mark.parametrize("name,precision", [("1d-graded", 0), ("2d-graded", 0), ("2d-graded", 1),
                                            ("2d-high", 0)])
def test_hp_solve_matches_oracle(name, precision):
    from paper_2412_13733_amd import hpg
    breaks, deg = _case(name)
    d = len(breaks)
    mesh, prob, om, sysm = _pair(breaks, deg, _data(d))
    ro = lvpp.solve(sysm, lvpp.Options())
    assert ro.converged
    kw = dict(fixed_prox_steps=ro.prox_steps)
    if precision:
        kw.update(precision=hpg.MIXED, newton_tol=1e-10, krylov_rtol=1e-6)
    u, psi, lam, st = prob.solve(hpg.default_opts(**kw), want_lambda=True)
    eu = sysm.l2_norm_u(u - ro.u) / sysm.l2_norm_u(ro.u)
    log("hp solve", name, "precision", precision, "oracle K", ro.prox_steps, "newton", ro.newton,
        "| gpu", st.as_dict(), "rel L2", eu)
    assert st.status == 0
    assert eu < (1e-8 if precision else 1e-10)


def _dip():
    deg = np.loadtxt(os.path.join(HERE, "golden", "dip_64x64_degrees.txt"), dtype=int).reshape(-1)
    return [W.uniform_breaks(64)] * 2, deg


@pytest.mark.timeout(600)
def test_hp_dip_64x64_fullsize():
    breaks, deg = _dip()
    mesh, prob, om, sysm = _pair(breaks, deg, W.w2d_dip(0))
    log("dip 64x64: n_u", mesh.n_u, "n_psi", mesh.n_psi)
    rng = np.random.default_rng(23)
    psi = 0.5 * rng.standard_normal(mesh.n_psi)
    alpha, beta = 8.0, 1e-4
    x = rng.standard_normal(mesh.n_u + mesh.n_psi)
    yu, yp = precond.apply_G(sysm, psi, alpha, beta, x[:mesh.n_u], x[mesh.n_u:])
    for prec, dt, tol in ((0, torch.float64, FP64_G), (1, torch.float32, FP32_G)):
        prob.op_setup(_dev(psi), alpha, beta, precision=prec)
        y = torch.zeros(mesh.n_u + mesh.n_psi, dtype=dt, device="cuda")
        prob.op_apply_G(_dev(x, dt), y)
        yg = y.double().cpu().numpy()
        log("  G prec", prec, rel(yg[:mesh.n_u], yu), rel(yg[mesh.n_u:], yp))
        assert rel(yg[:mesh.n_u], yu) < tol and rel(yg[mesh.n_u:], yp) < tol
    u = 0.1 * rng.standard_normal(mesh.n_u)
    pp = 0.5 * rng.standard_normal(mesh.n_psi)
    R = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_residual(_dev(u), _dev(psi), _dev(pp), alpha, R)
    Ru, Rp = sysm.residual(u, psi, pp, alpha)
    Rg = R.cpu().numpy()
    assert rel(Rg[:mesh.n_u], Ru) < FP64_RES and rel(Rg[mesh.n_u:], Rp) < FP64_RES
    # preconditioner (FP64): the block-Jacobi A-block in full ...
    prob.op_setup(_dev(psi), alpha, beta, precision=0)
    r = rng.standard_normal(mesh.n_u + mesh.n_psi)
    z = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float64, device="cuda")
    prob.op_apply_prec(_dev(r), z)
    zg = z.cpu().numpy()
    zu = precond.a_block(sysm, alpha, r[:mesh.n_u])
    log("  A-block", rel(zg[:mesh.n_u], zu))
    assert rel(zg[:mesh.n_u], zu) < FP64_P
    # ... and the psi-block on sampled cells: S_hat_K is cell-local, so each is
    # taken from a one-cell oracle mesh of the cell's degree and widths
    h = 1.0 / 64
    for c in rng.choice(mesh.n_cells, 16, replace=False):
        p = int(deg[c])
        one = OM.TensorMesh([np.array([0.0, h])] * 2, p)
        s1 = assemble.System(one, np.zeros(one.n_qp), np.zeros(one.n_qp))
        sl = om.psi_dofs(int(c))
        S = precond.schur_hat_cells(s1, psi[sl], alpha, beta, [0])[0]
        zo = np.linalg.solve(-S, r[mesh.n_u + sl])
        assert rel(zg[mesh.n_u + sl], zo) < FP64_P, (c, p)
