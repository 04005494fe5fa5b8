"""FP32 psi-block of a cell straddling the free boundary.

Where psi_h swings over two hundred units across one cell, e^{-psi} spans
some ninety orders of magnitude over its Gauss points and -S_hat_K has a
condition number near 1e11; a product with its inverse in FP32 then carries a
relative error far above one and <S^{-1} v, v> can come out negative (the FP32
MINRES breakdowns of high-degree requests).  The setup flags such cells
(1-norm condition above 1e6) and the FP32 preconditioner applies them with the
FP64 inverse.  Checked against the oracle's P_D (FP64) on a 3x3-cell p = 9
mesh whose centre cell carries such a psi, with the right-hand side along the
block's stiffest direction, where an FP32 product is least accurate (its
error there is about 4.5 relative to the block's result; the FP64 product's
2e-8)."""
import numpy as np
import pytest

from oracle import precond
import workloads as W

from gpu_common import FP32_P, build_pair, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def test_ill_conditioned_cell_is_applied_in_fp64_by_the_fp32_path():
    from paper_2412_13733_amd import hpg
    mesh, prob, sysm = build_pair(2, 3, 9, W.w2d(0))
    P = 8
    npc = P * P
    psi = np.zeros(mesh.n_psi)
    psi[::npc] = 1.6                                   # e^{-psi} ~ 0.2 in every cell ...
    c = 4                                              # ... but the centre cell: psi_h from about -10 to 207
    sl = slice(c * npc, (c + 1) * npc)
    psi[c * npc] = 98.5
    psi[c * npc + 1] = 108.0                           # the first Legendre mode along direction 0
    pq = sysm.psi_at_points(psi)[c, 0]
    log("centre cell psi at the Gauss points: %.1f .. %.1f" % (pq.min(), pq.max()))
    assert pq.min() < -5 and pq.max() > 150
    alpha, beta = 8.0, 0.0
    S = -np.asarray(precond.schur_hat_cells(sysm, psi, alpha, beta, [c])[0])
    Si = np.linalg.inv(S)
    cond1 = np.abs(S).sum(0).max() * np.abs(Si).sum(0).max()
    log("centre block 1-norm condition %.2e" % cond1)
    assert cond1 > 1e8                                 # well beyond the flagging limit
    # right-hand side: random, with the centre block's stiffest direction
    rng = np.random.default_rng(9)
    r = rng.standard_normal(mesh.n_u + mesh.n_psi)
    ev, V = np.linalg.eigh(0.5 * (Si + Si.T))
    r[mesh.n_u + c * npc:mesh.n_u + (c + 1) * npc] = V[:, 0] * np.linalg.norm(r[mesh.n_u:][:npc])
    # the FP32 path sees r rounded to FP32: the reference takes the same input
    # (along the stiff direction the rounding alone moves S^{-1} r by about
    # eps_32 cond relative; an FP32 product adds as much again, an FP64
    # product of the FP64 inverse about 2e-8 here)
    r = r.astype(np.float32).astype(np.float64)
    zu, zp = precond.apply_prec(sysm, psi, alpha, beta, r[:mesh.n_u], r[mesh.n_u:])
    prob.op_setup(_dev(psi), alpha, beta, precision=hpg.MIXED)
    z = torch.zeros(mesh.n_u + mesh.n_psi, dtype=torch.float32, device="cuda")
    prob.op_apply_prec(_dev(r, torch.float32), z)
    zg = z.double().cpu().numpy()
    zc, rc = zg[mesh.n_u:][sl], r[mesh.n_u:][sl]
    e_cell = rel(zc, zp[sl])
    e_all = rel(zg[mesh.n_u:], zp)
    log("FP32 path: centre block rel %.2e, psi-block rel %.2e, u-block rel %.2e, <z, r> centre %.3e "
        "(FP64 %.3e)" % (e_cell, e_all, rel(zg[:mesh.n_u], zu), float(zc @ rc), float(zp[sl] @ rc)))
    assert e_cell < FP32_P and e_all < FP32_P
    assert rel(zg[:mesh.n_u], zu) < FP32_P
    assert float(zc @ rc) > 0.0
    assert abs(float(zc @ rc) - float(zp[sl] @ rc)) < FP32_P * abs(float(zp[sl] @ rc))
