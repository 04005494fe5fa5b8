"""Pins of the oracle's per-cell-degree (hp) mesh: DOF count by hand,
H^1-conformity of the traces, exact reproduction of a polynomial that lies in
every hp space, equality with the uniform-degree oracle when all degrees
agree, the cell-locality of S_hat, and exactness of the block-Jacobi A-block
in 1-D (where the bubbles are A-orthogonal to everything else)."""
import numpy as np
import pytest

from oracle import assemble, basis, lvpp, precond, mesh as OM
from oracle.hpmesh import HpMesh

import workloads as W


def _system(mesh, f, phi):
    x = mesh.quadrature_points()
    return assemble.System(mesh, f(x), phi(x))


def _eval_cell(mesh, u, cidx, y):
    """u_h at reference points y (n, d) of cell cidx, from its local coefficients."""
    cno = mesh.cell_number(cidx)
    p = int(mesh.deg[cno])
    ug = mesh.u_dofs(cidx)
    loc = np.where(ug >= 0, u[np.maximum(ug, 0)], 0.0)
    L = p + 1
    vals = [basis.u_local(p, y[:, k])[0] for k in range(mesh.d)]   # (L, n) each
    out = np.zeros(y.shape[0])
    for j in range(L ** mesh.d):
        t = np.ones(y.shape[0])
        for k in range(mesh.d):
            t = t * vals[k][(j // L ** k) % L]
        out += loc[j] * t
    return out


def test_dof_count_by_hand():
    # 2 x 2 cells, degrees (cell (i, j) -> i + 2 j): 2, 3, 4, 5.  Interior vertex: 1;
    # edges: min(2,3)-1 + min(4,5)-1 + min(2,4)-1 + min(3,5)-1 = 1 + 3 + 1 + 2;
    # interiors: 1 + 4 + 9 + 16.
    m = HpMesh([W.uniform_breaks(2)] * 2, [2, 3, 4, 5])
    assert m.n_u == 1 + (1 + 3 + 1 + 2) + 30
    assert m.n_psi == 1 + 4 + 9 + 16
    assert m.n_qp == 9 + 16 + 25 + 36
    # every global unknown is reached from some cell, none twice within a cell
    seen = set()
    for cno, cidx in m.cells():
        g = m.u_dofs(cidx)
        g = g[g >= 0]
        assert len(set(g.tolist())) == g.size
        seen.update(g.tolist())
    assert seen == set(range(m.n_u))


@pytest.mark.parametrize("d", [2, 3])
def test_traces_agree_across_cells(d):
    rng = np.random.default_rng(5)
    m = 3
    deg = rng.integers(2, 6, size=m ** d)
    mesh = HpMesh([np.sort(np.r_[0.0, rng.uniform(0.1, 0.9, m - 1), 1.0])] * d, deg)
    u = rng.standard_normal(mesh.n_u)
    t = rng.uniform(-1, 1, size=(7, d))
    worst = 0.0
    for cno, cidx in mesh.cells():
        for k in range(d):
            if cidx[k] + 1 >= m:
                continue
            nb = list(cidx)
            nb[k] += 1
            ya, yb = t.copy(), t.copy()
            ya[:, k], yb[:, k] = 1.0, -1.0       # the shared face, seen from both sides
            va = _eval_cell(mesh, u, cidx, ya)
            vb = _eval_cell(mesh, u, tuple(nb), yb)
            worst = max(worst, np.max(np.abs(va - vb)))
    assert worst < 1e-12


def test_polynomial_in_every_hp_space_is_reproduced():
    # u* = x(1-x) y(1-y) has degree 2 per direction and vanishes on the boundary:
    # it lies in every hp space (p_K >= 2), so the Galerkin solution of
    # -Lap u = f, f = 2 y(1-y) + 2 x(1-x), is u* itself.
    rng = np.random.default_rng(8)
    deg = rng.integers(2, 7, size=16)
    br = np.array([0.0, 0.2, 0.55, 0.8, 1.0])
    mesh = HpMesh([br, br], deg)
    f = lambda x: 2 * x[:, 1] * (1 - x[:, 1]) + 2 * x[:, 0] * (1 - x[:, 0])
    sysm = _system(mesh, f, lambda x: np.ones(len(x)))
    import scipy.sparse.linalg as spla
    u = spla.spsolve(sysm.A.tocsc(), sysm.F)
    x = mesh.quadrature_points()
    ex = x[:, 0] * (1 - x[:, 0]) * x[:, 1] * (1 - x[:, 1])
    assert np.max(np.abs(sysm.u_at_points(u) - ex)) < 1e-13


def test_uniform_degrees_reproduce_the_tensor_oracle():
    f, phi = W.w2d(0)
    br = W.uniform_breaks(3)
    hp = HpMesh([br, br], [4] * 9)
    tm = OM.TensorMesh([br, br], 4)
    sh, st = _system(hp, f, phi), _system(tm, f, phi)
    assert hp.n_u == tm.n_u and hp.n_psi == tm.n_psi
    rh = lvpp.solve(sh, lvpp.Options())
    rt = lvpp.solve(st, lvpp.Options())
    assert rh.prox_steps == rt.prox_steps
    uh, ut = sh.u_at_points(rh.u), st.u_at_points(rt.u)
    assert np.max(np.abs(uh - ut)) < 1e-11 * np.max(np.abs(ut))
    assert np.max(np.abs(rh.psi - rt.psi)) < 1e-9 * np.max(np.abs(rt.psi))


def test_schur_hat_is_cell_local():
    # S_hat_K depends only on the cell's degree, widths and psi: compare a cell
    # of an hp mesh with the same cell of a uniform mesh of that degree
    rng = np.random.default_rng(9)
    br = W.uniform_breaks(3)
    deg = np.array([2, 3, 4, 5, 3, 2, 4, 4, 5])
    hp = HpMesh([br, br], deg)
    sh = _system(hp, *W.w2d(0))
    psi = 0.4 * rng.standard_normal(hp.n_psi)
    for c in (2, 4, 8):
        p = int(deg[c])
        tm = OM.TensorMesh([br, br], p)
        st = _system(tm, *W.w2d(0))
        psi_t = np.zeros(tm.n_psi)
        psi_t[tm.psi_dofs(c)] = psi[hp.psi_dofs(c)]
        Sh = precond.schur_hat_cells(sh, psi, 3.0, 1e-3, [c])[0]
        St = precond.schur_hat_cells(st, psi_t, 3.0, 1e-3, [c])[0]
        assert np.max(np.abs(Sh - St)) < 1e-12 * np.max(np.abs(St))


def test_block_jacobi_is_exact_in_1d():
    rng = np.random.default_rng(10)
    mesh = HpMesh([np.sort(np.r_[0.0, rng.uniform(0.05, 0.95, 6), 1.0])], [2, 5, 3, 7, 2, 4, 6])
    sysm = _system(mesh, lambda x: np.ones(len(x)), lambda x: np.ones(len(x)))
    r = rng.standard_normal(mesh.n_u)
    import scipy.sparse.linalg as spla
    z = precond.a_block(sysm, 2.5, r)
    ze = spla.spsolve((2.5 * sysm.A).tocsc(), r)
    assert np.max(np.abs(z - ze)) < 1e-12 * np.max(np.abs(ze))


def test_block_jacobi_is_spd_in_2d():
    rng = np.random.default_rng(11)
    br = W.uniform_breaks(3)
    mesh = HpMesh([br, br], rng.integers(2, 6, size=9))
    sysm = _system(mesh, lambda x: np.ones(len(x)), lambda x: np.ones(len(x)))
    n = mesh.n_u
    Pm = np.column_stack([precond.a_block(sysm, 1.0, e) for e in np.eye(n)])
    assert np.max(np.abs(Pm - Pm.T)) < 1e-12 * np.max(np.abs(Pm))
    assert np.min(np.linalg.eigvalsh(0.5 * (Pm + Pm.T))) > 0
