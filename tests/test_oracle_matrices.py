"""Pins of the oracle's assembled operators (paper Sec. 3 and Sec. 4.3-4.5):
closed-form 1-D matrices, tensor-product structure, sparsity facts and
residual/Jacobian consistency."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle import assemble, mesh as M, precond
import workloads as W


def _system(breaks, p, kind=M.OBSTACLE, f=None, phi=None):
    ms = M.TensorMesh(breaks, p, kind)
    x = ms.quadrature_points()
    f = f or W.const(1.0)
    phi = phi or W.const(1.0)
    return assemble.System(ms, f(x), phi(x))


BR1 = [np.array([0.0, 0.15, 0.4, 0.55, 1.0])]


@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_1d_stiffness_closed_form(p):
    s = _system(BR1, p)
    A = s.A.toarray()
    h = np.diff(BR1[0])
    m = len(h)
    ref = np.zeros_like(A)
    for v in range(1, m):                       # interior hats
        i = v * p - 1
        ref[i, i] = 1 / h[v - 1] + 1 / h[v]
        if v + 1 <= m - 1:
            j = (v + 1) * p - 1
            ref[i, j] = ref[j, i] = -1 / h[v]
    for c in range(m):                          # bubbles: 4 / (h (2n+3)) delta
        for n in range(p - 1):
            ref[c * p + n, c * p + n] = 4.0 / (h[c] * (2 * n + 3))
    assert np.allclose(A, ref, atol=1e-12, rtol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 6])
def test_1d_gram_closed_form(p):
    # B_ij = (v_i, zeta_j): (W_n, P_k)_K = (h/2)[2 d_nk/(2n+1) - 2 d_{k,n+2}/(2n+5)]/(2n+3),
    # (hat, P_0) = h/2, (hat_left-of-cell, P_1) = -h/6, (hat_right, P_1) = h/6.
    s = _system(BR1, p)
    B = s.B.toarray()
    h = np.diff(BR1[0])
    m, P = len(h), p - 1
    ref = np.zeros_like(B)
    for c in range(m):
        for n in range(p - 1):
            for k in range(P):
                val = 0.0
                if k == n:
                    val += 2.0 / (2 * n + 1)
                if k == n + 2:
                    val -= 2.0 / (2 * n + 5)
                ref[c * p + n, c * P + k] = 0.5 * h[c] * val / (2 * n + 3)
        if c >= 1:       # hat of vertex c is the left end of cell c
            ref[c * p - 1, c * P] += h[c] / 2
            if P > 1:
                ref[c * p - 1, c * P + 1] += -h[c] / 6
        if c + 1 <= m - 1:   # hat of vertex c+1 is the right end of cell c
            ref[(c + 1) * p - 1, c * P] += h[c] / 2
            if P > 1:
                ref[(c + 1) * p - 1, c * P + 1] += h[c] / 6
    assert np.allclose(B, ref, atol=1e-14)


@pytest.mark.parametrize("p", [2, 4, 7])
def test_psi_mass_is_diagonal(p):
    # Lemma (diagonal mass matrix): (zeta_i, zeta_j) = |K| delta_ij / (2n+1),
    # n the Legendre degree of zeta_i (in d-D the product over directions).
    br = [np.array([0.0, 0.3, 1.0]), np.array([0.0, 0.6, 1.0])]
    s = _system(br, p)
    Mp = s.Mpsi.toarray()
    P = p - 1
    ref = []
    for cno, cidx in s.mesh.cells():
        hx, hy = s.mesh.cell_widths(cidx)
        for ay in range(P):
            for ax in range(P):
                ref.append(hx * hy / ((2 * ax + 1) * (2 * ay + 1)))
    assert np.allclose(Mp, np.diag(ref), atol=1e-15)


def test_phi_hat_blocks_1d_closed_form():
    # A_hat_alpha = alpha (Y_m', Y_n')_K = alpha 4 (2n+3) / h delta (diagonal in 1-D, Sec. 4.5);
    # B_hat = (Y_m, P_n)_K = (h/2)[2 d_mn/(2n+1) - 2 d_{m+2,n}/(2n+1)].
    p, alpha = 6, 3.0
    s = _system(BR1, p)
    Ah, Bh = precond.phi_blocks(s, alpha)
    h = np.diff(BR1[0])
    P = p - 1
    refA = np.diag(np.concatenate([alpha * 4 * (2 * np.arange(P) + 3) / hc for hc in h]))
    assert np.allclose(Ah.toarray(), refA, rtol=1e-13)
    refB = np.zeros((len(h) * P, len(h) * P))
    for c, hc in enumerate(h):
        for mm in range(P):
            for n in range(P):
                v = (2.0 / (2 * n + 1)) * ((mm == n) - (mm + 2 == n))
                refB[c * P + mm, c * P + n] = 0.5 * hc * v
    assert np.allclose(Bh.toarray(), refB, atol=1e-14)


def test_tensor_structure_2d():
    # Sec. 3: the 2-D spaces are tensor products, so with u ordered direction-0
    # fastest A = M1_y (x) A1_x + A1_y (x) M1_x and the u-mass is M1_y (x) M1_x.
    p = 4
    bx = np.array([0.0, 0.2, 0.45, 1.0])
    by = np.array([0.0, 0.7, 1.0])
    s2 = _system([bx, by], p)
    sx = _system([bx], p)
    sy = _system([by], p)
    A2 = sp.kron(sy.Mu, sx.A) + sp.kron(sy.A, sx.Mu)
    assert abs(s2.A - A2).max() < 1e-13
    assert abs(s2.Mu - sp.kron(sy.Mu, sx.Mu)).max() < 1e-14
    # B = B1_y (x) B1_x up to the cell-major psi numbering
    Bk = sp.kron(sy.B, sx.B).toarray()
    P = p - 1
    mx, my = len(bx) - 1, len(by) - 1
    perm = []
    for cy in range(my):
        for cx in range(mx):
            for ay in range(P):
                for ax in range(P):
                    perm.append((cy * P + ay) * (mx * P) + cx * P + ax)
    assert np.allclose(s2.B.toarray(), Bk[:, perm], atol=1e-14)


@pytest.mark.parametrize("d,p", [(2, 5), (3, 3)])
def test_sparsity_facts(d, p):
    # D_psi is block-diagonal with dense cell blocks (Sec. 4.3); A, B have
    # O(p^d / h^d) nonzeros: at most (p+1)^d local couplings per cell.
    ms = M.uniform_mesh(d, 3, p)
    x = ms.quadrature_points()
    s = assemble.System(ms, W.const(1.0)(x), W.const(1.0)(x))
    rng = np.random.default_rng(0)
    D = s.Dpsi(rng.standard_normal(ms.n_psi)).tocoo()
    blk = ms.psi_per_cell
    assert np.all(D.row // blk == D.col // blk)
    assert D.nnz == ms.n_cells * blk * blk
    assert s.A.nnz <= ms.n_cells * (p + 1) ** (2 * d)
    assert s.B.nnz <= ms.n_cells * (p + 1) ** d * (p - 1) ** d


def test_phi_hat_has_4N_blocks_in_2d():
    # Sec. 4.5: A_hat is block-diagonal with 4N blocks in 2-D (N cells).
    ms = M.uniform_mesh(2, 3, 6)
    x = ms.quadrature_points()
    s = assemble.System(ms, W.const(1.0)(x), W.const(1.0)(x))
    Ah, _ = precond.phi_blocks(s, 1.0)
    Ah = Ah.tocoo()
    big = np.abs(Ah.data) > 1e-12 * np.abs(Ah.data).max()   # drop quadrature round-off
    Ah = sp.coo_matrix((Ah.data[big], (Ah.row[big], Ah.col[big])), shape=Ah.shape)
    ncomp, _ = connected_components(Ah, directed=False)
    assert ncomp == 4 * ms.n_cells
    # S_hat is cell-block diagonal
    S = precond.schur_hat(s, np.zeros(ms.n_psi), 2.0, 0.0).tocoo()
    blk = ms.psi_per_cell
    big = np.abs(S.data) > 1e-300
    assert np.all(S.row[big] // blk == S.col[big] // blk)


@pytest.mark.parametrize("d,p,kind", [(1, 4, M.OBSTACLE), (2, 3, M.OBSTACLE), (3, 2, M.OBSTACLE),
                                      (1, 3, M.GRADIENT), (2, 2, M.GRADIENT), (3, 1, M.GRADIENT)])
def test_residual_jacobian_consistency(d, p, kind):
    # central differences of the residual equal the Jacobian action to O(eps^2)
    ms = M.TensorMesh([np.array([0.0, 0.35, 1.0])] * d, p, kind)
    x = ms.quadrature_points()
    phi = W.const(0.4)
    f = lambda xx: 3.0 + np.sin(3 * np.atleast_2d(xx)[:, 0])
    s = assemble.System(ms, f(x), phi(x))
    rng = np.random.default_rng(1)
    u = rng.standard_normal(ms.n_u) * 0.1
    psi = rng.standard_normal(ms.n_psi) * 0.5
    psi_prev = rng.standard_normal(ms.n_psi) * 0.5
    alpha = 1.7
    G = s.jacobian(psi, alpha, 0.0)
    v = rng.standard_normal(ms.n_u + ms.n_psi)
    eps = 1e-5
    vu, vp = v[:ms.n_u], v[ms.n_u:]
    Rp = np.concatenate(s.residual(u + eps * vu, psi + eps * vp, psi_prev, alpha))
    Rm = np.concatenate(s.residual(u - eps * vu, psi - eps * vp, psi_prev, alpha))
    fd = (Rp - Rm) / (2 * eps)
    Gv = G @ v
    assert np.linalg.norm(fd - Gv) <= 1e-8 * np.linalg.norm(Gv)
    # G is symmetric (GL quadrature keeps D_psi symmetric)
    assert abs(G - G.T).max() < 1e-12 * abs(G).max()


@pytest.mark.parametrize("kind", [M.OBSTACLE, M.GRADIENT])
def test_schur_hat_cells_are_the_blocks_of_schur_hat(kind):
    # the per-cell accessor used by the full-size GPU checks must reproduce the
    # diagonal blocks of the (pinned) global S_hat, and S_hat must vanish
    # outside them
    om = M.TensorMesh([np.array([0, .3, .55, 1.0]), np.array([0, .4, 1.0])], 4, kind)
    f, phi = W.w2d(0)
    xo = om.quadrature_points()
    sysm = assemble.System(om, f(xo), np.abs(phi(xo)) + 0.1)
    rng = np.random.default_rng(3)
    psi = 0.7 * rng.standard_normal(om.n_psi)
    S = precond.schur_hat(sysm, psi, 2.5, 1e-3).toarray()
    cells = np.arange(om.n_cells)
    blocks = precond.schur_hat_cells(sysm, psi, 2.5, 1e-3, cells)
    mask = np.zeros_like(S, dtype=bool)
    for c, B in zip(cells, blocks):
        pg = om.psi_dofs(int(c))
        assert np.allclose(S[np.ix_(pg, pg)], B, rtol=1e-12, atol=1e-12 * np.abs(S).max())
        mask[np.ix_(pg, pg)] = True
    assert np.abs(S[~mask]).max() <= 1e-12 * np.abs(S).max()
