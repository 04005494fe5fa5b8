"""The block preconditioner of Sec. 4.4-4.6, assembled plainly.

Test infrastructure only (see ``oracle/__init__.py``).

P_D = diag(A_alpha, S) from the Schur factorisation eq. (schur4); the Schur
complement S = -(D_psi + E_beta + B^T A_alpha^{-1} B) is replaced by
* obstacle, eq. (schur-preconditioner):
      S_hat = -D_psi - E_beta - B_hat^T A_hat_alpha^{-1} B_hat,
      [A_hat_alpha]_ij = alpha (grad_h eta_i, grad_h eta_j),
      B_hat_ij = (eta_i, zeta_j), eta in Phi_h: per cell and direction the
      rescaled shape functions Y_0..Y_{p-2} (Sec. 3, Sec. 4.5);
* gradient, eq. (schur-preconditioner:gradient): S_hat = -D_psi - E_beta.

A symmetric Krylov method needs a positive definite preconditioner, so the
operator returned is the SPD form diag(alpha A, -S_hat) (a reading: the paper
writes P_D = diag(A_alpha, S_hat) for FGMRES, where the sign does not matter).

With one degree per cell (``HpMesh``) the u space is no longer a tensor
product and the A-block is replaced (reading) by the block-Jacobi operator
sum_g R_g^T (alpha A_gg)^{-1} R_g over the groups of ``mesh.u_groups()``: all
vertex unknowns together (the Q1 space of the mesh) and each edge, face and
cell-interior entity on its own.  It is SPD and exact on each group.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import _Coo, kron_dirs
from .mesh import OBSTACLE


def phi_blocks(system, alpha):
    """(A_hat_alpha, B_hat) of eq. (schur-preconditioner), sparse, on Phi_h."""
    mesh = system.mesh
    cA, cB = _Coo(), _Coo()
    for cno, cidx, W, Vpsi, pg, phq in system.cells:
        ref = system.cell_refs[cno]
        hs = mesh.cell_widths(cidx)
        VY = kron_dirs([ref.Y] * mesh.d)
        GY = []
        for k in range(mesh.d):
            tabs = [ref.Y] * mesh.d
            tabs[k] = ref.dY * (2.0 / hs[k])
            GY.append(kron_dirs(tabs))
        eta = pg   # Phi_h carries as many functions per cell as Psi_h (P_K^d)
        cA.add(eta, eta, alpha * sum(G.T @ (W[:, None] * G) for G in GY))
        cB.add(eta, pg, VY.T @ (W[:, None] * Vpsi))
    n_eta = mesh.n_psi
    return cA.csr((n_eta, n_eta)).tocsc(), cB.csr((n_eta, mesh.n_psi)).tocsc()


def schur_hat(system, psi, alpha, beta):
    """Sparse S_hat (n_psi x n_psi); cell-block diagonal by construction."""
    D = system.Dpsi(psi) + beta * system.Ebeta_unit
    if system.mesh.kind != OBSTACLE:
        return -D
    Ahat, Bhat = phi_blocks(system, alpha)
    X = spla.spsolve(Ahat, Bhat.toarray())
    return sp.csr_matrix(-D.toarray() - Bhat.T.toarray() @ X)


def schur_hat_cells(system, psi, alpha, beta, cells):
    """Dense cell blocks of S_hat for the listed cells (S_hat is block-diagonal
    by cells); the same matrices as schur_hat, restricted to each cell."""
    D = (system.Dpsi(psi) + beta * system.Ebeta_unit).tocsr()
    mesh = system.mesh
    if mesh.kind == OBSTACLE:
        Ahat, Bhat = phi_blocks(system, alpha)
        Ahat, Bhat = Ahat.tocsr(), Bhat.tocsr()
    out = []
    for c in cells:
        pg = mesh.psi_dofs(int(c))
        blk = -D[pg][:, pg].toarray()
        if mesh.kind == OBSTACLE:
            eta = pg
            Bk = Bhat[eta][:, pg].toarray()
            Ak = Ahat[eta][:, eta].toarray()
            blk = blk - Bk.T @ np.linalg.solve(Ak, Bk)
        out.append(blk)
    return out


def a_block(system, alpha, r_u):
    """z_u: (alpha A)^{-1} r_u, or the block-Jacobi operator on hp meshes."""
    if not getattr(system.mesh, "hp", False):
        return spla.spsolve((alpha * system.A).tocsc(), r_u)
    A = system.A.tocsr()
    z = np.zeros_like(r_u)
    for g in system.mesh.u_groups():
        if g.size:
            z[g] = np.linalg.solve(alpha * A[g][:, g].toarray(), r_u[g])
    return z


def apply_prec(system, psi, alpha, beta, r_u, r_psi):
    """z = diag(alpha A, -S_hat)^{-1} r (direct solves; A-block as a_block)."""
    zu = a_block(system, alpha, r_u)
    S = schur_hat(system, psi, alpha, beta)
    zpsi = np.linalg.solve(-S.toarray(), r_psi)
    return zu, zpsi


def apply_G(system, psi, alpha, beta, x_u, x_psi):
    """y = G x with G of eq. (pG-matrix) at the iterate psi."""
    G = system.jacobian(psi, alpha, beta)
    y = G @ np.concatenate([x_u, x_psi])
    return y[: system.mesh.n_u], y[system.mesh.n_u:]
