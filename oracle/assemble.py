"""Sparse FP64 assembly of the hpG matrices and nonlinear terms (paper Sec. 4).

Test infrastructure only (see ``oracle/__init__.py``).

Reading Q1 (quadrature): every integral is computed with the tensor
Gauss-Legendre rule of q = p + 1 points per direction on every cell.  It is
exact for A, B and the u-mass matrix; the nonlinear terms (exp(-psi) and the
gradient flux) are evaluated at these points, which keeps D_psi symmetric.
Data f and phi enter only through their values at these points.

Obstacle (Sec. 4.1, eq. (pG), eq. (pG-matrix)):
    A_ij = (grad v_i, grad v_j),  B_ij = (v_i, zeta_j),
    [D_psi]_ij = (zeta_i, exp(-psi_h) zeta_j),  [E_beta]_ij = beta (zeta_i, zeta_j),
    F_i = (f, v_i),  Phi_i = (phi, zeta_i),  E(psi)_i = (exp(-psi_h), zeta_i).
Gradient (Sec. 4.2, eq. (pG:gradient)):
    B_ij = (grad v_i, zeta_j) with zeta_j in Psi^d (component k pairs with d/dx_k),
    N(psi)_i = (phi psi_h / sqrt(1 + |psi_h|^2), zeta_i),
    [D_psi] = Frechet derivative of N,
    [E_beta]_ij = beta (grad_h eta_i, grad_h eta_j), eta in Phi_h^d (Y_n basis,
    identified index-for-index with zeta; Y_0..Y_{P-1} per direction).
Exponent guard (a reading: the paper does not say how exp(-psi) is kept
finite): exp(-psi) is evaluated as exp(min(-psi, 700)).
"""
import numpy as np
import scipy.sparse as sp

from . import basis
from .mesh import GRADIENT, OBSTACLE, kron_dirs

EXP_CAP = 700.0


class RefTables:
    """1-D reference tables at the q Gauss-Legendre nodes (degree p, P psi
    modes per direction); from a uniform mesh or given explicitly."""

    def __init__(self, mesh=None, p=None, P=None, q=None):
        if mesh is not None:
            p, P, q = mesh.p, mesh.P, mesh.q
        self.y, self.w = basis.gauss_legendre(q)
        V, D = basis.u_local(p, self.y)
        self.Vu = V.T                        # (q, p+1)
        self.Du = D.T                        # (q, p+1), d/dy
        self.Vpsi = basis.legendre(P - 1, self.y).T          # (q, P)
        self.Y = basis.spectral_galerkin(P - 1, self.y).T     # (q, P)
        self.dY = basis.spectral_galerkin_deriv(P - 1, self.y).T


def _cell_tables(mesh, ref, cidx):
    """d-D evaluation tables for one cell: values, physical gradients, weights."""
    d = mesh.d
    hs = mesh.cell_widths(cidx)
    J = np.prod([0.5 * hk for hk in hs])
    W = J * kron_dirs([ref.w[None, :]] * d).reshape(-1)
    Vu = kron_dirs([ref.Vu] * d)
    Gu = []
    for k in range(d):
        tabs = [ref.Vu] * d
        tabs = list(tabs)
        tabs[k] = ref.Du * (2.0 / hs[k])
        Gu.append(kron_dirs(tabs))
    Vpsi = kron_dirs([ref.Vpsi] * d)
    return W, Vu, Gu, Vpsi, hs


class _Coo:
    def __init__(self):
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, block):
        rr, cc = np.meshgrid(rows, cols, indexing="ij")
        keep = (rr >= 0) & (cc >= 0)
        self.r.append(rr[keep])
        self.c.append(cc[keep])
        self.v.append(block[keep])

    def csr(self, shape):
        if not self.r:
            return sp.csr_matrix(shape)
        return sp.coo_matrix((np.concatenate(self.v),
                              (np.concatenate(self.r), np.concatenate(self.c))),
                             shape=shape).tocsr()


class System:
    """The parameter-independent pieces of the hpG saddle system."""

    def __init__(self, mesh, f_qp, phi_qp):
        self.mesh = mesh
        self._refs = {}
        self.ref = None if getattr(mesh, "hp", False) else RefTables(mesh)
        f_qp = np.asarray(f_qp, dtype=np.float64).reshape(-1)
        phi_qp = np.asarray(phi_qp, dtype=np.float64).reshape(-1)
        if f_qp.size != mesh.n_qp or phi_qp.size != mesh.n_qp:
            raise ValueError("f and phi must be given at the n_qp quadrature points")
        self.f_qp, self.phi_qp = f_qp, phi_qp
        self._assemble()

    def ref_for(self, cno):
        """Reference tables of a cell (cached per degree)."""
        key = self.mesh.cell_p(cno)
        if key not in self._refs:
            self._refs[key] = RefTables(p=key[0], P=key[1], q=key[2])
        return self._refs[key]

    def _assemble(self):
        mesh = self.mesh
        d, nc = mesh.d, mesh.ncomp
        cA, cB, cMu, cMpsi, cEg = _Coo(), _Coo(), _Coo(), _Coo(), _Coo()
        F = np.zeros(mesh.n_u)
        Phi = np.zeros(mesh.n_psi)
        self.cells = []
        self.cell_refs = []
        for cno, cidx in mesh.cells():
            ref = self.ref_for(cno)
            W, Vu, Gu, Vpsi, hs = _cell_tables(mesh, ref, cidx)
            ug = mesh.u_dofs(cidx)
            pg = mesh.psi_dofs(cno)
            fq = self.f_qp[mesh.qp_slice(cno)]
            phq = self.phi_qp[mesh.qp_slice(cno)]
            A_K = sum(G.T @ (W[:, None] * G) for G in Gu)
            cA.add(ug, ug, A_K)
            cMu.add(ug, ug, Vu.T @ (W[:, None] * Vu))
            Mpsi_1 = Vpsi.T @ (W[:, None] * Vpsi)
            Fk = Vu.T @ (W * fq)
            keep = ug >= 0
            np.add.at(F, ug[keep], Fk[keep])
            if mesh.kind == OBSTACLE:
                cB.add(ug, pg, Vu.T @ (W[:, None] * Vpsi))
                cMpsi.add(pg, pg, Mpsi_1)
                Phi[pg] = Vpsi.T @ (W * phq)
            else:
                nP = Vpsi.shape[1]
                Bblk = np.hstack([G.T @ (W[:, None] * Vpsi) for G in Gu])
                cB.add(ug, pg, Bblk)
                cMpsi.add(pg, pg, np.kron(np.eye(nc), Mpsi_1))
                # Y-basis broken gradient stiffness (E_beta of Sec. 4.2)
                hsY = hs
                Ytabs = []
                for k in range(d):
                    tabs = [ref.Y] * d
                    tabs[k] = ref.dY * (2.0 / hsY[k])
                    Ytabs.append(kron_dirs(tabs))
                EY = sum(T.T @ (W[:, None] * T) for T in Ytabs)
                cEg.add(pg, pg, np.kron(np.eye(nc), EY))
                Phi[pg] = np.tile(Vpsi.T @ (W * phq), nc)
                assert nP == mesh.P ** d
            self.cells.append((cno, cidx, W, Vpsi, pg, phq))
            self.cell_refs.append(ref)
        self.A = cA.csr((mesh.n_u, mesh.n_u))
        self.B = cB.csr((mesh.n_u, mesh.n_psi))
        self.Mu = cMu.csr((mesh.n_u, mesh.n_u))
        self.Mpsi = cMpsi.csr((mesh.n_psi, mesh.n_psi))
        self.F = F
        self.Phi = Phi
        if mesh.kind == OBSTACLE:
            self.Ebeta_unit = self.Mpsi
        else:
            self.Ebeta_unit = cEg.csr((mesh.n_psi, mesh.n_psi))

    # ---- nonlinear terms ---------------------------------------------------
    def psi_at_points(self, psi):
        """psi_h at every quadrature point, shape (n_cells, ncomp, Q) (a list
        of (ncomp, Q_K) arrays when the degree varies by cell)."""
        mesh = self.mesh
        out = []
        for cno, cidx, W, Vpsi, pg, phq in self.cells:
            c = psi[pg].reshape(mesh.ncomp, Vpsi.shape[1])
            out.append(c @ Vpsi.T)
        return out if getattr(mesh, "hp", False) else np.array(out)

    def nonlinear(self, psi):
        """Obstacle: E(psi) of eq. (pG).  Gradient: N(psi) of eq. (pG:gradient)."""
        mesh = self.mesh
        out = np.zeros(mesh.n_psi)
        for cno, cidx, W, Vpsi, pg, phq in self.cells:
            nP = Vpsi.shape[1]
            c = psi[pg].reshape(mesh.ncomp, nP)
            pq = c @ Vpsi.T                      # (ncomp, Q)
            if mesh.kind == OBSTACLE:
                e = np.exp(np.minimum(-pq[0], EXP_CAP))
                out[pg] = Vpsi.T @ (W * e)
            else:
                s = 1.0 + np.sum(pq * pq, axis=0)
                flux = phq * pq / np.sqrt(s)         # (ncomp, Q)
                out[pg] = np.concatenate([Vpsi.T @ (W * flux[k]) for k in range(mesh.ncomp)])
        return out

    def Dpsi(self, psi):
        """Jacobian block D_psi (sparse, cell-block diagonal)."""
        mesh = self.mesh
        coo = _Coo()
        nc = mesh.ncomp
        for cno, cidx, W, Vpsi, pg, phq in self.cells:
            nP = Vpsi.shape[1]
            c = psi[pg].reshape(nc, nP)
            pq = c @ Vpsi.T
            if mesh.kind == OBSTACLE:
                om = W * np.exp(np.minimum(-pq[0], EXP_CAP))
                coo.add(pg, pg, Vpsi.T @ (om[:, None] * Vpsi))
            else:
                s = 1.0 + np.sum(pq * pq, axis=0)
                blk = np.zeros((nc * nP, nc * nP))
                for a in range(nc):
                    for b in range(nc):
                        Ft = (s * (a == b) - pq[a] * pq[b]) * s ** -1.5
                        om = W * phq * Ft
                        blk[a * nP:(a + 1) * nP, b * nP:(b + 1) * nP] = Vpsi.T @ (om[:, None] * Vpsi)
                coo.add(pg, pg, blk)
        return coo.csr((mesh.n_psi, mesh.n_psi))

    # ---- residual and Jacobian of the LVPP subproblem ----------------------
    def residual(self, u, psi, psi_prev, alpha):
        """(R_u, R_psi) of eq. (pG) / eq. (pG:gradient) at step size alpha."""
        Ru = alpha * (self.A @ u) + self.B @ (psi - psi_prev) - alpha * self.F
        if self.mesh.kind == OBSTACLE:
            Rpsi = self.B.T @ u + self.nonlinear(psi) - self.Phi
        else:
            Rpsi = self.B.T @ u - self.nonlinear(psi)
        return Ru, Rpsi

    def jacobian(self, psi, alpha, beta):
        """G of eq. (pG-matrix): [[alpha A, B], [B^T, -D_psi - E_beta]]."""
        br = -(self.Dpsi(psi) + beta * self.Ebeta_unit)
        return sp.bmat([[alpha * self.A, self.B], [self.B.T, br]], format="csc")

    # ---- function-space helpers ---------------------------------------------
    def l2_norm_u(self, u):
        return float(np.sqrt(max(u @ (self.Mu @ u), 0.0)))

    def grad_u_at_points(self, u):
        """Physical gradient of u_h at every quadrature point, shape (n_qp, d)."""
        mesh = self.mesh
        out = np.zeros((mesh.n_qp, mesh.d))
        for cno, cidx in mesh.cells():
            W, Vu, Gu, Vpsi, hs = _cell_tables(mesh, self.ref_for(cno), cidx)
            ug = mesh.u_dofs(cidx)
            loc = np.where(ug >= 0, u[np.maximum(ug, 0)], 0.0)
            for k in range(mesh.d):
                out[mesh.qp_slice(cno), k] = Gu[k] @ loc
        return out

    def u_at_points(self, u):
        mesh = self.mesh
        out = np.zeros(mesh.n_qp)
        for cno, cidx in mesh.cells():
            Vu = kron_dirs([self.ref_for(cno).Vu] * mesh.d)
            ug = mesh.u_dofs(cidx)
            loc = np.where(ug >= 0, u[np.maximum(ug, 0)], 0.0)
            out[mesh.qp_slice(cno)] = Vu @ loc
        return out
