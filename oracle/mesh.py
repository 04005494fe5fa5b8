"""Tensor-product meshes and the spaces U_{0,h,p}, Psi_{h,p} (paper Sec. 3).

Test infrastructure only (see ``oracle/__init__.py``).

Mesh: in each of the d directions a breakpoint vector a = x_0 < ... < x_m = b
(Sec. 3, first paragraph); cell (c_0, ..., c_{d-1}) is the box of the
per-direction intervals.  Cells are numbered lexicographically, direction 0
fastest.  One uniform partial degree p on every cell.

DOF numbering (a convention of this implementation; the paper fixes none):

* U_{0,h,p} in 1-D (m cells): the hat of interior vertex v (1 <= v <= m-1)
  is unknown v*p - 1; bubble W_n (0 <= n <= p-2) of cell c is unknown c*p + n.
  So n1 = m*p - 1 unknowns, and the d-D space (tensor product, Sec. 3) is
  numbered as the n1_0 x ... x n1_{d-1} array with direction 0 fastest.
* Psi_{h,p}: cell-major; inside a cell the Legendre multi-index (a_0, ...)
  with a_0 fastest, a_k in 0..P-1 (P = p-1 obstacle, P = p gradient).  For
  the gradient variant (Psi^d) a cell holds its d components one after the
  other (component-major).
* Quadrature points: cell-major; inside a cell the Gauss-Legendre multi-index
  with direction 0 fastest (q = p + 1 points per direction).
"""
import itertools

import numpy as np

from . import basis

OBSTACLE = "obstacle"
GRADIENT = "gradient"


class TensorMesh:
    def __init__(self, breaks, p, kind=OBSTACLE, q=None):
        self.breaks = [np.asarray(b, dtype=np.float64) for b in breaks]
        self.d = len(self.breaks)
        if self.d not in (1, 2, 3):
            raise ValueError("d must be 1, 2 or 3")
        for b in self.breaks:
            if len(b) < 2 or np.any(np.diff(b) <= 0):
                raise ValueError("breakpoints must be strictly increasing")
        self.kind = kind
        if kind == OBSTACLE and p < 2:
            raise ValueError("obstacle needs p >= 2 (psi has degree p-2)")
        if kind == GRADIENT and p < 1:
            raise ValueError("gradient constraint needs p >= 1")
        self.p = int(p)
        self.q = int(q) if q else self.p + 1
        self.P = self.p - 1 if kind == OBSTACLE else self.p
        self.m = [len(b) - 1 for b in self.breaks]
        self.h = [np.diff(b) for b in self.breaks]
        self.n1 = [mm * self.p - 1 for mm in self.m]
        self.n_u = int(np.prod(self.n1))
        self.n_cells = int(np.prod(self.m))
        self.ncomp = 1 if kind == OBSTACLE else self.d
        self.psi_per_cell = self.ncomp * self.P ** self.d
        self.n_psi = self.n_cells * self.psi_per_cell
        self.n_qp = self.n_cells * self.q ** self.d

    # ---- cells -------------------------------------------------------------
    def cells(self):
        """Yield (cell number, multi-index) with direction 0 fastest."""
        ranges = [range(mm) for mm in reversed(self.m)]
        for k, rev in enumerate(itertools.product(*ranges)):
            yield k, tuple(reversed(rev))

    def cell_widths(self, cidx):
        return [self.h[k][cidx[k]] for k in range(self.d)]

    # ---- DOF maps ----------------------------------------------------------
    def u_index_1d(self, k, c):
        """Global 1-D unknown of each local function l = 0..p of cell c in
        direction k (-1 where the function is a boundary hat)."""
        p, m = self.p, self.m[k]
        out = np.empty(p + 1, dtype=np.int64)
        out[0] = c * p - 1 if c >= 1 else -1          # hat of vertex c
        out[p] = (c + 1) * p - 1 if c + 1 <= m - 1 else -1  # hat of vertex c+1
        for n in range(p - 1):
            out[1 + n] = c * p + n                     # bubble W_n of cell c
        return out

    def u_dofs(self, cidx):
        """Global unknowns of the (p+1)^d local functions of a cell (local
        multi-index with direction 0 fastest); -1 marks a zero boundary hat."""
        idx1 = [self.u_index_1d(k, cidx[k]) for k in range(self.d)]
        stride = np.cumprod([1] + self.n1[:-1])
        glob = np.zeros(1, dtype=np.int64)
        valid = np.ones(1, dtype=bool)
        for k in range(self.d):   # build with direction 0 fastest
            g = idx1[k]
            glob = (glob[None, :] + (g[:, None] * stride[k])).reshape(-1) if k else g * stride[k]
            v = g >= 0
            valid = (valid[None, :] & v[:, None]).reshape(-1) if k else v
        glob = np.where(valid, glob, -1)
        return glob

    def psi_dofs(self, cell_no):
        s = self.psi_per_cell
        return np.arange(cell_no * s, (cell_no + 1) * s, dtype=np.int64)

    def cell_p(self, cell_no):
        """(p, P, q) of a cell: the same on every cell of this mesh."""
        return self.p, self.P, self.q

    def qp_slice(self, cell_no):
        Q = self.q ** self.d
        return slice(cell_no * Q, (cell_no + 1) * Q)

    # ---- quadrature --------------------------------------------------------
    def reference_rule(self):
        return basis.gauss_legendre(self.q)

    def quadrature_points(self):
        """(n_qp, d) physical Gauss-Legendre points, ordered as documented."""
        y, _ = self.reference_rule()
        pts = np.zeros((self.n_qp, self.d))
        Q = self.q ** self.d
        for cno, cidx in self.cells():
            axes = []
            for k in range(self.d):
                x0 = self.breaks[k][cidx[k]]
                hk = self.h[k][cidx[k]]
                axes.append(x0 + 0.5 * (y + 1.0) * hk)
            grid = np.meshgrid(*axes, indexing="ij")     # grid[k][i0, i1, ...]
            for k in range(self.d):
                # direction 0 fastest => transpose axis order before ravel
                pts[cno * Q:(cno + 1) * Q, k] = np.transpose(grid[k]).reshape(-1)
        return pts


def uniform_mesh(d, m, p, kind=OBSTACLE):
    return TensorMesh([np.linspace(0.0, 1.0, m + 1)] * d, p, kind)


def kron_dirs(tables):
    """Tensor-product table with direction 0 fastest in both row and column
    multi-indices: kron(T_{d-1}, ..., T_0)."""
    out = tables[-1]
    for T in reversed(tables[:-1]):
        out = np.kron(out, T)
    return out
