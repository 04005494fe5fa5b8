"""Tensor-product meshes with one degree per cell (obstacle constraint).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 3 builds U_{h,p} from the integrated-Legendre hierarchy (hats and the
bubbles W_n of eq. (Wn)) and lets the degree vary from cell to cell; its
multi-dimensional spaces are tensor products of 1-D hp spaces.  A degree per
cell that is the same in every direction (p_K) is not such a tensor product;
the conforming space used here (reading: the minimum rule) is

* every mesh entity (vertex, edge, face, cell interior) carries the degree
  p_E = min p_K over the cells K that contain it;
* a cell-local function prod_k phi_{l_k}(y_k) (l_k = 0: left hat, l_k = p_K:
  right hat, else bubble W_{l_k - 1}) belongs to the entity picked out by
  which factors are hats; the global function exists iff every bubble mode
  n_k = l_k - 1 satisfies n_k <= p_E - 2 and the entity is not on the boundary
  (homogeneous Dirichlet data).

Because the bubbles and hats are the same functions in every cell, the traces
on a shared entity agree and the space is H^1-conforming; for equal degrees
it is U_{0,h,p} of the uniform mesh (with a different numbering).

Numbering (a convention of this implementation): entities are the points of
the doubled grid e = (e_0, ..., e_{d-1}), e_k in 0..2 m_k (even: vertex
coordinate e_k / 2; odd: cell interval (e_k - 1) / 2); interior entities are
numbered lexicographically with direction 0 fastest, and inside an entity its
functions are numbered by the bubble modes of its odd directions, the first
odd direction fastest, each mode in 0..p_E - 2.  psi (Legendre, degree p_K - 2
per direction, P_K = p_K - 1) is cell-major with P_K^d values per cell; the
quadrature points are cell-major with q_K = p_K + 1 points per direction.
"""
import itertools

import numpy as np

from . import basis
from .mesh import OBSTACLE


class HpMesh:
    hp = True

    def __init__(self, breaks, degrees, kind=OBSTACLE):
        if kind != OBSTACLE:
            raise ValueError("per-cell degrees: obstacle constraint only")
        self.breaks = [np.asarray(b, dtype=np.float64) for b in breaks]
        self.d = len(self.breaks)
        if self.d not in (1, 2, 3):
            raise ValueError("d must be 1, 2 or 3")
        for b in self.breaks:
            if len(b) < 2 or np.any(np.diff(b) <= 0):
                raise ValueError("breakpoints must be strictly increasing")
        self.kind = kind
        self.m = [len(b) - 1 for b in self.breaks]
        self.h = [np.diff(b) for b in self.breaks]
        self.n_cells = int(np.prod(self.m))
        self.deg = np.asarray(degrees, dtype=np.int64).reshape(-1)
        if self.deg.size != self.n_cells or np.any(self.deg < 2):
            raise ValueError("one degree >= 2 per cell")
        self.ncomp = 1
        self._entities()
        Pk = self.deg - 1
        qk = self.deg + 1
        self.psi_off = np.concatenate([[0], np.cumsum(Pk ** self.d)])
        self.qp_off = np.concatenate([[0], np.cumsum(qk ** self.d)])
        self.n_psi = int(self.psi_off[-1])
        self.n_qp = int(self.qp_off[-1])
        self.psi_per_cell = None

    # ---- cells -------------------------------------------------------------
    def cells(self):
        ranges = [range(mm) for mm in reversed(self.m)]
        for k, rev in enumerate(itertools.product(*ranges)):
            yield k, tuple(reversed(rev))

    def cell_number(self, cidx):
        c, st = 0, 1
        for k in range(self.d):
            c += cidx[k] * st
            st *= self.m[k]
        return c

    def cell_widths(self, cidx):
        return [self.h[k][cidx[k]] for k in range(self.d)]

    def cell_p(self, cno):
        p = int(self.deg[cno])
        return p, p - 1, p + 1

    # ---- entities ----------------------------------------------------------
    def _containing_cells(self, e):
        """Cell multi-indices containing the entity at doubled position e."""
        opts = []
        for k in range(self.d):
            if e[k] % 2:
                opts.append([(e[k] - 1) // 2])
            else:
                v = e[k] // 2
                opts.append([c for c in (v - 1, v) if 0 <= c < self.m[k]])
        return list(itertools.product(*opts))

    def _entities(self):
        shape = [2 * mk + 1 for mk in self.m]
        self.ent_deg = {}
        self.ent_base = {}
        n = 0
        ranges = [range(s) for s in reversed(shape)]
        for rev in itertools.product(*ranges):
            e = tuple(reversed(rev))
            if any(e[k] == 0 or e[k] == 2 * self.m[k] for k in range(self.d)):
                continue
            pe = min(int(self.deg[self.cell_number(c)]) for c in self._containing_cells(e))
            nodd = sum(ek % 2 for ek in e)
            self.ent_deg[e] = pe
            self.ent_base[e] = n
            n += (pe - 1) ** nodd
        self.n_u = n

    def entity_dofs(self, e):
        pe = self.ent_deg[e]
        nodd = sum(ek % 2 for ek in e)
        return np.arange(self.ent_base[e], self.ent_base[e] + (pe - 1) ** nodd)

    # ---- DOF maps ----------------------------------------------------------
    def u_dofs(self, cidx):
        """Global unknowns of the (p_K+1)^d local functions (local multi-index,
        direction 0 fastest); -1 where the function is absent."""
        p = int(self.deg[self.cell_number(cidx)])
        L = p + 1
        out = np.full(L ** self.d, -1, dtype=np.int64)
        for j in range(L ** self.d):
            l = [(j // L ** k) % L for k in range(self.d)]
            e, modes = [], []
            for k in range(self.d):
                if l[k] == 0:
                    e.append(2 * cidx[k])
                elif l[k] == p:
                    e.append(2 * cidx[k] + 2)
                else:
                    e.append(2 * cidx[k] + 1)
                    modes.append(l[k] - 1)
            e = tuple(e)
            if e not in self.ent_base:
                continue
            pe = self.ent_deg[e]
            if any(nm > pe - 2 for nm in modes):
                continue
            idx, st = 0, 1
            for nm in modes:
                idx += nm * st
                st *= pe - 1
            out[j] = self.ent_base[e] + idx
        return out

    def psi_dofs(self, cno):
        return np.arange(self.psi_off[cno], self.psi_off[cno + 1], dtype=np.int64)

    def qp_slice(self, cno):
        return slice(int(self.qp_off[cno]), int(self.qp_off[cno + 1]))

    def u_groups(self):
        """Blocks of the A-preconditioner: all vertex unknowns (the Q1 space),
        then the unknowns of each edge / face / interior entity."""
        verts, rest = [], []
        for e in self.ent_base:
            if all(ek % 2 == 0 for ek in e):
                verts.append(self.ent_base[e])
            else:
                rest.append(self.entity_dofs(e))
        return [np.array(sorted(verts), dtype=np.int64)] + rest

    # ---- quadrature --------------------------------------------------------
    def quadrature_points(self):
        pts = np.zeros((self.n_qp, self.d))
        for cno, cidx in self.cells():
            q = int(self.deg[cno]) + 1
            y, _ = basis.gauss_legendre(q)
            axes = []
            for k in range(self.d):
                x0 = self.breaks[k][cidx[k]]
                hk = self.h[k][cidx[k]]
                axes.append(x0 + 0.5 * (y + 1.0) * hk)
            grid = np.meshgrid(*axes, indexing="ij")
            sl = self.qp_slice(cno)
            for k in range(self.d):
                pts[sl, k] = np.transpose(grid[k]).reshape(-1)
        return pts
