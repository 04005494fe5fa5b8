"""Pins of the oracle's multi-dimensional gradient-constraint assembly
(paper Sec. 4.2, eq. (pG:gradient): B_ij = (grad v_i, zeta_j) with zeta_j in
Psi_h^d, component k of zeta paired with d/dx_k).

Three checks that do not go through the assembly they test:
1. B^T u for a u_h known in closed form (an anisotropic polynomial that lies
   in U_h) equals the moments (d u / d x_k, P_a(x_0) P_b(x_1) ...)_K computed
   here from the analytic gradient with NumPy's Gauss-Legendre rule and
   Legendre series.
2. Each cell block of B equals the tensor product of the 1-D closed forms
   (v_l', P_a)_K = -2/(2a+1) delta_{a, n+1} (bubble W_n, from W_n' = -P_{n+1}),
   -/+ delta_{a0} (left / right hat) and (v_l, P_a)_K (Sec. 3 closed forms).
3. A 2-D gradient solve with data symmetric under x <-> y and x -> 1 - x
   returns u with those symmetries and psi components that map into each
   other as the components of grad u do.
Each check is also run on mutated copies of B (components swapped, one
component's sign flipped) and must reject them."""
import numpy as np
import pytest
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

from oracle import assemble, lvpp, mesh as M
import workloads as W


def _poly_u(d):
    """u = prod_k a_k(x_k) with a different cubic factor per direction
    (vanishing at 0 and 1), its gradient and -Laplacian."""
    facs = [np.array([0.0, 2.0, -1.0, -1.0]),      # x(1-x)(2+x)
            np.array([0.0, 1.0, -1.0]),            # x(1-x)
            np.array([0.0, 1.0, 2.0, -3.0])]       # x(1-x)(1+3x)
    facs = facs[:d]
    val = lambda c, x: np.polynomial.polynomial.polyval(x, c)
    der = [np.polynomial.polynomial.polyder(c) for c in facs]
    der2 = [np.polynomial.polynomial.polyder(c, 2) for c in facs]

    def u(x):
        return np.prod([val(facs[k], x[:, k]) for k in range(d)], axis=0)

    def grad(x):
        out = np.zeros_like(x)
        for k in range(d):
            t = val(der[k], x[:, k])
            for j in range(d):
                if j != k:
                    t = t * val(facs[j], x[:, j])
            out[:, k] = t
        return out

    def mlap(x):
        s = np.zeros(x.shape[0])
        for k in range(d):
            t = val(der2[k], x[:, k])
            for j in range(d):
                if j != k:
                    t = t * val(facs[j], x[:, j])
            s -= t
        return s

    return u, grad, mlap


def _grad_system(breaks, p, f=None, phi=None):
    ms = M.TensorMesh(breaks, p, M.GRADIENT)
    x = ms.quadrature_points()
    fv = f(x) if f is not None else np.ones(ms.n_qp)
    pv = phi(x) if phi is not None else np.full(ms.n_qp, 0.3)
    return assemble.System(ms, fv, pv)


def _moments_from_gradient(mesh, grad):
    """(d u / d x_k, P_a0(y_0) P_a1(y_1) ...)_K per cell, component-major,
    Legendre index 0 fastest, with NumPy's Gauss rule (exact here)."""
    d, P = mesh.d, mesh.P
    yq, wq = npleg.leggauss(mesh.p + 3)
    out = np.zeros(mesh.n_psi)
    eye = np.eye(P)
    Pv = np.array([npleg.legval(yq, eye[a]) for a in range(P)])   # (P, nq)
    for cno, cidx in mesh.cells():
        axes, wts = [], []
        for k in range(d):
            x0 = mesh.breaks[k][cidx[k]]
            hk = mesh.h[k][cidx[k]]
            axes.append(x0 + 0.5 * (yq + 1.0) * hk)
            wts.append(0.5 * hk * wq)
        grids = np.meshgrid(*axes, indexing="ij")
        pts = np.stack([g.reshape(-1) for g in grids], axis=1)    # index 0 slowest
        wgt = np.ones(1)
        for k in range(d):
            wgt = np.multiply.outer(wgt, wts[k]).reshape(-1) if k else wts[0]
        g = grad(pts)
        base = cno * mesh.psi_per_cell
        for comp in range(d):
            for j in range(P ** d):
                aa = [(j // P ** k) % P for k in range(d)]
                zeta = np.ones(pts.shape[0])
                for k in range(d):
                    zeta = zeta * np.repeat(np.tile(Pv[aa[k]], len(yq) ** k),
                                            len(yq) ** (d - 1 - k))
                out[base + comp * P ** d + j] = np.sum(wgt * g[:, comp] * zeta)
    return out


def _mutations(sysm):
    """B with the two first components swapped, and with component 0 negated."""
    mesh = sysm.mesh
    n = mesh.P ** mesh.d
    perm = np.arange(mesh.n_psi)
    sign = np.ones(mesh.n_psi)
    for c in range(mesh.n_cells):
        b = c * mesh.psi_per_cell
        perm[b:b + n], perm[b + n:b + 2 * n] = np.arange(b + n, b + 2 * n), np.arange(b, b + n)
        sign[b:b + n] = -1.0
    B = sysm.B.tocsc()
    return {"swap": B[:, perm].tocsr(), "sign": (B @ sp.diags(sign)).tocsr()}


CASES = [
    ([np.array([0.0, 0.3, 1.0]), np.array([0.0, 0.45, 0.8, 1.0])], 3),
    ([np.array([0.0, 0.6, 1.0]), np.array([0.0, 0.25, 1.0]), np.array([0.0, 0.5, 1.0])], 3),
]


@pytest.mark.parametrize("breaks,p", CASES)
def test_gradient_B_moments_of_an_exact_polynomial(breaks, p):
    d = len(breaks)
    u, grad, mlap = _poly_u(d)
    sysm = _grad_system(breaks, p, f=mlap)
    mesh = sysm.mesh
    # u lies in U_h (degree <= 3 <= p per direction, zero on the boundary), so
    # the Galerkin solution with f = -Laplace(u) reproduces it exactly
    import scipy.sparse.linalg as spla
    c = spla.spsolve(sysm.A.tocsc(), sysm.F)
    xq = mesh.quadrature_points()
    assert np.max(np.abs(sysm.u_at_points(c) - u(xq))) < 1e-12
    assert np.max(np.abs(sysm.grad_u_at_points(c) - grad(xq))) < 1e-11
    ref = _moments_from_gradient(mesh, grad)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(sysm.B.T @ c - ref)) < 1e-12 * scale
    for name, Bm in _mutations(sysm).items():
        err = np.max(np.abs(Bm.T @ c - ref))
        assert err > 1e-2 * scale, name


def _closed_form_1d(p, h):
    """(v_l', P_a)_K and (v_l, P_a)_K on a cell of width h, l = 0 (left hat),
    1..p-1 (bubbles W_0..W_{p-2}), p (right hat); a = 0..p-1 (gradient: P = p)."""
    L, P = p + 1, p
    der = np.zeros((L, P))
    val = np.zeros((L, P))
    der[0, 0], der[p, 0] = -1.0, 1.0
    val[0, 0], val[p, 0] = h / 2.0, h / 2.0
    if P > 1:
        val[0, 1], val[p, 1] = -h / 6.0, h / 6.0
    for n in range(p - 1):
        if n + 1 < P:
            der[1 + n, n + 1] = -2.0 / (2 * (n + 1) + 1)
        for a in range(P):
            v = (2.0 * (a == n) / (2 * n + 1) - 2.0 * (a == n + 2) / (2 * n + 5)) / (2 * n + 3)
            val[1 + n, a] = 0.5 * h * v
    return der, val


def _kron_block(mesh, cidx):
    d = mesh.d
    tabs = [_closed_form_1d(mesh.p, mesh.h[k][cidx[k]]) for k in range(d)]
    blocks = []
    for comp in range(d):
        mats = [tabs[k][0] if k == comp else tabs[k][1] for k in range(d)]
        blocks.append(M.kron_dirs(mats))
    return np.hstack(blocks)


@pytest.mark.parametrize("breaks,p", CASES + [([np.array([0.0, 0.4, 1.0])] * 2, 4)])
def test_gradient_B_is_the_tensor_product_of_1d_closed_forms(breaks, p):
    sysm = _grad_system(breaks, p)
    mesh = sysm.mesh

    def worst(B):
        Bd = B.toarray()
        e = 0.0
        for cno, cidx in mesh.cells():
            ug = mesh.u_dofs(cidx)
            keep = ug >= 0
            pg = mesh.psi_dofs(cno)
            # psi columns belong to one cell, so B restricted to them is
            # that cell's block alone
            blk = _kron_block(mesh, cidx)
            e = max(e, np.max(np.abs(Bd[np.ix_(ug[keep], pg)] - blk[keep])))
        return e

    assert worst(sysm.B) < 1e-13
    for name, Bm in _mutations(sysm).items():
        assert worst(Bm) > 1e-2, name


def _mirror_maps(m, p):
    """Permutation and signs of the 1-D unknowns under x -> 1 - x on m uniform
    cells (hat of vertex v -> vertex m - v; W_n of cell c -> (-1)^n W_n of
    cell m - 1 - c), and of the Legendre modes (P_a -> (-1)^a P_a)."""
    n1 = m * p - 1
    perm = np.zeros(n1, dtype=int)
    sgn = np.ones(n1)
    for v in range(1, m):
        perm[v * p - 1] = (m - v) * p - 1
    for c in range(m):
        for n in range(p - 1):
            perm[c * p + n] = (m - 1 - c) * p + n
            sgn[c * p + n] = (-1.0) ** n
    return perm, sgn


def _symmetry_errors(sysm, u, psi):
    mesh = sysm.mesh
    m, p, P = mesh.m[0], mesh.p, mesh.P
    n1 = mesh.n1[0]
    U = u.reshape(n1, n1)                       # U[j, i]: direction 0 fastest
    pm, sg = _mirror_maps(m, p)
    e_swap = np.max(np.abs(U - U.T))
    Um = np.zeros_like(U)
    Um[:, pm] = U * sg[None, :]                 # u(1 - x, y)
    e_mirror = np.max(np.abs(Um - U))
    # psi[cell (cx, cy), comp, (ay, ax)]
    Ps = psi.reshape(m, m, 2, P, P)             # [cy, cx, comp, ay, ax]
    # x <-> y maps component 0 to component 1 with cells and modes transposed
    e_pswap = np.max(np.abs(Ps[:, :, 0] - np.transpose(Ps[:, :, 1], (1, 0, 3, 2))))
    # x -> 1 - x: cell cx -> m-1-cx, mode ax -> (-1)^ax; component 0 (d/dx) flips sign
    sa = (-1.0) ** np.arange(P)
    Pm = Ps[:, ::-1] * sa[None, None, None, None, :]
    e_pmir = max(np.max(np.abs(Pm[:, :, 0] + Ps[:, :, 0])), np.max(np.abs(Pm[:, :, 1] - Ps[:, :, 1])))
    return e_swap, e_mirror, e_pswap, e_pmir


def test_gradient_solve_has_the_symmetries_of_the_data():
    m, p = 4, 3
    br = [np.linspace(0.0, 1.0, m + 1)] * 2
    f = W.const(20.0)
    phi = lambda x: 0.25 + 0.5 * ((x[:, 0] - 0.5) ** 2 + (x[:, 1] - 0.5) ** 2)
    sysm = _grad_system(br, p, f=f, phi=phi)
    opts = lvpp.Options(alpha0=2.0 ** -3, alpha_factor=2.0 ** 0.5, alpha_max=4.0, fixed_steps=8)
    r = lvpp.solve(sysm, opts)
    assert r.converged
    # the constraint is active somewhere (otherwise psi would carry no information)
    assert np.max(np.abs(r.psi)) > 0.1
    errs = _symmetry_errors(sysm, r.u, r.psi)
    scale = max(np.max(np.abs(r.u)), np.max(np.abs(r.psi)))
    assert max(errs) < 1e-9 * scale, errs
    # with a mutated coupling the solve returns (u, S psi) for the matching
    # component permutation or sign change S, which breaks the psi symmetries
    # (a negated component fails the x <-> y map, swapped ones the mirror)
    for name, Bm in _mutations(sysm).items():
        sysm.B = Bm
        r2 = lvpp.solve(sysm, opts)
        errs2 = _symmetry_errors(sysm, r2.u, r2.psi)
        assert max(errs2[2:]) > 1e-3 * scale, (name, errs2)


def test_max_violation_gradient_of_a_known_function():
    # u = x(1-x)y(1-y)(2+x)-type product: |grad u| at the Gauss points is known
    breaks = CASES[0][0]
    u, grad, mlap = _poly_u(2)
    sysm = _grad_system(breaks, 3, f=mlap, phi=W.const(0.05))
    import scipy.sparse.linalg as spla
    c = spla.spsolve(sysm.A.tocsc(), sysm.F)
    xq = sysm.mesh.quadrature_points()
    want = np.max(np.sqrt(np.sum(grad(xq) ** 2, axis=1)) - 0.05)
    assert abs(lvpp.max_violation_gradient(sysm, c) - want) < 1e-12
