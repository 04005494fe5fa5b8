"""Pins of the oracle's LVPP solve against closed forms, a brute-force QP and
invariants of the method (paper Sec. 2 and Sec. 4)."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble, lvpp, mesh as M
import workloads as W

A_FB = 3.0 / np.sqrt(220.0)   # free boundary of the 1-D workload, sqrt(0.225/5.5)


def u_star_obstacle_1d(x):
    """Closed form for f = 10, phi = 0.1 + 0.5 (x - 1/2)^2 on (0,1):
    u = -5 x^2 + (11 a - 1/2) x on [0, a], u = phi on [a, 1-a], mirrored."""
    x = np.asarray(x)
    xx = np.minimum(x, 1.0 - x)
    return np.where(xx <= A_FB, -5 * xx ** 2 + (11 * A_FB - 0.5) * xx, 0.1 + 0.5 * (x - 0.5) ** 2)


def solve(breaks, p, f, phi, kind=M.OBSTACLE, **kw):
    ms = M.TensorMesh(breaks, p, kind)
    x = ms.quadrature_points()
    s = assemble.System(ms, f(x), phi(x))
    return s, lvpp.solve(s, lvpp.Options(**kw)), x


def aligned_breaks():
    a = A_FB
    return [np.concatenate([np.linspace(0, a, 4), np.linspace(a, 1 - a, 9)[1:],
                            np.linspace(1 - a, 1, 4)[1:]])]


@pytest.mark.parametrize("p", [2, 3, 5])
def test_closed_form_obstacle_aligned_mesh(p):
    # with breakpoints at a, 1-a the exact solution is in U_h and lambda* = -11
    # (contact) / 0 lies in Psi_h, so the LVPP limit is u* itself
    f, phi = W.w1d()
    s, r, x = solve(aligned_breaks(), p, f, phi)
    assert r.converged
    err = np.max(np.abs(s.u_at_points(r.u) - u_star_obstacle_1d(x[:, 0])))
    assert err < 1e-9
    # lambda -> -11 on contact cells, 0 elsewhere (its P_0 coefficient)
    lam0 = r.lam.reshape(s.mesh.n_cells, -1)[:, 0]
    centres = 0.5 * (aligned_breaks()[0][1:] + aligned_breaks()[0][:-1])
    contact = (centres > A_FB) & (centres < 1 - A_FB)
    assert np.allclose(lam0[contact], -11.0, atol=1e-7)
    assert np.allclose(lam0[~contact], 0.0, atol=1e-7)
    cr, rel = lvpp.complementarity(s, r.psi, r.lam)
    assert rel < 1e-8


def test_closed_form_obstacle_uniform_rate():
    # uniform meshes do not align with a: the H^1 error is O(h^{3/2}) (Sec. 6.1,
    # u in H^{5/2-eps}); where a falls inside its cell makes single-step rates
    # oscillate, so pin the constant err * m^{3/2} and the overall decrease.
    f, phi = W.w1d()
    errs = []
    ms_list = (16, 32, 64, 128, 256, 512)
    for m in ms_list:
        ms = M.uniform_mesh(1, m, 4)
        x = ms.quadrature_points()
        s = assemble.System(ms, f(x), phi(x))
        r = lvpp.solve(s, lvpp.Options())
        # H^1 seminorm error by a finer Gauss rule on each cell
        from oracle import basis
        y, w = basis.gauss_legendre(12)
        V, D = basis.u_local(4, y)
        e2 = 0.0
        for cno, cidx in ms.cells():
            h = ms.h[0][cidx[0]]
            g = ms.u_dofs(cidx)
            loc = np.where(g >= 0, r.u[np.maximum(g, 0)], 0.0)
            xx = ms.breaks[0][cidx[0]] + 0.5 * (y + 1) * h
            du = (D.T @ loc) * 2 / h
            dstar = np.where(xx <= A_FB, -10 * xx + 11 * A_FB - 0.5,
                             np.where(xx >= 1 - A_FB, 10 * (1 - xx) - 11 * A_FB + 0.5, xx - 0.5))
            e2 += np.sum(w * (du - dstar) ** 2) * h / 2
        errs.append(np.sqrt(e2))
    errs = np.array(errs)
    assert np.all(errs * np.array(ms_list) ** 1.5 < 1.0), errs
    assert errs[-1] < errs[0] / 32, errs


def test_closed_form_gradient_1d():
    # |u'| <= phi, f = 10, phi = 1: u*' = clamp(f (1/2 - x), -phi, phi), kinks
    # at 1/2 -+ phi/f = 0.4, 0.6.  On a mesh aligned with the kinks the LVPP
    # limit is u*.
    br = [np.array([0.0, 0.2, 0.4, 0.5, 0.6, 0.8, 1.0])]
    f, phi = W.const(10.0), W.const(1.0)
    s, r, x = solve(br, 3, f, phi, kind=M.GRADIENT, max_prox=80)
    assert r.converged
    xx = x[:, 0]
    ustar = np.where(xx <= 0.4, xx, np.where(xx >= 0.6, 1 - xx,
                                               0.4 + 5 * xx - 5 * xx ** 2 - 1.2))
    assert np.max(np.abs(s.u_at_points(r.u) - ustar)) < 1e-8


def _qp_by_enumeration(H, g):
    """min 1/2 mu^T H mu - g^T mu over mu >= 0 by checking every active set."""
    n = len(g)
    best, best_mu = np.inf, None
    for mask in itertools.product([0, 1], repeat=n):
        idx = np.flatnonzero(mask)
        mu = np.zeros(n)
        if idx.size:
            mu[idx] = np.linalg.solve(H[np.ix_(idx, idx)], g[idx])
        if np.any(mu < -1e-12):
            continue
        grad = H @ mu - g
        if np.any(grad[mu <= 1e-14] < -1e-10):
            continue
        val = 0.5 * mu @ H @ mu - g @ mu
        if val < best:
            best, best_mu = val, mu
    return best_mu


def _qp_by_pgs(H, g, sweeps=20000):
    mu = np.zeros(len(g))
    for _ in range(sweeps):
        for i in range(len(g)):
            mu[i] = max(0.0, mu[i] + (g[i] - H[i] @ mu) / H[i, i])
    return mu


@pytest.mark.parametrize("d,m", [(1, 6), (1, 8), (2, 3)])
def test_p2_reduces_to_polyhedral_qp(d, m):
    # At p = 2, psi is piecewise constant and (exp(-psi), 1)_K = |K| exp(-psi_K) > 0,
    # so the LVPP limit solves min 1/2 u^T A u - F^T u s.t. B^T u <= Phi (cell
    # means).  Its dual over mu >= 0 is solved by brute force.
    f = lambda x: 40.0 * np.sin(np.pi * np.atleast_2d(x)[:, 0]) + 10.0
    phi = lambda x: 0.03 + 0.2 * np.sum((np.atleast_2d(x) - 0.45) ** 2, axis=1)
    ms = M.uniform_mesh(d, m, 2)
    x = ms.quadrature_points()
    s = assemble.System(ms, f(x), phi(x))
    r = lvpp.solve(s, lvpp.Options())
    assert r.converged
    A = s.A.toarray()
    B = s.B.toarray()
    AinvB = np.linalg.solve(A, B)
    AinvF = np.linalg.solve(A, s.F)
    H = B.T @ AinvB
    g = B.T @ AinvF - s.Phi
    mu_e = _qp_by_enumeration(H, g)
    mu_p = _qp_by_pgs(H, g)
    assert np.allclose(mu_e, mu_p, atol=1e-9)
    u_qp = AinvF - AinvB @ mu_e
    assert np.linalg.norm(r.u - u_qp) <= 1e-9 * np.linalg.norm(u_qp)
    assert np.allclose(-r.lam, mu_e, atol=1e-7 * max(1, np.abs(mu_e).max()))
    assert np.any(mu_e > 1e-6)     # the constraint is active somewhere


def test_beta_independence():
    # E_beta only enters the Jacobian (Sec. 4.1), so the converged iterates do
    # not depend on it.  A larger beta turns Newton into a slowly converging
    # quasi-Newton once D_psi -> 0 on contact cells, so use the Sec. 6.1 value.
    f, phi = W.w2d(0)
    ms = M.uniform_mesh(2, 4, 4)
    x = ms.quadrature_points()
    s = assemble.System(ms, f(x), phi(x))
    r0 = lvpp.solve(s, lvpp.Options(beta=0.0, fixed_steps=8))
    r1 = lvpp.solve(s, lvpp.Options(beta=1e-8, fixed_steps=8, max_newton=200))
    assert r0.converged and r1.converged
    assert np.linalg.norm(r0.u - r1.u) <= 1e-11 * np.linalg.norm(r0.u)
    assert np.linalg.norm(r0.psi - r1.psi) <= 1e-11 * np.linalg.norm(r0.psi)


@pytest.mark.parametrize("kind", [M.OBSTACLE, M.GRADIENT])
def test_unconstrained_limit(kind):
    # an inactive constraint leaves the plain Galerkin solution A u = F
    f, _ = W.w1d()
    phi = W.const(10.0) if kind == M.OBSTACLE else W.const(100.0)
    for d, m, p in ((1, 16, 4), (2, 4, 3)):
        ms = M.uniform_mesh(d, m, p, kind)
        x = ms.quadrature_points()
        s = assemble.System(ms, f(x), phi(x))
        r = lvpp.solve(s, lvpp.Options(max_prox=80))
        assert r.converged
        u0 = spla.spsolve(s.A.tocsc(), s.F)
        assert np.linalg.norm(r.u - u0) <= 1e-10 * np.linalg.norm(u0)


def test_symmetry_1d_and_3d():
    # data symmetric under x -> 1 - x (and the cube group in 3-D) give symmetric u
    f, phi = W.w1d()
    s, r, x = solve([np.linspace(0, 1, 17)], 4, f, phi)
    uq = s.u_at_points(r.u)
    # quadrature points are symmetric about 1/2: reversing the order mirrors them
    assert np.allclose(uq, uq[::-1], atol=1e-12)
    f3, phi3 = W.w3d()
    s3, r3, x3 = solve([np.linspace(0, 1, 4)] * 3, 2, f3, phi3)
    uq3 = s3.u_at_points(r3.u)
    key = np.round(x3, 12)
    perm_sets = [key[:, [1, 0, 2]], key[:, [2, 1, 0]], 1 - key]
    lookup = {tuple(k): i for i, k in enumerate(key)}
    for pk in perm_sets:
        j = np.array([lookup[tuple(np.round(k, 12))] for k in pk])
        assert np.allclose(uq3, uq3[j], atol=1e-10)


def test_feasibility_and_complementarity_1d_workload():
    # 1-D workload, 16 uniform cells, p = 4: u~ = phi - exp(-psi) <= phi by construction,
    # moment feasibility B^T u + E(psi) = Phi, complementarity below 1e-8
    f, phi = W.w1d()
    s, r, x = solve([np.linspace(0, 1, 17)], 4, f, phi)
    assert r.converged
    Ru, Rpsi = s.residual(r.u, r.psi, r.psi, 1.0)
    assert np.linalg.norm(Rpsi) <= 1e-10 * np.linalg.norm(s.Phi)
    cr, rel = lvpp.complementarity(s, r.psi, r.lam)
    assert rel < 1e-8
    # pointwise violation is at most the discretisation error of this mesh
    assert lvpp.max_violation(s, r.u) < 1e-3
