"""Latent-variable proximal point loop with Newton and sparse LU (paper Sec. 2, 4).

Test infrastructure only (see ``oracle/__init__.py``).

For k = 1, 2, ...: given alpha_k and psi_{k-1} (psi_0 = 0), solve the hpG
subproblem eq. (pG) (or eq. (pG:gradient)) for (u_k, psi_k) by Newton's
method, each step solving G delta = -R with G from eq. (pG-matrix) by a
direct sparse LU of the assembled saddle matrix (the strategy the paper
reports as surprisingly good at the start of Sec. 4.4).  Then
lambda_k = (psi_{k-1} - psi_k) / alpha_k (Sec. 2.1).

Readings where the paper is silent (shared with the GPU path):
* alpha schedule: alpha_k = alpha0 * factor^(k-1) (configured workloads use
  alpha0 = factor = 2, i.e. alpha_k = 2^k).
* Newton initial guess: the previous proximal iterate (u_{k-1}, psi_{k-1}).
* Newton stop: ||R_u||_2 / (alpha ||F||_2) + ||R_psi||_2 / s_psi <= tol,
  s_psi = ||Phi||_2 with Phi_i = (phi, zeta_i) (times sqrt(d) for the
  gradient variant, whose Phi is replicated per component).
* Globalisation (the paper only cites a line-search package): backtracking
  on the merit ||(R_u / alpha, R_psi)||_2: t = 1, halve while
  merit(x + t delta) > (1 - 1e-4 t) merit(x), at most 30 halvings.  If no
  step is accepted the residual has reached its rounding floor or Newton has
  failed: the subproblem counts as converged when the Newton error is then
  already <= stall_tol (1e-9), and as failed otherwise.
* Outer stop: ||u_k - u_{k-1}||_{L2} <= tol_prox ||u_k||_{L2}, or k = max_prox,
  or exactly ``fixed_steps`` proximal steps when that is given.
* E_beta enters the Jacobian only (Sec. 4.1: not needed for well-posedness),
  so the computed iterates do not depend on beta.
"""
import time

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import EXP_CAP, System
from .mesh import OBSTACLE


class Options:
    def __init__(self, alpha0=2.0, alpha_factor=2.0, alpha_max=np.inf,
                 max_prox=60, tol_prox=1e-10, newton_tol=1e-12, max_newton=60,
                 beta=0.0, fixed_steps=0, max_halvings=30, stall_tol=1e-9):
        self.alpha0 = alpha0
        self.alpha_factor = alpha_factor
        self.alpha_max = alpha_max
        self.max_prox = max_prox
        self.tol_prox = tol_prox
        self.newton_tol = newton_tol
        self.max_newton = max_newton
        self.beta = beta
        self.fixed_steps = fixed_steps
        self.max_halvings = max_halvings
        self.stall_tol = stall_tol


class Result:
    pass


def _scales(system):
    mesh = system.mesh
    sF = max(np.linalg.norm(system.F), 1e-300)
    sP = max(np.linalg.norm(system.Phi), 1e-300)
    return sF, sP


def newton_error(system, Ru, Rpsi, alpha):
    sF, sP = _scales(system)
    return np.linalg.norm(Ru) / (alpha * sF) + np.linalg.norm(Rpsi) / sP


def merit(Ru, Rpsi, alpha):
    return float(np.sqrt(np.dot(Ru, Ru) / alpha ** 2 + np.dot(Rpsi, Rpsi)))


def newton_subproblem(system, u, psi, psi_prev, alpha, opts, stats):
    """Solve one LVPP subproblem from (u, psi); returns (u, psi, converged)."""
    n_u = system.mesh.n_u
    for it in range(opts.max_newton + 1):
        Ru, Rpsi = system.residual(u, psi, psi_prev, alpha)
        err = newton_error(system, Ru, Rpsi, alpha)
        if not np.isfinite(err):
            return u, psi, False
        if err <= opts.newton_tol:
            return u, psi, True
        if it == opts.max_newton:
            return u, psi, False
        t0 = time.perf_counter()
        G = system.jacobian(psi, alpha, opts.beta)
        lu = spla.splu(G)
        delta = -lu.solve(np.concatenate([Ru, Rpsi]))
        stats.lu_seconds += time.perf_counter() - t0
        stats.newton += 1
        du, dpsi = delta[:n_u], delta[n_u:]
        m0 = merit(Ru, Rpsi, alpha)
        t = 1.0
        accepted = False
        for _ in range(opts.max_halvings + 1):
            ut, pt = u + t * du, psi + t * dpsi
            Rut, Rpt = system.residual(ut, pt, psi_prev, alpha)
            if merit(Rut, Rpt, alpha) <= (1.0 - 1e-4 * t) * m0:
                accepted = True
                break
            t *= 0.5
        if not accepted:
            return u, psi, bool(err <= opts.stall_tol)
        u, psi = ut, pt
    return u, psi, False


def solve(system, opts=None):
    """Run the LVPP loop; returns a Result with u, psi, lam and counts."""
    opts = opts or Options()
    mesh = system.mesh
    u = np.zeros(mesh.n_u)
    psi = np.zeros(mesh.n_psi)
    psi_prev = np.zeros(mesh.n_psi)
    res = Result()
    res.newton = 0
    res.lu_seconds = 0.0
    res.converged = True
    res.alphas = []
    t0 = time.perf_counter()
    alpha = opts.alpha0
    k = 0
    lam = np.zeros(mesh.n_psi)
    kmax = opts.fixed_steps if opts.fixed_steps else opts.max_prox
    while k < kmax:
        k += 1
        u_old = u
        u, psi, ok = newton_subproblem(system, u, psi, psi_prev, alpha, opts, res)
        res.alphas.append(alpha)
        if not ok:
            res.converged = False
            break
        lam = (psi_prev - psi) / alpha
        psi_prev = psi.copy()
        if not opts.fixed_steps:
            du = system.l2_norm_u(u - u_old)
            if du <= opts.tol_prox * system.l2_norm_u(u):
                break
        alpha = min(alpha * opts.alpha_factor, opts.alpha_max)
    res.u, res.psi, res.lam = u, psi, lam
    res.prox_steps = k
    res.seconds = time.perf_counter() - t0
    return res


# ---- diagnostics: feasibility and complementarity (readings of how the paper's
# feasible and complementary iterates are measured on the discrete level) -----
def complementarity(system, psi, lam):
    """CR = sum_K sum_q w |J| |lambda_h(x_q)| exp(-psi_h(x_q)), and its relative
    form CR / (||lambda||_{L1,h} ||phi||_inf) (obstacle only)."""
    cr, l1 = 0.0, 0.0
    # cell by cell: the number of Gauss points may differ between cells
    for cell, lq, pq in zip(system.cells, system.psi_at_points(lam),
                            system.psi_at_points(psi)):
        W = cell[2]
        e = np.exp(np.minimum(-pq[0], EXP_CAP))
        cr += float(np.sum(W * np.abs(lq[0]) * e))
        l1 += float(np.sum(W * np.abs(lq[0])))
    rel = cr / max(l1 * np.max(np.abs(system.phi_qp)), 1e-300)
    return cr, rel


def max_violation(system, u):
    """max over quadrature points of u_h - phi (pointwise feasibility at the
    Gauss points, a reading of the constraint u <= phi on the discrete level)."""
    return float(np.max(system.u_at_points(u) - system.phi_qp))


def max_violation_gradient(system, u):
    """max over quadrature points of |grad u_h| - phi (the gradient constraint
    |grad u| <= phi at the Gauss points)."""
    g = system.grad_u_at_points(u)
    return float(np.max(np.sqrt(np.sum(g * g, axis=1)) - system.phi_qp))
