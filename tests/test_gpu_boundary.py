"""GPU tests of the boundary's solve options and statistics.

* warm start / resume (Sec. 2.1: subproblem k depends only on psi_{k-1}): a
  solve resumed from (u_k0, psi_k0, k0) returns bit for bit what the
  uninterrupted FP64 solve returns;
* the per-solve diagnostics (complementarity sums with lambda_K, pointwise
  violation at the Gauss points) against the oracle's definitions evaluated
  on the same returned iterate;
* the point-function data setters against the array setters;
* option validation (q, krylov, warm start);
* the mixed path's FP64 recomputation counts and their caps;
* hpg_server_destroy with a caller blocked on a queued request."""
import threading

import numpy as np
import pytest

from oracle import assemble, lvpp, mesh as OM
from oracle.hpmesh import HpMesh
import workloads as W

from gpu_common import build_pair, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _hpg():
    from paper_2412_13733_amd import hpg
    return hpg


RESUME_CASES = [
    (1, 16, 4, "obstacle", 0),
    (2, 6, 4, "obstacle", 0),
    (3, 3, 3, "obstacle", 0),
    (2, 4, 3, "gradient", 0),
    (2, 6, 4, "obstacle", 1),
]


def _data(dim, kind):
    if kind == "gradient":
        # the sine family (seed 3) with a positive varying phi, as in the
        # gradient parity tests
        phi = lambda x: 0.2 + 0.3 * np.sum((np.atleast_2d(x) - 0.4) ** 2, axis=1)
        return W.sine_forcing(3)[0], phi
    return W.w1d() if dim == 1 else (W.w2d(0) if dim == 2 else W.w3d())


def _opts(kind, precision, **kw):
    hpg = _hpg()
    base = dict(precision=precision)
    if precision == hpg.MIXED:
        base.update(newton_tol=1e-10, krylov_rtol=1e-6)
    if kind == "gradient":
        base.update(alpha0=2.0 ** -5, alpha_factor=2.0 ** 0.5, alpha_max=4.0)
    base.update(kw)
    return hpg.default_opts(**base)


@pytest.mark.parametrize("dim,m,p,kind,precision", RESUME_CASES)
def test_resume_equals_uninterrupted_solve(dim, m, p, kind, precision):
    hpg = _hpg()
    okind = OM.GRADIENT if kind == "gradient" else OM.OBSTACLE
    log("resume", dim, m, p, kind, precision)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim, kind), kind=okind)
    K, k0 = 7, 3
    u, psi, lam, st = prob.solve(_opts(kind, precision, fixed_prox_steps=K), want_lambda=True)
    u0, psi0, _, st0 = prob.solve(_opts(kind, precision, fixed_prox_steps=k0))
    u1, psi1, lam1, st1 = prob.solve(_opts(kind, precision, fixed_prox_steps=K), want_lambda=True,
                                     warm=(u0, psi0, k0))
    log("  full", st.as_dict(), "\n  resumed", st1.as_dict())
    assert st.status == 0 and st0.status == 0 and st1.status == 0
    assert st1.prox_steps == K and st0.prox_steps == k0
    if precision == hpg.FP64 or (st.fp64_recomputations == 0 and st0.fp64_recomputations == 0):
        assert np.array_equal(u1, u) and np.array_equal(psi1, psi) and np.array_equal(lam1, lam)
        assert st0.newton_iters + st1.newton_iters == st.newton_iters
    else:
        assert sysm.l2_norm_u(u1 - u) <= 1e-8 * sysm.l2_norm_u(u)


def test_resume_with_adaptive_stop():
    # no fixed count: the outer stop of the resumed solve compares u_{k0+1}
    # with warm_u, so it stops at the same step as the uninterrupted solve
    mesh, prob, sysm = build_pair(1, 16, 4, W.w1d())
    hpg = _hpg()
    u, psi, lam, st = prob.solve(hpg.default_opts(), want_lambda=True)
    u0, psi0, _, st0 = prob.solve(hpg.default_opts(fixed_prox_steps=4))
    u1, psi1, lam1, st1 = prob.solve(hpg.default_opts(), want_lambda=True, warm=(u0, psi0, 4))
    assert st1.prox_steps == st.prox_steps
    assert np.array_equal(u1, u) and np.array_equal(psi1, psi) and np.array_equal(lam1, lam)


def _check_diagnostics(sysm, u, psi, lam, st, gradient=False):
    if gradient:
        mv = lvpp.max_violation_gradient(sysm, u)
        assert st.complementarity == 0.0 and st.complementarity_rel == 0.0
    else:
        mv = lvpp.max_violation(sysm, u)
        cr, crel = lvpp.complementarity(sysm, psi, lam)
        log("  complementarity gpu", st.complementarity, "oracle", cr, "rel", crel)
        # the sums weigh |lambda_h| where lambda_h nearly cancels (off the
        # contact set): compare in units of the normaliser ||lambda||_L1 ||phi||_inf
        unit = cr / crel if crel > 0 else 1.0
        assert abs(st.complementarity - cr) <= 1e-13 * unit
        assert abs(st.complementarity_rel - crel) <= 1e-13
    log("  max violation gpu", st.max_violation, "oracle", mv)
    scale = max(np.max(np.abs(sysm.phi_qp)), 1.0)
    assert abs(st.max_violation - mv) <= 1e-13 * scale


DIAG_CASES = [
    (1, 16, 4, "obstacle"),
    (2, 6, 4, "obstacle"),
    (2, 9, 3, "obstacle"),
    (3, 3, 3, "obstacle"),
    (2, 4, 3, "gradient"),
    (3, 2, 2, "gradient"),
]


@pytest.mark.parametrize("dim,m,p,kind", DIAG_CASES)
def test_solve_diagnostics_match_the_oracle_definitions(dim, m, p, kind):
    okind = OM.GRADIENT if kind == "gradient" else OM.OBSTACLE
    log("diagnostics", dim, m, p, kind)
    mesh, prob, sysm = build_pair(dim, m, p, _data(dim, kind), kind=okind)
    u, psi, lam, st = prob.solve(_opts(kind, 0, fixed_prox_steps=6), want_lambda=True)
    assert st.status == 0
    _check_diagnostics(sysm, u, psi, lam, st, gradient=kind == "gradient")


def test_converged_obstacle_solve_is_complementary():
    # the paper's limit: lambda exp(-psi) -> 0; with alpha_k = 2^k to the
    # 1e-10 outer tolerance the relative complementarity is far below 1e-8
    mesh, prob, sysm = build_pair(2, 8, 4, W.w2d(0))
    u, psi, lam, st = prob.solve(_hpg().default_opts(), want_lambda=True)
    log("  stats", st.as_dict())
    assert st.status == 0 and st.complementarity_rel < 1e-8
    _check_diagnostics(sysm, u, psi, lam, st)


def test_hp_diagnostics_match_the_oracle_definitions():
    hpg = _hpg()
    breaks = [W.uniform_breaks(4), np.array([0.0, 0.2, 0.5, 0.75, 1.0])]
    deg = np.random.default_rng(5).integers(2, 7, 16)
    f, phi = W.w2d(0)
    mesh = hpg.Mesh(2, [4, 4], 0, breaks=breaks, degree=deg)
    x = mesh.quadrature_points()
    prob = hpg.Problem(mesh)
    prob.set_forcing(f(x))
    prob.set_obstacle(phi(x))
    om = HpMesh(breaks, deg)
    xo = om.quadrature_points()
    sysm = assemble.System(om, f(xo), phi(xo))
    u, psi, lam, st = prob.solve(hpg.default_opts(fixed_prox_steps=5), want_lambda=True)
    assert st.status == 0
    _check_diagnostics(sysm, u, psi, lam, st)


def test_point_function_setters_equal_array_setters():
    hpg = _hpg()
    f, phi = W.w2d(0)
    mesh = hpg.Mesh(2, [5, 5], 3)
    x = mesh.quadrature_points()
    a = hpg.Problem(mesh)
    a.set_forcing(f(x))
    a.set_obstacle(phi(x))
    b = hpg.Problem(mesh)
    b.set_forcing_fn(lambda pt: f(pt[None, :])[0])
    b.set_obstacle_fn(lambda pt: phi(pt[None, :])[0])
    o = hpg.default_opts(fixed_prox_steps=4)
    ua, pa, _, _ = a.solve(o)
    ub, pb, _, _ = b.solve(o)
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb)
    with pytest.raises(hpg.HpgError) as e:
        b.set_obstacle_fn(lambda pt: float("nan"))
    assert e.value.status == hpg.ERR_NUMERIC


def test_option_validation():
    hpg = _hpg()
    mesh, prob, sysm = build_pair(1, 4, 3, W.w1d())
    u, psi, _, st = prob.solve(hpg.default_opts(q=4, fixed_prox_steps=2))   # q = p + 1
    assert st.status == 0
    bad = [dict(q=3), dict(q=5), dict(krylov=1), dict(k0=2), dict(k0=-1)]
    for kw in bad:
        with pytest.raises(hpg.HpgError) as e:
            prob.solve(hpg.default_opts(fixed_prox_steps=3, **kw))
        assert e.value.status == hpg.ERR_INVALID_ARG, kw
    with pytest.raises(hpg.HpgError) as e:   # k0 at the step cap
        prob.solve(hpg.default_opts(fixed_prox_steps=3), warm=(u, psi, 3))
    assert e.value.status == hpg.ERR_INVALID_ARG


def test_mixed_recomputation_caps():
    # a Krylov cap below what the FP32 solves need makes every FP32 direction
    # hit it, so each is recomputed in FP64 (itself capped, an inexact Newton
    # direction): three per proximal step, after which that step's directions
    # are FP64 from the start, and twelve over the solve, after which every
    # direction is.  Every subproblem takes at least three Newton steps, so
    # the count is exactly twelve and every direction is an FP64 one; the
    # inexact directions still converge to the same subproblem solutions.
    hpg = _hpg()
    mesh, prob, sysm = build_pair(2, 8, 4, W.w2d(0))
    ro = lvpp.solve(sysm, lvpp.Options())
    o = hpg.default_opts(fixed_prox_steps=ro.prox_steps, precision=hpg.MIXED, newton_tol=1e-10,
                         krylov_rtol=1e-6, max_krylov=15, max_newton=100)
    u, psi, lam, st = prob.solve(o, want_lambda=True)
    log("  stats", st.as_dict())
    assert st.status == 0
    assert st.fp64_recomputations == 12
    # after the twelfth, directions are FP64 from the start (counted as
    # fallbacks, not recomputations)
    assert st.fp64_recomputations < st.fp64_fallbacks <= st.newton_iters
    assert sysm.l2_norm_u(u - ro.u) <= 1e-8 * sysm.l2_norm_u(ro.u)
    # one proximal step with a cap no FP32 solve meets: three recomputations,
    # then every later direction of the step in FP64 (the counts hold whether
    # or not the step converges within its Newton cap)
    o1 = hpg.default_opts(fixed_prox_steps=1, precision=hpg.MIXED, newton_tol=1e-10,
                          krylov_rtol=1e-6, max_krylov=5, max_newton=30)
    _, _, _, s1 = prob.solve(o1)
    log("  one step", s1.as_dict())
    assert s1.fp64_recomputations == 3
    assert s1.fp64_fallbacks == s1.newton_iters


def test_server_destroy_wakes_a_waiter_on_a_queued_request():
    hpg = _hpg()
    srv = hpg.Server(device=0, max_slots=1)
    f, phi = W.w2d(0)
    meshes = [hpg.Mesh(2, [16, 16], 6), hpg.Mesh(2, [4, 4], 3)]
    tickets = []
    for ms in meshes:
        x = ms.quadrature_points()
        tickets.append(srv.submit(ms, f(x), phi(x), hpg.default_opts()))
    out = {}

    def waiter():
        try:
            out["res"] = srv.wait(tickets[1])
        except hpg.HpgError as e:
            out["err"] = e

    th = threading.Thread(target=waiter)
    th.start()
    srv.close()   # the second request is still queued behind the first
    th.join(timeout=120)
    assert not th.is_alive()
    # either it ran before destroy took the queue, or it failed as dropped
    assert "res" in out or (out["err"].status == hpg.ERR_INVALID_ARG
                            and "destroyed" in str(out["err"]))
