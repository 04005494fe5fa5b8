"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/hpg.h declares, and its host-only calls (mesh, DOF counts,
quadrature points, argument validation) behave as documented.  No kernel is
launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2412_13733_amd import hpg
from oracle import mesh as OM

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "hpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(hpg_[A-Za-z_0-9]+)\s*\(", src)
    return sorted(set(n for n in names))


def test_library_exports_every_declared_symbol():
    lib = hpg.load()
    declared = header_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(hpg.EXPORTS) == declared


@pytest.mark.parametrize("dim,m,p", [(1, 16, 4), (2, 5, 6), (3, 3, 2), (2, 7, 3)])
def test_mesh_info_and_counts(dim, m, p):
    mesh = hpg.Mesh(dim, [m] * dim, p)
    n1 = m * p - 1
    assert mesh.n_u == n1 ** dim
    assert mesh.n_psi == m ** dim * (p - 1) ** dim
    assert mesh.n_qp == m ** dim * (p + 1) ** dim
    om = OM.uniform_mesh(dim, m, p)
    assert (om.n_u, om.n_psi, om.n_qp) == (mesh.n_u, mesh.n_psi, mesh.n_qp)


@pytest.mark.parametrize("dim,p", [(1, 4), (2, 3), (3, 2)])
def test_quadrature_points_match_oracle(dim, p):
    br = [np.array([0.0, 0.13, 0.5, 1.0]), np.array([0.0, 0.7, 1.0]), np.array([0.0, 0.25, 1.0])][:dim]
    mesh = hpg.Mesh(dim, [len(b) - 1 for b in br], p, breaks=br)
    x = mesh.quadrature_points()
    xo = OM.TensorMesh(br, p).quadrature_points()
    assert np.max(np.abs(x - xo)) < 2e-16 * 4


def test_invalid_arguments_are_rejected():
    with pytest.raises(hpg.HpgError) as e:
        hpg.Mesh(2, [4, 4], 1)                  # obstacle needs p >= 2
    assert e.value.status == hpg.ERR_INVALID_ARG
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(4, [2, 2, 2, 2], 3)            # d <= 3
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(1, [0], 3)                      # at least one cell
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(1, [2], 3, breaks=[np.array([0.0, 0.7, 0.6])])   # not increasing
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(1, [2], 3, breaks=[np.array([0.0, 0.5, 2.0])])   # must end at 1
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(2, [1, 3], 1, constraint=hpg.GRADIENT)   # p = 1 on one cell: no u unknown
    assert hpg.Mesh(1, [2], 1, constraint=hpg.GRADIENT).n_u == 1
    m = hpg.Mesh(1, [3], 2, constraint=hpg.GRADIENT)
    assert m.P == 2 and m.n_psi == 3 * 2


def test_footprint_estimate_is_host_only_and_monotone():
    from paper_2412_13733_amd import hpg
    small = hpg.Mesh(2, [8, 8], 4)
    big = hpg.Mesh(2, [32, 32], 4)
    hi_p = hpg.Mesh(2, [8, 8], 8)
    f64, f32 = small.footprint(hpg.FP64), small.footprint(hpg.MIXED)
    # a mixed solve also reserves the FP64 buffers of the steps it recomputes in FP64
    assert 0 < f64 < f32
    assert big.footprint(hpg.FP64) > f64
    assert hi_p.footprint(hpg.FP64) > f64
    # at least the FP64 Newton state and Krylov vectors
    assert f64 > 8 * 15 * (small.n_u + small.n_psi)
    with pytest.raises(hpg.HpgError):
        small.footprint(7)


def test_gradient_footprint_counts_component_blocks():
    from paper_2412_13733_amd import hpg
    ob = hpg.Mesh(2, [8, 8], 4)
    gr = hpg.Mesh(2, [8, 8], 4, constraint=hpg.GRADIENT)
    assert gr.n_psi == 8 * 8 * 2 * 16      # d components of P^d = p^d modes per cell
    # psi blocks (d P^d)^2 per cell dominate the difference
    assert gr.footprint(hpg.FP64) - ob.footprint(hpg.FP64) > 8 * 64 * (32 * 32 - 9 * 9)


def test_per_cell_degree_mesh_matches_the_oracle_numbering_sizes():
    # host-only: unknown counts and Gauss points of hp meshes against the oracle
    from oracle.hpmesh import HpMesh
    rng = np.random.default_rng(3)
    for d, m in ((1, 6), (2, 4), (3, 2)):
        deg = rng.integers(2, 8, size=m ** d)
        br = [np.sort(np.r_[0.0, rng.uniform(0.05, 0.95, m - 1), 1.0]) for _ in range(d)]
        g = hpg.Mesh(d, [m] * d, 0, breaks=br, degree=deg)
        o = HpMesh(br, deg)
        assert (g.n_u, g.n_psi, g.n_qp, g.p) == (o.n_u, o.n_psi, o.n_qp, int(deg.max()))
        assert np.max(np.abs(g.quadrature_points() - o.quadrature_points())) < 1e-15
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(2, [2, 2], 0, constraint=hpg.GRADIENT, degree=[2, 2, 2, 2])
    with pytest.raises(hpg.HpgError):
        hpg.Mesh(2, [2, 2], 0, degree=[2, 1, 3, 2])
    a = hpg.Mesh(2, [16, 16], 0, degree=np.full(256, 6))
    b = hpg.Mesh(2, [16, 16], 0, degree=np.r_[np.full(128, 6), np.full(128, 3)])
    assert a.footprint(0) > b.footprint(0) > 0


def test_solve_options_struct_matches_the_library():
    # the binding's hpg_solve_opts layout must be the library's: the size field
    # hpg_default_opts writes is sizeof(hpg_solve_opts) in C, and every field
    # keeps its documented default
    o = hpg.default_opts()
    assert o.size == ctypes.sizeof(hpg.SolveOpts)
    assert (o.alpha0, o.alpha_factor, o.max_prox, o.max_newton, o.max_krylov) == (2.0, 2.0, 60, 60, 2000)
    assert (o.newton_tol, o.krylov_rtol, o.beta, o.precision) == (1e-12, 1e-10, 0.0, hpg.FP64)
    assert (o.krylov_chunk, o.inexact_newton, o.step_extension) == (16, 0, 0)
