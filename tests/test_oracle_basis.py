"""Pins of the oracle's 1-D bases and quadrature against what the paper and
the mathematics fix (Sec. 3 of the paper)."""
import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("q", [1, 2, 3, 5, 7, 13, 20])
def test_gauss_legendre_exact_on_monomials(q):
    # a q-point Gauss rule integrates x^k exactly for k <= 2q - 1
    x, w = basis.gauss_legendre(q)
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14 * max(1.0, q / 4)
    # and not at degree 2q: the nodes are the roots of P_q, so the rule gives 0
    # for (P_q, P_q) = 2/(2q+1) (guards against a rule with the wrong nodes)
    Pq = basis.legendre(q, x)[q]
    assert abs(np.dot(w, Pq * Pq)) < 1e-13


@pytest.mark.parametrize("q", [2, 5, 9, 16])
def test_gauss_legendre_matches_library(q):
    x, w = basis.gauss_legendre(q)
    xl, wl = np.polynomial.legendre.leggauss(q)
    assert np.max(np.abs(x - xl)) < 1e-15
    assert np.max(np.abs(w - wl)) < 1e-14


def test_legendre_against_closed_forms():
    y = np.linspace(-1, 1, 11)
    P = basis.legendre(4, y)
    assert np.allclose(P[2], 0.5 * (3 * y ** 2 - 1), atol=1e-15)
    assert np.allclose(P[3], 0.5 * (5 * y ** 3 - 3 * y), atol=1e-15)
    assert np.allclose(P[4], (35 * y ** 4 - 30 * y ** 2 + 3) / 8, atol=1e-15)
    assert np.allclose(basis.legendre(4, np.array([1.0]))[:, 0], 1.0)
    assert np.allclose(basis.legendre(4, np.array([-1.0]))[:, 0], [1, -1, 1, -1, 1])
    dP = basis.legendre_deriv(4, y)
    assert np.allclose(dP[3], 0.5 * (15 * y ** 2 - 3), atol=1e-14)


def test_legendre_orthogonality():
    # (P_n, P_m) = 2 delta_nm / (2n + 1)  (Sec. 3)
    x, w = basis.gauss_legendre(20)
    P = basis.legendre(15, x)
    G = (P * w) @ P.T
    assert np.allclose(G, np.diag(2.0 / (2 * np.arange(16) + 1)), atol=1e-14)


def test_bubble_definition_and_derivative():
    # eq. (Wn) with the stated normalisation W_n' = -P_{n+1}: check the Jacobi
    # definition against W_n(x) = -int_{-1}^x P_{n+1}(t) dt computed by an exact
    # Gauss rule on [-1, x], and against the Legendre form (P_n - P_{n+2})/(2n+3).
    n_max = 12
    xs = np.linspace(-1, 1, 17)
    W = basis.bubbles(n_max, xs)
    t, wt = basis.gauss_legendre(n_max + 2)
    for j, x in enumerate(xs):
        tt = -1 + (t + 1) * (x + 1) / 2
        integ = -(basis.legendre(n_max + 1, tt)[1:] @ wt) * (x + 1) / 2
        assert np.allclose(W[:, j], integ, atol=1e-14)
    P = basis.legendre(n_max + 2, xs)
    n = np.arange(n_max + 1)[:, None]
    assert np.allclose(W, (P[:-2] - P[2:]) / (2 * n + 3), atol=1e-14)
    # boundary values vanish
    assert np.allclose(basis.bubbles(n_max, np.array([-1.0, 1.0])), 0.0, atol=1e-15)
    # derivative table is -P_{n+1}; check one case with a finite difference
    h = 1e-6
    fd = (basis.bubbles(n_max, xs + h) - basis.bubbles(n_max, xs - h)) / (2 * h)
    inner = slice(1, -1)
    assert np.allclose(fd[:, inner], basis.bubbles_deriv(n_max, xs)[:, inner], atol=1e-7)


def test_spectral_galerkin_is_rescaled_bubble():
    # Y_n = P_n - P_{n+2} vanishes at +-1 and equals (2n+3) W_n (Sec. 3)
    xs = np.linspace(-1, 1, 9)
    Y = basis.spectral_galerkin(10, xs)
    W = basis.bubbles(10, xs)
    n = np.arange(11)[:, None]
    assert np.allclose(Y, (2 * n + 3) * W, atol=1e-13)
    assert np.allclose(basis.spectral_galerkin(10, np.array([-1.0, 1.0])), 0.0, atol=1e-14)
    # derivative of Y_n is -(2n+3) P_{n+1}
    dY = basis.spectral_galerkin_deriv(10, xs)
    assert np.allclose(dY, -(2 * n + 3) * basis.legendre(11, xs)[1:], atol=1e-12)


def test_u_local_hats():
    V, D = basis.u_local(4, np.array([-1.0, 0.0, 1.0]))
    assert np.allclose(V[0], [1, 0.5, 0]) and np.allclose(V[4], [0, 0.5, 1])
    assert np.allclose(D[0], -0.5) and np.allclose(D[4], 0.5)
    assert np.allclose(V[1:4][:, [0, 2]], 0.0)
