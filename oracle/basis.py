"""One-dimensional polynomial bases and quadrature (paper Sec. 3).

Test infrastructure only (see ``oracle/__init__.py``).

* Legendre P_n on [-1, 1] by the three-term recurrence; orthogonality
  (P_n, P_m) = 2 delta_nm / (2n+1) is the property Sec. 3 quotes.
* Bubbles W_n of eq. (Wn): (1 - x^2) P_n^{(1,1)}(x) / (2(n+1)), built from the
  Jacobi P^{(1,1)} recurrence, i.e. from the paper's definition.  The paper
  fixes the normalisation by W_n' = -P_{n+1}; the derivative below uses that
  stated property, and the tests check it against the Jacobi values.
* Hats on the reference cell: (1 - y)/2 (left vertex), (1 + y)/2 (right).
* Spectral-Galerkin Y_n = P_n - P_{n+2} (Sec. 3, last paragraph).
* Gauss-Legendre nodes/weights by Golub-Welsch (eigen-decomposition of the
  Legendre Jacobi matrix), polished by Newton steps on P_q.
"""
import numpy as np


def legendre(nmax, y):
    """Rows n = 0..nmax of P_n(y); shape (nmax+1, len(y))."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros((nmax + 1,) + y.shape)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = y
    for n in range(1, nmax):
        # (n+1) P_{n+1} = (2n+1) y P_n - n P_{n-1}
        out[n + 1] = ((2 * n + 1) * y * out[n] - n * out[n - 1]) / (n + 1)
    return out


def legendre_deriv(nmax, y):
    """Rows n = 0..nmax of P_n'(y) via P'_{n+1} = P'_{n-1} + (2n+1) P_n."""
    P = legendre(nmax, y)
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(P)
    if nmax >= 1:
        out[1] = 1.0
    for n in range(1, nmax):
        out[n + 1] = out[n - 1] + (2 * n + 1) * P[n]
    return out


def jacobi11(nmax, y):
    """Rows n = 0..nmax of the Jacobi polynomials P_n^{(1,1)}(y).

    Recurrence for alpha = beta = 1:
        n (n+2) P_n = (2n+1)(n+1) y P_{n-1} - n (n+1) P_{n-2},
    with P_0 = 1, P_1 = 2y.
    """
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros((nmax + 1,) + y.shape)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = 2.0 * y
    for n in range(2, nmax + 1):
        out[n] = ((2 * n + 1) * (n + 1) * y * out[n - 1]
                  - n * (n + 1) * out[n - 2]) / (n * (n + 2))
    return out


def bubbles(nmax, y):
    """Rows n = 0..nmax of W_n(y) = (1 - y^2) P_n^{(1,1)}(y) / (2(n+1)), eq. (Wn)."""
    y = np.asarray(y, dtype=np.float64)
    J = jacobi11(nmax, y)
    n = np.arange(nmax + 1).reshape((-1,) + (1,) * y.ndim)
    return (1.0 - y * y) * J / (2.0 * (n + 1))


def bubbles_deriv(nmax, y):
    """Rows n = 0..nmax of W_n'(y) = -P_{n+1}(y) (normalisation stated under eq. (Wn))."""
    return -legendre(nmax + 1, y)[1:]


def spectral_galerkin(nmax, y):
    """Rows n = 0..nmax of Y_n(y) = P_n(y) - P_{n+2}(y) (Sec. 3)."""
    P = legendre(nmax + 2, y)
    return P[: nmax + 1] - P[2: nmax + 3]


def spectral_galerkin_deriv(nmax, y):
    dP = legendre_deriv(nmax + 2, y)
    return dP[: nmax + 1] - dP[2: nmax + 3]


def gauss_legendre(q):
    """q-point Gauss-Legendre rule on [-1, 1]: (nodes ascending, weights).

    Golub-Welsch: the nodes are the eigenvalues of the symmetric tridiagonal
    Jacobi matrix of the Legendre recurrence, off-diagonal k / sqrt(4k^2 - 1);
    weight_j = 2 * (first eigenvector component)^2.  Two Newton steps on P_q
    polish the nodes; weights then follow from 2 / ((1 - x^2) P_q'(x)^2).
    """
    if q < 1:
        raise ValueError("q >= 1")
    if q == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, q, dtype=np.float64)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    T = np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(T)
    for _ in range(2):
        P = legendre(q, x)
        dP = legendre_deriv(q, x)
        x = x - P[q] / dP[q]
    dP = legendre_deriv(q, x)[q]
    w = 2.0 / ((1.0 - x * x) * dP * dP)
    order = np.argsort(x)
    return x[order], w[order]


def u_local(p, y):
    """Local U_{h,p} basis on the reference cell, rows l = 0..p.

    l = 0: left hat (1 - y)/2; l = p: right hat (1 + y)/2;
    l = 1..p-1: bubble W_{l-1}(y).  Returns (values, d/dy values).
    """
    y = np.asarray(y, dtype=np.float64)
    V = np.zeros((p + 1,) + y.shape)
    D = np.zeros((p + 1,) + y.shape)
    V[0] = 0.5 * (1.0 - y)
    D[0] = -0.5
    V[p] = 0.5 * (1.0 + y)
    D[p] = 0.5
    if p >= 2:
        V[1:p] = bubbles(p - 2, y)
        D[1:p] = bubbles_deriv(p - 2, y)
    return V, D
