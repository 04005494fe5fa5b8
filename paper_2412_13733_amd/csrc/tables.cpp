// Host-side 1-D bases, quadrature, global 1-D rows and the generalised
// eigen-decomposition used by the fast-diagonalisation A-block inverse.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "hpg_internal.h"

namespace hpg {

// P_0..P_nmax and derivatives at y by the three-term recurrence
// (n+1)P_{n+1} = (2n+1) y P_n - n P_{n-1},  P'_{n+1} = P'_{n-1} + (2n+1) P_n.
void legendre_all(int nmax, double y, double* P, double* dP) {
    P[0] = 1.0;
    if (dP) dP[0] = 0.0;
    if (nmax >= 1) {
        P[1] = y;
        if (dP) dP[1] = 1.0;
    }
    for (int n = 1; n < nmax; ++n) {
        P[n + 1] = ((2 * n + 1) * y * P[n] - n * P[n - 1]) / (n + 1);
        if (dP) dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n];
    }
}

// Gauss-Legendre: Newton iteration on P_q from the asymptotic guesses
// cos(pi (i + 3/4) / (q + 1/2)); weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    std::vector<double> P(q + 1), dP(q + 1);
    for (int i = 0; i < q; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            legendre_all(q, t, P.data(), dP.data());
            double dt = P[q] / dP[q];
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        legendre_all(q, t, P.data(), dP.data());
        x[q - 1 - i] = t;   // ascending order
        w[q - 1 - i] = 2.0 / ((1.0 - t * t) * dP[q] * dP[q]);
    }
    if (q % 2 == 1) x[q / 2] = 0.0;
}

void RefTables::build(int p_, int P_, int q_) {
    p = p_;
    P = P_;
    q = q_;
    gauss_legendre(q, y, w);
    const int L = p + 1;
    const int nmax = std::max(p + 1, P + 2);
    std::vector<double> Pl(nmax + 1), dPl(nmax + 1);
    Vu.assign(q * L, 0.0);
    Du.assign(q * L, 0.0);
    Vpsi.assign(q * P, 0.0);
    std::vector<double> Yv(q * P), Yd(q * P);
    for (int j = 0; j < q; ++j) {
        double t = y[j];
        legendre_all(nmax, t, Pl.data(), dPl.data());
        // local u basis: l = 0 left hat, l = p right hat, l = 1..p-1 bubble W_{l-1}
        Vu[j * L + 0] = 0.5 * (1.0 - t);
        Du[j * L + 0] = -0.5;
        Vu[j * L + p] = 0.5 * (1.0 + t);
        Du[j * L + p] = 0.5;
        for (int n = 0; n + 2 <= p; ++n) {
            Vu[j * L + 1 + n] = (Pl[n] - Pl[n + 2]) / (2 * n + 3);
            Du[j * L + 1 + n] = -Pl[n + 1];
        }
        for (int a = 0; a < P; ++a) {
            Vpsi[j * P + a] = Pl[a];
            Yv[j * P + a] = Pl[a] - Pl[a + 2];
            Yd[j * P + a] = dPl[a] - dPl[a + 2];
        }
    }
    auto quad = [&](const std::vector<double>& X, int nx, int i, const std::vector<double>& Z,
                    int nz, int k) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += w[j] * X[j * nx + i] * Z[j * nz + k];
        return s;
    };
    A1.assign(L * L, 0.0);
    M1.assign(L * L, 0.0);
    for (int i = 0; i < L; ++i)
        for (int k = 0; k < L; ++k) {
            A1[i * L + k] = quad(Du, L, i, Du, L, k);
            M1[i * L + k] = quad(Vu, L, i, Vu, L, k);
        }
    B1.assign(L * P, 0.0);
    G1.assign(L * P, 0.0);
    for (int i = 0; i < L; ++i)
        for (int a = 0; a < P; ++a) {
            B1[i * P + a] = quad(Vu, L, i, Vpsi, P, a);
            G1[i * P + a] = quad(Du, L, i, Vpsi, P, a);
        }
    MpsiDiag.assign(P, 0.0);
    for (int a = 0; a < P; ++a) MpsiDiag[a] = 2.0 / (2 * a + 1);
    AY.assign(P * P, 0.0);
    MY.assign(P * P, 0.0);
    BY.assign(P * P, 0.0);
    for (int i = 0; i < P; ++i)
        for (int k = 0; k < P; ++k) {
            AY[i * P + k] = quad(Yd, P, i, Yd, P, k);
            MY[i * P + k] = quad(Yv, P, i, Yv, P, k);
            BY[i * P + k] = quad(Yv, P, i, Vpsi, P, k);
        }
    // exact zeros of these integrals come out of the rule as round-off; clean
    // them so the sparse 1-D rows keep only the structural couplings
    auto clean = [](std::vector<double>& v) {
        double mx = 0.0;
        for (double t : v) mx = std::max(mx, std::fabs(t));
        for (double& t : v)
            if (std::fabs(t) < 1e-13 * mx) t = 0.0;
    };
    clean(A1);
    clean(M1);
    clean(B1);
    clean(G1);
    clean(AY);
    clean(MY);
    clean(BY);
}

// Global 1-D rows in direction k.  1-D unknown of local function l of cell c:
// g = c p + l - 1 (l = 0 left hat, l = p right hat, else bubble l-1), valid
// when 0 <= g < n1 (the hats of the two boundary vertices are absent).
void build_rows(const Mesh& M, int k, Rows1D& R, bool dense) {
    const int p = M.p, P = M.P, m = M.m[k], n1 = M.n1[k];
    const int L = p + 1;
    const RefTables& T = M.ref;
    R.n = n1;
    std::vector<std::map<int, std::pair<double, double>>> am(n1);
    std::vector<std::map<int, double>> bm(n1), gm(n1);
    for (int c = 0; c < m; ++c) {
        const double h = M.h(k, c);
        for (int l = 0; l < L; ++l) {
            int g = c * p + l - 1;
            if (g < 0 || g >= n1) continue;
            for (int l2 = 0; l2 < L; ++l2) {
                int g2 = c * p + l2 - 1;
                if (g2 < 0 || g2 >= n1) continue;
                double a = T.A1[l * L + l2] * (2.0 / h);
                double mm = T.M1[l * L + l2] * (0.5 * h);
                if (a == 0.0 && mm == 0.0) continue;
                auto& e = am[g][g2];
                e.first += a;
                e.second += mm;
            }
            for (int a = 0; a < P; ++a) {
                double b = T.B1[l * P + a] * (0.5 * h);
                if (b != 0.0) bm[g][c * P + a] += b;
                double gg = T.G1[l * P + a];   // (2/h) (h/2) = 1
                if (gg != 0.0) gm[g][c * P + a] += gg;
            }
        }
    }
    R.lenM.assign(n1, 0);
    R.colM.assign(n1 * Rows1D::WM, 0);
    R.aM.assign(n1 * Rows1D::WM, 0.0);
    R.mM.assign(n1 * Rows1D::WM, 0.0);
    R.lenB.assign(n1, 0);
    R.colB.assign(n1 * Rows1D::WB, 0);
    R.vB.assign(n1 * Rows1D::WB, 0.0);
    R.lenG.assign(n1, 0);
    R.colG.assign(n1 * Rows1D::WB, 0);
    R.vG.assign(n1 * Rows1D::WB, 0.0);
    if (dense) {
        R.Adense.assign((size_t)n1 * n1, 0.0);
        R.Mdense.assign((size_t)n1 * n1, 0.0);
    }
    for (int g = 0; g < n1; ++g) {
        if ((int)am[g].size() > Rows1D::WM || (int)bm[g].size() > Rows1D::WB ||
            (int)gm[g].size() > Rows1D::WB)
            fail(HPG_ERR_INVALID_ARG, "internal: 1-D row wider than expected");
        int e = 0;
        for (auto& kv : am[g]) {
            R.colM[g * Rows1D::WM + e] = kv.first;
            R.aM[g * Rows1D::WM + e] = kv.second.first;
            R.mM[g * Rows1D::WM + e] = kv.second.second;
            if (dense) {
                R.Adense[(size_t)g * n1 + kv.first] = kv.second.first;
                R.Mdense[(size_t)g * n1 + kv.first] = kv.second.second;
            }
            ++e;
        }
        R.lenM[g] = e;
        e = 0;
        for (auto& kv : bm[g]) {
            R.colB[g * Rows1D::WB + e] = kv.first;
            R.vB[g * Rows1D::WB + e] = kv.second;
            ++e;
        }
        R.lenB[g] = e;
        e = 0;
        for (auto& kv : gm[g]) {
            R.colG[g * Rows1D::WB + e] = kv.first;
            R.vG[g * Rows1D::WB + e] = kv.second;
            ++e;
        }
        R.lenG[g] = e;
    }
}

// ---------------------------------------------------------------------------
// Dense symmetric eigen-solver (n small: the 1-D unknowns of one direction).
// Step 1: Householder reduction T = Q^T S Q to tridiagonal form, reflectors
//         accumulated into Q.
// Step 2: implicit symmetric QR steps with the Wilkinson shift on the
//         unreduced trailing block, Givens rotations accumulated into Q,
//         deflating off-diagonals below eps (|t_ii| + |t_i+1,i+1|).
// On return S holds Q (column j = eigenvector j) and lam the eigenvalues.
static void sym_eig(int n, std::vector<double>& S, std::vector<double>& lam) {
    auto at = [n](std::vector<double>& M, int i, int j) -> double& {
        return M[(size_t)i * n + j];
    };
    std::vector<double> Q((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) at(Q, i, i) = 1.0;
    std::vector<double> v(n), pv(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        // reflector H = I - beta v v^T with H x = -sign(x0) |x| e0, x = S[k+1:, k]
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += at(S, i, k) * at(S, i, k);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        double x0 = at(S, k + 1, k);
        double alpha = (x0 >= 0.0) ? -xn : xn;
        for (int i = k + 1; i < n; ++i) v[i] = at(S, i, k);
        v[k + 1] = x0 - alpha;
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        double beta = 2.0 / vv;
        // S <- H S H on the trailing block: p = beta S v, w = p - (beta p.v / 2) v
        double pdotv = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += at(S, i, j) * v[j];
            pv[i] = beta * t;
            pdotv += pv[i] * v[i];
        }
        for (int i = k + 1; i < n; ++i) wv[i] = pv[i] - 0.5 * beta * pdotv * v[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) at(S, i, j) -= v[i] * wv[j] + wv[i] * v[j];
        at(S, k + 1, k) = at(S, k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) at(S, i, k) = at(S, k, i) = 0.0;
        // Q <- Q H
        for (int r = 0; r < n; ++r) {
            double t = 0.0;
            for (int j = k + 1; j < n; ++j) t += at(Q, r, j) * v[j];
            t *= beta;
            for (int j = k + 1; j < n; ++j) at(Q, r, j) -= t * v[j];
        }
    }
    std::vector<double> a(n), b(n, 0.0);   // diagonal, sub-diagonal b[i] = T(i+1, i)
    for (int i = 0; i < n; ++i) a[i] = at(S, i, i);
    for (int i = 0; i + 1 < n; ++i) b[i] = at(S, i + 1, i);
    const double eps = 2.2e-16;
    int hi = n - 1, sweeps = 0;
    while (hi > 0) {
        // deflate
        for (int i = 0; i < hi; ++i)
            if (std::fabs(b[i]) <= eps * (std::fabs(a[i]) + std::fabs(a[i + 1]))) b[i] = 0.0;
        if (b[hi - 1] == 0.0) {
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && b[lo - 1] != 0.0) --lo;
        if (++sweeps > 60 * n) fail(HPG_ERR_NUMERIC, "eigen-solver did not converge");
        // Wilkinson shift from the trailing 2x2 block of the unreduced part
        double dd = 0.5 * (a[hi - 1] - a[hi]);
        double bb = b[hi - 1] * b[hi - 1];
        double mu = a[hi] - bb / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::sqrt(dd * dd + bb));
        // bulge chase
        double x = a[lo] - mu, z = b[lo];
        for (int k = lo; k < hi; ++k) {
            double r = std::hypot(x, z);
            double c = x / r, s = -z / r;
            if (k > lo) b[k - 1] = r;
            // apply the rotation G^T T G to rows/cols k, k+1
            double akk = a[k], ak1 = a[k + 1], bk = b[k];
            a[k] = c * c * akk - 2.0 * c * s * bk + s * s * ak1;
            a[k + 1] = s * s * akk + 2.0 * c * s * bk + c * c * ak1;
            b[k] = c * s * (akk - ak1) + (c * c - s * s) * bk;
            if (k + 1 < hi) {
                x = b[k];
                z = -s * b[k + 1];
                b[k + 1] *= c;
            }
            for (int r2 = 0; r2 < n; ++r2) {
                double qk = at(Q, r2, k), q1 = at(Q, r2, k + 1);
                at(Q, r2, k) = c * qk - s * q1;
                at(Q, r2, k + 1) = s * qk + c * q1;
            }
        }
    }
    lam = a;
    S = Q;
}

// A V = B V Lambda with B = L L^T (Cholesky): C = L^{-1} A L^{-T} = Q Lambda Q^T,
// V = L^{-T} Q, so V^T B V = I and V^T A V = Lambda.  V row-major n x n,
// column j the j-th eigenvector.
void generalized_eig(int n, const std::vector<double>& A, const std::vector<double>& B,
                     std::vector<double>& V, std::vector<double>& lam) {
    std::vector<double> L(B);
    for (int j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (s <= 0.0) fail(HPG_ERR_NUMERIC, "mass matrix not positive definite");
        double dj = std::sqrt(s);
        L[(size_t)j * n + j] = dj;
        for (int i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / dj;
        }
        for (int k = j + 1; k < n; ++k) L[(size_t)j * n + k] = 0.0;
    }
    // C = L^{-1} A L^{-T}: first X = L^{-1} A (forward solves on columns)
    std::vector<double> X(A);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double t = X[(size_t)i * n + c];
            for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * X[(size_t)k * n + c];
            X[(size_t)i * n + c] = t / L[(size_t)i * n + i];
        }
    // C = X L^{-T}  <=>  C^T = L^{-1} X^T; C symmetric so solve rows
    std::vector<double> C((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) {
            double t = X[(size_t)r * n + i];
            for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * C[(size_t)r * n + k];
            C[(size_t)r * n + i] = t / L[(size_t)i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
            C[(size_t)i * n + j] = C[(size_t)j * n + i] = s;
        }
    sym_eig(n, C, lam);   // C now holds Q (columns)
    // V = L^{-T} Q: back substitution with L^T
    V.assign((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double t = C[(size_t)i * n + c];
            for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * V[(size_t)k * n + c];
            V[(size_t)i * n + c] = t / L[(size_t)i * n + i];
        }
}

}  // namespace hpg
