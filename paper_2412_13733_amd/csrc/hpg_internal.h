// Internal declarations of the hpG library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "hpg.h"

namespace hpg {

// ---------------------------------------------------------------------------
// Error plumbing: every API call catches hpg::Error and turns it into a status.
struct Error {
    hpg_status code;
    std::string msg;
};
[[noreturn]] void fail(hpg_status code, const std::string& msg);
void set_last_error(const std::string& msg);
// run fn, turning an hpg::Error or an allocation failure into a status code
template <typename F>
hpg_status guarded(F&& fn) {
    try {
        return fn();
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return HPG_ERR_NOMEM;
    } catch (...) {
        set_last_error("unexpected internal error");
        return HPG_ERR_DEVICE;
    }
}
#define HPG_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            ::hpg::fail(HPG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// 1-D reference tables on [-1, 1] (Sec. 3): Legendre P_n, hats, bubbles
// W_n = (P_n - P_{n+2})/(2n+3) with W_n' = -P_{n+1}, spectral-Galerkin
// Y_n = P_n - P_{n+2}, and a Gauss-Legendre rule.
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);
void legendre_all(int nmax, double y, double* P, double* dP);

struct RefTables {
    int p = 0, P = 0, q = 0;
    std::vector<double> y, w;          // q nodes / weights
    std::vector<double> Vu, Du;        // q x (p+1): local u basis and d/dy
    std::vector<double> Vpsi;          // q x P: Legendre modes
    std::vector<double> A1, M1;        // (p+1)^2 reference stiffness / mass (d/dy)
    std::vector<double> B1;            // (p+1) x P: (phi_l, P_a) on [-1,1]
    std::vector<double> G1;            // (p+1) x P: (phi_l', P_a) on [-1,1]
    std::vector<double> MpsiDiag;      // P: 2/(2a+1)
    // Phi_h (Y basis, P functions): gradient stiffness, mass, Gram with P_a
    std::vector<double> AY, MY, BY;    // P x P
    void build(int p, int P, int q);
};

// ---------------------------------------------------------------------------
// Host mesh (uniform partial degree p, tensor breakpoints).
struct Mesh {
    int d = 0, p = 0, P = 0, q = 0, kind = HPG_OBSTACLE;
    int m[3] = {1, 1, 1};
    int n1[3] = {1, 1, 1};
    std::vector<double> breaks[3];
    int64_t n_cells = 0, n_u = 0, n_psi = 0, n_qp = 0;
    int ncomp = 1;
    int64_t psi_per_cell = 0;   // ncomp * P^d
    int64_t Pd = 0, Qd = 0, Ld = 0;   // P^d, q^d, (p+1)^d
    RefTables ref;
    double h(int k, int c) const { return breaks[k][c + 1] - breaks[k][c]; }
    // One degree per cell (obstacle only; p, P, q, Pd, Qd, Ld above then
    // describe the largest degree).  Entities (vertices, edges, faces, cell
    // interiors) are the points of the doubled grid, 2 m_k + 1 per direction
    // (even: vertex, odd: cell interval), direction 0 fastest; each interior
    // entity carries the smallest degree of the cells containing it and
    // (p_E - 1)^(number of odd directions) consecutive unknowns starting at
    // ent_base (boundary entities: -1).
    bool hp = false;
    int pmin = 0;
    std::vector<int32_t> deg;              // n_cells
    std::vector<int64_t> psi_off, qp_off;  // n_cells + 1: P_K^d and q_K^d prefix sums
    std::vector<int64_t> ent_base;
    std::vector<int32_t> ent_deg;
    int64_t ent_index(const int e[3]) const {
        return e[0] + (int64_t)(2 * m[0] + 1) * (d > 1 ? e[1] + (int64_t)(2 * m[1] + 1) * (d > 2 ? e[2] : 0) : 0);
    }
};

// dense Cholesky solve A X = B (A n x n SPD, B n x m, row-major)
void chol_solve(int n, std::vector<double> A, std::vector<double>& B, int m);
// C_K = Bhat^T Ahat^{-1} Bhat of one cell shape (widths hk) at the mesh's P
std::vector<double> schur_block(const Mesh& M, const double* hk);
// contract axis ax of a d-D tensor (dims din, updated) with mat (nout x din[ax])
std::vector<double> hcontract(const std::vector<double>& in, int d, int din[3], int ax,
                              int nout, const std::vector<double>& mat, int ld, bool trans);

// number the unknowns of a per-cell-degree mesh (fills n_u, n_psi, n_qp,
// offsets and the entity tables from d, m, breaks and deg)
void hp_number(Mesh& M);
// global unknown of every local function of cell c ((p_K+1)^d, direction 0
// fastest; -1 where the function is absent), appended to out
void hp_cell_dofs(const Mesh& M, int64_t c, std::vector<int32_t>& out);

// Sparse 1-D global rows in direction k (assembled from the cell matrices):
// for every 1-D u unknown g: up to 7 (column, stiffness, mass) entries and up
// to 4 (psi 1-D index c*P + a, Gram value) entries; gradient adds up to 4
// (psi index, (phi', P_a)) entries.
struct Rows1D {
    static constexpr int WM = 7, WB = 4;
    int n = 0;
    std::vector<int32_t> lenM, colM;
    std::vector<double> aM, mM;
    std::vector<int32_t> lenB, colB;
    std::vector<double> vB;
    std::vector<int32_t> lenG, colG;
    std::vector<double> vG;
    std::vector<double> Adense, Mdense;   // n x n global 1-D stiffness and mass (for FDM)
};
void build_rows(const Mesh& M, int k, Rows1D& R, bool dense = false);

// Fast diagonalisation (Lynch-Rice-Thomas): A1 V = M1 V Lambda, V^T M1 V = I.
void generalized_eig(int n, const std::vector<double>& A, const std::vector<double>& B,
                     std::vector<double>& V, std::vector<double>& lam);

}  // namespace hpg
