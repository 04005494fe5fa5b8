// Kernel-side structs and launchers of the hpG library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpg {
namespace dev {

constexpr int MODE_APPLY = 0;
constexpr int MODE_RES = 1;

// mesh geometry, passed by value
struct Geo {
    int d, p, P, q;
    int m[3];
    int n1[3];
    int64_t n_u, n_psi, n_cells;
    int Pd, Qd, Ld;
    int S;    // per-cell LDS stride: max(p+1, q)^d
    int nc;   // psi components per cell: 1 (obstacle) or d (gradient)
};

// sparse global 1-D rows of one direction (see Rows1D on the host)
template <typename T>
struct URows {
    static constexpr int WM = 7, WB = 4;
    const int32_t* lenM;
    const int32_t* colM;
    const T* aM;
    const T* mM;
    const int32_t* lenB;
    const int32_t* cellB;
    const int32_t* modeB;
    const T* vB;
    // p <= 3: dense windows per 1-D unknown g, stored from row g + 1 (row 0 and
    // the tail are zero): stiffness and mass at columns g - p .. g + p, then the
    // psi coupling of cells g / p and g / p + 1 (P modes each)
    const T* win;
    // gradient constraint: rows of (v', zeta) in this direction (<= WB entries)
    const int32_t* lenG;
    const int32_t* cellG;
    const int32_t* modeG;
    const T* vG;
};

// 1-D reference tables and cell widths
template <typename T>
struct PsiTabs {
    const T* B1;     // (p+1) x P
    const T* Vpsi;   // q x P
    const T* Vu;     // q x (p+1)
    const T* w;      // q
    const T* Mdiag;  // P: 2/(2a+1)
    const T* h[3];   // cell widths per direction
    const T* G1;     // (p+1) x P: (phi_l', P_a) on [-1, 1] (gradient)
    const T* AY;     // P x P: (Y_a', Y_b') on [-1, 1] (gradient E_beta)
    const T* MY;     // P x P: (Y_a, Y_b) on [-1, 1]
};

// start/stop events recorded by the dispatch of one kernel launch itself
// (hipExtLaunchKernelGGL), used when kernel timing is enabled
struct KernelEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// MINRES scalar state (device)
struct KState {
    double gamma1, gamma, delta;
    double c, c_prev, s, s_prev, eta;
    double rtol;
    int iters, max_iters, done, breakdown;
};

// prm (device, may be null): prm[0] = alpha, prm[1] = beta, prm[2] = 1/alpha;
// when given it overrides the by-value alpha / beta
template <typename T>
void launch_u_side(const Geo& g, const URows<T>* r, T alpha, const T* xu, const T* xb,
                   const T* xb_prev, const double* F, T* yu, double* partial, const int* done,
                   int mode, hipStream_t s, const double* prm = nullptr);
template <typename T>
void launch_psi_side(const Geo& g, const PsiTabs<T>& tb, int cpb, T beta, const T* xu,
                     const T* xpsi, const T* omega, const double* Phi, T* ypsi, double* partial,
                     const int* done, int mode, hipStream_t s, const double* prm = nullptr);
// fused LDS-tiled G apply / residual with compile-time p (tile.hip); returns
// false when (d, p) has no compiled variant.  Partials: APPLY one per block
// (<x, Gx>-type sums), RES two per block (||R_u||^2, ||R_psi||^2).
bool tile_supported(const Geo& g);
int tile_grid(const Geo& g);          // capped grid (bounded partial count)
int64_t tile_count(const Geo& g);     // number of tiles
template <typename T>
bool launch_tile(const Geo& g, const URows<T>* r, const PsiTabs<T>& tb, T alpha, T beta,
                 const double* prm, const T* xu, const T* xpsi, const T* xpsi_prev, const T* omega,
                 const double* F, const double* Phi, T* yu, T* ypsi, double* partial,
                 const int* done, int mode, hipStream_t s, const KernelEvents* ev = nullptr);
// Obstacle setup: LDS bytes per cell with the block in LDS; and of the
// variants that form and invert the block in s64 (global memory), with or
// without (d = 3) the q P^4 contraction intermediate in LDS.
enum { SETUP_LDS = 0, SETUP_HBM_T2 = 1, SETUP_HBM = 2 };
size_t setup_smem_per_cell(const Geo& g);
size_t setup_big_smem(const Geo& g, bool t2);
void launch_setup(const Geo& g, const PsiTabs<double>& tb, int cpb, int big, const double* psi,
                  double alpha, double beta, const double* C, const int* cclass, double* om64,
                  float* om32, double* s64, float* s32, hipStream_t s);
template <typename T>
void launch_prec_psi(int64_t n_cells, int n, int cpb, const T* sinv, const T* r, T* z,
                     double* partial, const int* done, hipStream_t s);
// C_b = A_b B_b (row-major, M x K times K x N), batch strides sA, sB, sC,
// with the optional epilogues of GemmEpi
template <typename T>
struct GemmEpi {
    int scale_mode;
    int n0;
    const T* l0;
    const T* l1;
    const T* l2;
    const double* prm;
    const T* dotv;
    double* partial;
};
template <typename T>
void launch_gemm(int M, int N, int K, const T* A, int64_t lda, int64_t sA, const T* B,
                 int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC, int batch,
                 const int* done, const GemmEpi<T>& ep, hipStream_t s,
                 const KernelEvents* ev = nullptr);
template <typename T>
void launch_fdm_scale(const Geo& g, const T* l0, const T* l1, const T* l2, T inv_alpha, T* z,
                      const int* done, hipStream_t s);
template <typename T>
void launch_dot(int64_t n, const T* a, const T* b, double* partial, int nblocks, const int* done,
                hipStream_t s);
template <typename T>
void launch_kr_start(int64_t n, KState* st0, const double* partial, int np, double rtol,
                     int maxit, const T* b, const T* z, T* vcur, T* vprev, T* q, T* wprev,
                     T* wcur, T* x, hipStream_t s);
template <typename T>
void launch_kr_vhat(int64_t n, KState* st, const double* partial, int np, const T* Gq,
                    const T* vcur, T* vprev, hipStream_t s);
template <typename T>
void launch_kr_update(int64_t n, const KState* st_in, KState* st_out, const double* partial,
                      int np, T* q, T* wprev, const T* wcur, T* x, T* vprev, const T* z,
                      hipStream_t s);
template <typename TI, typename TO>
void launch_convert(int64_t n, const TI* a, TO* b, double scale, hipStream_t s);
template <typename T>
void launch_axpy_to(int64_t n, const double* x, double t, const T* d, double* y, hipStream_t s);
void launch_lambda(int64_t n, const double* psi_prev, const double* psi, double alpha,
                   double* lam, hipStream_t s);
void launch_l2(const Geo& g, const PsiTabs<double>& tb, int cpb, const double* u, const double* v,
               double* partial, hipStream_t s);

// ---- gradient constraint |grad u| <= phi (gradient.hip) ---------------------
// omega layout: [cell][pair (c <= l, row-major upper triangle)][q^d] of the
// symmetric d x d weights w_q |J| phi_q F(psi_h(x_q)).
template <typename T>
void launch_u_side_grad(const Geo& g, const URows<T>* r, T alpha, const T* xu, const T* xb,
                        const T* xb_prev, const double* F, T* yu, double* partial,
                        const int* done, int mode, hipStream_t s, const double* prm);
template <typename T>
int psi_side_grad_cpb(const Geo& g);
template <typename T>
void launch_psi_side_grad(const Geo& g, const PsiTabs<T>& tb, int cpb, T beta, const T* xu,
                          const T* xpsi, const T* omega, const double* phi_q, T* ypsi,
                          double* partial, const int* done, int mode, hipStream_t s,
                          const double* prm);
// Newton-step setup: omega and the inverses of -S_hat_K = D_K + beta E_K
// (n = d P^d); blocks that do not fit in LDS are inverted in place in sinv64
bool setup_grad_in_hbm(const Geo& g);
void launch_setup_grad(const Geo& g, const PsiTabs<double>& tb, const double* psi,
                       const double* phi_q, double beta, double* om64, float* om32, double* s64,
                       float* s32, hipStream_t s);
// psi-block preconditioner for blocks too large to stage in LDS: one block of
// threads per cell streams the symmetric inverse row by row
template <typename T>
void launch_prec_psi_big(int64_t n_cells, int n, const T* sinv, const T* r, T* z,
                         double* partial, int nblocks, const int* done, hipStream_t s);

}  // namespace dev
}  // namespace hpg
