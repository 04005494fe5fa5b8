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

// Batches of independent problems on one mesh: a launch covers nb requests,
// request b = blockIdx.y (blockIdx.z for the GEMM passes), and every pointer a
// kernel takes is offset by b times its stride below (0: shared).  Partial
// sums and done flags are per request, so each request's reductions run in
// the same fixed order as when it is solved alone.
struct TileBatch {
    int nb = 1;
    int64_t xu = 0, xp = 0, pprev = 0, om = 0, F = 0, Phi = 0, yu = 0, yp = 0, part = 0, done = 0;
    int64_t prm = 0;   // per-request (alpha, beta, 1/alpha) at prm + b * this
};
struct PsiBatch {
    int nb = 1;
    int64_t sinv = 0, r = 0, z = 0, part = 0, done = 0;
    int64_t flag = 0;   // per-request stride of the cell flags of PsiHi (cells)
};
// FP32 psi-block apply: the cells with flag[cell] != 0 (a Schur block too
// ill-conditioned for an FP32 product, see kFp32CondLimit) are applied with
// their FP64 inverse s64 and FP64 accumulation instead of the FP32 blocks
struct PsiHi {
    const double* s64 = nullptr;
    const int* flag = nullptr;
    // the inverse blocks (and s64) stored packed: the upper triangle row by row,
    // n (n + 1) / 2 values per cell (the blocks are symmetric)
    int packed = 0;
};
// values per psi-block: n^2, or n (n + 1) / 2 packed
__host__ __device__ inline int64_t psi_block_size(int n, int packed) {
    return packed ? (int64_t)n * (n + 1) / 2 : (int64_t)n * n;
}
// 1-norm condition number of -S_hat_K above which the FP32 path applies the
// cell's block in FP64: an FP32 product with a block of condition c carries a
// relative error up to about n eps_32 c, which turns <S^{-1} v, v> negative
// (a MINRES breakdown) once it passes 1
constexpr double kFp32CondLimit = 1e6;
struct VecBatch {
    int nb = 1;
    int64_t v = 0, part = 0;   // vector stride, partial-sum stride (the state: st + b)
    const int* mask = nullptr; // MINRES start: only the requests with mask[b] != 0
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
                 const int* done, int mode, hipStream_t s, const KernelEvents* ev = nullptr,
                 const TileBatch& bt = TileBatch());
// Obstacle setup: LDS bytes per cell with the block in LDS; and of the
// variants that form and invert the block in s64 (global memory), with or
// without (d = 3) the q P^4 contraction intermediate in LDS.
enum { SETUP_LDS = 0, SETUP_HBM_T2 = 1, SETUP_HBM = 2 };
size_t setup_smem_per_cell(const Geo& g);
size_t setup_big_smem(const Geo& g, bool t2);
// batches (g.n_cells = all requests' cells): prm_req (4 per request: alpha,
// beta, ..) overrides alpha and beta per request, and with mask only the
// cells of requests with mask[req] != 0 are written (req = cell / cpr)
void launch_setup(const Geo& g, const PsiTabs<double>& tb, int cpb, int big, const double* psi,
                  double alpha, double beta, const double* C, const int* cclass, double* om64,
                  float* om32, double* s64, float* s32, hipStream_t s,
                  const double* prm_req = nullptr, const int* mask = nullptr, int64_t cpr = 1,
                  int* sflag = nullptr, int packed = 0);
template <typename T>
void launch_prec_psi(int64_t n_cells, int n, int cpb, const T* sinv, const T* r, T* z,
                     double* partial, const int* done, hipStream_t s,
                     const PsiBatch& bt = PsiBatch(), const PsiHi& hi = PsiHi());
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
    // batches of requests: the GEMM batch bz belongs to request bz / bdiv, whose
    // done flag is done[request * dstride] and whose partial sums start at
    // partial[request * pstride] (pstride 0: one index over all batches)
    int bdiv;
    int64_t pstride, dstride;
    int64_t prmstride;   // per-request prm at prm + request * prmstride
    // block tile (16 ts) x (16 ts), ts = 1 or 2 (0: 1).  Every tile shape sums
    // in the same order, so the choice changes the time and never the result
    int ts;
};
template <typename T>
inline int gemm_ts(const GemmEpi<T>& ep) {
    return ep.ts == 2 ? 2 : 1;
}
template <typename T>
void launch_gemm(int M, int N, int K, const T* A, int64_t lda, int64_t sA, const T* B,
                 int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC, int batch,
                 const int* done, const GemmEpi<T>& ep, hipStream_t s,
                 const KernelEvents* ev = nullptr);
// launch_gemm (batch 1, no strides) and launch_prec_psi in one launch: the
// GEMM tiles and the psi-block cell groups are independent blocks of one grid
template <typename T>
void launch_gemm_prec(int M, int N, int K, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                      int64_t ldc, const int* done, const GemmEpi<T>& ep, int64_t n_cells, int n,
                      int cpb, const T* sinv, const T* r, T* z, double* ppart, hipStream_t s,
                      int64_t sA = 0, int64_t sC = 0, const PsiBatch& bt = PsiBatch(),
                      const PsiHi& hi = PsiHi());
template <typename T>
void launch_dot(int64_t n, const T* a, const T* b, double* partial, int nblocks, const int* done,
                hipStream_t s);
template <typename T>
void launch_kr_start(int64_t n, KState* st0, const double* partial, int np, double rtol,
                     int maxit, const T* b, const T* z, T* vcur, T* vprev, T* q, T* wprev,
                     T* wcur, T* x, hipStream_t s, const VecBatch& bt = VecBatch());
template <typename T>
void launch_kr_vhat(int64_t n, KState* st, const double* partial, int np, const T* Gq,
                    const T* vcur, const T* vprev, T* vhat, hipStream_t s,
                    const VecBatch& bt = VecBatch());
template <typename T>
void launch_kr_update(int64_t n, const KState* st_in, KState* st_out, const double* partial,
                      int np, T* q, T* wprev, const T* wcur, T* x, T* vprev, const T* vhat,
                      const T* z, hipStream_t s, const VecBatch& bt = VecBatch());
// launch_gemm_prec with the Lanczos step folded in: every block reduces the
// G-apply partials gpart (npg) to delta = <q, Gq> (stored in st), and the
// first pass (A = vhat, R x N with lda N, B = V, C) and the psi-block read
// vhat = Gq - delta vcur - gamma vprev, which is also stored to vhat (n_u +
// psi entries).  The psi-block partials go to ppart.
template <typename T>
void launch_vhat_gemm_prec(int M, int N, const T* B, T* C, const GemmEpi<T>& ep, int64_t n_cells,
                           int n, int cpb, const T* sinv, T* z, double* ppart, KState* st,
                           const double* gpart, int npg, const T* Gq, const T* vcur,
                           const T* vprev, T* vhat, int64_t n_u, hipStream_t s,
                           const PsiHi& hi = PsiHi());
template <typename TI, typename TO>
void launch_convert(int64_t n, const TI* a, TO* b, double scale, hipStream_t s);
template <typename T>
void launch_axpy_to(int64_t n, const double* x, double t, const T* d, double* y, hipStream_t s);
void launch_lambda(int64_t n, const double* psi_prev, const double* psi, double alpha,
                   double* lam, hipStream_t s);
void launch_l2(const Geo& g, const PsiTabs<double>& tb, int cpb, const double* u, const double* v,
               double* partial, hipStream_t s, const VecBatch& bt = VecBatch());
// Diagnostics of an iterate (diag.hip): per block b, partial[3 b] = sum w |J|
// |lambda_h| exp(-psi_h), partial[3 b + 1] = sum w |J| |lambda_h| (obstacle;
// 0 for the gradient constraint), partial[3 b + 2] = max over the block's
// Gauss points of u_h - phi (obstacle) or |grad u_h| - phi (gradient).  Du:
// q x (p+1) reference derivative table; phiq: phi at the Gauss points.
// At most nblocks blocks (one cell at a time each).
// Batched: request b = blockIdx.y reads u + b u_stride, psi and lam + b
// psi_stride, phiq + b qp_stride and writes partial + 3 nblocks b.
struct DiagBatch {
    int nb = 1;
    int64_t u = 0, psi = 0, qp = 0;
};
void launch_diag(const Geo& g, const PsiTabs<double>& tb, const double* Du, const double* u,
                 const double* psi, const double* lam, const double* phiq, double* partial,
                 int nblocks, hipStream_t s, const DiagBatch& bt = DiagBatch());

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

// ---- one degree per cell (hp.hip) -----------------------------------------
// Offsets of the reference tables of degree p (L = p+1 local u functions,
// P = p-1 psi modes, q = p+1 Gauss points per direction) in a packed array:
// A1, M1 (L x L), B1 (L x P), Vu (q x L), Vpsi (q x P), w (q), Mdiag (P).
struct HpTabOff {
    int64_t A1, M1, B1, Vu, Vpsi, w, Mdiag;
};
template <typename T>
struct HpTabs {
    const T* base;
    const HpTabOff* off;   // indexed by degree
    const T* h[3];         // cell widths per direction
};
// Cells are processed in work items: runs of up to item_count cells of equal
// degree item_p (cell numbers order[item_start .. item_start + count)).
struct HpGeo {
    int d;
    int m[3];
    int64_t n_cells, n_u, n_psi;
    int n_items, lds_elems;   // lds_elems: per-buffer LDS elements of the cell kernels
    int lmax;                 // largest p + 1
    const int32_t* cell_p;
    const int64_t* loc_off;   // prefix sums of (p_K+1)^d
    const int64_t* psi_off;   // prefix sums of P_K^d
    const int64_t* qp_off;    // prefix sums of q_K^d
    const int64_t* sinv_off;  // prefix sums of (P_K^d)^2
    const int32_t* loc2glob;  // local -> global u unknown (-1: absent)
    const int32_t* order;
    const int32_t* item_start;
    const int32_t* item_count;
    const int32_t* item_p;
};
constexpr int MODE_L2 = 2;
// Cell pass of G (MODE_APPLY: y_loc = alpha A_K x_K + B_K x_psi, y_psi =
// B_K^T x_K - (D_K + beta M_K) x_psi) or of the FP64 residual (MODE_RES:
// x_psi = psi, xpsi_prev = psi_{k-1}; y_loc = alpha A_K u_K + B_K (psi -
// psi_prev), y_psi = B_K^T u_K + E_K(psi) - Phi_K).  y_loc is per local
// function, summed into y_u by launch_hp_gather, which also takes both halves
// of the reduction.
// LDS bytes of the cell pass (element size tsize, MODE_APPLY or MODE_RES)
size_t hp_cell_lds(int d, int lds_elems, int lmax, size_t tsize, int mode);
template <typename T>
void launch_hp_cell(const HpGeo& g, const HpTabs<T>& tb, T alpha, T beta, const double* prm,
                    const T* xu, const T* xpsi, const T* xpsi_prev, const T* omega,
                    const double* Phi, T* yloc, T* ypsi, int nblocks, const int* done, int mode,
                    hipStream_t s);
// y_u[g] = sum of y_loc over the local functions of unknown g (fixed order),
// minus alpha F[g] in MODE_RES, in nblocks blocks; partial[0, nblocks) gets
// <y_u, x_u> (APPLY) or |y_u|^2 (RES) per block and partial[nblocks,
// 2 nblocks) <y_psi, x_psi> or |y_psi|^2 over fixed ranges of the psi unknowns
// (y_psi as the cell pass wrote it), independent of the work items
template <typename T>
void launch_hp_gather(int64_t n_u, const int32_t* inc_ptr, const int32_t* inc_idx, const T* yloc,
                      const double* F, double alpha, const T* xu, T* yu, int64_t n_psi,
                      const T* xpsi, const T* ypsi, double* partial, int nblocks, const int* done,
                      int mode, hipStream_t s);
// launch_diag on a mesh with one degree per cell (obstacle constraint)
void launch_hp_diag(const HpGeo& g, const HpTabs<double>& tb, const double* u, const double* psi,
                    const double* lam, const double* phiq, double* partial, int nblocks,
                    hipStream_t s);
// ||a - b||_{L2}^2 and ||a||_{L2}^2 per block (partial[2 i], partial[2 i + 1]);
// block i takes cells i, i + nblocks, ... (min(n_cells, nblocks) blocks)
void launch_hp_l2(const HpGeo& g, const HpTabs<double>& tb, const double* a, const double* b,
                  double* partial, int nblocks, hipStream_t s);
// Newton-step setup: omega_q = w_q |J| exp(-psi_h) at qp_off, and the inverse of
// -S_hat_K = D_K + beta M_K + C_K / alpha (C of cell K at C + c_off[cclass[K]]),
// one cell per block for the cells order[o0 .. o0 + ncell) (one degree per
// launch, so lds_bytes = hp_setup_lds_p of that degree), written to s64 / s32
// + sinv_off (either may be null when block_in_lds; otherwise the block is
// inverted in place in s64)
void launch_hp_setup(const HpGeo& g, const HpTabs<double>& tb, const double* psi, double alpha,
                     double beta, const double* C, const int64_t* c_off, const int32_t* cclass,
                     double* om64, float* om32, double* s64, float* s32, size_t lds_bytes,
                     bool block_in_lds, int o0, int ncell, hipStream_t s);
// LDS bytes of that setup for degrees 2..pmax
size_t hp_setup_lds(int d, int pmax, bool block_in_lds);
size_t hp_setup_lds_p(int d, int p, bool block_in_lds);   // one degree
// z_psi = (-S_hat_K)^{-1} r_psi per cell, partial <z_psi, r_psi>
template <typename T>
void launch_hp_prec_psi(const HpGeo& g, const T* sinv, const T* r, T* z, double* partial,
                        int nblocks, int nmax, const int* done, hipStream_t s);
// block-Jacobi A-block: out[t] = r[idx[t]] / z[idx[t]] = in[t] (vertex unknowns),
// and per edge/face/interior entity z_E = (1/alpha) Ainv_E r_E
template <typename T>
void launch_hp_vgather(int64_t n, const int32_t* idx, const T* r, T* out, const int* done,
                       hipStream_t s);
template <typename T>
void launch_hp_vscatter(int64_t n, const int32_t* idx, const T* in, T* z, const int* done,
                        hipStream_t s);
// Edge / face / interior entities of the block-Jacobi A-block, in chunks of
// entities that share one (deduplicated) inverse: a chunk's right-hand sides
// sit side by side in LDS, so each entry of the inverse is read once per
// chunk.  Entities of kHpEntRowMin..kHpEntRowMax unknowns: up to kHpEntChunk
// per chunk, a row (or a part of one) per thread for all of them; smaller
// ones: up to 256 / n per chunk, a thread per (entity, row); larger ones: one
// per chunk.
constexpr int kHpEntChunk = 8;
constexpr int kHpEntRowMin = 32, kHpEntRowMax = 768;
__host__ __device__ inline bool hp_ent_rows(int n) {
    return n >= kHpEntRowMin && n <= kHpEntRowMax;
}
__host__ __device__ inline int hp_ent_cap(int n) {
    return hp_ent_rows(n) ? kHpEntChunk : (n < kHpEntRowMin ? 256 / n : 1);
}
// row path: the 256 threads form groups that each sum a range of j for
// 256 / groups rows; the groups' sums meet in LDS
__host__ __device__ inline int hp_ent_groups(int n) { return n > 128 ? 1 : (n > 64 ? 2 : 4); }
__host__ __device__ inline int hp_ent_lds(int n) {   // LDS elements of a chunk
    if (!hp_ent_rows(n)) return hp_ent_cap(n) * n;
    const int g = hp_ent_groups(n);
    return kHpEntChunk * n + (g - 1) * (256 / g) * kHpEntChunk;
}
struct HpEnt {
    int nchunk;
    int lds;                  // largest hp_ent_lds over the entities
    const int32_t* cstart;    // chunk -> first position in list
    const int32_t* ccount;    // entities in the chunk
    const int32_t* list;      // entity numbers, chunk by chunk
    const int32_t* first;     // first unknown of each entity (its unknowns are consecutive)
    const int32_t* cnt;       // unknowns of each entity
    const int64_t* off;       // offset of each entity's inverse (row-major, symmetric)
};
// The psi-block (np blocks, LDS nmax values), the entity chunks (ne blocks,
// their <z, r> shares in epart[0..ne)) and the vertex gather (into cv) in one
// launch; hp_prec_entity_blocks gives ne for nchunk chunks.  The vertex
// scatter then adds its <z, r> shares (hp_vscatter_blocks(nv) of them).
int hp_prec_entity_blocks(int nchunk);
int hp_vscatter_blocks(int64_t nv);
template <typename T>
void launch_hp_prec_fused(const HpGeo& g, const T* sinv, int np, int nmax, int ne,
                          const HpEnt& ent, const T* inv, const double* prm, const int32_t* vidx,
                          int64_t nv, T* cv, const T* r, T* z, double* ppart, double* epart,
                          const int* done, hipStream_t s);
// 2-D vertex block of the preconditioner in one workgroup (n0, n1 <= 64
// interior vertices per direction): z[vidx] = (alpha A_VV)^{-1} rv by fast
// diagonalisation, rv = r[vidx] gathered beforehand (launch_hp_vgather or the
// fused launch) (V0, V1: eigenvectors row-major; l0, l1: eigenvalues; prm[2] =
// 1 / alpha), partial[0] = <z_V, r_V> and partial[1 .. npart) = 0
size_t hp_vsolve2_lds(int n0, int n1, size_t tsize);
template <typename T>
void launch_hp_vsolve2(int n0, int n1, const int32_t* vidx, const T* V0, const T* V1, const T* l0,
                       const T* l1, const double* prm, const T* rv, T* z, double* partial,
                       int npart, const int* done, hipStream_t s);
template <typename T>
void launch_hp_vscatter_dot(int64_t nv, const int32_t* idx, const T* in, const T* r, T* z,
                            double* partial, const int* done, hipStream_t s);
// the entity chunks alone (z_E = prm[2] Ainv_E r_E)
template <typename T>
void launch_hp_entity(const HpEnt& ent, const T* inv, const double* prm, const T* r, T* z,
                      const int* done, hipStream_t s);

}  // namespace dev
}  // namespace hpg
