// Kernels for meshes with one degree per cell (obstacle constraint).
//
// The u space is the conforming space of the minimum rule (every vertex, edge,
// face and cell interior carries the smallest degree of the cells containing
// it), so it is no longer a tensor product and the operator is applied cell by
// cell: a work item (a run of cells of equal degree p) gathers its local u
// coefficients through a local -> global map (absent functions read as zero),
// contracts them with the 1-D reference matrices of degree p along each
// direction (stiffness A_K = sum_k J (2/h_k)^2 A1 (x) M1 ..., coupling
// B_K = J (x) B1, paper Sec. 3-4), and writes one value per local function;
// a second pass sums those values into each global unknown in a fixed order
// (deterministic, no atomics).  The psi side (B^T u, D_psi, E(psi), the Schur
// blocks) is cell-local as in the uniform kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dev_util.h"
#include "kernels.h"

namespace hpg {
namespace dev {

template <typename T>
struct HpCellTabs {
    const T *A1, *M1, *B1, *Vu, *Vpsi, *w, *Mdiag;
};

template <typename T>
__device__ inline HpCellTabs<T> hp_tabs(const HpTabs<T>& tb, int p) {
    const HpTabOff o = tb.off[p];
    return {tb.base + o.A1, tb.base + o.M1,   tb.base + o.B1,   tb.base + o.Vu,
            tb.base + o.Vpsi, tb.base + o.w, tb.base + o.Mdiag};
}

template <typename T, int D>
__device__ inline T hp_jac(const HpGeo& g, const HpTabs<T>& tb, int64_t cell, T* hk) {
    T J = 1;
    int64_t c = cell;
    for (int k = 0; k < D; ++k) {
        const int ck = (int)(c % g.m[k]);
        c /= g.m[k];
        hk[k] = tb.h[k][ck];
        J *= (T)0.5 * hk[k];
    }
    return J;
}

// LDS layout of the 2-D cell pass: per-cell offsets (int64), then the
// buffers of lds_elems elements, the 1-D tables of the largest degree and the
// per-cell factors
struct HpCell2Lds {
    int cmax, nbuf, l2;
    size_t off_t, bytes;
};
__host__ __device__ inline HpCell2Lds hp_cell2_layout(int lds_elems, int lmax, int ts, int mode) {
    HpCell2Lds o;
    o.cmax = lds_elems / 9 + 1;   // (p + 1)^2 >= 9 local functions per cell
    o.nbuf = mode == MODE_RES ? 9 : 8;
    o.l2 = lmax * lmax;
    o.off_t = (size_t)3 * o.cmax * sizeof(int64_t);
    o.bytes = o.off_t + (size_t)ts * ((size_t)o.nbuf * lds_elems + 4 * o.l2 + 2 * lmax + 3 * o.cmax);
    return o;
}

size_t hp_cell_lds(int d, int lds_elems, int lmax, size_t tsize, int mode) {
    if (d == 2) return hp_cell2_layout(lds_elems, lmax, (int)tsize, mode).bytes;
    return (size_t)6 * lds_elems * tsize;
}

// ---------------------------------------------------------------------------
template <typename T, int D, int MODE>
__global__ __launch_bounds__(256) void k_hp_cell(HpGeo g, HpTabs<T> tb, T alpha, T beta,
                                                 const double* __restrict__ prm,
                                                 const T* __restrict__ xu,
                                                 const T* __restrict__ xpsi,
                                                 const T* __restrict__ xpsi_prev,
                                                 const T* __restrict__ omega,
                                                 const double* __restrict__ Phi,
                                                 T* __restrict__ yloc, T* __restrict__ ypsi,
                                                 const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    if (prm) {
        alpha = (T)prm[0];
        beta = (T)prm[1];
    }
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int SB = g.lds_elems;
    T* bU = sm;            // local u coefficients
    T* bX = sm + SB;       // psi coefficients (RES: psi - psi_prev)
    T* bY = sm + 2 * SB;   // A_K x_K
    T* bT = sm + 3 * SB;   // J B1^T x_K
    T* bA = sm + 4 * SB;
    T* bB = sm + 5 * SB;
    for (int it = blockIdx.x; it < g.n_items; it += gridDim.x) {
        const int p = g.item_p[it], L = p + 1, P = p - 1, q = p + 1;
        const int start = g.item_start[it], ncell = g.item_count[it];
        int S = 1, Pd = 1;
        for (int k = 0; k < D; ++k) {
            S *= L;
            Pd *= P;
        }
        const HpCellTabs<T> t = hp_tabs(tb, p);
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = e / S, l = e - ci * S;
            const int64_t cell = g.order[start + ci];
            const int gi = g.loc2glob[g.loc_off[cell] + l];
            bU[ci * S + l] = gi >= 0 ? xu[gi] : (T)0;
            bY[ci * S + l] = 0;
        }
        for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
            const int ci = e / Pd, a = e - ci * Pd;
            const int64_t o = g.psi_off[g.order[start + ci]] + a;
            bX[ci * S + a] = MODE == MODE_RES ? xpsi[o] - xpsi_prev[o] : xpsi[o];
        }
        __syncthreads();
        // A_K x_K = sum_k J (2/h_k)^2 (A1 in direction k, M1 elsewhere) x_K
        for (int k = 0; k < D; ++k) {
            for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) bA[e] = bU[e];
            __syncthreads();
            const T* mats[3] = {t.M1, t.M1, t.M1};
            mats[k] = t.A1;
            const T* r = contract_axes<T, D>(bA, bB, S, ncell, L, L, mats, L, false);
            for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
                const int ci = e / S;
                T hk[3];
                const T J = hp_jac<T, D>(g, tb, g.order[start + ci], hk);
                const T c = J * ((T)2 / hk[k]) * ((T)2 / hk[k]);
                bY[e] += c * r[e];
            }
            __syncthreads();
        }
        // + B_K x_psi, written per local function
        for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
            const int ci = e / Pd, a = e - ci * Pd;
            bA[ci * S + a] = bX[ci * S + a];
        }
        __syncthreads();
        {
            const T* r = contract_all<T, D>(bA, bB, S, ncell, P, L, t.B1, P, false);
            for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
                const int ci = e / S, l = e - ci * S;
                const int64_t cell = g.order[start + ci];
                T hk[3];
                const T J = hp_jac<T, D>(g, tb, cell, hk);
                yloc[g.loc_off[cell] + l] = alpha * bY[e] + J * r[e];
            }
        }
        __syncthreads();
        // psi side: J B1^T x_K
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) bA[e] = bU[e];
        __syncthreads();
        {
            const T* r = contract_all<T, D>(bA, bB, S, ncell, L, P, t.B1, P, true);
            for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                const int ci = e / Pd, a = e - ci * Pd;
                T hk[3];
                const T J = hp_jac<T, D>(g, tb, g.order[start + ci], hk);
                bT[ci * S + a] = J * r[ci * S + a];
            }
        }
        __syncthreads();
        // the psi coefficients (APPLY: x_psi; RES: psi) to the Gauss points
        for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
            const int ci = e / Pd, a = e - ci * Pd;
            bA[ci * S + a] =
                MODE == MODE_RES ? xpsi[g.psi_off[g.order[start + ci]] + a] : bX[ci * S + a];
        }
        __syncthreads();
        T* vq = contract_all<T, D>(bA, bB, S, ncell, P, q, t.Vpsi, P, false);
        T* other = (vq == bA) ? bB : bA;
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = e / S, j = e - ci * S;
            const int64_t cell = g.order[start + ci];
            if (MODE == MODE_RES) {
                T hk[3];
                const T J = hp_jac<T, D>(g, tb, cell, hk);
                int jj[3] = {j % q, (j / q) % q, j / (q * q)};
                T wq = J;
                for (int k = 0; k < D; ++k) wq *= t.w[jj[k]];
                const double arg = -(double)vq[e];
                vq[e] = (T)((double)wq * exp(arg < 700.0 ? arg : 700.0));
            } else {
                vq[e] *= omega[g.qp_off[cell] + j];
            }
        }
        __syncthreads();
        const T* dx = contract_all<T, D>(vq, other, S, ncell, q, P, t.Vpsi, P, true);
        for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
            const int ci = e / Pd, a = e - ci * Pd;
            const int64_t cell = g.order[start + ci];
            const int64_t o = g.psi_off[cell] + a;
            if (MODE == MODE_RES) {
                const double r = (double)bT[ci * S + a] + (double)dx[ci * S + a] - Phi[o];
                ypsi[o] = (T)r;
            } else {
                T hk[3];
                const T J = hp_jac<T, D>(g, tb, cell, hk);
                int aa[3] = {a % P, (a / P) % P, a / (P * P)};
                T md = J;
                for (int k = 0; k < D; ++k) md *= t.Mdiag[aa[k]];
                const T y = bT[ci * S + a] - dx[ci * S + a] - beta * md * bX[ci * S + a];
                ypsi[o] = y;
            }
        }
        __syncthreads();   // the LDS buffers are reused by the next item
    }
}

// ---------------------------------------------------------------------------
// The same cell pass in 2-D with the contractions grouped by axis: every
// quantity is contracted along direction 1 first, all of them in one step
// from one read of the input column (x_K: M1, A1, B1^T; x_psi: B1, Vpsi),
// then along direction 0 (A_K x_K and B_K x_psi go straight to y_loc), so an
// item takes six barriers.  The 1-D tables of the item's degree and the
// per-cell factors and offsets are staged in LDS; index arithmetic uses a
// float reciprocal with an exact integer correction.

// floor(n / d) for 0 <= n < 2^22, 1 <= d, rd = 1 / d
__device__ inline int hp_div(int n, int d, float rd) {
    int q = (int)((float)n * rd);
    const int r = n - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_hp_cell2(HpGeo g, HpTabs<T> tb, T alpha, T beta,
                                                  const double* __restrict__ prm,
                                                  const T* __restrict__ xu,
                                                  const T* __restrict__ xpsi,
                                                  const T* __restrict__ xpsi_prev,
                                                  const T* __restrict__ omega,
                                                  const double* __restrict__ Phi,
                                                  T* __restrict__ yloc, T* __restrict__ ypsi,
                                                  const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (done && *done) return;
    if (prm) {
        alpha = (T)prm[0];
        beta = (T)prm[1];
    }
    const HpCell2Lds lay = hp_cell2_layout(g.lds_elems, g.lmax, (int)sizeof(T), MODE);
    int64_t* cLo = reinterpret_cast<int64_t*>(smem_raw);   // per cell: local, psi, qp offsets
    int64_t* cPo = cLo + lay.cmax;
    int64_t* cQo = cPo + lay.cmax;
    T* const base = reinterpret_cast<T*>(smem_raw + lay.off_t);
    const int SB = g.lds_elems;
    T* bU = base;             // x_K; later the weighted values at the Gauss points
    T* bX = base + SB;        // x_psi (RES: psi - psi_prev)
    T* tM = base + 2 * SB;    // M1 along direction 1 of x_K; later Vpsi^T along 1
    T* tA = base + 3 * SB;    // A1 along direction 1 of x_K
    T* tBt = base + 4 * SB;   // B1^T along direction 1 of x_K
    T* tB = base + 5 * SB;    // B1 along direction 1 of x_psi
    T* tV = base + 6 * SB;    // Vpsi along direction 1 of x_psi (RES: of psi)
    T* bT = base + 7 * SB;    // J B_K^T x_K
    T* bP = MODE == MODE_RES ? base + 8 * SB : bX;   // psi (RES)
    T* sA1 = base + lay.nbuf * SB;
    T* sM1 = sA1 + lay.l2;
    T* sB1 = sM1 + lay.l2;
    T* sV = sB1 + lay.l2;
    T* sMd = sV + lay.l2;
    T* sw = sMd + g.lmax;
    T* cJ = sw + g.lmax;
    T* cC0 = cJ + lay.cmax;
    T* cC1 = cC0 + lay.cmax;
    for (int it = blockIdx.x; it < g.n_items; it += gridDim.x) {
        const int p = g.item_p[it], L = p + 1, P = p - 1;
        const int S = L * L, LP = L * P, PP = P * P;
        const float rS = 1.0f / (float)S, rL = 1.0f / (float)L, rP = 1.0f / (float)P;
        const float rLP = 1.0f / (float)LP, rPP = 1.0f / (float)PP;
        const int start = g.item_start[it], ncell = g.item_count[it];
        const HpCellTabs<T> t = hp_tabs(tb, p);
        for (int e = threadIdx.x; e < S; e += blockDim.x) {
            sA1[e] = t.A1[e];
            sM1[e] = t.M1[e];
        }
        for (int e = threadIdx.x; e < LP; e += blockDim.x) {
            sB1[e] = t.B1[e];
            sV[e] = t.Vpsi[e];
        }
        for (int e = threadIdx.x; e < L; e += blockDim.x) {
            if (e < P) sMd[e] = t.Mdiag[e];
            sw[e] = t.w[e];
        }
        for (int ci = threadIdx.x; ci < ncell; ci += blockDim.x) {
            const int64_t cell = g.order[start + ci];
            T hk[3];
            const T J = hp_jac<T, 2>(g, tb, cell, hk);
            cJ[ci] = J;
            cC0[ci] = J * ((T)2 / hk[0]) * ((T)2 / hk[0]);
            cC1[ci] = J * ((T)2 / hk[1]) * ((T)2 / hk[1]);
            cLo[ci] = g.loc_off[cell];
            cPo[ci] = g.psi_off[cell];
            cQo[ci] = g.qp_off[cell];
        }
        // the gathers index through the offsets staged above (two dependent
        // global reads instead of four)
        __syncthreads();
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = hp_div(e, S, rS);
            const int gi = g.loc2glob[cLo[ci] + (e - ci * S)];
            bU[e] = gi >= 0 ? xu[gi] : (T)0;
        }
        for (int e = threadIdx.x; e < ncell * PP; e += blockDim.x) {
            const int ci = hp_div(e, PP, rPP), a = e - ci * PP;
            const int64_t o = cPo[ci] + a;
            if (MODE == MODE_RES) {
                bX[ci * S + a] = xpsi[o] - xpsi_prev[o];
                bP[ci * S + a] = xpsi[o];
            } else {
                bX[ci * S + a] = xpsi[o];
            }
        }
        __syncthreads();
        // ---- direction 1: x_K columns -> M1, A1 (L rows), B1^T (P rows)
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = hp_div(e, S, rS), r = e - ci * S;
            const int i1 = hp_div(r, L, rL), j0 = r - i1 * L;
            const T* col = bU + ci * S + j0;
            T am = 0, aa = 0, ab = 0;
            for (int j1 = 0; j1 < L; ++j1) {
                const T xv = col[j1 * L];
                am += sM1[i1 * L + j1] * xv;
                aa += sA1[i1 * L + j1] * xv;
                if (i1 < P) ab += sB1[j1 * P + i1] * xv;
            }
            tM[e] = am;
            tA[e] = aa;
            if (i1 < P) tBt[ci * S + j0 + L * i1] = ab;
        }
        // x_psi columns -> B1 (L rows), Vpsi (q = L rows)
        for (int e = threadIdx.x; e < ncell * LP; e += blockDim.x) {
            const int ci = hp_div(e, LP, rLP), r = e - ci * LP;
            const int i1 = hp_div(r, P, rP), a0 = r - i1 * P;
            const T* colx = bX + ci * S + a0;
            const T* colp = bP + ci * S + a0;
            T sb = 0, sv = 0;
            for (int a1 = 0; a1 < P; ++a1) {
                sb += sB1[i1 * P + a1] * colx[a1 * P];
                sv += sV[i1 * P + a1] * colp[a1 * P];
            }
            tB[ci * S + r] = sb;
            tV[ci * S + r] = sv;
        }
        __syncthreads();
        // ---- direction 0: y_loc = alpha (c0 A1 (x) M1 + c1 M1 (x) A1) x_K + J B1 (x) B1 x_psi
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = hp_div(e, S, rS), r = e - ci * S;
            const int i1 = hp_div(r, L, rL), i0 = r - i1 * L;
            const T* rm = tM + ci * S + L * i1;
            const T* ra = tA + ci * S + L * i1;
            const T* rb = tB + ci * S + P * i1;
            T s0 = 0, s1 = 0, sb = 0;
            for (int j0 = 0; j0 < L; ++j0) {
                s0 += sA1[i0 * L + j0] * rm[j0];
                s1 += sM1[i0 * L + j0] * ra[j0];
            }
            for (int a0 = 0; a0 < P; ++a0) sb += sB1[i0 * P + a0] * rb[a0];
            yloc[cLo[ci] + r] = alpha * (cC0[ci] * s0 + cC1[ci] * s1) + cJ[ci] * sb;
        }
        // J B1^T (x) B1^T x_K
        for (int e = threadIdx.x; e < ncell * PP; e += blockDim.x) {
            const int ci = hp_div(e, PP, rPP), r = e - ci * PP;
            const int a1 = hp_div(r, P, rP), a0 = r - a1 * P;
            const T* rb = tBt + ci * S + L * a1;
            T sb = 0;
            for (int j0 = 0; j0 < L; ++j0) sb += sB1[j0 * P + a0] * rb[j0];
            bT[ci * S + r] = cJ[ci] * sb;
        }
        // psi_h at the Gauss points (q = L per direction), times the weights
        for (int e = threadIdx.x; e < ncell * S; e += blockDim.x) {
            const int ci = hp_div(e, S, rS), r = e - ci * S;
            const int j1 = hp_div(r, L, rL), j0 = r - j1 * L;
            const T* rv = tV + ci * S + P * j1;
            T v = 0;
            for (int a0 = 0; a0 < P; ++a0) v += sV[j0 * P + a0] * rv[a0];
            if (MODE == MODE_RES) {
                const T wq = cJ[ci] * sw[j0] * sw[j1];
                const double arg = -(double)v;
                bU[e] = (T)((double)wq * exp(arg < 700.0 ? arg : 700.0));
            } else {
                bU[e] = omega[cQo[ci] + r] * v;
            }
        }
        __syncthreads();
        // ---- back to the Legendre modes: Vpsi^T along direction 1 ...
        for (int e = threadIdx.x; e < ncell * LP; e += blockDim.x) {
            const int ci = hp_div(e, LP, rLP), r = e - ci * LP;
            const int a1 = hp_div(r, L, rL), j0 = r - a1 * L;
            const T* col = bU + ci * S + j0;
            T sv = 0;
            for (int j1 = 0; j1 < L; ++j1) sv += sV[j1 * P + a1] * col[j1 * L];
            tM[ci * S + r] = sv;
        }
        __syncthreads();
        // ... and along direction 0; y_psi
        for (int e = threadIdx.x; e < ncell * PP; e += blockDim.x) {
            const int ci = hp_div(e, PP, rPP), r = e - ci * PP;
            const int a1 = hp_div(r, P, rP), a0 = r - a1 * P;
            const T* rw = tM + ci * S + L * a1;
            T dx = 0;
            for (int j0 = 0; j0 < L; ++j0) dx += sV[j0 * P + a0] * rw[j0];
            const int64_t o = cPo[ci] + r;
            if (MODE == MODE_RES) {
                const double res = (double)bT[ci * S + r] + (double)dx - Phi[o];
                ypsi[o] = (T)res;
            } else {
                const T xp = bX[ci * S + r];
                const T md = cJ[ci] * sMd[a0] * sMd[a1];
                const T y = bT[ci * S + r] - dx - beta * md * xp;
                ypsi[o] = y;
            }
        }
        __syncthreads();   // the LDS buffers are reused by the next item
    }
}

// ---------------------------------------------------------------------------
// The psi half of the reduction is taken here too, over fixed index ranges of
// y_psi (written by the cell pass), so that no sum depends on how the cells
// are grouped into work items.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_hp_gather(int64_t n_u, const int32_t* __restrict__ ip,
                                                   const int32_t* __restrict__ ix,
                                                   const T* __restrict__ yloc,
                                                   const double* __restrict__ F, double alpha,
                                                   const T* __restrict__ xu, T* __restrict__ yu,
                                                   int64_t n_psi, const T* __restrict__ xpsi,
                                                   const T* __restrict__ ypsi,
                                                   double* __restrict__ partial,
                                                   const int* __restrict__ done) {
    __shared__ double red[4];
    if (done && *done) return;
    double part = 0.0;
    for (int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gi < n_u;
         gi += (int64_t)gridDim.x * blockDim.x) {
        T s = 0;
        for (int i = ip[gi]; i < ip[gi + 1]; ++i) s += yloc[ix[i]];
        if (MODE == MODE_RES) {
            const double r = (double)s - alpha * F[gi];
            yu[gi] = (T)r;
            part += r * r;
        } else {
            yu[gi] = s;
            part += (double)s * (double)xu[gi];
        }
    }
    if (!partial) return;
    double pp = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_psi;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double y = (double)ypsi[k];
        pp += MODE == MODE_RES ? y * y : y * (double)xpsi[k];
    }
    const double s = block_sum(part, red);
    const double sp = block_sum(pp, red);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        partial[gridDim.x + blockIdx.x] = sp;
    }
}

// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_hp_l2(HpGeo g, HpTabs<double> tb,
                                               const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int SB = g.lds_elems;
    double* bD = sm;
    double* bN = sm + SB;
    double* bA = sm + 2 * SB;
    double* bB = sm + 3 * SB;
    double pd = 0.0, pn = 0.0;
    // one cell at a time (cells blockIdx.x, + gridDim.x, ...): the sums do not
    // depend on the work items
    for (int64_t cell = blockIdx.x; cell < g.n_cells; cell += gridDim.x) {
        const int p = g.cell_p[cell], L = p + 1, q = p + 1;
        int S = 1;
        for (int k = 0; k < D; ++k) S *= L;
        const HpCellTabs<double> t = hp_tabs(tb, p);
        for (int l = threadIdx.x; l < S; l += blockDim.x) {
            const int gi = g.loc2glob[g.loc_off[cell] + l];
            bD[l] = gi >= 0 ? a[gi] - b[gi] : 0.0;
            bN[l] = gi >= 0 ? a[gi] : 0.0;
        }
        __syncthreads();
        const double* vd = contract_all<double, D>(bD, bA, S, 1, L, q, t.Vu, L, false);
        const double* vn = contract_all<double, D>(bN, bB, S, 1, L, q, t.Vu, L, false);
        for (int j = threadIdx.x; j < S; j += blockDim.x) {
            const int e = j;
            double hk[3];
            const double J = hp_jac<double, D>(g, tb, cell, hk);
            int jj[3] = {j % q, (j / q) % q, j / (q * q)};
            double wq = J;
            for (int k = 0; k < D; ++k) wq *= t.w[jj[k]];
            pd += wq * vd[e] * vd[e];
            pn += wq * vn[e] * vn[e];
        }
        __syncthreads();
    }
    const double s1 = block_sum(pd, red);
    const double s2 = block_sum(pn, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s1;
        partial[2 * blockIdx.x + 1] = s2;
    }
}

// ---------------------------------------------------------------------------
// Newton-step setup, one cell per block (sizes vary by cell): the block of
// -S_hat_K is formed and inverted in LDS (LDSD, when the largest block fits)
// or in place in s64 (global memory).  1024 threads: one block holds a CU's
// LDS, so its own waves hide the LDS latency of the elimination.
template <int D, bool LDSD>
__global__ __launch_bounds__(1024) void k_hp_setup(HpGeo g, HpTabs<double> tb,
                                                  const double* __restrict__ psi, double alpha,
                                                  double beta, const double* __restrict__ Cmat,
                                                  const int64_t* __restrict__ c_off,
                                                  const int32_t* __restrict__ cclass,
                                                  double* __restrict__ om64,
                                                  float* __restrict__ om32,
                                                  double* __restrict__ s64,
                                                  float* __restrict__ s32, int o0) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int64_t cell = g.order[o0 + (int)blockIdx.x];
    const int p = g.cell_p[cell], P = p - 1, q = p + 1;
    int n = 1, S = 1;
    for (int k = 0; k < D; ++k) {
        n *= P;
        S *= q;
    }
    const int sT1 = D == 1 ? 1 : (D == 2 ? q * P * P : q * q * P * P);
    double* bA = sm;
    double* bB = sm + S;
    double* T1 = sm + 2 * S;
    double* cr = T1 + sT1;
    const HpCellTabs<double> t = hp_tabs(tb, p);
    const int64_t po = g.psi_off[cell], qo = g.qp_off[cell];
    // cr: the pivot column and row (2n; 256 for the register elimination)
    double* Dm = LDSD ? cr + (2 * n > 256 ? 2 * n : 256) : s64 + g.sinv_off[cell];
    for (int a = threadIdx.x; a < n; a += blockDim.x) bA[a] = psi[po + a];
    __syncthreads();
    double* vq = contract_all<double, D>(bA, bB, S, 1, P, q, t.Vpsi, P, false);
    double hk[3];
    const double J = hp_jac<double, D>(g, tb, cell, hk);
    for (int j = threadIdx.x; j < S; j += blockDim.x) {
        int jj[3] = {j % q, (j / q) % q, j / (q * q)};
        double wq = J;
        for (int k = 0; k < D; ++k) wq *= t.w[jj[k]];
        const double arg = -vq[j];
        const double om = wq * exp(arg < 700.0 ? arg : 700.0);
        vq[j] = om;
        if (om64) om64[qo + j] = om;
        if (om32) om32[qo + j] = (float)om;
    }
    __syncthreads();
    if (D == 3)
        d_block3_direct(vq, t.Vpsi, P, q, T1, Dm, n);
    else
        d_block<D>(vq, t.Vpsi, P, q, T1, T1, Dm, n);
    const double ia = 1.0 / alpha;
    const double* C = Cmat + c_off[cclass[cell]];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = Dm[e] + ia * C[e];
        if (i == j) {
            int aa[3] = {i % P, (i / P) % P, i / (P * P)};
            double md = J;
            for (int k = 0; k < D; ++k) md *= t.Mdiag[aa[k]];
            v += beta * md;
        }
        Dm[e] = v;
    }
    __syncthreads();
    if (LDSD && n <= 128)
        gauss_jordan_spd_reg(Dm, n, cr);   // 1024 threads: the block in registers
    else
        gauss_jordan_spd(Dm, n, cr);
    const int64_t so = g.sinv_off[cell];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        if (j < i) continue;
        const double v = 0.5 * (Dm[(int64_t)i * n + j] + Dm[(int64_t)j * n + i]);
        if (LDSD) {
            if (s64) {
                s64[so + (int64_t)i * n + j] = v;
                s64[so + (int64_t)j * n + i] = v;
            }
        } else {
            Dm[(int64_t)i * n + j] = v;
            Dm[(int64_t)j * n + i] = v;
        }
        if (s32) {
            s32[so + (int64_t)i * n + j] = (float)v;
            s32[so + (int64_t)j * n + i] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// z_psi = (-S_hat_K)^{-1} r_psi, one cell per block (largest blocks first):
// the 256 threads split into nsplit groups that each sum a range of j for
// every row i (the inverse is symmetric: row j read as column j, coalesced),
// and the group sums are added in LDS in a fixed order
template <typename T>
__device__ inline void hp_prec_psi_body(int bid, int nblk, const HpGeo& g,
                                        const T* __restrict__ sinv, const T* __restrict__ r,
                                        T* __restrict__ z, double* __restrict__ partial, T* rb,
                                        T* acc_s, double* red) {
    double part = 0.0;
    for (int64_t b = bid; b < g.n_cells; b += nblk) {
        const int64_t cell = g.order[b];
        const int P = g.cell_p[cell] - 1;
        int n = 1;
        for (int k = 0; k < g.d; ++k) n *= P;
        const int64_t po = g.psi_off[cell];
        for (int i = threadIdx.x; i < n; i += blockDim.x) rb[i] = r[po + i];
        __syncthreads();
        const T* Sb = sinv + g.sinv_off[cell];
        const int nsplit = n >= 256 ? 1 : 256 / n;
        const int chunk = (n + nsplit - 1) / nsplit;
        for (int i0 = 0; i0 < n; i0 += 256 / nsplit) {
            const int t = threadIdx.x;
            const int grp = t / (256 / nsplit), i = i0 + t % (256 / nsplit);
            T acc = 0;
            if (grp < nsplit && i < n) {
                const int j1 = min(n, (grp + 1) * chunk);
                T a1 = 0, a2 = 0, a3 = 0;
                int j = grp * chunk;
                for (; j + 4 <= j1; j += 4) {
                    acc += Sb[(int64_t)j * n + i] * rb[j];
                    a1 += Sb[(int64_t)(j + 1) * n + i] * rb[j + 1];
                    a2 += Sb[(int64_t)(j + 2) * n + i] * rb[j + 2];
                    a3 += Sb[(int64_t)(j + 3) * n + i] * rb[j + 3];
                }
                for (; j < j1; ++j) acc += Sb[(int64_t)j * n + i] * rb[j];
                acc = (acc + a1) + (a2 + a3);
            }
            acc_s[t] = acc;
            __syncthreads();
            if (t < 256 / nsplit && i0 + t < n) {
                T s = 0;
                for (int q = 0; q < nsplit; ++q) s += acc_s[q * (256 / nsplit) + t];
                z[po + i0 + t] = s;
                part += (double)s * (double)rb[i0 + t];
            }
            __syncthreads();
        }
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[bid] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_hp_prec_psi(HpGeo g, const T* __restrict__ sinv,
                                                     const T* __restrict__ r,
                                                     T* __restrict__ z,
                                                     double* __restrict__ partial,
                                                     const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    __shared__ T acc_s[256];
    if (done && *done) return;
    hp_prec_psi_body<T>(blockIdx.x, gridDim.x, g, sinv, r, z, partial,
                        reinterpret_cast<T*>(smem_raw), acc_s, red);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_hp_vgather(int64_t n, const int32_t* __restrict__ idx,
                                                    const T* __restrict__ r, T* __restrict__ out,
                                                    const int* __restrict__ done) {
    if (done && *done) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = r[idx[i]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_hp_vscatter(int64_t n, const int32_t* __restrict__ idx,
                                                     const T* __restrict__ in,
                                                     T* __restrict__ z,
                                                     const int* __restrict__ done) {
    if (done && *done) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        z[idx[i]] = in[i];
}

// z_E = (1/alpha) Ainv_E r_E for the non-vertex entities, one chunk of
// entities sharing an inverse at a time: their r_E side by side in LDS (rs),
// then per row i of the inverse (read as column i, coalesced: it is
// symmetric) all the chunk's z_E[i] from one read of the row.  Optionally the
// block's share of <z, r> over those unknowns goes to partial[bid].
template <typename T>
__device__ inline void hp_entity_body(int64_t bid, int64_t nblk, const HpEnt& ent,
                                      const T* __restrict__ inv, T ia, const T* __restrict__ r,
                                      T* __restrict__ z, double* __restrict__ partial, T* rs,
                                      double* red) {
    double part = 0.0;
    for (int64_t ch = bid; ch < ent.nchunk; ch += nblk) {
        const int c0 = ent.cstart[ch], nc = ent.ccount[ch];
        const int n = ent.cnt[ent.list[c0]];
        const T* A = inv + ent.off[ent.list[c0]];
        const bool rows = hp_ent_rows(n);
        if (rows) {
            // the chunk's right-hand sides interleaved, rs[j kHpEntChunk + c]
            // (zeros past the last entity: the accumulators cover kHpEntChunk)
            for (int k = threadIdx.x; k < kHpEntChunk * n; k += blockDim.x) {
                const int j = k / kHpEntChunk, c = k - j * kHpEntChunk;
                rs[k] = c < nc ? r[ent.first[ent.list[c0 + c]] + j] : T(0);
            }
        } else {
            // entity by entity, rs[c n + j]
            for (int k = threadIdx.x; k < nc * n; k += blockDim.x) {
                const int c = k / n, j = k - c * n;
                rs[k] = r[ent.first[ent.list[c0 + c]] + j];
            }
        }
        __syncthreads();
        if (rows) {
            // ng groups of 256 / ng threads, group g summing j in its range for
            // the rows i0 + t; groups 1.. leave their sums in ps, group 0 adds
            // them in order of g
            const int ng = hp_ent_groups(n), rpg = 256 / ng, jc = (n + ng - 1) / ng;
            T* ps = rs + kHpEntChunk * n;
            const int t = threadIdx.x, grp = t / rpg;
            for (int i0 = 0; i0 < n; i0 += rpg) {
                const int i = i0 + t % rpg;
                T acc[kHpEntChunk];
#pragma unroll
                for (int c = 0; c < kHpEntChunk; ++c) acc[c] = 0;
                if (i < n) {
                    const int j1 = min(n, (grp + 1) * jc);
                    // U rows of loads in flight, then their products in order of
                    // j (FP32: 2, so that the fused launch's psi blocks, which
                    // share its register budget, keep their occupancy)
                    constexpr int U = sizeof(T) == sizeof(double) ? 8 : 2;
                    int j = grp * jc;
                    for (; j + U <= j1; j += U) {
                        T a[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) a[u] = A[(int64_t)(j + u) * n + i];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const T* rj = rs + (j + u) * kHpEntChunk;
#pragma unroll
                            for (int c = 0; c < kHpEntChunk; ++c) acc[c] += a[u] * rj[c];
                        }
                    }
                    for (; j < j1; ++j) {
                        const T a = A[(int64_t)j * n + i];
                        const T* rj = rs + j * kHpEntChunk;
#pragma unroll
                        for (int c = 0; c < kHpEntChunk; ++c) acc[c] += a * rj[c];
                    }
                }
                if (ng > 1) {
                    if (grp > 0) {
#pragma unroll
                        for (int c = 0; c < kHpEntChunk; ++c)
                            ps[((grp - 1) * rpg + t % rpg) * kHpEntChunk + c] = acc[c];
                    }
                    __syncthreads();
                    if (grp == 0) {
                        for (int q = 1; q < ng; ++q) {
#pragma unroll
                            for (int c = 0; c < kHpEntChunk; ++c)
                                acc[c] += ps[((q - 1) * rpg + t) * kHpEntChunk + c];
                        }
                    }
                    __syncthreads();   // ps is reused by the next rows
                }
                if (grp == 0 && i < n) {
#pragma unroll
                    for (int c = 0; c < kHpEntChunk; ++c) {
                        if (c < nc) {
                            const T zv = ia * acc[c];
                            z[ent.first[ent.list[c0 + c]] + i] = zv;
                            part += (double)zv * (double)rs[i * kHpEntChunk + c];
                        }
                    }
                }
            }
        } else {
            for (int k = threadIdx.x; k < nc * n; k += blockDim.x) {
                const int c = k / n, i = k - c * n;
                const T* rc = rs + c * n;
                T acc = 0;
                int j = 0;
                for (; j + 8 <= n; j += 8) {
                    T a[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) a[u] = A[(int64_t)(j + u) * n + i];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += a[u] * rc[j + u];
                }
                for (; j < n; ++j) acc += A[(int64_t)j * n + i] * rc[j];
                const T zv = ia * acc;
                z[ent.first[ent.list[c0 + c]] + i] = zv;
                part += (double)zv * (double)rs[k];
            }
        }
        __syncthreads();   // rs is refilled by the next chunk
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[bid] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_hp_entity(HpEnt ent, const T* __restrict__ inv,
                                                   const double* __restrict__ prm,
                                                   const T* __restrict__ r, T* __restrict__ z,
                                                   const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    if (done && *done) return;
    hp_entity_body<T>(blockIdx.x, gridDim.x, ent, inv, (T)prm[2], r, z, nullptr,
                      reinterpret_cast<T*>(smem_raw), red);
}

// The three independent parts of the block preconditioner in one grid:
// blocks [0, ne) the entity chunks (with their share of <z, r> in epart;
// first, so that their cache-bound work overlaps the streaming of the
// psi-blocks), [ne, ne + np) the psi-block cells, the rest gathers the vertex
// residual.
template <typename T>
__global__ __launch_bounds__(256) void k_hp_prec_fused(HpGeo g, const T* __restrict__ sinv,
                                                       int np, int ne, HpEnt ent, const T* inv,
                                                       const double* __restrict__ prm,
                                                       const int32_t* __restrict__ vidx,
                                                       int64_t nv, T* __restrict__ cv,
                                                       const T* __restrict__ r, T* __restrict__ z,
                                                       double* __restrict__ ppart,
                                                       double* __restrict__ epart,
                                                       const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    __shared__ T acc_s[256];
    if (done && *done) return;
    const int b = blockIdx.x;
    if (b < ne) {
        hp_entity_body<T>(b, ne, ent, inv, (T)prm[2], r, z, epart,
                          reinterpret_cast<T*>(smem_raw), red);
    } else if (b < ne + np) {
        hp_prec_psi_body<T>(b - ne, np, g, sinv, r + g.n_u, z + g.n_u, ppart,
                            reinterpret_cast<T*>(smem_raw), acc_s, red);
    } else {
        const int64_t nb = gridDim.x - np - ne;
        for (int64_t i = (int64_t)(b - np - ne) * blockDim.x + threadIdx.x; i < nv;
             i += nb * blockDim.x)
            cv[i] = r[vidx[i]];
    }
}

// z at the vertices from the coarse solution, with their share of <z, r>
template <typename T>
__global__ __launch_bounds__(256) void k_hp_vscatter_dot(int64_t n, const int32_t* __restrict__ idx,
                                                         const T* __restrict__ in,
                                                         const T* __restrict__ r,
                                                         T* __restrict__ z,
                                                         double* __restrict__ partial,
                                                         const int* __restrict__ done) {
    __shared__ double red[4];
    if (done && *done) return;
    double part = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gi = idx[i];
        z[gi] = in[i];
        part += (double)in[i] * (double)r[gi];
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// The vertex block of the 2-D preconditioner in one workgroup: (alpha A_VV)^{-1}
// r_V by fast diagonalisation, V1 [(V1^T R V0) / (alpha (lam1_i + lam0_j))] V0^T
// with R the interior-vertex residual as an n1 x n0 array, when the grid is at
// most 64 x 64.  The eigenvector matrices, R and the intermediates stay in LDS
// (zero-padded to multiples of 16; row pitch one more than that), and each
// product is a 16 x 16 MFMA tile per wave; gather, the four products, scatter
// and the vertex share of <z, r> take one launch instead of six.
typedef double hp_v4d __attribute__((ext_vector_type(4)));
typedef float hp_v4f __attribute__((ext_vector_type(4)));
__device__ inline hp_v4d hp_mfma(double a, double b, hp_v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline hp_v4f hp_mfma(float a, float b, hp_v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
struct HpV4 {
    using V = hp_v4d;
};
template <>
struct HpV4<float> {
    using V = hp_v4f;
};

// C (M x N) = op(A) op(B), K terms, all dimensions multiples of 16 (K of 4);
// TA: op(A)[i][k] = A[k][i]; TB: op(B)[k][j] = B[j][k].  (ri, ci): the tile
// row and column of each of the lane's four results.  epi(i, j, s) is stored.
template <typename T, bool TA, bool TB, typename Epi>
__device__ inline void hp_lds_gemm(const T* A, int lda, const T* B, int ldb, T* C, int ldc, int M,
                                   int N, int K, const int* ri, const int* ci, Epi epi) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int tn = N / 16, r = lane & 15, kk = lane >> 4;
    for (int t = w; t < (M / 16) * tn; t += nw) {
        const int i0 = (t / tn) * 16, j0 = (t % tn) * 16;
        // two accumulators (even / odd slabs of 4 terms) halve the MFMA chain
        typename HpV4<T>::V acc = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
#pragma unroll 4
        for (int k0 = 0; k0 < K; k0 += 8) {
            const int k = k0 + kk;
            const T a = TA ? A[k * lda + i0 + r] : A[(i0 + r) * lda + k];
            const T b = TB ? B[(j0 + r) * ldb + k] : B[k * ldb + j0 + r];
            acc = hp_mfma(a, b, acc);
            if (k0 + 4 < K) {
                const T a1 = TA ? A[(k + 4) * lda + i0 + r] : A[(i0 + r) * lda + k + 4];
                const T b1 = TB ? B[(j0 + r) * ldb + k + 4] : B[(k + 4) * ldb + j0 + r];
                acc1 = hp_mfma(a1, b1, acc1);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ri[v], j = j0 + ci[v];
            C[i * ldc + j] = epi(i, j, acc[v] + acc1[v]);
        }
    }
}

__host__ __device__ inline int hp_pad16(int n) { return (n + 15) & ~15; }

size_t hp_vsolve2_lds(int n0, int n1, size_t tsize) {
    const size_t N0 = hp_pad16(n0), N1 = hp_pad16(n1);
    return tsize * (N0 * (N0 + 1) + N1 * (N1 + 1) + 2 * N1 * (N0 + 1));
}

template <typename T>
__global__ __launch_bounds__(1024) void k_hp_vsolve2(int n0, int n1,
                                                     const int32_t* __restrict__ vidx,
                                                     const T* __restrict__ V0,
                                                     const T* __restrict__ V1,
                                                     const T* __restrict__ l0,
                                                     const T* __restrict__ l1,
                                                     const double* __restrict__ prm,
                                                     const T* __restrict__ rv, T* __restrict__ z,
                                                     double* __restrict__ partial, int npart,
                                                     const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    __shared__ T sl0[64], sl1[64];
    if (done && *done) return;
    const int N0 = hp_pad16(n0), N1 = hp_pad16(n1), P0 = N0 + 1, P1 = N1 + 1;
    T* sV0 = reinterpret_cast<T*>(smem_raw);   // N0 x N0, pitch P0
    T* sV1 = sV0 + N0 * P0;                      // N1 x N1, pitch P1
    T* X = sV1 + N1 * P1;                        // N1 x N0, pitch P0
    T* Y = X + N1 * P0;
    // every global load is issued before the first LDS store (each thread has
    // at most 4 entries of each 64 x 64 array), so the prologue waits for one
    // memory round trip: the vertex residual rv comes gathered (by the launch
    // before), the vertex indices are needed only for the scatter
    constexpr int NT = 1024, NE = 4;
    const int tid = (int)threadIdx.x, nv = n0 * n1;
    T a0[NE], a1[NE], rr[NE];
    int gi[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = tid + NT * m;
        const int i0 = e / N0, j0 = e - i0 * N0, i1 = e / N1, j1 = e - i1 * N1;
        a0[m] = (i0 < n0 && j0 < n0) ? V0[i0 * n0 + j0] : (T)0;
        a1[m] = (i1 < n1 && j1 < n1) ? V1[i1 * n1 + j1] : (T)0;
        gi[m] = e < nv ? vidx[e] : 0;
    }
    T el0 = tid < n0 ? l0[tid] : (T)1, el1 = tid < n1 ? l1[tid] : (T)1;
#pragma unroll
    for (int m = 0; m < NE; ++m) rr[m] = tid + NT * m < nv ? rv[tid + NT * m] : (T)0;
    if (tid < 64) {
        sl0[tid] = el0;
        sl1[tid] = el1;
    }
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = tid + NT * m;
        if (e < N0 * N0) sV0[(e / N0) * P0 + e % N0] = a0[m];
        if (e < N1 * N1) sV1[(e / N1) * P1 + e % N1] = a1[m];
        if (e < N1 * N0) {   // padding of X
            const int i = e / N0, j = e - i * N0;
            if (i >= n1 || j >= n0) X[i * P0 + j] = (T)0;
        }
        if (e < nv) X[(e / n0) * P0 + e % n0] = rr[m];
    }
    // tile positions of the four results of this lane: an MFMA with
    // A[i][0] = i, B[0][j] = 1 gives i, one with A[i][0] = 1, B[0][j] = j gives j
    const int lane = threadIdx.x & 63, kk = lane >> 4;
    const typename HpV4<T>::V zero = {0, 0, 0, 0};
    const typename HpV4<T>::V rid =
        hp_mfma(kk == 0 ? (T)(lane & 15) : (T)0, kk == 0 ? (T)1 : (T)0, zero);
    const typename HpV4<T>::V cid =
        hp_mfma(kk == 0 ? (T)1 : (T)0, kk == 0 ? (T)(lane & 15) : (T)0, zero);
    int ri[4], ci[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        ri[v] = (int)rid[v] & 15;
        ci[v] = (int)cid[v] & 15;
    }
    __syncthreads();
    auto same = [](int, int, T s) { return s; };
    hp_lds_gemm<T, false, false>(X, P0, sV0, P0, Y, P0, N1, N0, N0, ri, ci, same);   // R V0
    __syncthreads();
    const T ia = (T)prm[2];
    hp_lds_gemm<T, true, false>(sV1, P1, Y, P0, X, P0, N1, N0, N1, ri, ci,
                                [&](int i, int j, T s) {
                                    return (i < n1 && j < n0) ? s * ia / (sl1[i] + sl0[j]) : (T)0;
                                });   // V1^T (.), eigen-space division
    __syncthreads();
    hp_lds_gemm<T, false, true>(X, P0, sV0, P0, Y, P0, N1, N0, N0, ri, ci, same);    // (.) V0^T
    __syncthreads();
    hp_lds_gemm<T, false, false>(sV1, P1, Y, P0, X, P0, N1, N0, N1, ri, ci, same);   // V1 (.)
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = tid + NT * m;
        if (e < nv) {
            const T v = X[(e / n0) * P0 + e % n0];
            z[gi[m]] = v;
            part += (double)v * (double)rr[m];
        }
    }
    if (partial) {
        const double sum = block_sum(part, red);
        if (threadIdx.x == 0) partial[0] = sum;
        for (int i = 1 + (int)threadIdx.x; i < npart; i += blockDim.x) partial[i] = 0.0;
    }
}

template <typename T>
void launch_hp_vsolve2(int n0, int n1, const int32_t* vidx, const T* V0, const T* V1, const T* l0,
                       const T* l1, const double* prm, const T* rv, T* z, double* partial,
                       int npart, const int* done, hipStream_t s) {
    hipLaunchKernelGGL((k_hp_vsolve2<T>), dim3(1), dim3(1024), hp_vsolve2_lds(n0, n1, sizeof(T)),
                       s, n0, n1, vidx, V0, V1, l0, l1, prm, rv, z, partial, npart, done);
}

// ---------------------------------------------------------------------------
static inline unsigned grid_of(int64_t n, int b, int cap) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + b - 1) / b, cap));
}

template <typename T>
void launch_hp_cell(const HpGeo& g, const HpTabs<T>& tb, T alpha, T beta, const double* prm,
                    const T* xu, const T* xpsi, const T* xpsi_prev, const T* omega,
                    const double* Phi, T* yloc, T* ypsi, int nblocks, const int* done, int mode,
                    hipStream_t s) {
    const unsigned grid = (unsigned)std::max(1, std::min(g.n_items, nblocks));
    const size_t shm = hp_cell_lds(g.d, g.lds_elems, g.lmax, sizeof(T), mode);
    if (g.d == 2) {
        if (mode == MODE_RES)
            hipLaunchKernelGGL((k_hp_cell2<T, MODE_RES>), dim3(grid), dim3(256), shm, s, g, tb,
                               alpha, beta, prm, xu, xpsi, xpsi_prev, omega, Phi, yloc, ypsi,
                               done);
        else
            hipLaunchKernelGGL((k_hp_cell2<T, MODE_APPLY>), dim3(grid), dim3(256), shm, s, g, tb,
                               alpha, beta, prm, xu, xpsi, xpsi_prev, omega, Phi, yloc, ypsi,
                               done);
        return;
    }
#define HPG_HC(DD, MM)                                                                          \
    hipLaunchKernelGGL((k_hp_cell<T, DD, MM>), dim3(grid), dim3(256), shm, s, g, tb, alpha, beta, \
                       prm, xu, xpsi, xpsi_prev, omega, Phi, yloc, ypsi, done)
    if (mode == MODE_RES) {
        if (g.d == 1) HPG_HC(1, MODE_RES);
        else HPG_HC(3, MODE_RES);
    } else {
        if (g.d == 1) HPG_HC(1, MODE_APPLY);
        else HPG_HC(3, MODE_APPLY);
    }
#undef HPG_HC
}

template <typename T>
void launch_hp_gather(int64_t n_u, const int32_t* inc_ptr, const int32_t* inc_idx, const T* yloc,
                      const double* F, double alpha, const T* xu, T* yu, int64_t n_psi,
                      const T* xpsi, const T* ypsi, double* partial, int nblocks, const int* done,
                      int mode, hipStream_t s) {
    const unsigned grid = (unsigned)std::max(1, nblocks);
    if (mode == MODE_RES)
        hipLaunchKernelGGL((k_hp_gather<T, MODE_RES>), dim3(grid), dim3(256), 0, s, n_u, inc_ptr,
                           inc_idx, yloc, F, alpha, xu, yu, n_psi, xpsi, ypsi, partial, done);
    else
        hipLaunchKernelGGL((k_hp_gather<T, MODE_APPLY>), dim3(grid), dim3(256), 0, s, n_u, inc_ptr,
                           inc_idx, yloc, F, alpha, xu, yu, n_psi, xpsi, ypsi, partial, done);
}

void launch_hp_l2(const HpGeo& g, const HpTabs<double>& tb, const double* a, const double* b,
                  double* partial, int nblocks, hipStream_t s) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(g.n_cells, nblocks));
    const size_t shm = (size_t)4 * g.lds_elems * sizeof(double);
    if (g.d == 1)
        hipLaunchKernelGGL((k_hp_l2<1>), dim3(grid), dim3(256), shm, s, g, tb, a, b, partial);
    else if (g.d == 2)
        hipLaunchKernelGGL((k_hp_l2<2>), dim3(grid), dim3(256), shm, s, g, tb, a, b, partial);
    else
        hipLaunchKernelGGL((k_hp_l2<3>), dim3(grid), dim3(256), shm, s, g, tb, a, b, partial);
}

size_t hp_setup_lds_p(int d, int p, bool block_in_lds) {
    const size_t P = p - 1, q = p + 1;
    size_t n = 1, S = 1;
    for (int k = 0; k < d; ++k) {
        n *= P;
        S *= q;
    }
    const size_t sT1 = d == 1 ? 1 : (d == 2 ? q * P * P : q * q * P * P);
    return (2 * S + sT1 + std::max<size_t>(2 * n, 256) + (block_in_lds ? n * n : 0)) *
           sizeof(double);
}

size_t hp_setup_lds(int d, int pmax, bool block_in_lds) {
    size_t best = 0;
    for (int p = 2; p <= pmax; ++p) best = std::max(best, hp_setup_lds_p(d, p, block_in_lds));
    return best;
}

void launch_hp_setup(const HpGeo& g, const HpTabs<double>& tb, const double* psi, double alpha,
                     double beta, const double* C, const int64_t* c_off, const int32_t* cclass,
                     double* om64, float* om32, double* s64, float* s32, size_t lds_bytes,
                     bool block_in_lds, int o0, int ncell, hipStream_t s) {
    const unsigned grid = (unsigned)ncell;
#define HPG_HS(DD, LL)                                                                       \
    hipLaunchKernelGGL((k_hp_setup<DD, LL>), dim3(grid), dim3(1024), lds_bytes, s, g, tb, psi, \
                       alpha, beta, C, c_off, cclass, om64, om32, s64, s32, o0)
    if (block_in_lds) {
        if (g.d == 1) HPG_HS(1, true);
        else if (g.d == 2) HPG_HS(2, true);
        else HPG_HS(3, true);
    } else {
        if (g.d == 1) HPG_HS(1, false);
        else if (g.d == 2) HPG_HS(2, false);
        else HPG_HS(3, false);
    }
#undef HPG_HS
}

template <typename T>
void launch_hp_prec_psi(const HpGeo& g, const T* sinv, const T* r, T* z, double* partial,
                        int nblocks, int nmax, const int* done, hipStream_t s) {
    const unsigned grid = grid_of(g.n_cells, 1, nblocks);
    hipLaunchKernelGGL((k_hp_prec_psi<T>), dim3(grid), dim3(256), (size_t)nmax * sizeof(T), s, g,
                       sinv, r, z, partial, done);
}

template <typename T>
void launch_hp_vgather(int64_t n, const int32_t* idx, const T* r, T* out, const int* done,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_hp_vgather<T>), dim3(grid_of(n, 256, 1024)), dim3(256), 0, s, n, idx, r,
                       out, done);
}

template <typename T>
void launch_hp_vscatter(int64_t n, const int32_t* idx, const T* in, T* z, const int* done,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_hp_vscatter<T>), dim3(grid_of(n, 256, 1024)), dim3(256), 0, s, n, idx,
                       in, z, done);
}

template <typename T>
void launch_hp_entity(const HpEnt& ent, const T* inv, const double* prm, const T* r, T* z,
                      const int* done, hipStream_t s) {
    if (ent.nchunk <= 0) return;
    hipLaunchKernelGGL((k_hp_entity<T>), dim3(grid_of(ent.nchunk, 1, 8192)), dim3(256),
                       (size_t)ent.lds * sizeof(T), s, ent, inv, prm, r, z, done);
}

int hp_prec_entity_blocks(int nchunk) { return nchunk > 0 ? (int)grid_of(nchunk, 1, 2048) : 0; }
int hp_vscatter_blocks(int64_t nv) { return (int)grid_of(nv, 256, 256); }

template <typename T>
void launch_hp_prec_fused(const HpGeo& g, const T* sinv, int np, int nmax, int ne,
                          const HpEnt& ent, const T* inv, const double* prm, const int32_t* vidx,
                          int64_t nv, T* cv, const T* r, T* z, double* ppart, double* epart,
                          const int* done, hipStream_t s) {
    const int nvb = nv > 0 ? (int)grid_of(nv, 256, 64) : 0;
    const size_t lds = (size_t)std::max(nmax, ne > 0 ? ent.lds : 0) * sizeof(T);
    hipLaunchKernelGGL((k_hp_prec_fused<T>), dim3(np + ne + nvb), dim3(256), lds, s, g, sinv,
                       np, ne, ent, inv, prm, vidx, nv, cv, r, z, ppart, epart, done);
}

template <typename T>
void launch_hp_vscatter_dot(int64_t nv, const int32_t* idx, const T* in, const T* r, T* z,
                            double* partial, const int* done, hipStream_t s) {
    hipLaunchKernelGGL((k_hp_vscatter_dot<T>), dim3(hp_vscatter_blocks(nv)), dim3(256), 0, s, nv,
                       idx, in, r, z, partial, done);
}

#define HPG_INST(T)                                                                               \
    template void launch_hp_cell<T>(const HpGeo&, const HpTabs<T>&, T, T, const double*, const T*, \
                                    const T*, const T*, const T*, const double*, T*, T*, int,      \
                                    const int*, int, hipStream_t);                                 \
    template void launch_hp_gather<T>(int64_t, const int32_t*, const int32_t*, const T*,          \
                                      const double*, double, const T*, T*, int64_t, const T*,     \
                                      const T*, double*, int, const int*, int, hipStream_t);      \
    template void launch_hp_prec_psi<T>(const HpGeo&, const T*, const T*, T*, double*, int, int,  \
                                        const int*, hipStream_t);                                  \
    template void launch_hp_vgather<T>(int64_t, const int32_t*, const T*, T*, const int*,         \
                                       hipStream_t);                                               \
    template void launch_hp_vscatter<T>(int64_t, const int32_t*, const T*, T*, const int*,        \
                                        hipStream_t);                                              \
    template void launch_hp_prec_fused<T>(const HpGeo&, const T*, int, int, int, const HpEnt&,    \
                                          const T*, const double*, const int32_t*, int64_t, T*,   \
                                          const T*, T*, double*, double*, const int*,             \
                                          hipStream_t);                                            \
    template void launch_hp_vscatter_dot<T>(int64_t, const int32_t*, const T*, const T*, T*,     \
                                            double*, const int*, hipStream_t);                     \
    template void launch_hp_vsolve2<T>(int, int, const int32_t*, const T*, const T*, const T*,    \
                                       const T*, const double*, const T*, T*, double*, int,        \
                                       const int*, hipStream_t);                                   \
    template void launch_hp_entity<T>(const HpEnt&, const T*, const double*, const T*, T*,       \
                                      const int*, hipStream_t);
HPG_INST(double)
HPG_INST(float)
#undef HPG_INST

}  // namespace dev
}  // namespace hpg
