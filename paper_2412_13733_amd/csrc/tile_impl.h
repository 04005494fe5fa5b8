#pragma once
// Fused, LDS-tiled apply of the hpG saddle operator G (and the FP64 residual)
// with the degree p fixed at compile time.
//
// A block owns a tile of TC^d cells and the u unknowns whose 1-D indices lie
// in [t TC p - 1, (t+1) TC p - 1) in every direction (the tile's lower vertex
// hats belong to it, its upper ones to the next tile).  It stages in LDS
//   * the x_u box [t TC p - 1 - p, (t+1) TC p - 1] per direction (the sparse
//     1-D rows of an owned unknown reach at most p to the left and 1 to the
//     right of the owned range),
//   * the psi coefficients of the cells [t TC - 1, (t+1) TC) (an owned vertex
//     hat couples to the cells on both sides),
//   * the owned rows of the global 1-D stiffness/mass/Gram matrices,
// then computes
//   * y_u for the owned unknowns: alpha sum_k (A1 in k)(x)(M1 elsewhere) x_u
//     + (x)_k B1 x_psi as tensor products of 1-D rows read from LDS
//     (owner-computes: deterministic, no atomics),
//   * y_psi for the tile's cells: B_K^T x_uK - V^T diag(omega) V x_psiK
//     - beta M x_psiK by compile-time-sized sum-factorised contractions
//     (paper Sec. 4.3: D_psi block-diagonal, applied through the
//     Gauss-Legendre points),
// so each input is read from HBM once (the halo is re-read from L2) and each
// output written once.  Residual mode evaluates eq. (pG) instead: the Gram
// term acts on psi - psi_prev, R_u subtracts alpha F, and R_psi uses
// (exp(-psi_h), zeta) - Phi with the exponent guard exp(min(-psi, 700)).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace hpg {
namespace dev {

__device__ inline double block_sum_tile(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    return s;   // valid in thread 0
}

template <int D, int N>
struct Pw {
    static constexpr int v = N * Pw<D - 1, N>::v;
};
template <int N>
struct Pw<0, N> {
    static constexpr int v = 1;
};

template <int D, int PP, int TC>
struct TileCfg {
    static constexpr int L = PP + 1, P = PP - 1, Q = PP + 1;
    static constexpr int OW = TC * PP;          // owned u per direction
    // low p: 1-D rows as dense windows of 2p+1 columns (col - g in [-p, p]) and
    // 2 cells x P modes of psi (cells g/p and g/p + 1); the box and the psi
    // cells then extend one window further so every tap stays in LDS
    static constexpr bool DENSE = PP == 2 || (PP == 3 && D <= 2);
    static constexpr int WN = 2 * PP + 1, WBN = 2 * (PP - 1), WS = 2 * WN + WBN;
    static constexpr int XW = DENSE ? OW + 2 * PP : OW + PP + 1;   // x_u box width
    static constexpr int CW = DENSE ? TC + 2 : TC + 1;   // psi cells per direction (left halo)
    static constexpr int OWS = DENSE ? 1 : OW;   // sparse row tables (unused when DENSE)
    static constexpr int NWIN = DENSE ? D * OW * WS : 1;
    static constexpr int XS = Pw<D, XW>::v;
    static constexpr int CS = Pw<D, CW>::v;
    static constexpr int OWD = Pw<D, OW>::v;
    static constexpr int TCD = Pw<D, TC>::v;
    static constexpr int PD = Pw<D, P>::v;
    static constexpr int QD = Pw<D, Q>::v;
    static constexpr int LD = Pw<D, L>::v;
    static constexpr int SB = QD > LD ? QD : LD;   // per-cell contraction buffer
    // low p with many cells per tile: psi-side one cell per thread in registers
    static constexpr bool REG_PSI = PP == 2 && D <= 2 && TCD >= 64;
    static constexpr int NS = REG_PSI ? 1 : TCD * SB;   // LDS contraction buffers
    static constexpr int NT = REG_PSI ? 1 : TCD * PD;
    // u-side intermediates of the direction-by-direction stencil: 2-D
    // (owned 1) x (box 0); 3-D (owned 2) x (box 1) x (box 0) and
    // (owned 2) x (owned 1) x (box 0)
    static constexpr int NV = D == 3 ? OW * XW * XW : 1;
    static constexpr int NU = D == 1 ? 1 : (D == 2 ? OW * XW : OW * OW * XW);
    // the u-side intermediates and the psi-side buffers share one LDS region
    static constexpr int NSCR_U = 2 * NV + 2 * NU, NSCR_P = 2 * NS + NT;
    static constexpr int NSCR = NSCR_U > NSCR_P ? NSCR_U : NSCR_P;
};

// compile-time-sized contraction along axis AX of a batch of d-D cell
// tensors in LDS (axes < AX already of size NOUT, axes >= AX of size NIN):
// out[.., i, ..] = sum_j mat(i, j) in[.., j, ..], mat(i, j) = mat[i LD + j]
// or mat[j LD + i] (TRANS)
template <typename T, int D, int NIN, int NOUT, int AX, bool TRANS, int LDM>
__device__ inline void ctc(const T* __restrict__ in, T* __restrict__ out, int stride, int ncell,
                           const T* __restrict__ mat) {
    constexpr int di0 = (0 < AX) ? NOUT : NIN;
    constexpr int di1 = D > 1 ? ((1 < AX) ? NOUT : NIN) : 1;
    constexpr int do0 = (0 <= AX) ? NOUT : NIN;
    constexpr int do1 = D > 1 ? ((1 <= AX) ? NOUT : NIN) : 1;
    constexpr int do2 = D > 2 ? ((2 <= AX) ? NOUT : NIN) : 1;
    constexpr int TOT = do0 * do1 * do2;
    constexpr int SAX = AX == 0 ? 1 : (AX == 1 ? di0 : di0 * di1);
    for (int e = threadIdx.x; e < ncell * TOT; e += blockDim.x) {
        const int c = e / TOT, o = e - c * TOT;
        const int i0 = o % do0, r = o / do0, i1 = r % do1, i2 = r / do1;
        const int iout = AX == 0 ? i0 : (AX == 1 ? i1 : i2);
        const int base = (AX == 0 ? 0 : i0) + di0 * ((AX == 1 ? 0 : i1) + di1 * (AX == 2 ? 0 : i2));
        const T* src = in + c * stride + base;
        T acc = 0;
#pragma unroll
        for (int j = 0; j < NIN; ++j) acc += (TRANS ? mat[j * LDM + iout] : mat[iout * LDM + j]) * src[j * SAX];
        out[c * stride + o] = acc;
    }
}

// the same matrix along every axis; ping-pong a <-> b; returns the result buffer
template <typename T, int D, int NIN, int NOUT, bool TRANS, int LDM>
__device__ inline T* ctc_all(T* a, T* b, int stride, int ncell, const T* mat) {
    ctc<T, D, NIN, NOUT, 0, TRANS, LDM>(a, b, stride, ncell, mat);
    __syncthreads();
    if (D == 1) return b;
    ctc<T, D, NIN, NOUT, 1, TRANS, LDM>(b, a, stride, ncell, mat);
    __syncthreads();
    if (D == 2) return a;
    ctc<T, D, NIN, NOUT, 2, TRANS, LDM>(a, b, stride, ncell, mat);
    __syncthreads();
    return b;
}

template <typename T, int D, int PP, int TC, int MODE>
__global__ __launch_bounds__(256) void k_apply_tile(Geo g, URows<T> r0, URows<T> r1, URows<T> r2,
                                                    PsiTabs<T> tb, T alpha, T beta,
                                                    const double* __restrict__ prm,
                                                    const T* __restrict__ xu,
                                                    const T* __restrict__ xpsi,
                                                    const T* __restrict__ xpsi_prev,
                                                    const T* __restrict__ omega,
                                                    const double* __restrict__ F,
                                                    const double* __restrict__ Phi,
                                                    T* __restrict__ yu, T* __restrict__ ypsi,
                                                    double* __restrict__ partial,
                                                    const int* __restrict__ done, TileBatch bt) {
    using C = TileCfg<D, PP, TC>;
    constexpr int L = C::L, P = C::P, Q = C::Q, OW = C::OW, XW = C::XW, CW = C::CW;
    constexpr int W = URows<T>::WM, WB = URows<T>::WB;
    __shared__ T X[C::XS];
    __shared__ T PS[C::CS * C::PD];
    __shared__ T SCR[C::NSCR];
    T* const VA = SCR;
    T* const VM = SCR + C::NV;
    T* const UA = SCR + 2 * C::NV;
    T* const UM = UA + C::NU;
    T* const S1 = SCR;
    T* const S2 = SCR + C::NS;
    T* const TB = SCR + 2 * C::NS;
    __shared__ T tB1[L * P], tV[Q * P], tw[Q], tMd[P];
    // row tables entry-major ([dir][entry][row]) so lanes of consecutive rows
    // read consecutive LDS words
    __shared__ int16_t rc[D][W][C::OWS];
    __shared__ T ra[D][W][C::OWS], rm[D][W][C::OWS];
    __shared__ int8_t rl[D][C::OWS], bl[D][C::OWS];
    __shared__ int16_t bcell[D][WB][C::OWS], bmode[D][WB][C::OWS];
    __shared__ T bv[D][WB][C::OWS];
    __shared__ T WIN[C::NWIN];   // dense windows: [dir][owned row][A | M | B]
    __shared__ double red[4];
    {
        // request of a batched launch (blockIdx.y = 0 otherwise)
        const int64_t rb = blockIdx.y;
        xu += rb * bt.xu;
        xpsi += rb * bt.xp;
        if (xpsi_prev) xpsi_prev += rb * bt.pprev;
        if (omega) omega += rb * bt.om;
        if (F) F += rb * bt.F;
        if (Phi) Phi += rb * bt.Phi;
        yu += rb * bt.yu;
        ypsi += rb * bt.yp;
        if (partial) partial += rb * bt.part;
        if (done) done += rb * bt.done;
        if (prm) prm += rb * bt.prm;
    }
    if (done && *done) return;
    if (prm) {
        alpha = (T)prm[0];
        beta = (T)prm[1];
    }
    // reference tables
    for (int i = threadIdx.x; i < L * P; i += blockDim.x) tB1[i] = tb.B1[i];
    for (int i = threadIdx.x; i < Q * P; i += blockDim.x) tV[i] = tb.Vpsi[i];
    for (int i = threadIdx.x; i < Q; i += blockDim.x) tw[i] = tb.w[i];
    for (int i = threadIdx.x; i < P; i += blockDim.x) tMd[i] = tb.Mdiag[i];
    int ntile[3] = {1, 1, 1};
    int ntot = 1;
    for (int k = 0; k < D; ++k) {
        ntile[k] = (g.m[k] + TC - 1) / TC;
        ntot *= ntile[k];
    }
    // each block takes a contiguous run of tiles; workgroups go round-robin to
    // the 8 XCDs, so consecutive runs are given to blocks of the same XCD and
    // neighbouring tiles share halo lines in one L2
    const int nb = (int)gridDim.x;
    const int xcd = (int)blockIdx.x & 7, slot = (int)blockIdx.x >> 3;
    const int base_q = nb >> 3, base_r = nb & 7;
    const int lb = xcd * base_q + (xcd < base_r ? xcd : base_r) + slot;
    const int per = (ntot + nb - 1) / nb;
    const int t_begin = lb * per, t_end = min(ntot, t_begin + per);
    const int tid = (int)threadIdx.x;
    // origins of a tile: first owned 1-D index o0, box origin x0, first psi cell c0
    const int gn1[3] = {g.n1[0], g.n1[1], g.n1[2]};
    const int gm[3] = {g.m[0], g.m[1], g.m[2]};
    const T* const xu_l = xu;
    const T* const xpsi_l = xpsi;
    const T* const xprev_l = xpsi_prev;
    auto origins = [&](int tile, int* x0, int* o0, int* c0) {
        int t = tile;
        for (int k = 0; k < 3; ++k) {
            const int tk = k < D ? t % ntile[k] : 0;
            if (k < D) t /= ntile[k];
            o0[k] = k < D ? tk * OW - 1 : 0;
            x0[k] = k < D ? o0[k] - PP : 0;
            c0[k] = k < D ? tk * TC - 1 : 0;
        }
    };
    // the next tile's x_u box, psi and row windows are loaded into registers
    // while the current tile computes
    constexpr int NTH = 256;
    constexpr int NXR = (C::XS + NTH - 1) / NTH;
    constexpr int NPR = (C::CS * C::PD + NTH - 1) / NTH;
    constexpr int NWK = C::DENSE ? (OW * C::WS + NTH - 1) / NTH : 0;   // per direction
    constexpr int NWR = D * NWK;
    T xr[NXR], pr[NPR], wr[NWR > 0 ? NWR : 1];
    const T* const win0 = r0.win;
    const T* const win1 = r1.win;
    const T* const win2 = r2.win;
    auto fetch = [&](int tile) {
        int fx0[3], fo0[3], fc0[3];
        origins(tile, fx0, fo0, fc0);
#pragma unroll
        for (int r = 0; r < NXR; ++r) {
            const int e = tid + r * NTH;
            const int b0 = e % XW, b1 = (e / XW) % XW, b2 = e / (XW * XW);
            const int g0 = fx0[0] + b0, g1 = fx0[1] + b1, g2 = fx0[2] + b2;
            bool ok = e < C::XS && g0 >= 0 && g0 < gn1[0];
            if (D > 1) ok = ok && g1 >= 0 && g1 < gn1[1];
            if (D > 2) ok = ok && g2 >= 0 && g2 < gn1[2];
            int64_t flat = g0;
            if (D > 1) flat += (int64_t)g1 * gn1[0];
            if (D > 2) flat += (int64_t)g2 * gn1[0] * gn1[1];
            xr[r] = ok ? xu_l[flat] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < NPR; ++r) {
            const int e = tid + r * NTH;
            const int cl = e / C::PD, a = e - cl * C::PD;
            const int k0 = fc0[0] + cl % CW, k1 = fc0[1] + (cl / CW) % CW, k2 = fc0[2] + cl / (CW * CW);
            bool ok = e < C::CS * C::PD && k0 >= 0 && k0 < gm[0];
            if (D > 1) ok = ok && k1 >= 0 && k1 < gm[1];
            if (D > 2) ok = ok && k2 >= 0 && k2 < gm[2];
            int64_t cell = k0;
            if (D > 1) cell += (int64_t)k1 * gm[0];
            if (D > 2) cell += (int64_t)k2 * gm[0] * gm[1];
            T v = 0;
            if (ok) {
                v = xpsi_l[cell * C::PD + a];
                if (MODE == MODE_RES) v -= xprev_l[cell * C::PD + a];
            }
            pr[r] = v;
        }
        if constexpr (C::DENSE) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T* wk = k == 0 ? win0 : (k == 1 ? win1 : win2);
                const int64_t base = (int64_t)(fo0[k] + 1) * C::WS;
#pragma unroll
                for (int r = 0; r < NWK; ++r) {
                    const int o = tid + r * NTH;
                    wr[k * NWK + r] = o < OW * C::WS ? wk[base + o] : (T)0;
                }
            }
        }
    };
    // the low-degree path prefetches; at higher degree the registers are worth
    // more to occupancy and the staging is synchronous
    constexpr bool PREFETCH = C::DENSE;
    double part_u = 0.0, part_p = 0.0;
    if (PREFETCH && t_begin < t_end) fetch(t_begin);
    for (int tile = t_begin; tile < t_end; ++tile) {
        int x0[3], o0[3], c0[3];
        origins(tile, x0, o0, c0);
        if (!PREFETCH) fetch(tile);
        __syncthreads();   // previous tile done with LDS
#pragma unroll
        for (int r = 0; r < NXR; ++r)
            if (tid + r * NTH < C::XS) X[tid + r * NTH] = xr[r];
#pragma unroll
        for (int r = 0; r < NPR; ++r)
            if (tid + r * NTH < C::CS * C::PD) PS[tid + r * NTH] = pr[r];
        if constexpr (C::DENSE) {
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int r = 0; r < NWK; ++r)
                    if (tid + r * NTH < OW * C::WS) WIN[k * OW * C::WS + tid + r * NTH] = wr[k * NWK + r];
        }
        if (PREFETCH && tile + 1 < t_end) fetch(tile + 1);
        if constexpr (!C::DENSE) {
            // ---- stage owned 1-D rows (columns relative to the box / cell origin);
            // the owned rows of a direction are contiguous in the global tables, so
            // one thread per row entry reads them coalesced
            for (int e = threadIdx.x; e < D * OW * W; e += blockDim.x) {
                const int k = e / (OW * W), rj = e - k * OW * W, r = rj / W, j = rj - r * W;
                const URows<T>& R = k == 0 ? r0 : (k == 1 ? r1 : r2);
                const int gk = o0[k] + r;
                const bool ok = gk >= 0 && gk < g.n1[k];
                const int n = ok ? R.lenM[gk] : 0;
                if (j == 0) rl[k][r] = (int8_t)n;
                const bool v = j < n;
                rc[k][j][r] = (int16_t)(v ? R.colM[gk * W + j] - x0[k] : 0);
                ra[k][j][r] = v ? R.aM[gk * W + j] : (T)0;
                rm[k][j][r] = v ? R.mM[gk * W + j] : (T)0;
            }
            for (int e = threadIdx.x; e < D * OW * WB; e += blockDim.x) {
                const int k = e / (OW * WB), rj = e - k * OW * WB, r = rj / WB, j = rj - r * WB;
                const URows<T>& R = k == 0 ? r0 : (k == 1 ? r1 : r2);
                const int gk = o0[k] + r;
                const bool ok = gk >= 0 && gk < g.n1[k];
                const int nb = ok ? R.lenB[gk] : 0;
                if (j == 0) bl[k][r] = (int8_t)nb;
                const bool v = j < nb;
                bcell[k][j][r] = (int16_t)(v ? R.cellB[gk * WB + j] - c0[k] : 0);
                bmode[k][j][r] = (int16_t)(v ? R.modeB[gk * WB + j] : 0);
                bv[k][j][r] = v ? R.vB[gk * WB + j] : (T)0;
            }
        }
        __syncthreads();
        if constexpr (C::DENSE) {
            // ---- u-side stiffness / mass, one direction at a time, window taps
            constexpr int WN = C::WN, WS = C::WS;
            if constexpr (D == 2 && PP == 2) {
                // a thread takes R consecutive rows q1 of one box column b0 and
                // reads the R + WN - 1 box values they share once (p = 2; at p = 3
                // the registers would cost occupancy)
                constexpr int R = 4;
                static_assert(OW % R == 0, "owned rows in groups of R");
                for (int it = threadIdx.x; it < XW * (OW / R); it += blockDim.x) {
                    const int q1b = (it / XW) * R, b0 = it - (it / XW) * XW;
                    T xv[R + WN - 1];
#pragma unroll
                    for (int r = 0; r < R + WN - 1; ++r) xv[r] = X[(q1b + r) * XW + b0];
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        const T* w = WIN + (OW + q1b + i) * WS;
                        T sa = 0, sm = 0;
#pragma unroll
                        for (int j = 0; j < WN; ++j) {
                            sa += w[j] * xv[i + j];
                            sm += w[WN + j] * xv[i + j];
                        }
                        UA[(q1b + i) * XW + b0] = sa;
                        UM[(q1b + i) * XW + b0] = sm;
                    }
                }
                __syncthreads();
            } else if constexpr (D == 2) {
                for (int e = threadIdx.x; e < OW * XW; e += blockDim.x) {
                    const int q1 = e / XW, b0 = e - q1 * XW;
                    const T* w = WIN + (OW + q1) * WS;
                    T sa = 0, sm = 0;
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        const T xv = X[(q1 + j) * XW + b0];
                        sa += w[j] * xv;
                        sm += w[WN + j] * xv;
                    }
                    UA[e] = sa;
                    UM[e] = sm;
                }
                __syncthreads();
            } else if constexpr (D == 3) {
                for (int e = threadIdx.x; e < OW * XW * XW; e += blockDim.x) {
                    const int q2 = e / (XW * XW), b01 = e - q2 * (XW * XW);
                    const T* w = WIN + (2 * OW + q2) * WS;
                    T sa = 0, sm = 0;
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        const T xv = X[(q2 + j) * (XW * XW) + b01];
                        sa += w[j] * xv;
                        sm += w[WN + j] * xv;
                    }
                    VA[e] = sa;
                    VM[e] = sm;
                }
                __syncthreads();
                for (int e = threadIdx.x; e < OW * OW * XW; e += blockDim.x) {
                    const int b0 = e % XW, r = e / XW, q1 = r % OW, q2 = r / OW;
                    const T* w = WIN + (OW + q1) * WS;
                    T sa = 0, sm = 0;
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        const int o = (q2 * XW + q1 + j) * XW + b0;
                        const T vm = VM[o];
                        sm += w[WN + j] * vm;
                        sa += w[j] * vm + w[WN + j] * VA[o];
                    }
                    UA[e] = sa;
                    UM[e] = sm;
                }
                __syncthreads();
            }
        } else {
            // (A_0 M_1 M_2 + M_0 A_1 M_2 + M_0 M_1 A_2) x, direction 0 fastest
            if constexpr (D == 2) {
                for (int e = threadIdx.x; e < OW * XW; e += blockDim.x) {
                    const int b0 = e % XW, q1 = e / XW;
                    const int n1 = rl[1][q1];
                    T sa = 0, sm = 0;
                    for (int j = 0; j < n1; ++j) {
                        const T xv = X[rc[1][j][q1] * XW + b0];
                        sa += ra[1][j][q1] * xv;
                        sm += rm[1][j][q1] * xv;
                    }
                    UA[e] = sa;
                    UM[e] = sm;
                }
                __syncthreads();
            } else if constexpr (D == 3) {
                for (int e = threadIdx.x; e < OW * XW * XW; e += blockDim.x) {
                    const int b01 = e % (XW * XW), q2 = e / (XW * XW);
                    const int n2 = rl[2][q2];
                    T sa = 0, sm = 0;
                    for (int j = 0; j < n2; ++j) {
                        const T xv = X[rc[2][j][q2] * XW * XW + b01];
                        sa += ra[2][j][q2] * xv;
                        sm += rm[2][j][q2] * xv;
                    }
                    VA[e] = sa;
                    VM[e] = sm;
                }
                __syncthreads();
                for (int e = threadIdx.x; e < OW * OW * XW; e += blockDim.x) {
                    const int b0 = e % XW, q1 = (e / XW) % OW, q2 = e / (XW * OW);
                    const int n1 = rl[1][q1];
                    T sa = 0, sm = 0;
                    for (int j = 0; j < n1; ++j) {
                        const int o = (q2 * XW + rc[1][j][q1]) * XW + b0;
                        const T vm = VM[o];
                        sm += rm[1][j][q1] * vm;
                        sa += ra[1][j][q1] * vm + rm[1][j][q1] * VA[o];
                    }
                    UA[e] = sa;
                    UM[e] = sm;
                }
                __syncthreads();
            }
        }
        // ---- u-side: owned unknowns
        if constexpr (C::DENSE && D == 2 && PP == 2) {
            // a thread takes R consecutive rows q1 of one owned column q0 and
            // keeps the column's window taps (stiffness, mass, psi coupling) in
            // registers; the arithmetic per unknown is that of the loop below
            constexpr int WN = C::WN, WS = C::WS, R = 4;
            for (int it = threadIdx.x; it < OW * (OW / R); it += blockDim.x) {
                const int q1b = (it / OW) * R, q0 = it - (it / OW) * OW;
                const int g0 = o0[0] + q0;
                if (g0 < 0 || g0 >= g.n1[0]) continue;
                T wa[WN], wm[WN], b0w[2 * P];
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    wa[j] = WIN[q0 * WS + j];
                    wm[j] = WIN[q0 * WS + WN + j];
                }
#pragma unroll
                for (int i0 = 0; i0 < 2 * P; ++i0) b0w[i0] = WIN[q0 * WS + 2 * WN + i0];
                const int s0 = (q0 + PP - 1) / PP;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const int q1 = q1b + i, g1 = o0[1] + q1;
                    if (g1 < 0 || g1 >= g.n1[1]) continue;
                    const int ub = q1 * XW + q0;
                    T acc = 0;
#pragma unroll
                    for (int j = 0; j < WN; ++j) acc += wa[j] * UM[ub + j] + wm[j] * UA[ub + j];
                    acc *= alpha;
                    const T* b1w = WIN + (OW + q1) * WS + 2 * WN;
                    const int s1 = (q1 + PP - 1) / PP;
#pragma unroll
                    for (int i1 = 0; i1 < 2 * P; ++i1) {
                        const int sc1 = i1 / P, a1 = i1 - sc1 * P;
                        const T v1 = b1w[i1];
                        const T* ps = PS + ((s1 + sc1) * CW + s0) * C::PD + a1 * P;
#pragma unroll
                        for (int i0 = 0; i0 < 2 * P; ++i0) {
                            const int sc0 = i0 / P, a0 = i0 - sc0 * P;
                            acc += b0w[i0] * v1 * ps[sc0 * C::PD + a0];
                        }
                    }
                    const int64_t flat = g0 + (int64_t)g1 * g.n1[0];
                    if (MODE == MODE_RES) {
                        const double r = (double)acc - (double)alpha * F[flat];
                        yu[flat] = (T)r;
                        part_u += r * r;
                    } else {
                        yu[flat] = acc;
                        part_u += (double)acc * (double)X[(q0 + PP) + XW * (q1 + PP)];
                    }
                }
            }
        }
        for (int e = threadIdx.x; e < (C::DENSE && D == 2 && PP == 2 ? 0 : C::OWD);
             e += blockDim.x) {
            const int q0 = e % OW, q1 = (e / OW) % OW, q2 = e / (OW * OW);
            int gi[3] = {o0[0] + q0, D > 1 ? o0[1] + q1 : 0, D > 2 ? o0[2] + q2 : 0};
            bool ok = gi[0] >= 0 && gi[0] < g.n1[0];
            if (D > 1) ok = ok && gi[1] >= 0 && gi[1] < g.n1[1];
            if (D > 2) ok = ok && gi[2] >= 0 && gi[2] < g.n1[2];
            if (!ok) continue;
            T acc = 0;
            if constexpr (C::DENSE) {
                constexpr int WN = C::WN, WS = C::WS;
                const T* w0 = WIN + q0 * WS;
                if (D == 1) {
#pragma unroll
                    for (int j = 0; j < WN; ++j) acc += w0[j] * X[q0 + j];
                } else {
                    const int ub = (D == 2 ? q1 : q2 * OW + q1) * XW + q0;
#pragma unroll
                    for (int j = 0; j < WN; ++j) acc += w0[j] * UM[ub + j] + w0[WN + j] * UA[ub + j];
                }
                acc *= alpha;
                // psi coupling: cells (q + p - 1) / p and the next one (tile-relative)
                const T* b0w = w0 + 2 * WN;
                const int s0 = (q0 + PP - 1) / PP;
                if (D == 1) {
#pragma unroll
                    for (int sc = 0; sc < 2; ++sc)
#pragma unroll
                        for (int a = 0; a < P; ++a) acc += b0w[sc * P + a] * PS[(s0 + sc) * C::PD + a];
                } else if (D == 2) {
                    const T* b1w = WIN + (OW + q1) * WS + 2 * WN;
                    const int s1 = (q1 + PP - 1) / PP;
#pragma unroll
                    for (int i1 = 0; i1 < 2 * P; ++i1) {
                        const int sc1 = i1 / P, a1 = i1 - sc1 * P;
                        const T v1 = b1w[i1];
                        const T* ps = PS + ((s1 + sc1) * CW + s0) * C::PD + a1 * P;
#pragma unroll
                        for (int i0 = 0; i0 < 2 * P; ++i0) {
                            const int sc0 = i0 / P, a0 = i0 - sc0 * P;
                            acc += b0w[i0] * v1 * ps[sc0 * C::PD + a0];
                        }
                    }
                } else {
                    const T* b1w = WIN + (OW + q1) * WS + 2 * WN;
                    const T* b2w = WIN + (2 * OW + q2) * WS + 2 * WN;
                    const int s1 = (q1 + PP - 1) / PP, s2 = (q2 + PP - 1) / PP;
#pragma unroll
                    for (int i2 = 0; i2 < 2 * P; ++i2) {
                        const int sc2 = i2 / P, a2 = i2 - sc2 * P;
#pragma unroll
                        for (int i1 = 0; i1 < 2 * P; ++i1) {
                            const int sc1 = i1 / P, a1 = i1 - sc1 * P;
                            const T v12 = b1w[i1] * b2w[i2];
                            const T* ps = PS + (((s2 + sc2) * CW + s1 + sc1) * CW + s0) * C::PD +
                                          (a2 * P + a1) * P;
#pragma unroll
                            for (int i0 = 0; i0 < 2 * P; ++i0) {
                                const int sc0 = i0 / P, a0 = i0 - sc0 * P;
                                acc += b0w[i0] * v12 * ps[sc0 * C::PD + a0];
                            }
                        }
                    }
                }
            } else {
                const int n0 = rl[0][q0];
                if (D == 1) {
                    for (int j0 = 0; j0 < n0; ++j0) acc += ra[0][j0][q0] * X[rc[0][j0][q0]];
                } else {
                    const int ub = (D == 2 ? q1 : q2 * OW + q1) * XW;
                    for (int j0 = 0; j0 < n0; ++j0) {
                        const int o = ub + rc[0][j0][q0];
                        acc += ra[0][j0][q0] * UM[o] + rm[0][j0][q0] * UA[o];
                    }
                }
                acc *= alpha;
                const int nb0 = bl[0][q0];
                if (D == 1) {
                    for (int j0 = 0; j0 < nb0; ++j0)
                        acc += bv[0][j0][q0] * PS[bcell[0][j0][q0] * C::PD + bmode[0][j0][q0]];
                } else if (D == 2) {
                    const int nb1 = bl[1][q1];
                    for (int j1 = 0; j1 < nb1; ++j1) {
                        const int cb = bcell[1][j1][q1] * CW;
                        const int mb = bmode[1][j1][q1] * P;
                        const T v1 = bv[1][j1][q1];
                        for (int j0 = 0; j0 < nb0; ++j0)
                            acc += bv[0][j0][q0] * v1 *
                                   PS[(cb + bcell[0][j0][q0]) * C::PD + mb + bmode[0][j0][q0]];
                    }
                } else {
                    const int nb1 = bl[1][q1], nb2 = bl[2][q2];
                    for (int j2 = 0; j2 < nb2; ++j2)
                        for (int j1 = 0; j1 < nb1; ++j1) {
                            const int cb = (bcell[2][j2][q2] * CW + bcell[1][j1][q1]) * CW;
                            const int mb = (bmode[2][j2][q2] * P + bmode[1][j1][q1]) * P;
                            const T v12 = bv[1][j1][q1] * bv[2][j2][q2];
                            for (int j0 = 0; j0 < nb0; ++j0)
                                acc += bv[0][j0][q0] * v12 *
                                       PS[(cb + bcell[0][j0][q0]) * C::PD + mb + bmode[0][j0][q0]];
                        }
                }
            }
            int64_t flat = gi[0];
            if (D > 1) flat += (int64_t)gi[1] * g.n1[0];
            if (D > 2) flat += (int64_t)gi[2] * g.n1[0] * g.n1[1];
            if (MODE == MODE_RES) {
                const double r = (double)acc - (double)alpha * F[flat];
                yu[flat] = (T)r;
                part_u += r * r;
            } else {
                yu[flat] = acc;
                part_u += (double)acc * (double)X[(q0 + PP) + XW * ((D > 1 ? q1 + PP : 0) +
                                                                     XW * (D > 2 ? q2 + PP : 0))];
            }
        }
        // ---- psi-side, one cell per thread in registers (low p, many cells)
        if constexpr (C::REG_PSI) {
            for (int ci = threadIdx.x; ci < C::TCD; ci += blockDim.x) {
                const int c_0 = ci % TC, c_1 = (ci / TC) % TC, c_2 = ci / (TC * TC);
                int gc[3] = {c0[0] + 1 + c_0, D > 1 ? c0[1] + 1 + c_1 : 0,
                             D > 2 ? c0[2] + 1 + c_2 : 0};
                bool ok = gc[0] < g.m[0];
                if (D > 1) ok = ok && gc[1] < g.m[1];
                if (D > 2) ok = ok && gc[2] < g.m[2];
                if (!ok) continue;
                int64_t cell = gc[0];
                if (D > 1) cell += (int64_t)gc[1] * g.m[0];
                if (D > 2) cell += (int64_t)gc[2] * g.m[0] * g.m[1];
                T J = (T)0.5 * tb.h[0][gc[0]];
                if (D > 1) J *= (T)0.5 * tb.h[1][gc[1]];
                if (D > 2) J *= (T)0.5 * tb.h[2][gc[2]];
                // local u box
                T xl[C::LD];
#pragma unroll
                for (int l = 0; l < C::LD; ++l) {
                    const int l0 = l % L, l1 = (l / L) % L, l2 = l / (L * L);
                    int b = (c_0 * PP + l0 + PP);
                    if (D > 1) b += XW * (c_1 * PP + l1 + PP);
                    if (D > 2) b += XW * XW * (c_2 * PP + l2 + PP);
                    xl[l] = X[b];
                }
                T pk[C::PD];
#pragma unroll
                for (int a = 0; a < C::PD; ++a)
                    pk[a] = MODE == MODE_APPLY
                                ? PS[((D > 1 ? (c_1 + 1) * CW : 0) + c_0 + 1) * C::PD + a]
                                : xpsi[cell * C::PD + a];
                // psi_h at the Gauss points, weight, back-projection
                T dx[C::PD];
#pragma unroll
                for (int a = 0; a < C::PD; ++a) dx[a] = 0;
#pragma unroll
                for (int j = 0; j < C::QD; ++j) {
                    const int j0 = j % Q, j1 = (j / Q) % Q, j2 = j / (Q * Q);
                    T vq = 0;
#pragma unroll
                    for (int a = 0; a < C::PD; ++a) {
                        const int a0 = a % P, a1 = (a / P) % P, a2 = a / (P * P);
                        T v = tV[j0 * P + a0];
                        if (D > 1) v *= tV[j1 * P + a1];
                        if (D > 2) v *= tV[j2 * P + a2];
                        vq += v * pk[a];
                    }
                    T wv;
                    if (MODE == MODE_RES) {
                        T wq = J * tw[j0];
                        if (D > 1) wq *= tw[j1];
                        if (D > 2) wq *= tw[j2];
                        const double arg = -(double)vq;
                        wv = (T)((double)wq * exp(arg < 700.0 ? arg : 700.0));
                    } else {
                        wv = omega[cell * C::QD + j] * vq;
                    }
#pragma unroll
                    for (int a = 0; a < C::PD; ++a) {
                        const int a0 = a % P, a1 = (a / P) % P, a2 = a / (P * P);
                        T v = tV[j0 * P + a0];
                        if (D > 1) v *= tV[j1 * P + a1];
                        if (D > 2) v *= tV[j2 * P + a2];
                        dx[a] += v * wv;
                    }
                }
#pragma unroll
                for (int a = 0; a < C::PD; ++a) {
                    const int a0 = a % P, a1 = (a / P) % P, a2 = a / (P * P);
                    T bt = 0;
#pragma unroll
                    for (int l = 0; l < C::LD; ++l) {
                        const int l0 = l % L, l1 = (l / L) % L, l2 = l / (L * L);
                        T v = tB1[l0 * P + a0];
                        if (D > 1) v *= tB1[l1 * P + a1];
                        if (D > 2) v *= tB1[l2 * P + a2];
                        bt += v * xl[l];
                    }
                    bt *= J;
                    const int64_t o = cell * C::PD + a;
                    if (MODE == MODE_RES) {
                        const double r = (double)bt + (double)dx[a] - Phi[o];
                        ypsi[o] = (T)r;
                        part_p += r * r;
                    } else {
                        T md = J * tMd[a0];
                        if (D > 1) md *= tMd[a1];
                        if (D > 2) md *= tMd[a2];
                        const T y = bt - dx[a] - beta * md * pk[a];
                        ypsi[o] = y;
                        part_p += (double)y * (double)pk[a];
                    }
                }
            }
        } else {
            // ---- psi-side: the tile's cells (the first TC^d of the halo-extended set);
            // its buffers overlay the u-side intermediates
            __syncthreads();
            // gather the local u boxes: cell ci's box starts at ci p + p in the X box
            for (int e = threadIdx.x; e < C::TCD * C::LD; e += blockDim.x) {
                const int ci = e / C::LD, l = e - ci * C::LD;
                const int c_0 = ci % TC, c_1 = (ci / TC) % TC, c_2 = ci / (TC * TC);
                const int l0 = l % L, l1 = (l / L) % L, l2 = l / (L * L);
                int b = (c_0 * PP + l0 + PP);
                if (D > 1) b += XW * (c_1 * PP + l1 + PP);
                if (D > 2) b += XW * XW * (c_2 * PP + l2 + PP);
                S1[ci * C::SB + l] = X[b];
            }
            __syncthreads();
            {
                T* t = ctc_all<T, D, L, P, true, P>(S1, S2, C::SB, C::TCD, tB1);
                for (int e = threadIdx.x; e < C::TCD * C::PD; e += blockDim.x) {
                    const int ci = e / C::PD, a = e - ci * C::PD;
                    TB[e] = t[ci * C::SB + a];
                }
            }
            __syncthreads();
            // psi_K (the apply's x_psi, or psi itself in residual mode) -> quadrature points
            for (int e = threadIdx.x; e < C::TCD * C::PD; e += blockDim.x) {
                const int ci = e / C::PD, a = e - ci * C::PD;
                const int c_0 = ci % TC, c_1 = (ci / TC) % TC, c_2 = ci / (TC * TC);
                int gc[3] = {c0[0] + 1 + c_0, D > 1 ? c0[1] + 1 + c_1 : 0, D > 2 ? c0[2] + 1 + c_2 : 0};
                bool ok = gc[0] < g.m[0];
                if (D > 1) ok = ok && gc[1] < g.m[1];
                if (D > 2) ok = ok && gc[2] < g.m[2];
                T v = 0;
                if (ok) {
                    int64_t cell = gc[0];
                    if (D > 1) cell += (int64_t)gc[1] * g.m[0];
                    if (D > 2) cell += (int64_t)gc[2] * g.m[0] * g.m[1];
                    v = xpsi[cell * C::PD + a];
                }
                S1[ci * C::SB + a] = v;
            }
            __syncthreads();
            T* vq = ctc_all<T, D, P, Q, false, P>(S1, S2, C::SB, C::TCD, tV);
            T* oth = (vq == S1) ? S2 : S1;
            for (int e = threadIdx.x; e < C::TCD * C::QD; e += blockDim.x) {
                const int ci = e / C::QD, j = e - ci * C::QD;
                const int c_0 = ci % TC, c_1 = (ci / TC) % TC, c_2 = ci / (TC * TC);
                int gc[3] = {c0[0] + 1 + c_0, D > 1 ? c0[1] + 1 + c_1 : 0, D > 2 ? c0[2] + 1 + c_2 : 0};
                bool ok = gc[0] < g.m[0];
                if (D > 1) ok = ok && gc[1] < g.m[1];
                if (D > 2) ok = ok && gc[2] < g.m[2];
                T w = 0;
                if (ok) {
                    int64_t cell = gc[0];
                    if (D > 1) cell += (int64_t)gc[1] * g.m[0];
                    if (D > 2) cell += (int64_t)gc[2] * g.m[0] * g.m[1];
                    if (MODE == MODE_RES) {
                        T J = (T)0.5 * tb.h[0][gc[0]];
                        if (D > 1) J *= (T)0.5 * tb.h[1][gc[1]];
                        if (D > 2) J *= (T)0.5 * tb.h[2][gc[2]];
                        const int j0 = j % Q, j1 = (j / Q) % Q, j2 = j / (Q * Q);
                        T wq = J * tw[j0];
                        if (D > 1) wq *= tw[j1];
                        if (D > 2) wq *= tw[j2];
                        const double arg = -(double)vq[ci * C::SB + j];
                        w = (T)((double)wq * exp(arg < 700.0 ? arg : 700.0));
                    } else {
                        w = omega[cell * C::QD + j] * vq[ci * C::SB + j];
                    }
                }
                vq[ci * C::SB + j] = w;
            }
            __syncthreads();
            T* dx = ctc_all<T, D, Q, P, true, P>(vq, oth, C::SB, C::TCD, tV);
            for (int e = threadIdx.x; e < C::TCD * C::PD; e += blockDim.x) {
                const int ci = e / C::PD, a = e - ci * C::PD;
                const int c_0 = ci % TC, c_1 = (ci / TC) % TC, c_2 = ci / (TC * TC);
                int gc[3] = {c0[0] + 1 + c_0, D > 1 ? c0[1] + 1 + c_1 : 0, D > 2 ? c0[2] + 1 + c_2 : 0};
                bool ok = gc[0] < g.m[0];
                if (D > 1) ok = ok && gc[1] < g.m[1];
                if (D > 2) ok = ok && gc[2] < g.m[2];
                if (!ok) continue;
                int64_t cell = gc[0];
                if (D > 1) cell += (int64_t)gc[1] * g.m[0];
                if (D > 2) cell += (int64_t)gc[2] * g.m[0] * g.m[1];
                T J = (T)0.5 * tb.h[0][gc[0]];
                if (D > 1) J *= (T)0.5 * tb.h[1][gc[1]];
                if (D > 2) J *= (T)0.5 * tb.h[2][gc[2]];
                const T bt = TB[e] * J;
                const int64_t o = cell * C::PD + a;
                if (MODE == MODE_RES) {
                    const double r = (double)bt + (double)dx[ci * C::SB + a] - Phi[o];
                    ypsi[o] = (T)r;
                    part_p += r * r;
                } else {
                    const int a0 = a % P, a1 = (a / P) % P, a2 = a / (P * P);
                    T md = J * tMd[a0];
                    if (D > 1) md *= tMd[a1];
                    if (D > 2) md *= tMd[a2];
                    const T xp = xpsi[o];
                    const T y = bt - dx[ci * C::SB + a] - beta * md * xp;
                    ypsi[o] = y;
                    part_p += (double)y * (double)xp;
                }
            }
    
        }
    }
    if (partial) {
        if (MODE == MODE_RES) {
            const double su = block_sum_tile(part_u, red);
            __syncthreads();
            const double sp = block_sum_tile(part_p, red);
            if (threadIdx.x == 0) {
                partial[2 * blockIdx.x] = su;
                partial[2 * blockIdx.x + 1] = sp;
            }
        } else {
            const double s = block_sum_tile(part_u + part_p, red);
            if (threadIdx.x == 0) partial[blockIdx.x] = s;
        }
    }
}

// tile edge in cells for (d, p): 2-D tiles own about 12-24 u unknowns per
// direction, 3-D tiles one cell
constexpr int tile_cells(int D, int PP) {
    return D == 1 ? 16
                  : (D == 3 ? (PP == 2 ? 4 : 1)
                            : (PP == 2 ? 16 : PP == 3 ? 8 : PP == 4 ? 4 : PP == 5 ? 3 : PP == 6 ? 2 : 1));
}
constexpr int TILE_GRID_CAP = 2048;

template <typename T, int D, int PP, int MODE>
void launch_tile_impl(const Geo& g, const URows<T>* r, const PsiTabs<T>& tb, T alpha,
                             T beta, const double* prm, const T* xu, const T* xpsi,
                             const T* xpsi_prev, const T* omega, const double* F,
                             const double* Phi, T* yu, T* ypsi, double* partial, const int* done,
                             hipStream_t s, const KernelEvents* ev, const TileBatch& bt) {
    constexpr int TC = tile_cells(D, PP);
    // the prefetching path runs persistent blocks over contiguous runs of tiles;
    // otherwise one block per tile, unless per-block partial sums are written
    // (their count must fit the reduction buffer)
    const unsigned grid = (TileCfg<D, PP, TC>::DENSE || partial) ? (unsigned)tile_grid(g)
                                                                 : (unsigned)tile_count(g);
    const dim3 gd(grid, (unsigned)bt.nb);
    if (ev && ev->start)
        hipExtLaunchKernelGGL((k_apply_tile<T, D, PP, TC, MODE>), gd, dim3(256), 0, s,
                              ev->start, ev->stop, 0, g, r[0], r[1], r[2], tb, alpha, beta, prm, xu,
                              xpsi, xpsi_prev, omega, F, Phi, yu, ypsi, partial, done, bt);
    else
        hipLaunchKernelGGL((k_apply_tile<T, D, PP, TC, MODE>), gd, dim3(256), 0, s, g,
                           r[0], r[1], r[2], tb, alpha, beta, prm, xu, xpsi, xpsi_prev, omega, F,
                           Phi, yu, ypsi, partial, done, bt);
}

template <typename T, int D, int MODE>
bool launch_tile_d(const Geo& g, const URows<T>* r, const PsiTabs<T>& tb, T alpha, T beta,
                   const double* prm, const T* xu, const T* xpsi, const T* xpsi_prev,
                   const T* omega, const double* F, const double* Phi, T* yu, T* ypsi,
                   double* partial, const int* done, hipStream_t s, const KernelEvents* ev,
                   const TileBatch& bt) {
#define HPG_TC(PV)                                                                            \
    case PV:                                                                                  \
        launch_tile_impl<T, D, PV, MODE>(g, r, tb, alpha, beta, prm, xu, xpsi, xpsi_prev,    \
                                         omega, F, Phi, yu, ypsi, partial, done, s, ev, bt);  \
        return true;
    if constexpr (D == 3) {
        switch (g.p) {
            HPG_TC(2) HPG_TC(3) HPG_TC(4) HPG_TC(5) HPG_TC(6) HPG_TC(7)
            default: return false;
        }
    } else {
        switch (g.p) {
            HPG_TC(2) HPG_TC(3) HPG_TC(4) HPG_TC(5) HPG_TC(6) HPG_TC(7) HPG_TC(8) HPG_TC(9)
            HPG_TC(10) HPG_TC(11) HPG_TC(12)
            default: return false;
        }
    }
#undef HPG_TC
}

#define HPG_TILE_INST(T, DD, MM)                                                                 \
    template bool launch_tile_d<T, DD, MM>(const Geo&, const URows<T>*, const PsiTabs<T>&, T, T, \
                                           const double*, const T*, const T*, const T*,          \
                                           const T*, const double*, const double*, T*, T*,       \
                                           double*, const int*, hipStream_t, const KernelEvents*, \
                                           const TileBatch&);

}  // namespace dev
}  // namespace hpg
