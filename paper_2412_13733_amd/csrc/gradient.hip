// Gradient constraint |grad u| <= phi (Sec. 4.2, eq. (pG:gradient)).
//
// psi has d components per cell (component-major blocks of P^d Legendre
// coefficients, P = p).  The coupling is B_ij = (d/dx_c v_i, zeta_j^(c)):
// along direction c its 1-D factor is (phi_l', P_a), along the others the
// Gram (phi_l, P_a).  The nonlinear term is N(psi) = (phi psi_h / sqrt(1 +
// |psi_h|^2), zeta); its Frechet derivative D_psi has, at each Gauss point,
// the symmetric d x d weight w_q |J| phi_q F(psi_h) with
// F = ((1 + |psi|^2) I - psi psi^T) (1 + |psi|^2)^{-3/2}.  E_beta is the
// broken gradient stiffness of the Y_n basis per component, and the psi-block
// of the preconditioner is -S_hat = D_psi + beta E_beta
// (eq. (schur-preconditioner:gradient)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dev_util.h"
#include "kernels.h"

namespace hpg {
namespace dev {

// index of the component pair (c, l), c <= l, in the row-major upper triangle
__host__ __device__ inline int pair_index(int c, int l, int D) {
    if (c > l) {
        const int t = c;
        c = l;
        l = t;
    }
    return c * D - c * (c - 1) / 2 + (l - c);
}

// sum over the tensor product of one 1-D coupling row per direction of
// x_b (component comp); MODE_RES uses x_b - x_b_prev
template <typename T, int D, int MODE, int WB>
__device__ inline T couple(const Geo& g, const BRow<T, WB>& R0, const BRow<T, WB>& R1,
                           const BRow<T, WB>& R2, int comp, const T* __restrict__ xb,
                           const T* __restrict__ xb_prev) {
    const int P = g.P;
    const int64_t cs = (int64_t)g.nc * g.Pd;
    const int64_t coff = (int64_t)comp * g.Pd;
    T acc = 0;
    if (D == 1) {
#pragma unroll
        for (int e0 = 0; e0 < WB; ++e0)
            if (e0 < R0.n) {
                const int64_t j = R0.cell[e0] * cs + coff + R0.mode[e0];
                T xv = xb[j];
                if (MODE == MODE_RES) xv -= xb_prev[j];
                acc += R0.v[e0] * xv;
            }
    } else if (D == 2) {
#pragma unroll
        for (int e1 = 0; e1 < WB; ++e1) {
            if (e1 >= R1.n) continue;
            const int64_t cb = (int64_t)R1.cell[e1] * g.m[0];
            const int mb = R1.mode[e1] * P;
#pragma unroll
            for (int e0 = 0; e0 < WB; ++e0)
                if (e0 < R0.n) {
                    const int64_t j = (cb + R0.cell[e0]) * cs + coff + mb + R0.mode[e0];
                    T xv = xb[j];
                    if (MODE == MODE_RES) xv -= xb_prev[j];
                    acc += R0.v[e0] * R1.v[e1] * xv;
                }
        }
    } else {
#pragma unroll
        for (int e2 = 0; e2 < WB; ++e2)
#pragma unroll
            for (int e1 = 0; e1 < WB; ++e1) {
                if (e2 >= R2.n || e1 >= R1.n) continue;
                const int64_t cb = ((int64_t)R2.cell[e2] * g.m[1] + R1.cell[e1]) * g.m[0];
                const int mb = (R2.mode[e2] * P + R1.mode[e1]) * P;
                const T v12 = R1.v[e1] * R2.v[e2];
#pragma unroll
                for (int e0 = 0; e0 < WB; ++e0)
                    if (e0 < R0.n) {
                        const int64_t j = (cb + R0.cell[e0]) * cs + coff + mb + R0.mode[e0];
                        T xv = xb[j];
                        if (MODE == MODE_RES) xv -= xb_prev[j];
                        acc += R0.v[e0] * v12 * xv;
                    }
            }
    }
    return acc;
}

// ---------------------------------------------------------------------------
// u-side: y_u = alpha A x_u + sum_c B^(c) x_psi^(c)  (+ residual epilogue)
template <typename T, int D, int MODE>
__global__ __launch_bounds__(128) void k_u_side_grad(Geo g, URows<T> r0, URows<T> r1,
                                                     URows<T> r2, T alpha,
                                                     const T* __restrict__ xu,
                                                     const T* __restrict__ xb,
                                                     const T* __restrict__ xb_prev,
                                                     const double* __restrict__ F,
                                                     T* __restrict__ yu,
                                                     double* __restrict__ partial,
                                                     const int* __restrict__ done,
                                                     const double* __restrict__ prm) {
    __shared__ double red[2];
    if (done && *done) return;
    if (prm) alpha = (T)prm[0];
    constexpr int WB = URows<T>::WB;
    double part = 0.0;
    for (int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; I < g.n_u;
         I += (int64_t)gridDim.x * blockDim.x) {
        int gi[3] = {0, 0, 0};
        int64_t t = I;
        gi[0] = (int)(t % g.n1[0]);
        t /= g.n1[0];
        if (D >= 2) {
            gi[1] = (int)(t % g.n1[1]);
            t /= g.n1[1];
        }
        if (D >= 3) gi[2] = (int)t;
        T acc = stiff_mass_sum<T, D>(g, r0, r1, r2, gi, xu) * alpha;
        BRow<T, WB> B0, B1, B2, G0, G1, G2;
        B0.load(r0, gi[0]);
        G0.loadG(r0, gi[0]);
        B1.n = B2.n = G1.n = G2.n = 0;
        if (D >= 2) {
            B1.load(r1, gi[1]);
            G1.loadG(r1, gi[1]);
        }
        if (D >= 3) {
            B2.load(r2, gi[2]);
            G2.loadG(r2, gi[2]);
        }
        acc += couple<T, D, MODE, WB>(g, G0, B1, B2, 0, xb, xb_prev);
        if (D >= 2) acc += couple<T, D, MODE, WB>(g, B0, G1, B2, 1, xb, xb_prev);
        if (D >= 3) acc += couple<T, D, MODE, WB>(g, B0, B1, G2, 2, xb, xb_prev);
        if (MODE == MODE_RES) {
            const double r = (double)acc - (double)alpha * F[I];
            yu[I] = (T)r;
            part += r * r;
        } else {
            yu[I] = acc;
            part += (double)acc * (double)xu[I];
        }
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// psi-side (per component c):
//   apply:    y_c = B^(c)T x_u - sum_l D_cl x_l - beta E x_c
//   residual: y_c = B^(c)T u - N_c(psi)      (T = double; x_psi = psi)
// LDS per cell (stride S = max(p+1, q)^d): u box, then d buffers each of
// B^(c)T x_u, x_c and the values at the Gauss points, two work buffers and
// one E accumulator.
template <typename T, int D>
__host__ __device__ inline int grad_psi_bufs() {
    return 1 + 3 * D + 3;
}

template <typename T, int D, int MODE>
__global__ __launch_bounds__(256) void k_psi_side_grad(Geo g, PsiTabs<T> tb, int cpb, T beta,
                                                       const T* __restrict__ xu,
                                                       const T* __restrict__ xpsi,
                                                       const T* __restrict__ omega,
                                                       const double* __restrict__ phi_q,
                                                       T* __restrict__ ypsi,
                                                       double* __restrict__ partial,
                                                       const int* __restrict__ done,
                                                       const double* __restrict__ prm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    if (done && *done) return;
    if (prm) beta = (T)prm[1];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int S = g.S, L = g.p + 1, P = g.P, q = g.q, Pd = g.Pd, Qd = g.Qd;
    constexpr int NP = D * (D + 1) / 2;
    const int cs = cpb * S;   // one buffer for the block's cells
    T* bU = sm;
    T* bT = sm + cs;              // [c][cell][S]
    T* bX = bT + D * cs;
    T* bV = bX + D * cs;
    T* bA = bV + D * cs;
    T* bB = bA + cs;
    T* bE = bB + cs;
    double part = 0.0;
    const int64_t ngroups = (g.n_cells + cpb - 1) / cpb;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t cell0 = grp * cpb;
        const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
        gather_u<T, D>(g, xu, bU, S, cell0, ncell);
        for (int e = threadIdx.x; e < ncell * D * Pd; e += blockDim.x) {
            const int ci = e / (D * Pd), r = e - ci * D * Pd, c = r / Pd, a = r - c * Pd;
            bX[c * cs + ci * S + a] = xpsi[(cell0 + ci) * D * Pd + r];
        }
        __syncthreads();
        // B^(c)T x_u: G1 along direction c, B1 along the others ((p+1)^d -> P^d)
        for (int c = 0; c < D; ++c) {
            for (int e = threadIdx.x; e < ncell * g.Ld; e += blockDim.x) {
                const int ci = e / g.Ld, l = e - ci * g.Ld;
                bA[ci * S + l] = bU[ci * S + l];
            }
            __syncthreads();
            const T* mats[3] = {c == 0 ? tb.G1 : tb.B1, c == 1 ? tb.G1 : tb.B1,
                                c == 2 ? tb.G1 : tb.B1};
            T* t = contract_axes<T, D>(bA, bB, S, ncell, L, P, mats, P, true);
            for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                const int ci = e / Pd, a = e - ci * Pd;
                bT[c * cs + ci * S + a] = t[ci * S + a];
            }
            __syncthreads();
        }
        // components at the Gauss points (P^d -> q^d)
        for (int c = 0; c < D; ++c) {
            for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                const int ci = e / Pd, a = e - ci * Pd;
                bA[ci * S + a] = bX[c * cs + ci * S + a];
            }
            __syncthreads();
            T* vq = contract_all<T, D>(bA, bB, S, ncell, P, q, tb.Vpsi, P, false);
            for (int e = threadIdx.x; e < ncell * Qd; e += blockDim.x) {
                const int ci = e / Qd, j = e - ci * Qd;
                bV[c * cs + ci * S + j] = vq[ci * S + j];
            }
            __syncthreads();
        }
        // pointwise: weights (apply) or the flux phi psi / sqrt(1 + |psi|^2) (residual)
        for (int e = threadIdx.x; e < ncell * Qd; e += blockDim.x) {
            const int ci = e / Qd, j = e - ci * Qd;
            const int64_t cell = cell0 + ci;
            T v[3] = {0, 0, 0};
            for (int c = 0; c < D; ++c) v[c] = bV[c * cs + ci * S + j];
            if (MODE == MODE_RES) {
                T hk[3];
                const T J = cell_jac<T, D>(g, tb.h, cell, hk);
                int jj[3] = {j % q, (j / q) % q, j / (q * q)};
                double wq = (double)J;
                for (int k = 0; k < D; ++k) wq *= (double)tb.w[jj[k]];
                double s2 = 1.0;
                for (int c = 0; c < D; ++c) s2 += (double)v[c] * (double)v[c];
                const double sc = wq * phi_q[cell * Qd + j] / sqrt(s2);
                for (int c = 0; c < D; ++c) bV[c * cs + ci * S + j] = (T)(sc * (double)v[c]);
            } else {
                const T* om = omega + cell * (int64_t)NP * Qd;
                for (int c = 0; c < D; ++c) {
                    T w = 0;
                    for (int l = 0; l < D; ++l) w += om[pair_index(c, l, D) * Qd + j] * v[l];
                    bV[c * cs + ci * S + j] = w;
                }
            }
        }
        __syncthreads();
        for (int c = 0; c < D; ++c) {
            // back to the Legendre modes (q^d -> P^d)
            for (int e = threadIdx.x; e < ncell * Qd; e += blockDim.x) {
                const int ci = e / Qd, j = e - ci * Qd;
                bA[ci * S + j] = bV[c * cs + ci * S + j];
            }
            __syncthreads();
            T* dx = contract_all<T, D>(bA, bB, S, ncell, q, P, tb.Vpsi, P, true);
            for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                const int ci = e / Pd, a = e - ci * Pd;
                bV[c * cs + ci * S + a] = dx[ci * S + a];
            }
            __syncthreads();
            // E x_c = sum_k c_k (x)_j (j == k ? AY : MY) x_c, c_k = (2/h_k) prod_{j != k} h_j/2
            const bool with_e = MODE == MODE_APPLY && beta != (T)0;
            if (with_e) {
                for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                    const int ci = e / Pd, a = e - ci * Pd;
                    bE[ci * S + a] = 0;
                }
                for (int k = 0; k < D; ++k) {
                    for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                        const int ci = e / Pd, a = e - ci * Pd;
                        bA[ci * S + a] = bX[c * cs + ci * S + a];
                    }
                    __syncthreads();
                    const T* mats[3] = {k == 0 ? tb.AY : tb.MY, k == 1 ? tb.AY : tb.MY,
                                        k == 2 ? tb.AY : tb.MY};
                    T* ex = contract_axes<T, D>(bA, bB, S, ncell, P, P, mats, P, false);
                    for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                        const int ci = e / Pd, a = e - ci * Pd;
                        T hk[3];
                        const T J = cell_jac<T, D>(g, tb.h, cell0 + ci, hk);
                        const T ck = J * ((T)2 / hk[k]) * ((T)2 / hk[k]);
                        bE[ci * S + a] += ck * ex[ci * S + a];
                    }
                    __syncthreads();
                }
            }
            for (int e = threadIdx.x; e < ncell * Pd; e += blockDim.x) {
                const int ci = e / Pd, a = e - ci * Pd;
                const int64_t cell = cell0 + ci;
                T hk[3];
                const T J = cell_jac<T, D>(g, tb.h, cell, hk);
                const T bt = bT[c * cs + ci * S + a] * J * ((T)2 / hk[c]);   // prod_{k != c} h_k/2
                const int64_t o = cell * D * Pd + (int64_t)c * Pd + a;
                if (MODE == MODE_RES) {
                    const double r = (double)bt - (double)bV[c * cs + ci * S + a];
                    ypsi[o] = (T)r;
                    part += r * r;
                } else {
                    const T xv = bX[c * cs + ci * S + a];
                    T y = bt - bV[c * cs + ci * S + a];
                    if (with_e) y -= beta * bE[ci * S + a];
                    ypsi[o] = y;
                    part += (double)y * (double)xv;
                }
            }
            __syncthreads();
        }
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}


// Newton-step setup, one cell per block: the weights and the inverse of
// -S_hat_K = D_K + beta E_K (n = d P^d, SPD).  BIG: the block is formed and
// inverted in place in sinv64 (global memory) instead of LDS.
template <int D, bool BIG>
__global__ __launch_bounds__(256) void k_setup_grad(Geo g, PsiTabs<double> tb,
                                                    const double* __restrict__ psi,
                                                    const double* __restrict__ phi_q,
                                                    double beta, double* __restrict__ om64,
                                                    float* __restrict__ om32,
                                                    double* __restrict__ s64,
                                                    float* __restrict__ s32) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int S = g.S, P = g.P, q = g.q, Pd = g.Pd, Qd = g.Qd, n = D * Pd;
    constexpr int NP = D * (D + 1) / 2;
    const int PP = P * P;
    const int sT1 = D == 1 ? 1 : (D == 2 ? q * PP : q * q * PP);
    const int sT2 = D == 3 ? q * PP * PP : 1;
    const int64_t cell = blockIdx.x;
    double* bA = sm;
    double* bB = bA + S;
    double* bV = bB + S;            // D x S: components at the Gauss points
    double* W = bV + D * S;         // NP x Qd weights
    double* T1 = W + NP * Qd;
    double* T2 = T1 + sT1;
    double* Eb = T2 + sT2;          // Pd x Pd: E_K
    double* cr = Eb + Pd * Pd;      // 2n: pivot column / row
    double* Dm = BIG ? s64 + cell * (int64_t)n * n : cr + 2 * n;
    // components at the Gauss points
    for (int c = 0; c < D; ++c) {
        for (int a = threadIdx.x; a < Pd; a += blockDim.x) bA[a] = psi[cell * n + c * Pd + a];
        __syncthreads();
        double* vq = contract_all<double, D>(bA, bB, S, 1, P, q, tb.Vpsi, P, false);
        for (int j = threadIdx.x; j < Qd; j += blockDim.x) bV[c * S + j] = vq[j];
        __syncthreads();
    }
    double hk[3];
    const double J = cell_jac<double, D>(g, tb.h, cell, hk);
    // weights w_q |J| phi_q F_cl(psi_h(x_q))
    for (int j = threadIdx.x; j < Qd; j += blockDim.x) {
        int jj[3] = {j % q, (j / q) % q, j / (q * q)};
        double wq = J;
        for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
        double v[3] = {0, 0, 0}, s2 = 1.0;
        for (int c = 0; c < D; ++c) {
            v[c] = bV[c * S + j];
            s2 += v[c] * v[c];
        }
        const double f = wq * phi_q[cell * Qd + j] / (s2 * sqrt(s2));
        for (int c = 0; c < D; ++c)
            for (int l = c; l < D; ++l) {
                const double om = f * ((c == l ? s2 : 0.0) - v[c] * v[l]);
                const int pr = pair_index(c, l, D);
                W[pr * Qd + j] = om;
                const int64_t off = (cell * NP + pr) * (int64_t)Qd + j;
                if (om64) om64[off] = om;
                if (om32) om32[off] = (float)om;
            }
    }
    __syncthreads();
    // D blocks (c, l) and their mirror images
    for (int c = 0; c < D; ++c)
        for (int l = c; l < D; ++l) {
            double* blk = Dm + (int64_t)(c * Pd) * n + l * Pd;
            d_block<D>(W + pair_index(c, l, D) * Qd, tb.Vpsi, P, q, T1, T2, blk, n);
            if (l != c) {
                for (int e = threadIdx.x; e < Pd * Pd; e += blockDim.x) {
                    const int a = e / Pd, b = e % Pd;
                    Dm[(int64_t)(l * Pd + b) * n + c * Pd + a] = blk[(int64_t)a * n + b];
                }
                __syncthreads();
            }
        }
    // + beta E on the diagonal blocks: E_ab = sum_k c_k prod_j (j == k ? AY : MY)[a_j][b_j]
    if (beta != 0.0) {
        for (int e = threadIdx.x; e < Pd * Pd; e += blockDim.x) {
            const int a = e / Pd, b = e % Pd;
            int aa[3] = {a % P, (a / P) % P, a / (P * P)};
            int bb[3] = {b % P, (b / P) % P, b / (P * P)};
            double s = 0.0;
            for (int k = 0; k < D; ++k) {
                double t = J * (2.0 / hk[k]) * (2.0 / hk[k]);
                for (int j = 0; j < D; ++j)
                    t *= (j == k ? tb.AY : tb.MY)[aa[j] * P + bb[j]];
                s += t;
            }
            Eb[e] = beta * s;
        }
        __syncthreads();
        for (int c = 0; c < D; ++c)
            for (int e = threadIdx.x; e < Pd * Pd; e += blockDim.x) {
                const int a = e / Pd, b = e % Pd;
                Dm[(int64_t)(c * Pd + a) * n + c * Pd + b] += Eb[e];
            }
        __syncthreads();
    }
    gauss_jordan_spd(Dm, n, cr);
    // symmetrise (the exact inverse is symmetric) and store
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        if (j < i) continue;
        const double v = 0.5 * (Dm[(int64_t)i * n + j] + Dm[(int64_t)j * n + i]);
        const int64_t o1 = cell * (int64_t)n * n + (int64_t)i * n + j;
        const int64_t o2 = cell * (int64_t)n * n + (int64_t)j * n + i;
        if (!BIG) {
            if (s64) {
                s64[o1] = v;
                s64[o2] = v;
            }
        } else {
            Dm[(int64_t)i * n + j] = v;
            Dm[(int64_t)j * n + i] = v;
        }
        if (s32) {
            s32[o1] = (float)v;
            s32[o2] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// z_psi = (-S_hat_K)^{-1} r_psi for large blocks: the cell's residual in LDS,
// thread i forms z_i = sum_j S[j][i] r_j (S symmetric) reading row j of the
// inverse coalesced.  Partial dot <z, r> fused.
template <typename T>
__global__ __launch_bounds__(256) void k_prec_psi_big(int64_t n_cells, int n,
                                                      const T* __restrict__ sinv,
                                                      const T* __restrict__ r,
                                                      T* __restrict__ z,
                                                      double* __restrict__ partial,
                                                      const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    if (done && *done) return;
    T* rb = reinterpret_cast<T*>(smem_raw);
    double part = 0.0;
    for (int64_t cell = blockIdx.x; cell < n_cells; cell += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) rb[i] = r[cell * n + i];
        __syncthreads();
        const T* Sb = sinv + cell * (int64_t)n * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            T acc = 0;
            for (int j = 0; j < n; ++j) acc += Sb[(int64_t)j * n + i] * rb[j];
            z[cell * n + i] = acc;
            part += (double)acc * (double)rb[i];
        }
        __syncthreads();
    }
    if (partial) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned nblk_g(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_u_side_grad(const Geo& g, const URows<T>* r, T alpha, const T* xu, const T* xb,
                        const T* xb_prev, const double* F, T* yu, double* partial,
                        const int* done, int mode, hipStream_t s, const double* prm) {
    const unsigned grid = partial ? (unsigned)std::min<int64_t>(nblk_g(g.n_u, 128), 1024)
                                  : (unsigned)std::min<int64_t>(nblk_g(g.n_u, 128), 1 << 20);
#define HPG_UG(DD, MM)                                                                          \
    hipLaunchKernelGGL((k_u_side_grad<T, DD, MM>), dim3(grid), dim3(128), 0, s, g, r[0], r[1], \
                       r[2], alpha, xu, xb, xb_prev, F, yu, partial, done, prm)
    if (mode == MODE_RES) {
        if (g.d == 1) HPG_UG(1, MODE_RES);
        else if (g.d == 2) HPG_UG(2, MODE_RES);
        else HPG_UG(3, MODE_RES);
    } else {
        if (g.d == 1) HPG_UG(1, MODE_APPLY);
        else if (g.d == 2) HPG_UG(2, MODE_APPLY);
        else HPG_UG(3, MODE_APPLY);
    }
#undef HPG_UG
}

template <typename T>
int psi_side_grad_cpb(const Geo& g) {
    const size_t per = (size_t)(1 + 3 * g.d + 3) * g.S * sizeof(T);
    int cpb = std::max(1, 256 / std::max(1, g.Qd));
    while (cpb > 1 && (size_t)cpb * per > 48 * 1024) --cpb;
    return cpb;
}

template <typename T>
void launch_psi_side_grad(const Geo& g, const PsiTabs<T>& tb, int cpb, T beta, const T* xu,
                          const T* xpsi, const T* omega, const double* phi_q, T* ypsi,
                          double* partial, const int* done, int mode, hipStream_t s,
                          const double* prm) {
    const size_t smem = (size_t)(1 + 3 * g.d + 3) * g.S * cpb * sizeof(T);
    const int64_t ngroups = (g.n_cells + cpb - 1) / cpb;
    const unsigned grid = (unsigned)std::min<int64_t>(ngroups, 1024);
#define HPG_PG(DD, MM)                                                                        \
    hipLaunchKernelGGL((k_psi_side_grad<T, DD, MM>), dim3(grid), dim3(256), smem, s, g, tb, \
                       cpb, beta, xu, xpsi, omega, phi_q, ypsi, partial, done, prm)
    if (mode == MODE_RES) {
        if (g.d == 1) HPG_PG(1, MODE_RES);
        else if (g.d == 2) HPG_PG(2, MODE_RES);
        else HPG_PG(3, MODE_RES);
    } else {
        if (g.d == 1) HPG_PG(1, MODE_APPLY);
        else if (g.d == 2) HPG_PG(2, MODE_APPLY);
        else HPG_PG(3, MODE_APPLY);
    }
#undef HPG_PG
}

// LDS of the setup kernel (doubles), without the block itself
static size_t setup_grad_work(const Geo& g) {
    const int d = g.d, P = g.P, q = g.q, PP = P * P, n = d * g.Pd;
    const size_t sT1 = d == 1 ? 1 : (d == 2 ? (size_t)q * PP : (size_t)q * q * PP);
    const size_t sT2 = d == 3 ? (size_t)q * PP * PP : 1;
    return (size_t)(2 + d) * g.S + (size_t)(d * (d + 1) / 2) * g.Qd + sT1 + sT2 +
           (size_t)g.Pd * g.Pd + 2 * (size_t)n;
}

bool setup_grad_in_hbm(const Geo& g) {
    const size_t n = (size_t)g.d * g.Pd;
    return (setup_grad_work(g) + n * n) * sizeof(double) > 120 * 1024;
}

void launch_setup_grad(const Geo& g, const PsiTabs<double>& tb, const double* psi,
                       const double* phi_q, double beta, double* om64, float* om32, double* s64,
                       float* s32, hipStream_t s) {
    const int n = g.d * g.Pd;
    const size_t work = setup_grad_work(g);
    const bool big = setup_grad_in_hbm(g);
    const size_t smem = (work + (big ? 0 : (size_t)n * n)) * sizeof(double);
    const unsigned grid = (unsigned)g.n_cells;
#define HPG_SG(DD, BB)                                                                         \
    hipLaunchKernelGGL((k_setup_grad<DD, BB>), dim3(grid), dim3(256), smem, s, g, tb, psi,     \
                       phi_q, beta, om64, om32, s64, s32)
    if (g.d == 1) {
        if (big) HPG_SG(1, true); else HPG_SG(1, false);
    } else if (g.d == 2) {
        if (big) HPG_SG(2, true); else HPG_SG(2, false);
    } else {
        if (big) HPG_SG(3, true); else HPG_SG(3, false);
    }
#undef HPG_SG
}

template <typename T>
void launch_prec_psi_big(int64_t n_cells, int n, const T* sinv, const T* r, T* z,
                         double* partial, int nblocks, const int* done, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(n_cells, nblocks);
    hipLaunchKernelGGL((k_prec_psi_big<T>), dim3(grid), dim3(256), (size_t)n * sizeof(T), s,
                       n_cells, n, sinv, r, z, partial, done);
}

template void launch_u_side_grad<double>(const Geo&, const URows<double>*, double, const double*,
                                         const double*, const double*, const double*, double*,
                                         double*, const int*, int, hipStream_t, const double*);
template void launch_u_side_grad<float>(const Geo&, const URows<float>*, float, const float*,
                                        const float*, const float*, const double*, float*,
                                        double*, const int*, int, hipStream_t, const double*);
template int psi_side_grad_cpb<double>(const Geo&);
template int psi_side_grad_cpb<float>(const Geo&);
template void launch_psi_side_grad<double>(const Geo&, const PsiTabs<double>&, int, double,
                                           const double*, const double*, const double*,
                                           const double*, double*, double*, const int*, int,
                                           hipStream_t, const double*);
template void launch_psi_side_grad<float>(const Geo&, const PsiTabs<float>&, int, float,
                                          const float*, const float*, const float*,
                                          const double*, float*, double*, const int*, int,
                                          hipStream_t, const double*);
template void launch_prec_psi_big<double>(int64_t, int, const double*, const double*, double*,
                                          double*, int, const int*, hipStream_t);
template void launch_prec_psi_big<float>(int64_t, int, const float*, const float*, float*,
                                         double*, int, const int*, hipStream_t);

}  // namespace dev
}  // namespace hpg
