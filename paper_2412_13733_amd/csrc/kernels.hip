// Device kernels of the hpG Newton/Krylov path for gfx950 (wave64).
//
// Data layout in HBM (one problem):
//   u vectors : n1_0 x n1_1 x n1_2 array, direction 0 fastest (global 1-D
//               unknown of local function l of cell c is c*p + l - 1).
//   psi       : cell-major blocks of P^d Legendre coefficients.
//   omega     : cell-major blocks of q^d quadrature weights of D_psi.
//   Sinv      : cell-major dense (P^d)^2 inverses of -S_hat_K (symmetric).
//
// The u-side of G (alpha A x_u + B x_psi) is evaluated owner-computes: one
// thread per global u unknown sums the tensor products of the sparse global
// 1-D rows (stiffness/mass/Gram), so the assembly is deterministic and needs
// no atomics or scratch.  The psi-side (B^T x_u - D_psi x_psi - E_beta x_psi)
// is cell-local: a block stages several cells' coefficients in LDS and
// applies D_psi sum-factorised through the Gauss-Legendre points
// (paper Sec. 4.3: D_psi = V^T diag(omega) V per cell).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dev_util.h"
#include "kernels.h"

namespace hpg {
namespace dev {

// ---------------------------------------------------------------------------
// u-side: y_u = alpha A x_u + B x_b  (+ residual epilogue).  Each thread owns
// global u unknowns (grid-stride); the sparse 1-D rows of its multi-index are
// held in registers and the tensor-product sums are unrolled over the fixed
// row width with predication.
template <typename T, int D, int MODE>
__global__ __launch_bounds__(128) void k_u_side(Geo g, URows<T> r0, URows<T> r1, URows<T> r2,
                                                T alpha, const T* __restrict__ xu,
                                                const T* __restrict__ xb,
                                                const T* __restrict__ xb_prev,
                                                const double* __restrict__ F,
                                                T* __restrict__ yu, double* __restrict__ partial,
                                                const int* __restrict__ done,
                                                const double* __restrict__ prm) {
    __shared__ double red[2];
    if (done && *done) return;
    if (prm) alpha = (T)prm[0];   // linearisation parameters held on the device
    constexpr int W = URows<T>::WM, WB = URows<T>::WB;
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
        T acc = stiff_mass_sum<T, D>(g, r0, r1, r2, gi, xu);
        acc *= alpha;
        // Gram: (x)_k B1 applied to x_b = x_psi (or psi - psi_prev)
        BRow<T, WB> B0;
        B0.load(r0, gi[0]);
        const int P = g.P;
        if (D == 1) {
#pragma unroll
            for (int e0 = 0; e0 < WB; ++e0)
                if (e0 < B0.n) {
                    const int64_t j = (int64_t)B0.cell[e0] * g.Pd + B0.mode[e0];
                    T xv = xb[j];
                    if (MODE == MODE_RES) xv -= xb_prev[j];
                    acc += B0.v[e0] * xv;
                }
        } else if (D == 2) {
            BRow<T, WB> B1;
            B1.load(r1, gi[1]);
#pragma unroll
            for (int e1 = 0; e1 < WB; ++e1) {
                if (e1 >= B1.n) continue;
                const int64_t cbase = (int64_t)B1.cell[e1] * g.m[0];
                const int mbase = B1.mode[e1] * P;
#pragma unroll
                for (int e0 = 0; e0 < WB; ++e0)
                    if (e0 < B0.n) {
                        const int64_t j = (cbase + B0.cell[e0]) * g.Pd + mbase + B0.mode[e0];
                        T xv = xb[j];
                        if (MODE == MODE_RES) xv -= xb_prev[j];
                        acc += B0.v[e0] * B1.v[e1] * xv;
                    }
            }
        } else {
            BRow<T, WB> B1, B2;
            B1.load(r1, gi[1]);
            B2.load(r2, gi[2]);
#pragma unroll
            for (int e2 = 0; e2 < WB; ++e2)
#pragma unroll
                for (int e1 = 0; e1 < WB; ++e1) {
                    if (e2 >= B2.n || e1 >= B1.n) continue;
                    const int64_t cbase = ((int64_t)B2.cell[e2] * g.m[1] + B1.cell[e1]) * g.m[0];
                    const int mbase = (B2.mode[e2] * P + B1.mode[e1]) * P;
                    const T v12 = B1.v[e1] * B2.v[e2];
#pragma unroll
                    for (int e0 = 0; e0 < WB; ++e0)
                        if (e0 < B0.n) {
                            const int64_t j = (cbase + B0.cell[e0]) * g.Pd + mbase + B0.mode[e0];
                            T xv = xb[j];
                            if (MODE == MODE_RES) xv -= xb_prev[j];
                            acc += B0.v[e0] * v12 * xv;
                        }
                }
        }
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
        double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// psi-side of G (obstacle): y_psi = B_K^T x_u - D_K x_psi - beta M_psi x_psi
// residual mode (T = double): y_psi = B_K^T u + (exp(-psi_h), zeta) - Phi
template <typename T, int D, int MODE>
__global__ __launch_bounds__(256) void k_psi_side(Geo g, PsiTabs<T> tb, int cpb, T beta,
                                                  const T* __restrict__ xu,
                                                  const T* __restrict__ xpsi,
                                                  const T* __restrict__ omega,
                                                  const double* __restrict__ Phi,
                                                  T* __restrict__ ypsi,
                                                  double* __restrict__ partial,
                                                  const int* __restrict__ done,
                                                  const double* __restrict__ prm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    if (done && *done) return;
    if (prm) beta = (T)prm[1];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int S = g.S;   // per-cell buffer stride (max(p+1, q)^D)
    T* bU = sm;
    T* bX = sm + cpb * S;
    T* bT = sm + 2 * cpb * S;
    T* bA = sm + 3 * cpb * S;
    T* bB = sm + 4 * cpb * S;
    const int L = g.p + 1, P = g.P, q = g.q;
    double part = 0.0;
    const int64_t ngroups = (g.n_cells + cpb - 1) / cpb;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t cell0 = grp * cpb;
    const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
    gather_u<T, D>(g, xu, bU, S, cell0, ncell);
    for (int e = threadIdx.x; e < ncell * g.Pd; e += blockDim.x) {
        const int ci = e / g.Pd, a = e - ci * g.Pd;
        bX[ci * S + a] = xpsi[(cell0 + ci) * g.Pd + a];
    }
    __syncthreads();
    // t = (x)_k B1^T x_u  ((p+1)^D -> P^D), scaled by prod_k h_k/2 below
    T* t = contract_all<T, D>(bU, bT, S, ncell, L, P, tb.B1, P, true);
    if (t != bT) {
        for (int e = threadIdx.x; e < ncell * g.Pd; e += blockDim.x) {
            const int ci = e / g.Pd, a = e - ci * g.Pd;
            bT[ci * S + a] = t[ci * S + a];
        }
        __syncthreads();
    }
    // psi_h (or x_psi) at the quadrature points: P^D -> q^D
    for (int e = threadIdx.x; e < ncell * g.Pd; e += blockDim.x) {
        const int ci = e / g.Pd, a = e - ci * g.Pd;
        bA[ci * S + a] = bX[ci * S + a];
    }
    __syncthreads();
    T* vq = contract_all<T, D>(bA, bB, S, ncell, P, q, tb.Vpsi, P, false);
    T* other = (vq == bA) ? bB : bA;
    for (int e = threadIdx.x; e < ncell * g.Qd; e += blockDim.x) {
        const int ci = e / g.Qd, j = e - ci * g.Qd;
        const int64_t cell = cell0 + ci;
        if (MODE == MODE_RES) {
            T hk[3];
            const T J = cell_jac<T, D>(g, tb.h, cell, hk);
            int jj[3] = {j % q, (j / q) % q, j / (q * q)};
            T wq = J;
            for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
            const double arg = -(double)vq[ci * S + j];
            vq[ci * S + j] = (T)((double)wq * exp(arg < 700.0 ? arg : 700.0));
        } else {
            vq[ci * S + j] *= omega[cell * g.Qd + j];
        }
    }
    __syncthreads();
    T* dx = contract_all<T, D>(vq, other, S, ncell, q, P, tb.Vpsi, P, true);
    for (int e = threadIdx.x; e < ncell * g.Pd; e += blockDim.x) {
        const int ci = e / g.Pd, a = e - ci * g.Pd;
        const int64_t cell = cell0 + ci;
        T hk[3];
        const T J = cell_jac<T, D>(g, tb.h, cell, hk);
        const T bt = bT[ci * S + a] * J;   // B_K^T x_u: prod_k (h_k/2) B1^T
        T y;
        if (MODE == MODE_RES) {
            const double r = (double)bt + (double)dx[ci * S + a] - Phi[cell * g.Pd + a];
            y = (T)r;
            part += r * r;
        } else {
            int aa[3] = {a % P, (a / P) % P, a / (P * P)};
            T md = J;
            for (int k = 0; k < D; ++k) md *= tb.Mdiag[aa[k]];
            y = bt - dx[ci * S + a] - beta * md * bX[ci * S + a];
            part += (double)y * (double)bX[ci * S + a];
        }
        ypsi[cell * g.Pd + a] = y;
    }
    __syncthreads();   // the LDS buffers are reused by the next cell group
    }
    if (partial) {
        double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Newton-step setup (obstacle), FP64: omega_q = w_q |J| exp(-psi_h(x_q)),
// D_K = V^T diag(omega) V (sum-factorised), -S_hat_K = D_K + beta M_K + C_K/alpha,
// inverted in LDS by Gauss-Jordan (SPD: no pivoting needed).
template <int D>
__global__ __launch_bounds__(256) void k_setup(Geo g, PsiTabs<double> tb, int cpb,
                                               const double* __restrict__ psi, double alpha,
                                               double beta, const double* __restrict__ Cmat,
                                               const int* __restrict__ cclass,
                                               double* __restrict__ omega64,
                                               float* __restrict__ omega32,
                                               double* __restrict__ sinv64,
                                               float* __restrict__ sinv32,
                                               const double* __restrict__ prm_req,
                                               const int* __restrict__ mask, int64_t cpr,
                                               int* __restrict__ sflag, int packed) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int n = g.Pd, q = g.q, P = g.P, Qd = g.Qd;
    // batches: the request of a cell, whether it is set up now, its alpha and beta
    auto live = [&](int64_t cell) { return !mask || mask[cell / cpr] != 0; };
    auto a_of = [&](int64_t cell) { return prm_req ? prm_req[4 * (cell / cpr)] : alpha; };
    auto b_of = [&](int64_t cell) { return prm_req ? prm_req[4 * (cell / cpr) + 1] : beta; };
    const int S = g.S;
    // per cell: A, B (S each), T1 (q^(D-1) P^2), T2 (q P^4, D = 3), Dm (n^2), col/row (2n),
    // the 1-norm of -S_hat (1)
    const int sT1 = (D == 1) ? 1 : ((D == 2) ? q * P * P : q * q * P * P);
    const int sT2 = (D == 3) ? q * P * P * P * P : 1;
    const int per = 2 * S + sT1 + sT2 + n * n + 2 * n + 1;
    const int64_t cell0 = (int64_t)blockIdx.x * cpb;
    const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
    if (mask) {
        // a block none of whose cells is set up now has nothing to do
        bool any = false;
        for (int ci = 0; ci < ncell; ++ci) any = any || live(cell0 + ci);
        if (!any) return;
    }
    double* bA = sm;
    double* bB = sm + cpb * S;
    double* T1 = sm + 2 * cpb * S;
    double* T2 = T1 + cpb * sT1;
    double* Dm = T2 + cpb * sT2;
    double* cr = Dm + cpb * n * n;
    double* nrm = cr + cpb * 2 * n;
    // 1-norm of each block of Dm into nrm[ci] (column sums staged in cr)
    auto block_norm1 = [&]() {
        for (int e = threadIdx.x; e < ncell * n; e += blockDim.x) {
            const int ci = e / n, j = e - ci * n;
            double cs = 0.0;
            for (int i = 0; i < n; ++i) cs += fabs(Dm[ci * n * n + i * n + j]);
            cr[ci * 2 * n + j] = cs;
        }
        __syncthreads();
        for (int ci = threadIdx.x; ci < ncell; ci += blockDim.x) {
            double m = 0.0;
            for (int j = 0; j < n; ++j) m = fmax(m, cr[ci * 2 * n + j]);
            nrm[ci] = m;
        }
        __syncthreads();
    };
    for (int e = threadIdx.x; e < ncell * n; e += blockDim.x) {
        const int ci = e / n, a = e - ci * n;
        bA[ci * S + a] = psi[(cell0 + ci) * n + a];
    }
    __syncthreads();
    double* vq = contract_all<double, D>(bA, bB, S, ncell, P, q, tb.Vpsi, P, false);
    // omega
    for (int e = threadIdx.x; e < ncell * Qd; e += blockDim.x) {
        const int ci = e / Qd, j = e - ci * Qd;
        const int64_t cell = cell0 + ci;
        double hk[3];
        const double J = cell_jac<double, D>(g, tb.h, cell, hk);
        int jj[3] = {j % q, (j / q) % q, j / (q * q)};
        double wq = J;
        for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
        const double arg = -vq[ci * S + j];
        const double om = wq * exp(arg < 700.0 ? arg : 700.0);
        vq[ci * S + j] = om;
        if (!live(cell)) continue;
        if (omega64) omega64[cell * Qd + j] = om;
        if (omega32) omega32[cell * Qd + j] = (float)om;
    }
    __syncthreads();
    const double* V = tb.Vpsi;   // q x P
    const int PP = P * P;
    if (D == 1) {
        for (int e = threadIdx.x; e < ncell * PP; e += blockDim.x) {
            const int ci = e / PP, ab = e - ci * PP;
            const int a = ab / P, b = ab % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += vq[ci * S + j] * V[j * P + a] * V[j * P + b];
            Dm[ci * n * n + a * n + b] = s;
        }
        __syncthreads();
    } else if (D == 2) {
        // T1[q2][a1 b1] = sum_q1 omega[q2][q1] V[q1,a1] V[q1,b1]
        for (int e = threadIdx.x; e < ncell * q * PP; e += blockDim.x) {
            const int ci = e / (q * PP), r = e - ci * q * PP;
            const int q2 = r / PP, ab = r % PP, a1 = ab / P, b1 = ab % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j)
                s += vq[ci * S + q2 * q + j] * V[j * P + a1] * V[j * P + b1];
            T1[ci * sT1 + r] = s;
        }
        __syncthreads();
        // Dm[(a1 + P a2)][(b1 + P b2)] = sum_q2 V[q2,a2] V[q2,b2] T1[q2][a1 b1]
        for (int e = threadIdx.x; e < ncell * PP * PP; e += blockDim.x) {
            const int ci = e / (PP * PP), r = e - ci * PP * PP;
            const int ab2 = r / PP, ab1 = r % PP;
            const int a2 = ab2 / P, b2 = ab2 % P, a1 = ab1 / P, b1 = ab1 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += V[j * P + a2] * V[j * P + b2] * T1[ci * sT1 + j * PP + ab1];
            Dm[ci * n * n + (a1 + P * a2) * n + (b1 + P * b2)] = s;
        }
        __syncthreads();
    } else {
        // T1[q3][q2][a1 b1] = sum_q1 omega[q3][q2][q1] V[q1,a1] V[q1,b1]
        for (int e = threadIdx.x; e < ncell * q * q * PP; e += blockDim.x) {
            const int ci = e / (q * q * PP), r = e - ci * q * q * PP;
            const int q32 = r / PP, ab = r % PP, a1 = ab / P, b1 = ab % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j)
                s += vq[ci * S + q32 * q + j] * V[j * P + a1] * V[j * P + b1];
            T1[ci * sT1 + r] = s;
        }
        __syncthreads();
        // T2[q3][a2 b2][a1 b1] = sum_q2 V[q2,a2] V[q2,b2] T1[q3][q2][a1 b1]
        for (int e = threadIdx.x; e < ncell * q * PP * PP; e += blockDim.x) {
            const int ci = e / (q * PP * PP), r = e - ci * q * PP * PP;
            const int q3 = r / (PP * PP), rr = r % (PP * PP), ab2 = rr / PP, ab1 = rr % PP;
            const int a2 = ab2 / P, b2 = ab2 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j)
                s += V[j * P + a2] * V[j * P + b2] * T1[ci * sT1 + (q3 * q + j) * PP + ab1];
            T2[ci * sT2 + r] = s;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell * PP * PP * PP; e += blockDim.x) {
            const int ci = e / (PP * PP * PP), r = e - ci * PP * PP * PP;
            const int ab3 = r / (PP * PP), rr = r % (PP * PP), ab2 = rr / PP, ab1 = rr % PP;
            const int a3 = ab3 / P, b3 = ab3 % P, a2 = ab2 / P, b2 = ab2 % P, a1 = ab1 / P,
                      b1 = ab1 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j)
                s += V[j * P + a3] * V[j * P + b3] * T2[ci * sT2 + (j * PP + ab2) * PP + ab1];
            Dm[ci * n * n + (a1 + P * (a2 + P * a3)) * n + (b1 + P * (b2 + P * b3))] = s;
        }
        __syncthreads();
    }
    // -S_hat = D + beta M + C / alpha
    for (int e = threadIdx.x; e < ncell * n * n; e += blockDim.x) {
        const int ci = e / (n * n), r = e - ci * n * n;
        const int i = r / n, j = r % n;
        const int64_t cell = cell0 + ci;
        const double ia = 1.0 / a_of(cell);
        const double* C = Cmat + (int64_t)cclass[cell] * n * n;
        double v = Dm[ci * n * n + r] + ia * C[r];
        if (i == j) {
            double hk[3];
            const double J = cell_jac<double, D>(g, tb.h, cell, hk);
            int aa[3] = {i % P, (i / P) % P, i / (P * P)};
            double md = J;
            for (int k = 0; k < D; ++k) md *= tb.Mdiag[aa[k]];
            v += b_of(cell) * md;
        }
        Dm[ci * n * n + r] = v;
    }
    __syncthreads();
    double nrm_s = 0.0;   // ||-S_hat||_1 of this thread's cell (flagging threads)
    if (sflag) {
        block_norm1();
        nrm_s = threadIdx.x < ncell ? nrm[threadIdx.x] : 0.0;
        __syncthreads();
    }
    // in-place Gauss-Jordan inverse of each SPD block
    for (int k = 0; k < n; ++k) {
        for (int e = threadIdx.x; e < ncell * n; e += blockDim.x) {
            const int ci = e / n, i = e - ci * n;
            cr[ci * 2 * n + i] = Dm[ci * n * n + i * n + k];       // column k
            cr[ci * 2 * n + n + i] = Dm[ci * n * n + k * n + i];   // row k
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncell * n * n; e += blockDim.x) {
            const int ci = e / (n * n), r = e - ci * n * n;
            const int i = r / n, j = r % n;
            const double ip = 1.0 / cr[ci * 2 * n + k];
            const double rk = (j == k ? 1.0 : cr[ci * 2 * n + n + j]) * ip;
            double v;
            if (i == k)
                v = rk;
            else
                v = (j == k ? 0.0 : Dm[ci * n * n + r]) - cr[ci * 2 * n + i] * rk;
            Dm[ci * n * n + r] = v;
        }
        __syncthreads();
    }
    // FP32 solves: flag the cells whose 1-norm condition number exceeds
    // kFp32CondLimit (a non-finite one included); their FP64 inverse is kept
    // for the FP32 apply.  Without an FP64 linearisation (omega64 null) only
    // the flagged cells' inverses are written to sinv64.
    if (sflag) {
        block_norm1();
        if (threadIdx.x < ncell) {
            const int ci = threadIdx.x;
            const int f = !(nrm_s * nrm[ci] <= kFp32CondLimit);
            nrm[ci] = f ? 1.0 : 0.0;
            if (live(cell0 + ci)) sflag[cell0 + ci] = f;
        }
        __syncthreads();
    }
    const int64_t nt = psi_block_size(n, packed);
    for (int e = threadIdx.x; e < ncell * n * n; e += blockDim.x) {
        const int ci = e / (n * n), r = e - ci * n * n;
        // symmetrise (the exact inverse is symmetric)
        const int i = r / n, j = r % n;
        if (packed && j < i) continue;   // packed: the upper triangle, row by row
        const double v = 0.5 * (Dm[ci * n * n + i * n + j] + Dm[ci * n * n + j * n + i]);
        const int64_t off = (cell0 + ci) * nt +
                            (packed ? (int64_t)i * n - (int64_t)i * (i - 1) / 2 + (j - i) : r);
        if (!live(cell0 + ci)) continue;
        if (sinv64 && (!sflag || omega64 || nrm[ci] != 0.0)) sinv64[off] = v;
        if (sinv32) sinv32[off] = (float)v;
    }
    (void)per;
}

// ---------------------------------------------------------------------------
// The same setup for blocks too large for LDS (high P^d): one cell per block,
// -S_hat_K formed and inverted in place in its slot of s64 (global memory);
// LDS holds the weights, the contraction work space and the pivot row.
// T2: the d = 3 contraction keeps its q P^4 intermediate (else d_block3_direct).
template <int D, bool T2S>
__global__ __launch_bounds__(256) void k_setup_big(Geo g, PsiTabs<double> tb,
                                                   const double* __restrict__ psi, double alpha,
                                                   double beta, const double* __restrict__ Cmat,
                                                   const int* __restrict__ cclass,
                                                   double* __restrict__ omega64,
                                                   float* __restrict__ omega32,
                                                   double* __restrict__ s64,
                                                   float* __restrict__ s32) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int n = g.Pd, q = g.q, P = g.P, Qd = g.Qd, S = g.S;
    const int sT1 = (D == 1) ? 1 : ((D == 2) ? q * P * P : q * q * P * P);
    const int sT2 = (D == 3 && T2S) ? q * P * P * P * P : 1;
    const int64_t cell = blockIdx.x;
    double* bA = sm;
    double* bB = sm + S;
    double* T1 = sm + 2 * S;
    double* T2 = T1 + sT1;
    double* cr = T2 + sT2;
    double* Dm = s64 + cell * (int64_t)n * n;
    for (int a = threadIdx.x; a < n; a += blockDim.x) bA[a] = psi[cell * n + a];
    __syncthreads();
    double* vq = contract_all<double, D>(bA, bB, S, 1, P, q, tb.Vpsi, P, false);
    double hk[3];
    const double J = cell_jac<double, D>(g, tb.h, cell, hk);
    for (int j = threadIdx.x; j < Qd; j += blockDim.x) {
        int jj[3] = {j % q, (j / q) % q, j / (q * q)};
        double wq = J;
        for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
        const double arg = -vq[j];
        const double om = wq * exp(arg < 700.0 ? arg : 700.0);
        vq[j] = om;
        if (omega64) omega64[cell * Qd + j] = om;
        if (omega32) omega32[cell * Qd + j] = (float)om;
    }
    __syncthreads();
    if (D == 3 && !T2S)
        d_block3_direct(vq, tb.Vpsi, P, q, T1, Dm, n);
    else
        d_block<D>(vq, tb.Vpsi, P, q, T1, T2, Dm, n);
    // + beta M_K + C_K / alpha
    const double ia = 1.0 / alpha;
    const double* C = Cmat + (int64_t)cclass[cell] * n * n;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = Dm[e] + ia * C[e];
        if (i == j) {
            int aa[3] = {i % P, (i / P) % P, i / (P * P)};
            double md = J;
            for (int k = 0; k < D; ++k) md *= tb.Mdiag[aa[k]];
            v += beta * md;
        }
        Dm[e] = v;
    }
    __syncthreads();
    gauss_jordan_spd(Dm, n, cr);
    // symmetrise: the thread of (i, j), j >= i, owns both mirror entries
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        if (j < i) continue;
        const double v = 0.5 * (Dm[(int64_t)i * n + j] + Dm[(int64_t)j * n + i]);
        Dm[(int64_t)i * n + j] = v;
        Dm[(int64_t)j * n + i] = v;
        if (s32) {
            s32[cell * (int64_t)n * n + (int64_t)i * n + j] = (float)v;
            s32[cell * (int64_t)n * n + (int64_t)j * n + i] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// psi-block of the preconditioner: z_psi = (-S_hat_K)^{-1} r_psi per cell.
// A block copies the contiguous inverse blocks of cpb cells into LDS with
// coalesced loads, then one thread per (cell, row) forms the row product
// (the blocks are symmetric, so row i is read as column i: conflict-free).
// Partial dot <z, r> fused.
// fixed-order sum of np partials, identical in every block (valid in all threads)
__device__ inline double reduce_partials(const double* __restrict__ p, int np, double* red,
                                         double* bcast) {
    // eight loads in flight per thread (a loop of single loads waits one L2
    // round trip per element); the eight sums are combined in a fixed order
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int bd = (int)blockDim.x;
    int i = (int)threadIdx.x;
    for (; i + 7 * bd < np; i += 8 * bd) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[i + u * bd];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += v[u];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)   // fewer than eight left per thread
        if (i + u * bd < np) a[u] += p[i + u * bd];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = block_sum(s, red);
    if (threadIdx.x == 0) *bcast = s;
    __syncthreads();
    return *bcast;
}

// the next Lanczos vector formed where it is read: vhat = Gq - dl vcur - gm vprev
// (element i), optionally stored to out[i] by the one block that reads it
template <typename T>
struct VhatSrc {
    const T* Gq;
    const T* vcur;
    const T* vprev;
    T* out;
    T dl, gm;
    __device__ inline T at(int64_t i) const { return Gq[i] - dl * vcur[i] - gm * vprev[i]; }
};

template <typename T, bool VH = false, bool PK = false>
__device__ inline void prec_psi_body(int bid, int nblk, int64_t n_cells, int n, int cpb,
                                     const T* __restrict__ sinv, const T* __restrict__ r,
                                     T* __restrict__ z, double* __restrict__ partial,
                                     const int* __restrict__ done, T* Sb, double* red,
                                     const VhatSrc<T>* vs = nullptr, int64_t voff = 0,
                                     const double* __restrict__ s64h = nullptr,
                                     const int* __restrict__ flg = nullptr) {
    if (done && *done) return;
    const int nn = (int)psi_block_size(n, PK);   // values per block
    T* Rb = Sb + cpb * nn;
    double part = 0.0;
    const int64_t ngroups = (n_cells + cpb - 1) / cpb;
    for (int64_t grp = bid; grp < ngroups; grp += nblk) {
        const int64_t cell0 = grp * cpb;
        const int nc = (int)min((int64_t)cpb, n_cells - cell0);
        const T* src = sinv + cell0 * (int64_t)nn;
        const int tot = nc * nn;
        int e = threadIdx.x;
        for (; e + 3 * 256 < tot; e += 4 * 256) {
            const T v0 = src[e], v1 = src[e + 256], v2 = src[e + 512], v3 = src[e + 768];
            Sb[e] = v0;
            Sb[e + 256] = v1;
            Sb[e + 512] = v2;
            Sb[e + 768] = v3;
        }
        for (; e < tot; e += 256) Sb[e] = src[e];
        for (int i = threadIdx.x; i < nc * n; i += 256) {
            if (VH) {
                const int64_t gi = voff + cell0 * n + i;
                const T v = vs->at(gi);
                vs->out[gi] = v;
                Rb[i] = v;
            } else {
                Rb[i] = r[cell0 * n + i];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nc * n; i += 256) {
            const int ci = i / n, row = i - ci * n;
            const T* rr = Rb + ci * n;
            // z_row = sum_j S[j][row] r_j, j ascending.  Packed (upper triangle
            // row by row): S[j][row] sits at tri(j) + row - j for j < row, where
            // tri(j) = j n - j (j - 1) / 2 starts row j, and at tri(row) + j - row
            // after; the same values in the same order as the full block
            if (flg && flg[cell0 + ci]) {
                // a block too ill-conditioned for an FP32 product: its FP64
                // inverse with FP64 sums (the dot from the FP64 product)
                const double* S = s64h + (cell0 + ci) * (int64_t)nn;
                double acc = 0.0;
                if (PK) {
                    const int trow = row * n - row * (row - 1) / 2;
                    int tj = 0;   // tri(j)
                    for (int j = 0; j < n; ++j) {
                        acc += S[j < row ? tj + row - j : trow + j - row] * (double)rr[j];
                        tj += n - j;
                    }
                } else {
                    for (int j = 0; j < n; ++j) acc += S[(int64_t)j * n + row] * (double)rr[j];
                }
                z[cell0 * n + i] = (T)acc;
                part += acc * (double)rr[row];
                continue;
            }
            const T* S = Sb + ci * nn;
            T acc = 0;
            if (PK) {
                // one loop of n steps for every thread (no per-row trip counts)
                const int trow = row * n - row * (row - 1) / 2;
                int tj = 0;   // tri(j)
                for (int j = 0; j < n; ++j) {
                    acc += S[j < row ? tj + row - j : trow + j - row] * rr[j];
                    tj += n - j;
                }
            } else {
                for (int j = 0; j < n; ++j) acc += S[j * n + row] * rr[j];
            }
            z[cell0 * n + i] = acc;
            part += (double)acc * (double)rr[row];
        }
        __syncthreads();
    }
    if (partial) {
        double s2 = block_sum(part, red);
        if (threadIdx.x == 0) partial[bid] = s2;
    }
}


template <typename T, bool PK>
__global__ __launch_bounds__(256) void k_prec_psi(int64_t n_cells, int n, int cpb,
                                                  const T* __restrict__ sinv,
                                                  const T* __restrict__ r, T* __restrict__ z,
                                                  double* __restrict__ partial,
                                                  const int* __restrict__ done, PsiBatch bt,
                                                  PsiHi hi) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    const int64_t rb = blockIdx.y;
    prec_psi_body<T, false, PK>(blockIdx.x, gridDim.x, n_cells, n, cpb, sinv + rb * bt.sinv,
                                r + rb * bt.r, z + rb * bt.z,
                                partial ? partial + rb * bt.part : nullptr,
                                done ? done + rb * bt.done : nullptr,
                                reinterpret_cast<T*>(smem_raw), red, nullptr, 0,
                                hi.s64 ? hi.s64 + rb * bt.sinv : nullptr,
                                hi.flag ? hi.flag + rb * bt.flag : nullptr);
}

// ---------------------------------------------------------------------------
// Tensor-axis GEMMs of the fast-diagonalisation A-block inverse on the matrix
// cores: C_b = A_b (M x K) B_b (K x N), row-major, batch b = blockIdx.z.
// A block of 4 waves owns a (16 TS) x (16 TS) tile of C (TS = 1 or 2); the
// waves split K, each wave computes all TS x TS 16x16 sub-tiles over its part
// of K (v_mfma_*_16x16x4 operands: lane l supplies A[l%16][k] and B[k][l%16]
// for the k of its lane group; the 16x16 result sits 4 values per lane at
// positions the kernel reads off two index-valued MFMAs) and the four partial
// tiles are summed in LDS in a fixed order.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using V = v4d;
    static __device__ inline V op(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    using V = v4f;
    static __device__ inline V op(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// optional epilogues of a pass: divide by alpha (lam_k[row] + inner
// eigenvalues) (the eigen-space division of the fast diagonalisation) and/or
// accumulate <C, dotv> per block into partial[block]

// Summation order, the same for every tile shape: wave w takes the K slabs of
// four k0 = 4 w + 16 u (u = 0, 1, ..; the four lanes of a row read four
// consecutive k, so a row's loads share a cache line), MFMA k row kk adding
// k0 + kk (zero beyond K), even steps into one accumulator and odd steps into
// another;
// a 16x16 output element is (w0 + w1) + (w2 + w3) of the four waves' sums, and
// the fused dot's partials are one block_sum per 16x16 sub-tile.  So the tile
// shape never changes a bit of the result: it is a free (tuned) choice.
//
// One (16 TS)^2 tile (bx, by) of batch bz; the partial of the fused dot of
// 16x16 sub-tile (x, y) of the 16-grid goes to partial[(bz * gy + y) gx + x]
// (pstride 0) or partial[request * pstride + y gx + x].
template <typename T, int TS, bool VH = false>
__device__ inline void gemm_tile_body(int bx, int by, int bz, int M, int N, int K,
                                      const T* __restrict__ A, int64_t lda, int64_t sA,
                                      const T* __restrict__ B, int64_t ldb, int64_t sB,
                                      T* __restrict__ C, int64_t ldc, int64_t sC,
                                      const int* __restrict__ done, const GemmEpi<T>& ep,
                                      T* red, double* rsum, const VhatSrc<T>* vs = nullptr) {
    using V = typename Mfma<T>::V;
    // batched requests: batch bz belongs to request bz / bdiv
    const int64_t rq = ep.bdiv > 0 ? bz / ep.bdiv : 0;
    if (done) done += rq * ep.dstride;
    const double* eprm = ep.prm ? ep.prm + rq * ep.prmstride : nullptr;
    if (done && *done) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t b = bz;
    A += b * sA;
    B += b * sB;
    C += b * sC;
    const int i0 = by * 16 * TS, j0 = bx * 16 * TS;
    const int l16 = lane & 15, kk = lane >> 4;
    V acc[2][TS][TS];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int ta = 0; ta < TS; ++ta)
#pragma unroll
            for (int tb = 0; tb < TS; ++tb) acc[e][ta][tb] = V{0, 0, 0, 0};
    // the operands of twelve steps are loaded before their MFMAs, so K <= 192
    // costs one round trip (the row offsets of a lane are fixed, so every load
    // is the lane's base address plus a constant)
    int ar[TS], bc[TS];
    bool aok[TS], bok[TS];
#pragma unroll
    for (int t = 0; t < TS; ++t) {
        ar[t] = i0 + 16 * t + l16;
        bc[t] = j0 + 16 * t + l16;
        aok[t] = ar[t] < M;
        bok[t] = bc[t] < N;
    }
    for (int k0 = 4 * w; k0 < K; k0 += 16 * 12) {
        T a[12][TS], bb[12][TS];
#pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int k = k0 + 16 * u + kk;
            const bool kok = k < K;
#pragma unroll
            for (int t = 0; t < TS; ++t) {
                const int64_t gi = (int64_t)ar[t] * lda + k;
                if (VH) {
                    // A = vhat (batch 0, no stride): formed here; the blocks of
                    // the first tile column store it (each element once)
                    T v = (T)0;
                    if (kok && aok[t]) {
                        v = vs->at(gi);
                        if (bx == 0) vs->out[gi] = v;
                    }
                    a[u][t] = v;
                } else {
                    a[u][t] = (kok && aok[t]) ? A[gi] : (T)0;
                }
                bb[u][t] = (kok && bok[t]) ? B[(int64_t)k * ldb + bc[t]] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < 12; ++u)
#pragma unroll
            for (int ta = 0; ta < TS; ++ta)
#pragma unroll
                for (int tb = 0; tb < TS; ++tb)
                    acc[u & 1][ta][tb] = Mfma<T>::op(a[u][ta], bb[u][tb], acc[u & 1][ta][tb]);
    }
    // where each of the 4 result values of this lane sits in a 16x16 tile:
    // one MFMA with A[i][0] = i, B[0][j] = 1 gives D[i][j] = i, one with
    // A[i][0] = 1, B[0][j] = j gives D[i][j] = j (exact small integers)
    const V zero = {0, 0, 0, 0};
    const V rid = Mfma<T>::op(kk == 0 ? (T)l16 : (T)0, kk == 0 ? (T)1 : (T)0, zero);
    const V cid = Mfma<T>::op(kk == 0 ? (T)1 : (T)0, kk == 0 ? (T)l16 : (T)0, zero);
#pragma unroll
    for (int ta = 0; ta < TS; ++ta)
#pragma unroll
        for (int tb = 0; tb < TS; ++tb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ri = (int)rid[v] & 15, ci = (int)cid[v] & 15;
                red[((w * TS + ta) * TS + tb) * 256 + ri * 16 + ci] =
                    acc[0][ta][tb][v] + acc[1][ta][tb][v];
            }
    __syncthreads();
    const int t = threadIdx.x, r = t >> 4, c = t & 15;
    const int gx16 = (N + 15) >> 4, gy16 = (M + 15) >> 4;
    const int64_t pbase = ep.pstride ? rq * ep.pstride + (b - rq * ep.bdiv) * gx16 * gy16
                                     : b * gx16 * gy16;
#pragma unroll
    for (int ta = 0; ta < TS; ++ta)
#pragma unroll
        for (int tb = 0; tb < TS; ++tb) {
            const int sub = ta * TS + tb, st = TS * TS * 256;
            T s = (red[sub * 256 + t] + red[st + sub * 256 + t]) +
                  (red[2 * st + sub * 256 + t] + red[3 * st + sub * 256 + t]);
            const int row = i0 + 16 * ta + r, col = j0 + 16 * tb + c;
            const bool in = row < M && col < N;
            double part = 0.0;
            if (in) {
                if (ep.scale_mode) {
                    T lam;
                    if (ep.scale_mode == 1)
                        lam = ep.l0[col];
                    else if (ep.scale_mode == 2)
                        lam = ep.l1[row] + ep.l0[col];
                    else
                        lam = ep.l2[row] + ep.l0[col % ep.n0] + ep.l1[col / ep.n0];
                    s = s * (T)eprm[2] / lam;
                }
                C[(int64_t)row * ldc + col] = s;
                if (ep.dotv)
                    part = (double)s * (double)ep.dotv[b * sC + (int64_t)row * ldc + col];
            }
            // sub-tiles beyond the matrix are not part of the 16-grid
            if (ep.partial && i0 + 16 * ta < M && j0 + 16 * tb < N) {
                const double tot = block_sum(part, rsum);
                if (t == 0)
                    ep.partial[pbase + (int64_t)(by * TS + ta) * gx16 + bx * TS + tb] = tot;
            }
        }
}

template <typename T, int TS>
__global__ __launch_bounds__(256) void k_gemm_mfma(int M, int N, int K, const T* __restrict__ A,
                                                   int64_t lda, int64_t sA,
                                                   const T* __restrict__ B, int64_t ldb,
                                                   int64_t sB, T* __restrict__ C, int64_t ldc,
                                                   int64_t sC, const int* __restrict__ done,
                                                   GemmEpi<T> ep) {
    __shared__ T red[4 * TS * TS * 256];
    __shared__ double rsum[4];
    gemm_tile_body<T, TS>(blockIdx.x, blockIdx.y, blockIdx.z, M, N, K, A, lda, sA, B, ldb, sB, C,
                          ldc, sC, done, ep, red, rsum);
}

// The first fast-diagonalisation pass (one GEMM, batch 1) and the psi-block
// preconditioner in one launch: both read the same residual and are
// independent, so blocks [0, gx gy) take GEMM tiles and the remaining np
// blocks the psi-block cell groups.  Saves a dependent launch per iteration.
// As k_gemm_prec, with the MINRES step that forms the next Lanczos vector
// folded in: every block reduces the G-apply partials of <q, Gq> in the same
// fixed order (delta, stored by block 0), then the GEMM tiles and the
// psi-block cells read vhat = Gq - delta v_cur - gamma v_prev where they load
// the residual, and store it to vhat (each element by exactly one block).
template <typename T, int TS, bool PK>
__global__ __launch_bounds__(256) void k_vhat_gemm_prec(int M, int N, int K, const T* __restrict__ B,
                                                        int64_t ldb, T* __restrict__ C,
                                                        int64_t ldc, GemmEpi<T> ep, int gx,
                                                        int gy, int64_t n_cells, int n, int cpb,
                                                        const T* __restrict__ sinv,
                                                        T* __restrict__ z,
                                                        double* __restrict__ ppart, KState* st,
                                                        const double* __restrict__ gpart, int npg,
                                                        const T* Gq, const T* vcur,
                                                        const T* vprev, T* vhat, int64_t n_u,
                                                        PsiHi hi) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red[4 * TS * TS * 256];
    __shared__ double rsum[4];
    __shared__ double bc;
    if (st->done) return;
    const double delta = reduce_partials(gpart, npg, rsum, &bc);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->delta = delta;
    VhatSrc<T> vs{Gq, vcur, vprev, vhat, (T)delta, (T)st->gamma};
    const int ng = gx * gy;
    if ((int)blockIdx.x < ng) {
        const int bx = blockIdx.x % gx, by = blockIdx.x / gx;
        gemm_tile_body<T, TS, true>(bx, by, 0, M, N, K, nullptr, N, 0, B, ldb, 0, C, ldc, 0,
                                    nullptr, ep, red, rsum, &vs);
    } else {
        prec_psi_body<T, true, PK>(blockIdx.x - ng, gridDim.x - ng, n_cells, n, cpb, sinv, nullptr,
                               z, ppart, nullptr, reinterpret_cast<T*>(smem_raw), rsum, &vs, n_u,
                               hi.s64, hi.flag);
    }
}

template <typename T, int TS, bool PK>
__global__ __launch_bounds__(256) void k_gemm_prec(int M, int N, int K, const T* __restrict__ A,
                                                   int64_t lda, const T* __restrict__ B,
                                                   int64_t ldb, T* __restrict__ C, int64_t ldc,
                                                   const int* __restrict__ done, GemmEpi<T> ep,
                                                   int gx, int gy, int64_t n_cells, int n, int cpb,
                                                   const T* __restrict__ sinv,
                                                   const T* __restrict__ r, T* __restrict__ z,
                                                   double* __restrict__ ppart, int64_t sA,
                                                   int64_t sC, PsiBatch bt, PsiHi hi) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red[4 * TS * TS * 256];
    __shared__ double rsum[4];
    const int ng = gx * gy;
    const int64_t rb = blockIdx.y;   // request of a batched launch
    if ((int)blockIdx.x < ng) {
        const int bx = blockIdx.x % gx, by = blockIdx.x / gx;
        GemmEpi<T> e2 = ep;
        if (e2.prm) e2.prm += rb * e2.prmstride;
        gemm_tile_body<T, TS>(bx, by, 0, M, N, K, A + rb * sA, lda, 0, B, ldb, 0, C + rb * sC,
                              ldc, 0, done ? done + rb * bt.done : nullptr, e2, red, rsum);
    } else {
        prec_psi_body<T, false, PK>(blockIdx.x - ng, gridDim.x - ng, n_cells, n, cpb,
                                    sinv + rb * bt.sinv,
                         r + rb * bt.r, z + rb * bt.z, ppart ? ppart + rb * bt.part : nullptr,
                         done ? done + rb * bt.done : nullptr, reinterpret_cast<T*>(smem_raw),
                         rsum, nullptr, 0, hi.s64 ? hi.s64 + rb * bt.sinv : nullptr,
                         hi.flag ? hi.flag + rb * bt.flag : nullptr);
    }
}

// ---------------------------------------------------------------------------
// Preconditioned MINRES for the symmetric indefinite G with an SPD
// preconditioner M (Lanczos on M^{-1} G in the M-inner product, QR of the
// tridiagonal by Givens rotations).  The scalar recurrences are folded into
// the vector kernels: every block reduces the partial sums of the preceding
// dot product itself, in one fixed order, so all blocks hold bit-identical
// scalars; block 0 stores them.  The state is double-buffered by iteration
// parity (iteration j reads st[j&1] and writes st[(j+1)&1]), so no block
// reads a field that another block of the same kernel writes.  Once a state
// is marked done every later kernel of the loop returns at once.


// start: gamma1 = sqrt(<z1, b>), v_cur = b/gamma1, q = z1/gamma1, w = v_prev = x = 0
template <typename T>
__global__ __launch_bounds__(256) void k_kr_start(int64_t n, KState* st0, const double* partial,
                                                  int np, double rtol, int maxit, const T* b,
                                                  const T* z, T* vcur, T* vprev, T* q, T* wprev,
                                                  T* wcur, T* x, VecBatch bt) {
    __shared__ double red[4];
    __shared__ double bc;
    if (bt.mask && !bt.mask[blockIdx.y]) return;   // a request not starting now
    {
        const int64_t rb = blockIdx.y, o = rb * bt.v;
        st0 += rb;
        partial += rb * bt.part;
        b += o;
        z += o;
        vcur += o;
        vprev += o;
        q += o;
        wprev += o;
        wcur += o;
        x += o;
    }
    const double g2 = reduce_partials(partial, np, red, &bc);
    const double g1 = sqrt(g2 > 0.0 ? g2 : 0.0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        KState s;
        s.gamma1 = g1;
        s.gamma = g1;
        s.delta = 0.0;
        s.c = s.c_prev = 1.0;
        s.s = s.s_prev = 0.0;
        s.eta = g1;
        s.rtol = rtol;
        s.iters = 0;
        s.max_iters = maxit;
        s.breakdown = 0;
        s.done = (g1 > 0.0 && g1 == g1) ? 0 : 1;
        *st0 = s;
    }
    const double ig = g1 > 0.0 ? 1.0 / g1 : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        vcur[i] = (T)((double)b[i] * ig);
        q[i] = (T)((double)z[i] * ig);
        vprev[i] = 0;
        wprev[i] = 0;
        wcur[i] = 0;
        x[i] = 0;
    }
}

// delta = <G q, q>;  vhat = G q - delta v_cur - gamma v_prev   (over v_prev)
template <typename T>
__global__ __launch_bounds__(256) void k_kr_vhat(int64_t n, KState* st, const double* partial,
                                                 int np, const T* Gq, const T* vcur,
                                                 const T* vprev, T* vhat, VecBatch bt) {
    __shared__ double red[4];
    __shared__ double bc;
    {
        const int64_t rb = blockIdx.y, o = rb * bt.v;
        st += rb;
        partial += rb * bt.part;
        Gq += o;
        vcur += o;
        vprev += o;
        vhat += o;
    }
    if (st->done) return;
    const double delta = reduce_partials(partial, np, red, &bc);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->delta = delta;
    const T dl = (T)delta, gm = (T)st->gamma;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        vhat[i] = Gq[i] - dl * vcur[i] - gm * vprev[i];
}

// gamma_new = sqrt(<z, vhat>), Givens rotation, then
// w_new = (q - a3 w_prev - a2 w_cur)/a1 (over w_prev), x += c_new eta w_new,
// v_prev <- vhat / gamma_new, q <- z / gamma_new; the new state goes to st_out
template <typename T>
__global__ __launch_bounds__(256) void k_kr_update(int64_t n, const KState* st_in, KState* st_out,
                                                   const double* partial, int np, T* q, T* wprev,
                                                   const T* wcur, T* x, T* vprev, const T* vhat,
                                                   const T* z, VecBatch bt) {
    __shared__ double red[4];
    __shared__ double bc;
    __shared__ double sc[6];   // a1, a2, a3, step, 1/gamma_new, skip
    {
        const int64_t rb = blockIdx.y, o = rb * bt.v;
        st_in += rb;
        st_out += rb;
        partial += rb * bt.part;
        q += o;
        wprev += o;
        wcur += o;
        x += o;
        vprev += o;
        vhat += o;
        z += o;
    }
    if (st_in->done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *st_out = *st_in;
        return;
    }
    const double g2 = reduce_partials(partial, np, red, &bc);
    if (threadIdx.x == 0) {
        KState s = *st_in;
        const double gnew = sqrt(g2 > 0.0 ? g2 : 0.0);
        const double delta = s.delta, gcur = s.gamma;
        const double a0 = s.c * delta - s.c_prev * s.s * gcur;
        const double a1 = sqrt(a0 * a0 + gnew * gnew);
        const double a2 = s.s * delta + s.c_prev * s.c * gcur;
        const double a3 = s.s_prev * gcur;
        if (a1 == 0.0 || !(a1 == a1)) {   // breakdown or NaN: stop without an update
            s.done = 1;
            s.breakdown = 1;
            sc[5] = 1.0;
        } else {
            s.c_prev = s.c;
            s.s_prev = s.s;
            s.c = a0 / a1;
            s.s = gnew / a1;
            sc[0] = a1;
            sc[1] = a2;
            sc[2] = a3;
            sc[3] = s.c * s.eta;
            sc[4] = gnew > 0.0 ? 1.0 / gnew : 0.0;
            sc[5] = 0.0;
            s.eta = -s.s * s.eta;
            s.gamma = gnew;
            s.iters += 1;
            if (fabs(s.eta) <= s.rtol * s.gamma1 || s.iters >= s.max_iters || gnew == 0.0)
                s.done = 1;
            // a negative preconditioned norm of the next Lanczos vector means the
            // preconditioner lost definiteness in the working precision: stop and
            // report it rather than take it for convergence
            if (g2 < 0.0) s.breakdown = 1;
        }
        if (blockIdx.x == 0) *st_out = s;
    }
    __syncthreads();
    if (sc[5] != 0.0) return;
    const double ia1 = 1.0 / sc[0];
    const T a2 = (T)sc[1], a3 = (T)sc[2], step = (T)sc[3];
    const double ig = sc[4];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T wn = (T)((double)(q[i] - a3 * wprev[i] - a2 * wcur[i]) * ia1);
        wprev[i] = wn;
        x[i] += step * wn;
        vprev[i] = (T)((double)vhat[i] * ig);
        q[i] = (T)((double)z[i] * ig);
    }
}

// ---------------------------------------------------------------------------
// partial[b] = sum over block b's grid-stride slice of a_i b_i (FP64 accumulation)
template <typename T>
__global__ __launch_bounds__(256) void k_dot(int64_t n, const T* __restrict__ a,
                                             const T* __restrict__ b, double* __restrict__ partial,
                                             const int* __restrict__ done) {
    __shared__ double red[4];
    if (done && *done) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += (double)a[i] * (double)b[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// small vector kernels
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(int64_t n, const TI* a, TO* b, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (TO)((double)a[i] * scale);
}

// y = x + t * d (FP64 x, y; d of type T)
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_to(int64_t n, const double* x, double t,
                                                 const T* d, double* y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + t * (double)d[i];
}

// lam = (psi_prev - psi) / alpha
__global__ __launch_bounds__(256) void k_lambda(int64_t n, const double* psi_prev,
                                                const double* psi, double alpha, double* lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) lam[i] = (psi_prev[i] - psi[i]) / alpha;
}

// ---------------------------------------------------------------------------
// L2 norms of u_h - v_h and u_h by Gauss-Legendre (exact for degree 2p):
// partial[2 b] = sum W (u - v)^2, partial[2 b + 1] = sum W u^2
template <int D>
__global__ __launch_bounds__(256) void k_l2(Geo g, PsiTabs<double> tb, int cpb,
                                            const double* __restrict__ u,
                                            const double* __restrict__ v,
                                            double* __restrict__ partial, VecBatch bt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    u += (int64_t)blockIdx.y * bt.v;
    v += (int64_t)blockIdx.y * bt.v;
    partial += (int64_t)blockIdx.y * bt.part;
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int S = g.S;
    double* a = sm;
    double* b = sm + cpb * S;
    double* c = sm + 2 * cpb * S;
    double* d2 = sm + 3 * cpb * S;
    const int64_t cell0 = (int64_t)blockIdx.x * cpb;
    const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
    const int L = g.p + 1, q = g.q;
    gather_u<double, D>(g, u, a, S, cell0, ncell);
    gather_u<double, D>(g, v, c, S, cell0, ncell);
    __syncthreads();
    double* uq = contract_all<double, D>(a, b, S, ncell, L, q, tb.Vu, L, false);
    double* vq = contract_all<double, D>(c, d2, S, ncell, L, q, tb.Vu, L, false);
    double s1 = 0.0, s2 = 0.0;
    for (int e = threadIdx.x; e < ncell * g.Qd; e += blockDim.x) {
        const int ci = e / g.Qd, j = e - ci * g.Qd;
        double hk[3];
        const double J = cell_jac<double, D>(g, tb.h, cell0 + ci, hk);
        int jj[3] = {j % q, (j / q) % q, j / (q * q)};
        double wq = J;
        for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
        const double du = uq[ci * S + j] - vq[ci * S + j];
        s1 += wq * du * du;
        s2 += wq * uq[ci * S + j] * uq[ci * S + j];
    }
    double t1 = block_sum(s1, red);
    __syncthreads();
    double t2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = t1;
        partial[2 * blockIdx.x + 1] = t2;
    }
}

// ---------------------------------------------------------------------------
// explicit instantiation through launcher functions (see kernels.h)
static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_u_side(const Geo& g, const URows<T>* r, T alpha, const T* xu, const T* xb,
                   const T* xb_prev, const double* F, T* yu, double* partial, const int* done,
                   int mode, hipStream_t s, const double* prm) {
    dim3 grid((unsigned)std::min<int64_t>((g.n_u + 127) / 128, 1024)), blk(128);
#define HPG_U(DD, MM)                                                                       \
    hipLaunchKernelGGL((k_u_side<T, DD, MM>), grid, blk, 0, s, g, r[0], r[1], r[2], alpha, \
                       xu, xb, xb_prev, F, yu, partial, done, prm)
    if (mode == MODE_APPLY) {
        if (g.d == 1) HPG_U(1, MODE_APPLY);
        else if (g.d == 2) HPG_U(2, MODE_APPLY);
        else HPG_U(3, MODE_APPLY);
    } else {
        if (g.d == 1) HPG_U(1, MODE_RES);
        else if (g.d == 2) HPG_U(2, MODE_RES);
        else HPG_U(3, MODE_RES);
    }
#undef HPG_U
}

template <typename T>
void launch_psi_side(const Geo& g, const PsiTabs<T>& tb, int cpb, T beta, const T* xu,
                     const T* xpsi, const T* omega, const double* Phi, T* ypsi, double* partial,
                     const int* done, int mode, hipStream_t s, const double* prm) {
    dim3 grid((unsigned)std::min<int64_t>((g.n_cells + cpb - 1) / cpb, 1024)), blk(256);
    size_t shm = (size_t)5 * cpb * g.S * sizeof(T);
#define HPG_P(DD, MM)                                                                      \
    hipLaunchKernelGGL((k_psi_side<T, DD, MM>), grid, blk, shm, s, g, tb, cpb, beta, xu, \
                       xpsi, omega, Phi, ypsi, partial, done, prm)
    if (mode == MODE_APPLY) {
        if (g.d == 1) HPG_P(1, MODE_APPLY);
        else if (g.d == 2) HPG_P(2, MODE_APPLY);
        else HPG_P(3, MODE_APPLY);
    } else {
        if (g.d == 1) HPG_P(1, MODE_RES);
        else if (g.d == 2) HPG_P(2, MODE_RES);
        else HPG_P(3, MODE_RES);
    }
#undef HPG_P
}

size_t setup_smem_per_cell(const Geo& g) {
    const int n = g.Pd, q = g.q, P = g.P;
    const int sT1 = (g.d == 1) ? 1 : ((g.d == 2) ? q * P * P : q * q * P * P);
    const int sT2 = (g.d == 3) ? q * P * P * P * P : 1;
    return (size_t)(2 * g.S + sT1 + sT2 + n * n + 2 * n + 1) * sizeof(double);
}

size_t setup_big_smem(const Geo& g, bool t2) {
    const int n = g.Pd, q = g.q, P = g.P;
    const int sT1 = (g.d == 1) ? 1 : ((g.d == 2) ? q * P * P : q * q * P * P);
    const int sT2 = (g.d == 3 && t2) ? q * P * P * P * P : 1;
    return (size_t)(2 * g.S + sT1 + sT2 + 2 * n) * sizeof(double);
}

void launch_setup(const Geo& g, const PsiTabs<double>& tb, int cpb, int big, const double* psi,
                  double alpha, double beta, const double* C, const int* cclass, double* om64,
                  float* om32, double* s64, float* s32, hipStream_t s, const double* prm_req,
                  const int* mask, int64_t cpr, int* sflag, int packed) {
    if (big) {
        const bool t2 = big == SETUP_HBM_T2;
        const size_t shm = setup_big_smem(g, t2);
#define HPG_SB(DD, TT)                                                                      \
    hipLaunchKernelGGL((k_setup_big<DD, TT>), dim3((unsigned)g.n_cells), dim3(256), shm, s, \
                       g, tb, psi, alpha, beta, C, cclass, om64, om32, s64, s32)
        if (g.d == 1) HPG_SB(1, true);
        else if (g.d == 2) HPG_SB(2, true);
        else if (t2) HPG_SB(3, true);
        else HPG_SB(3, false);
#undef HPG_SB
        return;
    }
    dim3 grid(nblk(g.n_cells, cpb)), blk(256);
    size_t shm = setup_smem_per_cell(g) * cpb;
#define HPG_S(DD)                                                                        \
    hipLaunchKernelGGL((k_setup<DD>), grid, blk, shm, s, g, tb, cpb, psi, alpha, beta, C, \
                       cclass, om64, om32, s64, s32, prm_req, mask, cpr, sflag, packed)
    if (g.d == 1) HPG_S(1);
    else if (g.d == 2) HPG_S(2);
    else HPG_S(3);
#undef HPG_S
}

template <typename T>
void launch_prec_psi(int64_t n_cells, int n, int cpb, const T* sinv, const T* r, T* z,
                     double* partial, const int* done, hipStream_t s, const PsiBatch& bt,
                     const PsiHi& hi) {
    const size_t shm = (size_t)cpb * (psi_block_size(n, hi.packed) + n) * sizeof(T);
    const unsigned grid = (unsigned)std::min<int64_t>((n_cells + cpb - 1) / cpb, 1024);
    if (hi.packed)
        hipLaunchKernelGGL((k_prec_psi<T, true>), dim3(grid, (unsigned)bt.nb), dim3(256), shm, s,
                           n_cells, n, cpb, sinv, r, z, partial, done, bt, hi);
    else
        hipLaunchKernelGGL((k_prec_psi<T, false>), dim3(grid, (unsigned)bt.nb), dim3(256), shm, s,
                           n_cells, n, cpb, sinv, r, z, partial, done, bt, hi);
}

template <typename T>
void launch_gemm(int M, int N, int K, const T* A, int64_t lda, int64_t sA, const T* B,
                 int64_t ldb, int64_t sB, T* C, int64_t ldc, int64_t sC, int batch,
                 const int* done, const GemmEpi<T>& ep, hipStream_t s, const KernelEvents* ev) {
    const int e = 16 * gemm_ts(ep);
    dim3 grid((N + e - 1) / e, (M + e - 1) / e, batch);
#define HPG_G(TS)                                                                               \
    do {                                                                                        \
        if (ev && ev->start)                                                                    \
            hipExtLaunchKernelGGL((k_gemm_mfma<T, TS>), grid, dim3(256), 0, s, ev->start,        \
                                  ev->stop, 0, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, done, \
                                  ep);                                                          \
        else                                                                                    \
            hipLaunchKernelGGL((k_gemm_mfma<T, TS>), grid, dim3(256), 0, s, M, N, K, A, lda, sA, \
                               B, ldb, sB, C, ldc, sC, done, ep);                               \
    } while (0)
    if (e == 32) HPG_G(2);
    else HPG_G(1);
#undef HPG_G
}

template <typename T>
void launch_gemm_prec(int M, int N, int K, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                      int64_t ldc, const int* done, const GemmEpi<T>& ep, int64_t n_cells, int n,
                      int cpb, const T* sinv, const T* r, T* z, double* ppart, hipStream_t s,
                      int64_t sA, int64_t sC, const PsiBatch& bt, const PsiHi& hi) {
    const int e = 16 * gemm_ts(ep);
    const int gx = (N + e - 1) / e, gy = (M + e - 1) / e;
    const int np = (int)std::min<int64_t>((n_cells + cpb - 1) / cpb, 1024);
    const size_t shm = (size_t)cpb * (psi_block_size(n, hi.packed) + n) * sizeof(T);
#define HPG_G(TS, PK)                                                                             \
    hipLaunchKernelGGL((k_gemm_prec<T, TS, PK>), dim3(gx * gy + np, (unsigned)bt.nb), dim3(256),   \
                       shm, s, M, N, K, A, lda, B, ldb, C, ldc, done, ep, gx, gy, n_cells, n, cpb,  \
                       sinv, r, z, ppart, sA, sC, bt, hi)
    if (e == 32 && hi.packed) HPG_G(2, true);
    else if (e == 32) HPG_G(2, false);
    else if (hi.packed) HPG_G(1, true);
    else HPG_G(1, false);
#undef HPG_G
}

template <typename T>
void launch_vhat_gemm_prec(int M, int N, const T* B, T* C, const GemmEpi<T>& ep, int64_t n_cells,
                           int n, int cpb, const T* sinv, T* z, double* ppart, KState* st,
                           const double* gpart, int npg, const T* Gq, const T* vcur,
                           const T* vprev, T* vhat, int64_t n_u, hipStream_t s,
                           const PsiHi& hi) {
    const int e = 16 * gemm_ts(ep);
    const int gx = (N + e - 1) / e, gy = (M + e - 1) / e;
    const int np = (int)std::min<int64_t>((n_cells + cpb - 1) / cpb, 1024);
    const size_t shm = (size_t)cpb * (psi_block_size(n, hi.packed) + n) * sizeof(T);
#define HPG_G(TS, PK)                                                                             \
    hipLaunchKernelGGL((k_vhat_gemm_prec<T, TS, PK>), dim3(gx * gy + np), dim3(256), shm, s, M, N, \
                       N, B, N, C, N, ep, gx, gy, n_cells, n, cpb, sinv, z, ppart, st, gpart, npg,  \
                       Gq, vcur, vprev, vhat, n_u, hi)
    if (e == 32 && hi.packed) HPG_G(2, true);
    else if (e == 32) HPG_G(2, false);
    else if (hi.packed) HPG_G(1, true);
    else HPG_G(1, false);
#undef HPG_G
}

template <typename T>
void launch_dot(int64_t n, const T* a, const T* b, double* partial, int nblocks, const int* done,
                hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(nblocks), dim3(256), 0, s, n, a, b, partial, done);
}

static inline unsigned vec_grid(int64_t n) {
    return (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
}
template <typename T>
void launch_kr_start(int64_t n, KState* st0, const double* partial, int np, double rtol,
                     int maxit, const T* b, const T* z, T* vcur, T* vprev, T* q, T* wprev,
                     T* wcur, T* x, hipStream_t s, const VecBatch& bt) {
    hipLaunchKernelGGL((k_kr_start<T>), dim3(vec_grid(n), (unsigned)bt.nb), dim3(256), 0, s, n,
                       st0, partial, np, rtol, maxit, b, z, vcur, vprev, q, wprev, wcur, x, bt);
}
template <typename T>
void launch_kr_vhat(int64_t n, KState* st, const double* partial, int np, const T* Gq,
                    const T* vcur, const T* vprev, T* vhat, hipStream_t s, const VecBatch& bt) {
    hipLaunchKernelGGL((k_kr_vhat<T>), dim3(vec_grid(n), (unsigned)bt.nb), dim3(256), 0, s, n, st,
                       partial, np, Gq, vcur, vprev, vhat, bt);
}
template <typename T>
void launch_kr_update(int64_t n, const KState* st_in, KState* st_out, const double* partial,
                      int np, T* q, T* wprev, const T* wcur, T* x, T* vprev, const T* vhat,
                      const T* z, hipStream_t s, const VecBatch& bt) {
    hipLaunchKernelGGL((k_kr_update<T>), dim3(vec_grid(n), (unsigned)bt.nb), dim3(256), 0, s, n,
                       st_in, st_out, partial, np, q, wprev, wcur, x, vprev, vhat, z, bt);
}
template <typename TI, typename TO>
void launch_convert(int64_t n, const TI* a, TO* b, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3(nblk(n)), dim3(256), 0, s, n, a, b, scale);
}
template <typename T>
void launch_axpy_to(int64_t n, const double* x, double t, const T* d, double* y, hipStream_t s) {
    hipLaunchKernelGGL((k_axpy_to<T>), dim3(nblk(n)), dim3(256), 0, s, n, x, t, d, y);
}
void launch_lambda(int64_t n, const double* psi_prev, const double* psi, double alpha,
                   double* lam, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda, dim3(nblk(n)), dim3(256), 0, s, n, psi_prev, psi, alpha, lam);
}
void launch_l2(const Geo& g, const PsiTabs<double>& tb, int cpb, const double* u, const double* v,
               double* partial, hipStream_t s, const VecBatch& bt) {
    dim3 grid(nblk(g.n_cells, cpb), (unsigned)bt.nb);
    size_t shm = (size_t)4 * cpb * g.S * sizeof(double);
    if (g.d == 1)
        hipLaunchKernelGGL((k_l2<1>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial, bt);
    else if (g.d == 2)
        hipLaunchKernelGGL((k_l2<2>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial, bt);
    else
        hipLaunchKernelGGL((k_l2<3>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial, bt);
}

#define HPG_INST(T)                                                                              \
    template void launch_u_side<T>(const Geo&, const URows<T>*, T, const T*, const T*, const T*, \
                                   const double*, T*, double*, const int*, int, hipStream_t,    \
                                   const double*);                                               \
    template void launch_psi_side<T>(const Geo&, const PsiTabs<T>&, int, T, const T*, const T*, \
                                     const T*, const double*, T*, double*, const int*, int,     \
                                     hipStream_t, const double*);                                \
    template void launch_prec_psi<T>(int64_t, int, int, const T*, const T*, T*, double*,         \
                                     const int*, hipStream_t, const PsiBatch&, const PsiHi&);    \
    template void launch_gemm<T>(int, int, int, const T*, int64_t, int64_t, const T*, int64_t,    \
                                 int64_t, T*, int64_t, int64_t, int, const int*,                 \
                                 const GemmEpi<T>&, hipStream_t, const KernelEvents*);           \
    template void launch_gemm_prec<T>(int, int, int, const T*, int64_t, const T*, int64_t, T*,   \
                                      int64_t, const int*, const GemmEpi<T>&, int64_t, int, int,  \
                                      const T*, const T*, T*, double*, hipStream_t, int64_t,     \
                                      int64_t, const PsiBatch&, const PsiHi&);                   \
    template void launch_kr_start<T>(int64_t, KState*, const double*, int, double, int, const T*, \
                                     const T*, T*, T*, T*, T*, T*, T*, hipStream_t,              \
                                     const VecBatch&);                                           \
    template void launch_kr_vhat<T>(int64_t, KState*, const double*, int, const T*, const T*,   \
                                    const T*, T*, hipStream_t, const VecBatch&);                 \
    template void launch_kr_update<T>(int64_t, const KState*, KState*, const double*, int, T*, T*, \
                                      const T*, T*, T*, const T*, const T*, hipStream_t,         \
                                      const VecBatch&);                                          \
    template void launch_vhat_gemm_prec<T>(int, int, const T*, T*, const GemmEpi<T>&, int64_t,   \
                                           int, int, const T*, T*, double*, KState*,             \
                                           const double*, int, const T*, const T*, const T*, T*, \
                                           int64_t, hipStream_t, const PsiHi&);                  \
    template void launch_axpy_to<T>(int64_t, const double*, double, const T*, double*,          \
                                    hipStream_t);                                                \
    template void launch_dot<T>(int64_t, const T*, const T*, double*, int, const int*, hipStream_t);
HPG_INST(double)
HPG_INST(float)
template void launch_convert<double, float>(int64_t, const double*, float*, double, hipStream_t);
template void launch_convert<float, double>(int64_t, const float*, double*, double, hipStream_t);
template void launch_convert<double, double>(int64_t, const double*, double*, double, hipStream_t);

}  // namespace dev
}  // namespace hpg
