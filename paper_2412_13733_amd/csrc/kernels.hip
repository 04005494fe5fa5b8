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
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace hpg {
namespace dev {

// ---------------------------------------------------------------------------
// block reduction of a double (fixed order: wave shuffle tree, then waves in order)
__device__ inline double block_sum(double v, double* red) {
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

// ---------------------------------------------------------------------------
// u-side: y_u = alpha A x_u + B x_b  (+ residual epilogue)
template <typename T, int D, int MODE>
__global__ __launch_bounds__(256) void k_u_side(Geo g, URows<T> r0, URows<T> r1, URows<T> r2,
                                                T alpha, const T* __restrict__ xu,
                                                const T* __restrict__ xb,
                                                const T* __restrict__ xb_prev,
                                                const double* __restrict__ F,
                                                T* __restrict__ yu, double* __restrict__ partial,
                                                const int* __restrict__ done) {
    __shared__ double red[4];
    if (done && *done) return;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double part = 0.0;
    if (I < g.n_u) {
        int gi[3] = {0, 0, 0};
        int64_t t = I;
        gi[0] = (int)(t % g.n1[0]);
        t /= g.n1[0];
        if (D >= 2) {
            gi[1] = (int)(t % g.n1[1]);
            t /= g.n1[1];
        }
        if (D >= 3) gi[2] = (int)t;
        const int W = URows<T>::WM, WB = URows<T>::WB;
        T acc = 0;
        // ---- stiffness: alpha sum_k (A1 in k) (x) (M1 elsewhere)
        const int l0 = r0.lenM[gi[0]];
        const int* c0 = r0.colM + gi[0] * W;
        const T* a0 = r0.aM + gi[0] * W;
        const T* m0 = r0.mM + gi[0] * W;
        if (D == 1) {
            for (int e = 0; e < l0; ++e) acc += a0[e] * xu[c0[e]];
        } else if (D == 2) {
            const int l1 = r1.lenM[gi[1]];
            const int* c1 = r1.colM + gi[1] * W;
            const T* a1 = r1.aM + gi[1] * W;
            const T* m1 = r1.mM + gi[1] * W;
            for (int e1 = 0; e1 < l1; ++e1) {
                const T* row = xu + (int64_t)c1[e1] * g.n1[0];
                for (int e0 = 0; e0 < l0; ++e0)
                    acc += (a0[e0] * m1[e1] + m0[e0] * a1[e1]) * row[c0[e0]];
            }
        } else {
            const int l1 = r1.lenM[gi[1]];
            const int* c1 = r1.colM + gi[1] * W;
            const T* a1 = r1.aM + gi[1] * W;
            const T* m1 = r1.mM + gi[1] * W;
            const int l2 = r2.lenM[gi[2]];
            const int* c2 = r2.colM + gi[2] * W;
            const T* a2 = r2.aM + gi[2] * W;
            const T* m2 = r2.mM + gi[2] * W;
            for (int e2 = 0; e2 < l2; ++e2)
                for (int e1 = 0; e1 < l1; ++e1) {
                    const T* row = xu + ((int64_t)c2[e2] * g.n1[1] + c1[e1]) * g.n1[0];
                    const T am = a1[e1] * m2[e2], ma = m1[e1] * a2[e2], mm = m1[e1] * m2[e2];
                    for (int e0 = 0; e0 < l0; ++e0)
                        acc += (a0[e0] * mm + m0[e0] * (am + ma)) * row[c0[e0]];
                }
        }
        acc *= alpha;
        // ---- Gram: (x)_k B1 applied to x_b = x_psi (or psi - psi_prev)
        const int b0 = r0.lenB[gi[0]];
        const int* cc0 = r0.cellB + gi[0] * WB;
        const int* md0 = r0.modeB + gi[0] * WB;
        const T* v0 = r0.vB + gi[0] * WB;
        const int P = g.P;
        if (D == 1) {
            for (int e0 = 0; e0 < b0; ++e0) {
                const int64_t j = (int64_t)cc0[e0] * g.Pd + md0[e0];
                T xv = xb[j];
                if (MODE == MODE_RES) xv -= xb_prev[j];
                acc += v0[e0] * xv;
            }
        } else if (D == 2) {
            const int b1 = r1.lenB[gi[1]];
            const int* cc1 = r1.cellB + gi[1] * WB;
            const int* md1 = r1.modeB + gi[1] * WB;
            const T* v1 = r1.vB + gi[1] * WB;
            for (int e1 = 0; e1 < b1; ++e1)
                for (int e0 = 0; e0 < b0; ++e0) {
                    const int64_t cell = (int64_t)cc1[e1] * g.m[0] + cc0[e0];
                    const int64_t j = cell * g.Pd + md1[e1] * P + md0[e0];
                    T xv = xb[j];
                    if (MODE == MODE_RES) xv -= xb_prev[j];
                    acc += v0[e0] * v1[e1] * xv;
                }
        } else {
            const int b1 = r1.lenB[gi[1]];
            const int* cc1 = r1.cellB + gi[1] * WB;
            const int* md1 = r1.modeB + gi[1] * WB;
            const T* v1 = r1.vB + gi[1] * WB;
            const int b2 = r2.lenB[gi[2]];
            const int* cc2 = r2.cellB + gi[2] * WB;
            const int* md2 = r2.modeB + gi[2] * WB;
            const T* v2 = r2.vB + gi[2] * WB;
            for (int e2 = 0; e2 < b2; ++e2)
                for (int e1 = 0; e1 < b1; ++e1)
                    for (int e0 = 0; e0 < b0; ++e0) {
                        const int64_t cell =
                            ((int64_t)cc2[e2] * g.m[1] + cc1[e1]) * g.m[0] + cc0[e0];
                        const int64_t j = cell * g.Pd + (md2[e2] * P + md1[e1]) * P + md0[e0];
                        T xv = xb[j];
                        if (MODE == MODE_RES) xv -= xb_prev[j];
                        acc += v0[e0] * v1[e1] * v2[e2] * xv;
                    }
        }
        if (MODE == MODE_RES) {
            const double r = (double)acc - (double)alpha * F[I];
            yu[I] = (T)r;
            part = r * r;
        } else {
            yu[I] = acc;
            part = (double)acc * (double)xu[I];
        }
    }
    if (partial) {
        double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// sum-factorised contraction along one axis of a batch of cell tensors in LDS:
// out[.., i, ..] = sum_j mat(i, j) in[.., j, ..], mat(i, j) = mat[i*ld + j] or
// mat[j*ld + i] (trans).  din: input dims (direction 0 fastest).
template <typename T>
__device__ inline void contract_axis(const T* in, T* out, int stride, int ncell, int ax,
                                     const int din[3], int nout, const T* mat, int ld,
                                     bool trans) {
    int dout[3] = {din[0], din[1], din[2]};
    dout[ax] = nout;
    const int tot = dout[0] * dout[1] * dout[2];
    const int nin = din[ax];
    const int sax = (ax == 0) ? 1 : (ax == 1 ? din[0] : din[0] * din[1]);
    for (int e = threadIdx.x; e < ncell * tot; e += blockDim.x) {
        const int c = e / tot, o = e - c * tot;
        int idx[3];
        idx[0] = o % dout[0];
        const int r = o / dout[0];
        idx[1] = r % dout[1];
        idx[2] = r / dout[1];
        const int iout = idx[ax];
        idx[ax] = 0;
        const T* src = in + c * stride + idx[0] + din[0] * (idx[1] + din[1] * idx[2]);
        T acc = 0;
        if (trans)
            for (int j = 0; j < nin; ++j) acc += mat[j * ld + iout] * src[j * sax];
        else
            for (int j = 0; j < nin; ++j) acc += mat[iout * ld + j] * src[j * sax];
        out[c * stride + o] = acc;
    }
}

// apply the same matrix along every axis 0..D-1: buffers ping-pong between
// a and b; returns the buffer holding the result
template <typename T, int D>
__device__ inline T* contract_all(T* a, T* b, int stride, int ncell, int nin, int nout,
                                  const T* mat, int ld, bool trans) {
    int dims[3] = {1, 1, 1};
    for (int k = 0; k < D; ++k) dims[k] = nin;
    T* src = a;
    T* dst = b;
    for (int k = 0; k < D; ++k) {
        contract_axis<T>(src, dst, stride, ncell, k, dims, nout, mat, ld, trans);
        __syncthreads();
        dims[k] = nout;
        T* t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// gather the (p+1)^D local u coefficients of the block's cells into LDS
template <typename T, int D>
__device__ inline void gather_u(const Geo& g, const T* __restrict__ xu, T* buf, int stride,
                                int64_t cell0, int ncell) {
    const int L = g.p + 1;
    const int Ld = g.Ld;
    for (int e = threadIdx.x; e < ncell * Ld; e += blockDim.x) {
        const int ci = e / Ld, l = e - ci * Ld;
        int64_t cell = cell0 + ci;
        int cc[3] = {0, 0, 0};
        cc[0] = (int)(cell % g.m[0]);
        cell /= g.m[0];
        if (D >= 2) {
            cc[1] = (int)(cell % g.m[1]);
            cell /= g.m[1];
        }
        if (D >= 3) cc[2] = (int)cell;
        int ll[3] = {l % L, (l / L) % L, l / (L * L)};
        int64_t flat = 0, stridek = 1;
        bool ok = true;
        for (int k = 0; k < D; ++k) {
            const int gk = cc[k] * g.p + ll[k] - 1;
            ok = ok && gk >= 0 && gk < g.n1[k];
            flat += (int64_t)gk * stridek;
            stridek *= g.n1[k];
        }
        buf[ci * stride + l] = ok ? xu[flat] : (T)0;
    }
}

template <typename T, int D>
__device__ inline T cell_jac(const Geo& g, const T* const* hw, int64_t cell, T* hk) {
    T J = 1;
    int64_t c = cell;
    for (int k = 0; k < D; ++k) {
        const int ck = (int)(c % g.m[k]);
        c /= g.m[k];
        hk[k] = hw[k][ck];
        J *= (T)0.5 * hk[k];
    }
    return J;
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
                                                  const int* __restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    if (done && *done) return;
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int S = g.S;   // per-cell buffer stride (max(p+1, q)^D)
    T* bU = sm;
    T* bX = sm + cpb * S;
    T* bT = sm + 2 * cpb * S;
    T* bA = sm + 3 * cpb * S;
    T* bB = sm + 4 * cpb * S;
    const int64_t cell0 = (int64_t)blockIdx.x * cpb;
    const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
    const int L = g.p + 1, P = g.P, q = g.q;
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
    double part = 0.0;
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
                                               float* __restrict__ sinv32) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int n = g.Pd, q = g.q, P = g.P, Qd = g.Qd;
    const int S = g.S;
    // per cell: A, B (S each), T1 (q^(D-1) P^2), T2 (q P^4, D = 3), Dm (n^2), col/row (2n)
    const int sT1 = (D == 1) ? 1 : ((D == 2) ? q * P * P : q * q * P * P);
    const int sT2 = (D == 3) ? q * P * P * P * P : 1;
    const int per = 2 * S + sT1 + sT2 + n * n + 2 * n;
    const int64_t cell0 = (int64_t)blockIdx.x * cpb;
    const int ncell = (int)min((int64_t)cpb, g.n_cells - cell0);
    double* bA = sm;
    double* bB = sm + cpb * S;
    double* T1 = sm + 2 * cpb * S;
    double* T2 = T1 + cpb * sT1;
    double* Dm = T2 + cpb * sT2;
    double* cr = Dm + cpb * n * n;
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
    const double ia = 1.0 / alpha;
    for (int e = threadIdx.x; e < ncell * n * n; e += blockDim.x) {
        const int ci = e / (n * n), r = e - ci * n * n;
        const int i = r / n, j = r % n;
        const int64_t cell = cell0 + ci;
        const double* C = Cmat + (int64_t)cclass[cell] * n * n;
        double v = Dm[ci * n * n + r] + ia * C[r];
        if (i == j) {
            double hk[3];
            const double J = cell_jac<double, D>(g, tb.h, cell, hk);
            int aa[3] = {i % P, (i / P) % P, i / (P * P)};
            double md = J;
            for (int k = 0; k < D; ++k) md *= tb.Mdiag[aa[k]];
            v += beta * md;
        }
        Dm[ci * n * n + r] = v;
    }
    __syncthreads();
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
    for (int e = threadIdx.x; e < ncell * n * n; e += blockDim.x) {
        const int ci = e / (n * n), r = e - ci * n * n;
        // symmetrise (the exact inverse is symmetric)
        const int i = r / n, j = r % n;
        const double v = 0.5 * (Dm[ci * n * n + i * n + j] + Dm[ci * n * n + j * n + i]);
        const int64_t off = (cell0 + ci) * (int64_t)n * n + r;
        if (sinv64) sinv64[off] = v;
        if (sinv32) sinv32[off] = (float)v;
    }
    (void)per;
}

// ---------------------------------------------------------------------------
// psi-block of the preconditioner: z_psi = (-S_hat_K)^{-1} r_psi per cell;
// one thread per (cell, row); the block is symmetric, so thread i reads
// column i (coalesced across threads).  Partial dot <z, r> fused.
template <typename T>
__global__ __launch_bounds__(256) void k_prec_psi(int64_t n_cells, int n,
                                                  const T* __restrict__ sinv,
                                                  const T* __restrict__ r, T* __restrict__ z,
                                                  double* __restrict__ partial,
                                                  const int* __restrict__ done) {
    __shared__ double red[4];
    if (done && *done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double part = 0.0;
    if (e < n_cells * n) {
        const int64_t cell = e / n;
        const int i = (int)(e - cell * n);
        const T* Sb = sinv + cell * (int64_t)n * n;
        const T* rb = r + cell * n;
        T acc = 0;
        for (int j = 0; j < n; ++j) acc += Sb[(int64_t)j * n + i] * rb[j];
        z[e] = acc;
        part = (double)acc * (double)r[e];
    }
    if (partial) {
        double s = block_sum(part, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Tensor-axis GEMMs of the fast-diagonalisation A-block inverse.
// right:  Y[r][i] = sum_j X[r][j] Mat[i][j]         (axis 0; rows = other axes)
// left :  Y[o][i][c] = sum_j Mat[i][j] X[o][j][c]   (axis k > 0; o outer, c inner)
// 64x64 output tiles, 16-deep K slabs staged in LDS, 4x4 outputs per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_right(int64_t R, int N, const T* __restrict__ X,
                                                    const T* __restrict__ Mat,
                                                    T* __restrict__ Y,
                                                    const int* __restrict__ done) {
    __shared__ T sx[16][64 + 1];
    __shared__ T sm[16][64 + 1];
    if (done && *done) return;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t r0 = (int64_t)blockIdx.y * 64;
    const int i0 = blockIdx.x * 64;
    T acc[4][4] = {};
    for (int k0 = 0; k0 < N; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e % 16, rr = e / 16;
            const int64_t row = r0 + rr;
            const int col = k0 + kk;
            sx[kk][rr] = (row < R && col < N) ? X[row * N + col] : (T)0;
            const int irow = i0 + rr;
            sm[kk][rr] = (irow < N && col < N) ? Mat[(int64_t)irow * N + col] : (T)0;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) {
            T a[4], b[4];
            for (int u = 0; u < 4; ++u) a[u] = sx[kk][ty * 4 + u];
            for (int v = 0; v < 4; ++v) b[v] = sm[kk][tx * 4 + v];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u) {
        const int64_t row = r0 + ty * 4 + u;
        if (row >= R) continue;
        for (int v = 0; v < 4; ++v) {
            const int col = i0 + tx * 4 + v;
            if (col < N) Y[row * N + col] = acc[u][v];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_left(int64_t O, int N, int64_t C,
                                                   const T* __restrict__ X,
                                                   const T* __restrict__ Mat,
                                                   T* __restrict__ Y,
                                                   const int* __restrict__ done) {
    __shared__ T sm[16][64 + 1];
    __shared__ T sx[16][64 + 1];
    if (done && *done) return;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t o = blockIdx.z;
    const int i0 = blockIdx.y * 64;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const T* Xo = X + o * (int64_t)N * C;
    T* Yo = Y + o * (int64_t)N * C;
    T acc[4][4] = {};
    for (int k0 = 0; k0 < N; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e % 16, ii = e / 16;
            const int irow = i0 + ii, col = k0 + kk;
            sm[kk][ii] = (irow < N && col < N) ? Mat[(int64_t)irow * N + col] : (T)0;
            const int cc = e % 64, kk2 = e / 64;
            const int krow = k0 + kk2;
            const int64_t ccol = c0 + cc;
            sx[kk2][cc] = (krow < N && ccol < C) ? Xo[(int64_t)krow * C + ccol] : (T)0;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) {
            T a[4], b[4];
            for (int u = 0; u < 4; ++u) a[u] = sm[kk][ty * 4 + u];
            for (int v = 0; v < 4; ++v) b[v] = sx[kk][tx * 4 + v];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u) {
        const int irow = i0 + ty * 4 + u;
        if (irow >= N) continue;
        for (int v = 0; v < 4; ++v) {
            const int64_t ccol = c0 + tx * 4 + v;
            if (ccol < C) Yo[(int64_t)irow * C + ccol] = acc[u][v];
        }
    }
}

// z *= 1 / (alpha (lam_0[i0] + lam_1[i1] + lam_2[i2]))  (eigen-space division)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_fdm_scale(Geo g, const T* __restrict__ l0,
                                                   const T* __restrict__ l1,
                                                   const T* __restrict__ l2, T inv_alpha,
                                                   T* __restrict__ z,
                                                   const int* __restrict__ done) {
    if (done && *done) return;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.n_u) return;
    int64_t t = I;
    const int i0 = (int)(t % g.n1[0]);
    t /= g.n1[0];
    T lam = l0[i0];
    if (D >= 2) {
        lam += l1[(int)(t % g.n1[1])];
        t /= g.n1[1];
    }
    if (D >= 3) lam += l2[(int)t];
    z[I] *= inv_alpha / lam;
}

// ---------------------------------------------------------------------------
// MINRES scalar recurrences and vector updates (preconditioned MINRES for a
// symmetric indefinite G with an SPD preconditioner M).
__device__ inline double sum_partials(const double* p, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    return s;
}

// after <G q, q>: delta
__global__ void k_kr_delta(KState* st, const double* partial, int np) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    st->delta = sum_partials(partial, np);
}

// vhat = Gq - delta v_cur - gamma v_prev   (written over v_prev)
template <typename T>
__global__ __launch_bounds__(256) void k_kr_vhat(int64_t n, const KState* st, const T* Gq,
                                                 const T* vcur, T* vprev,
                                                 const int* __restrict__ done) {
    if (*done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T dl = (T)st->delta, gm = (T)st->gamma;
    vprev[i] = Gq[i] - dl * vcur[i] - gm * vprev[i];
}

// after <z, vhat>: new gamma, Givens rotation, convergence test
__global__ void k_kr_rotate(KState* st, const double* partial, int np, int* done) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    double g2 = sum_partials(partial, np);
    const double gnew = sqrt(g2 > 0.0 ? g2 : 0.0);
    const double delta = st->delta, gcur = st->gamma;
    const double a0 = st->c * delta - st->c_prev * st->s * gcur;
    const double a1 = sqrt(a0 * a0 + gnew * gnew);
    const double a2 = st->s * delta + st->c_prev * st->c * gcur;
    const double a3 = st->s_prev * gcur;
    st->c_prev = st->c;
    st->s_prev = st->s;
    if (a1 == 0.0 || !(a1 == a1)) {   // breakdown or NaN: stop
        st->done = 1;
        st->breakdown = 1;
        *done = 1;
        st->a1 = 1.0;
        st->a2 = 0.0;
        st->a3 = 0.0;
        st->step = 0.0;
        return;
    }
    st->c = a0 / a1;
    st->s = gnew / a1;
    st->a1 = a1;
    st->a2 = a2;
    st->a3 = a3;
    st->step = st->c * st->eta;
    st->eta = -st->s * st->eta;
    st->gamma_new = gnew;
    st->iters += 1;
    if (fabs(st->eta) <= st->rtol * st->gamma1 || st->iters >= st->max_iters || gnew == 0.0) {
        st->done = 1;
    }
}

// w_new = (q - a3 w_prev - a2 w_cur) / a1 (over w_prev); x += step w_new;
// v_prev <- vhat / gamma_new (vhat lives in v_prev, v_cur kept for the swap),
// q <- z / gamma_new
template <typename T>
__global__ __launch_bounds__(256) void k_kr_update(int64_t n, const KState* st, T* q,
                                                   T* wprev, const T* wcur, T* x, T* vprev,
                                                   const T* z, const int* __restrict__ done) {
    if (*done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ia1 = 1.0 / st->a1;
    const T a2 = (T)st->a2, a3 = (T)st->a3;
    const T wn = (T)((double)(q[i] - a3 * wprev[i] - a2 * wcur[i]) * ia1);
    wprev[i] = wn;
    x[i] += (T)st->step * wn;
    const double gn = st->gamma_new;
    const double ig = gn > 0.0 ? 1.0 / gn : 0.0;
    vprev[i] = (T)((double)vprev[i] * ig);
    q[i] = (T)((double)z[i] * ig);
}

// finish an iteration: gamma <- gamma_new; raise the host-visible flag
__global__ void k_kr_finish(KState* st, int* done) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (*done) return;
    st->gamma = st->gamma_new;
    if (st->done) *done = 1;
}

// initialisation: gamma1 = sqrt(<z1, b>), v_cur = b / gamma1, q = z1 / gamma1
__global__ void k_kr_init(KState* st, const double* partial, int np, double rtol, int maxit,
                          int* done) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double g2 = sum_partials(partial, np);
    const double g1 = sqrt(g2 > 0.0 ? g2 : 0.0);
    st->gamma1 = g1;
    st->gamma = g1;
    st->gamma_new = g1;
    st->eta = g1;
    st->c = st->c_prev = 1.0;
    st->s = st->s_prev = 0.0;
    st->iters = 0;
    st->max_iters = maxit;
    st->rtol = rtol;
    st->breakdown = 0;
    st->done = (g1 == 0.0 || !(g1 == g1)) ? 1 : 0;
    *done = st->done;
}

template <typename T>
__global__ __launch_bounds__(256) void k_kr_start(int64_t n, const KState* st, const T* b,
                                                  const T* z, T* vcur, T* vprev, T* q, T* wprev,
                                                  T* wcur, T* x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g1 = st->gamma1;
    const double ig = g1 > 0.0 ? 1.0 / g1 : 0.0;
    vcur[i] = (T)((double)b[i] * ig);
    q[i] = (T)((double)z[i] * ig);
    vprev[i] = 0;
    wprev[i] = 0;
    wcur[i] = 0;
    x[i] = 0;
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
                                            double* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
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
                   int mode, hipStream_t s) {
    dim3 grid(nblk(g.n_u)), blk(256);
#define HPG_U(DD, MM)                                                                       \
    hipLaunchKernelGGL((k_u_side<T, DD, MM>), grid, blk, 0, s, g, r[0], r[1], r[2], alpha, \
                       xu, xb, xb_prev, F, yu, partial, done)
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
                     const int* done, int mode, hipStream_t s) {
    dim3 grid(nblk(g.n_cells, cpb)), blk(256);
    size_t shm = (size_t)5 * cpb * g.S * sizeof(T);
#define HPG_P(DD, MM)                                                                      \
    hipLaunchKernelGGL((k_psi_side<T, DD, MM>), grid, blk, shm, s, g, tb, cpb, beta, xu, \
                       xpsi, omega, Phi, ypsi, partial, done)
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
    return (size_t)(2 * g.S + sT1 + sT2 + n * n + 2 * n) * sizeof(double);
}

void launch_setup(const Geo& g, const PsiTabs<double>& tb, int cpb, const double* psi,
                  double alpha, double beta, const double* C, const int* cclass, double* om64,
                  float* om32, double* s64, float* s32, hipStream_t s) {
    dim3 grid(nblk(g.n_cells, cpb)), blk(256);
    size_t shm = setup_smem_per_cell(g) * cpb;
#define HPG_S(DD)                                                                        \
    hipLaunchKernelGGL((k_setup<DD>), grid, blk, shm, s, g, tb, cpb, psi, alpha, beta, C, \
                       cclass, om64, om32, s64, s32)
    if (g.d == 1) HPG_S(1);
    else if (g.d == 2) HPG_S(2);
    else HPG_S(3);
#undef HPG_S
}

template <typename T>
void launch_prec_psi(int64_t n_cells, int n, const T* sinv, const T* r, T* z, double* partial,
                     const int* done, hipStream_t s) {
    hipLaunchKernelGGL((k_prec_psi<T>), dim3(nblk(n_cells * n)), dim3(256), 0, s, n_cells, n,
                       sinv, r, z, partial, done);
}

template <typename T>
void launch_gemm_right(int64_t R, int N, const T* X, const T* Mat, T* Y, const int* done,
                       hipStream_t s) {
    dim3 grid((N + 63) / 64, (unsigned)((R + 63) / 64));
    hipLaunchKernelGGL((k_gemm_right<T>), grid, dim3(256), 0, s, R, N, X, Mat, Y, done);
}

template <typename T>
void launch_gemm_left(int64_t O, int N, int64_t C, const T* X, const T* Mat, T* Y,
                      const int* done, hipStream_t s) {
    dim3 grid((unsigned)((C + 63) / 64), (N + 63) / 64, (unsigned)O);
    hipLaunchKernelGGL((k_gemm_left<T>), grid, dim3(256), 0, s, O, N, C, X, Mat, Y, done);
}

template <typename T>
void launch_fdm_scale(const Geo& g, const T* l0, const T* l1, const T* l2, T inv_alpha, T* z,
                      const int* done, hipStream_t s) {
    dim3 grid(nblk(g.n_u));
    if (g.d == 1)
        hipLaunchKernelGGL((k_fdm_scale<T, 1>), grid, dim3(256), 0, s, g, l0, l1, l2, inv_alpha,
                           z, done);
    else if (g.d == 2)
        hipLaunchKernelGGL((k_fdm_scale<T, 2>), grid, dim3(256), 0, s, g, l0, l1, l2, inv_alpha,
                           z, done);
    else
        hipLaunchKernelGGL((k_fdm_scale<T, 3>), grid, dim3(256), 0, s, g, l0, l1, l2, inv_alpha,
                           z, done);
}

template <typename T>
void launch_dot(int64_t n, const T* a, const T* b, double* partial, int nblocks, const int* done,
                hipStream_t s) {
    hipLaunchKernelGGL((k_dot<T>), dim3(nblocks), dim3(256), 0, s, n, a, b, partial, done);
}

void launch_kr_delta(KState* st, const double* partial, int np, hipStream_t s) {
    hipLaunchKernelGGL(k_kr_delta, dim3(1), dim3(64), 0, s, st, partial, np);
}
template <typename T>
void launch_kr_vhat(int64_t n, const KState* st, const T* Gq, const T* vcur, T* vprev,
                    const int* done, hipStream_t s) {
    hipLaunchKernelGGL((k_kr_vhat<T>), dim3(nblk(n)), dim3(256), 0, s, n, st, Gq, vcur, vprev,
                       done);
}
void launch_kr_rotate(KState* st, const double* partial, int np, int* done, hipStream_t s) {
    hipLaunchKernelGGL(k_kr_rotate, dim3(1), dim3(64), 0, s, st, partial, np, done);
}
template <typename T>
void launch_kr_update(int64_t n, const KState* st, T* q, T* wprev, const T* wcur, T* x, T* vprev,
                      const T* z, const int* done, hipStream_t s) {
    hipLaunchKernelGGL((k_kr_update<T>), dim3(nblk(n)), dim3(256), 0, s, n, st, q, wprev, wcur,
                       x, vprev, z, done);
}
void launch_kr_finish(KState* st, int* done, hipStream_t s) {
    hipLaunchKernelGGL(k_kr_finish, dim3(1), dim3(64), 0, s, st, done);
}
void launch_kr_init(KState* st, const double* partial, int np, double rtol, int maxit, int* done,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_kr_init, dim3(1), dim3(64), 0, s, st, partial, np, rtol, maxit, done);
}
template <typename T>
void launch_kr_start(int64_t n, const KState* st, const T* b, const T* z, T* vcur, T* vprev,
                     T* q, T* wprev, T* wcur, T* x, hipStream_t s) {
    hipLaunchKernelGGL((k_kr_start<T>), dim3(nblk(n)), dim3(256), 0, s, n, st, b, z, vcur, vprev,
                       q, wprev, wcur, x);
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
               double* partial, hipStream_t s) {
    dim3 grid(nblk(g.n_cells, cpb));
    size_t shm = (size_t)4 * cpb * g.S * sizeof(double);
    if (g.d == 1)
        hipLaunchKernelGGL((k_l2<1>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial);
    else if (g.d == 2)
        hipLaunchKernelGGL((k_l2<2>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial);
    else
        hipLaunchKernelGGL((k_l2<3>), grid, dim3(256), shm, s, g, tb, cpb, u, v, partial);
}

#define HPG_INST(T)                                                                              \
    template void launch_u_side<T>(const Geo&, const URows<T>*, T, const T*, const T*, const T*, \
                                   const double*, T*, double*, const int*, int, hipStream_t);   \
    template void launch_psi_side<T>(const Geo&, const PsiTabs<T>&, int, T, const T*, const T*, \
                                     const T*, const double*, T*, double*, const int*, int,     \
                                     hipStream_t);                                               \
    template void launch_prec_psi<T>(int64_t, int, const T*, const T*, T*, double*, const int*, \
                                     hipStream_t);                                               \
    template void launch_gemm_right<T>(int64_t, int, const T*, const T*, T*, const int*,        \
                                       hipStream_t);                                             \
    template void launch_gemm_left<T>(int64_t, int, int64_t, const T*, const T*, T*, const int*, \
                                      hipStream_t);                                              \
    template void launch_fdm_scale<T>(const Geo&, const T*, const T*, const T*, T, T*,          \
                                      const int*, hipStream_t);                                  \
    template void launch_kr_vhat<T>(int64_t, const KState*, const T*, const T*, T*, const int*, \
                                    hipStream_t);                                                \
    template void launch_kr_update<T>(int64_t, const KState*, T*, T*, const T*, T*, T*,         \
                                      const T*, const int*, hipStream_t);                        \
    template void launch_kr_start<T>(int64_t, const KState*, const T*, const T*, T*, T*, T*, T*, \
                                     T*, T*, hipStream_t);                                       \
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
