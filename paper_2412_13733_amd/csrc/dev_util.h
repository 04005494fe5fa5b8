// Device helpers shared by the kernels of the hpG library: block reductions,
// register copies of the sparse 1-D rows, and the sum-factorised per-cell
// contractions staged in LDS.
#pragma once

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

// register copies of one sparse 1-D row (stiffness/mass, and psi coupling)
template <typename T, int W>
struct Row {
    int n;
    int c[W];
    T a[W], m[W];
    __device__ inline void load(const URows<T>& r, int g) {
        n = r.lenM[g];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const bool ok = e < n;
            c[e] = ok ? r.colM[g * W + e] : 0;
            a[e] = ok ? r.aM[g * W + e] : (T)0;
            m[e] = ok ? r.mM[g * W + e] : (T)0;
        }
    }
};
template <typename T, int W>
struct BRow {
    int n;
    int cell[W], mode[W];
    T v[W];
    __device__ inline void load(const URows<T>& r, int g) {
        n = r.lenB[g];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const bool ok = e < n;
            cell[e] = ok ? r.cellB[g * W + e] : 0;
            mode[e] = ok ? r.modeB[g * W + e] : 0;
            v[e] = ok ? r.vB[g * W + e] : (T)0;
        }
    }
    // the (v', zeta) coupling rows of the gradient constraint
    __device__ inline void loadG(const URows<T>& r, int g) {
        n = r.lenG[g];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const bool ok = e < n;
            cell[e] = ok ? r.cellG[g * W + e] : 0;
            mode[e] = ok ? r.modeG[g * W + e] : 0;
            v[e] = ok ? r.vG[g * W + e] : (T)0;
        }
    }
};

// (A_0 M_1 M_2 + M_0 A_1 M_2 + M_0 M_1 A_2) x_u at the global unknown with
// 1-D indices gi: tensor products of the sparse 1-D rows held in registers
template <typename T, int D>
__device__ inline T stiff_mass_sum(const Geo& g, const URows<T>& r0, const URows<T>& r1,
                                   const URows<T>& r2, const int gi[3], const T* __restrict__ xu) {
    constexpr int W = URows<T>::WM;
    Row<T, W> R0;
    R0.load(r0, gi[0]);
    T acc = 0;
    if (D == 1) {
#pragma unroll
        for (int e0 = 0; e0 < W; ++e0)
            if (e0 < R0.n) acc += R0.a[e0] * xu[R0.c[e0]];
    } else if (D == 2) {
        Row<T, W> R1;
        R1.load(r1, gi[1]);
#pragma unroll
        for (int e1 = 0; e1 < W; ++e1) {
            if (e1 < R1.n) {
                const T* row = xu + (int64_t)R1.c[e1] * g.n1[0];
                const T m1 = R1.m[e1], a1 = R1.a[e1];
#pragma unroll
                for (int e0 = 0; e0 < W; ++e0)
                    if (e0 < R0.n) acc += (R0.a[e0] * m1 + R0.m[e0] * a1) * row[R0.c[e0]];
            }
        }
    } else {
        Row<T, W> R1, R2;
        R1.load(r1, gi[1]);
        R2.load(r2, gi[2]);
#pragma unroll
        for (int e2 = 0; e2 < W; ++e2) {
            if (e2 >= R2.n) continue;
#pragma unroll
            for (int e1 = 0; e1 < W; ++e1) {
                if (e1 >= R1.n) continue;
                const T* row = xu + ((int64_t)R2.c[e2] * g.n1[1] + R1.c[e1]) * g.n1[0];
                const T am = R1.a[e1] * R2.m[e2] + R1.m[e1] * R2.a[e2];
                const T mm = R1.m[e1] * R2.m[e2];
#pragma unroll
                for (int e0 = 0; e0 < W; ++e0)
                    if (e0 < R0.n) acc += (R0.a[e0] * mm + R0.m[e0] * am) * row[R0.c[e0]];
            }
        }
    }
    return acc;
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

// a different matrix along each axis k (mats[k], all nin -> nout, leading
// dimension ld); returns the buffer holding the result
template <typename T, int D>
__device__ inline T* contract_axes(T* a, T* b, int stride, int ncell, int nin, int nout,
                                   const T* const* mats, int ld, bool trans) {
    int dims[3] = {1, 1, 1};
    for (int k = 0; k < D; ++k) dims[k] = nin;
    T* src = a;
    T* dst = b;
    for (int k = 0; k < D; ++k) {
        contract_axis<T>(src, dst, stride, ncell, k, dims, nout, mats[k], ld, trans);
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

// D block of one weight field on one cell: out[a * ldo + b] (+)= sum_q w(q)
// V_a(q) V_b(q), a, b in [0, P^d), sum-factorised direction by direction
// (T1: q^(d-1) P^2, T2: q P^4 (d = 3) of work space)
template <int D>
__device__ inline void d_block(const double* w, const double* V, int P, int q, double* T1,
                               double* T2, double* out, int ldo) {
    const int PP = P * P;
    if (D == 1) {
        for (int e = threadIdx.x; e < PP; e += blockDim.x) {
            const int a = e / P, b = e % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += w[j] * V[j * P + a] * V[j * P + b];
            out[a * ldo + b] = s;
        }
        __syncthreads();
    } else if (D == 2) {
        for (int e = threadIdx.x; e < q * PP; e += blockDim.x) {
            const int q2 = e / PP, ab = e % PP, a1 = ab / P, b1 = ab % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += w[q2 * q + j] * V[j * P + a1] * V[j * P + b1];
            T1[e] = s;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
            const int ab2 = e / PP, ab1 = e % PP;
            const int a2 = ab2 / P, b2 = ab2 % P, a1 = ab1 / P, b1 = ab1 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += V[j * P + a2] * V[j * P + b2] * T1[j * PP + ab1];
            out[(a1 + P * a2) * ldo + (b1 + P * b2)] = s;
        }
        __syncthreads();
    } else {
        for (int e = threadIdx.x; e < q * q * PP; e += blockDim.x) {
            const int q32 = e / PP, ab = e % PP, a1 = ab / P, b1 = ab % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += w[q32 * q + j] * V[j * P + a1] * V[j * P + b1];
            T1[e] = s;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < q * PP * PP; e += blockDim.x) {
            const int q3 = e / (PP * PP), rr = e % (PP * PP), ab2 = rr / PP, ab1 = rr % PP;
            const int a2 = ab2 / P, b2 = ab2 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j)
                s += V[j * P + a2] * V[j * P + b2] * T1[(q3 * q + j) * PP + ab1];
            T2[e] = s;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < PP * PP * PP; e += blockDim.x) {
            const int ab3 = e / (PP * PP), rr = e % (PP * PP), ab2 = rr / PP, ab1 = rr % PP;
            const int a3 = ab3 / P, b3 = ab3 % P, a2 = ab2 / P, b2 = ab2 % P, a1 = ab1 / P,
                      b1 = ab1 % P;
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += V[j * P + a3] * V[j * P + b3] * T2[(j * PP + ab2) * PP + ab1];
            out[(a1 + P * (a2 + P * a3)) * ldo + (b1 + P * (b2 + P * b3))] = s;
        }
        __syncthreads();
    }
}

// d = 3 form of d_block without the q P^4 work space: the last two
// directions are summed together (q^2 terms per entry instead of q)
__device__ inline void d_block3_direct(const double* w, const double* V, int P, int q,
                                       double* T1, double* out, int ldo) {
    const int PP = P * P;
    for (int e = threadIdx.x; e < q * q * PP; e += blockDim.x) {
        const int q32 = e / PP, ab = e % PP, a1 = ab / P, b1 = ab % P;
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += w[q32 * q + j] * V[j * P + a1] * V[j * P + b1];
        T1[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < PP * PP * PP; e += blockDim.x) {
        const int ab3 = e / (PP * PP), rr = e % (PP * PP), ab2 = rr / PP, ab1 = rr % PP;
        const int a3 = ab3 / P, b3 = ab3 % P, a2 = ab2 / P, b2 = ab2 % P, a1 = ab1 / P,
                  b1 = ab1 % P;
        double s = 0.0;
        for (int j3 = 0; j3 < q; ++j3) {
            double t = 0.0;
            for (int j2 = 0; j2 < q; ++j2)
                t += V[j2 * P + a2] * V[j2 * P + b2] * T1[(j3 * q + j2) * PP + ab1];
            s += V[j3 * P + a3] * V[j3 * P + b3] * t;
        }
        out[(a1 + P * (a2 + P * a3)) * ldo + (b1 + P * (b2 + P * b3))] = s;
    }
    __syncthreads();
}

// In-place inverse of one SPD n x n block (row-major, any memory space) by
// Gauss-Jordan elimination without pivoting; cr: 2n doubles of LDS for the
// pivot column and row.  Every thread of the block takes part (blockDim a
// multiple of 32): half-waves sweep rows, lanes sweep columns.
__device__ inline void gauss_jordan_spd(double* Dm, int n, double* cr) {
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5, ny = blockDim.x >> 5;
    for (int k = 0; k < n; ++k) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            cr[i] = Dm[(int64_t)i * n + k];
            cr[n + i] = Dm[(int64_t)k * n + i];
        }
        __syncthreads();
        const double ip = 1.0 / cr[k];
        for (int i = ty; i < n; i += ny) {
            const double ci = cr[i];
            double* row = Dm + (int64_t)i * n;
            for (int j = tx; j < n; j += 32) {
                const double rk = (j == k ? 1.0 : cr[n + j]) * ip;
                row[j] = (i == k) ? rk : ((j == k ? 0.0 : row[j]) - ci * rk);
            }
        }
        __syncthreads();
    }
}

// The same elimination with the block held in registers: blockDim = 1024
// threads as a 32 x 32 grid, thread (ty, tx) owning the 4 x 4 elements
// (ty + 32 a, tx + 32 b), so n <= 128.  Per pass the owners publish the pivot
// column (cr[0, 128)) and row (cr[128, 256)) to LDS and every thread updates
// its elements in registers; the arithmetic per element is that of
// gauss_jordan_spd.  Elements beyond n are zero and stay zero (their pivot
// column and row entries are zero), so the update runs without bounds tests.
// cr: 256 doubles.  The block is read from and written back to Dm.
__device__ inline void gauss_jordan_spd_reg(double* Dm, int n, double* cr) {
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double v[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 32 * a, j = tx + 32 * b;
            v[a][b] = (i < n && j < n) ? Dm[i * n + j] : 0.0;
        }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // k lies in register column / row kb (uniform) of the owners tx = kr / ty = kr
        const int kb = k >> 5, kr = k & 31;
        if (tx == kr) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b == kb)
#pragma unroll
                    for (int a = 0; a < 4; ++a) cr[ty + 32 * a] = v[a][b];
        }
        if (ty == kr) {
            // the row's own pivot entry is published as 1, so rk = cr[128 + j] / pivot
            // needs no case for j = k
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a == kb)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        cr[128 + tx + 32 * b] = (tx == kr && b == kb) ? 1.0 : v[a][b];
        }
        __syncthreads();
        const double ip = 1.0 / cr[k];
        double rk[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) rk[b] = cr[128 + tx + 32 * b] * ip;
        // column k restarts from zero (its new value is -c_i rk_k) ...
        if (tx == kr) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b == kb)
#pragma unroll
                    for (int a = 0; a < 4; ++a) v[a][b] = 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double ci = cr[ty + 32 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) v[a][b] -= ci * rk[b];
        }
        // ... and row k becomes rk
        if (ty == kr) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a == kb)
#pragma unroll
                    for (int b = 0; b < 4; ++b) v[a][b] = rk[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 32 * a, j = tx + 32 * b;
            if (i < n && j < n) Dm[i * n + j] = v[a][b];
        }
    __syncthreads();
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

}  // namespace dev
}  // namespace hpg
