// Diagnostics of a computed iterate at the Gauss points of every cell:
// the complementarity sums of the multiplier lambda = (psi_{k-1} - psi_k) /
// alpha_k (Sec. 2.1) against the latent gap exp(-psi_h) (obstacle), and the
// largest pointwise violation of the constraint, u_h - phi (obstacle) or
// |grad u_h| - phi (gradient).  Run once per solve, so each point is
// evaluated directly from the cell's coefficients (staged in LDS) rather than
// by sum factorisation: (p+1)^d products per value.
//
// partial[3 b + 0] = sum w |J| |lambda_h| exp(-psi_h), partial[3 b + 1] =
// sum w |J| |lambda_h|, partial[3 b + 2] = max violation, for block b; the
// host adds the sums of all blocks in block order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>

#include "dev_util.h"
#include "kernels.h"

namespace hpg {
namespace dev {

namespace {

constexpr double kExpCap = 700.0;   // exp(-psi) evaluated as exp(min(-psi, 700))

__device__ inline double block_max(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = -DBL_MAX;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s = fmax(s, red[i]);
    }
    return s;   // valid in thread 0
}

// value at Gauss point jj of a cell tensor of n modes per direction:
// sum_a prod_k tab[jj[k] * n + a_k] c[a]
template <int D>
__device__ inline double eval_point(const double* c, const double* tab, int n, const int* jj) {
    double s = 0.0;
    if (D == 1) {
        for (int a = 0; a < n; ++a) s += tab[jj[0] * n + a] * c[a];
    } else if (D == 2) {
        for (int b = 0; b < n; ++b) {
            double t = 0.0;
            for (int a = 0; a < n; ++a) t += tab[jj[0] * n + a] * c[b * n + a];
            s += tab[jj[1] * n + b] * t;
        }
    } else {
        for (int e = 0; e < n; ++e) {
            double t2 = 0.0;
            for (int b = 0; b < n; ++b) {
                double t = 0.0;
                for (int a = 0; a < n; ++a) t += tab[jj[0] * n + a] * c[(e * n + b) * n + a];
                t2 += tab[jj[1] * n + b] * t;
            }
            s += tab[jj[2] * n + e] * t2;
        }
    }
    return s;
}

// d/dy_c of the local u tensor at Gauss point jj: the reference derivative
// table Du along direction c, values Vu along the others
template <int D>
__device__ inline double eval_deriv(const double* c, const double* Vu, const double* Du, int L,
                                    const int* jj, int dir) {
    const double* t0 = dir == 0 ? Du : Vu;
    const double* t1 = dir == 1 ? Du : Vu;
    const double* t2 = dir == 2 ? Du : Vu;
    double s = 0.0;
    if (D == 1) {
        for (int a = 0; a < L; ++a) s += t0[jj[0] * L + a] * c[a];
    } else if (D == 2) {
        for (int b = 0; b < L; ++b) {
            double t = 0.0;
            for (int a = 0; a < L; ++a) t += t0[jj[0] * L + a] * c[b * L + a];
            s += t1[jj[1] * L + b] * t;
        }
    } else {
        for (int e = 0; e < L; ++e) {
            double u2 = 0.0;
            for (int b = 0; b < L; ++b) {
                double t = 0.0;
                for (int a = 0; a < L; ++a) t += t0[jj[0] * L + a] * c[(e * L + b) * L + a];
                u2 += t1[jj[1] * L + b] * t;
            }
            s += t2[jj[2] * L + e] * u2;
        }
    }
    return s;
}

}  // namespace

// uniform-degree tensor meshes: one cell at a time per block
template <int D, bool GRAD>
__global__ __launch_bounds__(256) void k_diag(Geo g, PsiTabs<double> tb,
                                              const double* __restrict__ Du,
                                              const double* __restrict__ u,
                                              const double* __restrict__ psi,
                                              const double* __restrict__ lam,
                                              const double* __restrict__ phiq,
                                              double* __restrict__ partial, DiagBatch bt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    {
        const int64_t rb = blockIdx.y;
        u += rb * bt.u;
        psi += rb * bt.psi;
        lam += rb * bt.psi;
        phiq += rb * bt.qp;
        partial += rb * 3 * (int64_t)gridDim.x;
    }
    double* su = reinterpret_cast<double*>(smem_raw);   // Ld
    double* sp = su + g.Ld;                             // Pd (obstacle)
    double* sl = sp + g.Pd;                             // Pd
    const int L = g.p + 1, q = g.q, P = g.P;
    double cr = 0.0, l1 = 0.0, mv = -DBL_MAX;
    for (int64_t cell = blockIdx.x; cell < g.n_cells; cell += gridDim.x) {
        int cc[3] = {0, 0, 0};
        int64_t t = cell;
        for (int k = 0; k < D; ++k) {
            cc[k] = (int)(t % g.m[k]);
            t /= g.m[k];
        }
        for (int l = threadIdx.x; l < g.Ld; l += blockDim.x) {
            const int ll[3] = {l % L, (l / L) % L, l / (L * L)};
            int64_t flat = 0, sk = 1;
            bool ok = true;
            for (int k = 0; k < D; ++k) {
                const int gk = cc[k] * g.p + ll[k] - 1;
                ok = ok && gk >= 0 && gk < g.n1[k];
                flat += (int64_t)gk * sk;
                sk *= g.n1[k];
            }
            su[l] = ok ? u[flat] : 0.0;
        }
        if (!GRAD)
            for (int a = threadIdx.x; a < g.Pd; a += blockDim.x) {
                sp[a] = psi[cell * g.Pd + a];
                sl[a] = lam[cell * g.Pd + a];
            }
        __syncthreads();
        double hk[3];
        const double J = cell_jac<double, D>(g, tb.h, cell, hk);
        for (int j = threadIdx.x; j < g.Qd; j += blockDim.x) {
            const int jj[3] = {j % q, (j / q) % q, j / (q * q)};
            const double ph = phiq[cell * g.Qd + j];
            if (GRAD) {
                double g2 = 0.0;
                for (int c = 0; c < D; ++c) {
                    const double dv = eval_deriv<D>(su, tb.Vu, Du, L, jj, c) * (2.0 / hk[c]);
                    g2 += dv * dv;
                }
                mv = fmax(mv, sqrt(g2) - ph);
            } else {
                double wq = J;
                for (int k = 0; k < D; ++k) wq *= tb.w[jj[k]];
                const double uv = eval_point<D>(su, tb.Vu, L, jj);
                const double pv = eval_point<D>(sp, tb.Vpsi, P, jj);
                const double lv = eval_point<D>(sl, tb.Vpsi, P, jj);
                cr += wq * fabs(lv) * exp(fmin(-pv, kExpCap));
                l1 += wq * fabs(lv);
                mv = fmax(mv, uv - ph);
            }
        }
        __syncthreads();
    }
    const double s1 = block_sum(cr, red);
    __syncthreads();
    const double s2 = block_sum(l1, red);
    __syncthreads();
    const double s3 = block_max(mv, red);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = s1;
        partial[3 * blockIdx.x + 1] = s2;
        partial[3 * blockIdx.x + 2] = s3;
    }
}

size_t diag_lds(const Geo& g) { return (size_t)(g.Ld + 2 * g.Pd) * sizeof(double); }

void launch_diag(const Geo& g, const PsiTabs<double>& tb, const double* Du, const double* u,
                 const double* psi, const double* lam, const double* phiq, double* partial,
                 int nblocks, hipStream_t s, const DiagBatch& bt) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(g.n_cells, nblocks));
    const size_t shm = diag_lds(g);
    const bool grad = g.nc > 1 || g.P == g.p;   // gradient constraint: P = p modes
#define HPG_DIAG(DD, GG)                                                                      \
    hipLaunchKernelGGL((k_diag<DD, GG>), dim3(grid, (unsigned)bt.nb), dim3(256), shm, s, g, tb, \
                       Du, u, psi, lam, phiq, partial, bt)
    if (grad) {
        if (g.d == 1) HPG_DIAG(1, true);
        else if (g.d == 2) HPG_DIAG(2, true);
        else HPG_DIAG(3, true);
    } else {
        if (g.d == 1) HPG_DIAG(1, false);
        else if (g.d == 2) HPG_DIAG(2, false);
        else HPG_DIAG(3, false);
    }
#undef HPG_DIAG
}

// one degree per cell (obstacle): cells through the local -> global map
template <int D>
__global__ __launch_bounds__(256) void k_hp_diag(HpGeo g, HpTabs<double> tb,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ psi,
                                                 const double* __restrict__ lam,
                                                 const double* __restrict__ phiq,
                                                 double* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[4];
    double* su = reinterpret_cast<double*>(smem_raw);
    double cr = 0.0, l1 = 0.0, mv = -DBL_MAX;
    for (int64_t cell = blockIdx.x; cell < g.n_cells; cell += gridDim.x) {
        const int p = g.cell_p[cell], L = p + 1, P = p - 1, q = p + 1;
        const int nl = (int)(g.loc_off[cell + 1] - g.loc_off[cell]);
        const int np = (int)(g.psi_off[cell + 1] - g.psi_off[cell]);
        double* sp = su + nl;
        double* sl = sp + np;
        for (int l = threadIdx.x; l < nl; l += blockDim.x) {
            const int gi = g.loc2glob[g.loc_off[cell] + l];
            su[l] = gi >= 0 ? u[gi] : 0.0;
        }
        for (int a = threadIdx.x; a < np; a += blockDim.x) {
            sp[a] = psi[g.psi_off[cell] + a];
            sl[a] = lam[g.psi_off[cell] + a];
        }
        __syncthreads();
        const HpTabOff o = tb.off[p];
        const double* Vu = tb.base + o.Vu;
        const double* Vpsi = tb.base + o.Vpsi;
        const double* w = tb.base + o.w;
        double J = 1.0;
        int64_t t = cell;
        for (int k = 0; k < D; ++k) {
            J *= 0.5 * tb.h[k][(int)(t % g.m[k])];
            t /= g.m[k];
        }
        const int nq = (int)(g.qp_off[cell + 1] - g.qp_off[cell]);
        for (int j = threadIdx.x; j < nq; j += blockDim.x) {
            const int jj[3] = {j % q, (j / q) % q, j / (q * q)};
            double wq = J;
            for (int k = 0; k < D; ++k) wq *= w[jj[k]];
            const double uv = eval_point<D>(su, Vu, L, jj);
            const double pv = eval_point<D>(sp, Vpsi, P, jj);
            const double lv = eval_point<D>(sl, Vpsi, P, jj);
            cr += wq * fabs(lv) * exp(fmin(-pv, kExpCap));
            l1 += wq * fabs(lv);
            mv = fmax(mv, uv - phiq[g.qp_off[cell] + j]);
        }
        __syncthreads();
    }
    const double s1 = block_sum(cr, red);
    __syncthreads();
    const double s2 = block_sum(l1, red);
    __syncthreads();
    const double s3 = block_max(mv, red);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = s1;
        partial[3 * blockIdx.x + 1] = s2;
        partial[3 * blockIdx.x + 2] = s3;
    }
}

size_t hp_diag_lds(const HpGeo& g) {
    size_t L = 1, P = 1;
    for (int k = 0; k < g.d; ++k) {
        L *= (size_t)g.lmax;
        P *= (size_t)(g.lmax - 2);
    }
    return (L + 2 * P) * sizeof(double);
}

void launch_hp_diag(const HpGeo& g, const HpTabs<double>& tb, const double* u, const double* psi,
                    const double* lam, const double* phiq, double* partial, int nblocks,
                    hipStream_t s) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(g.n_cells, nblocks));
    const size_t shm = hp_diag_lds(g);
    if (g.d == 1)
        hipLaunchKernelGGL((k_hp_diag<1>), dim3(grid), dim3(256), shm, s, g, tb, u, psi, lam, phiq,
                           partial);
    else if (g.d == 2)
        hipLaunchKernelGGL((k_hp_diag<2>), dim3(grid), dim3(256), shm, s, g, tb, u, psi, lam, phiq,
                           partial);
    else
        hipLaunchKernelGGL((k_hp_diag<3>), dim3(grid), dim3(256), shm, s, g, tb, u, psi, lam, phiq,
                           partial);
}

}  // namespace dev
}  // namespace hpg
