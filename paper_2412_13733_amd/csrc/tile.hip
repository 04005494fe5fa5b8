// Dispatch of the fused tiled G apply / residual over (d, p).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace hpg {
namespace dev {

// tile edge in cells for (d, p): 2-D tiles own about 12-24 u unknowns per
// direction, 3-D tiles one cell
constexpr int tile_cells(int D, int PP) {
    return D == 1 ? 16
                  : (D == 3 ? (PP == 2 ? 4 : 1)
                            : (PP == 2 ? 16 : PP == 3 ? 8 : PP == 4 ? 4 : PP == 5 ? 3 : PP == 6 ? 2 : 1));
}
constexpr int TILE_GRID_CAP = 2048;

int64_t tile_count(const Geo& g) {
    const int TC = tile_cells(g.d, g.p);
    int64_t n = 1;
    for (int k = 0; k < g.d; ++k) n *= (g.m[k] + TC - 1) / TC;
    return n;
}

int tile_grid(const Geo& g) {
    const int TC = tile_cells(g.d, g.p);
    int64_t n = 1;
    for (int k = 0; k < g.d; ++k) n *= (g.m[k] + TC - 1) / TC;
    return (int)std::min<int64_t>(n, TILE_GRID_CAP);
}

bool tile_supported(const Geo& g) {
    if (g.P != g.p - 1 || g.q != g.p + 1) return false;   // obstacle pairing, q = p + 1
    if (g.d == 3) return g.p >= 2 && g.p <= 7;
    return g.p >= 2 && g.p <= 12;
}

template <typename T, int D, int MODE>
bool launch_tile_d(const Geo& g, const URows<T>* r, const PsiTabs<T>& tb, T alpha, T beta,
                   const double* prm, const T* xu, const T* xpsi, const T* xpsi_prev,
                   const T* omega, const double* F, const double* Phi, T* yu, T* ypsi,
                   double* partial, const int* done, hipStream_t s, const KernelEvents* ev,
                   const TileBatch& bt);

template <typename T>
bool launch_tile(const Geo& g, const URows<T>* r, const PsiTabs<T>& tb, T alpha, T beta,
                 const double* prm, const T* xu, const T* xpsi, const T* xpsi_prev, const T* omega,
                 const double* F, const double* Phi, T* yu, T* ypsi, double* partial,
                 const int* done, int mode, hipStream_t s, const KernelEvents* ev,
                 const TileBatch& bt) {
    if (!tile_supported(g)) return false;
#define HPG_TD(DD, MM)                                                                        \
    return launch_tile_d<T, DD, MM>(g, r, tb, alpha, beta, prm, xu, xpsi, xpsi_prev, omega, F, \
                                    Phi, yu, ypsi, partial, done, s, ev, bt)
    if (mode == MODE_APPLY) {
        if (g.d == 1) HPG_TD(1, MODE_APPLY);
        if (g.d == 2) HPG_TD(2, MODE_APPLY);
        HPG_TD(3, MODE_APPLY);
    }
    if (g.d == 1) HPG_TD(1, MODE_RES);
    if (g.d == 2) HPG_TD(2, MODE_RES);
    HPG_TD(3, MODE_RES);
#undef HPG_TD
}

template bool launch_tile<double>(const Geo&, const URows<double>*, const PsiTabs<double>&, double,
                                  double, const double*, const double*, const double*,
                                  const double*, const double*, const double*, const double*,
                                  double*, double*, double*, const int*, int, hipStream_t,
                                  const KernelEvents*, const TileBatch&);
template bool launch_tile<float>(const Geo&, const URows<float>*, const PsiTabs<float>&, float,
                                 float, const double*, const float*, const float*, const float*,
                                 const float*, const double*, const double*, float*, float*,
                                 double*, const int*, int, hipStream_t, const KernelEvents*,
                                 const TileBatch&);

}  // namespace dev
}  // namespace hpg
