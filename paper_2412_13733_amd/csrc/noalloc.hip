// hpg_op_residual_noalloc: the FP64 Newton residual with every scratch
// buffer of its kernels in a fixed device array of the library, so that the
// call allocates no memory (for callers that cannot allocate: code under
// graph capture, serving loops, harnesses that forbid allocation).
//
// The array holds the kernels' per-block partial sums of ||R_u||^2 and
// ||R_psi||^2 and, on meshes with one degree per cell, the per-local-function
// values of the cell pass.  Every block writes its partial sums and the cell
// pass writes every local value before the gather reads it, so nothing has to
// be cleared between calls.  The host copy of the partial sums goes to a
// per-thread static buffer.  One array per device, shared by every call on
// that device: calls that overlap on one device race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "problem.h"

namespace hpg {
namespace {

constexpr int kMaxPartials = 8192;                        // partial sums (doubles)
constexpr size_t kScratchDoubles = (size_t)1 << 20;      // 8 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// device address of this device's copy of the array (looked up once per
// device, with that device current: the array's host-side name is not a
// device address)
double* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) fail(HPG_ERR_INVALID_ARG, "device ordinal too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        HPG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(HPG_ERR_DEVICE, "no device address for the residual scratch array");
        g_scratch[device] = static_cast<double*>(ptr);
    }
    return g_scratch[device];
}

thread_local double t_host_part[kMaxPartials];

}  // namespace
}  // namespace hpg

using namespace hpg;

extern "C" {

hpg_status hpg_op_residual_noalloc(hpg_problem* prob, const double* d_u, const double* d_psi,
                                   const double* d_psi_prev, double alpha, double* d_R,
                                   double* norms2, void* stream) {
    return guarded([&]() -> hpg_status {
        if (!prob) fail(HPG_ERR_INVALID_ARG, "problem handle is NULL");
        HPG_HIP(hipSetDevice(prob->P.device));
        if (!d_u || !d_psi || !d_psi_prev || !d_R) fail(HPG_ERR_INVALID_ARG, "NULL buffer");
        if (!(alpha > 0)) fail(HPG_ERR_INVALID_ARG, "alpha must be > 0");
        Problem& P = prob->P;
        const int npart = P.residual_partials();
        const int64_t nloc = P.residual_local_values();
        if (npart > kMaxPartials || nloc > (int64_t)(kScratchDoubles - kMaxPartials))
            fail(HPG_ERR_INVALID_ARG,
                 "mesh too large for the allocation-free residual (at most 8192 partial sums and "
                 "1040384 local values)");
        double* base = scratch_on(P.device);
        Problem::ResScratch sc{base, nloc ? base + kMaxPartials : nullptr, t_host_part};
        double a = 0.0, b = 0.0;
        P.residual(d_u, d_psi, d_psi_prev, alpha, d_R, P.stream(stream), &a, &b, &sc);
        if (norms2) {
            norms2[0] = a;
            norms2[1] = b;
        }
        return HPG_OK;
    });
}

}  // extern "C"
