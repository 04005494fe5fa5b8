// Batched solves: nb independent problems on one mesh (the same breakpoints,
// degree and obstacle constraint, each with its own f and phi) solved
// together, so that every step of the inner Newton solve of all requests is
// one launch: the fused tiled G apply over (request, tile) items, the
// fast-diagonalisation passes as GEMMs batched over requests (the tables and
// eigenvectors are shared), the psi-block over (request, cell group), the
// Lanczos kernels over (request, slice), the Newton residual, the setup of
// the linearisation over all cells of all requests, and the line search.
//
// Every reduction is per request and in the order of a solve of that request
// alone: partial sums have a per-request stride, MINRES keeps one scalar
// state per request, and each request's Newton and proximal decisions (step
// acceptance, convergence, FP64 recomputation of a mixed-precision direction)
// are taken from its own quantities only.  A request's result therefore does
// not depend on the others in the batch.  Requests that have converged, or
// whose outer loop has stopped, stay in the launches with a zero right-hand
// side (MINRES returns at once) and a zero step.
//
// The method is that of Problem::solve (Sec. 2.1 proximal loop, Newton with
// backtracking on each subproblem eq. (pG), MINRES with P_D of eq. (schur4)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <vector>

#include "problem.h"

namespace hpg {
namespace {

// ---- small batched vector kernels -------------------------------------------

// y_b = x_b + t_b d_b (y_b = x_b exactly where t_b = 0); element i of request b
// at b * stride + i
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_strided(int64_t n, const double* __restrict__ x,
                                                      int64_t sx, const double* __restrict__ t,
                                                      const T* __restrict__ d, int64_t sd,
                                                      double* __restrict__ y, int64_t sy) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double tb = t[b];
    const double xv = x[b * sx + i];
    y[b * sy + i] = tb == 0.0 ? xv : xv + tb * (double)d[b * sd + i];
}

// x_b = 0 for the requests with mask_b = 0 (n values per request)
template <typename T>
__global__ __launch_bounds__(256) void k_mask(int64_t n, const int* __restrict__ mask,
                                              T* __restrict__ x) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !mask[b]) x[b * n + i] = (T)0;
}

// lam_b = (psi_prev_b - psi_b) / alpha for the requests with mask_b = 1
__global__ __launch_bounds__(256) void k_lambda_masked(int64_t n, const int* __restrict__ mask,
                                                       const double* __restrict__ pp,
                                                       const double* __restrict__ p, double alpha,
                                                       double* __restrict__ lam) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mask[b]) lam[b * n + i] = (pp[b * n + i] - p[b * n + i]) / alpha;
}

// y_b = (double) x_b for the requests with mask_b = 1 (n values per request)
template <typename T>
__global__ __launch_bounds__(256) void k_copy_masked(int64_t n, const int* __restrict__ mask,
                                                     const T* __restrict__ x,
                                                     double* __restrict__ y) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mask[b]) y[b * n + i] = (double)x[b * n + i];
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
struct BKrylov {
    DBuf z, vcur, vprev, vhat, q, Gq, wprev, wcur, t1, t2, x;
};

// FP64 and FP32 views of the shared tables
template <typename T>
struct BSel;
template <>
struct BSel<double> {
    static const DevRows<double>* rows(const Problem& p) { return p.rows64; }
    static const DevTabs<double>& tabs(const Problem& p) { return p.tab64; }
    static const DevFdm<double>& fdm(const Problem& p) { return p.fdm64; }
    static constexpr int prec = HPG_FP64;
};
template <>
struct BSel<float> {
    static const DevRows<float>* rows(const Problem& p) { return p.rows32; }
    static const DevTabs<float>& tabs(const Problem& p) { return p.tab32; }
    static const DevFdm<float>& fdm(const Problem& p) { return p.fdm32; }
    static constexpr int prec = HPG_MIXED;
};

}  // namespace

struct Batch {
    Problem P;   // the shared mesh: tables, eigenvectors, geometry (its own data unused)
    int nb = 1;
    int64_t nu = 0, np = 0, n = 0, ncell = 0, nqp = 0;
    int PS = 0;          // per-request partial-sum stride
    DBuf F, Phi, PhiQ, cclass_rep;
    std::vector<double> normF, normPhi, phimax;
    bool have_data = false;
    // linearisation (FP64 always; FP32 as well for mixed solves)
    DBuf om64, om32, s64, s32;
    bool lin32 = false;
    double alpha = 1.0, beta = 0.0;
    BKrylov<double> k64;
    BKrylov<float> k32;
    DBuf part, gpart, kst, mask, tvec, diagp;
    // Newton state
    DBuf u, psi, pp, ut, pt, R, uold, d64, rhs32, d32, rhs64, lam;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<dev::KState> hst;
    std::vector<int> last_iters, last_breakdown;

    ~Batch() {
        if (P.own_stream) (void)hipStreamSynchronize(P.own_stream);
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    }
    void build(const Mesh& M, int nbatch, int device);
    void set_data(const double* f, const double* phi);
    void setup(const double* d_psi, double a, double b, bool want32, hipStream_t s);
    template <typename T>
    void apply_G(const T* x, T* y, double* gp, const int* done, hipStream_t s);
    template <typename T>
    void apply_prec(const T* r, T* z, double* pr, const int* done, hipStream_t s);
    template <typename T>
    void iterations(int count, T*& vcur, T*& vprev, T*& wprev, T*& wcur, T* q, T* Gq, T* z, T* x,
                    hipStream_t s);
    template <typename T>
    void minres(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t s);
    void residual(const double* uu, const double* ps, const double* ppv, double a, double* RR,
                  hipStream_t s, double* nu2, double* np2);
    void l2_diff(const double* a, const double* b, hipStream_t s, double* d, double* nrm);
    hpg_status solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* st, double* d_u_out,
                     double* d_psi_out, double* d_lam_out);
    template <typename T>
    BKrylov<T>& kw();
    static int kstride() { return (int)(sizeof(dev::KState) / sizeof(int)); }
};

template <>
BKrylov<double>& Batch::kw<double>() { return k64; }
template <>
BKrylov<float>& Batch::kw<float>() { return k32; }

void Batch::build(const Mesh& M, int nbatch, int device) {
    if (M.hp) fail(HPG_ERR_INVALID_ARG, "batched solves: one degree on every cell only");
    if (M.kind != HPG_OBSTACLE) fail(HPG_ERR_INVALID_ARG, "batched solves: obstacle constraint only");
    P.single_stream = true;
    P.build(M, device);
    if (!P.use_tile || P.setup_mode != dev::SETUP_LDS || P.prec_big || !P.fdm_dot_fused)
        fail(HPG_ERR_INVALID_ARG,
             "batched solves need the fused tiled apply (p <= 12 in 1-D/2-D, <= 7 in 3-D) with "
             "Schur blocks in LDS");
    // requests run along the second grid dimension, and along the third
    // together with the outer batches of a 3-D middle pass (both <= 65535)
    if (nbatch > 65535 || (M.d == 3 && (int64_t)nbatch * M.n1[2] > 65535))
        fail(HPG_ERR_INVALID_ARG, "too many requests in one batch for this mesh");
    nb = nbatch;
    nu = M.n_u;
    np = M.n_psi;
    n = nu + np;
    ncell = M.n_cells;
    nqp = M.n_qp;
    PS = P.np_cap;
    const size_t B = (size_t)nb;
    std::vector<int32_t> cc((size_t)ncell);
    HPG_HIP(hipMemcpy(cc.data(), P.cclass.p, cc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> rep(B * ncell);
    for (size_t b = 0; b < B; ++b) std::copy(cc.begin(), cc.end(), rep.begin() + b * ncell);
    upload(cclass_rep, rep);
    part.alloc(B * PS * sizeof(double));
    gpart.alloc(B * PS * sizeof(double));
    kst.alloc(2 * B * sizeof(dev::KState));
    mask.alloc(B * sizeof(int));
    tvec.alloc(B * sizeof(double));
    diagp.alloc(B * 3 * 1024 * sizeof(double));
    hst.resize(B);
    last_iters.assign(B, 0);
    last_breakdown.assign(B, 0);
}

void Batch::set_data(const double* f, const double* phi) {
    // each request's F, Phi and phi at the Gauss points, through the shared
    // problem's own (host) projection of the data
    const size_t B = (size_t)nb;
    std::vector<double> Fh(B * nu), Ph(B * np);
    normF.assign(B, 1.0);
    normPhi.assign(B, 1.0);
    phimax.assign(B, 0.0);
    for (size_t b = 0; b < B; ++b) {
        P.set_data(f + b * nqp, phi + b * nqp);
        HPG_HIP(hipMemcpy(Fh.data() + b * nu, P.F.p, nu * sizeof(double), hipMemcpyDeviceToHost));
        HPG_HIP(hipMemcpy(Ph.data() + b * np, P.Phi.p, np * sizeof(double), hipMemcpyDeviceToHost));
        normF[b] = P.normF;
        normPhi[b] = P.normPhi;
        phimax[b] = P.phi_absmax;
    }
    upload(F, Fh);
    upload(Phi, Ph);
    upload(PhiQ, std::vector<double>(phi, phi + B * nqp));
    have_data = true;
}

void Batch::setup(const double* d_psi, double a, double b, bool want32, hipStream_t s) {
    alpha = a;
    beta = b;
    const size_t B = (size_t)nb;
    const size_t nq = (size_t)ncell * P.geo.Qd, ns = (size_t)ncell * P.geo.Pd * P.geo.Pd;
    om64.alloc(B * nq * sizeof(double));
    s64.alloc(B * ns * sizeof(double));
    if (want32) {
        om32.alloc(B * nq * sizeof(float));
        s32.alloc(B * ns * sizeof(float));
    }
    lin32 = want32;
    P.alpha = a;
    P.beta = b;
    P.hparams[0] = a;
    P.hparams[1] = b;
    P.hparams[2] = 1.0 / a;
    HPG_HIP(hipMemcpyAsync(P.params.p, P.hparams, sizeof(P.hparams), hipMemcpyHostToDevice, s));
    // the cells of all requests in one launch: psi, the weights and the blocks
    // are request-major, the cell geometry repeats per request
    dev::Geo gb = P.geo;
    gb.n_cells = (int64_t)nb * ncell;
    P.tstart("setup", s);
    dev::launch_setup(gb, P.tab64.view(), P.cpb_setup, dev::SETUP_LDS, d_psi, a, b, P.C.as<double>(),
                      cclass_rep.as<int>(), om64.as<double>(), want32 ? om32.as<float>() : nullptr,
                      s64.as<double>(), want32 ? s32.as<float>() : nullptr, s);
    P.tstop("setup", s);
    HPG_HIP(hipGetLastError());
}

template <typename T>
void Batch::apply_G(const T* x, T* y, double* gp, const int* done, hipStream_t s) {
    const DevRows<T>* rw = BSel<T>::rows(P);
    dev::URows<T> r[3] = {rw[0].view(), rw[1].view(), rw[2].view()};
    dev::TileBatch bt;
    bt.nb = nb;
    bt.xu = bt.xp = bt.yu = bt.yp = n;
    bt.om = (int64_t)ncell * P.geo.Qd;
    bt.part = PS;
    bt.done = kstride();
    const T* om = BSel<T>::prec == HPG_FP64 ? (const T*)om64.p : (const T*)om32.p;
    const dev::KernelEvents ke = P.kernel_events("apply_G");
    dev::launch_tile<T>(P.geo, r, BSel<T>::tabs(P).view(), (T)alpha, (T)beta, P.params.as<double>(),
                        x, x + nu, nullptr, om, nullptr, nullptr, y, y + nu, gp, done,
                        dev::MODE_APPLY, s, &ke, bt);
}

template <typename T>
void Batch::apply_prec(const T* r, T* z, double* pr, const int* done, hipStream_t s) {
    P.ensure_fdm();
    BKrylov<T>& K = kw<T>();
    const DevFdm<T>& Fd = BSel<T>::fdm(P);
    T* t1 = K.t1.template as<T>();
    T* t2 = K.t2.template as<T>();
    const T* sinv = BSel<T>::prec == HPG_FP64 ? (const T*)s64.p : (const T*)s32.p;
    const Mesh& M = P.M;
    const int d = M.d, npass = 2 * d, Pd = P.geo.Pd;
    const int ks = kstride();
    dev::PsiBatch pb;
    pb.nb = nb;
    pb.sinv = (int64_t)ncell * Pd * Pd;
    pb.r = pb.z = n;
    pb.part = PS;
    pb.done = ks;
    const T* src = r;
    int pass = 0;
    for (int ph = 0; ph < 2; ++ph) {
        for (int k = 0; k < d; ++k) {
            ++pass;
            T* dst = (pass == npass) ? z : ((src == t1) ? t2 : t1);
            dev::GemmEpi<T> ep{};
            if (ph == 0 && k == d - 1) {
                ep.scale_mode = d;
                ep.n0 = M.n1[0];
                ep.l0 = Fd.lam[0].template as<T>();
                ep.l1 = Fd.lam[1].template as<T>();
                ep.l2 = Fd.lam[2].template as<T>();
                ep.prm = P.params.as<double>();
            }
            if (pass == npass) {
                ep.dotv = r;
                ep.partial = pr;
            }
            ep.pstride = PS;
            ep.dstride = ks;
            const int N = M.n1[k];
            const int64_t ss = src == r ? n : nu, ds = dst == z ? n : nu;
            const dev::KernelEvents ke = P.kernel_events("fdm");
            if (k == 0) {
                const T* Bm = ph == 0 ? Fd.V[k].template as<T>() : Fd.Vt[k].template as<T>();
                const int R = (int)(nu / N);
                ep.bdiv = 1;
                if (pass == 1)
                    dev::launch_gemm_prec<T>(R, N, N, src, N, Bm, N, dst, N, done, ep, ncell, Pd,
                                             P.cpb_prec, sinv, r + nu, z + nu,
                                             pr ? pr + P.np_dot : nullptr, s, ss, ds, pb);
                else
                    dev::launch_gemm<T>(R, N, N, src, N, ss, Bm, N, 0, dst, N, ds, nb, done, ep, s,
                                        &ke);
            } else {
                const T* Am = ph == 0 ? Fd.Vt[k].template as<T>() : Fd.V[k].template as<T>();
                int64_t inner = 1;
                for (int j = 0; j < k; ++j) inner *= M.n1[j];
                const int64_t outer = nu / (inner * N);
                ep.bdiv = (int)outer;
                // within a request the outer batches are N inner apart; the
                // intermediate buffers hold the requests nu apart, which is
                // outer N inner, so one stride covers all; the output z (n
                // apart) is written only by the last pass, where outer = 1
                const int64_t sa = (int64_t)N * inner;
                const int64_t sc = dst == z ? n : (int64_t)N * inner;
                dev::launch_gemm<T>(N, (int)inner, N, Am, N, 0, src, inner, sa, dst, inner, sc,
                                    (int)(outer * nb), done, ep, s, &ke);
            }
            src = dst;
        }
    }
}

template <typename T>
void Batch::iterations(int count, T*& vcur, T*& vprev, T*& wprev, T*& wcur, T* q, T* Gq, T* z,
                       T* x, hipStream_t s) {
    auto* st = kst.as<dev::KState>();
    double* pr = part.as<double>();
    double* gp = gpart.as<double>();
    T* vhat = kw<T>().vhat.template as<T>();
    const int npG = dev::tile_grid(P.geo), npP = P.np_dot + P.np_prec;
    dev::VecBatch vg, vp;
    vg.nb = vp.nb = nb;
    vg.v = vp.v = n;
    vg.part = vp.part = PS;
    int par = 0;
    for (int j = 0; j < count; ++j) {
        dev::KState* cur = st + (size_t)par * nb;
        dev::KState* nxt = st + (size_t)(1 - par) * nb;
        const int* dn = &cur->done;
        apply_G<T>(q, Gq, gp, dn, s);
        P.tstart("minres_vec", s);
        dev::launch_kr_vhat<T>(n, cur, gp, npG, Gq, vcur, vprev, vhat, s, vg);
        P.tstop("minres_vec", s);
        apply_prec<T>(vhat, z, pr, dn, s);
        P.tstart("minres_vec", s);
        dev::launch_kr_update<T>(n, cur, nxt, pr, npP, q, wprev, wcur, x, vprev, vhat, z, s, vp);
        P.tstop("minres_vec", s);
        std::swap(vprev, vcur);
        std::swap(wprev, wcur);
        par = 1 - par;
    }
}

template <typename T>
void Batch::minres(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t s) {
    BKrylov<T>& K = kw<T>();
    const size_t bytes = (size_t)nb * n * sizeof(T), bu = (size_t)nb * nu * sizeof(T);
    K.z.alloc(bytes);
    K.vcur.alloc(bytes);
    K.vprev.alloc(bytes);
    K.vhat.alloc(bytes);
    K.q.alloc(bytes);
    K.Gq.alloc(bytes);
    K.wprev.alloc(bytes);
    K.wcur.alloc(bytes);
    K.t1.alloc(bu);
    K.t2.alloc(bu);
    T* z = K.z.template as<T>();
    T* vcur = K.vcur.template as<T>();
    T* vprev = K.vprev.template as<T>();
    T* q = K.q.template as<T>();
    T* Gq = K.Gq.template as<T>();
    T* wprev = K.wprev.template as<T>();
    T* wcur = K.wcur.template as<T>();
    auto* st = kst.as<dev::KState>();
    double* pr = part.as<double>();
    const int npP = P.np_dot + P.np_prec;
    apply_prec<T>(b, z, pr, nullptr, s);
    dev::VecBatch vp;
    vp.nb = nb;
    vp.v = n;
    vp.part = PS;
    dev::launch_kr_start<T>(n, st, pr, npP, rtol, maxit, b, z, vcur, vprev, q, wprev, wcur, x, s,
                            vp);
    HPG_HIP(hipGetLastError());
    chunk = std::max(2, chunk + (chunk & 1));
    hipGraphExec_t exec = nullptr;
    if (!P.timing) {
        const GraphKey key{BSel<T>::prec, chunk, (const void*)b, (const void*)x};
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            T *vc = vcur, *vpp = vprev, *wp = wprev, *wc = wcur;
            hipGraph_t g;
            std::lock_guard<std::recursive_mutex> api(device_api_mutex());
            HPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            iterations<T>(chunk, vc, vpp, wp, wc, q, Gq, z, x, s);
            HPG_HIP(hipStreamEndCapture(s, &g));
            HPG_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
            HPG_HIP(hipGraphDestroy(g));
            graphs[key] = exec;
        } else {
            exec = it->second;
        }
    }
    int it = 0;
    while (it < maxit) {
        if (exec) {
            HPG_HIP(hipGraphLaunch(exec, s));
        } else {
            T *vc = vcur, *vpp = vprev, *wp = wprev, *wc = wcur;
            iterations<T>(chunk, vc, vpp, wp, wc, q, Gq, z, x, s);
        }
        it += chunk;
        // an even chunk leaves every request's state in st[0 .. nb)
        HPG_HIP(hipMemcpyAsync(hst.data(), st, (size_t)nb * sizeof(dev::KState),
                               hipMemcpyDeviceToHost, s));
        HPG_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int b2 = 0; b2 < nb && all; ++b2) all = hst[b2].done != 0;
        if (all) break;
    }
    HPG_HIP(hipGetLastError());
    for (int b2 = 0; b2 < nb; ++b2) {
        last_iters[b2] = hst[b2].iters;
        last_breakdown[b2] = hst[b2].breakdown;
    }
}

void Batch::residual(const double* uu, const double* ps, const double* ppv, double a, double* RR,
                     hipStream_t s, double* nu2, double* np2) {
    const DevRows<double>* rw = P.rows64;
    dev::URows<double> r[3] = {rw[0].view(), rw[1].view(), rw[2].view()};
    dev::TileBatch bt;
    bt.nb = nb;
    bt.xu = nu;
    bt.xp = bt.pprev = np;
    bt.F = nu;
    bt.Phi = np;
    bt.yu = bt.yp = n;
    bt.part = PS;
    double* pr = part.as<double>();
    P.tstart("residual", s);
    dev::launch_tile<double>(P.geo, r, P.tab64.view(), a, 0.0, nullptr, uu, ps, ppv, nullptr,
                             F.as<double>(), Phi.as<double>(), RR, RR + nu, pr, nullptr,
                             dev::MODE_RES, s, nullptr, bt);
    P.tstop("residual", s);
    HPG_HIP(hipGetLastError());
    const int tg = dev::tile_grid(P.geo);
    std::vector<double> h((size_t)nb * PS);
    HPG_HIP(hipMemcpyAsync(h.data(), pr, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
        double x = 0.0, y = 0.0;
        const double* hb = h.data() + (size_t)b * PS;
        for (int i = 0; i < tg; ++i) {
            x += hb[2 * i];
            y += hb[2 * i + 1];
        }
        nu2[b] = x;
        np2[b] = y;
    }
}

void Batch::l2_diff(const double* a, const double* b, hipStream_t s, double* d, double* nrm) {
    // ||a_b - b_b||, ||a_b|| per request
    dev::VecBatch vb;
    vb.nb = nb;
    vb.v = nu;
    vb.part = PS;
    double* pr = part.as<double>();
    dev::launch_l2(P.geo, P.tab64.view(), P.cpb_l2, a, b, pr, s, vb);
    HPG_HIP(hipGetLastError());
    const int nbl = (int)((ncell + P.cpb_l2 - 1) / P.cpb_l2);
    std::vector<double> h((size_t)nb * PS);
    HPG_HIP(hipMemcpyAsync(h.data(), pr, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nb; ++r) {
        double d2 = 0.0, a2 = 0.0;
        const double* hb = h.data() + (size_t)r * PS;
        for (int i = 0; i < nbl; ++i) {
            d2 += hb[2 * i];
            a2 += hb[2 * i + 1];
        }
        d[r] = std::sqrt(std::max(d2, 0.0));
        nrm[r] = std::sqrt(std::max(a2, 0.0));
    }
}

// MINRES tolerance of an FP64 recomputation and the caps on them, as in a
// single solve
constexpr double kBatchFallbackRtol = 1e-10;
constexpr int kBatchMaxFallbacksPerStep = 3;
constexpr int kBatchMaxFallbacksPerSolve = 12;

hpg_status Batch::solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* stats,
                        double* d_u_out, double* d_psi_out, double* d_lam_out) {
    if (!have_data) fail(HPG_ERR_INVALID_ARG, "forcing and obstacle must be set");
    if (o.step_extension || o.inexact_newton || o.warm_u || o.k0)
        fail(HPG_ERR_INVALID_ARG,
             "batched solves: step_extension, inexact_newton and warm starts are not supported");
    const int kmax = o.fixed_prox_steps > 0 ? o.fixed_prox_steps : o.max_prox;
    if (o.q != 0 && o.q != P.M.q)
        fail(HPG_ERR_INVALID_ARG, "only the Gauss rule with q = p + 1 points per direction is built");
    const auto t0 = std::chrono::steady_clock::now();
    const bool mixed = o.precision == HPG_MIXED;
    const size_t B = (size_t)nb;
    u.alloc(B * nu * sizeof(double));
    ut.alloc(B * nu * sizeof(double));
    uold.alloc(B * nu * sizeof(double));
    psi.alloc(B * np * sizeof(double));
    pt.alloc(B * np * sizeof(double));
    pp.alloc(B * np * sizeof(double));
    lam.alloc(B * np * sizeof(double));
    R.alloc(B * n * sizeof(double));
    d64.alloc(B * n * sizeof(double));
    k64.x.alloc(B * n * sizeof(double));
    rhs64.alloc(B * n * sizeof(double));
    if (mixed) {
        rhs32.alloc(B * n * sizeof(float));
        d32.alloc(B * n * sizeof(float));
    }
    double* du = u.as<double>();
    double* dp = psi.as<double>();
    double* dut = ut.as<double>();
    double* dpt = pt.as<double>();
    double* dpp = pp.as<double>();
    double* dR = R.as<double>();
    double* dd = d64.as<double>();
    double* xk = k64.x.as<double>();
    int* dmask = mask.as<int>();
    double* dt = tvec.as<double>();
    HPG_HIP(hipMemsetAsync(du, 0, B * nu * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(dp, 0, B * np * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(dpp, 0, B * np * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(lam.p, 0, B * np * sizeof(double), s));
    std::vector<hpg_solve_stats> S(B);
    for (auto& x : S) {
        std::memset(&x, 0, sizeof(x));
        x.status = HPG_OK;
    }
    std::vector<int> running(B, 1), stop_now(B, 0), recomputed(B, 0), fb_step(B, 0);
    std::vector<double> nu2(B), np2(B), a2(B), b2(B), err(B), m0(B), t(B), diff(B), nrm(B);
    std::vector<int> conv(B), act(B), acc(B), need64(B);
    double alpha_k = o.alpha0;
    int k = 0;
    auto upload_mask = [&](const std::vector<int>& m) {
        HPG_HIP(hipMemcpyAsync(dmask, m.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
    };
    auto upload_t = [&](const std::vector<double>& tv) {
        HPG_HIP(hipMemcpyAsync(dt, tv.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
    };
    const dim3 gu(blocks_of(nu), (unsigned)nb), gp(blocks_of(np), (unsigned)nb),
        gn(blocks_of(n), (unsigned)nb);
    // trial iterates (u, psi) + t_b delta_b of every request (t_b = 0: a copy)
    auto trial = [&]() {
        upload_t(t);
        hipLaunchKernelGGL((k_axpy_strided<double>), gu, dim3(256), 0, s, nu, du, nu, dt, dd, n,
                           dut, nu);
        hipLaunchKernelGGL((k_axpy_strided<double>), gp, dim3(256), 0, s, np, dp, np, dt, dd + nu,
                           n, dpt, np);
    };
    // MINRES for the Newton directions of the requests in sel (FP32 operator in
    // a mixed solve, else FP64 at tolerance rt) from the residual in dR; the
    // other requests solve with a zero right-hand side.  The directions go to
    // dd for the selected requests only.
    auto directions = [&](const std::vector<int>& sel, bool fp32, double rt) {
        upload_mask(sel);
        if (fp32) {
            float* b32 = rhs32.as<float>();
            float* x32 = d32.as<float>();
            dev::launch_convert<double, float>((int64_t)B * n, dR, b32, -1.0, s);
            hipLaunchKernelGGL((k_mask<float>), gn, dim3(256), 0, s, n, dmask, b32);
            minres<float>(b32, x32, rt, o.max_krylov, o.krylov_chunk, s);
            hipLaunchKernelGGL((k_copy_masked<float>), gn, dim3(256), 0, s, n, dmask, x32, dd);
        } else {
            dev::launch_convert<double, double>((int64_t)B * n, dR, rhs64.as<double>(), -1.0, s);
            hipLaunchKernelGGL((k_mask<double>), gn, dim3(256), 0, s, n, dmask, rhs64.as<double>());
            minres<double>(rhs64.as<double>(), xk, rt, o.max_krylov, o.krylov_chunk, s);
            hipLaunchKernelGGL((k_copy_masked<double>), gn, dim3(256), 0, s, n, dmask, xk, dd);
        }
        for (size_t b = 0; b < B; ++b)
            if (sel[b]) S[b].krylov_iters += last_iters[b];
    };
    // backtracking line search of the requests in open0 from t = 1; requests
    // with fixed[b] keep their step t[b] (already accepted) and the rest take
    // no step.  Sets acc[b] for the requests it accepts.
    auto line_search = [&](const std::vector<int>& open0, const std::vector<int>& fixed) {
        std::vector<int> open(B, 0);
        for (size_t b = 0; b < B; ++b) {
            if (open0[b]) {
                t[b] = 1.0;
                acc[b] = 0;
                open[b] = 1;
            } else if (!fixed[b]) {
                t[b] = 0.0;
            }
        }
        for (int halvings = 0; halvings <= 30; ++halvings) {
            bool any = false;
            for (size_t b = 0; b < B; ++b) any = any || open[b];
            if (!any) break;
            trial();
            residual(dut, dpt, dpp, alpha_k, dR, s, a2.data(), b2.data());
            for (size_t b = 0; b < B; ++b) {
                if (!open[b]) continue;
                const double m1 = std::sqrt(a2[b] / (alpha_k * alpha_k) + b2[b]);
                if (m1 <= (1.0 - 1e-4 * t[b]) * m0[b]) {
                    acc[b] = 1;
                    open[b] = 0;
                } else if (halvings == 30) {
                    open[b] = 0;
                    t[b] = 0.0;
                } else {
                    t[b] *= 0.5;
                    S[b].line_search_halvings += 1;
                }
            }
        }
    };
    while (k < kmax) {
        ++k;
        bool any_running = false;
        for (size_t b = 0; b < B; ++b) any_running = any_running || running[b];
        if (!any_running) break;
        HPG_HIP(hipMemcpyAsync(uold.p, du, B * nu * sizeof(double), hipMemcpyDeviceToDevice, s));
        for (size_t b = 0; b < B; ++b) {
            conv[b] = 0;
            act[b] = running[b];
            fb_step[b] = 0;
        }
        for (int it = 0; it <= o.max_newton; ++it) {
            residual(du, dp, dpp, alpha_k, dR, s, nu2.data(), np2.data());
            bool any = false;
            for (size_t b = 0; b < B; ++b) {
                if (!act[b]) continue;
                err[b] = std::sqrt(nu2[b]) / (alpha_k * normF[b]) + std::sqrt(np2[b]) / normPhi[b];
                S[b].newton_error = err[b];
                if (!std::isfinite(err[b])) {
                    act[b] = 0;
                } else if (err[b] <= o.newton_tol) {
                    conv[b] = 1;
                    act[b] = 0;
                } else if (it == o.max_newton) {
                    act[b] = 0;
                }
                m0[b] = std::sqrt(nu2[b] / (alpha_k * alpha_k) + np2[b]);
                any = any || act[b];
            }
            if (!any) break;
            std::vector<int> sel32(B, 0), sel64(B, 0);
            bool any32 = false, any64 = false;
            for (size_t b = 0; b < B; ++b) {
                acc[b] = 0;
                need64[b] = 0;
                if (!act[b]) continue;
                const bool u32 = mixed && fb_step[b] < kBatchMaxFallbacksPerStep &&
                                 recomputed[b] < kBatchMaxFallbacksPerSolve;
                (u32 ? sel32 : sel64)[b] = 1;
                any32 = any32 || u32;
                any64 = any64 || !u32;
                S[b].newton_iters += 1;
                if (mixed && !u32) S[b].fp64_fallbacks += 1;
            }
            // linearise at every request's psi (FP64, and FP32 for a mixed solve)
            setup(dp, alpha_k, o.beta, mixed, s);
            if (any32) {
                directions(sel32, true, o.krylov_rtol);
                for (size_t b = 0; b < B; ++b)
                    need64[b] = sel32[b] && (last_breakdown[b] || last_iters[b] >= o.max_krylov);
            }
            if (any64)
                directions(sel64, false, mixed ? std::min(o.krylov_rtol, kBatchFallbackRtol)
                                               : o.krylov_rtol);
            std::vector<int> ls(B, 0), none(B, 0);
            for (size_t b = 0; b < B; ++b) ls[b] = act[b] && !need64[b];
            line_search(ls, none);
            // FP32 directions that broke down, hit the cap or were rejected by
            // the line search: computed again with the FP64 operator
            std::vector<int> redo(B, 0), kept(B, 0);
            bool any_redo = false;
            for (size_t b = 0; b < B; ++b) {
                redo[b] = sel32[b] && (need64[b] || !acc[b]);
                kept[b] = acc[b];
                any_redo = any_redo || redo[b];
            }
            if (any_redo) {
                residual(du, dp, dpp, alpha_k, dR, s, a2.data(), b2.data());
                directions(redo, false, std::min(o.krylov_rtol, kBatchFallbackRtol));
                for (size_t b = 0; b < B; ++b)
                    if (redo[b]) {
                        S[b].fp64_fallbacks += 1;
                        S[b].fp64_recomputations += 1;
                        fb_step[b] += 1;
                        recomputed[b] += 1;
                    }
                line_search(redo, kept);
            }
            // requests without an accepted step leave the Newton loop: converged
            // at the stall tolerance, or failed
            for (size_t b = 0; b < B; ++b) {
                if (!act[b]) continue;
                if (!acc[b]) {
                    conv[b] = err[b] <= o.stall_tol;
                    act[b] = 0;
                }
            }
            // the trial buffers take every request's step (t = 0 where none was
            // accepted: an exact copy), then become the current iterates
            for (size_t b = 0; b < B; ++b)
                if (!acc[b]) t[b] = 0.0;
            trial();
            std::swap(du, dut);
            std::swap(dp, dpt);
        }
        // outer step: per request
        for (size_t b = 0; b < B; ++b) stop_now[b] = 0;
        l2_diff(du, uold.as<double>(), s, diff.data(), nrm.data());
        std::vector<int> lm(B, 0);
        for (size_t b = 0; b < B; ++b) {
            if (!running[b]) continue;
            S[b].prox_steps = k;
            S[b].alpha_last = alpha_k;
            if (!conv[b]) {
                S[b].status = HPG_NOT_CONVERGED;
                stop_now[b] = 1;
            } else {
                const bool last = k == kmax;
                stop_now[b] = o.fixed_prox_steps > 0 ? last : (diff[b] <= o.prox_tol * nrm[b] || last);
            }
            lm[b] = stop_now[b];
        }
        upload_mask(lm);
        hipLaunchKernelGGL(k_lambda_masked, gp, dim3(256), 0, s, np, dmask, dpp, dp, alpha_k,
                           lam.as<double>());
        HPG_HIP(hipMemcpyAsync(dpp, dp, B * np * sizeof(double), hipMemcpyDeviceToDevice, s));
        for (size_t b = 0; b < B; ++b)
            if (stop_now[b]) running[b] = 0;
        alpha_k = std::min(alpha_k * o.alpha_factor, o.alpha_max);
    }
    if (d_u_out) HPG_HIP(hipMemcpyAsync(d_u_out, du, B * nu * 8, hipMemcpyDeviceToDevice, s));
    if (d_psi_out) HPG_HIP(hipMemcpyAsync(d_psi_out, dp, B * np * 8, hipMemcpyDeviceToDevice, s));
    if (d_lam_out)
        HPG_HIP(hipMemcpyAsync(d_lam_out, lam.p, B * np * 8, hipMemcpyDeviceToDevice, s));
    // diagnostics of every request (one launch)
    {
        constexpr int kDiagBlocks = 1024;
        const int nbl = (int)std::min<int64_t>(ncell, kDiagBlocks);
        dev::DiagBatch db;
        db.nb = nb;
        db.u = nu;
        db.psi = np;
        db.qp = nqp;
        double* dg = diagp.as<double>();
        dev::launch_diag(P.geo, P.tab64.view(), P.Du64.as<double>(), du, dp, lam.as<double>(),
                         PhiQ.as<double>(), dg, nbl, s, db);
        HPG_HIP(hipGetLastError());
        std::vector<double> h(B * 3 * nbl);
        HPG_HIP(hipMemcpyAsync(h.data(), dg, h.size() * 8, hipMemcpyDeviceToHost, s));
        HPG_HIP(hipStreamSynchronize(s));
        for (size_t b = 0; b < B; ++b) {
            double c = 0.0, l1 = 0.0, mv = -std::numeric_limits<double>::infinity();
            for (int i = 0; i < nbl; ++i) {
                const double* e = h.data() + (b * nbl + i) * 3;
                c += e[0];
                l1 += e[1];
                mv = std::max(mv, e[2]);
            }
            S[b].complementarity = c;
            S[b].complementarity_rel = c / std::max(l1 * phimax[b], 1e-300);
            S[b].max_violation = mv;
        }
    }
    HPG_HIP(hipStreamSynchronize(s));
    // keep the batch's buffers pointing at the final iterates
    if (du != u.as<double>()) u.swap(ut);
    if (dp != psi.as<double>()) psi.swap(pt);
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    hpg_status worst = HPG_OK;
    for (size_t b = 0; b < B; ++b) {
        S[b].seconds = sec;
        if (S[b].status != HPG_OK) worst = S[b].status;
        if (stats) stats[b] = S[b];
    }
    return worst;
}

}  // namespace hpg

struct hpg_batch {
    hpg::Batch B;
    int op_prec = HPG_FP64;
    bool op_ready = false;
};

using namespace hpg;

extern "C" {

hpg_status hpg_create_batch(const hpg_mesh* mesh, int32_t nbatch, int device, hpg_batch** out) {
    return guarded([&]() -> hpg_status {
        if (!mesh || !out) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        if (nbatch < 1 || nbatch > (1 << 20)) fail(HPG_ERR_INVALID_ARG, "nbatch must be 1..2^20");
        auto* b = new hpg_batch();
        try {
            b->B.build(mesh->M, nbatch, device);
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
        return HPG_OK;
    });
}

void hpg_destroy_batch(hpg_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->B.P.device);
    delete b;
}

static void check_batch(hpg_batch* b) {
    if (!b) fail(HPG_ERR_INVALID_ARG, "batch handle is NULL");
    HPG_HIP(hipSetDevice(b->B.P.device));
}

hpg_status hpg_batch_set_data(hpg_batch* b, const double* f_qp, const double* phi_qp,
                              size_t n_values) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        Batch& Bt = b->B;
        if (!f_qp || !phi_qp) fail(HPG_ERR_INVALID_ARG, "NULL data");
        if (n_values != (size_t)Bt.nb * (size_t)Bt.nqp)
            fail(HPG_ERR_INVALID_ARG, "f and phi need nbatch * n_qp values each");
        for (size_t i = 0; i < n_values; ++i)
            if (!std::isfinite(f_qp[i]) || !std::isfinite(phi_qp[i]))
                fail(HPG_ERR_NUMERIC, "non-finite f or phi");
        Bt.set_data(f_qp, phi_qp);
        return HPG_OK;
    });
}

hpg_status hpg_batch_solve(hpg_batch* b, const hpg_solve_opts* opts, double* u_out,
                           double* psi_out, double* lam_out, hpg_solve_stats* stats) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        hpg_solve_opts o = checked_opts(opts);
        Batch& Bt = b->B;
        hipStream_t s = Bt.P.own_stream;
        const hpg_status st = Bt.solve(o, s, stats, nullptr, nullptr, nullptr);
        const size_t B = (size_t)Bt.nb;
        if (u_out)
            HPG_HIP(hipMemcpy(u_out, Bt.u.p, B * Bt.nu * sizeof(double), hipMemcpyDeviceToHost));
        if (psi_out)
            HPG_HIP(hipMemcpy(psi_out, Bt.psi.p, B * Bt.np * sizeof(double), hipMemcpyDeviceToHost));
        if (lam_out)
            HPG_HIP(hipMemcpy(lam_out, Bt.lam.p, B * Bt.np * sizeof(double), hipMemcpyDeviceToHost));
        b->op_ready = false;   // the solve's linearisation replaced the operator's
        return st;
    });
}

hpg_status hpg_batch_op_setup(hpg_batch* b, const double* d_psi, double alpha, double beta,
                              int32_t precision, void* stream) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        if (!d_psi) fail(HPG_ERR_INVALID_ARG, "psi is NULL");
        if (!(alpha > 0) || !(beta >= 0)) fail(HPG_ERR_INVALID_ARG, "alpha > 0, beta >= 0");
        if (precision != HPG_FP64 && precision != HPG_MIXED)
            fail(HPG_ERR_INVALID_ARG, "precision must be HPG_FP64 or HPG_MIXED");
        hipStream_t s = (hipStream_t)stream;
        b->B.setup(d_psi, alpha, beta, precision == HPG_MIXED, s);
        HPG_HIP(hipStreamSynchronize(s));
        b->op_prec = precision;
        b->op_ready = true;
        return HPG_OK;
    });
}

hpg_status hpg_batch_op_apply_G(hpg_batch* b, const void* d_x, void* d_y, void* stream) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        if (!b->op_ready) fail(HPG_ERR_INVALID_ARG, "operator not set up (hpg_batch_op_setup)");
        if (!d_x || !d_y || d_x == d_y) fail(HPG_ERR_INVALID_ARG, "x, y must be distinct buffers");
        hipStream_t s = (hipStream_t)stream;
        Batch& Bt = b->B;
        Bt.gpart.alloc((size_t)Bt.nb * Bt.PS * sizeof(double));
        if (b->op_prec == HPG_FP64)
            Bt.apply_G<double>((const double*)d_x, (double*)d_y, nullptr, nullptr, s);
        else
            Bt.apply_G<float>((const float*)d_x, (float*)d_y, nullptr, nullptr, s);
        HPG_HIP(hipGetLastError());
        HPG_HIP(hipStreamSynchronize(s));
        return HPG_OK;
    });
}

hpg_status hpg_batch_set_kernel_timing(hpg_batch* b, const char* group) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        Problem& P = b->B.P;
        HPG_HIP(hipDeviceSynchronize());
        P.timing = group != nullptr;
        P.timing_group = group ? group : "";
        for (auto& kv : P.groups) kv.second.used = 0;
        return HPG_OK;
    });
}

hpg_status hpg_batch_kernel_time(hpg_batch* b, const char* group, int64_t* launches,
                                 double* total_ms) {
    return guarded([&]() -> hpg_status {
        check_batch(b);
        if (!group || !launches || !total_ms) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        Problem& P = b->B.P;
        *launches = 0;
        *total_ms = 0.0;
        auto it = P.groups.find(group);
        if (it == P.groups.end()) return HPG_OK;
        HPG_HIP(hipDeviceSynchronize());
        double tot = 0.0;
        for (size_t i = 0; i < it->second.used; ++i) {
            float ms = 0.f;
            HPG_HIP(hipEventElapsedTime(&ms, it->second.start[i], it->second.stop[i]));
            tot += ms;
        }
        *launches = (int64_t)it->second.used;
        *total_ms = tot;
        return HPG_OK;
    });
}

}  // extern "C"
