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
#include <cstdio>
#include <cstdlib>
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

// lam_b = (psi_prev_b - psi_b) / alpha_b for the requests with mask_b = 1
// (alpha_b = prm[4 b])
__global__ __launch_bounds__(256) void k_lambda_masked(int64_t n, const int* __restrict__ mask,
                                                       const double* __restrict__ pp,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ prm,
                                                       double* __restrict__ lam) {
    const int64_t b = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mask[b]) lam[b * n + i] = (pp[b * n + i] - p[b * n + i]) / prm[4 * b];
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
    // the requests (host, after projection) and the slots' device copies
    int nreq = 0;
    std::vector<double> hF, hPhi, hPhiQ, rnormF, rnormPhi, rphimax;
    DBuf F, Phi, PhiQ, cclass_rep;
    std::vector<double> normF, normPhi, phimax;
    bool have_data = false;
    // results per request
    std::vector<double> ru, rpsi, rlam;
    std::vector<hpg_solve_stats> rstats;
    // per-request (alpha, beta, 1 / alpha, 0) of the current linearisation
    DBuf prm;
    std::vector<double> hprm;
    // linearisation (FP64 always; FP32 as well for mixed solves)
    DBuf om64, om32, s64, s32;
    DBuf sflag;   // mixed: cells whose FP32 psi-block apply uses s64 (kFp32CondLimit)
    // MINRES engines: FP64 and FP32 work vectors, right-hand sides, solutions
    // and per-request states (two parities each)
    BKrylov<double> k64;
    BKrylov<float> k32;
    DBuf rhs64, rhs32, kst64, kst32;
    DBuf part, gpart, mask, mask2, tvec, diagp;
    // Newton state
    DBuf u, psi, pp, ut, pt, R, uold, d64, lam;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<dev::KState> hst;

    ~Batch() {
        if (P.own_stream) (void)hipStreamSynchronize(P.own_stream);
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    }
    void build(const Mesh& M, int nbatch, int device);
    void set_data(const double* f, const double* phi, int nrequests);
    void upload_prm(hipStream_t s);
    void setup(const double* d_psi, const int* d_mask, bool want32, hipStream_t s);
    template <typename T>
    void apply_G(const T* x, T* y, double* gp, const int* done, hipStream_t s);
    template <typename T>
    void apply_prec(const T* r, T* z, double* pr, const int* done, int dstride, hipStream_t s);
    template <typename T>
    void iterations(int count, T*& vcur, T*& vprev, T*& wprev, T*& wcur, T* q, T* Gq, T* z, T* x,
                    hipStream_t s);
    template <typename T>
    void ensure_engine();
    template <typename T>
    void start(const std::vector<int>& entrants, double rtol, int maxit, hipStream_t s);
    template <typename T>
    void chunk(int count, hipStream_t s);
    template <typename T>
    void poll(hipStream_t s);
    void residual(const double* uu, const double* ps, const double* ppv, double* RR,
                  hipStream_t s, double* nu2, double* np2);
    void l2_diff(const double* a, const double* b, hipStream_t s, double* d, double* nrm);
    hpg_status solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* st);
    template <typename T>
    BKrylov<T>& kw();
    template <typename T>
    dev::KState* kst();
    template <typename T>
    T* rhs();
    static int kstride() { return (int)(sizeof(dev::KState) / sizeof(int)); }
};

template <>
BKrylov<double>& Batch::kw<double>() { return k64; }
template <>
BKrylov<float>& Batch::kw<float>() { return k32; }
template <>
dev::KState* Batch::kst<double>() { return kst64.as<dev::KState>(); }
template <>
dev::KState* Batch::kst<float>() { return kst32.as<dev::KState>(); }
template <>
double* Batch::rhs<double>() { return rhs64.as<double>(); }
template <>
float* Batch::rhs<float>() { return rhs32.as<float>(); }

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
    kst64.alloc(2 * B * sizeof(dev::KState));
    kst32.alloc(2 * B * sizeof(dev::KState));
    mask.alloc(B * sizeof(int));
    mask2.alloc(B * sizeof(int));
    tvec.alloc(B * sizeof(double));
    diagp.alloc(B * 3 * 1024 * sizeof(double));
    prm.alloc(B * 4 * sizeof(double));
    hprm.assign(B * 4, 0.0);
    hst.resize(B);
}

void Batch::set_data(const double* f, const double* phi, int nrequests) {
    // each request's F, Phi and phi at the Gauss points, through the shared
    // problem's own (host) projection of the data; the slots load them as
    // they take the requests
    const size_t Rn = (size_t)nrequests, B = (size_t)nb;
    nreq = nrequests;
    hF.assign(Rn * nu, 0.0);
    hPhi.assign(Rn * np, 0.0);
    hPhiQ.assign(phi, phi + Rn * nqp);
    rnormF.assign(Rn, 1.0);
    rnormPhi.assign(Rn, 1.0);
    rphimax.assign(Rn, 0.0);
    for (size_t r = 0; r < Rn; ++r) {
        P.set_data(f + r * nqp, phi + r * nqp);
        HPG_HIP(hipMemcpy(hF.data() + r * nu, P.F.p, nu * sizeof(double), hipMemcpyDeviceToHost));
        HPG_HIP(hipMemcpy(hPhi.data() + r * np, P.Phi.p, np * sizeof(double), hipMemcpyDeviceToHost));
        rnormF[r] = P.normF;
        rnormPhi[r] = P.normPhi;
        rphimax[r] = P.phi_absmax;
    }
    F.alloc(B * nu * sizeof(double));
    Phi.alloc(B * np * sizeof(double));
    PhiQ.alloc(B * nqp * sizeof(double));
    normF.assign(B, 1.0);
    normPhi.assign(B, 1.0);
    phimax.assign(B, 0.0);
    have_data = true;
}

void Batch::upload_prm(hipStream_t s) {
    HPG_HIP(hipMemcpyAsync(prm.p, hprm.data(), hprm.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
}

// linearisation of the requests with d_mask[b] != 0 (all if null) at their
// psi with their own (alpha, beta) from prm
void Batch::setup(const double* d_psi, const int* d_mask, bool want32, hipStream_t s) {
    const size_t B = (size_t)nb;
    const size_t nq = (size_t)ncell * P.geo.Qd, ns = (size_t)ncell * P.geo.Pd * P.geo.Pd;
    om64.alloc(B * nq * sizeof(double));
    s64.alloc(B * ns * sizeof(double));
    if (want32) {
        om32.alloc(B * nq * sizeof(float));
        s32.alloc(B * ns * sizeof(float));
        sflag.alloc(B * (size_t)ncell * sizeof(int));
    }
    // the cells of all requests in one launch: psi, the weights and the blocks
    // are request-major, the cell geometry repeats per request
    dev::Geo gb = P.geo;
    gb.n_cells = (int64_t)nb * ncell;
    P.tstart("setup", s);
    dev::launch_setup(gb, P.tab64.view(), P.cpb_setup, dev::SETUP_LDS, d_psi, 1.0, 0.0,
                      P.C.as<double>(), cclass_rep.as<int>(), om64.as<double>(),
                      want32 ? om32.as<float>() : nullptr, s64.as<double>(),
                      want32 ? s32.as<float>() : nullptr, s, prm.as<double>(), d_mask, ncell,
                      want32 ? sflag.as<int>() : nullptr, 1);
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
    bt.prm = 4;
    const T* om = BSel<T>::prec == HPG_FP64 ? (const T*)om64.p : (const T*)om32.p;
    const dev::KernelEvents ke = P.kernel_events("apply_G");
    dev::launch_tile<T>(P.geo, r, BSel<T>::tabs(P).view(), (T)1, (T)0, prm.as<double>(), x,
                        x + nu, nullptr, om, nullptr, nullptr, y, y + nu, gp, done,
                        dev::MODE_APPLY, s, &ke, bt);
}

template <typename T>
void Batch::apply_prec(const T* r, T* z, double* pr, const int* done, int dstride, hipStream_t s) {
    P.ensure_fdm();
    BKrylov<T>& K = kw<T>();
    const DevFdm<T>& Fd = BSel<T>::fdm(P);
    T* t1 = K.t1.template as<T>();
    T* t2 = K.t2.template as<T>();
    const T* sinv = BSel<T>::prec == HPG_FP64 ? (const T*)s64.p : (const T*)s32.p;
    const Mesh& M = P.M;
    const int d = M.d, npass = 2 * d, Pd = P.geo.Pd;
    dev::PsiBatch pb;
    pb.nb = nb;
    pb.sinv = (int64_t)ncell * dev::psi_block_size(Pd, 1);   // packed blocks
    pb.r = pb.z = n;
    pb.part = PS;
    pb.done = dstride;
    pb.flag = ncell;
    dev::PsiHi hi;
    hi.packed = 1;
    if (BSel<T>::prec == HPG_MIXED) {
        hi.s64 = s64.as<double>();
        hi.flag = sflag.as<int>();
    }
    const T* src = r;
    int pass = 0;
    for (int ph = 0; ph < 2; ++ph) {
        for (int k = 0; k < d; ++k) {
            ++pass;
            T* dst = (pass == npass) ? z : ((src == t1) ? t2 : t1);
            dev::GemmEpi<T> ep{};
            ep.ts = P.fdm_tile<T>();
            if (ph == 0 && k == d - 1) {
                ep.scale_mode = d;
                ep.n0 = M.n1[0];
                ep.l0 = Fd.lam[0].template as<T>();
                ep.l1 = Fd.lam[1].template as<T>();
                ep.l2 = Fd.lam[2].template as<T>();
                ep.prm = prm.as<double>();
                ep.prmstride = 4;
            }
            if (pass == npass) {
                ep.dotv = r;
                ep.partial = pr;
            }
            ep.pstride = PS;
            ep.dstride = dstride;
            const int N = M.n1[k];
            const int64_t ss = src == r ? n : nu, ds = dst == z ? n : nu;
            if (k == 0) {
                const T* Bm = ph == 0 ? Fd.V[k].template as<T>() : Fd.Vt[k].template as<T>();
                const int R = (int)(nu / N);
                ep.bdiv = 1;
                if (pass == 1) {
                    dev::launch_gemm_prec<T>(R, N, N, src, N, Bm, N, dst, N, done, ep, ncell, Pd,
                                             P.cpb_prec, sinv, r + nu, z + nu,
                                             pr ? pr + P.np_dot : nullptr, s, ss, ds, pb, hi);
                } else {
                    const dev::KernelEvents ke = P.kernel_events("fdm");   // one GEMM per event pair
                    dev::launch_gemm<T>(R, N, N, src, N, ss, Bm, N, 0, dst, N, ds, nb, done, ep, s,
                                        &ke);
                }
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
                const dev::KernelEvents ke = P.kernel_events("fdm");
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
    dev::KState* st = kst<T>();
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
        apply_prec<T>(vhat, z, pr, dn, kstride(), s);
        P.tstart("minres_vec", s);
        dev::launch_kr_update<T>(n, cur, nxt, pr, npP, q, wprev, wcur, x, vprev, vhat, z, s, vp);
        P.tstop("minres_vec", s);
        std::swap(vprev, vcur);
        std::swap(wprev, wcur);
        par = 1 - par;
    }
}

template <typename T>
void Batch::ensure_engine() {
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
    K.x.alloc(bytes);
    K.t1.alloc(bu);
    K.t2.alloc(bu);
    (BSel<T>::prec == HPG_FP64 ? rhs64 : rhs32).alloc(bytes);
}

// MINRES starts for the requests flagged in entrants (their right-hand side
// -R from the residual buffer); the other requests' states are untouched, so
// the ones in the middle of their own MINRES go on where they are
template <typename T>
void Batch::start(const std::vector<int>& entrants, double rtol, int maxit, hipStream_t s) {
    ensure_engine<T>();
    BKrylov<T>& K = kw<T>();
    int& ts = P.fdm_ts<T>();
    if (!ts) {
        // the GEMM tile of this batch size, timed on zero vectors before the
        // first Krylov graph is captured
        const int* ign = mask2.as<int>();
        HPG_HIP(hipMemsetAsync(mask2.p, 0, nb * sizeof(int), s));
        HPG_HIP(hipMemsetAsync(K.vhat.p, 0, (size_t)nb * n * sizeof(T), s));
        const bool tm = P.timing;
        P.timing = false;
        ts = pick_gemm_tile(
            s,
            [&](int c) {
                ts = c;
                apply_prec<T>(K.vhat.template as<T>(), K.Gq.template as<T>(), nullptr, ign, 1, s);
            },
            sizeof(T) == 4 ? "batched FP32 preconditioner" : "batched FP64 preconditioner");
        P.timing = tm;
    }
    T* b = rhs<T>();
    int* dm = mask.as<int>();
    int* skip = mask2.as<int>();
    std::vector<int> sk(entrants.size());
    for (size_t i = 0; i < entrants.size(); ++i) sk[i] = entrants[i] ? 0 : 1;
    HPG_HIP(hipMemcpyAsync(dm, entrants.data(), entrants.size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
    HPG_HIP(hipMemcpyAsync(skip, sk.data(), sk.size() * sizeof(int), hipMemcpyHostToDevice, s));
    dev::launch_convert<double, T>((int64_t)nb * n, R.as<double>(), b, -1.0, s);
    double* pr = part.as<double>();
    apply_prec<T>(b, K.z.template as<T>(), pr, skip, 1, s);
    dev::VecBatch vp;
    vp.nb = nb;
    vp.v = n;
    vp.part = PS;
    vp.mask = dm;
    dev::launch_kr_start<T>(n, kst<T>(), pr, P.np_dot + P.np_prec, rtol, maxit, b,
                            K.z.template as<T>(), K.vcur.template as<T>(),
                            K.vprev.template as<T>(), K.q.template as<T>(),
                            K.wprev.template as<T>(), K.wcur.template as<T>(),
                            K.x.template as<T>(), s, vp);
    HPG_HIP(hipGetLastError());
}

// count (even) MINRES iterations of every running request, replayed from a
// captured graph (kernel timing: launched directly)
template <typename T>
void Batch::chunk(int count, hipStream_t s) {
    BKrylov<T>& K = kw<T>();
    T* vcur = K.vcur.template as<T>();
    T* vprev = K.vprev.template as<T>();
    T* wprev = K.wprev.template as<T>();
    T* wcur = K.wcur.template as<T>();
    T* q = K.q.template as<T>();
    T* Gq = K.Gq.template as<T>();
    T* z = K.z.template as<T>();
    T* x = K.x.template as<T>();
    if (P.timing) {
        iterations<T>(count, vcur, vprev, wprev, wcur, q, Gq, z, x, s);
        return;
    }
    const GraphKey key{BSel<T>::prec, count, (const void*)rhs<T>(), (const void*)x};
    auto it = graphs.find(key);
    hipGraphExec_t exec;
    if (it == graphs.end()) {
        hipGraph_t g;
        std::lock_guard<std::recursive_mutex> api(device_api_mutex());
        HPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        iterations<T>(count, vcur, vprev, wprev, wcur, q, Gq, z, x, s);
        HPG_HIP(hipStreamEndCapture(s, &g));
        HPG_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
        HPG_HIP(hipGraphDestroy(g));
        graphs[key] = exec;
    } else {
        exec = it->second;
    }
    HPG_HIP(hipGraphLaunch(exec, s));
}

// every request's MINRES state after an even chunk (in the first parity)
template <typename T>
void Batch::poll(hipStream_t s) {
    HPG_HIP(hipMemcpyAsync(hst.data(), kst<T>(), (size_t)nb * sizeof(dev::KState),
                           hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
}

void Batch::residual(const double* uu, const double* ps, const double* ppv, double* RR,
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
    bt.prm = 4;
    double* pr = part.as<double>();
    P.tstart("residual", s);
    dev::launch_tile<double>(P.geo, r, P.tab64.view(), 1.0, 0.0, prm.as<double>(), uu, ps, ppv,
                             nullptr, F.as<double>(), Phi.as<double>(), RR, RR + nu, pr, nullptr,
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
constexpr int kBatchChunk = 16;

// Every request runs its own proximal / Newton / line-search sequence (that
// of Problem::solve) at its own pace: in each round of the loop the requests
// that need a residual get one (one launch for all), those whose direction is
// due start MINRES (setup and start for them alone), every request in MINRES
// advances by one chunk (one graph of launches per precision), and the
// requests whose MINRES ended take their line search (one launch per trial
// for all of them) and move on.  A request therefore never waits for the
// Krylov solves of the others.
hpg_status Batch::solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* stats) {
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
    double* du = u.as<double>();
    double* dp = psi.as<double>();
    double* dut = ut.as<double>();
    double* dpt = pt.as<double>();
    double* dpp = pp.as<double>();
    double* dR = R.as<double>();
    double* dd = d64.as<double>();
    int* dmask = mask.as<int>();
    double* dt = tvec.as<double>();
    HPG_HIP(hipMemsetAsync(du, 0, B * nu * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(uold.p, 0, B * nu * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(dp, 0, B * np * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(dpp, 0, B * np * sizeof(double), s));
    HPG_HIP(hipMemsetAsync(lam.p, 0, B * np * sizeof(double), s));
    std::vector<hpg_solve_stats> S(B);
    for (auto& x : S) {
        std::memset(&x, 0, sizeof(x));
        x.status = HPG_OK;
    }
    enum Phase { TOP, REDO, KRYLOV, SEARCH, STEP_END, DONE };
    std::vector<int> ph(B, TOP), k(B, 1), it(B, 0), conv(B, 0), fb_step(B, 0), recomputed(B, 0);
    std::vector<int> eng32(B, 0), first32(B, 0), halv(B, 0);
    std::vector<double> alpha(B, o.alpha0), err(B, 0.0), m0(B, 0.0), t(B, 0.0);
    std::vector<double> nu2(B), np2(B), a2(B), b2(B), diff(B), nrm(B);
    auto set_prm = [&](size_t b) {
        hprm[4 * b] = alpha[b];
        hprm[4 * b + 1] = o.beta;
        hprm[4 * b + 2] = 1.0 / alpha[b];
        hprm[4 * b + 3] = 0.0;
    };
    // requests are taken by the slots in order; a slot whose request finishes
    // takes the next one
    const size_t Rn = (size_t)nreq;
    ru.assign(Rn * nu, 0.0);
    rpsi.assign(Rn * np, 0.0);
    rlam.assign(Rn * np, 0.0);
    rstats.assign(Rn, hpg_solve_stats{});
    std::vector<int> slot_req(B, -1);
    std::vector<std::chrono::steady_clock::time_point> t_load(B, t0);
    int next = 0;
    auto load = [&](size_t b, int r) {
        slot_req[b] = r;
        t_load[b] = std::chrono::steady_clock::now();
        HPG_HIP(hipMemcpyAsync(F.as<double>() + b * nu, hF.data() + (size_t)r * nu,
                               nu * sizeof(double), hipMemcpyHostToDevice, s));
        HPG_HIP(hipMemcpyAsync(Phi.as<double>() + b * np, hPhi.data() + (size_t)r * np,
                               np * sizeof(double), hipMemcpyHostToDevice, s));
        HPG_HIP(hipMemcpyAsync(PhiQ.as<double>() + b * nqp, hPhiQ.data() + (size_t)r * nqp,
                               nqp * sizeof(double), hipMemcpyHostToDevice, s));
        normF[b] = rnormF[r];
        normPhi[b] = rnormPhi[r];
        phimax[b] = rphimax[r];
        HPG_HIP(hipMemsetAsync(du + b * nu, 0, nu * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(uold.as<double>() + b * nu, 0, nu * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(dp + b * np, 0, np * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(dpp + b * np, 0, np * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(lam.as<double>() + b * np, 0, np * sizeof(double), s));
        std::memset(&S[b], 0, sizeof(S[b]));
        S[b].status = HPG_OK;
        ph[b] = TOP;
        k[b] = 1;
        it[b] = 0;
        conv[b] = 0;
        fb_step[b] = 0;
        recomputed[b] = 0;
        eng32[b] = 0;
        alpha[b] = o.alpha0;
        set_prm(b);
    };
    for (size_t b = 0; b < B; ++b) {
        if (next < nreq) {
            load(b, next++);
        } else {
            ph[b] = DONE;
            alpha[b] = o.alpha0;
            set_prm(b);
        }
    }
    upload_prm(s);
    auto upload_mask = [&](const std::vector<int>& m) {
        HPG_HIP(hipMemcpyAsync(dmask, m.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
    };
    const dim3 gu(blocks_of(nu), (unsigned)nb), gp(blocks_of(np), (unsigned)nb),
        gn(blocks_of(n), (unsigned)nb);
    auto count = [&](int p) {
        size_t c = 0;
        for (size_t b = 0; b < B; ++b) c += ph[b] == p;
        return c;
    };
    const double rtol64 = mixed ? std::min(o.krylov_rtol, kBatchFallbackRtol) : o.krylov_rtol;
    bool run64 = false, run32 = false;   // an engine with requests in MINRES
    int rounds = 0, chunks = 0, searches = 0, starts = 0;
    while (count(DONE) < B) {
        ++rounds;
        // ---- A: residuals; Newton stops; MINRES starts
        if (count(TOP) + count(REDO) > 0) {
            residual(du, dp, dpp, dR, s, nu2.data(), np2.data());
            std::vector<int> e32(B, 0), e64(B, 0);
            for (size_t b = 0; b < B; ++b) {
                if (ph[b] == TOP) {
                    err[b] = std::sqrt(nu2[b]) / (alpha[b] * normF[b]) + std::sqrt(np2[b]) / normPhi[b];
                    S[b].newton_error = err[b];
                    if (!std::isfinite(err[b])) {
                        conv[b] = 0;
                        ph[b] = STEP_END;
                    } else if (err[b] <= o.newton_tol) {
                        conv[b] = 1;
                        ph[b] = STEP_END;
                    } else if (it[b] == o.max_newton) {
                        conv[b] = 0;
                        ph[b] = STEP_END;
                    } else {
                        m0[b] = std::sqrt(nu2[b] / (alpha[b] * alpha[b]) + np2[b]);
                        const bool u32 = mixed && fb_step[b] < kBatchMaxFallbacksPerStep &&
                                         recomputed[b] < kBatchMaxFallbacksPerSolve;
                        S[b].newton_iters += 1;
                        if (mixed && !u32) S[b].fp64_fallbacks += 1;
                        eng32[b] = u32;
                        (u32 ? e32 : e64)[b] = 1;
                        ph[b] = KRYLOV;
                    }
                } else if (ph[b] == REDO) {
                    // an FP32 direction that broke down, hit the cap or was
                    // rejected: computed again with the FP64 operator
                    S[b].fp64_fallbacks += 1;
                    S[b].fp64_recomputations += 1;
                    fb_step[b] += 1;
                    recomputed[b] += 1;
                    eng32[b] = 0;
                    e64[b] = 1;
                    ph[b] = KRYLOV;
                }
            }
            bool any32 = false, any64 = false;
            std::vector<int> ent(B, 0);
            for (size_t b = 0; b < B; ++b) {
                ent[b] = e32[b] | e64[b];
                any32 = any32 || e32[b];
                any64 = any64 || e64[b];
            }
            if (any32 || any64) {
                upload_mask(ent);
                setup(dp, dmask, mixed, s);
                ++starts;
            }
            if (any32) {
                start<float>(e32, o.krylov_rtol, o.max_krylov, s);
                run32 = true;
            }
            if (any64) {
                start<double>(e64, rtol64, o.max_krylov, s);
                run64 = true;
            }
        }
        // ---- B: ends of proximal steps
        if (count(STEP_END) > 0) {
            l2_diff(du, uold.as<double>(), s, diff.data(), nrm.data());
            std::vector<int> lm(B, 0), adv(B, 0);
            for (size_t b = 0; b < B; ++b) {
                if (ph[b] != STEP_END) continue;
                S[b].prox_steps = k[b];
                S[b].alpha_last = alpha[b];
                bool stop;
                if (!conv[b]) {
                    S[b].status = HPG_NOT_CONVERGED;
                    stop = true;
                } else {
                    const bool last = k[b] == kmax;
                    stop = o.fixed_prox_steps > 0 ? last : (diff[b] <= o.prox_tol * nrm[b] || last);
                }
                lm[b] = 1;   // lambda of this step (kept only by the stopping requests)
                if (stop) {
                    ph[b] = DONE;
                } else {
                    adv[b] = 1;
                }
            }
            // lambda_k and psi_prev <- psi, u_old <- u for the requests that go on
            upload_mask(lm);
            hipLaunchKernelGGL(k_lambda_masked, gp, dim3(256), 0, s, np, dmask, dpp, dp,
                               prm.as<double>(), lam.as<double>());
            hipLaunchKernelGGL((k_copy_masked<double>), gp, dim3(256), 0, s, np, dmask, dp, dpp);
            upload_mask(adv);
            hipLaunchKernelGGL((k_copy_masked<double>), gu, dim3(256), 0, s, nu, dmask, du,
                               uold.as<double>());
            // finished requests: diagnostics, results, and the slot takes the next request
            std::vector<size_t> fin;
            for (size_t b = 0; b < B; ++b)
                if (lm[b] && !adv[b]) fin.push_back(b);
            if (!fin.empty()) {
                constexpr int kDiagBlocks = 1024;
                const int nbl = (int)std::min<int64_t>(ncell, kDiagBlocks);
                dev::DiagBatch db;
                db.nb = nb;
                db.u = nu;
                db.psi = np;
                db.qp = nqp;
                double* dg = diagp.as<double>();
                dev::launch_diag(P.geo, P.tab64.view(), P.Du64.as<double>(), du, dp,
                                 lam.as<double>(), PhiQ.as<double>(), dg, nbl, s, db);
                HPG_HIP(hipGetLastError());
                std::vector<double> h(B * 3 * nbl);
                HPG_HIP(hipMemcpyAsync(h.data(), dg, h.size() * 8, hipMemcpyDeviceToHost, s));
                for (size_t b : fin) {
                    const size_t r = (size_t)slot_req[b];
                    HPG_HIP(hipMemcpyAsync(ru.data() + r * nu, du + b * nu, nu * 8,
                                           hipMemcpyDeviceToHost, s));
                    HPG_HIP(hipMemcpyAsync(rpsi.data() + r * np, dp + b * np, np * 8,
                                           hipMemcpyDeviceToHost, s));
                    HPG_HIP(hipMemcpyAsync(rlam.data() + r * np, lam.as<double>() + b * np, np * 8,
                                           hipMemcpyDeviceToHost, s));
                }
                HPG_HIP(hipStreamSynchronize(s));
                const auto now = std::chrono::steady_clock::now();
                for (size_t b : fin) {
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
                    S[b].seconds = std::chrono::duration<double>(now - t_load[b]).count();
                    rstats[(size_t)slot_req[b]] = S[b];
                    slot_req[b] = -1;
                    if (next < nreq) load(b, next++);
                }
            }
            for (size_t b = 0; b < B; ++b) {
                if (!adv[b]) continue;
                k[b] += 1;
                alpha[b] = std::min(alpha[b] * o.alpha_factor, o.alpha_max);
                set_prm(b);
                it[b] = 0;
                fb_step[b] = 0;
                ph[b] = TOP;
            }
            upload_prm(s);
            continue;   // the advanced requests need their first residual
        }
        // ---- C: one chunk of MINRES iterations per engine in use
        std::vector<int> fin(B, 0);
        for (int e = 0; e < 2; ++e) {
            const bool f32 = e == 1;
            if (!(f32 ? run32 : run64)) continue;
            ++chunks;
            if (f32) {
                chunk<float>(kBatchChunk, s);
                poll<float>(s);
            } else {
                chunk<double>(kBatchChunk, s);
                poll<double>(s);
            }
            bool still = false;
            std::vector<int> harvest(B, 0);
            for (size_t b = 0; b < B; ++b) {
                if (ph[b] != KRYLOV || eng32[b] != (int)f32) continue;
                if (!hst[b].done) {
                    still = true;
                    continue;
                }
                S[b].krylov_iters += hst[b].iters;
                harvest[b] = 1;
                fin[b] = 1;
                const bool need64 = f32 && (hst[b].breakdown || hst[b].iters >= o.max_krylov);
                if (need64) {
                    ph[b] = REDO;
                    harvest[b] = 0;
                } else {
                    first32[b] = f32;
                    ph[b] = SEARCH;
                    t[b] = 1.0;
                    halv[b] = 0;
                }
            }
            upload_mask(harvest);
            if (f32)
                hipLaunchKernelGGL((k_copy_masked<float>), gn, dim3(256), 0, s, n, dmask,
                                   k32.x.as<float>(), dd);
            else
                hipLaunchKernelGGL((k_copy_masked<double>), gn, dim3(256), 0, s, n, dmask,
                                   k64.x.as<double>(), dd);
            (f32 ? run32 : run64) = still;
        }
        (void)fin;
        // ---- D: line searches of the requests whose direction is in
        while (count(SEARCH) > 0) {
            ++searches;
            std::vector<double> tt(B, 0.0);
            for (size_t b = 0; b < B; ++b) tt[b] = ph[b] == SEARCH ? t[b] : 0.0;
            HPG_HIP(hipMemcpyAsync(dt, tt.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL((k_axpy_strided<double>), gu, dim3(256), 0, s, nu, du, nu, dt, dd,
                               n, dut, nu);
            hipLaunchKernelGGL((k_axpy_strided<double>), gp, dim3(256), 0, s, np, dp, np, dt,
                               dd + nu, n, dpt, np);
            residual(dut, dpt, dpp, dR, s, a2.data(), b2.data());
            std::vector<int> acc(B, 0);
            bool any_acc = false;
            for (size_t b = 0; b < B; ++b) {
                if (ph[b] != SEARCH) continue;
                const double m1 = std::sqrt(a2[b] / (alpha[b] * alpha[b]) + b2[b]);
                if (m1 <= (1.0 - 1e-4 * t[b]) * m0[b]) {
                    acc[b] = 1;
                    any_acc = true;
                } else if (halv[b] == 30) {
                    if (first32[b]) {
                        ph[b] = REDO;   // the FP32 direction is recomputed once in FP64
                    } else {
                        conv[b] = err[b] <= o.stall_tol;
                        ph[b] = STEP_END;
                    }
                } else {
                    t[b] *= 0.5;
                    halv[b] += 1;
                    S[b].line_search_halvings += 1;
                }
            }
            if (any_acc) {
                // accepted steps: the trial iterates become the current ones
                upload_mask(acc);
                hipLaunchKernelGGL((k_copy_masked<double>), gu, dim3(256), 0, s, nu, dmask, dut,
                                   du);
                hipLaunchKernelGGL((k_copy_masked<double>), gp, dim3(256), 0, s, np, dmask, dpt,
                                   dp);
                for (size_t b = 0; b < B; ++b)
                    if (acc[b]) {
                        it[b] += 1;
                        ph[b] = TOP;
                    }
            }
        }
    }
    HPG_HIP(hipStreamSynchronize(s));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (std::getenv("HPG_TRACE"))
        std::fprintf(stderr, "hpg batch: %d requests, %.3f s, %d rounds, %d setups, %d chunks, %d "
                             "line-search trials\n", nb, sec, rounds, starts, chunks, searches);
    hpg_status worst = HPG_OK;
    for (size_t r = 0; r < Rn; ++r) {
        if (rstats[r].status != HPG_OK) worst = rstats[r].status;
        if (stats) stats[r] = rstats[r];
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
        if (n_values == 0 || n_values % (size_t)Bt.nqp != 0 ||
            n_values / (size_t)Bt.nqp > (size_t)(1 << 30))
            fail(HPG_ERR_INVALID_ARG, "f and phi need a positive multiple of n_qp values each");
        for (size_t i = 0; i < n_values; ++i)
            if (!std::isfinite(f_qp[i]) || !std::isfinite(phi_qp[i]))
                fail(HPG_ERR_NUMERIC, "non-finite f or phi");
        Bt.set_data(f_qp, phi_qp, (int)(n_values / (size_t)Bt.nqp));
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
        const hpg_status st = Bt.solve(o, s, stats);
        if (u_out) std::memcpy(u_out, Bt.ru.data(), Bt.ru.size() * sizeof(double));
        if (psi_out) std::memcpy(psi_out, Bt.rpsi.data(), Bt.rpsi.size() * sizeof(double));
        if (lam_out) std::memcpy(lam_out, Bt.rlam.data(), Bt.rlam.size() * sizeof(double));
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
        Batch& Bt = b->B;
        for (int r = 0; r < Bt.nb; ++r) {
            Bt.hprm[4 * r] = alpha;
            Bt.hprm[4 * r + 1] = beta;
            Bt.hprm[4 * r + 2] = 1.0 / alpha;
            Bt.hprm[4 * r + 3] = 0.0;
        }
        Bt.upload_prm(s);
        Bt.setup(d_psi, nullptr, precision == HPG_MIXED, s);
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
