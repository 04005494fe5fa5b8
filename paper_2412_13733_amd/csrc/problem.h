// Problem state of the hpG library: device tables, data and work buffers.
#pragma once

#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "hp_host.h"
#include "hpg_internal.h"
#include "kernels.h"

struct hpg_mesh {
    hpg::Mesh M;
};

namespace hpg {

// device buffer with RAII
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int device = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf();
    // exchange the underlying blocks (pointer, size and device together)
    void swap(DBuf& o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(device, o.device);
    }
    void alloc(size_t b);
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

template <typename T>
struct DevRows {
    DBuf lenM, colM, aM, mM, lenB, cellB, modeB, vB, win, lenG, cellG, modeG, vG;
    dev::URows<T> view() const;
};

template <typename T>
struct DevTabs {
    DBuf B1, Vpsi, Vu, w, Mdiag, h[3], G1, AY, MY;
    dev::PsiTabs<T> view() const;
};

template <typename T>
struct DevFdm {
    DBuf V[3], Vt[3], lam[3];
};

// MINRES workspace of one precision (vhat: the next Lanczos vector before
// normalisation)
template <typename T>
struct KrylovWork {
    DBuf z, vcur, vprev, vhat, q, Gq, wprev, wcur, t1, t2;
    int64_t n = 0;
    void ensure(int64_t n_, int64_t n_u);
};

// the Lanczos step folded into the preconditioner's first launch: its input
// vhat = Gq - delta vcur - gamma vprev is formed there from the G-apply
// partials gpart (npg of them) and the MINRES state st, and stored to vhat
template <typename T>
struct VhatIn {
    dev::KState* st;
    const double* gpart;
    int npg;
    const T* Gq;
    const T* vcur;
    const T* vprev;
    T* vhat;
};

struct TimingGroup {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
};

struct GraphKey {
    int prec, chunk;
    const void* b;
    const void* x;
    bool operator<(const GraphKey& o) const {
        return std::tie(prec, chunk, b, x) < std::tie(o.prec, o.chunk, o.b, o.x);
    }
};

// HPG_GEMM_TILE as a tile (1 or 2), else fallback
int forced_gemm_tile(int fallback);

struct Problem {
    Mesh M;
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t side = nullptr;            // second stream for the concurrent psi-side work
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_enter = nullptr, ev_leave = nullptr;
    bool use_graphs = true;
    // every launch on the one stream (no fork/join onto the side stream): the
    // default, since a captured fork/join cost more per Krylov iteration than
    // the overlap it bought (measured), and required for problems solved
    // concurrently by the server, where waits between streams that share
    // hardware queues with other problems' streams could block them
    bool single_stream = true;
    bool use_tile = false;                 // fused tiled G apply / residual available for (d, p)
    std::map<GraphKey, hipGraphExec_t> graphs;
    bool fdm_dot_fused = true;
    DBuf params;                           // alpha, beta, 1/alpha of the linearisation
    double hparams[4] = {1.0, 0.0, 1.0, 0.0};
    dev::Geo geo{};
    int cpb_psi = 1, cpb_setup = 1, cpb_l2 = 1, cpb_prec = 1;
    DevRows<double> rows64[3];
    DevRows<float> rows32[3];
    DevTabs<double> tab64;
    DevTabs<float> tab32;
    DevFdm<double> fdm64;
    DevFdm<float> fdm32;
    DBuf C, cclass;
    // one degree per cell (M.hp): host tables, their device copies, the cell
    // kernels' geometry, and the coarse (vertex) fast diagonalisation
    HpHost hph;
    struct HpDev {
        DBuf cell_p, loc_off, psi_off, qp_off, sinv_off, loc2glob, inc_ptr, inc_idx, order;
        DBuf item_start, item_count, item_p, cclass, c_off, C, vert, ent_first, ent_n, ent_off;
        DBuf ent_list, ent_cstart, ent_ccount;
        DBuf inv64, inv32, tab64, tab32, toff, h64[3], h32[3], yloc64, yloc32, cv64, cv32;
    } hpd;
    dev::HpGeo hgeo{};
    dev::HpEnt hent{};
    int hp_lds_elems = 256, hp_nmax = 1, np_gath = 0, np_cell = 0, np_hpl2 = 0;
    size_t hp_setup_bytes = 0;
    bool hp_setup_in_lds = false;
    struct HpRun {
        int p, first, count;   // cells order[first .. first + count) have degree p
    };
    std::vector<HpRun> hp_runs;
    DevFdm<double> cfdm64;
    DevFdm<float> cfdm32;
    int hp_smax = 1, hp_item_elems = 256;  // (p_max+1)^d; the tuned work-item budget
    void build_hp();
    void set_hp_items(int item_elems);
    void tune_hp_items();
    void ensure_fdm_hp();
    void set_data_hp(const double* f, const double* phi);
    template <typename T>
    dev::HpTabs<T> hp_tabs() const;
    template <typename T>
    void apply_G_hp(const T* x, T* y, double* part, const int* dn, hipStream_t s);
    template <typename T>
    void apply_prec_hp(const T* r, T* z, double* part, const int* dn, hipStream_t s);
    // data
    std::vector<double> f_qp, phi_qp;
    bool have_f = false, have_phi = false;
    DBuf F, Phi;
    DBuf PhiQ;                             // phi at the Gauss points (FP64)
    double phi_absmax = 0.0;               // max |phi| over the Gauss points
    DBuf Du64;                             // q x (p+1) reference derivatives of the u basis
    DBuf diag_part;                        // per-block sums of the solve diagnostics
    bool gradient = false;                 // constraint |grad u| <= phi
    bool prec_big = false;                 // psi blocks streamed from HBM (too large for LDS)
    int setup_mode = 0;                    // obstacle Schur blocks: dev::SETUP_LDS / _HBM_T2 / _HBM
    double normF = 1.0, normPhi = 1.0;
    // linearisation (hpg_op_setup / Newton setup)
    double alpha = 1.0, beta = 0.0;
    int precision = HPG_FP64;
    bool linearised = false;
    DBuf om64, om32, sinv64, sinv32;
    DBuf sflag;   // mixed: per cell, 1 if its psi-block is applied from sinv64 (kFp32CondLimit)
    // Krylov
    KrylovWork<double> kw64;
    KrylovWork<float> kw32;
    DBuf partial, partial_g, kstate;       // partial_g: the G apply's partial sums
    int np_u = 0, np_psi = 0, np_dot = 0, np_prec = 0, np_cap = 0;
    // Newton state
    DBuf u, psi, psi_prev, ut, pt, R, u_old, delta64, delta32, rhs32, xk64;
    DBuf ux, px;   // trial iterate of an extended Newton step
    // timing
    bool timing = false;
    std::string timing_group;
    std::map<std::string, TimingGroup> groups;

    // device-buffer calls run on the caller's stream; NULL is the HIP null stream
    hipStream_t stream(void* s) const { return (hipStream_t)s; }
    size_t lds_max = 65536;
    void build(const Mesh& mesh, int device);
    void set_data(const double* f, const double* phi);
    void ensure_work();
    void ensure_linearisation_buffers();
    bool fdm_ready = false;
    void ensure_fdm();
    // block tile of the fast-diagonalisation GEMMs per Krylov precision (0:
    // FP64, 1: FP32): 1 (16x16) or 2 (32x32), 0 until tuned on this problem
    int gemm_ts[2] = {0, 0};
    template <typename T>
    int& fdm_ts() {
        return gemm_ts[sizeof(T) == 4 ? 1 : 0];
    }
    // the tile in use: the tuned one, else HPG_GEMM_TILE, else 16x16
    template <typename T>
    int fdm_tile() {
        const int t = fdm_ts<T>();
        return t ? t : forced_gemm_tile(1);
    }
    template <typename T>
    void tune_fdm(hipStream_t s);

    // operations (all enqueue on stream s)
    void setup(const double* d_psi, double alpha, double beta, int precision, hipStream_t s);
    template <typename T>
    void apply_G(const T* x, T* y, double* partial, const int* done, hipStream_t s);
    template <typename T>
    void apply_prec(const T* r, T* z, double* partial, const int* done, hipStream_t s,
                    const VhatIn<T>* vin = nullptr);
    // the FP64 blocks of the ill-conditioned cells for an FP32 psi-block apply
    // (uniform-degree obstacle meshes with LDS-formed blocks; empty otherwise)
    bool flags_psi() const { return !M.hp && !gradient && !setup_mode; }
    // psi-block inverses stored packed (upper triangle): the same meshes,
    // with blocks applied from LDS
    bool packed_psi() const { return flags_psi() && !prec_big; }
    template <typename T>
    dev::PsiHi psi_hi() const {
        dev::PsiHi h;
        if (sizeof(T) == 4 && flags_psi() && sflag.p) {
            h.s64 = sinv64.as<double>();
            h.flag = sflag.as<int>();
        }
        h.packed = packed_psi() ? 1 : 0;
        return h;
    }
    template <typename T>
    int minres(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t s);
    template <typename T>
    int minres_on(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t s);
    template <typename T>
    void minres_iterations(int count, int par0, T*& vcur, T*& vprev, T*& wprev, T*& wcur, T* q,
                           T* Gq, T* z, T* x, hipStream_t s);
    void fork(hipStream_t s);
    void join(hipStream_t s);
    // residual into R; returns (||R_u||^2, ||R_psi||^2) (synchronises).  With sc
    // the partial sums (residual_partials() values), the per-local-function
    // values of a per-cell-degree mesh (residual_local_values()) and the host
    // copy of the partials use the caller's memory and nothing is allocated.
    struct ResScratch {
        double* part;   // device
        double* yloc;   // device (per-cell degrees only)
        double* host;   // host
    };
    void residual(const double* u, const double* psi, const double* psi_prev, double alpha,
                  double* R, hipStream_t s, double* nu2, double* np2,
                  const ResScratch* sc = nullptr);
    int residual_partials() const;
    int64_t residual_local_values() const;
    double l2_diff(const double* a, const double* b, double* norm_a, hipStream_t s);
    void diagnostics(const double* u, const double* psi, const double* lam, hipStream_t s,
                     double* cr, double* cr_rel, double* mv);
    hpg_status solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* st, double* d_u_out,
                     double* d_psi_out, double* d_lam_out);
    int newton_direction64(const double* dR, double* dd, double eta, const hpg_solve_opts& o,
                           hipStream_t s);
    bool last_minres_breakdown = false;    // the last MINRES stopped on a breakdown

    // events for one timed launch of group grp (recorded by the dispatch), or
    // none when the group is not being timed
    dev::KernelEvents kernel_events(const char* grp);
    void tstart(const char* grp, hipStream_t s);
    void tstop(const char* grp, hipStream_t s);
    ~Problem();
};

}  // namespace hpg

namespace hpg {
template <typename TO>
std::vector<TO> cast(const std::vector<double>& v) {
    return std::vector<TO>(v.begin(), v.end());
}
// bytes hipMalloc'ed by DBuf on the calling thread (accounting for the server)
size_t& device_bytes_counter();
// serialises the calls that act on the whole device (allocation, synchronous
// copies, stream/graph creation and destruction) with graph capture, so that
// problems solved on several host threads never invalidate each other's capture
std::recursive_mutex& device_api_mutex();
// device memory of one problem's solve at the given precision (upper estimate)
size_t footprint_bytes(const Mesh& M, int precision);
size_t footprint_bytes_hp(const Mesh& M, int precision);
// blocking host -> device copy into a freshly sized buffer
template <typename T>
void upload(DBuf& d, const std::vector<T>& h) {
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    d.alloc(h.size() * sizeof(T));
    if (!h.empty()) HPG_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}
// solve options with defaults filled in and validated (throws Error)
hpg_solve_opts checked_opts(const hpg_solve_opts* in);
// The faster GEMM block tile (1: 16x16, 2: 32x32) for run(ts), the work of
// one preconditioner apply enqueued on s, timed after a warm-up.  The tiles
// sum in the same order, so this picks a time and never a result.
// HPG_GEMM_TILE=16 or 32 forces a tile.
int pick_gemm_tile(hipStream_t s, const std::function<void(int)>& run, const char* what);

}  // namespace hpg

struct hpg_problem {
    hpg::Problem P;
};
