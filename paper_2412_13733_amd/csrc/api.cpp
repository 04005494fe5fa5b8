// extern "C" entry points of the hpG library (declared in include/hpg.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "problem.h"

namespace hpg {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }
[[noreturn]] void fail(hpg_status code, const std::string& msg) { throw Error{code, msg}; }

static void check_problem(hpg_problem* p) {
    if (!p) fail(HPG_ERR_INVALID_ARG, "problem handle is NULL");
    HPG_HIP(hipSetDevice(p->P.device));
}

hpg_solve_opts checked_opts(const hpg_solve_opts* in) {
    hpg_solve_opts o;
    hpg_default_opts(&o);
    if (in) {
        if (in->size != (int32_t)sizeof(hpg_solve_opts))
            fail(HPG_ERR_INVALID_ARG, "hpg_solve_opts.size mismatch");
        o = *in;
    }
    if (!(o.alpha0 > 0) || !(o.alpha_factor >= 1.0) || !(o.alpha_max > 0))
        fail(HPG_ERR_INVALID_ARG, "alpha schedule must be positive and non-decreasing");
    if (o.max_prox < 1 || o.max_newton < 1 || o.max_krylov < 1 || o.krylov_chunk < 1)
        fail(HPG_ERR_INVALID_ARG, "iteration caps must be >= 1");
    if (!(o.newton_tol > 0) || !(o.krylov_rtol > 0) || !(o.prox_tol >= 0))
        fail(HPG_ERR_INVALID_ARG, "tolerances must be positive");
    if (o.precision != HPG_FP64 && o.precision != HPG_MIXED)
        fail(HPG_ERR_INVALID_ARG, "precision must be HPG_FP64 or HPG_MIXED");
    if (!(o.beta >= 0)) fail(HPG_ERR_INVALID_ARG, "beta must be >= 0");
    if (o.step_extension != 0 && o.step_extension != 1)
        fail(HPG_ERR_INVALID_ARG, "step_extension must be 0 or 1");
    if (o.krylov != HPG_KRYLOV_MINRES) fail(HPG_ERR_INVALID_ARG, "krylov must be HPG_KRYLOV_MINRES");
    if (o.q < 0) fail(HPG_ERR_INVALID_ARG, "q must be 0 (p + 1) or p + 1");
    if ((o.warm_u == nullptr) != (o.warm_psi == nullptr))
        fail(HPG_ERR_INVALID_ARG, "warm start needs both warm_u and warm_psi");
    if (o.k0 < 0 || (o.k0 > 0 && !o.warm_u))
        fail(HPG_ERR_INVALID_ARG, "k0 must be >= 0, and 0 without a warm start");
    return o;
}

}  // namespace hpg

using namespace hpg;

extern "C" {

const char* hpg_last_error(void) { return hpg::g_last_error.c_str(); }

hpg_status hpg_create_mesh(int dim, const int32_t* ncells, const double* const* breaks,
                           const int32_t* degree, int32_t p, int32_t constraint, hpg_mesh** out) {
    return guarded([&]() -> hpg_status {
        if (!out) fail(HPG_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (dim < 1 || dim > 3) fail(HPG_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
        if (!ncells) fail(HPG_ERR_INVALID_ARG, "ncells is NULL");
        if (constraint != HPG_OBSTACLE && constraint != HPG_GRADIENT)
            fail(HPG_ERR_INVALID_ARG, "constraint must be HPG_OBSTACLE or HPG_GRADIENT");
        int64_t ncell_total = 1;
        for (int k = 0; k < dim; ++k) {
            if (ncells[k] < 1 || ncells[k] > (1 << 20)) fail(HPG_ERR_INVALID_ARG, "ncells out of range");
            ncell_total *= ncells[k];
        }
        std::vector<int32_t> deg;
        int pmin = 0;
        if (degree) {
            // one degree per cell: p is the largest one
            if (constraint != HPG_OBSTACLE)
                fail(HPG_ERR_INVALID_ARG, "per-cell degrees: obstacle constraint only");
            if (ncell_total > (int64_t)1 << 26) fail(HPG_ERR_INVALID_ARG, "too many cells");
            deg.assign(degree, degree + ncell_total);
            p = 0;
            pmin = 1 << 30;
            for (int32_t v : deg) {
                if (v < 2 || v > 24) fail(HPG_ERR_INVALID_ARG, "per-cell degree outside 2..24");
                p = std::max(p, v);
                pmin = std::min(pmin, v);
            }
        }
        if (constraint == HPG_OBSTACLE && p < 2)
            fail(HPG_ERR_INVALID_ARG, "obstacle constraint needs p >= 2");
        if (constraint == HPG_GRADIENT && p < 1)
            fail(HPG_ERR_INVALID_ARG, "gradient constraint needs p >= 1");
        if (p > 24) fail(HPG_ERR_INVALID_ARG, "p > 24 is not supported");
        auto* m = new hpg_mesh();
        Mesh& M = m->M;
        M.d = dim;
        M.p = p;
        M.q = p + 1;
        M.kind = constraint;
        M.P = constraint == HPG_OBSTACLE ? p - 1 : p;
        M.ncomp = constraint == HPG_OBSTACLE ? 1 : dim;
        for (int k = 0; k < dim; ++k) {
            if (ncells[k] < 1 || ncells[k] > (1 << 20)) {
                delete m;
                fail(HPG_ERR_INVALID_ARG, "ncells out of range");
            }
            M.m[k] = ncells[k];
            M.breaks[k].resize(ncells[k] + 1);
            for (int c = 0; c <= ncells[k]; ++c) {
                double v = breaks && breaks[k] ? breaks[k][c] : (double)c / ncells[k];
                if (!std::isfinite(v)) {
                    delete m;
                    fail(HPG_ERR_INVALID_ARG, "non-finite breakpoint");
                }
                M.breaks[k][c] = v;
            }
            if (breaks && breaks[k]) {
                if (std::fabs(M.breaks[k][0]) > 1e-14 || std::fabs(M.breaks[k][ncells[k]] - 1.0) > 1e-14) {
                    delete m;
                    fail(HPG_ERR_INVALID_ARG, "breakpoints must start at 0 and end at 1");
                }
                for (int c = 0; c < ncells[k]; ++c)
                    if (!(M.breaks[k][c + 1] > M.breaks[k][c])) {
                        delete m;
                        fail(HPG_ERR_INVALID_ARG, "breakpoints must be strictly increasing");
                    }
            }
            M.n1[k] = ncells[k] * p - 1;
            if (M.n1[k] < 1) {
                // only p = 1 on one cell: the H^1_0 space in that direction is empty
                delete m;
                fail(HPG_ERR_INVALID_ARG, "ncells * p must be at least 2 in every direction");
            }
        }
        M.n_cells = 1;
        M.n_u = 1;
        M.Pd = M.Qd = M.Ld = 1;
        for (int k = 0; k < dim; ++k) {
            M.n_cells *= M.m[k];
            M.n_u *= M.n1[k];
            M.Pd *= M.P;
            M.Qd *= M.q;
            M.Ld *= (p + 1);
        }
        M.psi_per_cell = M.ncomp * M.Pd;
        M.n_psi = M.n_cells * M.psi_per_cell;
        M.n_qp = M.n_cells * M.Qd;
        M.ref.build(p, M.P, M.q);
        if (degree) {
            M.hp = true;
            M.pmin = pmin;
            M.deg = std::move(deg);
            hp_number(M);
            if (M.n_u >= ((int64_t)1 << 31) || M.n_psi >= ((int64_t)1 << 40)) {
                delete m;
                fail(HPG_ERR_INVALID_ARG, "mesh too large");
            }
        }
        *out = m;
        return HPG_OK;
    });
}

void hpg_destroy_mesh(hpg_mesh* mesh) { delete mesh; }

hpg_status hpg_get_mesh_info(const hpg_mesh* mesh, hpg_mesh_info* out) {
    return guarded([&]() -> hpg_status {
        if (!mesh || !out) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        const Mesh& M = mesh->M;
        out->dim = M.d;
        out->p = M.p;
        out->q = M.q;
        out->P = M.P;
        out->constraint = M.kind;
        for (int k = 0; k < 3; ++k) out->ncells[k] = k < M.d ? M.m[k] : 1;
        out->n_cells = M.n_cells;
        out->n_u = M.n_u;
        out->n_psi = M.n_psi;
        out->n_qp = M.n_qp;
        return HPG_OK;
    });
}

hpg_status hpg_quadrature_points(const hpg_mesh* mesh, double* xyz) {
    return guarded([&]() -> hpg_status {
        if (!mesh || !xyz) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        const Mesh& M = mesh->M;
        const int d = M.d;
        if (M.hp) {
            // cell-major, each cell with its own q_K = p_K + 1 points per direction
            std::vector<std::vector<double>> nodes(M.p + 2);
            for (int64_t c = 0; c < M.n_cells; ++c) {
                const int q = M.deg[c] + 1;
                if (nodes[q].empty()) {
                    std::vector<double> w;
                    gauss_legendre(q, nodes[q], w);
                }
                int64_t t = c;
                int cc[3] = {0, 0, 0};
                for (int k = 0; k < d; ++k) {
                    cc[k] = (int)(t % M.m[k]);
                    t /= M.m[k];
                }
                const int64_t Qd = M.qp_off[c + 1] - M.qp_off[c];
                for (int64_t j = 0; j < Qd; ++j) {
                    int jj[3] = {(int)(j % q), (int)((j / q) % q), (int)(j / ((int64_t)q * q))};
                    double* o = xyz + (M.qp_off[c] + j) * d;
                    for (int k = 0; k < d; ++k)
                        o[k] = M.breaks[k][cc[k]] + 0.5 * (nodes[q][jj[k]] + 1.0) * M.h(k, cc[k]);
                }
            }
            return HPG_OK;
        }
        const int q = M.q;
        for (int64_t c = 0; c < M.n_cells; ++c) {
            int64_t t = c;
            int cc[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) {
                cc[k] = (int)(t % M.m[k]);
                t /= M.m[k];
            }
            for (int64_t j = 0; j < M.Qd; ++j) {
                int jj[3] = {(int)(j % q), (int)((j / q) % q), (int)(j / ((int64_t)q * q))};
                double* o = xyz + (c * M.Qd + j) * d;
                for (int k = 0; k < d; ++k)
                    o[k] = M.breaks[k][cc[k]] + 0.5 * (M.ref.y[jj[k]] + 1.0) * M.h(k, cc[k]);
            }
        }
        return HPG_OK;
    });
}

hpg_status hpg_create_problem(const hpg_mesh* mesh, int device, hpg_problem** out) {
    return guarded([&]() -> hpg_status {
        if (!mesh || !out) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        auto* p = new hpg_problem();
        try {
            p->P.build(mesh->M, device);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return HPG_OK;
    });
}

void hpg_destroy_problem(hpg_problem* prob) {
    if (!prob) return;
    (void)hipSetDevice(prob->P.device);
    (void)hipStreamSynchronize(prob->P.own_stream);
    delete prob;
}

static void check_values(const double* v, size_t n, size_t want, const char* what) {
    if (!v) fail(HPG_ERR_INVALID_ARG, std::string(what) + " is NULL");
    if (n != want) fail(HPG_ERR_INVALID_ARG, std::string(what) + ": wrong number of values");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) fail(HPG_ERR_NUMERIC, std::string(what) + ": non-finite value");
}

hpg_status hpg_set_forcing(hpg_problem* prob, const double* f_qp, size_t n_qp) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        check_values(f_qp, n_qp, (size_t)prob->P.M.n_qp, "f");
        prob->P.set_data(f_qp, nullptr);
        return HPG_OK;
    });
}

hpg_status hpg_set_obstacle(hpg_problem* prob, const double* phi_qp, size_t n_qp) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        check_values(phi_qp, n_qp, (size_t)prob->P.M.n_qp, "phi");
        if (prob->P.M.kind == HPG_GRADIENT)
            for (size_t i = 0; i < n_qp; ++i)
                if (!(phi_qp[i] > 0.0)) fail(HPG_ERR_INVALID_ARG, "gradient constraint needs phi > 0");
        prob->P.set_data(nullptr, phi_qp);
        return HPG_OK;
    });
}

// values of fn at the problem's quadrature points (host)
static std::vector<double> eval_at_points(hpg_problem* prob, hpg_point_fn fn, void* ctx) {
    if (!fn) fail(HPG_ERR_INVALID_ARG, "fn is NULL");
    const Mesh& M = prob->P.M;
    hpg_mesh tmp;
    tmp.M = M;
    std::vector<double> x((size_t)M.n_qp * M.d), v((size_t)M.n_qp);
    const hpg_status st = hpg_quadrature_points(&tmp, x.data());
    if (st != HPG_OK) fail(st, "quadrature points");
    for (int64_t i = 0; i < M.n_qp; ++i) v[i] = fn(x.data() + i * M.d, ctx);
    return v;
}

hpg_status hpg_set_forcing_fn(hpg_problem* prob, hpg_point_fn fn, void* ctx) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        const std::vector<double> v = eval_at_points(prob, fn, ctx);
        return hpg_set_forcing(prob, v.data(), v.size());
    });
}

hpg_status hpg_set_obstacle_fn(hpg_problem* prob, hpg_point_fn fn, void* ctx) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        const std::vector<double> v = eval_at_points(prob, fn, ctx);
        return hpg_set_obstacle(prob, v.data(), v.size());
    });
}

void hpg_default_opts(hpg_solve_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->size = sizeof(hpg_solve_opts);
    o->alpha0 = 2.0;
    o->alpha_factor = 2.0;
    o->alpha_max = 1e300;
    o->max_prox = 60;
    o->prox_tol = 1e-10;
    o->fixed_prox_steps = 0;
    o->newton_tol = 1e-12;
    o->stall_tol = 1e-9;
    o->max_newton = 60;
    o->krylov_rtol = 1e-10;
    o->max_krylov = 2000;
    o->beta = 0.0;
    o->precision = HPG_FP64;
    o->krylov_chunk = 16;
    o->inexact_newton = 0;
    o->step_extension = 0;
    o->q = 0;
    o->krylov = HPG_KRYLOV_MINRES;
    o->warm_u = nullptr;
    o->warm_psi = nullptr;
    o->k0 = 0;
}


hpg_status hpg_solve(hpg_problem* prob, const hpg_solve_opts* opts, double* u_out,
                     double* psi_out, double* lam_out, hpg_solve_stats* stats) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        hpg_solve_opts o = checked_opts(opts);
        Problem& P = prob->P;
        hipStream_t s = P.own_stream;
        DBuf lam;
        if (lam_out) lam.alloc(P.M.n_psi * sizeof(double));
        hpg_status st = P.solve(o, s, stats, nullptr, nullptr, lam_out ? lam.as<double>() : nullptr);
        if (u_out)
            HPG_HIP(hipMemcpy(u_out, P.u.p, P.M.n_u * sizeof(double), hipMemcpyDeviceToHost));
        if (psi_out)
            HPG_HIP(hipMemcpy(psi_out, P.psi.p, P.M.n_psi * sizeof(double), hipMemcpyDeviceToHost));
        if (lam_out)
            HPG_HIP(hipMemcpy(lam_out, lam.p, P.M.n_psi * sizeof(double), hipMemcpyDeviceToHost));
        return st;
    });
}

hpg_status hpg_solve_device(hpg_problem* prob, const hpg_solve_opts* opts, double* d_u,
                            double* d_psi, void* stream, hpg_solve_stats* stats) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        hpg_solve_opts o = checked_opts(opts);
        Problem& P = prob->P;
        return P.solve(o, P.stream(stream), stats, d_u, d_psi, nullptr);   // NULL: null stream
    });
}

hpg_status hpg_op_setup(hpg_problem* prob, const double* d_psi, double alpha, double beta,
                        int32_t precision, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_psi) fail(HPG_ERR_INVALID_ARG, "psi is NULL");
        if (!(alpha > 0) || !(beta >= 0)) fail(HPG_ERR_INVALID_ARG, "alpha > 0, beta >= 0");
        if (precision != HPG_FP64 && precision != HPG_MIXED)
            fail(HPG_ERR_INVALID_ARG, "precision must be HPG_FP64 or HPG_MIXED");
        hipStream_t s = prob->P.stream(stream);
        prob->P.setup(d_psi, alpha, beta, precision, s);
        HPG_HIP(hipStreamSynchronize(s));
        return HPG_OK;
    });
}

hpg_status hpg_op_apply_G(hpg_problem* prob, const void* d_x, void* d_y, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_x || !d_y || d_x == d_y) fail(HPG_ERR_INVALID_ARG, "x, y must be distinct buffers");
        Problem& P = prob->P;
        hipStream_t s = P.stream(stream);
        if (P.precision == HPG_FP64)
            P.apply_G<double>((const double*)d_x, (double*)d_y, nullptr, nullptr, s);
        else
            P.apply_G<float>((const float*)d_x, (float*)d_y, nullptr, nullptr, s);
        HPG_HIP(hipGetLastError());
        HPG_HIP(hipStreamSynchronize(s));
        return HPG_OK;
    });
}

hpg_status hpg_op_apply_prec(hpg_problem* prob, const void* d_r, void* d_z, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_r || !d_z || d_r == d_z) fail(HPG_ERR_INVALID_ARG, "r, z must be distinct buffers");
        Problem& P = prob->P;
        hipStream_t s = P.stream(stream);
        if (P.precision == HPG_FP64)
            P.apply_prec<double>((const double*)d_r, (double*)d_z, nullptr, nullptr, s);
        else
            P.apply_prec<float>((const float*)d_r, (float*)d_z, nullptr, nullptr, s);
        HPG_HIP(hipGetLastError());
        HPG_HIP(hipStreamSynchronize(s));
        return HPG_OK;
    });
}

hpg_status hpg_op_minres(hpg_problem* prob, const void* d_b, void* d_x, double rtol,
                         int32_t max_iters, int32_t* iters, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_b || !d_x || d_b == d_x) fail(HPG_ERR_INVALID_ARG, "b, x must be distinct buffers");
        if (!(rtol > 0) || max_iters < 1) fail(HPG_ERR_INVALID_ARG, "rtol > 0, max_iters >= 1");
        Problem& P = prob->P;
        hipStream_t s = P.stream(stream);
        int it;
        if (P.precision == HPG_FP64)
            it = P.minres<double>((const double*)d_b, (double*)d_x, rtol, max_iters, 16, s);
        else
            it = P.minres<float>((const float*)d_b, (float*)d_x, rtol, max_iters, 16, s);
        if (iters) *iters = it;
        return HPG_OK;
    });
}

hpg_status hpg_op_residual(hpg_problem* prob, const double* d_u, const double* d_psi,
                           const double* d_psi_prev, double alpha, double* d_R, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_u || !d_psi || !d_psi_prev || !d_R) fail(HPG_ERR_INVALID_ARG, "NULL buffer");
        if (!(alpha > 0)) fail(HPG_ERR_INVALID_ARG, "alpha must be > 0");
        Problem& P = prob->P;
        double a, b;
        P.residual(d_u, d_psi, d_psi_prev, alpha, d_R, P.stream(stream), &a, &b);
        (void)a;
        (void)b;
        return HPG_OK;
    });
}

hpg_status hpg_l2_diff(hpg_problem* prob, const double* d_a, const double* d_b, double* diff,
                       double* norm_b, void* stream) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!d_a || !d_b || !diff || !norm_b) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        Problem& P = prob->P;
        *diff = P.l2_diff(d_b, d_a, norm_b, P.stream(stream));
        return HPG_OK;
    });
}

hpg_status hpg_set_kernel_timing(hpg_problem* prob, const char* group) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        Problem& P = prob->P;
        HPG_HIP(hipDeviceSynchronize());
        P.timing = group != nullptr;
        P.timing_group = group ? group : "";
        for (auto& kv : P.groups) kv.second.used = 0;
        return HPG_OK;
    });
}

hpg_status hpg_kernel_time(hpg_problem* prob, const char* group, int64_t* launches,
                           double* total_ms) {
    return guarded([&]() -> hpg_status {
        check_problem(prob);
        if (!group || !launches || !total_ms) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        Problem& P = prob->P;
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
