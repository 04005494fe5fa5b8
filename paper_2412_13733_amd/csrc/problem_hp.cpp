// Problem methods for meshes with one degree per cell (obstacle constraint):
// table upload, data, the operator and the preconditioner.  The A-block of
// the preconditioner is block Jacobi: the vertex unknowns (the Q1 space of the
// mesh, a tensor product) by fast diagonalisation, each edge / face / interior
// entity by its stored inverse; the psi-block is -S_hat_K^{-1} per cell as on
// uniform meshes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "problem.h"

namespace hpg {

static KrylovWork<double>& kw_of(Problem& P, const double*) { return P.kw64; }
static KrylovWork<float>& kw_of(Problem& P, const float*) { return P.kw32; }
static const DevFdm<double>& cfdm_of(const Problem& P, const double*) { return P.cfdm64; }
static const DevFdm<float>& cfdm_of(const Problem& P, const float*) { return P.cfdm32; }

template <typename T>
dev::HpTabs<T> Problem::hp_tabs() const {
    dev::HpTabs<T> t;
    const bool dbl = sizeof(T) == sizeof(double);
    t.base = (dbl ? hpd.tab64 : hpd.tab32).template as<T>();
    t.off = hpd.toff.as<dev::HpTabOff>();
    for (int k = 0; k < 3; ++k) t.h[k] = (dbl ? hpd.h64[k] : hpd.h32[k]).template as<T>();
    return t;
}
template dev::HpTabs<double> Problem::hp_tabs<double>() const;
template dev::HpTabs<float> Problem::hp_tabs<float>() const;

void Problem::build_hp() {
    if (gradient) fail(HPG_ERR_INVALID_ARG, "per-cell degrees: obstacle constraint only");
    int Smax = 1, nmax = 1;
    for (int k = 0; k < M.d; ++k) {
        Smax *= M.p + 1;
        nmax *= M.p - 1;
    }
    hp_lds_elems = std::max(256, Smax);
    if (dev::hp_cell_lds(M.d, hp_lds_elems, M.p + 1, sizeof(double), dev::MODE_RES) > lds_max)
        fail(HPG_ERR_INVALID_ARG, "(p+1)^d too large for the per-cell-degree kernels");
    hp_smax = Smax;
    // Schur blocks formed in LDS when the largest one fits, else in place in HBM
    hp_setup_in_lds = dev::hp_setup_lds(M.d, M.p, true) <= lds_max;
    hp_setup_bytes = dev::hp_setup_lds(M.d, M.p, hp_setup_in_lds);
    if (hp_setup_bytes > lds_max)
        fail(HPG_ERR_INVALID_ARG, "P^d too large for the per-cell-degree Schur block setup");
    hp_nmax = nmax;
    hp_build_host(M, hp_lds_elems, hph);
    const HpHost& H = hph;
    hp_runs.clear();
    for (size_t i = 0; i < H.order.size();) {
        size_t j = i;
        const int p = M.deg[H.order[i]];
        while (j < H.order.size() && M.deg[H.order[j]] == p) ++j;
        hp_runs.push_back({p, (int)i, (int)(j - i)});
        i = j;
    }
    upload(hpd.cell_p, M.deg);
    upload(hpd.loc_off, H.loc_off);
    upload(hpd.psi_off, M.psi_off);
    upload(hpd.qp_off, M.qp_off);
    upload(hpd.sinv_off, H.sinv_off);
    upload(hpd.loc2glob, H.loc2glob);
    upload(hpd.inc_ptr, H.inc_ptr);
    upload(hpd.inc_idx, H.inc_idx);
    upload(hpd.order, H.order);
    upload(hpd.item_start, H.item_start);
    upload(hpd.item_count, H.item_count);
    upload(hpd.item_p, H.item_p);
    upload(hpd.cclass, H.cclass);
    upload(hpd.c_off, H.c_off);
    upload(hpd.C, H.C.empty() ? std::vector<double>(1, 0.0) : H.C);
    upload(hpd.vert, H.vert.empty() ? std::vector<int32_t>(1, 0) : H.vert);
    upload(hpd.ent_first, H.ent_first.empty() ? std::vector<int32_t>(1, 0) : H.ent_first);
    upload(hpd.ent_n, H.ent_n.empty() ? std::vector<int32_t>(1, 0) : H.ent_n);
    upload(hpd.ent_off, H.ent_off.empty() ? std::vector<int64_t>(1, 0) : H.ent_off);
    upload(hpd.ent_list, H.ent_list.empty() ? std::vector<int32_t>(1, 0) : H.ent_list);
    upload(hpd.ent_cstart, H.ent_cstart.empty() ? std::vector<int32_t>(1, 0) : H.ent_cstart);
    upload(hpd.ent_ccount, H.ent_ccount.empty() ? std::vector<int32_t>(1, 0) : H.ent_ccount);
    if ((size_t)std::max(H.ent_lds, hp_nmax) * sizeof(double) + 4096 > lds_max)
        fail(HPG_ERR_INVALID_ARG, "entity blocks too large for the preconditioner's LDS");
    hent.nchunk = (int)H.ent_cstart.size();
    hent.lds = H.ent_lds;
    hent.cstart = hpd.ent_cstart.as<int32_t>();
    hent.ccount = hpd.ent_ccount.as<int32_t>();
    hent.list = hpd.ent_list.as<int32_t>();
    hent.first = hpd.ent_first.as<int32_t>();
    hent.cnt = hpd.ent_n.as<int32_t>();
    hent.off = hpd.ent_off.as<int64_t>();
    upload(hpd.inv64, H.inv.empty() ? std::vector<double>(1, 0.0) : H.inv);
    upload(hpd.inv32, cast<float>(H.inv.empty() ? std::vector<double>(1, 0.0) : H.inv));
    upload(hpd.tab64, H.tab);
    upload(hpd.tab32, cast<float>(H.tab));
    upload(hpd.toff, H.toff);
    for (int k = 0; k < 3; ++k) {
        std::vector<double> hv;
        if (k < M.d)
            for (int c = 0; c < M.m[k]; ++c) hv.push_back(M.h(k, c));
        else
            hv.push_back(2.0);
        upload(hpd.h64[k], hv);
        upload(hpd.h32[k], cast<float>(hv));
    }
    hgeo.d = M.d;
    for (int k = 0; k < 3; ++k) hgeo.m[k] = M.m[k];
    hgeo.n_cells = M.n_cells;
    hgeo.n_u = M.n_u;
    hgeo.n_psi = M.n_psi;
    hgeo.n_items = (int)H.item_p.size();
    hgeo.lds_elems = hp_lds_elems;
    hgeo.lmax = M.p + 1;
    hgeo.cell_p = hpd.cell_p.as<int32_t>();
    hgeo.loc_off = hpd.loc_off.as<int64_t>();
    hgeo.psi_off = hpd.psi_off.as<int64_t>();
    hgeo.qp_off = hpd.qp_off.as<int64_t>();
    hgeo.sinv_off = hpd.sinv_off.as<int64_t>();
    hgeo.loc2glob = hpd.loc2glob.as<int32_t>();
    hgeo.order = hpd.order.as<int32_t>();
    hgeo.item_start = hpd.item_start.as<int32_t>();
    hgeo.item_count = hpd.item_count.as<int32_t>();
    hgeo.item_p = hpd.item_p.as<int32_t>();
    tune_hp_items();
    // reduction layout: G apply = [u sums | psi sums] of the gather blocks
    // (the u / psi halves of the generic layout; both over fixed index ranges,
    // so the sums do not depend on the tuned work items), preconditioner =
    // [dot blocks | psi blocks]
    np_gath = (int)std::max<int64_t>(1, std::min<int64_t>((M.n_u + 255) / 256, 1024));
    np_cell = std::min(hgeo.n_items, 4096);   // one block per work item up to 4096
    np_hpl2 = (int)std::min<int64_t>(M.n_cells, 2048);
    np_u = np_gath;
    np_psi = np_gath;
    // <z_u, r_u>: the entity blocks' shares, then the vertex scatter's
    np_dot = dev::hp_prec_entity_blocks(hent.nchunk) +
             (H.vert.empty() ? 0 : dev::hp_vscatter_blocks((int64_t)H.vert.size()));
    np_prec = (int)std::min<int64_t>(M.n_cells, 4096);
    fdm_dot_fused = false;
    use_tile = false;
    np_cap = std::max({np_u + np_psi, np_dot + np_prec, 2 * np_hpl2});
    partial.alloc((size_t)np_cap * sizeof(double));
    partial_g.alloc((size_t)np_cap * sizeof(double));
    params.alloc(4 * sizeof(double));
    kstate.alloc(2 * sizeof(dev::KState));
}

// Work items of the cell pass (a project-side autotuner): the cell pass is
// timed, as an FP32 G apply on zero data, with items of at most 256, 384, 512,
// 768 and 1024 local functions (more cells per item amortise its barriers, fewer
// give more blocks), and the fastest is kept.  HPG_HP_ITEM_ELEMS fixes it.
void Problem::set_hp_items(int item_elems) {
    const int lds = std::max(item_elems, hp_smax);
    hp_make_items(M, lds, item_elems, hph);
    upload(hpd.item_start, hph.item_start);
    upload(hpd.item_count, hph.item_count);
    upload(hpd.item_p, hph.item_p);
    hp_lds_elems = lds;
    hgeo.n_items = (int)hph.item_p.size();
    hgeo.lds_elems = lds;
    hgeo.item_start = hpd.item_start.as<int32_t>();
    hgeo.item_count = hpd.item_count.as<int32_t>();
    hgeo.item_p = hpd.item_p.as<int32_t>();
    hp_item_elems = item_elems;
}

void Problem::tune_hp_items() {
    std::vector<int> cands;
    if (const char* e = std::getenv("HPG_HP_ITEM_ELEMS")) {
        cands.push_back(std::max(1, std::atoi(e)));
    } else {
        for (int c : {256, 384, 512, 768, 1024})
            if (dev::hp_cell_lds(M.d, std::max(c, hp_smax), M.p + 1, sizeof(double),
                                 dev::MODE_RES) <= lds_max)
                cands.push_back(c);
    }
    if (cands.size() == 1) {
        set_hp_items(cands[0]);
        return;
    }
    const int64_t n = M.n_u + M.n_psi, nloc = hph.loc_off.back();
    DBuf x, y, om, yl;
    x.alloc(n * sizeof(float));
    y.alloc(n * sizeof(float));
    om.alloc(M.n_qp * sizeof(float));
    yl.alloc(nloc * sizeof(float));
    HPG_HIP(hipMemset(x.p, 0, x.bytes));
    HPG_HIP(hipMemset(om.p, 0, om.bytes));
    hipEvent_t e0, e1;
    HPG_HIP(hipEventCreate(&e0));
    HPG_HIP(hipEventCreate(&e1));
    const hipStream_t s = own_stream;
    float best = 1e30f;
    int best_c = cands[0];
    for (int c : cands) {
        set_hp_items(c);
        auto run = [&]() {
            dev::launch_hp_cell<float>(hgeo, hp_tabs<float>(), 1.0f, 0.0f, nullptr, x.as<float>(),
                                       x.as<float>() + M.n_u, nullptr, om.as<float>(), nullptr,
                                       yl.as<float>(), y.as<float>() + M.n_u,
                                       std::min(hgeo.n_items, 4096), nullptr, dev::MODE_APPLY, s);
        };
        run();
        run();
        HPG_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r) run();
        HPG_HIP(hipEventRecord(e1, s));
        HPG_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        HPG_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (std::getenv("HPG_TRACE"))
            std::fprintf(stderr, "[hpg] cell pass with work items of <= %d local functions: "
                                 "%d items, %.1f us\n", c, hgeo.n_items, 1e3 * ms / 5);
        if (ms < best) {
            best = ms;
            best_c = c;
        }
    }
    HPG_HIP(hipEventDestroy(e0));
    HPG_HIP(hipEventDestroy(e1));
    HPG_HIP(hipGetLastError());
    if (best_c != hp_item_elems) set_hp_items(best_c);
}

// Q1 stiffness / mass of the interior vertices of direction k (tridiagonal):
// the hat functions of the hierarchical basis are the Q1 hats
void Problem::ensure_fdm_hp() {
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    if (fdm_ready) return;
    for (int k = 0; k < 3; ++k) {
        std::vector<double> V = {1.0}, lam = {0.0};
        int n = 1;
        if (k < M.d && M.m[k] > 1) {
            n = M.m[k] - 1;
            std::vector<double> A((size_t)n * n, 0.0), B((size_t)n * n, 0.0);
            for (int v = 1; v <= n; ++v) {
                const double hl = M.h(k, v - 1), hr = M.h(k, v);
                const int i = v - 1;
                A[(size_t)i * n + i] = 1.0 / hl + 1.0 / hr;
                B[(size_t)i * n + i] = (hl + hr) / 3.0;
                if (v < n) {
                    A[(size_t)i * n + i + 1] = A[(size_t)(i + 1) * n + i] = -1.0 / hr;
                    B[(size_t)i * n + i + 1] = B[(size_t)(i + 1) * n + i] = hr / 6.0;
                }
            }
            generalized_eig(n, A, B, V, lam);
        }
        std::vector<double> Vt(V.size());
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Vt[(size_t)i * n + j] = V[(size_t)j * n + i];
        upload(cfdm64.V[k], V);
        upload(cfdm64.Vt[k], Vt);
        upload(cfdm64.lam[k], lam);
        upload(cfdm32.V[k], cast<float>(V));
        upload(cfdm32.Vt[k], cast<float>(Vt));
        upload(cfdm32.lam[k], cast<float>(lam));
    }
    const size_t nv = hph.vert.size();
    hpd.cv64.alloc(std::max<size_t>(nv, 1) * sizeof(double));
    hpd.cv32.alloc(std::max<size_t>(nv, 1) * sizeof(float));
    fdm_ready = true;
}

// F_i = (f, v_i) and Phi_i = (phi, zeta_i) cell by cell, with each cell's rule
void Problem::set_data_hp(const double* f, const double* phi) {
    const int d = M.d;
    const HpHost& H = hph;
    std::vector<double> Fh, Ph;
    if (f) Fh.assign(M.n_u, 0.0);
    if (phi) Ph.assign(M.n_psi, 0.0);
    for (int64_t c = 0; c < M.n_cells; ++c) {
        const int p = M.deg[c], L = p + 1, P = p - 1, q = p + 1;
        const RefTables& T = H.ref[p];
        int64_t t = c;
        double J = 1.0;
        for (int k = 0; k < d; ++k) {
            J *= 0.5 * M.h(k, (int)(t % M.m[k]));
            t /= M.m[k];
        }
        const int64_t Qd = M.qp_off[c + 1] - M.qp_off[c];
        std::vector<double> wq(Qd);
        for (int64_t j = 0; j < Qd; ++j) {
            int jj[3] = {(int)(j % q), (int)((j / q) % q), (int)(j / ((int64_t)q * q))};
            double w = J;
            for (int k = 0; k < d; ++k) w *= T.w[jj[k]];
            wq[j] = w;
        }
        if (f) {
            std::vector<double> cur(Qd);
            for (int64_t j = 0; j < Qd; ++j) cur[j] = wq[j] * f[M.qp_off[c] + j];
            int din[3] = {1, 1, 1};
            for (int k = 0; k < d; ++k) din[k] = q;
            for (int k = 0; k < d; ++k) cur = hcontract(cur, d, din, k, L, T.Vu, L, true);
            for (size_t l = 0; l < cur.size(); ++l) {
                const int32_t g = H.loc2glob[H.loc_off[c] + l];
                if (g >= 0) Fh[g] += cur[l];
            }
        }
        if (phi) {
            std::vector<double> cur(Qd);
            for (int64_t j = 0; j < Qd; ++j) cur[j] = wq[j] * phi[M.qp_off[c] + j];
            int din[3] = {1, 1, 1};
            for (int k = 0; k < d; ++k) din[k] = q;
            for (int k = 0; k < d; ++k) cur = hcontract(cur, d, din, k, P, T.Vpsi, P, true);
            for (size_t a = 0; a < cur.size(); ++a) Ph[M.psi_off[c] + a] = cur[a];
        }
    }
    if (f) {
        double s = 0.0;
        for (double v : Fh) s += v * v;
        normF = std::max(std::sqrt(s), 1e-300);
        upload(F, Fh);
        have_f = true;
    }
    if (phi) {
        double s = 0.0;
        for (double v : Ph) s += v * v;
        normPhi = std::max(std::sqrt(s), 1e-300);
        upload(Phi, Ph);
        have_phi = true;
    }
}

template <typename T>
void Problem::apply_G_hp(const T* x, T* y, double* part, const int* dn, hipStream_t s) {
    const bool dbl = sizeof(T) == sizeof(double);
    DBuf& yl = dbl ? hpd.yloc64 : hpd.yloc32;   // sized by ensure_linearisation_buffers
    const T* om = (dbl ? om64 : om32).template as<T>();
    tstart("apply_G", s);
    dev::launch_hp_cell<T>(hgeo, hp_tabs<T>(), (T)alpha, (T)beta, params.as<double>(), x,
                           x + M.n_u, nullptr, om, nullptr, yl.as<T>(), y + M.n_u, np_cell, dn,
                           dev::MODE_APPLY, s);
    dev::launch_hp_gather<T>(M.n_u, hpd.inc_ptr.as<int32_t>(), hpd.inc_idx.as<int32_t>(),
                             yl.as<T>(), nullptr, 0.0, x, y, M.n_psi, x + M.n_u, y + M.n_u, part,
                             np_gath, dn, dev::MODE_APPLY, s);
    tstop("apply_G", s);
}

template <typename T>
void Problem::apply_prec_hp(const T* r, T* z, double* part, const int* dn, hipStream_t s) {
    const bool dbl = sizeof(T) == sizeof(double);
    KrylovWork<T>& kw = kw_of(*this, r);
    kw.ensure(M.n_u + M.n_psi, M.n_u);
    ensure_fdm_hp();
    const DevFdm<T>& F = cfdm_of(*this, r);
    const double* prm = params.as<double>();
    const T* sinv = (dbl ? sinv64 : sinv32).template as<T>();
    const T* inv = (dbl ? hpd.inv64 : hpd.inv32).template as<T>();
    const int64_t nv = (int64_t)hph.vert.size();
    const int ne = dev::hp_prec_entity_blocks(hent.nchunk);
    T* cv = (dbl ? hpd.cv64 : hpd.cv32).template as<T>();
    const int32_t* vidx = hpd.vert.as<int32_t>();
    // 2-D vertex grids up to 64 x 64: gather, solve and scatter in one workgroup
    const bool vs2 = nv > 0 && M.d == 2 && hph.nv[0] <= 64 && hph.nv[1] <= 64 &&
                     dev::hp_vsolve2_lds(hph.nv[0], hph.nv[1], sizeof(T)) <= lds_max;
    if (vs2 && (int64_t)hph.nv[0] * hph.nv[1] != nv)
        fail(HPG_ERR_NUMERIC, "interior-vertex list does not match its grid");
    if (timing) {
        // one launch per part, each bracketed by its timing group
        tstart("prec_psi", s);
        dev::launch_hp_prec_psi<T>(hgeo, sinv, r + M.n_u, z + M.n_u,
                                   part ? part + np_dot : nullptr, np_prec, hp_nmax, dn, s);
        tstop("prec_psi", s);
        tstart("prec_u", s);
        if (!hph.ent_n.empty())
            dev::launch_hp_entity<T>(hent, inv, prm, r, z, dn, s);
        if (nv > 0) dev::launch_hp_vgather<T>(nv, vidx, r, cv, dn, s);
    } else {
        // psi-block, entity blocks (with their <z, r> shares) and the vertex
        // gather in one launch
        tstart("prec_u", s);
        dev::launch_hp_prec_fused<T>(hgeo, sinv, np_prec, hp_nmax, ne, hent, inv, prm, vidx, nv,
                                     cv, r, z, part ? part + np_dot : nullptr, part, dn, s);
    }
    // vertices: (alpha A_VV)^{-1} by fast diagonalisation on the interior-vertex grid
    if (vs2) {
        dev::launch_hp_vsolve2<T>(hph.nv[0], hph.nv[1], vidx, F.V[0].template as<T>(),
                                  F.V[1].template as<T>(), F.lam[0].template as<T>(),
                                  F.lam[1].template as<T>(), prm, cv, z,
                                  (part && !timing) ? part + ne : nullptr,
                                  dev::hp_vscatter_blocks(nv), dn, s);
    } else if (nv > 0) {
        T* t1 = kw.t1.template as<T>();
        T* t2 = kw.t2.template as<T>();
        const int d = M.d;
        const int* n1 = hph.nv;
        const T* src = cv;
        int pass = 0;
        const int npass = 2 * d;
        for (int ph = 0; ph < 2; ++ph)
            for (int k = 0; k < d; ++k) {
                ++pass;
                T* dst = (pass == npass) ? cv : ((src == t1) ? t2 : t1);
                dev::GemmEpi<T> ep{};
                ep.ts = fdm_tile<T>();
                if (ph == 0 && k == d - 1) {
                    ep.scale_mode = d;
                    ep.n0 = n1[0];
                    ep.l0 = F.lam[0].template as<T>();
                    ep.l1 = F.lam[1].template as<T>();
                    ep.l2 = F.lam[2].template as<T>();
                    ep.prm = prm;
                }
                const int N = n1[k];
                if (k == 0) {
                    const T* Bm = ph == 0 ? F.V[k].template as<T>() : F.Vt[k].template as<T>();
                    const int R = (int)(nv / N);
                    dev::launch_gemm<T>(R, N, N, src, N, 0, Bm, N, 0, dst, N, 0, 1, dn, ep, s);
                } else {
                    const T* Am = ph == 0 ? F.Vt[k].template as<T>() : F.V[k].template as<T>();
                    int64_t inner = 1;
                    for (int j = 0; j < k; ++j) inner *= n1[j];
                    const int64_t outer = nv / (inner * N);
                    dev::launch_gemm<T>(N, (int)inner, N, Am, N, 0, src, inner, (int64_t)N * inner,
                                        dst, inner, (int64_t)N * inner, (int)outer, dn, ep, s);
                }
                src = dst;
            }
        if (timing)
            dev::launch_hp_vscatter<T>(nv, vidx, cv, z, dn, s);
        else
            dev::launch_hp_vscatter_dot<T>(nv, vidx, cv, r, z, part ? part + ne : nullptr, dn, s);
    }
    if (part && timing) dev::launch_dot<T>(M.n_u, z, r, part, np_dot, dn, s);
    tstop("prec_u", s);
}

template void Problem::apply_G_hp<double>(const double*, double*, double*, const int*, hipStream_t);
template void Problem::apply_G_hp<float>(const float*, float*, double*, const int*, hipStream_t);
template void Problem::apply_prec_hp<double>(const double*, double*, double*, const int*,
                                             hipStream_t);
template void Problem::apply_prec_hp<float>(const float*, float*, double*, const int*,
                                            hipStream_t);

size_t footprint_bytes_hp(const Mesh& M, int precision) {
    const double n = (double)(M.n_u + M.n_psi), nu = (double)M.n_u;
    double loc = 0.0, blk = 0.0;
    for (int64_t c = 0; c < M.n_cells; ++c) {
        double l = 1.0, b = 1.0;
        for (int k = 0; k < M.d; ++k) {
            l *= M.deg[c] + 1;
            b *= M.deg[c] - 1;
        }
        loc += l;
        blk += b * b;
    }
    const double nq = (double)M.n_qp;
    double b = 0.0;
    b += loc * 8.0 + (nu + loc) * 4.0 + M.n_cells * 80.0;   // maps, incidence, offsets, items
    b += 2.0 * blk * 8.0;                                     // C_K classes and entity inverses (bound)
    b += 16.0 * n + 40.0 * n + 8.0 * 2 * 4096 * 2;
    b += 8.0 * blk;                                           // -S_hat blocks (formed in FP64)
    b += 8.0 * nq;                                            // phi at the Gauss points
    if (precision == HPG_FP64) {
        b += 8.0 * n + 8.0 * (7 * n + 2 * nu) + 8.0 * nq + 8.0 * loc;
    } else {
        b += 8.0 * n + 4.0 * (7 * n + 2 * nu) + 4.0 * nq + 4.0 * blk + 4.0 * loc;
        b += 8.0 * n + 8.0 * (7 * n + 2 * nu) + 8.0 * nq + 8.0 * loc;   // FP64 fallback steps
    }
    return (size_t)(1.15 * b) + ((size_t)8 << 20);
}

}  // namespace hpg
