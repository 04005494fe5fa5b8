// Host side of meshes with one degree per cell: the numbering of the
// minimum-rule space and the tables the hp kernels read.
#include <algorithm>
#include <climits>
#include <cmath>
#include <map>

#include "hp_host.h"

namespace hpg {

static void cell_index(const Mesh& M, int64_t c, int cc[3]) {
    cc[0] = cc[1] = cc[2] = 0;
    for (int k = 0; k < M.d; ++k) {
        cc[k] = (int)(c % M.m[k]);
        c /= M.m[k];
    }
}

static int64_t cell_number(const Mesh& M, const int cc[3]) {
    int64_t c = 0, st = 1;
    for (int k = 0; k < M.d; ++k) {
        c += cc[k] * st;
        st *= M.m[k];
    }
    return c;
}

void hp_number(Mesh& M) {
    const int d = M.d;
    int E[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) E[k] = 2 * M.m[k] + 1;
    const int64_t total = (int64_t)E[0] * E[1] * E[2];
    M.ent_base.assign(total, -1);
    M.ent_deg.assign(total, 0);
    int64_t n = 0;
    int e[3];
    for (e[2] = 0; e[2] < E[2]; ++e[2])
        for (e[1] = 0; e[1] < E[1]; ++e[1])
            for (e[0] = 0; e[0] < E[0]; ++e[0]) {
                bool bnd = false;
                for (int k = 0; k < d; ++k) bnd = bnd || e[k] == 0 || e[k] == E[k] - 1;
                if (bnd) continue;
                // cells containing the entity: per direction one interval (odd)
                // or the two intervals next to a vertex (even)
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                int nodd = 0;
                for (int k = 0; k < d; ++k) {
                    if (e[k] % 2) {
                        lo[k] = hi[k] = (e[k] - 1) / 2;
                        ++nodd;
                    } else {
                        lo[k] = std::max(0, e[k] / 2 - 1);
                        hi[k] = std::min(M.m[k] - 1, e[k] / 2);
                    }
                }
                int pe = INT_MAX;
                int c[3];
                for (c[2] = lo[2]; c[2] <= hi[2]; ++c[2])
                    for (c[1] = lo[1]; c[1] <= hi[1]; ++c[1])
                        for (c[0] = lo[0]; c[0] <= hi[0]; ++c[0])
                            pe = std::min(pe, M.deg[cell_number(M, c)]);
                const int64_t id = M.ent_index(e);
                M.ent_deg[id] = pe;
                M.ent_base[id] = n;
                int64_t cnt = 1;
                for (int j = 0; j < nodd; ++j) cnt *= pe - 1;
                n += cnt;
            }
    M.n_u = n;
    M.psi_off.assign(M.n_cells + 1, 0);
    M.qp_off.assign(M.n_cells + 1, 0);
    for (int64_t c = 0; c < M.n_cells; ++c) {
        int64_t pd = 1, qd = 1;
        for (int k = 0; k < d; ++k) {
            pd *= M.deg[c] - 1;
            qd *= M.deg[c] + 1;
        }
        M.psi_off[c + 1] = M.psi_off[c] + pd;
        M.qp_off[c + 1] = M.qp_off[c] + qd;
    }
    M.n_psi = M.psi_off[M.n_cells];
    M.n_qp = M.qp_off[M.n_cells];
}

void hp_cell_dofs(const Mesh& M, int64_t c, std::vector<int32_t>& out) {
    const int d = M.d, p = M.deg[c], L = p + 1;
    int cc[3];
    cell_index(M, c, cc);
    int64_t Ld = 1;
    for (int k = 0; k < d; ++k) Ld *= L;
    for (int64_t j = 0; j < Ld; ++j) {
        int e[3] = {0, 0, 0}, mode[3] = {0, 0, 0};
        bool odd[3] = {false, false, false};
        int64_t t = j;
        for (int k = 0; k < d; ++k) {
            const int l = (int)(t % L);
            t /= L;
            if (l == 0) {
                e[k] = 2 * cc[k];
            } else if (l == p) {
                e[k] = 2 * cc[k] + 2;
            } else {
                e[k] = 2 * cc[k] + 1;
                odd[k] = true;
                mode[k] = l - 1;
            }
        }
        const int64_t id = M.ent_index(e);
        const int64_t base = M.ent_base[id];
        int32_t g = -1;
        if (base >= 0) {
            const int pe = M.ent_deg[id];
            int64_t idx = 0, st = 1;
            bool ok = true;
            for (int k = 0; k < d; ++k)
                if (odd[k]) {
                    ok = ok && mode[k] <= pe - 2;
                    idx += mode[k] * st;
                    st *= pe - 1;
                }
            if (ok) g = (int32_t)(base + idx);
        }
        out.push_back(g);
    }
}

// Cholesky inverse of an SPD block (row-major)
static std::vector<double> spd_inverse(int n, const std::vector<double>& A) {
    std::vector<double> X((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) X[(size_t)i * n + i] = 1.0;
    chol_solve(n, A, X, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (X[(size_t)i * n + j] + X[(size_t)j * n + i]);
            X[(size_t)i * n + j] = X[(size_t)j * n + i] = s;
        }
    return X;
}

void hp_make_items(const Mesh& M, int lds_elems, int item_elems, HpHost& H) {
    const int64_t N = M.n_cells;
    H.item_start.clear();
    H.item_count.clear();
    H.item_p.clear();
    for (int64_t i = 0; i < N;) {
        const int p = M.deg[H.order[i]];
        int S = 1;
        for (int k = 0; k < M.d; ++k) S *= p + 1;
        const int cap = std::max(1, std::min(lds_elems, item_elems) / S);
        int64_t j = i;
        while (j < N && M.deg[H.order[j]] == p && j - i < cap) ++j;
        H.item_start.push_back((int32_t)i);
        H.item_count.push_back((int32_t)(j - i));
        H.item_p.push_back(p);
        i = j;
    }
}

void hp_build_host(const Mesh& M, int lds_elems, HpHost& H) {
    const int d = M.d;
    const int64_t N = M.n_cells;
    // per-degree reference tables
    H.ref.assign(M.p + 1, RefTables());
    H.toff.assign(M.p + 1, dev::HpTabOff{});
    H.tab.clear();
    for (int p = 2; p <= M.p; ++p) {
        RefTables& T = H.ref[p];
        T.build(p, p - 1, p + 1);
        auto put = [&](const std::vector<double>& v) {
            const int64_t o = (int64_t)H.tab.size();
            H.tab.insert(H.tab.end(), v.begin(), v.end());
            return o;
        };
        dev::HpTabOff& o = H.toff[p];
        o.A1 = put(T.A1);
        o.M1 = put(T.M1);
        o.B1 = put(T.B1);
        o.Vu = put(T.Vu);
        o.Vpsi = put(T.Vpsi);
        o.w = put(T.w);
        o.Mdiag = put(T.MpsiDiag);
    }
    // local -> global maps and their offsets
    H.loc_off.assign(N + 1, 0);
    H.sinv_off.assign(N + 1, 0);
    H.loc2glob.clear();
    for (int64_t c = 0; c < N; ++c) {
        hp_cell_dofs(M, c, H.loc2glob);
        H.loc_off[c + 1] = (int64_t)H.loc2glob.size();
        const int64_t n = M.psi_off[c + 1] - M.psi_off[c];
        H.sinv_off[c + 1] = H.sinv_off[c] + n * n;
    }
    // incidence lists (unknown -> local positions), ascending local position
    std::vector<int32_t> cnt(M.n_u + 1, 0);
    for (int32_t g : H.loc2glob)
        if (g >= 0) ++cnt[g + 1];
    H.inc_ptr.assign(M.n_u + 1, 0);
    for (int64_t i = 0; i < M.n_u; ++i) H.inc_ptr[i + 1] = H.inc_ptr[i] + cnt[i + 1];
    H.inc_idx.assign(H.inc_ptr[M.n_u], 0);
    std::vector<int32_t> fill(H.inc_ptr.begin(), H.inc_ptr.end() - 1);
    for (int64_t l = 0; l < (int64_t)H.loc2glob.size(); ++l) {
        const int32_t g = H.loc2glob[l];
        if (g >= 0) H.inc_idx[fill[g]++] = (int32_t)l;
    }
    // work items: cells sorted by degree (largest first), runs of equal degree
    H.order.resize(N);
    for (int64_t c = 0; c < N; ++c) H.order[c] = (int32_t)c;
    std::stable_sort(H.order.begin(), H.order.end(),
                     [&](int32_t a, int32_t b) { return M.deg[a] > M.deg[b]; });
    hp_make_items(M, lds_elems, 256, H);
    // C_K = Bhat^T Ahat^{-1} Bhat per (degree, widths) class
    std::map<std::vector<double>, int> cls;
    H.cclass.assign(N, 0);
    H.c_off.clear();
    H.C.clear();
    for (int64_t c = 0; c < N; ++c) {
        int cc[3];
        cell_index(M, c, cc);
        double hk[3] = {1, 1, 1};
        std::vector<double> key = {(double)M.deg[c]};
        for (int k = 0; k < d; ++k) {
            hk[k] = M.h(k, cc[k]);
            key.push_back(hk[k]);
        }
        auto it = cls.find(key);
        if (it == cls.end()) {
            Mesh T;
            T.d = d;
            T.p = M.deg[c];
            T.P = T.p - 1;
            T.q = T.p + 1;
            T.ref = H.ref[T.p];
            const std::vector<double> Cb = schur_block(T, hk);
            H.c_off.push_back((int64_t)H.C.size());
            H.C.insert(H.C.end(), Cb.begin(), Cb.end());
            it = cls.emplace(key, (int)H.c_off.size() - 1).first;
        }
        H.cclass[c] = it->second;
    }
    // block-Jacobi A-block: interior vertices in tensor order ...
    H.vert.clear();
    for (int k = 0; k < 3; ++k) H.nv[k] = k < d ? M.m[k] - 1 : 1;
    {
        int v[3];
        for (v[2] = 1; v[2] <= (d > 2 ? M.m[2] - 1 : 1); ++v[2])
            for (v[1] = 1; v[1] <= (d > 1 ? M.m[1] - 1 : 1); ++v[1])
                for (v[0] = 1; v[0] <= M.m[0] - 1; ++v[0]) {
                    int e[3] = {2 * v[0], d > 1 ? 2 * v[1] : 0, d > 2 ? 2 * v[2] : 0};
                    H.vert.push_back((int32_t)M.ent_base[M.ent_index(e)]);
                }
    }
    // ... and the inverse of A restricted to each other entity, assembled from
    // the cells containing it (deduplicated: equal blocks share storage)
    H.ent_first.clear();
    H.ent_n.clear();
    H.ent_off.clear();
    H.inv.clear();
    std::map<std::vector<double>, int64_t> blocks;
    int E[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) E[k] = 2 * M.m[k] + 1;
    int e[3];
    for (e[2] = 0; e[2] < E[2]; ++e[2])
        for (e[1] = 0; e[1] < E[1]; ++e[1])
            for (e[0] = 0; e[0] < E[0]; ++e[0]) {
                const int64_t id = M.ent_index(e);
                if (M.ent_base[id] < 0) continue;
                int nodd = 0;
                for (int k = 0; k < d; ++k) nodd += e[k] % 2;
                if (nodd == 0) continue;   // vertices: the coarse (Q1) block
                const int pe = M.ent_deg[id];
                int n = 1;
                for (int j = 0; j < nodd; ++j) n *= pe - 1;
                std::vector<double> A((size_t)n * n, 0.0);
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                for (int k = 0; k < d; ++k) {
                    if (e[k] % 2) {
                        lo[k] = hi[k] = (e[k] - 1) / 2;
                    } else {
                        lo[k] = std::max(0, e[k] / 2 - 1);
                        hi[k] = std::min(M.m[k] - 1, e[k] / 2);
                    }
                }
                int c[3];
                for (c[2] = lo[2]; c[2] <= hi[2]; ++c[2])
                    for (c[1] = lo[1]; c[1] <= hi[1]; ++c[1])
                        for (c[0] = lo[0]; c[0] <= hi[0]; ++c[0]) {
                            const int64_t cn = cell_number(M, c);
                            const int p = M.deg[cn], L = p + 1;
                            const RefTables& T = H.ref[p];
                            double hk[3], J = 1.0;
                            for (int k = 0; k < d; ++k) {
                                hk[k] = M.h(k, c[k]);
                                J *= 0.5 * hk[k];
                            }
                            // local 1-D index of entity function i in direction k
                            std::vector<int> li((size_t)n * d);
                            for (int i = 0; i < n; ++i) {
                                int t = i;
                                for (int k = 0; k < d; ++k) {
                                    if (e[k] % 2) {
                                        li[i * d + k] = 1 + t % (pe - 1);
                                        t /= pe - 1;
                                    } else {
                                        li[i * d + k] = (e[k] / 2 == c[k]) ? 0 : p;
                                    }
                                }
                            }
                            for (int i = 0; i < n; ++i)
                                for (int j = 0; j < n; ++j) {
                                    double s = 0.0;
                                    for (int k = 0; k < d; ++k) {
                                        double t = J * (2.0 / hk[k]) * (2.0 / hk[k]);
                                        for (int jj = 0; jj < d; ++jj) {
                                            const int a = li[i * d + jj], b = li[j * d + jj];
                                            t *= (jj == k ? T.A1 : T.M1)[a * L + b];
                                        }
                                        s += t;
                                    }
                                    A[(size_t)i * n + j] += s;
                                }
                        }
                auto it = blocks.find(A);
                if (it == blocks.end()) {
                    const std::vector<double> X = spd_inverse(n, A);
                    it = blocks.emplace(A, (int64_t)H.inv.size()).first;
                    H.inv.insert(H.inv.end(), X.begin(), X.end());
                }
                H.ent_first.push_back((int32_t)M.ent_base[id]);
                H.ent_n.push_back(n);
                H.ent_off.push_back(it->second);
            }
    // chunks: entities with one inverse (equal offsets, so equal sizes) next to
    // each other, larger entities first
    const int ne = (int)H.ent_n.size();
    H.ent_list.resize(ne);
    for (int e = 0; e < ne; ++e) H.ent_list[e] = e;
    std::stable_sort(H.ent_list.begin(), H.ent_list.end(), [&](int32_t a, int32_t b) {
        if (H.ent_n[a] != H.ent_n[b]) return H.ent_n[a] > H.ent_n[b];
        return H.ent_off[a] < H.ent_off[b];
    });
    H.ent_cstart.clear();
    H.ent_ccount.clear();
    H.ent_lds = 0;
    for (int k = 0; k < ne;) {
        const int n = H.ent_n[H.ent_list[k]], cap = dev::hp_ent_cap(n);
        int j = k;
        while (j < ne && j - k < cap && H.ent_off[H.ent_list[j]] == H.ent_off[H.ent_list[k]]) ++j;
        H.ent_cstart.push_back(k);
        H.ent_ccount.push_back(j - k);
        H.ent_lds = std::max(H.ent_lds, dev::hp_ent_lds(n));
        k = j;
    }
}

}  // namespace hpg
