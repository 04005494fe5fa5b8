// Host-side problem set-up, operator entry points, MINRES and the
// Newton / proximal-point drivers of the hpG library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "problem.h"

namespace hpg {

// ---------------------------------------------------------------------------
// Device buffers come from a per-device cache of freed blocks, so problems that
// are created and destroyed while other solves run (the server) reuse memory
// without a hipFree between them.  Blocks freed while the cache holds more than
// a quarter of the device's memory go back to HIP.
namespace {
struct BlockCache {
    std::mutex mu;
    std::multimap<size_t, void*> blocks;
    size_t cached = 0, cap = 0;
};
BlockCache& block_cache(int device) {
    static BlockCache caches[64];
    return caches[device & 63];
}
size_t round_block(size_t b) {
    const size_t small = 256, big = (size_t)2 << 20;
    return b < ((size_t)1 << 20) ? (b + small - 1) / small * small : (b + big - 1) / big * big;
}
}  // namespace

std::recursive_mutex& device_api_mutex() {
    static std::recursive_mutex m;
    return m;
}

size_t& device_bytes_counter() {
    static thread_local size_t n = 0;
    return n;
}

static void release_block(int device, void* p, size_t bytes) {
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    BlockCache& c = block_cache(device);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.cap == 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) c.cap = tot / 4;
        }
        if (c.cached + bytes <= c.cap) {
            c.blocks.emplace(bytes, p);
            c.cached += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

DBuf::~DBuf() {
    if (p) release_block(device, p, bytes);
}
void DBuf::alloc(size_t b) {
    if (p && bytes >= b) return;
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    if (p) {
        release_block(device, p, bytes);
        p = nullptr;
    }
    bytes = 0;
    if (b == 0) b = 16;
    const size_t rb = round_block(b);
    int dev = 0;
    HPG_HIP(hipGetDevice(&dev));
    BlockCache& c = block_cache(dev);
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.blocks.lower_bound(rb);
        if (it != c.blocks.end() && it->first <= 2 * rb) {
            p = it->second;
            bytes = it->first;
            c.cached -= it->first;
            c.blocks.erase(it);
        }
    }
    if (!p) {
        hipError_t e = hipMalloc(&p, rb);
        if (e != hipSuccess) {
            p = nullptr;
            fail(e == hipErrorOutOfMemory ? HPG_ERR_NOMEM : HPG_ERR_DEVICE,
                 std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        bytes = rb;
    }
    device = dev;
    device_bytes_counter() += bytes;
}

// Device memory one problem needs for a solve at the given precision: the
// buffers allocated by build, set_data, the linearisation, the Newton state,
// the Krylov work vectors and the fast-diagonalisation factors, plus a margin
// for allocation granularity.
size_t footprint_bytes(const Mesh& M, int precision) {
    if (M.hp) return footprint_bytes_hp(M, precision);
    const double n = (double)(M.n_u + M.n_psi), nu = (double)M.n_u;
    const double nc = (double)M.n_cells;
    double b = 0.0;
    for (int k = 0; k < M.d; ++k) {
        const double n1 = M.n1[k];
        b += n1 * 2.0 * (4 + Rows1D::WM * 20.0 + 4 + Rows1D::WB * 20.0);   // sparse rows, 2 precisions
        b += (n1 + 16.0 * M.p + 3) * (2 * (2 * M.p + 1) + 2 * M.P) * 12.0;    // dense windows
        b += n1 * n1 * 24.0 + n1 * 12.0;                                       // FDM factors
        b += M.m[k] * 12.0;
    }
    b += 16.0 * n;                        // F, Phi
    b += 40.0 * n;                        // Newton state: u, psi, psi_prev, ut, pt, u_old, R, delta
    b += 8.0 * 2 * 4096 * 2;              // partial sums, parameters, Krylov scalars
    const double npair = M.ncomp * (M.ncomp + 1) / 2.0;
    const double blk = (double)M.psi_per_cell * (double)M.psi_per_cell;
    b += 8.0 * nc * (double)M.Qd;                                   // phi at the Gauss points
    if (precision == HPG_FP64) {
        b += 8.0 * n;                                                  // Krylov solution
        b += 8.0 * (7 * n + 2 * nu);                                   // Krylov work vectors
        b += 8.0 * nc * (double)M.Qd * npair + 8.0 * nc * blk;         // weights, psi blocks
    } else {
        b += 8.0 * n;                                                  // FP32 rhs and correction
        b += 4.0 * (7 * n + 2 * nu);
        b += 4.0 * nc * (double)M.Qd * npair + 4.0 * nc * blk;
        // FP64 operator, Krylov vectors and solution of the steps that fall back to FP64
        b += 8.0 * n + 8.0 * (7 * n + 2 * nu);
        b += 8.0 * nc * (double)M.Qd * npair + 8.0 * nc * blk;
        b += 4.0 * nc;                                                 // ill-conditioned cell flags
    }
    return (size_t)(1.15 * b) + ((size_t)8 << 20);
}


// Dense-window form of the 1-D rows for p <= 3 (the fused apply's low-degree
// path): row g + 1 holds the stiffness and mass entries of columns g - p .. g + p,
// then the psi coupling of cells g / p and g / p + 1; row 0 and 16 p + 2 tail
// rows stay zero so that every tile's owned rows read in bounds.
static std::vector<double> dense_windows(const Mesh& M, const Rows1D& R) {
    const int p = M.p, P = std::max(1, M.P), WN = 2 * p + 1, WS = 2 * WN + 2 * P;
    if (p > 3 || M.P != p - 1) return std::vector<double>(1, 0.0);   // obstacle pairing only
    const int n = R.n;
    std::vector<double> w((size_t)(n + 1 + 16 * p + 2) * WS, 0.0);
    for (int gi = 0; gi < n; ++gi) {
        double* row = w.data() + (size_t)(gi + 1) * WS;
        for (int j = 0; j < R.lenM[gi]; ++j) {
            const int off = R.colM[(size_t)gi * Rows1D::WM + j] - gi + p;
            if (off < 0 || off >= WN) fail(HPG_ERR_NUMERIC, "1-D row wider than its window");
            row[off] = R.aM[(size_t)gi * Rows1D::WM + j];
            row[WN + off] = R.mM[(size_t)gi * Rows1D::WM + j];
        }
        for (int j = 0; j < R.lenB[gi]; ++j) {
            const int col = R.colB[(size_t)gi * Rows1D::WB + j];
            const int sc = col / P - gi / p, a = col % P;
            if (sc < 0 || sc > 1) fail(HPG_ERR_NUMERIC, "1-D psi coupling outside cells g/p, g/p+1");
            row[2 * WN + sc * P + a] = R.vB[(size_t)gi * Rows1D::WB + j];
        }
    }
    return w;
}

template <typename T>
dev::URows<T> DevRows<T>::view() const {
    dev::URows<T> r;
    r.lenM = lenM.as<int32_t>();
    r.colM = colM.as<int32_t>();
    r.aM = aM.as<T>();
    r.mM = mM.as<T>();
    r.lenB = lenB.as<int32_t>();
    r.cellB = cellB.as<int32_t>();
    r.modeB = modeB.as<int32_t>();
    r.vB = vB.as<T>();
    r.win = win.as<T>();
    r.lenG = lenG.as<int32_t>();
    r.cellG = cellG.as<int32_t>();
    r.modeG = modeG.as<int32_t>();
    r.vG = vG.as<T>();
    return r;
}
template <typename T>
dev::PsiTabs<T> DevTabs<T>::view() const {
    dev::PsiTabs<T> t;
    t.B1 = B1.as<T>();
    t.Vpsi = Vpsi.as<T>();
    t.Vu = Vu.as<T>();
    t.w = w.as<T>();
    t.Mdiag = Mdiag.as<T>();
    for (int k = 0; k < 3; ++k) t.h[k] = h[k].as<T>();
    t.G1 = G1.as<T>();
    t.AY = AY.as<T>();
    t.MY = MY.as<T>();
    return t;
}

template struct DevRows<double>;
template struct DevRows<float>;
template struct DevTabs<double>;
template struct DevTabs<float>;

template <typename T>
void KrylovWork<T>::ensure(int64_t n_, int64_t n_u) {
    if (n >= n_) return;
    const size_t b = n_ * sizeof(T), bu = n_u * sizeof(T);
    z.alloc(b);
    vcur.alloc(b);
    vprev.alloc(b);
    vhat.alloc(b);
    q.alloc(b);
    Gq.alloc(b);
    wprev.alloc(b);
    wcur.alloc(b);
    t1.alloc(bu);
    t2.alloc(bu);
    n = n_;
}

Problem::~Problem() {
    // device buffers return to the block cache when the members are destroyed:
    // the problem's own work must be finished first
    if (own_stream) (void)hipStreamSynchronize(own_stream);
    if (side) (void)hipStreamSynchronize(side);
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_enter) (void)hipEventDestroy(ev_enter);
    if (ev_leave) (void)hipEventDestroy(ev_leave);
    for (auto& kv : groups) {
        for (auto e : kv.second.start) (void)hipEventDestroy(e);
        for (auto e : kv.second.stop) (void)hipEventDestroy(e);
    }
    if (own_stream) (void)hipStreamDestroy(own_stream);
}

// ---------------------------------------------------------------------------
// small host tensor helper: contract axis ax of a d-D tensor (dims din,
// direction 0 fastest) with mat(i, j) = mat[i*ld + j] (or transposed)
std::vector<double> hcontract(const std::vector<double>& in, int d, int din[3], int ax,
                              int nout, const std::vector<double>& mat, int ld, bool trans) {
    int dout[3] = {din[0], din[1], din[2]};
    dout[ax] = nout;
    std::vector<double> out((size_t)dout[0] * dout[1] * dout[2], 0.0);
    const int sax = ax == 0 ? 1 : (ax == 1 ? din[0] : din[0] * din[1]);
    for (int i2 = 0; i2 < dout[2]; ++i2)
        for (int i1 = 0; i1 < dout[1]; ++i1)
            for (int i0 = 0; i0 < dout[0]; ++i0) {
                int idx[3] = {i0, i1, i2};
                const int io = idx[ax];
                idx[ax] = 0;
                const double* src = in.data() + idx[0] + din[0] * (idx[1] + din[1] * idx[2]);
                double s = 0.0;
                for (int j = 0; j < din[ax]; ++j)
                    s += (trans ? mat[j * ld + io] : mat[io * ld + j]) * src[j * sax];
                out[i0 + dout[0] * (i1 + dout[1] * i2)] = s;
            }
    (void)d;
    din[ax] = nout;
    return out;
}

// dense Cholesky solve A X = B (A n x n SPD, B n x m), row-major
void chol_solve(int n, std::vector<double> A, std::vector<double>& B, int m) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (s <= 0.0) fail(HPG_ERR_NUMERIC, "Phi-basis stiffness not positive definite");
        s = std::sqrt(s);
        A[j * n + j] = s;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / s;
        }
    }
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < n; ++i) {
            double t = B[i * m + c];
            for (int k = 0; k < i; ++k) t -= A[i * n + k] * B[k * m + c];
            B[i * m + c] = t / A[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double t = B[i * m + c];
            for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * B[k * m + c];
            B[i * m + c] = t / A[i * n + i];
        }
    }
}

static std::vector<double> kron(const std::vector<double>& A, int ar, int ac,
                                const std::vector<double>& B, int br, int bc) {
    std::vector<double> K((size_t)ar * br * ac * bc);
    for (int i = 0; i < ar; ++i)
        for (int j = 0; j < ac; ++j)
            for (int k = 0; k < br; ++k)
                for (int l = 0; l < bc; ++l)
                    K[(size_t)(i * br + k) * (ac * bc) + j * bc + l] = A[i * ac + j] * B[k * bc + l];
    return K;
}

// C_K = Bhat^T Ahat^{-1} Bhat for one cell shape (Sec. 4.5, alpha factored out):
// Ahat = sum_k (x)(AY (2/h_k) in slot k, MY (h_k/2) elsewhere), Bhat = (x)_k BY h_k/2
std::vector<double> schur_block(const Mesh& M, const double* hk) {
    const int P = M.P, d = M.d;
    const RefTables& T = M.ref;
    std::vector<double> Ah, Bh;
    int n = 1;
    for (int k = 0; k < d; ++k) {
        // kron with direction k as the slow factor: kron(X_k, current)
        std::vector<double> ak(P * P), mk(P * P), bk(P * P);
        for (int i = 0; i < P * P; ++i) {
            ak[i] = T.AY[i] * (2.0 / hk[k]);
            mk[i] = T.MY[i] * (0.5 * hk[k]);
            bk[i] = T.BY[i] * (0.5 * hk[k]);
        }
        if (k == 0) {
            Ah = ak;
            Bh = bk;
            n = P;
            continue;
        }
        // current Ah is the (k)-direction sum on the faster factors; mass of the faster ones:
        // rebuild Mfast = kron of MY over directions < k
        std::vector<double> Mf = {1.0};
        int nf = 1;
        for (int j = 0; j < k; ++j) {
            std::vector<double> mj(P * P);
            for (int i = 0; i < P * P; ++i) mj[i] = T.MY[i] * (0.5 * hk[j]);
            Mf = kron(mj, P, P, Mf, nf, nf);
            nf *= P;
        }
        std::vector<double> A1 = kron(mk, P, P, Ah, n, n);
        std::vector<double> A2 = kron(ak, P, P, Mf, nf, nf);
        for (size_t i = 0; i < A1.size(); ++i) A1[i] += A2[i];
        Ah = A1;
        Bh = kron(bk, P, P, Bh, n, n);
        n *= P;
    }
    // X = Ahat^{-1} Bhat; C = Bhat^T X
    std::vector<double> X(Bh);
    chol_solve(n, Ah, X, n);
    std::vector<double> C((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += Bh[(size_t)k * n + i] * X[(size_t)k * n + j];
            C[(size_t)i * n + j] = s;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
            C[(size_t)i * n + j] = C[(size_t)j * n + i] = s;
        }
    return C;
}

static int pick_cpb(int per_cell_elems, int elem_bytes, int work_per_cell, size_t budget) {
    int cpb = std::max(1, 256 / std::max(1, work_per_cell));
    while (cpb > 1 && (size_t)cpb * per_cell_elems * elem_bytes > budget) --cpb;
    return cpb;
}

void Problem::build(const Mesh& mesh, int dev_) {
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    M = mesh;
    device = dev_;
    int ndev = 0;
    HPG_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(HPG_ERR_INVALID_ARG, "no such HIP device");
    HPG_HIP(hipSetDevice(device));
    HPG_HIP(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
    HPG_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    HPG_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    HPG_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    HPG_HIP(hipEventCreateWithFlags(&ev_enter, hipEventDisableTiming));
    HPG_HIP(hipEventCreateWithFlags(&ev_leave, hipEventDisableTiming));
    {
        hipDeviceProp_t prop;
        HPG_HIP(hipGetDeviceProperties(&prop, device));
        lds_max = std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
    }
    gradient = M.kind == HPG_GRADIENT;
    if (M.hp) {
        build_hp();
        return;
    }
    // geometry
    geo.d = M.d;
    geo.p = M.p;
    geo.P = M.P;
    geo.q = M.q;
    for (int k = 0; k < 3; ++k) {
        geo.m[k] = M.m[k];
        geo.n1[k] = M.n1[k];
    }
    geo.n_u = M.n_u;
    geo.n_psi = M.n_psi;
    geo.n_cells = M.n_cells;
    geo.Pd = (int)M.Pd;
    geo.Qd = (int)M.Qd;
    geo.Ld = (int)M.Ld;
    int sb = std::max(M.p + 1, M.q), S = 1;
    for (int k = 0; k < M.d; ++k) S *= sb;
    geo.S = S;
    geo.nc = M.ncomp;
    // per-kernel cells per block
    if ((size_t)5 * S * 8 > lds_max || (size_t)4 * S * 8 > lds_max)
        fail(HPG_ERR_INVALID_ARG, "(p+1)^d too large for the LDS-staged cell kernels");
    cpb_l2 = pick_cpb(4 * S, 8, geo.Qd, std::min<size_t>(48 * 1024, lds_max));
    const int64_t nblk = M.psi_per_cell;   // psi block per cell: ncomp P^d
    if (gradient) {
        cpb_psi = dev::psi_side_grad_cpb<double>(geo);
        if ((size_t)(1 + 3 * M.d + 3) * S * 8 > std::min<size_t>(48 * 1024, lds_max))
            fail(HPG_ERR_INVALID_ARG, "(p+1)^d too large for the gradient psi-side kernel");
    } else {
        cpb_psi = pick_cpb(5 * S, 8, geo.Qd, std::min<size_t>(48 * 1024, lds_max));
        // Schur blocks: formed and inverted in LDS when one fits, else in place
        // in global memory (one cell per workgroup)
        const size_t setup_cell = dev::setup_smem_per_cell(geo);
        setup_mode = dev::SETUP_LDS;
        if (setup_cell > lds_max) {
            setup_mode = dev::setup_big_smem(geo, true) <= lds_max ? dev::SETUP_HBM_T2
                                                                   : dev::SETUP_HBM;
            if (dev::setup_big_smem(geo, false) > lds_max)
                fail(HPG_ERR_INVALID_ARG, "P^d too large for the Schur block setup");
        }
        cpb_setup = 1;
        if (!setup_mode) {
            cpb_setup = std::max(1, std::min(256 / std::max(1, geo.Pd), (int)(lds_max / setup_cell)));
            while (cpb_setup > 1 && setup_cell * cpb_setup > std::min<size_t>(64 * 1024, lds_max))
                --cpb_setup;
        }
    }
    // psi-block preconditioner: ~16 KB of inverse blocks per block of 256
    // threads; blocks beyond 48 KB are streamed from HBM one cell per block
    prec_big = (size_t)(nblk * nblk + nblk) * 8 > 48 * 1024;
    // packed blocks (uniform-degree obstacle meshes) hold twice the cells per
    // group in the same LDS, and use more of the block's threads (one per row)
    const int64_t nbs = dev::psi_block_size((int)nblk, packed_psi() ? 1 : 0);
    cpb_prec = std::max(1, (int)(2048 / std::max<int64_t>(1, nbs)));
    while (cpb_prec > 1 && (size_t)cpb_prec * (nbs + nblk) * 8 > 48 * 1024) --cpb_prec;
    // 1-D rows per direction
    for (int k = 0; k < 3; ++k) {
        Rows1D R;
        if (k < M.d) {
            build_rows(M, k, R);
        } else {
            R.n = 1;
            R.lenM = {0};
            R.colM.assign(Rows1D::WM, 0);
            R.aM.assign(Rows1D::WM, 0.0);
            R.mM.assign(Rows1D::WM, 0.0);
            R.lenB = {0};
            R.colB.assign(Rows1D::WB, 0);
            R.vB.assign(Rows1D::WB, 0.0);
        }
        std::vector<int32_t> cellB(R.colB.size()), modeB(R.colB.size());
        for (size_t i = 0; i < R.colB.size(); ++i) {
            cellB[i] = R.colB[i] / std::max(1, M.P);
            modeB[i] = R.colB[i] % std::max(1, M.P);
        }
        upload(rows64[k].lenM, R.lenM);
        upload(rows64[k].colM, R.colM);
        upload(rows64[k].aM, R.aM);
        upload(rows64[k].mM, R.mM);
        upload(rows64[k].lenB, R.lenB);
        upload(rows64[k].cellB, cellB);
        upload(rows64[k].modeB, modeB);
        upload(rows64[k].vB, R.vB);
        upload(rows32[k].lenM, R.lenM);
        upload(rows32[k].colM, R.colM);
        upload(rows32[k].aM, cast<float>(R.aM));
        upload(rows32[k].mM, cast<float>(R.mM));
        upload(rows32[k].lenB, R.lenB);
        upload(rows32[k].cellB, cellB);
        upload(rows32[k].modeB, modeB);
        upload(rows32[k].vB, cast<float>(R.vB));
        if (R.lenG.empty()) {
            R.lenG.assign(R.n, 0);
            R.colG.assign((size_t)R.n * Rows1D::WB, 0);
            R.vG.assign((size_t)R.n * Rows1D::WB, 0.0);
        }
        std::vector<int32_t> cellG(R.colG.size()), modeG(R.colG.size());
        for (size_t i = 0; i < R.colG.size(); ++i) {
            cellG[i] = R.colG[i] / std::max(1, M.P);
            modeG[i] = R.colG[i] % std::max(1, M.P);
        }
        upload(rows64[k].lenG, R.lenG);
        upload(rows64[k].cellG, cellG);
        upload(rows64[k].modeG, modeG);
        upload(rows64[k].vG, R.vG);
        upload(rows32[k].lenG, R.lenG);
        upload(rows32[k].cellG, cellG);
        upload(rows32[k].modeG, modeG);
        upload(rows32[k].vG, cast<float>(R.vG));
        const std::vector<double> win = dense_windows(M, R);
        upload(rows64[k].win, win);
        upload(rows32[k].win, cast<float>(win));
    }
    // reference tables
    const RefTables& T = M.ref;
    upload(tab64.B1, T.B1);
    upload(tab64.Vpsi, T.Vpsi);
    upload(tab64.Vu, T.Vu);
    upload(Du64, T.Du);
    upload(tab64.w, T.w);
    upload(tab64.Mdiag, T.MpsiDiag);
    upload(tab32.B1, cast<float>(T.B1));
    upload(tab32.Vpsi, cast<float>(T.Vpsi));
    upload(tab32.Vu, cast<float>(T.Vu));
    upload(tab32.w, cast<float>(T.w));
    upload(tab32.Mdiag, cast<float>(T.MpsiDiag));
    upload(tab64.G1, T.G1);
    upload(tab64.AY, T.AY);
    upload(tab64.MY, T.MY);
    upload(tab32.G1, cast<float>(T.G1));
    upload(tab32.AY, cast<float>(T.AY));
    upload(tab32.MY, cast<float>(T.MY));
    for (int k = 0; k < 3; ++k) {
        std::vector<double> hv;
        if (k < M.d)
            for (int c = 0; c < M.m[k]; ++c) hv.push_back(M.h(k, c));
        else
            hv.push_back(2.0);   // unused direction: h/2 = 1
        upload(tab64.h[k], hv);
        upload(tab32.h[k], cast<float>(hv));
    }
    // C_K per distinct cell shape: distinct widths per direction, class =
    // mixed-radix index of the width indices (one class on uniform meshes)
    std::vector<int> widx[3];
    std::vector<double> wval[3];
    for (int k = 0; k < 3; ++k) {
        if (k >= M.d) {
            widx[k] = {0};
            wval[k] = {2.0};
            continue;
        }
        std::map<double, int> seen;
        widx[k].resize(M.m[k]);
        for (int c = 0; c < M.m[k]; ++c) {
            const double hk = M.h(k, c);
            auto it = seen.find(hk);
            if (it == seen.end()) {
                const int id = (int)wval[k].size();
                seen[hk] = id;
                wval[k].push_back(hk);
                widx[k][c] = id;
            } else {
                widx[k][c] = it->second;
            }
        }
    }
    const int nw0 = (int)wval[0].size(), nw1 = (int)wval[1].size(), nw2 = (int)wval[2].size();
    std::vector<double> Call;
    for (int i2 = 0; i2 < (gradient ? 0 : nw2); ++i2)
        for (int i1 = 0; i1 < nw1; ++i1)
            for (int i0 = 0; i0 < nw0; ++i0) {
                const double hk[3] = {wval[0][i0], wval[1][i1], wval[2][i2]};
                std::vector<double> Cb = schur_block(M, hk);
                Call.insert(Call.end(), Cb.begin(), Cb.end());
            }
    std::vector<int32_t> cc(M.n_cells);
    for (int64_t c = 0; c < M.n_cells; ++c) {
        int64_t t = c;
        int ci[3] = {0, 0, 0};
        for (int k = 0; k < M.d; ++k) {
            ci[k] = widx[k][(int)(t % M.m[k])];
            t /= M.m[k];
        }
        cc[c] = ci[0] + nw0 * (ci[1] + nw1 * ci[2]);
    }
    if (Call.empty()) Call.assign(1, 0.0);   // the gradient preconditioner has no C_K term
    upload(C, Call);
    upload(cclass, cc);
    // reduction scratch
    np_u = (int)std::min<int64_t>((M.n_u + 127) / 128, 1024);
    np_psi = (int)std::min<int64_t>((M.n_cells + cpb_psi - 1) / cpb_psi, 1024);
    // partial sums of <z_u, r_u>: fused into the last fast-diagonalisation pass
    // when that pass has few enough blocks, else a separate 512-block kernel
    {
        int64_t nb_last;
        if (M.d == 1) {
            nb_last = (M.n1[0] + 15) / 16;
        } else {
            int64_t inner = 1;
            for (int j = 0; j < M.d - 1; ++j) inner *= M.n1[j];
            nb_last = ((inner + 15) / 16) * ((M.n1[M.d - 1] + 15) / 16);
        }
        fdm_dot_fused = nb_last <= 2048;
        np_dot = fdm_dot_fused ? (int)nb_last : 512;
    }
    const int np_l2 = 2 * (int)((M.n_cells + cpb_l2 - 1) / cpb_l2);
    np_prec = (int)std::min<int64_t>((M.n_cells + cpb_prec - 1) / cpb_prec, 1024);
    use_tile = dev::tile_supported(geo) && std::getenv("HPG_GENERIC_APPLY") == nullptr;
    np_cap = std::max({np_u + np_psi, np_dot + np_prec, np_l2, 2 * dev::tile_grid(geo)});
    partial.alloc((size_t)np_cap * sizeof(double));
    partial_g.alloc((size_t)np_cap * sizeof(double));
    params.alloc(4 * sizeof(double));
    kstate.alloc(2 * sizeof(dev::KState));
}

// Fast diagonalisation of the 1-D pairs (A1, M1) per direction, built on the
// first preconditioner apply (an O(n1^3) host eigen-decomposition, cached
// process-wide by (p, breakpoints) so repeated meshes reuse it).
namespace {
struct FdmEntry {
    std::vector<double> V, lam;
};
std::mutex g_fdm_mutex;
std::map<std::pair<int, std::vector<double>>, std::shared_ptr<FdmEntry>> g_fdm_cache;
}  // namespace

void Problem::ensure_fdm() {
    if (M.hp) return ensure_fdm_hp();
    std::lock_guard<std::recursive_mutex> api(device_api_mutex());
    if (fdm_ready) return;
    for (int k = 0; k < 3; ++k) {
        std::shared_ptr<FdmEntry> e;
        int n = 1;
        if (k < M.d) {
            n = M.n1[k];
            auto key = std::make_pair(M.p, M.breaks[k]);
            {
                std::lock_guard<std::mutex> lk(g_fdm_mutex);
                auto it = g_fdm_cache.find(key);
                if (it != g_fdm_cache.end()) e = it->second;
            }
            if (!e) {
                Rows1D R;
                build_rows(M, k, R, true);
                e = std::make_shared<FdmEntry>();
                generalized_eig(R.n, R.Adense, R.Mdense, e->V, e->lam);
                std::lock_guard<std::mutex> lk(g_fdm_mutex);
                g_fdm_cache[key] = e;
            }
        } else {
            e = std::make_shared<FdmEntry>();
            e->V = {1.0};
            e->lam = {0.0};
        }
        std::vector<double> Vt(e->V.size());
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Vt[(size_t)i * n + j] = e->V[(size_t)j * n + i];
        upload(fdm64.V[k], e->V);
        upload(fdm64.Vt[k], Vt);
        upload(fdm64.lam[k], e->lam);
        upload(fdm32.V[k], cast<float>(e->V));
        upload(fdm32.Vt[k], cast<float>(Vt));
        upload(fdm32.lam[k], cast<float>(e->lam));
    }
    fdm_ready = true;
}

// F_i = (f, v_i), Phi_i = (phi, zeta_i) by the Gauss-Legendre rule (sum-factorised)
void Problem::set_data(const double* f, const double* phi) {
    // phi at the Gauss points: the gradient constraint's weights and every
    // solve's feasibility diagnostic read it
    if (phi) {
        upload(PhiQ, std::vector<double>(phi, phi + M.n_qp));
        phi_absmax = 0.0;
        for (int64_t i = 0; i < M.n_qp; ++i) phi_absmax = std::max(phi_absmax, std::fabs(phi[i]));
    }
    if (M.hp) return set_data_hp(f, phi);
    const int d = M.d, q = M.q, L = M.p + 1, P = M.P;
    const RefTables& T = M.ref;
    if (f) {
        std::vector<double> Fh(M.n_u, 0.0);
        std::vector<double> vals(M.Qd);
        for (int64_t c = 0; c < M.n_cells; ++c) {
            int64_t t = c;
            int cc[3] = {0, 0, 0};
            double hk[3] = {2, 2, 2};
            double J = 1.0;
            for (int k = 0; k < d; ++k) {
                cc[k] = (int)(t % M.m[k]);
                t /= M.m[k];
                hk[k] = M.h(k, cc[k]);
                J *= 0.5 * hk[k];
            }
            for (int64_t j = 0; j < M.Qd; ++j) {
                int jj[3] = {(int)(j % q), (int)((j / q) % q), (int)(j / (q * q))};
                double wq = J;
                for (int k = 0; k < d; ++k) wq *= T.w[jj[k]];
                vals[j] = wq * f[c * M.Qd + j];
            }
            int din[3] = {1, 1, 1};
            for (int k = 0; k < d; ++k) din[k] = q;
            std::vector<double> cur = vals;
            for (int k = 0; k < d; ++k) cur = hcontract(cur, d, din, k, L, T.Vu, L, true);
            for (int64_t l = 0; l < M.Ld; ++l) {
                int ll[3] = {(int)(l % L), (int)((l / L) % L), (int)(l / (L * L))};
                int64_t flat = 0, st = 1;
                bool ok = true;
                for (int k = 0; k < d; ++k) {
                    int g = cc[k] * M.p + ll[k] - 1;
                    ok = ok && g >= 0 && g < M.n1[k];
                    flat += (int64_t)g * st;
                    st *= M.n1[k];
                }
                if (ok) Fh[flat] += cur[l];
            }
        }
        double s = 0.0;
        for (double v : Fh) s += v * v;
        normF = std::max(std::sqrt(s), 1e-300);
        upload(F, Fh);
        have_f = true;
    }
    if (phi) {
        std::vector<double> Ph(M.n_psi, 0.0);
        std::vector<double> vals(M.Qd);
        for (int64_t c = 0; c < M.n_cells; ++c) {
            int64_t t = c;
            double J = 1.0;
            for (int k = 0; k < d; ++k) {
                J *= 0.5 * M.h(k, (int)(t % M.m[k]));
                t /= M.m[k];
            }
            for (int64_t j = 0; j < M.Qd; ++j) {
                int jj[3] = {(int)(j % q), (int)((j / q) % q), (int)(j / (q * q))};
                double wq = J;
                for (int k = 0; k < d; ++k) wq *= T.w[jj[k]];
                vals[j] = wq * phi[c * M.Qd + j];
            }
            int din[3] = {1, 1, 1};
            for (int k = 0; k < d; ++k) din[k] = q;
            std::vector<double> cur = vals;
            for (int k = 0; k < d; ++k) cur = hcontract(cur, d, din, k, P, T.Vpsi, P, true);
            // gradient: Phi (the scale of the psi residual) repeats per component
            for (int comp = 0; comp < M.ncomp; ++comp)
                for (int64_t a = 0; a < M.Pd; ++a) Ph[(c * M.ncomp + comp) * M.Pd + a] = cur[a];
        }
        double s = 0.0;
        for (double v : Ph) s += v * v;
        normPhi = std::max(std::sqrt(s), 1e-300);
        upload(Phi, Ph);
        have_phi = true;
    }
}

void Problem::ensure_linearisation_buffers() {
    if (M.hp) {
        // weights at every cell's Gauss points; -S_hat blocks formed in FP64 in place
        // (and the per-local-function output of the cell pass: allocated here,
        // outside any graph capture of the Krylov iteration)
        const size_t nq = (size_t)M.n_qp, ns = (size_t)hph.sinv_off.back();
        const size_t nl = (size_t)hph.loc_off.back();
        sinv64.alloc(ns * sizeof(double));
        if (precision == HPG_FP64) {
            om64.alloc(nq * sizeof(double));
            if (!hpd.yloc64.p) hpd.yloc64.alloc(nl * sizeof(double));
        } else {
            om32.alloc(nq * sizeof(float));
            sinv32.alloc(ns * sizeof(float));
            if (!hpd.yloc32.p) hpd.yloc32.alloc(nl * sizeof(float));
        }
        return;
    }
    const size_t npair = (size_t)M.ncomp * (M.ncomp + 1) / 2;
    const size_t nq = (size_t)M.n_cells * M.Qd * npair;
    const size_t ns = (size_t)M.n_cells * M.psi_per_cell * M.psi_per_cell;
    if (precision == HPG_FP64) {
        om64.alloc(nq * sizeof(double));
        sinv64.alloc(ns * sizeof(double));
    } else {
        om32.alloc(nq * sizeof(float));
        sinv32.alloc(ns * sizeof(float));
        // blocks too large for LDS are formed and inverted in FP64 in place;
        // LDS-formed obstacle blocks keep the FP64 inverses of the cells too
        // ill-conditioned for an FP32 product
        if ((gradient && dev::setup_grad_in_hbm(geo)) || (!gradient && setup_mode))
            sinv64.alloc(ns * sizeof(double));
        if (flags_psi()) {
            sinv64.alloc(ns * sizeof(double));
            sflag.alloc((size_t)M.n_cells * sizeof(int));
        }
    }
}

void Problem::ensure_work() {
    const int64_t n = M.n_u + M.n_psi;
    const size_t b = n * sizeof(double);
    u.alloc(M.n_u * sizeof(double));
    psi.alloc(M.n_psi * sizeof(double));
    psi_prev.alloc(M.n_psi * sizeof(double));
    ut.alloc(M.n_u * sizeof(double));
    pt.alloc(M.n_psi * sizeof(double));
    u_old.alloc(M.n_u * sizeof(double));
    R.alloc(b);
    delta64.alloc(b);
}

// ---------------------------------------------------------------------------
static bool timed(const Problem& P, const char* grp) {
    return P.timing && (P.timing_group == "all" || P.timing_group == grp);
}

void Problem::tstart(const char* grp, hipStream_t s) {
    if (!timed(*this, grp)) return;
    TimingGroup& g = groups[grp];
    if (g.used == g.start.size()) {
        hipEvent_t a, b;
        HPG_HIP(hipEventCreate(&a));
        HPG_HIP(hipEventCreate(&b));
        g.start.push_back(a);
        g.stop.push_back(b);
    }
    HPG_HIP(hipEventRecord(g.start[g.used], s));
}
dev::KernelEvents Problem::kernel_events(const char* grp) {
    dev::KernelEvents ev;
    if (!timed(*this, grp)) return ev;
    TimingGroup& g = groups[grp];
    if (g.used == g.start.size()) {
        hipEvent_t a, b;
        HPG_HIP(hipEventCreate(&a));
        HPG_HIP(hipEventCreate(&b));
        g.start.push_back(a);
        g.stop.push_back(b);
    }
    ev.start = g.start[g.used];
    ev.stop = g.stop[g.used];
    g.used++;
    return ev;
}

void Problem::tstop(const char* grp, hipStream_t s) {
    if (!timed(*this, grp)) return;
    TimingGroup& g = groups[grp];
    HPG_HIP(hipEventRecord(g.stop[g.used], s));
    g.used++;
}

void Problem::setup(const double* d_psi, double alpha_, double beta_, int prec, hipStream_t s) {
    alpha = alpha_;
    beta = beta_;
    precision = prec;
    ensure_linearisation_buffers();
    hparams[0] = alpha;
    hparams[1] = beta;
    hparams[2] = 1.0 / alpha;
    HPG_HIP(hipMemcpyAsync(params.p, hparams, sizeof(hparams), hipMemcpyHostToDevice, s));
    tstart("setup", s);
    if (M.hp) {
        // one launch per degree (cells are ordered by degree), each with the LDS
        // of its own blocks, so low-degree cells are not held to the largest
        for (const HpRun& r : hp_runs) {
            const bool in_lds = dev::hp_setup_lds_p(M.d, r.p, true) <= lds_max;
            dev::launch_hp_setup(hgeo, hp_tabs<double>(), d_psi, alpha, beta, hpd.C.as<double>(),
                                 hpd.c_off.as<int64_t>(), hpd.cclass.as<int32_t>(),
                                 prec == HPG_FP64 ? om64.as<double>() : nullptr,
                                 prec == HPG_FP64 ? nullptr : om32.as<float>(),
                                 (prec == HPG_FP64 || !in_lds) ? sinv64.as<double>() : nullptr,
                                 prec == HPG_FP64 ? nullptr : sinv32.as<float>(),
                                 dev::hp_setup_lds_p(M.d, r.p, in_lds), in_lds, r.first, r.count, s);
        }
    } else if (gradient) {
        const bool hbm = dev::setup_grad_in_hbm(geo);
        dev::launch_setup_grad(geo, tab64.view(), d_psi, PhiQ.as<double>(), beta,
                               prec == HPG_FP64 ? om64.as<double>() : nullptr,
                               prec == HPG_FP64 ? nullptr : om32.as<float>(),
                               (prec == HPG_FP64 || hbm) ? sinv64.as<double>() : nullptr,
                               prec == HPG_FP64 ? nullptr : sinv32.as<float>(), s);
    } else {
        const bool fl = prec != HPG_FP64 && flags_psi();
        dev::launch_setup(geo, tab64.view(), cpb_setup, setup_mode, d_psi, alpha, beta,
                          C.as<double>(), cclass.as<int>(),
                          prec == HPG_FP64 ? om64.as<double>() : nullptr,
                          prec == HPG_FP64 ? nullptr : om32.as<float>(),
                          (prec == HPG_FP64 || setup_mode || fl) ? sinv64.as<double>() : nullptr,
                          prec == HPG_FP64 ? nullptr : sinv32.as<float>(), s, nullptr, nullptr, 1,
                          fl ? sflag.as<int>() : nullptr, packed_psi() ? 1 : 0);
    }
    tstop("setup", s);
    HPG_HIP(hipGetLastError());
    linearised = true;
}

template <typename T>
struct Sel;
template <>
struct Sel<double> {
    static const DevRows<double>* rows(const Problem& p) { return p.rows64; }
    static const DevTabs<double>& tabs(const Problem& p) { return p.tab64; }
    static const DevFdm<double>& fdm(const Problem& p) { return p.fdm64; }
    static const double* om(const Problem& p) { return p.om64.as<double>(); }
    static const double* sinv(const Problem& p) { return p.sinv64.as<double>(); }
    static KrylovWork<double>& kw(Problem& p) { return p.kw64; }
    static constexpr int prec = HPG_FP64;
};
template <>
struct Sel<float> {
    static const DevRows<float>* rows(const Problem& p) { return p.rows32; }
    static const DevTabs<float>& tabs(const Problem& p) { return p.tab32; }
    static const DevFdm<float>& fdm(const Problem& p) { return p.fdm32; }
    static const float* om(const Problem& p) { return p.om32.as<float>(); }
    static const float* sinv(const Problem& p) { return p.sinv32.as<float>(); }
    static KrylovWork<float>& kw(Problem& p) { return p.kw32; }
    static constexpr int prec = HPG_MIXED;
};

// fork work onto the side stream: everything enqueued on s2 after fork()
// runs concurrently with s until join()
void Problem::fork(hipStream_t s) {
    HPG_HIP(hipEventRecord(ev_fork, s));
    HPG_HIP(hipStreamWaitEvent(side, ev_fork, 0));
}
void Problem::join(hipStream_t s) {
    HPG_HIP(hipEventRecord(ev_join, side));
    HPG_HIP(hipStreamWaitEvent(s, ev_join, 0));
}

template <typename T>
void Problem::apply_G(const T* x, T* y, double* part, const int* dn, hipStream_t s) {
    if (!linearised || precision != Sel<T>::prec)
        fail(HPG_ERR_INVALID_ARG, "operator not set up for this precision (call hpg_op_setup)");
    if (M.hp) return apply_G_hp<T>(x, y, part, dn, s);
    const DevRows<T>* rw = Sel<T>::rows(*this);
    dev::URows<T> r[3] = {rw[0].view(), rw[1].view(), rw[2].view()};
    const double* prm = params.as<double>();
    if (use_tile) {
        // one fused LDS-tiled launch for both sides of G
        const dev::KernelEvents ke = kernel_events("apply_G");
        dev::launch_tile<T>(geo, r, Sel<T>::tabs(*this).view(), (T)alpha, (T)beta, prm, x,
                            x + M.n_u, nullptr, Sel<T>::om(*this), nullptr, nullptr, y, y + M.n_u,
                            part, dn, dev::MODE_APPLY, s, &ke);
        return;
    }
    const bool par = !timing && !single_stream;   // timed runs keep every launch on one stream
    hipStream_t s_psi = par ? side : s;
    if (par) fork(s);
    tstart("apply_G_psi", s_psi);
    if (gradient)
        dev::launch_psi_side_grad<T>(geo, Sel<T>::tabs(*this).view(), cpb_psi, (T)beta, x,
                                     x + M.n_u, Sel<T>::om(*this), nullptr, y + M.n_u,
                                     part ? part + np_u : nullptr, dn, dev::MODE_APPLY, s_psi, prm);
    else
        dev::launch_psi_side<T>(geo, Sel<T>::tabs(*this).view(), cpb_psi, (T)beta, x, x + M.n_u,
                                Sel<T>::om(*this), nullptr, y + M.n_u,
                                part ? part + np_u : nullptr, dn, dev::MODE_APPLY, s_psi, prm);
    tstop("apply_G_psi", s_psi);
    tstart("apply_G_u", s);
    if (gradient)
        dev::launch_u_side_grad<T>(geo, r, (T)alpha, x, x + M.n_u, nullptr, nullptr, y, part, dn,
                                   dev::MODE_APPLY, s, prm);
    else
        dev::launch_u_side<T>(geo, r, (T)alpha, x, x + M.n_u, nullptr, nullptr, y, part, dn,
                              dev::MODE_APPLY, s, prm);
    tstop("apply_G_u", s);
    if (par) join(s);
}

template <typename T>
void Problem::apply_prec(const T* r, T* z, double* part, const int* dn, hipStream_t s,
                         const VhatIn<T>* vin) {
    if (!linearised || precision != Sel<T>::prec)
        fail(HPG_ERR_INVALID_ARG, "operator not set up for this precision (call hpg_op_setup)");
    if (M.hp) return apply_prec_hp<T>(r, z, part, dn, s);
    KrylovWork<T>& kw = Sel<T>::kw(*this);
    kw.ensure(M.n_u + M.n_psi, M.n_u);
    ensure_fdm();
    const DevFdm<T>& F = Sel<T>::fdm(*this);
    T* t1 = kw.t1.template as<T>();
    T* t2 = kw.t2.template as<T>();
    const double* prm = params.as<double>();
    // psi-block: z_psi = (-S_hat_K)^{-1} r_psi.  Untimed, with LDS-staged
    // blocks, it shares one launch with the first fast-diagonalisation pass
    // (extra blocks of that grid); otherwise it runs on the side stream
    // concurrently with the A-block (timed runs: one stream, one group each)
    const bool merged = !prec_big && !timing;
    if (vin && (!merged || r != vin->vhat))
        fail(HPG_ERR_INVALID_ARG, "internal: folded Lanczos step without the merged first pass");
    const bool par = !merged && !timing && !single_stream;
    hipStream_t s_psi = par ? side : s;
    if (par) fork(s);
    if (!merged) {
        tstart("prec_psi", s_psi);
        if (prec_big)
            dev::launch_prec_psi_big<T>(M.n_cells, (int)M.psi_per_cell, Sel<T>::sinv(*this),
                                        r + M.n_u, z + M.n_u, part ? part + np_dot : nullptr,
                                        np_prec, dn, s_psi);
        else
            dev::launch_prec_psi<T>(M.n_cells, (int)M.psi_per_cell, cpb_prec, Sel<T>::sinv(*this),
                                    r + M.n_u, z + M.n_u, part ? part + np_dot : nullptr, dn, s_psi,
                                    dev::PsiBatch(), psi_hi<T>());
        tstop("prec_psi", s_psi);
    }
    // A-block: z_u = (alpha A)^{-1} r_u by fast diagonalisation: d forward
    // passes with V^T (the last one divides by alpha (lam_0 + ... )), then d
    // backward passes with V (the last one forms the partial sums of <z_u, r_u>)
    const int d = M.d;
    const T* src = r;
    int pass = 0;
    const int npass = 2 * d;
    const bool fuse_dot = part && fdm_dot_fused;
    for (int ph = 0; ph < 2; ++ph) {
        for (int k = 0; k < d; ++k) {
            ++pass;
            T* dst = (pass == npass) ? z : ((src == t1) ? t2 : t1);
            dev::GemmEpi<T> ep{};
            ep.ts = fdm_tile<T>();
            if (ph == 0 && k == d - 1) {
                ep.scale_mode = d;   // 1, 2, 3 as documented in the kernel
                ep.n0 = M.n1[0];
                ep.l0 = F.lam[0].template as<T>();
                ep.l1 = F.lam[1].template as<T>();
                ep.l2 = F.lam[2].template as<T>();
                ep.prm = prm;
            }
            if (pass == npass && fuse_dot) {
                ep.dotv = r;
                ep.partial = part;
            }
            const int N = M.n1[k];
            const dev::KernelEvents ke = kernel_events("fdm");   // timed per pass (one GEMM)
            if (k == 0) {
                // Y (R x N) = X (R x N) Mat^T with Mat = V^T (forward) / V (backward)
                const T* Bm = ph == 0 ? F.V[k].template as<T>() : F.Vt[k].template as<T>();
                const int R = (int)(M.n_u / N);
                if (vin && pass == 1)
                    dev::launch_vhat_gemm_prec<T>(R, N, Bm, dst, ep, M.n_cells,
                                                  (int)M.psi_per_cell, cpb_prec,
                                                  Sel<T>::sinv(*this), z + M.n_u,
                                                  part ? part + np_dot : nullptr, vin->st,
                                                  vin->gpart, vin->npg, vin->Gq, vin->vcur,
                                                  vin->vprev, vin->vhat, M.n_u, s, psi_hi<T>());
                else if (merged && pass == 1)
                    dev::launch_gemm_prec<T>(R, N, N, src, N, Bm, N, dst, N, dn, ep, M.n_cells,
                                             (int)M.psi_per_cell, cpb_prec, Sel<T>::sinv(*this),
                                             r + M.n_u, z + M.n_u,
                                             part ? part + np_dot : nullptr, s, 0, 0,
                                             dev::PsiBatch(), psi_hi<T>());
                else
                    dev::launch_gemm<T>(R, N, N, src, N, 0, Bm, N, 0, dst, N, 0, 1, dn, ep, s,
                                        &ke);
            } else {
                // Y_o (N x inner) = Mat (N x N) X_o (N x inner)
                const T* Am = ph == 0 ? F.Vt[k].template as<T>() : F.V[k].template as<T>();
                int64_t inner = 1;
                for (int j = 0; j < k; ++j) inner *= M.n1[j];
                const int64_t outer = M.n_u / (inner * N);
                dev::launch_gemm<T>(N, (int)inner, N, Am, N, 0, src, inner, (int64_t)N * inner, dst,
                                    inner, (int64_t)N * inner, (int)outer, dn, ep, s, &ke);
            }
            src = dst;
        }
    }
    if (part && !fuse_dot) dev::launch_dot<T>(M.n_u, z, r, part, np_dot, dn, s);
    if (par) join(s);
}

int forced_gemm_tile(int fallback) {
    const char* e = std::getenv("HPG_GEMM_TILE");
    if (!e) return fallback;
    return std::atoi(e) == 32 ? 2 : 1;
}

int pick_gemm_tile(hipStream_t s, const std::function<void(int)>& run, const char* what) {
    if (std::getenv("HPG_GEMM_TILE")) return forced_gemm_tile(1);
    hipEvent_t e0, e1;
    HPG_HIP(hipEventCreate(&e0));
    HPG_HIP(hipEventCreate(&e1));
    // the tiles alternate over several rounds and each keeps its best round,
    // so a clock still ramping up from idle does not favour the later one
    float best[3] = {1e30f, 1e30f, 1e30f};
    run(1);
    run(2);
    for (int round = 0; round < 5; ++round) {
        for (int ts : {1, 2}) {
            HPG_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < 3; ++r) run(ts);
            HPG_HIP(hipEventRecord(e1, s));
            HPG_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            HPG_HIP(hipEventElapsedTime(&ms, e0, e1));
            best[ts] = std::min(best[ts], ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (std::getenv("HPG_TRACE"))
        std::fprintf(stderr, "[hpg] %s: GEMM tile 16x16 %.1f us, 32x32 %.1f us per apply\n", what,
                     1e3 * best[1] / 3, 1e3 * best[2] / 3);
    // the 32x32 tile only when clearly faster (the 16x16 one has 4x the blocks,
    // the safer choice where the two are within timing noise)
    return best[2] < 0.95f * best[1] ? 2 : 1;
}

// times one preconditioner apply with each GEMM tile on zero vectors (the
// linearisation in place) and keeps the faster; runs before the first Krylov
// graph of this precision is captured
template <typename T>
void Problem::tune_fdm(hipStream_t s) {
    int& ts = fdm_ts<T>();
    if (ts) return;
    const int64_t n = M.n_u + M.n_psi;
    DBuf tmp;
    tmp.alloc((size_t)2 * n * sizeof(T));
    HPG_HIP(hipMemsetAsync(tmp.p, 0, tmp.bytes, s));
    T* r = tmp.as<T>();
    const bool tm = timing;
    timing = false;
    ts = pick_gemm_tile(
        s,
        [&](int c) {
            ts = c;
            apply_prec<T>(r, r + n, nullptr, nullptr, s);
        },
        sizeof(T) == 4 ? "FP32 preconditioner" : "FP64 preconditioner");
    timing = tm;
    HPG_HIP(hipStreamSynchronize(s));
}

static double host_sum(const double* d_part, int n, hipStream_t s) {
    std::vector<double> h(n);
    HPG_HIP(hipMemcpyAsync(h.data(), d_part, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : h) t += v;
    return t;
}

template <typename T>
void Problem::minres_iterations(int count, int par0, T*& vcur, T*& vprev, T*& wprev, T*& wcur,
                                T* q, T* Gq, T* z, T* x, hipStream_t s) {
    auto* st = kstate.as<dev::KState>();
    double* part = partial.as<double>();
    double* gpart = partial_g.as<double>();   // the G apply's partials, apart from the preconditioner's
    T* vhat = Sel<T>::kw(*this).vhat.template as<T>();
    const int64_t n = M.n_u + M.n_psi;
    const int npG = use_tile ? dev::tile_grid(geo) : np_u + np_psi, npP = np_dot + np_prec;
    // untimed uniform-degree solves form vhat inside the preconditioner's first launch
    const bool fold = !M.hp && !prec_big && !timing;
    int par = par0;
    for (int j = 0; j < count; ++j) {
        dev::KState* cur = st + par;
        dev::KState* nxt = st + (1 - par);
        const int* dn = &cur->done;
        apply_G<T>(q, Gq, gpart, dn, s);
        if (fold) {
            const VhatIn<T> vin{cur, gpart, npG, Gq, vcur, vprev, vhat};
            apply_prec<T>(vhat, z, part, dn, s, &vin);
        } else {
            tstart("minres_vec", s);
            dev::launch_kr_vhat<T>(n, cur, gpart, npG, Gq, vcur, vprev, vhat, s);
            tstop("minres_vec", s);
            apply_prec<T>(vhat, z, part, dn, s);
        }
        tstart("minres_vec", s);
        dev::launch_kr_update<T>(n, cur, nxt, part, npP, q, wprev, wcur, x, vprev, vhat, z, s);
        tstop("minres_vec", s);
        std::swap(vprev, vcur);
        std::swap(wprev, wcur);
        par = 1 - par;
    }
}

template <typename T>
int Problem::minres(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t caller) {
    // run on the library's own stream (capturable, unlike the legacy null
    // stream), ordered after the caller's earlier work and before its later work
    hipStream_t s = own_stream;
    if (caller != s) {
        HPG_HIP(hipEventRecord(ev_enter, caller));
        HPG_HIP(hipStreamWaitEvent(s, ev_enter, 0));
    }
    const int iters = minres_on(b, x, rtol, maxit, chunk, s);
    if (caller != s) {
        HPG_HIP(hipEventRecord(ev_leave, s));
        HPG_HIP(hipStreamWaitEvent(caller, ev_leave, 0));
    }
    return iters;
}

template <typename T>
int Problem::minres_on(const T* b, T* x, double rtol, int maxit, int chunk, hipStream_t s) {
    const int64_t n = M.n_u + M.n_psi;
    KrylovWork<T>& kw = Sel<T>::kw(*this);
    kw.ensure(n, M.n_u);
    T* z = kw.z.template as<T>();
    T* vcur = kw.vcur.template as<T>();
    T* vprev = kw.vprev.template as<T>();
    T* q = kw.q.template as<T>();
    T* Gq = kw.Gq.template as<T>();
    T* wprev = kw.wprev.template as<T>();
    T* wcur = kw.wcur.template as<T>();
    double* part = partial.as<double>();
    auto* st = kstate.as<dev::KState>();   // st[0], st[1]: state by iteration parity
    const int npP = np_dot + np_prec;
    tune_fdm<T>(s);
    // z1 = M^{-1} b, gamma1^2 = <z1, b>
    apply_prec<T>(b, z, part, nullptr, s);
    dev::launch_kr_start<T>(n, st, part, npP, rtol, maxit, b, z, vcur, vprev, q, wprev, wcur, x,
                            s);
    HPG_HIP(hipGetLastError());
    chunk = std::max(2, chunk + (chunk & 1));   // even: buffer roles and parity repeat
    // a chunk of iterations is captured once per (precision, b, x) and replayed;
    // timed runs launch directly so each kernel can be bracketed by events
    hipGraphExec_t exec = nullptr;
    if (use_graphs && !timing) {
        const GraphKey key{Sel<T>::prec, chunk, (const void*)b, (const void*)x};
        auto it = graphs.find(key);
        if (it == graphs.end()) {
            T *vc = vcur, *vp = vprev, *wp = wprev, *wc = wcur;
            hipGraph_t g;
            std::lock_guard<std::recursive_mutex> api(device_api_mutex());
            HPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            minres_iterations<T>(chunk, 0, vc, vp, wp, wc, q, Gq, z, x, s);
            HPG_HIP(hipStreamEndCapture(s, &g));
            HPG_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
            HPG_HIP(hipGraphDestroy(g));
            graphs[key] = exec;
        } else {
            exec = it->second;
        }
    }
    int it = 0;
    dev::KState hs;
    while (it < maxit) {
        if (exec) {
            HPG_HIP(hipGraphLaunch(exec, s));
            it += chunk;
        } else {
            const int nc = std::min(chunk, maxit - it);
            minres_iterations<T>(nc, 0, vcur, vprev, wprev, wcur, q, Gq, z, x, s);
            it += nc;
            if (nc & 1) {   // odd tail: the state of the last iteration sits in st[1]
                HPG_HIP(hipMemcpyAsync(&hs, st + 1, sizeof(hs), hipMemcpyDeviceToHost, s));
                HPG_HIP(hipStreamSynchronize(s));
                break;
            }
        }
        HPG_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        HPG_HIP(hipStreamSynchronize(s));
        if (hs.done) break;
    }
    HPG_HIP(hipGetLastError());
    if (!(hs.gamma1 == hs.gamma1)) fail(HPG_ERR_NUMERIC, "MINRES: non-finite right-hand side");
    if (hs.breakdown && hs.iters == 0 && hs.gamma1 != 0.0 && Sel<T>::prec == HPG_FP64)
        fail(HPG_ERR_NUMERIC, "MINRES breakdown");
    last_minres_breakdown = hs.breakdown != 0;
    return hs.iters;
}

int Problem::residual_partials() const {
    if (use_tile) return 2 * dev::tile_grid(geo);
    return np_u + np_psi;
}

int64_t Problem::residual_local_values() const {
    return M.hp ? (int64_t)hph.loc_off.back() : 0;
}

void Problem::residual(const double* uu, const double* pp, const double* pprev, double alpha_,
                       double* RR, hipStream_t s, double* nu2, double* np2, const ResScratch* sc) {
    if (!have_f || !have_phi) fail(HPG_ERR_INVALID_ARG, "forcing and obstacle must be set");
    dev::URows<double> r[3] = {rows64[0].view(), rows64[1].view(), rows64[2].view()};
    double* part = sc ? sc->part : partial.as<double>();
    // host copy of the partial sums: the caller's buffer, else a vector
    const int npart = residual_partials();
    std::vector<double> hv;
    double* h = sc ? sc->host : nullptr;
    if (!h) {
        hv.resize(npart);
        h = hv.data();
    }
    tstart("residual", s);
    double a = 0.0, b = 0.0;
    if (use_tile) {
        dev::launch_tile<double>(geo, r, tab64.view(), alpha_, 0.0, nullptr, uu, pp, pprev, nullptr,
                                 F.as<double>(), Phi.as<double>(), RR, RR + M.n_u, part, nullptr,
                                 dev::MODE_RES, s);
        tstop("residual", s);
        HPG_HIP(hipGetLastError());
        const int nb = npart / 2;
        HPG_HIP(hipMemcpyAsync(h, part, npart * sizeof(double), hipMemcpyDeviceToHost, s));
        HPG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < nb; ++i) {
            a += h[2 * i];
            b += h[2 * i + 1];
        }
    } else {
        if (M.hp) {
            double* yloc = sc ? sc->yloc : nullptr;
            if (!yloc) {
                if (!hpd.yloc64.p) hpd.yloc64.alloc((size_t)hph.loc_off.back() * sizeof(double));
                yloc = hpd.yloc64.as<double>();
            }
            dev::launch_hp_cell<double>(hgeo, hp_tabs<double>(), alpha_, 0.0, nullptr, uu, pp,
                                        pprev, nullptr, Phi.as<double>(), yloc, RR + M.n_u,
                                        np_cell, nullptr, dev::MODE_RES, s);
            dev::launch_hp_gather<double>(M.n_u, hpd.inc_ptr.as<int32_t>(),
                                          hpd.inc_idx.as<int32_t>(), yloc, F.as<double>(), alpha_,
                                          uu, RR, M.n_psi, nullptr, RR + M.n_u, part, np_gath,
                                          nullptr, dev::MODE_RES, s);
        } else if (gradient) {
            dev::launch_u_side_grad<double>(geo, r, alpha_, uu, pp, pprev, F.as<double>(), RR,
                                            part, nullptr, dev::MODE_RES, s, nullptr);
            dev::launch_psi_side_grad<double>(geo, tab64.view(), cpb_psi, 0.0, uu, pp, nullptr,
                                              PhiQ.as<double>(), RR + M.n_u, part + np_u,
                                              nullptr, dev::MODE_RES, s, nullptr);
        } else {
            dev::launch_u_side<double>(geo, r, alpha_, uu, pp, pprev, F.as<double>(), RR, part,
                                       nullptr, dev::MODE_RES, s);
            dev::launch_psi_side<double>(geo, tab64.view(), cpb_psi, 0.0, uu, pp, nullptr,
                                         Phi.as<double>(), RR + M.n_u, part + np_u, nullptr,
                                         dev::MODE_RES, s);
        }
        tstop("residual", s);
        HPG_HIP(hipGetLastError());
        HPG_HIP(hipMemcpyAsync(h, part, npart * sizeof(double), hipMemcpyDeviceToHost, s));
        HPG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < np_u; ++i) a += h[i];
        for (int i = 0; i < np_psi; ++i) b += h[np_u + i];
    }
    *nu2 = a;
    *np2 = b;
}

// complementarity sums and pointwise violation of an iterate at the Gauss
// points (launch_diag), reduced on the host in block order (synchronises)
void Problem::diagnostics(const double* du, const double* dp, const double* dlam, hipStream_t s,
                          double* cr, double* cr_rel, double* mv) {
    constexpr int kDiagBlocks = 1024;
    const int nb = (int)std::min<int64_t>(M.n_cells, kDiagBlocks);
    if (!diag_part.p) diag_part.alloc((size_t)3 * kDiagBlocks * sizeof(double));
    double* part = diag_part.as<double>();
    if (M.hp)
        dev::launch_hp_diag(hgeo, hp_tabs<double>(), du, dp, dlam, PhiQ.as<double>(), part, nb, s);
    else
        dev::launch_diag(geo, tab64.view(), Du64.as<double>(), du, dp, dlam, PhiQ.as<double>(),
                         part, nb, s);
    HPG_HIP(hipGetLastError());
    std::vector<double> h((size_t)3 * nb);
    HPG_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
    double c = 0.0, l1 = 0.0, m = -std::numeric_limits<double>::infinity();
    for (int i = 0; i < nb; ++i) {
        c += h[3 * i];
        l1 += h[3 * i + 1];
        m = std::max(m, h[3 * i + 2]);
    }
    *cr = c;
    *cr_rel = c / std::max(l1 * phi_absmax, 1e-300);
    *mv = m;
}

double Problem::l2_diff(const double* a, const double* b, double* norm_a, hipStream_t s) {
    double* part = partial.as<double>();
    int nb;
    if (M.hp) {
        dev::launch_hp_l2(hgeo, hp_tabs<double>(), a, b, part, np_hpl2, s);
        nb = np_hpl2;
    } else {
        dev::launch_l2(geo, tab64.view(), cpb_l2, a, b, part, s);
        nb = (int)((M.n_cells + cpb_l2 - 1) / cpb_l2);
    }
    HPG_HIP(hipGetLastError());
    std::vector<double> h(2 * nb);
    HPG_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HPG_HIP(hipStreamSynchronize(s));
    double d2 = 0.0, a2 = 0.0;
    for (int i = 0; i < nb; ++i) {
        d2 += h[2 * i];
        a2 += h[2 * i + 1];
    }
    *norm_a = std::sqrt(std::max(a2, 0.0));
    return std::sqrt(std::max(d2, 0.0));
}

// MINRES tolerance of a mixed-precision Newton step recomputed in FP64 (the
// FP64 path's default): a direction accurate only to the FP32 tolerance does
// not reduce the merit function near the Newton tolerance
constexpr double kFallbackKrylovRtol = 1e-10;
// after this many FP64 recomputations within one proximal step, a mixed solve
// computes the remaining Newton directions of that step in FP64 directly (a
// subproblem whose FP32 solves keep breaking down would pay for both)
constexpr int kMaxFallbacksPerStep = 3;
// ... and after this many over the whole solve, every later direction
constexpr int kMaxFallbacksPerSolve = 12;
// longest extended Newton step (step_extension), in multiples of the direction
constexpr double kMaxStepExtension = 8.0;

// Newton direction with the FP64 operator: b = -R, MINRES into xk64, delta = xk64
int Problem::newton_direction64(const double* dR, double* dd, double eta, const hpg_solve_opts& o,
                                hipStream_t s) {
    const int64_t n = M.n_u + M.n_psi;
    xk64.alloc(n * sizeof(double));
    dev::launch_convert<double, double>(n, dR, dd, -1.0, s);
    const int its = minres<double>(dd, xk64.as<double>(), eta, o.max_krylov, o.krylov_chunk, s);
    HPG_HIP(hipMemcpyAsync(dd, xk64.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return its;
}

// ---------------------------------------------------------------------------
// The proximal-point loop with Newton (paper Sec. 2.1 / Sec. 4; readings on
// the alpha schedule, the Newton stop, the backtracking line search and the
// outer stop are the ones documented in the oracle and in hpg.h).
hpg_status Problem::solve(const hpg_solve_opts& o, hipStream_t s, hpg_solve_stats* st,
                          double* d_u_out, double* d_psi_out, double* d_lam_out) {
    if (!have_f || !have_phi) fail(HPG_ERR_INVALID_ARG, "forcing and obstacle must be set");
    auto t0 = std::chrono::steady_clock::now();
    ensure_work();
    const int64_t n = M.n_u + M.n_psi;
    const bool mixed = o.precision == HPG_MIXED;
    if (mixed) {
        delta32.alloc(n * sizeof(float));
        rhs32.alloc(n * sizeof(float));
    } else {
        xk64.alloc(n * sizeof(double));
    }
    if (o.step_extension) {
        ux.alloc(M.n_u * sizeof(double));
        px.alloc(M.n_psi * sizeof(double));
    }
    double* du = u.as<double>();
    double* dp = psi.as<double>();
    double* dpp = psi_prev.as<double>();
    double* dut = ut.as<double>();
    double* dpt = pt.as<double>();
    double* dR = R.as<double>();
    double* dd = delta64.as<double>();
    const int kmax = o.fixed_prox_steps > 0 ? o.fixed_prox_steps : o.max_prox;
    if (o.q != 0 && o.q != M.q)
        fail(HPG_ERR_INVALID_ARG, "only the Gauss rule with q = p + 1 points per direction is built");
    if ((o.warm_u == nullptr) != (o.warm_psi == nullptr))
        fail(HPG_ERR_INVALID_ARG, "warm start needs both warm_u and warm_psi");
    if (o.k0 < 0 || o.k0 >= kmax || (o.k0 > 0 && !o.warm_u))
        fail(HPG_ERR_INVALID_ARG, "k0 must be 0 without a warm start and below the step cap");
    // u_0 = psi_0 = 0 (Sec. 2.1), or the state after k0 steps (warm start;
    // host or device pointers, the copy direction is inferred)
    if (o.warm_u) {
        HPG_HIP(hipMemcpyAsync(du, o.warm_u, M.n_u * sizeof(double), hipMemcpyDefault, s));
        HPG_HIP(hipMemcpyAsync(dp, o.warm_psi, M.n_psi * sizeof(double), hipMemcpyDefault, s));
        HPG_HIP(hipMemcpyAsync(dpp, o.warm_psi, M.n_psi * sizeof(double), hipMemcpyDefault, s));
    } else {
        HPG_HIP(hipMemsetAsync(du, 0, M.n_u * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(dp, 0, M.n_psi * sizeof(double), s));
        HPG_HIP(hipMemsetAsync(dpp, 0, M.n_psi * sizeof(double), s));
    }
    hpg_solve_stats S{};
    S.status = HPG_OK;
    // alpha_{k0+1}: the schedule's own recurrence, so a resumed solve takes the
    // same step sizes as the uninterrupted one
    double alpha_k = o.alpha0;
    for (int i = 0; i < o.k0; ++i) alpha_k = std::min(alpha_k * o.alpha_factor, o.alpha_max);
    int k = o.k0;
    bool ok = true;
    int recomputed = 0;   // FP32 directions computed again in FP64 over the solve (mixed)
    bool have_lam = false;
    double* dlam = dR;    // lambda of the last step: the residual buffer is free after the loop
    double last_err = 0.0;
    double alpha_used = alpha_k;
    // HPG_TRACE=1: one line per Newton step on stderr (proximal step, Newton
    // step, error, Krylov iterations, accepted step length)
    const bool trace = std::getenv("HPG_TRACE") != nullptr;
    while (k < kmax) {
        ++k;
        HPG_HIP(hipMemcpyAsync(u_old.p, du, M.n_u * sizeof(double), hipMemcpyDeviceToDevice, s));
        // ---- Newton on the subproblem with (alpha_k, psi_prev)
        bool conv = false;
        int fb_step = 0;   // FP64 recomputations in this proximal step (mixed)
        for (int it = 0; it <= o.max_newton; ++it) {
            double nu2, np2;
            residual(du, dp, dpp, alpha_k, dR, s, &nu2, &np2);
            const double err = std::sqrt(nu2) / (alpha_k * normF) + std::sqrt(np2) / normPhi;
            last_err = err;
            if (!std::isfinite(err)) break;
            if (err <= o.newton_tol) {
                conv = true;
                break;
            }
            if (it == o.max_newton) break;
            const bool use32 = mixed && fb_step < kMaxFallbacksPerStep &&
                               recomputed < kMaxFallbacksPerSolve;
            setup(dp, alpha_k, o.beta, use32 ? HPG_MIXED : HPG_FP64, s);
            // inexact Newton (optional): a linear-solve tolerance proportional
            // to the current error.  MINRES measures the residual in the
            // preconditioner's norm, which is much looser than the Newton
            // error measure, hence the small factor.
            const double eta = o.inexact_newton
                                   ? std::min(1e-6, std::max(o.krylov_rtol, 1e-6 * err))
                                   : o.krylov_rtol;
            int its;
            bool need64 = false;   // FP32 Krylov solve broke down or hit its cap
            if (use32) {
                float* b32 = rhs32.as<float>();
                float* x32 = delta32.as<float>();
                dev::launch_convert<double, float>(n, dR, b32, -1.0, s);
                its = minres<float>(b32, x32, eta, o.max_krylov, o.krylov_chunk, s);
                dev::launch_convert<float, double>(n, x32, dd, 1.0, s);
                need64 = last_minres_breakdown || its >= o.max_krylov;
            } else if (mixed) {
                its = newton_direction64(dR, dd, std::min(eta, kFallbackKrylovRtol), o, s);
                S.fp64_fallbacks += 1;
            } else {
                its = newton_direction64(dR, dd, eta, o, s);
            }
            S.krylov_iters += its;
            S.newton_iters += 1;
            // backtracking on ||(R_u / alpha, R_psi)||; a step from the FP32
            // Krylov solve that the line search rejects is recomputed once in FP64
            const double m0 = std::sqrt(nu2 / (alpha_k * alpha_k) + np2);
            double t = 1.0;
            bool acc = false;
            for (int attempt = need64 ? 1 : 0; attempt < (use32 ? 2 : 1) && !acc; ++attempt) {
                if (attempt == 1) {
                    if (trace)
                        std::fprintf(stderr, "hpg: prox %d newton %d fp32 direction %s, fp64 recomputed\n",
                                     k, it, need64 ? (last_minres_breakdown ? "broke down" : "hit the cap")
                                                   : "rejected by the line search");
                    residual(du, dp, dpp, alpha_k, dR, s, &nu2, &np2);
                    setup(dp, alpha_k, o.beta, HPG_FP64, s);
                    its = newton_direction64(dR, dd, std::min(eta, kFallbackKrylovRtol), o, s);
                    S.krylov_iters += its;
                    S.fp64_fallbacks += 1;   // the next Newton step sets up FP32 again
                    ++fb_step;
                    ++recomputed;
                }
                t = 1.0;
                for (int hv = 0; hv <= 30; ++hv) {
                    dev::launch_axpy_to<double>(M.n_u, du, t, dd, dut, s);
                    dev::launch_axpy_to<double>(M.n_psi, dp, t, dd + M.n_u, dpt, s);
                    double a2, b2;
                    residual(dut, dpt, dpp, alpha_k, dR, s, &a2, &b2);
                    const double m1 = std::sqrt(a2 / (alpha_k * alpha_k) + b2);
                    if (m1 <= (1.0 - 1e-4 * t) * m0) {
                        acc = true;
                        // optional extension of a full step (2, 4, 8 times the
                        // direction) while the merit keeps falling
                        double mb = m1;
                        const bool full = t == 1.0;
                        for (double te = 2.0; o.step_extension && full && te <= kMaxStepExtension;
                             te *= 2.0) {
                            double* ue = ux.as<double>();
                            double* pe = px.as<double>();
                            dev::launch_axpy_to<double>(M.n_u, du, te, dd, ue, s);
                            dev::launch_axpy_to<double>(M.n_psi, dp, te, dd + M.n_u, pe, s);
                            residual(ue, pe, dpp, alpha_k, dR, s, &a2, &b2);
                            const double me = std::sqrt(a2 / (alpha_k * alpha_k) + b2);
                            if (!(me < mb)) break;
                            mb = me;
                            HPG_HIP(hipMemcpyAsync(dut, ue, M.n_u * sizeof(double),
                                                   hipMemcpyDeviceToDevice, s));
                            HPG_HIP(hipMemcpyAsync(dpt, pe, M.n_psi * sizeof(double),
                                                   hipMemcpyDeviceToDevice, s));
                            S.step_extensions += 1;
                            t = te;
                        }
                        break;
                    }
                    t *= 0.5;
                    S.line_search_halvings += 1;
                }
            }
            if (trace)
                std::fprintf(stderr, "hpg: prox %d newton %d err %.3e krylov %d step %s\n", k, it,
                             err, its, acc ? std::to_string(t).c_str() : "rejected");
            if (!acc) {
                conv = err <= o.stall_tol;
                break;
            }
            std::swap(du, dut);
            std::swap(dp, dpt);
        }
        alpha_used = alpha_k;
        if (trace)
            std::fprintf(stderr, "hpg: prox %d alpha %g %s err %.3e\n", k, alpha_k,
                         conv ? "converged" : "NOT converged", last_err);
        if (!conv) {
            ok = false;
            // the multiplier of the unfinished step, for the diagnostics
            dev::launch_lambda(M.n_psi, dpp, dp, alpha_k, dlam, s);
            have_lam = true;
            break;
        }
        // lambda_k and psi_prev <- psi
        const bool last_possible = (k == kmax);
        double nrm_u;
        const double diff = l2_diff(du, u_old.as<double>(), &nrm_u, s);
        const bool stop = o.fixed_prox_steps > 0 ? last_possible
                                                 : (diff <= o.prox_tol * nrm_u || last_possible);
        if (stop) {
            dev::launch_lambda(M.n_psi, dpp, dp, alpha_k, dlam, s);
            have_lam = true;
        }
        HPG_HIP(hipMemcpyAsync(dpp, dp, M.n_psi * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (stop) break;
        alpha_k = std::min(alpha_k * o.alpha_factor, o.alpha_max);
    }
    // outputs
    if (!have_lam) HPG_HIP(hipMemsetAsync(dlam, 0, M.n_psi * sizeof(double), s));
    if (d_lam_out)
        HPG_HIP(hipMemcpyAsync(d_lam_out, dlam, M.n_psi * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_u_out) HPG_HIP(hipMemcpyAsync(d_u_out, du, M.n_u * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_psi_out)
        HPG_HIP(hipMemcpyAsync(d_psi_out, dp, M.n_psi * sizeof(double), hipMemcpyDeviceToDevice, s));
    diagnostics(du, dp, dlam, s, &S.complementarity, &S.complementarity_rel, &S.max_violation);
    HPG_HIP(hipStreamSynchronize(s));
    S.fp64_recomputations = recomputed;
    // keep the internal buffers pointing at the final iterate
    if (du != u.as<double>()) u.swap(ut);
    if (dp != psi.as<double>()) psi.swap(pt);
    auto t1 = std::chrono::steady_clock::now();
    S.prox_steps = k;
    S.newton_error = last_err;
    S.alpha_last = alpha_used;
    S.seconds = std::chrono::duration<double>(t1 - t0).count();
    S.status = ok ? HPG_OK : HPG_NOT_CONVERGED;
    if (st) *st = S;
    return S.status;
}

template void Problem::apply_G<double>(const double*, double*, double*, const int*, hipStream_t);
template void Problem::apply_G<float>(const float*, float*, double*, const int*, hipStream_t);
template void Problem::apply_prec<double>(const double*, double*, double*, const int*, hipStream_t,
                                          const VhatIn<double>*);
template void Problem::apply_prec<float>(const float*, float*, double*, const int*, hipStream_t,
                                         const VhatIn<float>*);
template int Problem::minres<double>(const double*, double*, double, int, int, hipStream_t);
template int Problem::minres_on<double>(const double*, double*, double, int, int, hipStream_t);
template int Problem::minres_on<float>(const float*, float*, double, int, int, hipStream_t);
template void Problem::minres_iterations<double>(int, int, double*&, double*&, double*&, double*&,
                                                 double*, double*, double*, double*, hipStream_t);
template void Problem::minres_iterations<float>(int, int, float*&, float*&, float*&, float*&,
                                                float*, float*, float*, float*, hipStream_t);
template int Problem::minres<float>(const float*, float*, double, int, int, hipStream_t);
template void Problem::tune_fdm<double>(hipStream_t);
template void Problem::tune_fdm<float>(hipStream_t);

}  // namespace hpg
