/*
 * hpg.h - C ABI of the MI355X hierarchical proximal Galerkin (hpG) library.
 *
 * The library solves the obstacle problem (u <= phi) and the gradient-type
 * problem (|grad u| <= phi) for the Dirichlet energy on a tensor-product
 * domain (0,1)^d, d = 1, 2, 3 (paper: Sec. 2 problem setup; d = 3 as in
 * Sec. 6.5), with homogeneous Dirichlet conditions, by the latent-variable
 * proximal point method discretised with the hierarchical p-FEM basis
 * (Sec. 2.1-2.2, Sec. 3, Sec. 4).  Each proximal subproblem eq. (pG) /
 * eq. (pG:gradient) is solved by Newton's method; every Newton system
 * eq. (pG-matrix) is solved matrix-free on the GPU by preconditioned MINRES
 * with the block-diagonal preconditioner P_D of eq. (schur4) and the Schur
 * approximation of eq. (schur-preconditioner) (obstacle) or
 * eq. (schur-preconditioner:gradient) (gradient).
 *
 * Conventions used by every call:
 *  - Mesh: per direction k a breakpoint vector 0 = x_0 < ... < x_{m_k} = 1
 *    (Sec. 3).  Cells are numbered lexicographically, direction 0 fastest.
 *    One partial degree p on every cell (p >= 2 obstacle, p >= 1 gradient).
 *  - u unknowns (U_{0,h,p}): per direction n1_k = m_k p - 1; the hat of
 *    interior vertex v is 1-D unknown v p - 1, bubble W_n of cell c is
 *    c p + n; the d-D vector is the n1_0 x ... x n1_{d-1} array, direction 0
 *    fastest.  Coefficients are w.r.t. the hats and W_n of eq. (Wn).
 *  - psi unknowns (Psi_{h,p}, Legendre P_n, Sec. 3): cell-major; inside a cell
 *    the Legendre multi-index with direction 0 fastest, P = p-1 (obstacle) or
 *    P = p (gradient) modes per direction; gradient: d components per cell,
 *    component-major.
 *  - Quadrature points: tensor Gauss-Legendre, q = p+1 per direction per
 *    cell; cell-major, direction 0 fastest inside a cell.  Data f and phi are
 *    given by their values at these points, which define the discrete problem.
 *  - All host pointers are owned by the caller and only read/written during
 *    the call.  Device pointers (hpg_solve_device, hpg_op_*) are caller-owned
 *    device memory on the problem's device; work is enqueued on the given HIP
 *    stream (NULL = the HIP null stream, as for HIP runtime calls) and the
 *    call returns after that stream has finished.  hpg_solve (host buffers)
 *    runs on a stream the library owns.
 *  - Every call returns a status; none aborts.  On error hpg_last_error()
 *    returns a thread-local message.
 */
#ifndef HPG_H
#define HPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hpg_status;
#define HPG_OK 0
#define HPG_NOT_CONVERGED 1      /* outputs written: best iterate so far */
#define HPG_PENDING 2            /* serving: result not ready yet */
#define HPG_ERR_INVALID_ARG (-1)
#define HPG_ERR_NOMEM (-2)
#define HPG_ERR_DEVICE (-3)
#define HPG_ERR_NUMERIC (-4)
#define HPG_ERR_BUDGET (-5)

#define HPG_OBSTACLE 0
#define HPG_GRADIENT 1

#define HPG_FP64 0               /* every GPU operation in FP64 */
#define HPG_MIXED 1              /* FP32 Krylov operator/preconditioner, FP64 Newton */

#define HPG_KRYLOV_MINRES 0      /* preconditioned MINRES on G with the SPD form of P_D */

typedef struct hpg_mesh hpg_mesh;
typedef struct hpg_problem hpg_problem;

/* Thread-local text of the last error (never NULL). */
const char* hpg_last_error(void);

/* ---- mesh (paper Sec. 3) ------------------------------------------------
 * dim: 1..3.  ncells[k]: cells in direction k (>= 1).  breaks: NULL for
 * uniform cells on (0,1), else breaks[k] points to ncells[k]+1 strictly
 * increasing values with breaks[k][0] = 0 and breaks[k][ncells[k]] = 1.
 * degree: NULL for one partial degree p on every cell (obstacle 2..24,
 * gradient 1..24; ncells[k] * p >= 2, so that every direction has an
 * interior u unknown).  Otherwise one degree per cell (2..24, cells numbered
 * with direction 0 fastest; obstacle constraint only; p is then ignored and
 * hpg_get_mesh_info reports the largest degree).  With per-cell degrees the u
 * space is the conforming one in which every vertex, edge, face and cell
 * interior carries the smallest degree of the cells containing it (the
 * hierarchical hats and bubbles of Sec. 3 are shared across cells); its
 * unknowns are numbered entity by entity: entities are the points of the
 * doubled grid (2 ncells[k] + 1 per direction, even = vertex coordinate, odd
 * = cell interval), direction 0 fastest, and inside an entity by the bubble
 * modes of its odd directions (first odd direction fastest, 0..p_E - 2).
 * psi holds (p_K - 1)^dim Legendre values per cell (cell-major) and each
 * cell has (p_K + 1)^dim Gauss points (cell-major, as hpg_quadrature_points
 * returns them).  constraint: HPG_OBSTACLE or HPG_GRADIENT.
 * Inputs are copied; the handle is freed with hpg_destroy_mesh.
 * Errors: HPG_ERR_INVALID_ARG for any out-of-range argument. */
hpg_status hpg_create_mesh(int dim, const int32_t* ncells, const double* const* breaks,
                           const int32_t* degree, int32_t p, int32_t constraint, hpg_mesh** out);
void hpg_destroy_mesh(hpg_mesh* mesh);

typedef struct hpg_mesh_info {
    int32_t dim, p, q, P, constraint;
    int32_t ncells[3];
    int64_t n_cells, n_u, n_psi, n_qp;
} hpg_mesh_info;

hpg_status hpg_get_mesh_info(const hpg_mesh* mesh, hpg_mesh_info* out);

/* Physical Gauss-Legendre points, xyz[i*dim + k] for point i (documented order). */
hpg_status hpg_quadrature_points(const hpg_mesh* mesh, double* xyz);

/* ---- problem: mesh + data + device state --------------------------------
 * device: HIP device ordinal.  Allocates the device tables and work buffers
 * (HPG_ERR_NOMEM / HPG_ERR_DEVICE on failure).  The mesh may be destroyed
 * afterwards (the problem keeps its own copy). */
hpg_status hpg_create_problem(const hpg_mesh* mesh, int device, hpg_problem** out);
/* Waits for the problem's own streams; work the caller enqueued on its own
 * streams through hpg_op_* must be complete before this call (the problem's
 * device buffers are handed to later problems of the process). */
void hpg_destroy_problem(hpg_problem* prob);

/* f and phi at the n_qp quadrature points (host arrays).  Non-finite values
 * give HPG_ERR_NUMERIC; for the gradient constraint phi must be > 0
 * (Sec. 2.2) else HPG_ERR_INVALID_ARG. */
hpg_status hpg_set_forcing(hpg_problem* prob, const double* f_qp, size_t n_qp);
hpg_status hpg_set_obstacle(hpg_problem* prob, const double* phi_qp, size_t n_qp);

/* Convenience forms: fn(x, ctx) is called on the calling thread once per
 * quadrature point, x = the point's dim coordinates (the order of
 * hpg_quadrature_points), and the values are then set as by hpg_set_forcing /
 * hpg_set_obstacle (same validation).  fn must not call into the library for
 * the same problem.  NULL fn: HPG_ERR_INVALID_ARG. */
typedef double (*hpg_point_fn)(const double* x, void* ctx);
hpg_status hpg_set_forcing_fn(hpg_problem* prob, hpg_point_fn fn, void* ctx);
hpg_status hpg_set_obstacle_fn(hpg_problem* prob, hpg_point_fn fn, void* ctx);

/* ---- solve options and statistics ---------------------------------------- */
typedef struct hpg_solve_opts {
    int32_t size;           /* sizeof(hpg_solve_opts), for ABI evolution */
    double alpha0;          /* alpha_1 (default 2) */
    double alpha_factor;    /* alpha_{k+1} = min(alpha_k * factor, alpha_max) (default 2) */
    double alpha_max;       /* default 1e300 (uncapped) */
    int32_t max_prox;       /* proximal step cap (default 60) */
    double prox_tol;        /* ||u_k - u_{k-1}||_L2 <= prox_tol ||u_k||_L2 (default 1e-10) */
    int32_t fixed_prox_steps; /* > 0: run exactly this many proximal steps */
    double newton_tol;      /* default 1e-12 (FP64), 1e-10 suggested for MIXED */
    double stall_tol;       /* line search failure accepted below this (default 1e-9) */
    int32_t max_newton;     /* per subproblem (default 60) */
    double krylov_rtol;     /* MINRES relative tolerance (default 1e-10) */
    int32_t max_krylov;     /* per Newton step (default 2000) */
    double beta;            /* E_beta weight, Jacobian only (default 0) */
    int32_t precision;      /* HPG_FP64 or HPG_MIXED */
    int32_t krylov_chunk;   /* iterations enqueued between convergence checks (default 16) */
    int32_t inexact_newton; /* 1: MINRES tolerance eta_k = clamp(1e-6 err_k, krylov_rtol, 1e-6)
                               from the current Newton error err_k (default 0: krylov_rtol) */
    int32_t step_extension; /* 1: when the full Newton step passes the line search, steps of
                               2, 4 and 8 times the direction are tried in turn and the last
                               one that lowers the merit further is taken (default 0: the
                               backtracking search alone) */
    int32_t q;              /* Gauss-Legendre points per direction: 0 (default) or p + 1, the
                               only rule built; any other value is HPG_ERR_INVALID_ARG */
    int32_t krylov;         /* HPG_KRYLOV_MINRES (default); any other value is
                               HPG_ERR_INVALID_ARG */
    /* Warm start / resume (Sec. 2.1: subproblem k depends only on psi_{k-1}):
     * with k0 >= 0 and both vectors given, the solve starts from the state
     * after k0 proximal steps, (u_{k0}, psi_{k0}) = (warm_u, warm_psi): step
     * k0 + 1 uses alpha_{k0+1} = min(alpha0 factor^k0, alpha_max), psi_prev =
     * warm_psi and the Newton initial guess (warm_u, warm_psi); the outer
     * stop compares u_{k0+1} with warm_u; max_prox and fixed_prox_steps count
     * from step 1, so a solve resumed at k0 runs steps k0 + 1 .. of the same
     * sequence and, in FP64 mode, returns bit for bit what the uninterrupted
     * solve returns (a mixed solve restarts its count of FP64 recomputations).
     * Pointers: host memory for hpg_solve and hpg_server_submit (copied),
     * device memory on the problem's device for hpg_solve_device; read only.
     * Both NULL (default): u_0 = psi_0 = 0 and k0 must be 0.  Exactly one
     * NULL, k0 < 0 or k0 >= the step cap: HPG_ERR_INVALID_ARG. */
    const double* warm_u;
    const double* warm_psi;
    int32_t k0;
} hpg_solve_opts;

void hpg_default_opts(hpg_solve_opts* opts);

typedef struct hpg_solve_stats {
    int32_t status;
    int32_t prox_steps;
    int32_t newton_iters;
    int32_t line_search_halvings;
    int64_t krylov_iters;
    double newton_error;    /* last Newton error of the last subproblem */
    double seconds;         /* wall time of the solve */
    double alpha_last;
    int32_t fp64_fallbacks; /* HPG_MIXED: Newton directions computed with the FP64 operator:
                               the FP64 recomputations below, and, after three of those
                               within one proximal step, the rest of that step's directions
                               (after twelve over the solve, every later direction) */
    int32_t step_extensions; /* Newton steps lengthened beyond the full step (step_extension) */
    int32_t fp64_recomputations; /* HPG_MIXED: FP32 directions that broke down, hit the Krylov
                                    cap or were rejected by the line search, and were computed
                                    again with the FP64 operator */
    /* Diagnostics of the returned iterate, evaluated on the device at the
     * n_qp Gauss points with lambda = (psi_{K-1} - psi_K) / alpha_K of the
     * last proximal step K (Sec. 2.1):
     * complementarity = sum_K sum_q w_q |J_K| |lambda_h(x_q)| exp(-psi_h(x_q))
     *   (obstacle; the products of the multiplier and the latent gap
     *   exp(-psi) = phi - u~ vanish at the limit), complementarity_rel = that
     *   sum / (sum_K sum_q w_q |J_K| |lambda_h(x_q)| * max_q |phi_q|); both 0
     *   for the gradient constraint, whose multiplier is a vector field;
     * max_violation = max_q (u_h(x_q) - phi_q) (obstacle) or
     *   max_q (|grad u_h(x_q)| - phi_q) (gradient): pointwise feasibility at
     *   the Gauss points (<= 0 when feasible there). */
    double complementarity;
    double complementarity_rel;
    double max_violation;
} hpg_solve_stats;

/* Solve; u_out[n_u], psi_out[n_psi] (psi may be NULL), lam_out[n_psi]
 * (lambda_K = (psi_{K-1} - psi_K)/alpha_K, may be NULL).  Host buffers.
 * Returns HPG_OK, HPG_NOT_CONVERGED (outputs hold the last iterate) or an error. */
hpg_status hpg_solve(hpg_problem* prob, const hpg_solve_opts* opts, double* u_out,
                     double* psi_out, double* lam_out, hpg_solve_stats* stats);

/* Same with caller-owned device buffers d_u[n_u], d_psi[n_psi] (FP64) on the
 * problem's device, enqueued on `stream` (a hipStream_t; NULL = null stream). */
hpg_status hpg_solve_device(hpg_problem* prob, const hpg_solve_opts* opts, double* d_u,
                            double* d_psi, void* stream, hpg_solve_stats* stats);

/* ---- operator-level calls (the Newton linear system of eq. (pG-matrix)) ---
 * hpg_op_setup linearises at psi (device, FP64, n_psi) for step size alpha
 * and E_beta weight beta: computes the quadrature weights omega of D_psi
 * (Sec. 4.3) and the inverted cell blocks of -S_hat (Sec. 4.5/4.6).
 * precision selects the element type of the hpg_op_apply_* vectors:
 * double for HPG_FP64, float for HPG_MIXED.  Vectors have n_u + n_psi
 * entries, u first. */
hpg_status hpg_op_setup(hpg_problem* prob, const double* d_psi, double alpha, double beta,
                        int32_t precision, void* stream);
/* y = G x, G = [[alpha A, B], [B^T, -D_psi - E_beta]] (eq. (pG-matrix)). */
hpg_status hpg_op_apply_G(hpg_problem* prob, const void* d_x, void* d_y, void* stream);
/* z = diag(alpha A, -S_hat)^{-1} r (SPD form of P_D, eq. (schur4)). */
hpg_status hpg_op_apply_prec(hpg_problem* prob, const void* d_r, void* d_z, void* stream);
/* Solve G x = b by preconditioned MINRES from x = 0; *iters = iterations. */
hpg_status hpg_op_minres(hpg_problem* prob, const void* d_b, void* d_x, double rtol,
                         int32_t max_iters, int32_t* iters, void* stream);
/* FP64 residual of eq. (pG) / eq. (pG:gradient) at (u, psi) with previous
 * latent iterate psi_prev and step alpha: R (n_u + n_psi, FP64, u first). */
hpg_status hpg_op_residual(hpg_problem* prob, const double* d_u, const double* d_psi,
                           const double* d_psi_prev, double alpha, double* d_R, void* stream);
/* hpg_op_residual for callers that cannot allocate memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * kernels and the same R, with their scratch (per-block partial sums and, on
 * meshes with one degree per cell, the per-local-function values of the cell
 * pass) in a fixed device array of the library, 8 MiB per device, held until
 * the process ends; the call allocates no device or host memory.  norms2
 * (host, may be NULL) receives ||R_u||_2^2 and ||R_psi||_2^2.  Meshes needing
 * more than 8192 partial sums or 1040384 local values: HPG_ERR_INVALID_ARG.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (several host threads or streams) race and must be serialised
 * by the caller.  Returns after `stream` has finished the call's work. */
hpg_status hpg_op_residual_noalloc(hpg_problem* prob, const double* d_u, const double* d_psi,
                                   const double* d_psi_prev, double alpha, double* d_R,
                                   double* norms2, void* stream);

/* L2 norms in function space (Gauss-Legendre, exact for degree 2p):
 * *diff = ||a_h - b_h||_{L2(Omega)}, *norm_b = ||b_h||_{L2(Omega)} for u
 * coefficient vectors a, b (device, FP64, n_u). */
hpg_status hpg_l2_diff(hpg_problem* prob, const double* d_a, const double* d_b, double* diff,
                       double* norm_b, void* stream);

/* ---- kernel timing (for measurement harnesses) ----------------------------
 * group NULL disables timing; "all" times every group; otherwise only the
 * named group ("apply_G" (fused tiled apply), "apply_G_u", "apply_G_psi" (the
 * two-kernel apply used where no tiled variant exists), "fdm", "prec_psi",
 * "minres_vec", "setup", "residual") is timed.  While enabled, every launch of a timed
 * group gets a pair of HIP events: recorded by the kernel's dispatch itself for
 * "apply_G" and "fdm" (one GEMM pass per launch), recorded on the launch stream
 * around the group's launches for the others;
 * hpg_kernel_time returns the number of bracketed launches and their summed
 * duration in milliseconds.  Enabling resets the counters. */
hpg_status hpg_set_kernel_timing(hpg_problem* prob, const char* group);
hpg_status hpg_kernel_time(hpg_problem* prob, const char* group, int64_t* launches,
                           double* total_ms);

/* ---- batched solves: many problems of one mesh shape in each launch -------
 * Independent problems on the same mesh (the same breakpoints, degree p and
 * obstacle constraint; the Sec. 2 problem with its own f and phi each) solved
 * together in nbatch slots: each step of the inner Newton solve (Sec. 4: the
 * G apply of eq. (pG-matrix), the preconditioner P_D of eq. (schur4), the
 * Lanczos updates, the Newton residual, the linearisation) of the requests in
 * the slots is one launch, with per-request reductions in the order of a
 * solve of that request alone.  Each request runs its own proximal, Newton
 * and line-search sequence at its own pace (a request whose Krylov solve
 * ends goes on while the others' continue), and a slot whose request
 * finishes takes the next one, so its result does not depend on the others.
 * Supported: obstacle constraint, one degree on every cell, p <= 12 in
 * 1-D/2-D and p <= 7 in 3-D (the fused tiled apply) with Schur blocks of at
 * most 48 KB (HPG_ERR_INVALID_ARG otherwise).
 * hpg_batch_set_data: f and phi of nreq requests (n_values = nreq n_qp, any
 *   nreq >= 1), request-major: request r's values are [r n_qp, (r+1) n_qp).
 * hpg_batch_solve: options as for hpg_solve (step_extension, inexact_newton
 *   and warm starts: HPG_ERR_INVALID_ARG); outputs per request, request-major
 *   (u_out[nreq n_u], psi_out and lam_out [nreq n_psi], stats[nreq], where
 *   seconds is the time from the request's start in a slot to its end);
 *   returns HPG_OK if every request converged, else HPG_NOT_CONVERGED
 *   (outputs written for all).
 * hpg_batch_op_setup / hpg_batch_op_apply_G: the linearisation and G of all
 *   requests at once (device psi[nbatch n_psi], x and y [nbatch (n_u + n_psi)],
 *   request b's vector at offset b (n_u + n_psi), u first; float vectors for
 *   HPG_MIXED).
 * hpg_batch_set_kernel_timing / hpg_batch_kernel_time: as the hpg_problem
 *   forms, for the batch's launches. */
typedef struct hpg_batch hpg_batch;
hpg_status hpg_create_batch(const hpg_mesh* mesh, int32_t nbatch, int device, hpg_batch** out);
void hpg_destroy_batch(hpg_batch* batch);
hpg_status hpg_batch_set_data(hpg_batch* batch, const double* f_qp, const double* phi_qp,
                              size_t n_values);
hpg_status hpg_batch_solve(hpg_batch* batch, const hpg_solve_opts* opts, double* u_out,
                           double* psi_out, double* lam_out, hpg_solve_stats* stats);
hpg_status hpg_batch_op_setup(hpg_batch* batch, const double* d_psi, double alpha, double beta,
                              int32_t precision, void* stream);
hpg_status hpg_batch_op_apply_G(hpg_batch* batch, const void* d_x, void* d_y, void* stream);
hpg_status hpg_batch_set_kernel_timing(hpg_batch* batch, const char* group);
hpg_status hpg_batch_kernel_time(hpg_batch* batch, const char* group, int64_t* launches,
                                 double* total_ms);

/* ---- serving: continuous batching of independent solves on one GPU --------
 * A request is one whole LVPP solve (the problem statement of Sec. 2 on its
 * own mesh, degree and constraint).  The server admits requests in arrival
 * order while both a slot and HBM are free: the sum of the admitted requests'
 * footprints (hpg_problem_footprint) stays within hbm_budget and at most
 * max_slots solves run at once.  Each admitted request gets its own device
 * buffers and HIP streams and runs on its own worker thread, so requests that
 * arrive while others are on the GPU start as soon as a slot and memory free
 * up and their kernels overlap on the device.  The result of a request does
 * not depend on what else runs (every reduction has a fixed order).
 *
 * hpg_problem_footprint: upper estimate, in bytes, of the device memory a
 *   solve on `mesh` at `precision` (HPG_FP64 / HPG_MIXED) allocates.
 * hpg_server_create: `device` is the HIP device; hbm_budget in bytes (0 = 90%
 *   of the device's free memory at creation); max_slots >= 1 worker threads.
 * hpg_server_submit: copies the mesh, f and phi at the mesh's n_qp quadrature
 *   points (hpg_quadrature_points) and the options; returns a ticket.  The
 *   caller may free its inputs on return.  HPG_ERR_BUDGET if the request's
 *   footprint alone exceeds the budget; HPG_ERR_INVALID_ARG for bad input.
 * hpg_server_poll: HPG_PENDING while the request is queued or running.  Once
 *   done it writes u_out[n_u], psi_out[n_psi], *stats and *info (each may be
 *   NULL), releases the ticket and returns the solve's status; a later call
 *   with the same ticket is HPG_ERR_INVALID_ARG.  A solve that failed returns
 *   its error status and hpg_last_error() its message.
 * hpg_server_wait: as poll, blocking until the request is done.
 * hpg_server_stats: counts, latency percentiles (submission to completion)
 *   and throughput over the requests completed so far.
 * hpg_server_destroy: queued requests complete at once with
 *   HPG_ERR_INVALID_ARG ("server destroyed before the request ran"), which
 *   wakes callers blocked in hpg_server_wait on them; running requests finish;
 *   callers already inside hpg_server_poll / hpg_server_wait return before the
 *   server is freed.  No call on the handle may start once destroy has begun.
 * Warm starts (hpg_solve_opts.warm_u / warm_psi, host pointers) are copied by
 * hpg_server_submit. */
typedef struct hpg_server hpg_server;

typedef struct hpg_request_info {
    double queue_s;           /* submission to admission */
    double run_s;             /* admission to completion */
    double latency_s;         /* submission to completion */
    uint64_t footprint;       /* bytes reserved at admission */
    uint64_t device_bytes;    /* bytes the solve actually allocated */
} hpg_request_info;

typedef struct hpg_serving_stats {
    int64_t submitted, completed, failed, queued, running;
    int32_t max_running;      /* most solves on the device at once */
    double p50_latency_s, p99_latency_s, mean_latency_s, max_latency_s;
    double span_s;            /* first submission to last completion */
    double solves_per_s;      /* completed / span_s */
    double dof_krylov_per_s;  /* sum over completed of (n_u + n_psi) * Krylov iterations / span_s */
    uint64_t hbm_budget, hbm_reserved, hbm_peak_reserved;
} hpg_serving_stats;

/* Device bytes one solve of this mesh holds at precision (HPG_FP64 / HPG_MIXED)
 * with default options; a request with step_extension on is admitted with
 * (n_u + n_psi) doubles more. */
hpg_status hpg_problem_footprint(const hpg_mesh* mesh, int32_t precision, uint64_t* bytes);
hpg_status hpg_server_create(int device, uint64_t hbm_budget, int32_t max_slots,
                             hpg_server** out);
hpg_status hpg_server_submit(hpg_server* srv, const hpg_mesh* mesh, const double* f_qp,
                             const double* phi_qp, const hpg_solve_opts* opts, uint64_t* ticket);
hpg_status hpg_server_poll(hpg_server* srv, uint64_t ticket, double* u_out, double* psi_out,
                           hpg_solve_stats* stats, hpg_request_info* info);
hpg_status hpg_server_wait(hpg_server* srv, uint64_t ticket, double* u_out, double* psi_out,
                           hpg_solve_stats* stats, hpg_request_info* info);
hpg_status hpg_server_stats(hpg_server* srv, hpg_serving_stats* out);
void hpg_server_destroy(hpg_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* HPG_H */
