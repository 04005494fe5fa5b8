// Serving: continuous batching of independent LVPP solves on one GPU.
//
// Each request is a whole solve of the problem of Sec. 2 on its own mesh.
// Worker threads (one per slot) take requests in arrival order as soon as a
// slot is free and the request's HBM footprint fits in what the running
// requests leave of the budget; each runs on its own device buffers and
// non-blocking HIP streams, so the solves of different requests overlap on
// the device.  Nothing is shared between requests except the block cache of
// the device allocator, so a result is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "problem.h"

namespace hpg {
namespace {

using Clock = std::chrono::steady_clock;

double seconds_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
}

struct Request {
    enum State { QUEUED, RUNNING, DONE };
    uint64_t ticket = 0;
    Mesh mesh;
    std::vector<double> f, phi;
    std::vector<double> warm_u, warm_psi;   // copies of a warm start's vectors
    hpg_solve_opts opts{};
    size_t footprint = 0;
    Clock::time_point t_submit, t_start, t_done;
    State state = QUEUED;
    hpg_status status = HPG_OK;
    std::string error;
    std::vector<double> u, psi;
    hpg_solve_stats stats{};
    size_t device_bytes = 0;
};

}  // namespace

struct Server {
    int device = 0;
    size_t budget = 0;
    int slots = 1;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> live;   // not yet retrieved
    uint64_t next_ticket = 1;
    size_t reserved = 0, peak_reserved = 0;
    int running = 0, max_running = 0;
    bool stop = false;
    int waiters = 0;   // calls inside hpg_server_poll / hpg_server_wait

    int64_t submitted = 0, completed = 0, failed = 0;
    std::vector<double> latencies;
    double dof_iters = 0.0;
    bool any_submit = false;
    Clock::time_point first_submit, last_done;

    std::vector<std::thread> workers;

    void worker_loop();
    void run(Request& r);
};

// one request on a fresh problem (own buffers, own streams); the problem's
// destructor waits for its streams before its buffers are released
void Server::run(Request& r) {
    size_t& counter = device_bytes_counter();
    const size_t before = counter;
    Problem P;
    P.single_stream = true;
    P.build(r.mesh, device);
    P.set_data(r.f.data(), r.phi.data());
    r.status = P.solve(r.opts, P.own_stream, &r.stats, nullptr, nullptr, nullptr);
    r.u.resize(r.mesh.n_u);
    r.psi.resize(r.mesh.n_psi);
    HPG_HIP(hipMemcpyAsync(r.u.data(), P.u.p, r.u.size() * sizeof(double), hipMemcpyDeviceToHost,
                           P.own_stream));
    HPG_HIP(hipMemcpyAsync(r.psi.data(), P.psi.p, r.psi.size() * sizeof(double),
                           hipMemcpyDeviceToHost, P.own_stream));
    HPG_HIP(hipStreamSynchronize(P.own_stream));
    r.device_bytes = counter - before;
}

void Server::worker_loop() {
    const hipError_t dev_err = hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // admit the oldest request once a slot and its memory are free; a lone
        // request always fits (its footprint was checked against the budget)
        cv_work.wait(lk, [&] {
            return stop || (!queue.empty() &&
                            (running == 0 || reserved + queue.front()->footprint <= budget));
        });
        if (stop) return;
        std::shared_ptr<Request> r = queue.front();
        queue.pop_front();
        reserved += r->footprint;
        peak_reserved = std::max(peak_reserved, reserved);
        ++running;
        max_running = std::max(max_running, running);
        r->state = Request::RUNNING;
        r->t_start = Clock::now();
        lk.unlock();
        if (dev_err != hipSuccess) {
            r->status = HPG_ERR_DEVICE;
            r->error = std::string("hipSetDevice: ") + hipGetErrorString(dev_err);
        } else {
            try {
                run(*r);
            } catch (const Error& e) {
                r->status = e.code;
                r->error = e.msg;
            } catch (const std::bad_alloc&) {
                r->status = HPG_ERR_NOMEM;
                r->error = "host allocation failed";
            } catch (...) {
                r->status = HPG_ERR_DEVICE;
                r->error = "unexpected internal error";
            }
        }
        const auto t_done = Clock::now();
        lk.lock();
        r->t_done = t_done;
        r->state = Request::DONE;
        reserved -= r->footprint;
        --running;
        if (r->status < 0) {
            ++failed;
        } else {
            ++completed;
            latencies.push_back(seconds_between(r->t_submit, t_done));
            dof_iters += (double)(r->mesh.n_u + r->mesh.n_psi) * (double)r->stats.krylov_iters;
            last_done = t_done;
        }
        r->f.clear();
        r->f.shrink_to_fit();
        r->phi.clear();
        r->phi.shrink_to_fit();
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    // nearest-rank percentile
    const size_t k = (size_t)std::ceil(q * (double)v.size());
    return v[std::min(v.size() - 1, k == 0 ? 0 : k - 1)];
}

}  // namespace hpg

struct hpg_server {
    hpg::Server S;
};

using namespace hpg;

namespace {

// copy out a finished request and release its ticket (lock held by caller)
hpg_status retrieve(Server& S, std::map<uint64_t, std::shared_ptr<Request>>::iterator it,
                    double* u_out, double* psi_out, hpg_solve_stats* stats,
                    hpg_request_info* info) {
    std::shared_ptr<Request> r = it->second;
    S.live.erase(it);
    if (u_out && !r->u.empty()) std::memcpy(u_out, r->u.data(), r->u.size() * sizeof(double));
    if (psi_out && !r->psi.empty())
        std::memcpy(psi_out, r->psi.data(), r->psi.size() * sizeof(double));
    if (stats) *stats = r->stats;
    if (info) {
        info->queue_s = seconds_between(r->t_submit, r->t_start);
        info->run_s = seconds_between(r->t_start, r->t_done);
        info->latency_s = seconds_between(r->t_submit, r->t_done);
        info->footprint = r->footprint;
        info->device_bytes = r->device_bytes;
    }
    if (r->status < 0) fail(r->status, r->error);
    return r->status;
}

hpg_status poll_or_wait(hpg_server* srv, uint64_t ticket, double* u_out, double* psi_out,
                        hpg_solve_stats* stats, hpg_request_info* info, bool block) {
    return guarded([&]() -> hpg_status {
        if (!srv) fail(HPG_ERR_INVALID_ARG, "server handle is NULL");
        Server& S = srv->S;
        std::unique_lock<std::mutex> lk(S.mu);
        // counted while inside, so that hpg_server_destroy frees the server
        // only after the last caller has left (destructor runs with lk held)
        struct Inside {
            Server& S;
            explicit Inside(Server& s) : S(s) { ++S.waiters; }
            ~Inside() {
                --S.waiters;
                S.cv_done.notify_all();
            }
        } inside(S);
        auto it = S.live.find(ticket);
        if (it == S.live.end()) fail(HPG_ERR_INVALID_ARG, "unknown or already retrieved ticket");
        if (block) {
            std::shared_ptr<Request> r = it->second;
            S.cv_done.wait(lk, [&] { return r->state == Request::DONE; });
            it = S.live.find(ticket);
            if (it == S.live.end()) fail(HPG_ERR_INVALID_ARG, "ticket retrieved by another caller");
        } else if (it->second->state != Request::DONE) {
            return HPG_PENDING;
        }
        return retrieve(S, it, u_out, psi_out, stats, info);
    });
}

}  // namespace

extern "C" {

hpg_status hpg_problem_footprint(const hpg_mesh* mesh, int32_t precision, uint64_t* bytes) {
    return guarded([&]() -> hpg_status {
        if (!mesh || !bytes) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        if (precision != HPG_FP64 && precision != HPG_MIXED)
            fail(HPG_ERR_INVALID_ARG, "precision must be HPG_FP64 or HPG_MIXED");
        *bytes = footprint_bytes(mesh->M, precision);
        return HPG_OK;
    });
}

hpg_status hpg_server_create(int device, uint64_t hbm_budget, int32_t max_slots,
                             hpg_server** out) {
    return guarded([&]() -> hpg_status {
        if (!out) fail(HPG_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (max_slots < 1 || max_slots > 256) fail(HPG_ERR_INVALID_ARG, "max_slots must be 1..256");
        int ndev = 0;
        HPG_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) fail(HPG_ERR_INVALID_ARG, "no such device");
        HPG_HIP(hipSetDevice(device));
        size_t budget = hbm_budget;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            HPG_HIP(hipMemGetInfo(&fr, &tot));
            budget = (size_t)(0.9 * (double)fr);
        }
        auto* srv = new hpg_server();
        Server& S = srv->S;
        S.device = device;
        S.budget = budget;
        S.slots = max_slots;
        try {
            for (int i = 0; i < max_slots; ++i) S.workers.emplace_back([&S] { S.worker_loop(); });
        } catch (...) {
            {
                std::lock_guard<std::mutex> lk(S.mu);
                S.stop = true;
            }
            S.cv_work.notify_all();
            for (auto& t : S.workers) t.join();
            delete srv;
            throw;
        }
        *out = srv;
        return HPG_OK;
    });
}

hpg_status hpg_server_submit(hpg_server* srv, const hpg_mesh* mesh, const double* f_qp,
                             const double* phi_qp, const hpg_solve_opts* opts, uint64_t* ticket) {
    return guarded([&]() -> hpg_status {
        if (!srv || !mesh || !f_qp || !phi_qp || !ticket)
            fail(HPG_ERR_INVALID_ARG, "NULL argument");
        *ticket = 0;
        Server& S = srv->S;
        auto r = std::make_shared<Request>();
        r->mesh = mesh->M;
        r->opts = checked_opts(opts);
        if (r->opts.warm_u) {
            r->warm_u.assign(r->opts.warm_u, r->opts.warm_u + r->mesh.n_u);
            r->warm_psi.assign(r->opts.warm_psi, r->opts.warm_psi + r->mesh.n_psi);
            r->opts.warm_u = r->warm_u.data();
            r->opts.warm_psi = r->warm_psi.data();
        }
        const size_t nq = (size_t)r->mesh.n_qp;
        r->f.assign(f_qp, f_qp + nq);
        r->phi.assign(phi_qp, phi_qp + nq);
        for (size_t i = 0; i < nq; ++i) {
            if (!std::isfinite(r->f[i]) || !std::isfinite(r->phi[i]))
                fail(HPG_ERR_NUMERIC, "non-finite f or phi");
            if (r->mesh.kind == HPG_GRADIENT && !(r->phi[i] > 0.0))
                fail(HPG_ERR_INVALID_ARG, "gradient constraint needs phi > 0");
        }
        r->footprint = footprint_bytes(r->mesh, r->opts.precision);
        if (r->opts.step_extension)   // the trial iterate of an extended Newton step
            r->footprint += (size_t)(r->mesh.n_u + r->mesh.n_psi) * sizeof(double);
        if (r->footprint > S.budget)
            fail(HPG_ERR_BUDGET, "request footprint exceeds the server's HBM budget");
        {
            std::lock_guard<std::mutex> lk(S.mu);
            if (S.stop) fail(HPG_ERR_INVALID_ARG, "server is shutting down");
            r->ticket = S.next_ticket++;
            r->t_submit = Clock::now();
            if (!S.any_submit) {
                S.any_submit = true;
                S.first_submit = r->t_submit;
            }
            ++S.submitted;
            S.live[r->ticket] = r;
            S.queue.push_back(r);
            *ticket = r->ticket;
        }
        S.cv_work.notify_one();
        return HPG_OK;
    });
}

hpg_status hpg_server_poll(hpg_server* srv, uint64_t ticket, double* u_out, double* psi_out,
                           hpg_solve_stats* stats, hpg_request_info* info) {
    return poll_or_wait(srv, ticket, u_out, psi_out, stats, info, false);
}

hpg_status hpg_server_wait(hpg_server* srv, uint64_t ticket, double* u_out, double* psi_out,
                           hpg_solve_stats* stats, hpg_request_info* info) {
    return poll_or_wait(srv, ticket, u_out, psi_out, stats, info, true);
}

hpg_status hpg_server_stats(hpg_server* srv, hpg_serving_stats* out) {
    return guarded([&]() -> hpg_status {
        if (!srv || !out) fail(HPG_ERR_INVALID_ARG, "NULL argument");
        Server& S = srv->S;
        std::lock_guard<std::mutex> lk(S.mu);
        std::memset(out, 0, sizeof(*out));
        out->submitted = S.submitted;
        out->completed = S.completed;
        out->failed = S.failed;
        out->queued = (int64_t)S.queue.size();
        out->running = S.running;
        out->max_running = S.max_running;
        out->p50_latency_s = percentile(S.latencies, 0.50);
        out->p99_latency_s = percentile(S.latencies, 0.99);
        double sum = 0.0, mx = 0.0;
        for (double v : S.latencies) {
            sum += v;
            mx = std::max(mx, v);
        }
        out->mean_latency_s = S.latencies.empty() ? 0.0 : sum / (double)S.latencies.size();
        out->max_latency_s = mx;
        if (S.completed > 0) {
            out->span_s = seconds_between(S.first_submit, S.last_done);
            if (out->span_s > 0) {
                out->solves_per_s = (double)S.completed / out->span_s;
                out->dof_krylov_per_s = S.dof_iters / out->span_s;
            }
        }
        out->hbm_budget = S.budget;
        out->hbm_reserved = S.reserved;
        out->hbm_peak_reserved = S.peak_reserved;
        return HPG_OK;
    });
}

void hpg_server_destroy(hpg_server* srv) {
    if (!srv) return;
    Server& S = srv->S;
    {
        // queued requests never run: they complete with an error, which wakes
        // any caller blocked in hpg_server_wait on them
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
        const auto now = Clock::now();
        for (auto& r : S.queue) {
            r->state = Request::DONE;
            r->status = HPG_ERR_INVALID_ARG;
            r->error = "server destroyed before the request ran";
            r->t_start = r->t_done = now;
            ++S.failed;
        }
        S.queue.clear();
    }
    S.cv_done.notify_all();
    S.cv_work.notify_all();
    for (auto& t : S.workers) t.join();
    {
        // callers already inside poll / wait leave before the server is freed
        std::unique_lock<std::mutex> lk(S.mu);
        S.cv_done.wait(lk, [&] { return S.waiters == 0; });
    }
    delete srv;
}

}  // extern "C"
