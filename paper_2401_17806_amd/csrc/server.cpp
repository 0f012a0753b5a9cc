// Continuous-batching server for independent pressure solves (the serving form of the
// Schur-CG) and IMEX time steps: requests are queued as they arrive, admitted while the
// device-memory budget and a free worker allow, and run concurrently on per-worker HIP
// streams, so work of different requests overlaps on the GPU.  A request owns its disc (CG
// workspace, and an IMEX step also its state) while it runs; requests on the same disc run one
// after another.  Results do not depend on the mix: every kernel uses fixed grids and
// fixed-order reductions, so a request's result is bitwise the same alone or overlapped.
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sld_internal.h"
#include "state_internal.h"

namespace {

struct Request {
    uint64_t ticket = 0;
    sld_disc disc = nullptr;
    const double* b = nullptr;
    double* p = nullptr;
    sld_cg_params params{};
    // IMEX step requests (state != nullptr): the step's parameters, time step and velocity
    sld_state state = nullptr;
    sld_imex_params iparams{};
    double dt = 0.0;
    double* v = nullptr;
    uint64_t bytes = 0;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream at submit
};

struct Result {
    bool done = false;
    int status = 0;
    sld_cg_report report{};
};

}  // namespace

struct sld_server_s {
    int device = 0;
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Result> results;
    std::unordered_set<sld_disc> busy;
    uint64_t in_flight_bytes = 0;
    uint64_t next_ticket = 1;
    uint64_t completed = 0;
    int running = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
};

uint64_t sld_disc_bytes(const sld_disc_s* d) {
    const uint64_t ne = d->mesh->ne, n = ne * (uint64_t)d->nphi;
    const uint64_t G = (uint64_t)d->cg.grid;
    // FP64 state (x, r/q/d ping-pong, b) + FP32 state + partials + operators
    return n * 8 * 8 + n * 4 * 7 + G * 8 * 20 + d->ops_bytes * 2;
}

namespace {

void worker_main(sld_server_s* s) {
    (void)hipSetDevice(s->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    while (true) {
        Request req;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            while (true) {
                if (s->stopping && s->queue.empty()) {
                    if (stream) (void)hipStreamDestroy(stream);
                    return;
                }
                // first queued request whose disc is free and that fits the budget (a request
                // is always admitted when nothing else runs, so none can starve)
                auto it = s->queue.begin();
                for (; it != s->queue.end(); ++it) {
                    if (s->busy.count(it->disc)) continue;
                    if (s->running == 0 || s->in_flight_bytes + it->bytes <= s->budget) break;
                }
                if (it != s->queue.end()) {
                    req = *it;
                    s->queue.erase(it);
                    s->busy.insert(req.disc);
                    s->in_flight_bytes += req.bytes;
                    ++s->running;
                    break;
                }
                s->cv_work.wait(lk);
            }
        }
        sld_cg_report rep{};
        int st = SLD_E_HIP;
        if (stream && hipStreamWaitEvent(stream, req.ready, 0) == hipSuccess) {
            if (req.state) {
                sld_imex_report irep{};
                st = sld_imex_step(req.state, &req.iparams, req.dt, req.v, req.p, &irep, stream);
                rep = irep.pressure;
            } else {
                st = sld_cg_solve(req.disc, req.b, req.p, &req.params, &rep, stream);
            }
        }
        (void)hipEventDestroy(req.ready);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            Result& r = s->results[req.ticket];
            r.done = true;
            r.status = st;
            r.report = rep;
            s->busy.erase(req.disc);
            s->in_flight_bytes -= req.bytes;
            --s->running;
            ++s->completed;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

sld_status sld_disc_footprint(sld_disc d, uint64_t* bytes) {
    if (!d || !bytes) {
        sld_set_error("sld_disc_footprint: NULL argument");
        return SLD_E_INVALID;
    }
    // + the mesh tables per triangle: geo, geo_i (32 B each), geo_nb (96 B), nbr, nbr_i, tedges
    // (16 B each), perm (4 B), the padded halo lists (a few B), the wall flags (1 B)
    *bytes = sld_disc_bytes(d) + uint64_t(d->mesh->ne) * 224;
    return SLD_OK;
}

sld_status sld_server_create(int32_t device, uint64_t hbm_budget_bytes, int32_t nworkers,
                             sld_server* out) {
    if (!out) {
        sld_set_error("sld_server_create: out is NULL");
        return SLD_E_INVALID;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        sld_set_error("sld_server_create: bad device ordinal");
        return SLD_E_INVALID;
    }
    if (nworkers < 1 || nworkers > 64 || hbm_budget_bytes == 0) {
        sld_set_error("sld_server_create: need 1 <= nworkers <= 64 and a nonzero budget");
        return SLD_E_INVALID;
    }
    sld_server_s* s = new (std::nothrow) sld_server_s();
    if (!s) {
        sld_set_error("sld_server_create: host allocation failed");
        return SLD_E_NOMEM;
    }
    s->device = device;
    s->budget = hbm_budget_bytes;
    for (int k = 0; k < nworkers; ++k) s->workers.emplace_back(worker_main, s);
    *out = s;
    return SLD_OK;
}

}  // extern "C"

namespace {

// Record the submitter's stream position and queue the request.
sld_status enqueue(sld_server s, Request r, void* stream, uint64_t* ticket) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    hipError_t e = hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r.ready, (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        if (r.ready) (void)hipEventDestroy(r.ready);
        sld_set_error(std::string("sld_server_submit: ") + hipGetErrorString(e));
        return SLD_E_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            (void)hipEventDestroy(r.ready);
            sld_set_error("sld_server_submit: server is shutting down");
            return SLD_E_INVALID;
        }
        r.ticket = s->next_ticket++;
        s->results[r.ticket] = Result{};
        s->queue.push_back(r);
        *ticket = r.ticket;
    }
    s->cv_work.notify_one();
    return SLD_OK;
}

}  // namespace

extern "C" {

sld_status sld_server_submit(sld_server s, sld_disc d, const double* b, double* p,
                             const sld_cg_params* params, void* stream, uint64_t* ticket) {
    if (!s || !d || !b || !p || !params || !ticket) {
        sld_set_error("sld_server_submit: NULL argument");
        return SLD_E_INVALID;
    }
    if (d->mesh->device != s->device) {
        sld_set_error("sld_server_submit: disc lives on another device");
        return SLD_E_INVALID;
    }
    uint64_t bytes = 0;
    (void)sld_disc_footprint(d, &bytes);
    bytes += uint64_t(d->mesh->ne) * d->nphi * 16;  // the request's b and p
    if (bytes > s->budget) {
        sld_set_error("sld_server_submit: the request alone exceeds the memory budget");
        return SLD_E_BUDGET;
    }
    Request r;
    r.disc = d;
    r.b = b;
    r.p = p;
    r.params = *params;
    r.bytes = bytes;
    return enqueue(s, r, stream, ticket);
}

sld_status sld_server_submit_imex(sld_server s, sld_state state, const sld_imex_params* params,
                                  double dt, double* v, double* p, void* stream, uint64_t* ticket) {
    if (!s || !state || !params || !v || !p || !ticket) {
        sld_set_error("sld_server_submit_imex: NULL argument");
        return SLD_E_INVALID;
    }
    sld_disc d = state->disc;
    if (d->mesh->device != s->device) {
        sld_set_error("sld_server_submit_imex: state lives on another device");
        return SLD_E_INVALID;
    }
    uint64_t bytes = 0;
    (void)sld_disc_footprint(d, &bytes);
    // + the state's workspace and the request's v and p
    bytes += sld_state_bytes(state) + 8 * (uint64_t(d->mesh->nd) * 2 * d->npsi +
                                           uint64_t(d->mesh->ne) * d->nphi);
    if (bytes > s->budget) {
        sld_set_error("sld_server_submit_imex: the request alone exceeds the memory budget");
        return SLD_E_BUDGET;
    }
    Request r;
    r.disc = d;
    r.p = p;
    r.state = state;
    r.iparams = *params;
    r.dt = dt;
    r.v = v;
    r.bytes = bytes;
    return enqueue(s, r, stream, ticket);
}

sld_status sld_server_poll(sld_server s, uint64_t ticket, int32_t wait, int32_t* done,
                           int32_t* status, sld_cg_report* report) {
    if (!s || !done) {
        sld_set_error("sld_server_poll: NULL argument");
        return SLD_E_INVALID;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) {
        sld_set_error("sld_server_poll: unknown ticket");
        return SLD_E_INVALID;
    }
    if (wait)
        s->cv_done.wait(lk, [&] { return s->results[ticket].done; });
    const Result& r = s->results[ticket];
    *done = r.done ? 1 : 0;
    if (r.done) {
        if (status) *status = r.status;
        if (report) *report = r.report;
        s->results.erase(ticket);
    }
    return SLD_OK;
}

sld_status sld_server_stats(sld_server s, int32_t* queued, int32_t* running, uint64_t* in_flight_bytes,
                            uint64_t* completed) {
    if (!s) {
        sld_set_error("sld_server_stats: NULL server");
        return SLD_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int32_t)s->queue.size();
    if (running) *running = s->running;
    if (in_flight_bytes) *in_flight_bytes = s->in_flight_bytes;
    if (completed) *completed = s->completed;
    return SLD_OK;
}

void sld_server_destroy(sld_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    delete s;
}

}  // extern "C"
