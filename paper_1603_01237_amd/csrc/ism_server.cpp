// libism serving loop: many independent ISM solves on one device.
//
// Admission is in arrival order against a device-memory budget; every admitted request
// owns a problem handle (and so its own HIP stream), which lets the small launches of
// different requests run side by side on the 256 CUs.  Work is issued in chunks of
// iterations; each chunk ends with an asynchronous copy of J, F and the status flags to
// pinned host memory and an event, which ism_server_progress polls without blocking.
// A request runs exactly the launches a lone ism_iterate would run, so its result does
// not depend on the rest of the load.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "ism_internal.h"
#include "ism_paths.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// per-request host record; the request's pointers are re-targeted to owned copies
struct Req {
    uint64_t ticket = 0;
    ism_request r{};
    std::vector<double> H0, Hc, V0, V1, psi0, target, u0, u_out;
    ism_result res{};
    ism_problem* h = nullptr;
    hipEvent_t ev = nullptr;
    int slot = -1;
    int issued = 0;          // iterations in the chunk in flight (0: the initial boundary pass)
    bool inflight = false;
    size_t est = 0;          // footprint estimate used for admission
};

constexpr int kSlotDoubles = 8;   // J, F, flags[4] (as ints), padding

bool finite_vec(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

}  // namespace

struct ism_server {
    int device = 0;
    size_t budget = 0;
    int ipr = 1;
    int max_running = 1;
    size_t in_use = 0, peak = 0;
    uint64_t next = 1, submitted = 0, completed = 0, failed = 0;
    std::deque<Req*> queue;
    std::vector<Req*> running;
    std::unordered_map<uint64_t, Req*> all;
    double* pinned = nullptr;
    std::vector<int> free_slots;
    std::vector<hipEvent_t> ev_pool;
    double busy = 0.0, busy_since = -1.0;
};

namespace {

void busy_mark(ism_server* s) {
    const double t = now_s();
    if (!s->running.empty() && s->busy_since < 0) s->busy_since = t;
    if (s->running.empty() && s->busy_since >= 0) {
        s->busy += t - s->busy_since;
        s->busy_since = -1.0;
    }
}

void release(ism_server* s, Req* r) {
    if (r->h) {
        ism_problem_destroy(r->h);     // waits for the handle's stream
        r->h = nullptr;
        s->in_use -= r->res.device_bytes;
    }
    if (r->ev) {
        s->ev_pool.push_back(r->ev);
        r->ev = nullptr;
    }
    if (r->slot >= 0) {
        s->free_slots.push_back(r->slot);
        r->slot = -1;
    }
    r->inflight = false;
    // the inputs are no longer needed once the request has left the device
    std::vector<double>().swap(r->H0);
    std::vector<double>().swap(r->Hc);
    std::vector<double>().swap(r->V0);
    std::vector<double>().swap(r->V1);
    std::vector<double>().swap(r->psi0);
    std::vector<double>().swap(r->target);
    std::vector<double>().swap(r->u0);
}

void fail(ism_server* s, Req* r, int status) {
    release(s, r);
    r->res.state = ISM_REQ_FAILED;
    r->res.status = status;
    r->res.t_done = now_s();
    s->failed += 1;
}

int finish(ism_server* s, Req* r) {
    r->u_out.resize((size_t)r->r.K * (r->r.model == ISM_REQ_GPE ? 1 : r->r.n_ctrl));
    const int st = ism_get_controls(r->h, r->u_out.data());
    if (st) return st;
    release(s, r);
    r->res.state = ISM_REQ_DONE;
    r->res.t_done = now_s();
    s->completed += 1;
    return ISM_OK;
}

// enqueue the D2H copy of J, F, flags into the request's pinned slot and its event
int mark_chunk(ism_server* s, Req* r) {
    ism_problem* p = r->h;
    double* slot = s->pinned + (size_t)r->slot * kSlotDoubles;
    if (hipMemcpyAsync(slot, p->J, sizeof(double), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(slot + 1, p->F, sizeof(double), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(slot + 2, p->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, p->stream) ||
        hipEventRecord(r->ev, p->stream))
        return ISM_E_DEVICE;
    r->inflight = true;
    return ISM_OK;
}

int issue_chunk(ism_server* s, Req* r) {
    const int n = std::min(s->ipr, r->r.max_iter - r->res.iters);
    const int st = ism::serve_chunk(r->h, n, r->r.rho, r->r.fid_stop);
    if (st) return st;
    r->issued = n;
    return mark_chunk(s, r);
}

int create_handle(ism_server* s, Req* r) {
    ism_options o;
    ism_default_options(&o);
    o.precision = r->r.precision;
    o.kind = r->r.kind;
    o.device = s->device;
    o.alloc_async = 1;      // retiring a request must not wait for the other requests' work
    const ism_request& q = r->r;
    if (q.model == ISM_REQ_GPE)
        return ism_problem_create_gpe(&r->h, q.n_grid, q.L, q.g, q.V0, q.V1, q.V2, q.psi0,
                                      q.target, q.T, q.K, q.N, &o);
    return ism_problem_create(&r->h, q.d, q.n_ctrl, q.H0, q.Hc, q.psi0, q.target, q.T, q.K, q.N,
                              &o);
}

int admit(ism_server* s, Req* r) {
    int st = create_handle(s, r);
    if (st) {
        r->h = nullptr;
        return st;
    }
    ism_info info;
    ism_problem_info(r->h, &info);
    r->res.device_bytes = std::max(r->est, info.device_bytes);
    s->in_use += r->res.device_bytes;
    s->peak = std::max(s->peak, s->in_use);
    r->res.t_admit = now_s();
    r->res.state = ISM_REQ_RUNNING;
    if ((st = ism_set_controls(r->h, r->u0.data()))) return st;
    if (s->free_slots.empty()) return ISM_E_STATE;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    if (!s->ev_pool.empty()) {
        r->ev = s->ev_pool.back();
        s->ev_pool.pop_back();
    } else if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
        r->ev = nullptr;
        return ISM_E_DEVICE;
    }
    if ((st = ism::serve_begin(r->h, r->r.fid_stop))) return st;
    r->issued = 0;
    return mark_chunk(s, r);
}

// a chunk (or the initial boundary pass) has completed: account for it, then finish the
// request or issue its next chunk
int advance(ism_server* s, Req* r) {
    const double* slot = s->pinned + (size_t)r->slot * kSlotDoubles;
    int fl[4];
    memcpy(fl, slot + 2, sizeof(fl));
    r->inflight = false;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    r->res.J = slot[0];
    r->res.F = slot[1];
    bool active;
    if (r->issued == 0) {
        active = fl[1] > 0;
    } else {
        // frozen instances stay frozen, so the chunk's boundary passes saw a run of active
        // ones followed by frozen ones; the update before the first frozen pass counts
        const int c = fl[1];
        active = c == r->issued;
        r->res.iters += active ? r->issued : c + 1;
    }
    if (!active || r->res.iters >= r->r.max_iter) return finish(s, r);
    return issue_chunk(s, r);
}

}  // namespace

extern "C" {

double ism_server_clock(void) { return now_s(); }

int ism_server_create(ism_server** out, int device, size_t hbm_budget, int iters_per_round,
                      int max_running) {
    if (!out || iters_per_round < 1 || max_running < 1 || hbm_budget == 0) return ISM_E_ARG;
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
            return ISM_E_DEVICE;
        if (hipSetDevice(device) != hipSuccess) return ISM_E_DEVICE;
        ism_server* s = new ism_server();
        s->device = device;
        s->budget = hbm_budget;
        s->ipr = iters_per_round;
        s->max_running = max_running;
        if (hipHostMalloc((void**)&s->pinned, (size_t)max_running * kSlotDoubles * sizeof(double),
                          hipHostMallocDefault) != hipSuccess) {
            delete s;
            return ISM_E_NOMEM;
        }
        for (int i = max_running - 1; i >= 0; --i) s->free_slots.push_back(i);
        *out = s;
        return ISM_OK;
    } catch (...) {
        return ISM_E_NOMEM;
    }
}

int ism_server_submit(ism_server* s, const ism_request* q, double t_arrival, uint64_t* ticket) {
    if (!s || !q || !ticket) return ISM_E_ARG;
    if (q->model != ISM_REQ_FINITE && q->model != ISM_REQ_GPE) return ISM_E_ARG;
    if (q->K < 1 || q->N < 1 || q->N > q->K || !(q->T > 0.0) || q->max_iter < 0 ||
        !std::isfinite(q->rho) || std::isnan(q->fid_stop) || !q->psi0 || !q->target || !q->u0)
        return ISM_E_ARG;
    if (q->precision != ISM_FP64 && q->precision != ISM_FP32_MIXED) return ISM_E_ARG;
    size_t est, n_state, n_ctrl;
    if (q->model == ISM_REQ_GPE) {
        if (q->n_grid < 1 || !q->V0 || !q->V1) return ISM_E_ARG;
        est = ism_problem_footprint(1, 1, q->K, q->N, 1, ISM_STATE, q->precision, q->n_grid);
        n_state = q->n_grid;
        n_ctrl = 1;
    } else {
        if (q->d < 1 || q->n_ctrl < 1 || !q->H0 || !q->Hc) return ISM_E_ARG;
        if (q->kind != ISM_STATE && q->kind != ISM_GATE) return ISM_E_ARG;
        est = ism_problem_footprint(q->d, q->n_ctrl, q->K, q->N, 1, q->kind, q->precision, 0);
        n_state = q->kind == ISM_GATE ? (size_t)q->d * q->d : (size_t)q->d;
        n_ctrl = q->n_ctrl;
    }
    if (est == 0) return ISM_E_ARG;
    if (est > s->budget) return ISM_E_BUDGET;
    if (!finite_vec(q->u0, (size_t)q->K * n_ctrl)) return ISM_E_ARG;
    try {
        Req* r = new Req();
        r->r = *q;
        r->est = est;
        if (q->model == ISM_REQ_GPE) {
            r->V0.assign(q->V0, q->V0 + q->n_grid);
            r->V1.assign(q->V1, q->V1 + q->n_grid);
            r->r.V0 = r->V0.data();
            r->r.V1 = r->V1.data();
            r->r.H0 = r->r.Hc = nullptr;
        } else {
            const size_t dd = (size_t)q->d * q->d;
            r->H0.assign(q->H0, q->H0 + 2 * dd);
            r->Hc.assign(q->Hc, q->Hc + 2 * dd * q->n_ctrl);
            r->r.H0 = r->H0.data();
            r->r.Hc = r->Hc.data();
            r->r.V0 = r->r.V1 = nullptr;
        }
        r->psi0.assign(q->psi0, q->psi0 + 2 * n_state);
        r->target.assign(q->target, q->target + 2 * n_state);
        r->u0.assign(q->u0, q->u0 + (size_t)q->K * n_ctrl);
        r->r.psi0 = r->psi0.data();
        r->r.target = r->target.data();
        r->r.u0 = r->u0.data();
        r->ticket = s->next++;
        r->res.state = ISM_REQ_QUEUED;
        r->res.status = ISM_OK;
        r->res.t_arrival = t_arrival < 0 ? now_s() : t_arrival;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
        s->submitted += 1;
        *ticket = r->ticket;
        return ISM_OK;
    } catch (...) {
        return ISM_E_NOMEM;
    }
}

int ism_server_progress(ism_server* s, int* n_queued, int* n_running) {
    if (!s) return ISM_E_ARG;
    try {
        if (hipSetDevice(s->device) != hipSuccess) return ISM_E_DEVICE;
        busy_mark(s);
        // 1. completed chunks
        std::vector<Req*> still;
        still.reserve(s->running.size());
        for (Req* r : s->running) {
            if (r->inflight) {
                const hipError_t q = hipEventQuery(r->ev);
                if (q == hipErrorNotReady) {
                    still.push_back(r);
                    continue;
                }
                if (q != hipSuccess) {
                    fail(s, r, ISM_E_DEVICE);
                    continue;
                }
            }
            const int st = advance(s, r);
            if (st) {
                fail(s, r, st);
                continue;
            }
            if (r->res.state == ISM_REQ_RUNNING) still.push_back(r);
        }
        s->running.swap(still);
        // 2. admission in arrival order while the head of the queue fits
        while (!s->queue.empty() && (int)s->running.size() < s->max_running) {
            Req* r = s->queue.front();
            if (s->in_use + r->est > s->budget) break;
            s->queue.pop_front();
            const int st = admit(s, r);
            if (st) {
                fail(s, r, st);
                continue;
            }
            s->running.push_back(r);
        }
        busy_mark(s);
        if (n_queued) *n_queued = (int)s->queue.size();
        if (n_running) *n_running = (int)s->running.size();
        return ISM_OK;
    } catch (...) {
        return ISM_E_NOMEM;
    }
}

int ism_server_poll(ism_server* s, uint64_t ticket, ism_result* res) {
    if (!s || !res) return ISM_E_ARG;
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return ISM_E_ARG;
    *res = it->second->res;
    return ISM_OK;
}

int ism_server_take(ism_server* s, uint64_t ticket, ism_result* res, double* u_out) {
    if (!s) return ISM_E_ARG;
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return ISM_E_ARG;
    Req* r = it->second;
    if (r->res.state != ISM_REQ_DONE && r->res.state != ISM_REQ_FAILED) return ISM_E_STATE;
    if (res) *res = r->res;
    if (u_out && r->res.state == ISM_REQ_DONE)
        memcpy(u_out, r->u_out.data(), r->u_out.size() * sizeof(double));
    s->all.erase(it);
    delete r;
    return ISM_OK;
}

int ism_server_stats_get(ism_server* s, ism_server_stats* st) {
    if (!s || !st) return ISM_E_ARG;
    busy_mark(s);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->queued = (int)s->queue.size();
    st->running = (int)s->running.size();
    st->bytes_in_use = s->in_use;
    st->bytes_peak = s->peak;
    st->busy_s = s->busy + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
    return ISM_OK;
}

void ism_server_destroy(ism_server* s) {
    if (!s) return;
    hipSetDevice(s->device);
    for (Req* r : s->running) release(s, r);
    for (auto& kv : s->all) delete kv.second;
    for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
    if (s->pinned) hipHostFree(s->pinned);
    delete s;
}

}  // extern "C"
