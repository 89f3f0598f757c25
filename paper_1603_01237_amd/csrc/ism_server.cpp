// libism serving loop: many independent ISM solves on one device.
//
// Admission is in arrival order against a device-memory budget.  The head of the queue is
// admitted together with every queued request that differs from it only in the diagonal of
// H0 (same model, shape, generators, initial and target states, time grid, step and stopping
// rule): they become the instances of one batched handle, so one set of launches serves them
// all (the kernels work on each instance independently, so every instance's arithmetic is
// that of its lone run).  Each group owns a handle and so its own HIP stream, which lets the
// launches of different groups run side by side on the 256 CUs.  Work is issued in chunks of
// iterations; each chunk ends with an asynchronous copy of the per-instance J, F, active
// flags and update counts to pinned host memory and an event, which ism_server_progress polls
// without blocking.  An instance freezes on its own (F >= fid_stop, or max_iter updates); its
// request is then finished (its controls copied out) while the rest of the group goes on.
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

struct Group;

// per-request host record; the request's pointers are re-targeted to owned copies
struct Req {
    uint64_t ticket = 0;
    ism_request r{};
    std::vector<double> H0, Hc, V0, V1, psi0, target, u0, u_out;
    ism_result res{};
    Group* g = nullptr;
    int b = -1;              // instance index in its group
    size_t est = 0;          // footprint estimate of a lone run
};

constexpr int kMaxBatch = 256;     // instances per merged group

// one admitted handle and the requests it serves
struct Group {
    ism_problem* h = nullptr;
    std::vector<Req*> mem;   // instance b = mem[b]
    std::vector<char> live;  // request b still running
    int n_live = 0;
    hipEvent_t ev = nullptr;
    int slot = -1;           // readback slot (pinned host memory and device counters)
    int* count = nullptr;    // device: updates per instance (the slot's part of the server's array)
    int issued = 0;          // iterations in the chunk in flight (0: the initial boundary pass)
    int iters = 0;           // iterations issued so far
    bool inflight = false;
    size_t bytes = 0;        // charged against the budget
};

// pinned readback slot of a group: J[B], F[B] (doubles), then flags[4], active[B], count[B]
constexpr size_t kSlotBytes = (size_t)kMaxBatch * 16 + 16 + (size_t)kMaxBatch * 8;

bool finite_vec(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

size_t state_len(const ism_request& q) {
    if (q.model == ISM_REQ_GPE) return (size_t)q.n_grid;
    return q.kind == ISM_GATE ? (size_t)q.d * q.d : (size_t)q.d;
}

// may b join a group headed by a?  Both finite state problems (the batched sparse path), equal
// in everything but the diagonal of H0; or both condensate problems (one workgroup per
// instance in every kernel of that path), equal in everything but the initial controls
bool mergeable(const Req* a, const Req* b) {
    const ism_request &x = a->r, &y = b->r;
    if (x.model == ISM_REQ_GPE && y.model == ISM_REQ_GPE) {
        if (x.precision != y.precision || x.n_grid != y.n_grid || x.L != y.L || x.g != y.g ||
            x.V2 != y.V2 || x.K != y.K || x.N != y.N || x.T != y.T || x.rho != y.rho ||
            x.fid_stop != y.fid_stop || x.max_iter != y.max_iter)
            return false;
        return a->V0 == b->V0 && a->V1 == b->V1 && a->psi0 == b->psi0 && a->target == b->target;
    }
    if (x.model != ISM_REQ_FINITE || y.model != ISM_REQ_FINITE) return false;
    if (x.kind != ISM_STATE || y.kind != ISM_STATE) return false;
    if (x.precision != y.precision || x.d != y.d || x.n_ctrl != y.n_ctrl || x.K != y.K ||
        x.N != y.N || x.T != y.T || x.rho != y.rho || x.fid_stop != y.fid_stop ||
        x.max_iter != y.max_iter)
        return false;
    if (a->Hc != b->Hc || a->psi0 != b->psi0 || a->target != b->target) return false;
    const int d = x.d;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            if (r == c) continue;
            const size_t k = 2 * ((size_t)r * d + c);
            if (a->H0[k] != b->H0[k] || a->H0[k + 1] != b->H0[k + 1]) return false;
        }
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
    std::vector<Group*> running;
    int n_req_running = 0;
    std::unordered_map<uint64_t, Req*> all;
    unsigned char* pinned = nullptr;
    int* counts = nullptr;   // device: kMaxBatch update counters per slot
    std::vector<int> free_slots;
    std::vector<hipEvent_t> ev_pool;
    double busy = 0.0, busy_since = -1.0;
    uint64_t groups = 0, merged = 0;
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

void drop_inputs(Req* r) {
    std::vector<double>().swap(r->H0);
    std::vector<double>().swap(r->Hc);
    std::vector<double>().swap(r->V0);
    std::vector<double>().swap(r->V1);
    std::vector<double>().swap(r->psi0);
    std::vector<double>().swap(r->target);
    std::vector<double>().swap(r->u0);
}

void release(ism_server* s, Group* g) {
    if (g->h) {
        ism_problem_destroy(g->h);     // waits for the handle's stream
        g->h = nullptr;
        s->in_use -= g->bytes;
    }
    g->count = nullptr;
    if (g->ev) {
        s->ev_pool.push_back(g->ev);
        g->ev = nullptr;
    }
    if (g->slot >= 0) {
        s->free_slots.push_back(g->slot);
        g->slot = -1;
    }
    for (Req* r : g->mem) {
        r->g = nullptr;
        drop_inputs(r);
    }
    delete g;
}

void fail_req(ism_server* s, Req* r, int status) {
    r->res.state = ISM_REQ_FAILED;
    r->res.status = status;
    r->res.t_done = now_s();
    s->failed += 1;
    s->n_req_running -= 1;
}

// every live member of the group fails (a device error or a non-finite value in the batch)
void fail_group(ism_server* s, Group* g, int status) {
    for (size_t b = 0; b < g->mem.size(); ++b)
        if (g->live[b]) {
            g->live[b] = 0;
            fail_req(s, g->mem[b], status);
        }
    g->n_live = 0;
}

unsigned char* slot_of(ism_server* s, const Group* g) {
    return s->pinned + (size_t)g->slot * kSlotBytes;
}

// enqueue the D2H copies of J, F, flags, active flags and update counts into the group's
// pinned slot, and its event
int mark_chunk(ism_server* s, Group* g) {
    ism_problem* p = g->h;
    const int B = p->B;
    unsigned char* sl = slot_of(s, g);
    double* J = reinterpret_cast<double*>(sl);
    double* F = J + kMaxBatch;
    int* fl = reinterpret_cast<int*>(F + kMaxBatch);
    int* act = fl + 4;
    int* cnt = act + kMaxBatch;
    if (hipMemcpyAsync(J, p->J, B * sizeof(double), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(F, p->F, B * sizeof(double), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(fl, p->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(act, p->active, B * sizeof(int), hipMemcpyDeviceToHost, p->stream) ||
        hipMemcpyAsync(cnt, g->count, B * sizeof(int), hipMemcpyDeviceToHost, p->stream) ||
        hipEventRecord(g->ev, p->stream))
        return ISM_E_DEVICE;
    g->inflight = true;
    return ISM_OK;
}

int issue_chunk(ism_server* s, Group* g) {
    const int max_iter = g->mem[0]->r.max_iter;
    const int n = std::min(s->ipr, max_iter - g->iters);
    const int st = ism::serve_chunk(g->h, n, g->mem[0]->r.rho, g->mem[0]->r.fid_stop, g->count);
    if (st) return st;
    g->issued = n;
    g->iters += n;
    return mark_chunk(s, g);
}

int create_handle(Group* g, int device) {
    const ism_request& q = g->mem[0]->r;
    const int B = (int)g->mem.size();
    ism_options o;
    ism_default_options(&o);
    o.precision = q.precision;
    o.kind = q.kind;
    o.device = device;
    o.batch = B;
    o.alloc_async = 1;      // retiring a group must not wait for the other groups' work
    if (q.model == ISM_REQ_GPE)
        return ism_problem_create_gpe(&g->h, q.n_grid, q.L, q.g, q.V0, q.V1, q.V2, q.psi0,
                                      q.target, q.T, q.K, q.N, &o);
    if (B == 1)
        return ism_problem_create(&g->h, q.d, q.n_ctrl, q.H0, q.Hc, q.psi0, q.target, q.T, q.K,
                                  q.N, &o);
    const size_t dd2 = 2 * (size_t)q.d * q.d;
    std::vector<double> H0(dd2 * B);
    for (int b = 0; b < B; ++b) std::copy(g->mem[b]->H0.begin(), g->mem[b]->H0.end(), H0.begin() + dd2 * b);
    o.h0_batched = 1;
    return ism_problem_create(&g->h, q.d, q.n_ctrl, H0.data(), q.Hc, q.psi0, q.target, q.T, q.K,
                              q.N, &o);
}

int admit(ism_server* s, Group* g) {
    int st = create_handle(g, s->device);
    if (st) {
        g->h = nullptr;
        return st;
    }
    ism_problem* p = g->h;
    ism_info info;
    ism_problem_info(p, &info);
    size_t est = 0;
    for (Req* r : g->mem) est += r->est;
    g->bytes = std::max(est, info.device_bytes);
    s->in_use += g->bytes;
    s->peak = std::max(s->peak, s->in_use);
    const double t = now_s();
    const ism_request& q = g->mem[0]->r;
    const size_t KC = (size_t)q.K * (q.model == ISM_REQ_GPE ? 1 : q.n_ctrl);
    std::vector<double> u((size_t)g->mem.size() * KC);
    for (size_t b = 0; b < g->mem.size(); ++b) {
        Req* r = g->mem[b];
        r->res.t_admit = t;
        r->res.state = ISM_REQ_RUNNING;
        r->g = g;
        r->b = (int)b;
        std::copy(r->u0.begin(), r->u0.end(), u.begin() + KC * b);
    }
    if ((st = ism_set_controls(p, u.data()))) return st;
    if (s->free_slots.empty()) return ISM_E_STATE;
    g->slot = s->free_slots.back();
    s->free_slots.pop_back();
    if (!s->ev_pool.empty()) {
        g->ev = s->ev_pool.back();
        s->ev_pool.pop_back();
    } else if (hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess) {
        g->ev = nullptr;
        return ISM_E_DEVICE;
    }
    g->count = s->counts + (size_t)g->slot * kMaxBatch;
    if (ism::launch_fill_i32(g->count, 0, (int)g->mem.size(), p->stream) != hipSuccess)
        return ISM_E_DEVICE;
    if ((st = ism::serve_begin(p, q.fid_stop))) return st;
    g->issued = 0;
    return mark_chunk(s, g);
}

// the request of instance b is done: its controls (frozen from here on) are copied out
int finish_member(ism_server* s, Group* g, int b) {
    Req* r = g->mem[b];
    ism_problem* p = g->h;
    const size_t KC = (size_t)r->r.K * (r->r.model == ISM_REQ_GPE ? 1 : r->r.n_ctrl);
    r->u_out.resize(KC);
    if (hipMemcpyAsync(r->u_out.data(), p->u + KC * b, KC * sizeof(double),
                       hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return ISM_E_DEVICE;
    g->live[b] = 0;
    g->n_live -= 1;
    r->res.state = ISM_REQ_DONE;
    r->res.t_done = now_s();
    s->completed += 1;
    s->n_req_running -= 1;
    return ISM_OK;
}

// a chunk (or the initial boundary pass) has completed: account for it per instance, finish
// the requests whose instance froze or ran out of iterations, issue the next chunk
int advance(ism_server* s, Group* g) {
    const unsigned char* sl = slot_of(s, g);
    const double* J = reinterpret_cast<const double*>(sl);
    const double* F = J + kMaxBatch;
    const int* fl = reinterpret_cast<const int*>(F + kMaxBatch);
    const int* act = fl + 4;
    const int* cnt = act + kMaxBatch;
    g->inflight = false;
    if (fl[0] & 2) return ISM_E_UNSUPPORTED;
    if (fl[0]) return ISM_E_NUMERIC;
    const int max_iter = g->mem[0]->r.max_iter;
    int st;
    for (size_t b = 0; b < g->mem.size(); ++b) {
        if (!g->live[b]) continue;
        Req* r = g->mem[b];
        r->res.J = J[b];
        r->res.F = F[b];
        r->res.iters = cnt[b];
        if (!act[b] || g->iters >= max_iter)
            if ((st = finish_member(s, g, (int)b))) return st;
    }
    if (g->n_live == 0) return ISM_OK;
    return issue_chunk(s, g);
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
        if (hipHostMalloc((void**)&s->pinned, (size_t)max_running * kSlotBytes,
                          hipHostMallocDefault) != hipSuccess) {
            delete s;
            return ISM_E_NOMEM;
        }
        if (hipMalloc((void**)&s->counts, (size_t)max_running * kMaxBatch * sizeof(int)) !=
            hipSuccess) {
            hipHostFree(s->pinned);
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

// the admission candidate headed by the queue's front: it and the queued requests that may
// share its handle, in arrival order, as many as fit the budget (at least the head, or none)
static std::vector<Req*> admission_group(ism_server* s) {
    std::vector<Req*> g;
    Req* head = s->queue.front();
    g.push_back(head);
    for (size_t i = 1; i < s->queue.size() && (int)g.size() < kMaxBatch; ++i)
        if (mergeable(head, s->queue[i])) g.push_back(s->queue[i]);
    while (!g.empty()) {
        const ism_request& q = head->r;
        const bool gpe = q.model == ISM_REQ_GPE;
        const size_t est = g.size() == 1
                               ? head->est
                               : ism_problem_footprint(gpe ? 1 : q.d, gpe ? 1 : q.n_ctrl, q.K, q.N,
                                                       (int)g.size(), gpe ? ISM_STATE : q.kind,
                                                       q.precision, gpe ? q.n_grid : 0);
        if (est != 0 && s->in_use + est <= s->budget) break;
        g.pop_back();
    }
    return g;
}

int ism_server_progress(ism_server* s, int* n_queued, int* n_running) {
    if (!s) return ISM_E_ARG;
    try {
        if (hipSetDevice(s->device) != hipSuccess) return ISM_E_DEVICE;
        busy_mark(s);
        // 1. completed chunks
        std::vector<Group*> still;
        still.reserve(s->running.size());
        for (Group* g : s->running) {
            if (g->inflight) {
                const hipError_t q = hipEventQuery(g->ev);
                if (q == hipErrorNotReady) {
                    still.push_back(g);
                    continue;
                }
                if (q != hipSuccess) {
                    fail_group(s, g, ISM_E_DEVICE);
                    release(s, g);
                    continue;
                }
            }
            const int st = advance(s, g);
            if (st) fail_group(s, g, st);
            if (g->n_live > 0) still.push_back(g);
            else release(s, g);
        }
        s->running.swap(still);
        // 2. admission in arrival order while the head of the queue fits, with the queued
        //    requests that can share its handle
        while (!s->queue.empty() && (int)s->running.size() < s->max_running) {
            std::vector<Req*> mem = admission_group(s);
            if (mem.empty()) break;
            std::deque<Req*> rest;
            for (Req* r : s->queue)
                if (std::find(mem.begin(), mem.end(), r) == mem.end()) rest.push_back(r);
            s->queue.swap(rest);
            Group* g = new Group();
            g->mem = mem;
            g->live.assign(mem.size(), 1);
            g->n_live = (int)mem.size();
            s->n_req_running += (int)mem.size();
            s->groups += 1;
            s->merged += mem.size() - 1;
            const int st = admit(s, g);
            if (st) {
                fail_group(s, g, st);
                release(s, g);
                continue;
            }
            s->running.push_back(g);
        }
        busy_mark(s);
        if (n_queued) *n_queued = (int)s->queue.size();
        if (n_running) *n_running = s->n_req_running;
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
    st->running = s->n_req_running;
    st->groups = s->groups;
    st->merged = s->merged;
    st->bytes_in_use = s->in_use;
    st->bytes_peak = s->peak;
    st->busy_s = s->busy + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
    return ISM_OK;
}

void ism_server_destroy(ism_server* s) {
    if (!s) return;
    hipSetDevice(s->device);
    for (Group* g : s->running) release(s, g);
    for (auto& kv : s->all) delete kv.second;
    for (hipEvent_t e : s->ev_pool) hipEventDestroy(e);
    if (s->pinned) hipHostFree(s->pinned);
    if (s->counts) hipFree(s->counts);
    delete s;
}

}  // extern "C"
