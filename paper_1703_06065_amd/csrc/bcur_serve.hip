// Continuous-batching request loop for Block CUR decompositions.
//
// A server owns `max_slots` worker slots.  Each slot is a library context
// with its own HIP stream (default priority) and its own host thread, so
// requests running in different slots overlap on the device: one request's
// latency-bound steps (the one-workgroup eigensolver, the small
// factorizations, the host round trip after sampling) run while another's
// GEMMs fill the machine.  Requests are admitted in arrival order (FIFO) as
// soon as a slot is free and the device memory they need fits the budget:
// the budget counts the workspace every slot holds; when the request at the
// head does not fit, idle slots give their workspace back first.  A request
// that can never fit is refused at submission.  Results (indices, scores,
// scalars) are kept per ticket until collected; U is written to the caller's
// device buffer.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bcur.h"

namespace {

using clk = std::chrono::steady_clock;

struct Ticket {
    uint64_t id = 0;
    // request (host arrays copied, device pointers borrowed)
    const float* A = nullptr;
    int64_t m = 0, n = 0, lda = 0;
    std::vector<int64_t> col_off, row_off, col_map, row_map;
    bcur_params params{};   // its map pointers point into col_map / row_map
    const float* omega = nullptr;
    std::vector<uint64_t> draws;
    float* U = nullptr;
    int64_t ldu = 0, u_rows_cap = 0;
    hipEvent_t ready = nullptr;   // recorded on the submitter's stream
    size_t footprint = 0;
    // result
    std::vector<int64_t> idx, idx_r;
    std::vector<double> weights, scores, ritz, row_scores;
    bcur_result res{};
    bcur_status status = BCUR_PENDING;
    clk::time_point t_submit, t_start, t_done;
};

struct Slot {
    bcur_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    size_t held = 0;   // device workspace the slot's context holds
    bool busy = false;
    std::thread th;
};

}  // namespace

struct bcur_server {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Ticket*> queue;
    std::map<uint64_t, Ticket*> tickets;
    std::vector<Slot> slots;
    uint64_t next_id = 1;
    bool stopping = false;
    // stats
    std::vector<double> latencies_ms;
    int64_t completed = 0, failed = 0;
    size_t peak_held = 0;
    int64_t peak_inflight = 0;
    clk::time_point t_first, t_last;
    bool any = false;
};

namespace {

size_t held_total(const bcur_server* s) {
    size_t t = 0;
    for (const Slot& sl : s->slots) t += sl.held;
    return t;
}

void worker(bcur_server* srv, int si) {
    Slot& me = srv->slots[si];
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        Ticket* t = nullptr;
        while (!srv->stopping) {
            if (!srv->queue.empty()) {
                Ticket* head = srv->queue.front();
                const size_t need = head->footprint;
                const size_t others = held_total(srv) - me.held;
                if (others + std::max(need, me.held) <= srv->budget) {
                    t = head;
                    srv->queue.pop_front();
                    break;
                }
                // give back idle slots' workspace (including ours) and retry
                bool freed = false;
                for (size_t j = 0; j < srv->slots.size(); ++j) {
                    Slot& o = srv->slots[j];
                    if (!o.busy && o.held > 0) {
                        (void)bcur_release_workspace(o.ctx);
                        o.held = 0;
                        freed = true;
                    }
                }
                if (freed) continue;
            }
            srv->cv_work.wait(lk);
        }
        if (!t) return;   // stopping
        me.busy = true;
        me.held = std::max(me.held, t->footprint);
        srv->peak_held = std::max(srv->peak_held, held_total(srv));
        int64_t inflight = 0;
        for (const Slot& sl : srv->slots) inflight += sl.busy;
        srv->peak_inflight = std::max(srv->peak_inflight, inflight);
        t->t_start = clk::now();
        lk.unlock();

        if (t->ready) (void)hipStreamWaitEvent(me.stream, t->ready, 0);
        t->res.idx = t->idx.data();
        t->res.weights = t->weights.data();
        t->res.scores = t->scores.data();
        t->res.ritz = t->ritz.data();
        t->res.U = t->U;
        t->res.ldu = t->ldu;
        t->res.u_rows_cap = t->u_rows_cap;
        t->res.idx_r = t->idx_r.empty() ? nullptr : t->idx_r.data();
        t->res.row_scores = t->row_scores.empty() ? nullptr : t->row_scores.data();
        const int64_t G = (int64_t)t->col_off.size() - 1;
        const int64_t Gr = t->row_off.empty() ? 0 : (int64_t)t->row_off.size() - 1;
        const bcur_status st = bcur_decompose(me.ctx, t->A, t->m, t->n, t->lda, t->col_off.data(), G,
                                              Gr ? t->row_off.data() : nullptr, Gr, &t->params, t->omega,
                                              t->draws.data(), &t->res);
        const size_t ws = bcur_workspace_bytes(me.ctx);

        lk.lock();
        me.held = ws;
        srv->peak_held = std::max(srv->peak_held, held_total(srv));
        me.busy = false;
        t->status = st;
        t->t_done = clk::now();
        if (st == BCUR_OK) {
            ++srv->completed;
            srv->latencies_ms.push_back(std::chrono::duration<double, std::milli>(t->t_done - t->t_submit).count());
        } else {
            ++srv->failed;
        }
        srv->t_last = t->t_done;
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
}

void copy_out(const Ticket* t, bcur_result* out) {
    const int64_t s = t->params.s;
    const int64_t s_r = t->idx_r.size();
    if (out->idx) memcpy(out->idx, t->idx.data(), s * sizeof(int64_t));
    if (out->weights) memcpy(out->weights, t->weights.data(), s * sizeof(double));
    if (out->scores) memcpy(out->scores, t->scores.data(), t->scores.size() * sizeof(double));
    if (out->ritz) memcpy(out->ritz, t->ritz.data(), t->ritz.size() * sizeof(double));
    if (out->idx_r && s_r) memcpy(out->idx_r, t->idx_r.data(), s_r * sizeof(int64_t));
    if (out->row_scores && !t->row_scores.empty())
        memcpy(out->row_scores, t->row_scores.data(), t->row_scores.size() * sizeof(double));
    out->c = t->res.c;
    out->r = t->res.r;
    out->frob2 = t->res.frob2;
    out->err = t->res.err;
    out->rel_err = t->res.rel_err;
    out->min_margin = t->res.min_margin;
    out->flags = t->res.flags;
    out->rr_sweeps = t->res.rr_sweeps;
    out->kappa = t->res.kappa;
    out->cond_c = t->res.cond_c;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)floor(pos), hi = (size_t)ceil(pos);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

extern "C" {

bcur_status bcur_server_create(bcur_server** out, int device, size_t hbm_budget, int32_t max_slots) {
    if (!out || max_slots < 1 || max_slots > 64 || hbm_budget == 0) return BCUR_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BCUR_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return BCUR_E_HIP;
    bcur_server* srv = new (std::nothrow) bcur_server;
    if (!srv) return BCUR_E_NOMEM;
    srv->device = device;
    srv->budget = hbm_budget;
    srv->slots.resize(max_slots);
    for (int i = 0; i < max_slots; ++i) {
        Slot& sl = srv->slots[i];
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            bcur_create(&sl.ctx, device, sl.stream, 0) != BCUR_OK) {
            for (int j = 0; j <= i; ++j) {
                if (srv->slots[j].ctx) bcur_destroy(srv->slots[j].ctx);
                if (srv->slots[j].stream) (void)hipStreamDestroy(srv->slots[j].stream);
            }
            delete srv;
            return BCUR_E_HIP;
        }
    }
    for (int i = 0; i < max_slots; ++i) srv->slots[i].th = std::thread(worker, srv, i);
    *out = srv;
    return BCUR_OK;
}

bcur_status bcur_server_destroy(bcur_server* srv) {
    if (!srv) return BCUR_E_ARG;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        // finish what is running and queued, then stop the workers
        srv->cv_done.wait(lk, [&] {
            bool busy = false;
            for (const Slot& sl : srv->slots) busy |= sl.busy;
            return srv->queue.empty() && !busy;
        });
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (Slot& sl : srv->slots)
        if (sl.th.joinable()) sl.th.join();
    for (Slot& sl : srv->slots) {
        bcur_destroy(sl.ctx);
        (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : srv->tickets) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    delete srv;
    return BCUR_OK;
}

bcur_status bcur_server_submit(bcur_server* srv, const bcur_request* rq, uint64_t* ticket) {
    if (!srv || !rq || !ticket || !rq->col_off || !rq->draws) return BCUR_E_ARG;
    const bcur_params& p = rq->params;
    if (rq->G < 1 || p.s < 1 || p.k < 1 || p.l < p.k || rq->m < 1 || rq->n < 1) return BCUR_E_ARG;
    const bool rowv = rq->row_off && p.s_r > 0;
    size_t fp = 0;
    if (bcur_footprint(rq->m, rq->n, rq->col_off, rq->G, rowv ? rq->row_off : nullptr, rowv ? rq->Gr : 0, &p,
                       rq->U ? 0 : 1, &fp) != BCUR_OK)
        return BCUR_E_ARG;
    if (fp > srv->budget) return BCUR_E_ADMIT;
    Ticket* t = new (std::nothrow) Ticket;
    if (!t) return BCUR_E_NOMEM;
    t->A = rq->A;
    t->m = rq->m;
    t->n = rq->n;
    t->lda = rq->lda;
    t->col_off.assign(rq->col_off, rq->col_off + rq->G + 1);
    if (rowv) t->row_off.assign(rq->row_off, rq->row_off + rq->Gr + 1);
    t->params = p;
    if (p.col_map) t->col_map.assign(p.col_map, p.col_map + rq->n);
    if (rowv && p.row_map) t->row_map.assign(p.row_map, p.row_map + rq->m);
    t->params.col_map = p.col_map ? t->col_map.data() : nullptr;
    t->params.row_map = rowv && p.row_map ? t->row_map.data() : nullptr;
    t->omega = rq->omega;
    t->draws.assign(rq->draws, rq->draws + p.s + (rowv ? p.s_r : 0));
    t->U = rq->U;
    t->ldu = rq->ldu;
    t->u_rows_cap = rq->u_rows_cap;
    t->footprint = fp;
    t->idx.resize(p.s);
    t->weights.resize(p.s);
    t->scores.resize(rq->G);
    t->ritz.resize(p.l);
    if (rowv) {
        t->idx_r.resize(p.s_r);
        t->row_scores.resize(rq->Gr);
    }
    if (rq->stream) {
        if (hipEventCreateWithFlags(&t->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(t->ready, (hipStream_t)rq->stream) != hipSuccess) {
            if (t->ready) (void)hipEventDestroy(t->ready);
            delete t;
            return BCUR_E_HIP;
        }
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    t->id = srv->next_id++;
    t->t_submit = clk::now();
    if (!srv->any) {
        srv->any = true;
        srv->t_first = t->t_submit;
    }
    srv->tickets[t->id] = t;
    srv->queue.push_back(t);
    *ticket = t->id;
    srv->cv_work.notify_all();
    return BCUR_OK;
}

static bcur_status collect(bcur_server* srv, std::unique_lock<std::mutex>& lk, uint64_t ticket, bcur_result* out,
                           bool wait) {
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return BCUR_E_STATE;
    Ticket* t = it->second;
    if (wait) srv->cv_done.wait(lk, [&] { return t->status != BCUR_PENDING; });
    if (t->status == BCUR_PENDING) return BCUR_PENDING;
    const bcur_status st = t->status;
    if (st == BCUR_OK && out) copy_out(t, out);
    srv->tickets.erase(it);
    lk.unlock();
    if (t->ready) (void)hipEventDestroy(t->ready);
    delete t;
    return st;
}

bcur_status bcur_server_poll(bcur_server* srv, uint64_t ticket, bcur_result* out) {
    if (!srv) return BCUR_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    return collect(srv, lk, ticket, out, false);
}

bcur_status bcur_server_wait(bcur_server* srv, uint64_t ticket, bcur_result* out) {
    if (!srv) return BCUR_E_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    return collect(srv, lk, ticket, out, true);
}

bcur_status bcur_server_stats(bcur_server* srv, bcur_stats* out) {
    if (!srv || !out) return BCUR_E_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->queued = (int64_t)srv->queue.size();
    int64_t busy = 0;
    for (const Slot& sl : srv->slots) busy += sl.busy;
    out->running = busy;
    out->p50_ms = percentile(srv->latencies_ms, 0.50);
    out->p99_ms = percentile(srv->latencies_ms, 0.99);
    out->mean_ms = 0.0;
    for (double v : srv->latencies_ms) out->mean_ms += v;
    if (!srv->latencies_ms.empty()) out->mean_ms /= (double)srv->latencies_ms.size();
    const double span = srv->any ? std::chrono::duration<double>(srv->t_last - srv->t_first).count() : 0.0;
    out->throughput = span > 0.0 ? (double)srv->completed / span : 0.0;
    out->hbm_held = held_total(srv);
    out->hbm_peak = srv->peak_held;
    out->peak_running = srv->peak_inflight;
    return BCUR_OK;
}

}  // extern "C"
