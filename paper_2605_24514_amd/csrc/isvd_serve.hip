// Serving loop over many streams: continuous batching of update requests
// into ticks, admission of streams by HBM budget, and per-request latency
// stamps.  Host-side scheduling only; every update runs through isvd_tick.
//
// Requests queue per stream in arrival order.  A scheduling step retires
// streams whose lifetime is complete, admits waiting streams in FIFO order
// while their footprint fits the budget (isvd_init), and launches one tick
// made of the oldest queued request of every admitted stream -- so requests
// that arrive while earlier ticks run on the device join the next tick, and
// up to max_inflight ticks overlap on the device.  A request whose shape no
// longer matches its stream completes at once with the error status and is
// not part of any tick.  Completion times come from an event recorded after
// each tick's last work, converted to the server's host clock through a
// reference event taken when the server was created.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "../../include/isvd.h"

namespace {

struct Pending {
    isvd_request r;
    double arrival;
    int64_t req;
};

struct Ticket {
    isvd_config cfg;
    const void* A0 = nullptr;
    int64_t lda = 0;
    int32_t dtype = 0;
    int64_t lifetime = 0;          // requests until the stream is released (0 = never)
    uint64_t bytes = 0;            // device footprint
    int state = 0;                 // 0 waiting, 1 admitted, 2 retired
    isvd_id id = -1;
    double admit_s = -1.0;
    int64_t completed = 0;
    std::deque<Pending> queue;
};

// A tick's work ends on the rotation lane (U rotations left pending by a
// pipelined tick) or on the server's stream (every other form, deferred U
// included): its completion is the later of two events, one on each.
struct InFlight {
    hipEvent_t done = nullptr;    // on the rotation lane
    hipEvent_t done2 = nullptr;   // on the server's stream
    double launch_s = 0.0;
    std::vector<Pending> reqs;
    std::vector<int64_t> tickets;
};

}  // namespace

struct isvd_server {
    isvd_engine* eng = nullptr;
    hipStream_t st = nullptr;
    isvd_server_config cfg{};
    std::vector<Ticket> tickets;
    std::deque<int64_t> waiting;
    uint64_t used = 0;
    std::deque<InFlight> inflight;
    std::vector<hipEvent_t> free_events;
    std::vector<isvd_completion> done;
    hipEvent_t ref = nullptr;
    double ref_s = 0.0;
    std::chrono::steady_clock::time_point t0;
    int64_t next_req = 0;
    size_t rr = 0;
    int64_t ticks = 0, tick_requests = 0;
    double t_admit = 0.0, t_tick = 0.0, t_wait = 0.0, t_release = 0.0;
    std::string err;
};

namespace {

double now_s(const isvd_server* s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

isvd_status sfail(isvd_server* s, isvd_status st, const char* msg) {
    if (s) s->err = msg;
    return st;
}

// A stream that has completed its lifetime of requests (successful or not)
// and has nothing queued releases its HBM.
isvd_status retire_if_done(isvd_server* s, Ticket& t) {
    if (t.lifetime > 0 && t.completed >= t.lifetime && t.queue.empty() && t.state == 1) {
        const double r0 = now_s(s);
        const isvd_status rc = isvd_release(s->eng, t.id);
        s->t_release += now_s(s) - r0;
        if (rc != ISVD_OK) return ISVD_E_DEVICE;
        t.state = 2;
        s->used -= t.bytes;
    }
    return ISVD_OK;
}

void complete(isvd_server* s, const Pending& p, int64_t ticket, int32_t status, double launch_s, double done_s) {
    isvd_completion c{};
    c.req = p.req;
    c.ticket = ticket;
    c.kind = p.r.kind;
    c.status = status;
    c.arrival_s = p.arrival;
    c.admit_s = s->tickets[ticket].admit_s;
    c.launch_s = launch_s;
    c.done_s = done_s;
    s->done.push_back(c);
}

// Stamp the oldest in-flight tick (waiting for it when `block`).
isvd_status finish_oldest(isvd_server* s, bool block, bool* finished) {
    *finished = false;
    if (s->inflight.empty()) return ISVD_OK;
    InFlight& f = s->inflight.front();
    float ms = 0.f;
    for (hipEvent_t ev : {f.done, f.done2}) {
        const double w0 = block ? now_s(s) : 0.0;
        hipError_t q = block ? hipEventSynchronize(ev) : hipEventQuery(ev);
        if (block) s->t_wait += now_s(s) - w0;
        if (q == hipErrorNotReady) return ISVD_OK;
        if (q != hipSuccess) return sfail(s, ISVD_E_DEVICE, "tick completion event failed");
        float e_ms = 0.f;
        if (hipEventElapsedTime(&e_ms, s->ref, ev) != hipSuccess) return sfail(s, ISVD_E_DEVICE, "event timing failed");
        ms = std::max(ms, e_ms);
    }
    const double done_s = s->ref_s + 1e-3 * ms;
    for (size_t q2 = 0; q2 < f.reqs.size(); ++q2) {
        complete(s, f.reqs[q2], f.tickets[q2], ISVD_OK, f.launch_s, done_s);
        Ticket& t = s->tickets[f.tickets[q2]];
        t.completed += 1;
        if (retire_if_done(s, t) != ISVD_OK) return sfail(s, ISVD_E_DEVICE, "release failed");
    }
    s->free_events.push_back(f.done);
    s->free_events.push_back(f.done2);
    s->inflight.pop_front();
    *finished = true;
    return ISVD_OK;
}

bool shape_ok(isvd_server* s, const Ticket& t, const isvd_request& r) {
    int64_t m = 0, n = 0;
    int32_t k = 0;
    if (isvd_shape(s->eng, t.id, &m, &n, &k) != ISVD_OK) return false;
    if (r.kind == ISVD_ROW) return r.len == n && m < t.cfg.m_cap;
    if (r.kind == ISVD_COL) return r.len == m && n < t.cfg.n_cap;
    if (r.kind == ISVD_ENTRY) return r.i >= 0 && r.i < m && r.j >= 0 && r.j < n;
    return false;
}

}  // namespace

extern "C" {

isvd_status isvd_server_create(isvd_engine* eng, const isvd_server_config* cfg, void* hip_stream,
                               isvd_server** out) {
    if (!eng || !cfg || !out) return ISVD_E_INVAL;
    if (cfg->max_inflight < 1 || cfg->max_batch < 0) return ISVD_E_INVAL;
    isvd_server* s = new isvd_server();
    s->eng = eng;
    s->st = (hipStream_t)hip_stream;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    if (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, s->st) != hipSuccess ||
        hipEventSynchronize(s->ref) != hipSuccess) {
        delete s;
        return ISVD_E_DEVICE;
    }
    s->ref_s = now_s(s);
    *out = s;
    return ISVD_OK;
}

isvd_status isvd_server_destroy(isvd_server* s) {
    if (!s) return ISVD_OK;
    for (InFlight& f : s->inflight) {
        for (hipEvent_t ev : {f.done, f.done2}) {
            (void)hipEventSynchronize(ev);
            (void)hipEventDestroy(ev);
        }
    }
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    if (s->ref) (void)hipEventDestroy(s->ref);
    delete s;
    return ISVD_OK;
}

double isvd_server_clock(isvd_server* s) { return s ? now_s(s) : 0.0; }

const char* isvd_server_error(isvd_server* s) { return s ? s->err.c_str() : ""; }

isvd_status isvd_server_add_stream(isvd_server* s, const isvd_config* cfg, const void* A0, int64_t lda,
                                   int32_t dtype, int64_t lifetime, int64_t* ticket) {
    if (!s || !cfg || !A0 || !ticket || lifetime < 0) return sfail(s, ISVD_E_INVAL, "bad stream arguments");
    const uint64_t bytes = isvd_stream_bytes(cfg);
    if (bytes == 0) return sfail(s, ISVD_E_INVAL, "invalid stream configuration");
    if (s->cfg.hbm_budget && bytes > s->cfg.hbm_budget) return sfail(s, ISVD_E_BUDGET, "stream exceeds the budget");
    Ticket t;
    t.cfg = *cfg;
    t.A0 = A0;
    t.lda = lda;
    t.dtype = dtype;
    t.lifetime = lifetime;
    t.bytes = bytes;
    s->tickets.push_back(t);
    *ticket = (int64_t)s->tickets.size() - 1;
    s->waiting.push_back(*ticket);
    return ISVD_OK;
}

isvd_status isvd_server_submit(isvd_server* s, int64_t ticket, const isvd_request* r, double arrival_s,
                               int64_t* req_id) {
    if (!s || !r || !req_id) return sfail(s, ISVD_E_INVAL, "null argument");
    if (ticket < 0 || ticket >= (int64_t)s->tickets.size() || s->tickets[ticket].state == 2)
        return sfail(s, ISVD_E_STATE, "unknown or retired ticket");
    if (r->kind != ISVD_ROW && r->kind != ISVD_COL && r->kind != ISVD_ENTRY)
        return sfail(s, ISVD_E_INVAL, "bad request kind");
    Pending p;
    p.r = *r;
    p.arrival = arrival_s;
    p.req = s->next_req++;
    s->tickets[ticket].queue.push_back(p);
    *req_id = p.req;
    return ISVD_OK;
}

isvd_status isvd_server_submit_many(isvd_server* s, int32_t count, const int64_t* tickets, const isvd_request* reqs,
                                    const double* arrival_s, int64_t* req_ids) {
    if (!s || count < 0 || (count > 0 && (!tickets || !reqs || !arrival_s))) return sfail(s, ISVD_E_INVAL, "null argument");
    for (int32_t q = 0; q < count; ++q) {
        int64_t id = -1;
        isvd_status rc = isvd_server_submit(s, tickets[q], &reqs[q], arrival_s[q], &id);
        if (rc != ISVD_OK) return rc;
        if (req_ids) req_ids[q] = id;
    }
    return ISVD_OK;
}

isvd_status isvd_server_step(isvd_server* s, int32_t* launched) {
    if (!s) return ISVD_E_INVAL;
    if (launched) *launched = 0;
    bool fin = true;
    while (fin) {
        isvd_status rc = finish_oldest(s, false, &fin);
        if (rc != ISVD_OK) return rc;
    }
    // admission: FIFO while the footprint fits, the admitted streams created
    // in one call (their initial SVDs batched)
    {
        std::vector<int64_t> adm;
        uint64_t used = s->used;
        for (int64_t ti : s->waiting) {
            const Ticket& t = s->tickets[ti];
            if (s->cfg.hbm_budget && used + t.bytes > s->cfg.hbm_budget) break;
            used += t.bytes;
            adm.push_back(ti);
        }
        if (!adm.empty()) {
            const size_t na = adm.size();
            std::vector<isvd_config> cfgs(na);
            std::vector<const void*> a0(na);
            std::vector<int64_t> lda(na);
            std::vector<int32_t> dt(na);
            std::vector<isvd_id> ids(na, -1);
            for (size_t q = 0; q < na; ++q) {
                const Ticket& t = s->tickets[adm[q]];
                cfgs[q] = t.cfg;
                a0[q] = t.A0;
                lda[q] = t.lda;
                dt[q] = t.dtype;
            }
            int32_t made = 0;
            const double a0s = now_s(s);
            isvd_status rc = isvd_init_batch(s->eng, (int32_t)na, cfgs.data(), a0.data(), lda.data(), dt.data(),
                                             s->st, ids.data(), &made);
            const double a1s = now_s(s);
            s->t_admit += a1s - a0s;
            for (int32_t q = 0; q < made; ++q) {
                Ticket& t = s->tickets[adm[q]];
                t.id = ids[q];
                t.state = 1;
                t.admit_s = a1s;
                s->used += t.bytes;
                s->waiting.pop_front();
            }
            if (rc != ISVD_OK) return sfail(s, rc, "admission failed");
        }
    }
    // at most max_inflight ticks on the device
    while ((int)s->inflight.size() >= s->cfg.max_inflight) {
        isvd_status rc = finish_oldest(s, true, &fin);
        if (rc != ISVD_OK) return rc;
    }
    // one tick: the oldest queued request of each admitted stream
    std::vector<isvd_request> batch;
    InFlight f;
    const size_t nt = s->tickets.size();
    const double tnow = now_s(s);
    for (size_t q = 0; q < nt; ++q) {
        const size_t ti = (s->rr + q) % nt;
        Ticket& t = s->tickets[ti];
        if (t.state != 1 || t.queue.empty()) continue;
        // a request stamped with a later arrival time has not arrived yet
        if (t.queue.front().arrival > tnow) continue;
        if (s->cfg.max_batch && (int)batch.size() >= s->cfg.max_batch) break;
        // a stream whose refresh still runs waits for a later tick, so the
        // refresh overlaps the other streams' updates
        int32_t busy = 0;
        isvd_status brc = isvd_stream_busy(s->eng, t.id, &busy);
        if (brc != ISVD_OK) return sfail(s, brc, "refresh of a stream failed");
        if (busy) continue;
        Pending p = t.queue.front();
        t.queue.pop_front();
        if (!shape_ok(s, t, p.r)) {
            complete(s, p, (int64_t)ti, ISVD_E_SHAPE, tnow, tnow);
            t.completed += 1;
            if (retire_if_done(s, t) != ISVD_OK) return sfail(s, ISVD_E_DEVICE, "release failed");
            continue;
        }
        p.r.id = t.id;
        batch.push_back(p.r);
        f.reqs.push_back(p);
        f.tickets.push_back((int64_t)ti);
    }
    if (nt) s->rr = (s->rr + 1) % nt;
    if (batch.empty()) return ISVD_OK;
    const double k0 = now_s(s);
    isvd_status rc = isvd_tick(s->eng, (int32_t)batch.size(), batch.data(), s->st);
    s->t_tick += now_s(s) - k0;
    s->ticks += 1;
    s->tick_requests += (int64_t)batch.size();
    if (rc != ISVD_OK) {
        for (size_t q = 0; q < f.reqs.size(); ++q) {
            complete(s, f.reqs[q], f.tickets[q], rc, tnow, tnow);
            Ticket& t = s->tickets[f.tickets[q]];
            t.completed += 1;
            (void)retire_if_done(s, t);
        }
        return sfail(s, rc, "tick failed");
    }
    while (s->free_events.size() < 2) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return sfail(s, ISVD_E_DEVICE, "event creation failed");
        s->free_events.push_back(ev);
    }
    f.done = s->free_events.back();
    s->free_events.pop_back();
    f.done2 = s->free_events.back();
    s->free_events.pop_back();
    void* lane = nullptr;
    if (isvd_rotation_stream(s->eng, &lane) != ISVD_OK ||
        hipEventRecord(f.done, (hipStream_t)lane) != hipSuccess || hipEventRecord(f.done2, s->st) != hipSuccess)
        return sfail(s, ISVD_E_DEVICE, "tick event failed");
    f.launch_s = tnow;
    if (launched) *launched = (int32_t)batch.size();
    s->inflight.push_back(std::move(f));
    return ISVD_OK;
}

isvd_status isvd_server_drain(isvd_server* s) {
    if (!s) return ISVD_E_INVAL;
    bool fin = true;
    while (!s->inflight.empty()) {
        isvd_status rc = finish_oldest(s, true, &fin);
        if (rc != ISVD_OK) return rc;
    }
    return ISVD_OK;
}

isvd_status isvd_server_poll(isvd_server* s, isvd_completion* out, int32_t cap, int32_t* count) {
    if (!s || !count || (cap > 0 && !out)) return ISVD_E_INVAL;
    const int32_t n = (int32_t)std::min<size_t>((size_t)std::max(cap, 0), s->done.size());
    for (int32_t q = 0; q < n; ++q) out[q] = s->done[q];
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *count = n;
    return ISVD_OK;
}

isvd_status isvd_server_stats(isvd_server* s, isvd_server_stats_t* out) {
    if (!s || !out) return ISVD_E_INVAL;
    isvd_server_stats_t st{};
    for (const Ticket& t : s->tickets) {
        st.waiting += t.state == 0;
        st.admitted += t.state == 1;
        st.retired += t.state == 2;
        st.queued += (int64_t)t.queue.size();
    }
    st.inflight_ticks = (int32_t)s->inflight.size();
    st.hbm_used = s->used;
    st.ticks = s->ticks;
    st.tick_requests = s->tick_requests;
    st.host_admit_s = s->t_admit;
    st.host_tick_s = s->t_tick;
    st.host_wait_s = s->t_wait;
    st.host_release_s = s->t_release;
    *out = st;
    return ISVD_OK;
}

isvd_status isvd_server_stream(isvd_server* s, int64_t ticket, isvd_id* id, int32_t* state) {
    if (!s || ticket < 0 || ticket >= (int64_t)s->tickets.size()) return ISVD_E_INVAL;
    if (id) *id = s->tickets[ticket].id;
    if (state) *state = s->tickets[ticket].state;
    return ISVD_OK;
}

}  // extern "C"
