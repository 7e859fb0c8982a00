// Request loop with continuous batching, built on the library's C ABI.
//
// One worker thread owns the device work of the running sessions.  Each
// round it admits queued requests in arrival order while the summed
// footprint of the admitted sessions stays within the budget, advances every
// running session by the same number of time steps (one batch per storage
// precision), and then lets sessions that reached an event take it: an
// optimisation iteration's exchange step (Sec. 2.2), or completion (outlet
// statistics of Sec. 4.2, state digest, release of the device memory).
// Admitted sessions are created by a second thread on a stream of its own
// (the host-side map generation and uploads overlap the rounds) and join the
// rounds once created, their handles moved to the worker's stream.
// Submitting threads only touch the queues; every queue is under one mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

double now_seconds() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Session {
    uint64_t id = 0;
    lbm_request req{};
    size_t bytes = 0;
    lbm_handle *h = nullptr;
    int64_t to_go = 0;   // steps left before the next event
    int64_t steps = 0;   // steps taken
    int32_t iter = 0;    // exchange steps taken
    int status = LBM_OK;
    double t_submit = 0, t_admit = 0;
};

// The batch of one precision and the handles it was built for.
struct Group {
    lbm_batch *b = nullptr;
    std::vector<lbm_handle *> members;
};

bool valid_request(const lbm_request *r) {
    if (!r) return false;
    if (r->kind != LBM_REQ_SOLVE && r->kind != LBM_REQ_OPTIMIZE) return false;
    if (r->iterations < 0 || r->solve_steps < 0 || r->steps_per_iteration < 0) return false;
    if (r->kind == LBM_REQ_OPTIMIZE) {
        const lbm_shape_params &p = r->shape;
        if (!(p.frac >= 0.0 && p.frac <= 1.0)) return false;
        if (p.band_x < 1 || p.band_y < 1) return false;
        if (2 * p.band_x >= r->geom.nx || 2 * p.band_y >= r->geom.ny) return false;
    }
    return lbm_footprint_bytes(&r->geom) > 0;
}

}  // namespace

struct lbm_server {
    lbm_server_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Session> queue;          // submitted, not admitted
    std::deque<Session> to_create;      // admitted, handle not made yet
    std::deque<Session> created;        // handle made (or failed), not yet running
    std::condition_variable cv_create;
    std::deque<lbm_result> results;     // completed, not polled
    uint64_t next_id = 1;
    int64_t pending = 0;                // submitted and not completed
    bool stop = false;
    lbm_server_stats st{};

    // worker-owned
    std::vector<Session> active;
    std::map<int, Group> groups;
    std::map<int, std::pair<int32_t, int32_t>> tuned;  // precision -> (variant, order)
    size_t used = 0;        // footprint of the admitted sessions
    int64_t creating = 0;   // admitted sessions not yet running
    std::thread worker;
    // creation thread
    std::thread creator;
    hipStream_t create_stream = nullptr;

    void complete(Session &s) {
        lbm_result r{};
        r.id = s.id;
        r.status = s.status;
        r.iterations_done = s.iter;
        r.steps = s.steps;
        r.cells = (int64_t)s.req.geom.nx * s.req.geom.ny;
        r.t_submit = s.t_submit;
        r.t_admit = s.t_admit;
        if (s.h && s.status == LBM_OK) {
            std::vector<double> flow(4096);
            int rc = lbm_outlet_stats(s.h, flow.data(), (int32_t)flow.size(), &r.stats);
            if (rc == LBM_OK) rc = lbm_state_digest(s.h, &r.digest);
            if (rc != LBM_OK) r.status = rc;
        }
        if (s.h) {
            lbm_destroy(s.h);
            s.h = nullptr;
            used -= s.bytes;
        }
        r.t_done = now_seconds();
        std::lock_guard<std::mutex> g(mu);
        results.push_back(r);
        --pending;
        ++st.completed;
        --st.active;
        cv_done.notify_all();
    }

    // Take the exchange steps the given sessions have reached, all due ones
    // in one lbm_shape_update_many call (repeated while an iteration of zero
    // steps leaves a session due again).  A session is done once it is due
    // with no iteration left, or failed.
    void take_events(std::vector<Session *> &ss) {
        for (;;) {
            std::vector<Session *> due;
            for (Session *s : ss)
                if (s->status == LBM_OK && s->to_go == 0 && s->req.kind == LBM_REQ_OPTIMIZE &&
                    s->iter < s->req.iterations)
                    due.push_back(s);
            if (due.empty()) return;
            std::vector<lbm_handle *> hs;
            std::vector<lbm_shape_params> ps;
            for (Session *s : due) {
                lbm_shape_params p = s->req.shape;
                p.seed = s->req.shape.seed + (uint64_t)s->iter;
                hs.push_back(s->h);
                ps.push_back(p);
            }
            std::vector<lbm_shape_result> rs(due.size());
            std::vector<int32_t> st(due.size(), LBM_OK);
            const double t0 = now_seconds();
            (void)lbm_shape_update_many(hs.data(), ps.data(), (int32_t)due.size(), rs.data(),
                                        st.data());
            {
                std::lock_guard<std::mutex> g(mu);
                this->st.exchange_seconds += now_seconds() - t0;
                this->st.exchanges += (int64_t)due.size();
                ++this->st.exchange_calls;
            }
            for (size_t k = 0; k < due.size(); ++k) {
                Session *s = due[k];
                if (st[k] != LBM_OK) {
                    s->status = st[k];
                    continue;
                }
                ++s->iter;
                s->to_go = s->req.steps_per_iteration;
            }
        }
    }
    static bool still_going(const Session &s) { return s.status == LBM_OK && s.to_go > 0; }

    void drop_group(int precision) {
        auto it = groups.find(precision);
        if (it == groups.end()) return;
        if (it->second.b) lbm_batch_destroy(it->second.b);
        groups.erase(it);
    }

    // Sessions whose handles the creation thread has made: failed ones
    // complete, the others take the events due at step 0 and start running.
    void start(std::vector<Session> &made) {
        for (Session &s : made) {
            --creating;
            if (s.status != LBM_OK) {  // no handle: release the budget it held
                used -= s.bytes;
                complete(s);
                continue;
            }
            s.to_go = s.req.solve_steps;
            std::vector<Session *> one{&s};
            take_events(one);
            if (!still_going(s)) {
                complete(s);
                continue;
            }
            active.push_back(s);
        }
    }

    // The creation thread: makes each admitted session's handle on its own
    // stream, then moves the handle to the worker's stream.
    void create_loop() {
        (void)hipSetDevice(device);
        for (;;) {
            Session s;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_create.wait(lk, [&] { return stop || !to_create.empty(); });
                if (stop) return;
                s = to_create.front();
                to_create.pop_front();
            }
            const double t0 = now_seconds();
            s.t_admit = t0;
            const int rc = lbm_create_geometry(&s.req.geom, nullptr, create_stream, &s.h);
            if (rc == LBM_OK) {
                lbm::handle_set_stream(s.h, stream);
            } else {
                s.status = rc;
                s.h = nullptr;
            }
            {
                std::lock_guard<std::mutex> g(mu);
                created.push_back(s);
                st.admit_seconds += now_seconds() - t0;
            }
            cv_work.notify_one();
        }
    }

    // Batch configuration: the configured one, else the autotuner's choice,
    // measured once per precision on the first batch of at least 8 members
    // (its trials restore every member's state); smaller batches before
    // that run one step per launch.
    int configure_batch(int precision, lbm_batch *b, int32_t members) {
        if (cfg.variant >= 0) return lbm_batch_configure(b, cfg.variant, cfg.order);
        auto it = tuned.find(precision);
        if (it != tuned.end()) return lbm_batch_configure(b, it->second.first, it->second.second);
        if (members >= 8) {
            int32_t v = 0, o = 0;
            const int rc = lbm_batch_tune(b, cfg.quantum, &v, &o, nullptr, 0);
            if (rc != LBM_OK) return rc;
            tuned[precision] = {v, o};
            return LBM_OK;
        }
        return lbm_batch_configure(b, lbm_tb_variant_count(precision), cfg.order);
    }

    void round() {
        const double t0 = now_seconds();
        int64_t q = cfg.quantum;
        for (const Session &s : active) q = std::min(q, s.to_go);
        // one batch per precision, rebuilt when its membership changed
        std::map<int, std::vector<lbm_handle *>> want;
        for (const Session &s : active) want[s.req.geom.precision].push_back(s.h);
        for (auto it = groups.begin(); it != groups.end();) {
            if (!want.count(it->first)) {
                if (it->second.b) lbm_batch_destroy(it->second.b);
                it = groups.erase(it);
            } else {
                ++it;
            }
        }
        std::map<int, int> failed;  // precision -> status
        int64_t nonsolid = 0;
        for (auto &kv : want) {
            Group &g = groups[kv.first];
            if (g.b && g.members != kv.second) {
                lbm_batch_destroy(g.b);
                g.b = nullptr;
            }
            int rc = LBM_OK;
            if (!g.b) {
                g.members = kv.second;
                rc = lbm_batch_create(g.members.data(), (int32_t)g.members.size(), stream, &g.b);
                if (rc == LBM_OK) rc = lbm_batch_set_graphs(g.b, 0);
                if (rc == LBM_OK) rc = configure_batch(kv.first, g.b, (int32_t)g.members.size());
            }
            if (rc == LBM_OK) rc = lbm_batch_run(g.b, q, nullptr);
            int64_t ns = 0;
            if (rc == LBM_OK) rc = lbm_batch_info(g.b, nullptr, nullptr, &ns);
            nonsolid += ns;
            if (rc != LBM_OK) failed[kv.first] = rc;
        }
        const double t1 = now_seconds();
        int64_t cells = 0;
        std::vector<Session *> all;
        for (Session &s : active) {
            auto f = failed.find(s.req.geom.precision);
            if (f != failed.end()) {
                s.status = f->second;
            } else {
                s.to_go -= q;
                s.steps += q;
                cells += (int64_t)s.req.geom.nx * s.req.geom.ny;
            }
            all.push_back(&s);
        }
        take_events(all);
        std::vector<Session> still;
        std::vector<Session> finished;
        for (Session &s : active) (still_going(s) ? still : finished).push_back(s);
        // batches hold the handles: drop the affected ones before releasing
        for (const Session &s : finished) drop_group(s.req.geom.precision);
        for (Session &s : finished) complete(s);
        active.swap(still);
        std::lock_guard<std::mutex> g(mu);
        const double t2 = now_seconds();
        ++st.rounds;
        st.cell_steps += cells * q;
        st.nonsolid_cell_steps += nonsolid * q;
        st.busy_seconds += t2 - t0;
        st.sweep_seconds += t1 - t0;
        st.event_seconds += t2 - t1;
    }

    void run() {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Session> made;
            {
                std::unique_lock<std::mutex> lk(mu);
                auto admissible = [&] {
                    return !queue.empty() &&
                           (int64_t)active.size() + creating < (int64_t)cfg.max_sessions &&
                           used + queue.front().bytes <= cfg.hbm_budget;
                };
                cv_work.wait(lk, [&] {
                    return stop || admissible() || !created.empty() || !active.empty();
                });
                if (stop) break;
                // admit in arrival order: the budget is taken now, the handle is
                // made by the creation thread
                bool any = false;
                while (admissible()) {
                    Session &q = queue.front();
                    used += q.bytes;
                    ++creating;
                    to_create.push_back(q);
                    queue.pop_front();
                    ++st.active;
                    --st.queued;
                    any = true;
                }
                st.peak_bytes = std::max(st.peak_bytes, used);
                if (any) cv_create.notify_one();
                made.assign(created.begin(), created.end());
                created.clear();
            }
            if (!made.empty()) {
                const double t0 = now_seconds();
                start(made);
                std::lock_guard<std::mutex> g(mu);
                st.busy_seconds += now_seconds() - t0;
            }
            if (!active.empty()) round();
        }
        for (auto &kv : groups)
            if (kv.second.b) lbm_batch_destroy(kv.second.b);
        groups.clear();
        for (Session &s : active)
            if (s.h) lbm_destroy(s.h);
        active.clear();
    }
};

extern "C" {

int lbm_server_create(const lbm_server_config *cfg, void *hip_stream, lbm_server **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget == 0 || cfg->max_sessions < 1 || cfg->quantum < 1 ||
        cfg->order < 0 || cfg->order > 1 || cfg->variant < -1)
        return LBM_EINVAL;
    lbm_server *s = new (std::nothrow) lbm_server;
    if (!s) return LBM_ENOMEM;
    s->cfg = *cfg;
    s->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return LBM_EHIP;
    }
    if (hipStreamCreateWithFlags(&s->create_stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return LBM_EHIP;
    }
    try {
        s->worker = std::thread([s] { s->run(); });
    } catch (...) {
        (void)hipStreamDestroy(s->create_stream);
        delete s;
        return LBM_ENOMEM;
    }
    try {
        s->creator = std::thread([s] { s->create_loop(); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
        (void)hipStreamDestroy(s->create_stream);
        delete s;
        return LBM_ENOMEM;
    }
    *out = s;
    return LBM_OK;
}

int lbm_server_submit(lbm_server *s, const lbm_request *req, uint64_t *id) {
    if (!s || !valid_request(req)) return LBM_EINVAL;
    Session ses;
    ses.req = *req;
    ses.bytes = lbm_footprint_bytes(&req->geom);
    ses.t_submit = now_seconds();
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return LBM_EINVAL;
    ses.id = s->next_id++;
    if (id) *id = ses.id;
    ++s->st.submitted;
    if (ses.bytes > s->cfg.hbm_budget) {
        lbm_result r{};
        r.id = ses.id;
        r.status = LBM_ENOMEM;
        r.cells = (int64_t)req->geom.nx * req->geom.ny;
        r.t_submit = r.t_admit = r.t_done = ses.t_submit;
        s->results.push_back(r);
        ++s->st.rejected;
        ++s->st.completed;
        s->cv_done.notify_all();
        return LBM_OK;
    }
    s->queue.push_back(ses);
    ++s->pending;
    ++s->st.queued;
    s->cv_work.notify_one();
    return LBM_OK;
}

int lbm_server_poll(lbm_server *s, lbm_result *out, int32_t cap, int32_t wait_ms) {
    if (!s || cap < 0 || (cap > 0 && !out)) return LBM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->results.empty() || (wait_ms < 0 && s->pending == 0); };
    if (wait_ms < 0)
        s->cv_done.wait(lk, ready);
    else if (wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
    int n = 0;
    while (n < cap && !s->results.empty()) {
        out[n++] = s->results.front();
        s->results.pop_front();
    }
    return n;
}

int lbm_server_drain(lbm_server *s) {
    if (!s) return LBM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->pending == 0; });
    return LBM_OK;
}

int lbm_server_stats_get(lbm_server *s, lbm_server_stats *st) {
    if (!s || !st) return LBM_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *st = s->st;
    return LBM_OK;
}

void lbm_server_destroy(lbm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_create.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->creator.joinable()) s->creator.join();
    // handles made but never run
    for (Session &x : s->created)
        if (x.h) lbm_destroy(x.h);
    (void)hipStreamDestroy(s->create_stream);
    delete s;
}

}  // extern "C"
