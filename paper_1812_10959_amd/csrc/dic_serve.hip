// Serving: a request loop over resident databases with continuous batching.
//
// One worker thread owns an Engine (its own stream).  Requests queue in
// arrival order; the worker admits the head of the queue whenever a slot is
// free and the request's memory bound fits the remaining budget, runs the
// admitted requests' first passes, and then advances every admitted request
// together a few stops at a time (one launch per kernel per stop for all of
// them), so requests that arrive while others are running join at the next
// stop chunk.  Finished requests free their slot and budget at once.
//
// The budget counts device memory: each admitted request's bound
// (job_bytes_bound: pool, per-item records, frequent-item bitsets, trace)
// and, once while any admitted request uses it, each database's resident
// rows and bitsets.  A request whose candidate pool overflows gives its
// memory back and goes to the head of the queue with the bound of the four
// times larger pool; it runs again when that fits, and fails with
// DIC_E_CAPACITY if it can never fit.  The engine's own tables (a few MB,
// allocated once) are not counted.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "dic_internal.h"

using namespace dic;

namespace dic {
// accessors implemented next to the database object
const uint64_t *db_rows(dic_db *db);
const uint64_t *db_vert(dic_db *db);
uint64_t db_n(dic_db *db);
uint32_t db_m(dic_db *db);
uint32_t db_W(dic_db *db);
void db_ref(dic_db *db, int delta);
uint64_t db_bytes(dic_db *db);
}  // namespace dic

namespace {

using clk = std::chrono::steady_clock;

// Stops advanced between admission checks: small enough that an arriving
// request waits at most a few stops, large enough to amortise a readback.
constexpr uint32_t SERVE_STEPS = 8;

struct Req {
    uint64_t ticket;
    dic_db *db;
    double minsup;
    uint64_t M;
    uint64_t bytes;  // budget charged while admitted (without the database)
    MineRequest again{};  // after a pool overflow: the rerun (again.mult > 1)
    clk::time_point submit;
    bool admitted = false, done = false;
    int status = DIC_OK;
    std::string error;
    MineOutput out;
};

}  // namespace

struct dic_server {
    uint64_t budget = 0;
    uint32_t max_active = 64;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    uint64_t used = 0, peak = 0;
    std::map<dic_db *, uint32_t> resident;  // databases of admitted requests
    uint32_t active = 0;
    bool stopping = false;
    std::vector<double> lat_ms;
    bool any = false;
    clk::time_point first_submit, last_done;
    int device = 0;
    std::thread worker;
};

namespace {

// Budget a request needs to be admitted now (its database counts once).
uint64_t need_of(dic_server *S, const Req *r)
{
    return r->bytes + (S->resident.count(r->db) ? 0 : db_bytes(r->db));
}

// Give an admitted request's memory back (called with S->mu held).
void release(dic_server *S, Req *r)
{
    if (!r->admitted)
        return;
    S->used -= r->bytes;
    auto it = S->resident.find(r->db);
    if (it != S->resident.end() && --it->second == 0) {
        S->used -= db_bytes(r->db);
        S->resident.erase(it);
    }
    S->active--;
    r->admitted = false;
}

// Hand a request's outcome over (called with S->mu held; the request holds
// no budget any more).
void complete(dic_server *S, Req *r, int status, MineOutput &&o)
{
    r->status = status;
    r->out = std::move(o);
    r->done = true;
    db_ref(r->db, -1);
    const auto now = clk::now();
    S->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->submit).count());
    S->last_done = now;
}

void finish(dic_server *S, Req *r, int status, MineOutput &&o)
{
    release(S, r);
    complete(S, r, status, std::move(o));
}

void worker_main(dic_server *S)
{
    (void)hipSetDevice(S->device);
    Engine eng(nullptr, S->max_active);  // its own stream: step graphs can be captured
    eng.set_requeue(true);  // overflowed requests come back through admission
    std::vector<std::pair<uint64_t, MineOutput>> done;
    for (;;) {
        std::vector<MineRequest> add;
        std::vector<uint64_t> ids;
        {
            std::unique_lock<std::mutex> g(S->mu);
            for (;;) {
                // admit from the head of the queue while slots and budget allow
                while (!S->queue.empty() && S->active < S->max_active) {
                    Req *r = S->reqs[S->queue.front()].get();
                    const uint64_t need = need_of(S, r);
                    if (S->used + need > S->budget)
                        break;
                    S->queue.pop_front();
                    r->admitted = true;
                    S->used += need;
                    S->resident[r->db]++;
                    S->peak = std::max(S->peak, S->used);
                    S->active++;
                    if (r->again.mult > 1) {
                        add.push_back(r->again);
                    } else {
                        add.push_back({db_rows(r->db), db_vert(r->db), (uint32_t)db_n(r->db),
                                       db_m(r->db), r->minsup, r->M});
                    }
                    ids.push_back(r->ticket);
                }
                if (!add.empty() || eng.size() > 0)
                    break;
                if (S->stopping)
                    return;
                S->cv_work.wait(g);
            }
        }
        int rc = DIC_OK;
        if (!add.empty()) {
            rc = eng.add(add, ids);
            if (rc) {
                std::lock_guard<std::mutex> g(S->mu);
                for (uint64_t t : ids) {
                    MineOutput o;
                    finish(S, S->reqs[t].get(), rc, std::move(o));
                }
                S->cv_done.notify_all();
            }
        }
        if (eng.size() > 0) {
            rc = eng.advance(SERVE_STEPS);
            done.clear();
            if (!rc)
                rc = eng.harvest(done);
            std::lock_guard<std::mutex> g(S->mu);
            bool any_done = false;
            for (auto &d : done) {
                Req *r = S->reqs[d.first].get();
                if (!d.second.requeue) {
                    finish(S, r, d.second.status, std::move(d.second));
                    any_done = true;
                    continue;
                }
                // pool overflow: back to the head of the queue with the
                // larger pool's bound, or fail if that can never fit
                release(S, r);
                r->again = d.second.again;
                r->bytes = job_bytes_bound(db_m(r->db), db_n(r->db), r->M, r->again.mult);
                if (r->bytes + db_bytes(r->db) > S->budget) {
                    r->error = "the request's candidate pool outgrew the budget";
                    MineOutput o;
                    complete(S, r, DIC_E_CAPACITY, std::move(o));
                    any_done = true;
                } else {
                    S->queue.push_front(r->ticket);
                }
            }
            if (any_done)
                S->cv_done.notify_all();
            if (!done.empty())
                S->cv_work.notify_one();
            if (rc) {
                // a device error: fail everything still in the engine and stop
                // using it; queued requests fail the same way, later submits too
                S->stopping = true;
                for (auto &kv : S->reqs)
                    if (!kv.second->done && kv.second->admitted) {
                        MineOutput o;
                        finish(S, kv.second.get(), rc, std::move(o));
                    }
                for (uint64_t t : S->queue) {
                    Req *r = S->reqs[t].get();
                    r->status = rc;
                    r->done = true;
                    db_ref(r->db, -1);
                }
                S->queue.clear();
                S->cv_done.notify_all();
                return;
            }
        }
    }
}

int take(dic_server *S, uint64_t ticket, dic_result **out, std::unique_lock<std::mutex> &g)
{
    (void)g;
    auto it = S->reqs.find(ticket);
    Req *r = it->second.get();
    int rc = r->status;
    if (!rc) {
        dic_result *res = new (std::nothrow) dic_result;
        if (!res) {
            rc = DIC_E_NOMEM;
        } else {
            res->W = db_W(r->db);
            res->masks = std::move(r->out.masks);
            res->counts = std::move(r->out.counts);
            res->trace = std::move(r->out.trace);
            res->stats = r->out.stats;
            *out = res;
        }
    } else {
        set_error(r->error.empty() ? std::string("request failed") : r->error);
    }
    S->reqs.erase(it);
    return rc;
}

}  // namespace

extern "C" {

int dic_serve_create(uint64_t hbm_budget_bytes, const dic_serve_opts *opts, dic_server **out)
{
    if (!out) {
        set_error("dic_serve_create: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    if (hbm_budget_bytes == 0) {
        set_error("dic_serve_create: budget must be > 0");
        return DIC_E_INVAL;
    }
    dic_server *S = new (std::nothrow) dic_server;
    if (!S) {
        set_error("host allocation failed");
        return DIC_E_NOMEM;
    }
    S->budget = hbm_budget_bytes;
    if (opts && opts->max_active)
        S->max_active = std::min<uint32_t>(opts->max_active, 4096);
    if (hipGetDevice(&S->device) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        set_error("dic_serve_create: no device");
        return DIC_E_DEVICE;
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return DIC_OK;
}

int dic_serve_submit(dic_server *S, dic_db *db, double minsup, uint64_t M, uint64_t *ticket)
{
    if (!S || !db || !ticket || !(minsup > 0.0) || M == 0) {
        set_error("dic_serve_submit: bad argument");
        return DIC_E_INVAL;
    }
    const uint64_t bytes = job_bytes_bound(db_m(db), db_n(db), M, 1);
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stopping) {
        set_error("dic_serve_submit: server is shutting down");
        return DIC_E_INVAL;
    }
    if (bytes + db_bytes(db) > S->budget) {
        set_error("dic_serve_submit: the request's memory bound exceeds the budget");
        return DIC_E_CAPACITY;
    }
    auto r = std::make_unique<Req>();
    r->ticket = S->next_ticket++;
    r->db = db;
    r->minsup = minsup;
    r->M = M;
    r->bytes = bytes;
    r->submit = clk::now();
    if (!S->any) {
        S->any = true;
        S->first_submit = r->submit;
    }
    db_ref(db, +1);
    *ticket = r->ticket;
    S->queue.push_back(r->ticket);
    S->reqs[r->ticket] = std::move(r);
    S->cv_work.notify_one();
    return DIC_OK;
}

int dic_serve_poll(dic_server *S, uint64_t ticket, dic_result **out)
{
    if (!S || !out) {
        set_error("dic_serve_poll: bad argument");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    std::unique_lock<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("dic_serve_poll: unknown ticket");
        return DIC_E_NOTFOUND;
    }
    if (!it->second->done)
        return DIC_E_PENDING;
    return take(S, ticket, out, g);
}

int dic_serve_wait(dic_server *S, uint64_t ticket, int64_t timeout_ms, dic_result **out)
{
    if (!S || !out) {
        set_error("dic_serve_wait: bad argument");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    std::unique_lock<std::mutex> g(S->mu);
    auto ready = [&] {
        auto it = S->reqs.find(ticket);
        return it == S->reqs.end() || it->second->done;
    };
    if (timeout_ms < 0) {
        S->cv_done.wait(g, ready);
    } else if (!S->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), ready)) {
        set_error("dic_serve_wait: timed out");
        return DIC_E_TIMEOUT;
    }
    if (S->reqs.find(ticket) == S->reqs.end()) {
        set_error("dic_serve_wait: unknown ticket");
        return DIC_E_NOTFOUND;
    }
    return take(S, ticket, out, g);
}

int dic_serve_stats(dic_server *S, double *p50_ms, double *p99_ms, double *throughput_rps)
{
    if (!S) {
        set_error("dic_serve_stats: server is NULL");
        return DIC_E_INVAL;
    }
    std::lock_guard<std::mutex> g(S->mu);
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) -> double {
        if (v.empty())
            return 0.0;
        // nearest rank
        size_t r = (size_t)std::ceil(p / 100.0 * (double)v.size());
        r = std::max<size_t>(1, std::min(r, v.size()));
        return v[r - 1];
    };
    if (p50_ms)
        *p50_ms = pct(50);
    if (p99_ms)
        *p99_ms = pct(99);
    if (throughput_rps) {
        double secs = v.empty() ? 0.0
                                : std::chrono::duration<double>(S->last_done - S->first_submit)
                                      .count();
        *throughput_rps = secs > 0 ? (double)v.size() / secs : 0.0;
    }
    return DIC_OK;
}

int dic_serve_usage(dic_server *S, uint64_t *used, uint64_t *peak, uint64_t *budget)
{
    if (!S) {
        set_error("dic_serve_usage: server is NULL");
        return DIC_E_INVAL;
    }
    std::lock_guard<std::mutex> g(S->mu);
    if (used)
        *used = S->used;
    if (peak)
        *peak = S->peak;
    if (budget)
        *budget = S->budget;
    return DIC_OK;
}

int dic_serve_destroy(dic_server *S)
{
    if (!S)
        return DIC_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stopping = true;
        // queued requests are dropped; running ones finish
        for (uint64_t t : S->queue) {
            Req *r = S->reqs[t].get();
            r->status = DIC_E_INVAL;
            r->done = true;
            db_ref(r->db, -1);
        }
        S->queue.clear();
        S->cv_work.notify_all();
    }
    if (S->worker.joinable())
        S->worker.join();
    delete S;
    return DIC_OK;
}

}  // extern "C"
