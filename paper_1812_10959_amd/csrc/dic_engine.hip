// Host engine: drives the per-stop kernels for a changing set of jobs.
//
// Life of a job:
//   add      -> FirstPass (item supports, frequent items) for the new jobs,
//               one readback to size each candidate pool, then the pair
//               candidates are written on the device;
//   advance  -> the host enqueues S stops for every unfinished job without
//               looking at the device (each kernel reads its job's state from
//               device memory and does nothing for a finished job), then reads
//               the small job states back once.  S is at most the number of
//               stops the live candidates certainly still need, so enqueued
//               stops are not idle;
//   harvest  -> solid boxes are gathered, sorted canonically and returned;
//               a job whose pool overflowed is rerun with POOL_GROWTH times
//               the room (or handed back to its server for that).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <mutex>
#include <numeric>

#include "dic_internal.h"

namespace dic {

namespace {

#define HIP_TRY(x)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string(#x) + " failed: " + hipGetErrorString(e_));            \
            return DIC_E_DEVICE;                                                         \
        }                                                                                \
    } while (0)

constexpr uint32_t FP_ROWS = 4096;    // rows per first-pass work item (kernel side too)
constexpr uint32_t FPV_WORDS = 4096;  // bitset words per first-pass work item (kernel side too)
constexpr uint32_t TRACE_INIT = 512;
constexpr uint32_t MAX_RESTARTS = 4;
// Pool growth after an overflow.  A restart repeats the run from its first
// stop, so the larger step: a run that needs 256 times the first pool
// restarts twice instead of four times.
constexpr uint32_t POOL_GROWTH = 16;

bool canon_less(const uint64_t *A, const uint64_t *B, uint32_t W, uint32_t ka, uint32_t kb)
{
    if (ka != kb)
        return ka < kb;
    // Equal sizes: the ascending item list that holds the smallest item of
    // the symmetric difference is the lexicographically smaller one.
    for (uint32_t w = 0; w < W; ++w) {
        uint64_t x = A[w] ^ B[w];
        if (x)
            return (A[w] & (x & (~x + 1))) != 0;
    }
    return false;
}

std::atomic<int> g_profile{0};
std::atomic<uint32_t> g_layout{LAYOUT_VERTICAL};
std::atomic<uint32_t> g_init{0};  // 0: FirstPass, 1: classic DIC initialisation
std::atomic<bool> g_graphs{true};
std::atomic<int> g_poison{0};
std::mutex g_knob_mu;
Knobs g_knobs;
constexpr uint32_t GRAPH_STEPS = 8;  // stops per captured step graph

}  // namespace

bool profiling() { return g_profile.load() != 0; }
void set_profiling(int on) { g_profile.store(on); }
uint32_t count_layout() { return g_layout.load(); }
uint32_t init_mode() { return g_init.load(); }
void set_init_mode(uint32_t mode) { g_init.store(mode); }
bool use_graphs() { return g_graphs.load(); }
int poison() { return g_poison.load(); }
void set_poison(int byte) { g_poison.store(byte); }

Knobs knobs()
{
    std::lock_guard<std::mutex> g(g_knob_mu);
    return g_knobs;
}

int set_knob(const char *name, int64_t v)
{
    std::lock_guard<std::mutex> g(g_knob_mu);
    const std::string n(name);
    if (n == "vt_target" && v >= 64 && v <= 65536)
        g_knobs.vt_target = (uint32_t)v;
    else if (n == "vt_wave_k" && v >= 0 && v <= (1 << 30))
        g_knobs.vt_wave_k = (uint32_t)v;
    else if (n == "vt_tile_words" && v >= 1 && v <= VT_MAXW)
        g_knobs.vt_tile_words = (uint32_t)v;
    else if (n == "count_grid" && v >= 64 && v <= 65536)
        g_knobs.count_grid = (uint32_t)v;
    else if (n == "count_target" && v >= 64 && v <= 65536)
        g_knobs.count_target = (uint32_t)v;
    else if (n == "cells_clear" && v == 1) {
        std::fill(std::begin(g_knobs.cell_mode), std::end(g_knobs.cell_mode), (uint16_t)0);
        std::fill(std::begin(g_knobs.cell_target), std::end(g_knobs.cell_target), (uint16_t)0);
    } else if (n.compare(0, 5, "cell:") == 0) {
        // "cell:<block band>:<survivor band>": mode * 65536 + target
        unsigned b = 0, k = 0;
        char tail = 0;
        if (std::sscanf(n.c_str() + 5, "%u:%u%c", &b, &k, &tail) != 2 || b >= TUNE_BB ||
            k >= TUNE_KB)
            return DIC_E_INVAL;
        const int64_t mode = v >> 16, target = v & 0xFFFF;
        if (v < 0 || mode > 2 || (target != 0 && (target < 64 || target > 65535)))
            return DIC_E_INVAL;
        g_knobs.cell_mode[b * TUNE_KB + k] = (uint16_t)mode;
        g_knobs.cell_target[b * TUNE_KB + k] = (uint16_t)target;
    } else
        return DIC_E_INVAL;
    return DIC_OK;
}
void set_use_graphs(bool on) { g_graphs.store(on); }
void set_count_layout(uint32_t layout) { g_layout.store(layout); }

// ---------------------------------------------------------------------------
// threshold and sizes
// ---------------------------------------------------------------------------

bool threshold(double minsup, uint64_t n, uint64_t *tau)
{
    if (!(minsup > 0.0) || n == 0)
        return false;
    const double x = minsup * (double)n;
    uint64_t t;
    if (!(x < 9007199254740992.0)) {
        t = n + 1;
    } else {
        const double r = std::nearbyint(x);
        const double scale = x > 1.0 ? x : 1.0;
        t = std::fabs(x - r) <= 1e-9 * scale ? (uint64_t)r : (uint64_t)std::ceil(x);
    }
    if (t > n + 1)
        t = n + 1;
    if (t < 1)
        t = 1;
    *tau = t;
    return true;
}

uint64_t trace_bound(uint64_t n, uint64_t M, uint64_t cap)
{
    const uint64_t Mp = std::max<uint64_t>(1, std::min(M, n));
    const uint64_t stop_max = (n + Mp - 1) / Mp;
    uint32_t lg = 0;
    while (lg < 63 && (2ull << lg) <= cap)
        ++lg;
    return std::min<uint64_t>((lg + 3ull) * (stop_max + 1) + 2, 0x7FFFFFFFull);
}

uint64_t job_bytes_bound(uint32_t m, uint64_t n, uint64_t M, uint32_t mult)
{
    const uint32_t W = (m + 63u) / 64u;
    const uint64_t nw = (n + 63) / 64;
    const uint64_t cap = pool_cap_for(m, mult);
    const uint64_t tr = std::max<uint64_t>(TRACE_INIT, trace_bound(n, M, cap));
    return alloc_bytes(PoolLayout(cap, W).bytes) + alloc_bytes(12ull * m + 768) +
           alloc_bytes(8ull * m * nw) + 2 * alloc_bytes(tr * sizeof(dic_stop_trace));
}

// ---------------------------------------------------------------------------
// per-job host record
// ---------------------------------------------------------------------------

struct ActiveJob {
    uint64_t id = 0;
    MineRequest req{};
    uint32_t W = 0, Mp = 0, stop_max = 0, tau = 0;
    uint32_t mult = 1, restarts = 0;
    uint32_t cap = 0, nL1 = 0, trace_cap = TRACE_INIT;
    int slot = -1;
    void *small = nullptr;  // item counts, frequent items
    void *pool = nullptr;   // candidate pool
    void *fvert = nullptr;  // frequent items' bitsets (item-bitset jobs with an infrequent item)
    void *trace = nullptr;
    Job job{};
    uint32_t layout = LAYOUT_VERTICAL;
    uint32_t classic = 0;   // classic DIC start: every 1-itemset a candidate, no FirstPass
    bool in_loop = false;   // first candidates written, taking part in stops
    double count_ms = 0;
    uint64_t count_launches = 0;
    double first_pass_ms = 0;
    std::vector<uint32_t> stop_ns;  // per stop: its launch's duration (profiled runs)
    std::chrono::steady_clock::time_point t0;

    void release()
    {
        dev_free(small);
        dev_free(pool);
        dev_free(fvert);
        dev_free(trace);
        small = pool = fvert = trace = nullptr;
    }
    ~ActiveJob() { release(); }
};

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------

Engine::Engine(hipStream_t s, uint32_t max_jobs)
    : s_(s), max_jobs_(std::min(MAX_JOBS, std::max(1u, max_jobs)))
{
    if (!s_) {
        if (hipStreamCreateWithFlags(&s_, hipStreamNonBlocking) == hipSuccess)
            own_stream_ = true;
        else
            s_ = nullptr;
    }
    for (int i = (int)max_jobs_ - 1; i >= 0; --i)
        free_slots_.push_back(i);
    st_.resize(max_jobs_);
}

Engine::~Engine()
{
    (void)hipStreamSynchronize(s_);
    for (ActiveJob *j : jobs_)
        delete j;
    dev_free(slab_);
    dev_free(table_);
    dev_free(table_aux_);
    dev_free(plan_buf_);
    if (pinned_)
        (void)hipHostFree(pinned_);
    for (hipEvent_t e : events_)
        (void)hipEventDestroy(e);
    for (auto &a : graphs_)
        for (hipGraphExec_t g : a)
            if (g)
                (void)hipGraphExecDestroy(g);
    if (own_stream_)
        (void)hipStreamDestroy(s_);
}

// Run at least S stops for every job in the step table: replays of a
// captured GRAPH_STEPS-stop graph when graphs are on, direct launches
// otherwise.  With profiling, events bracket each CountSupport launch and
// *count_ms receives their summed elapsed time.
int Engine::launch_steps(uint32_t S, bool rows, bool vert, bool prof, double *count_ms,
                         uint32_t *steps_done)
{
    *count_ms = 0;
    launch_ms_.clear();
    if (prof) {
        const uint32_t need = 2 * std::max(S, GRAPH_STEPS);
        while (events_.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            events_.push_back(e);
        }
    }
    auto add_event_times = [&](uint32_t n) -> int {
        for (uint32_t k = 0; k < n; ++k) {
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, events_[2 * k], events_[2 * k + 1]));
            *count_ms += t;
            launch_ms_.push_back(t);
        }
        return DIC_OK;
    };
    const uint32_t grid = knobs().count_grid;
    launch_begin((Job *)table_, d_plan_step_, s_);
    // Events recorded inside a captured graph cannot be timed: profile directly.
    if (!use_graphs() || !own_stream_ || prof) {
        for (uint32_t k = 0; k < S; ++k)
            launch_step((const Job *)table_, d_plan_step_, s_, rows, vert, grid,
                        prof ? events_[2 * k] : nullptr, prof ? events_[2 * k + 1] : nullptr);
        HIP_TRY(hipGetLastError());
        *steps_done = S;
        if (prof) {
            HIP_TRY(hipStreamSynchronize(s_));
            return add_event_times(S);
        }
        return DIC_OK;
    }
    hipGraphExec_t &g = graphs_[rows][vert];
    if (g && graph_grid_[rows][vert] != grid) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    if (!g) {
        graph_grid_[rows][vert] = grid;
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
        for (uint32_t k = 0; k < GRAPH_STEPS; ++k)
            launch_step((const Job *)table_, d_plan_step_, s_, rows, vert, grid);
        const hipError_t le = hipGetLastError();
        HIP_TRY(hipStreamEndCapture(s_, &graph));
        HIP_TRY(le);
        const hipError_t ie = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_TRY(ie);
    }
    const uint32_t reps = (S + GRAPH_STEPS - 1) / GRAPH_STEPS;
    for (uint32_t r = 0; r < reps; ++r)
        HIP_TRY(hipGraphLaunch(g, s_));
    *steps_done = reps * GRAPH_STEPS;
    return DIC_OK;
}

bool Engine::running() const
{
    for (ActiveJob *j : jobs_) {
        const JobState &s = st_[j->slot];
        if (j->in_loop && job_running(s, j->cap))
            return true;
    }
    return false;
}

int Engine::read_states()
{
    int hi = -1;
    for (ActiveJob *j : jobs_)
        hi = std::max(hi, j->slot);
    if (hi >= 0)
        HIP_TRY(hipMemcpyAsync(st_.data(), slab_, sizeof(JobState) * (hi + 1),
                               hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));
    return DIC_OK;
}

int Engine::add(const std::vector<MineRequest> &reqs, const std::vector<uint64_t> &ids)
{
    if (reqs.size() > free_slots_.size()) {
        set_error("too many jobs for this engine");
        return DIC_E_INVAL;
    }
    std::vector<ActiveJob *> fresh;
    const auto now = std::chrono::steady_clock::now();
    const uint32_t layout = count_layout();
    const uint32_t classic = init_mode();
    for (size_t i = 0; i < reqs.size(); ++i) {
        ActiveJob *a = new ActiveJob;
        a->id = ids[i];
        a->req = reqs[i];
        a->mult = std::max(1u, reqs[i].mult);
        a->restarts = reqs[i].restarts;
        a->count_ms = reqs[i].count_ms;
        a->count_launches = reqs[i].count_launches;
        a->t0 = now;
        a->layout = reqs[i].vert ? layout : LAYOUT_ROWS;
        a->classic = classic;
        fresh.push_back(a);
    }
    return add_internal(fresh);
}

int Engine::add_internal(std::vector<ActiveJob *> &fresh)
{
    const int rc = add_impl(fresh);
    if (rc) {
        // drop the jobs of a failed add; the caller reports them
        for (ActiveJob *a : fresh) {
            auto it = std::find(jobs_.begin(), jobs_.end(), a);
            if (it != jobs_.end())
                jobs_.erase(it);
            if (a->slot >= 0)
                free_slots_.push_back(a->slot);
            delete a;
        }
        fresh.clear();
        (void)hipStreamSynchronize(s_);
    }
    return rc;
}

int Engine::add_impl(std::vector<ActiveJob *> &fresh)
{
    if (fresh.empty())
        return DIC_OK;
    // one first-pass kernel per layout: split a mixed set
    std::vector<ActiveJob *> same, other;
    for (ActiveJob *a : fresh)
        (a->layout == fresh[0]->layout ? same : other).push_back(a);
    if (!other.empty()) {
        int rc = add_impl(same);
        return rc ? rc : add_impl(other);
    }
    // one-time device buffers
    if (!slab_) {
        slab_ = dev_alloc(sizeof(JobState) * max_jobs_ + 4ull * max_jobs_);
        table_ = dev_alloc(sizeof(Job) * max_jobs_);
        table_aux_ = dev_alloc(sizeof(Job) * max_jobs_);
        Carver c;
        const size_t p0 = c.take(sizeof(Plan)), p1 = c.take(sizeof(Plan));
        const size_t a0 = c.take(4ull * (max_jobs_ + 1));
        const size_t av = c.take(4ull * (max_jobs_ + 1)), bv = c.take(4ull * (max_jobs_ + 1));
        const size_t a2 = c.take(8ull * (max_jobs_ + 1)), a3 = c.take(8ull * (max_jobs_ + 1));
        const size_t b0 = c.take(4ull * (max_jobs_ + 1));
        const size_t b2 = c.take(8ull * (max_jobs_ + 1)), b3 = c.take(8ull * (max_jobs_ + 1));
        const size_t tk = c.take(4ull * TICKET_WORDS);
        plan_buf_ = dev_alloc(c.off);
        if (!slab_ || !table_ || !table_aux_ || !plan_buf_) {
            set_error("device allocation failed (engine tables)");
            return DIC_E_NOMEM;
        }
        char *pb = (char *)plan_buf_;
        d_plan_step_ = (Plan *)(pb + p0);
        d_plan_aux_ = (Plan *)(pb + p1);
        plan_step_.pre_count = (uint32_t *)(pb + a0);
        plan_step_.pre_countv = (uint32_t *)(pb + av);
        plan_aux_.pre_countv = (uint32_t *)(pb + bv);
        plan_step_.pre_cg = (unsigned long long *)(pb + a2);
        plan_step_.pre_fp = (unsigned long long *)(pb + a3);
        plan_aux_.pre_count = (uint32_t *)(pb + b0);
        plan_aux_.pre_cg = (unsigned long long *)(pb + b2);
        plan_aux_.pre_fp = (unsigned long long *)(pb + b3);
        plan_step_.tickets = plan_aux_.tickets = (uint32_t *)(pb + tk);
        HIP_TRY(hipMemsetAsync(pb + tk, 0, 4ull * TICKET_WORDS, s_));
        HIP_TRY(hipMemsetAsync(slab_, 0, sizeof(JobState) * max_jobs_ + 4ull * max_jobs_, s_));
    }
    JobState *states = (JobState *)slab_;
    uint32_t *outn = (uint32_t *)(states + max_jobs_);

    // ---- per-job small buffers and records
    const uint32_t nf = (uint32_t)fresh.size();
    int rc = DIC_OK;
    for (ActiveJob *a : fresh) {
        const MineRequest &r = a->req;
        uint64_t tau = 0;
        threshold(r.minsup, r.n, &tau);  // validated by the caller
        a->W = (r.m + 63u) / 64u;
        a->Mp = (uint32_t)std::min<uint64_t>(r.M, r.n);
        a->stop_max = (uint32_t)((r.n + a->Mp - 1) / a->Mp);
        a->tau = (uint32_t)tau;
        jobs_.push_back(a);  // owned by the engine from here on
        if (free_slots_.empty()) {
            set_error("too many jobs for this engine");
            return DIC_E_INVAL;
        }
        a->slot = free_slots_.back();
        free_slots_.pop_back();
        a->small = dev_alloc(12ull * r.m + 768);
        a->trace = dev_alloc(sizeof(dic_stop_trace) * a->trace_cap);
        if (!a->small || !a->trace) {
            rc = DIC_E_NOMEM;
            set_error("device allocation failed (job records)");
        } else if (const int pb = poison()) {
            HIP_TRY(hipMemsetAsync(a->small, pb, 12ull * r.m + 768, s_));
            HIP_TRY(hipMemsetAsync(a->trace, pb, sizeof(dic_stop_trace) * a->trace_cap, s_));
        }
    }
    if (rc)
        return rc;
    aux_host_.assign(nf, Job{});
    for (uint32_t i = 0; i < nf; ++i) {
        ActiveJob *a = fresh[i];
        Job &J = a->job;
        std::memset(&J, 0, sizeof(Job));
        J.rows = a->req.rows;
        J.vert = a->req.vert;
        J.nw = (a->req.n + 63u) / 64u;
        J.layout = a->layout;
        J.classic = a->classic;
        J.n = a->req.n;
        J.m = a->req.m;
        J.W = a->W;
        J.Mp = a->Mp;
        J.stop_max = a->stop_max;
        J.tau = a->tau;
        J.item_cnt = (uint32_t *)a->small;
        J.l1 = (uint32_t *)((char *)a->small + align_up(4ull * a->req.m, 256));
        J.l1pos = (uint32_t *)((char *)a->small + 2 * align_up(4ull * a->req.m, 256));
        J.st = states + a->slot;
        J.out_n = outn + a->slot;
        J.trace = (dic_stop_trace *)a->trace;
        J.trace_cap = a->trace_cap;
        HIP_TRY(hipMemsetAsync(J.st, 0, sizeof(JobState), s_));
        HIP_TRY(hipMemsetAsync(J.item_cnt, 0, 4ull * a->req.m, s_));
        aux_host_[i] = J;
    }

    // ---- FirstPass for the new jobs (all of one layout: the option at add time)
    const bool vert = fresh[0]->layout == LAYOUT_VERTICAL;
    pre_host_.assign(nf + 1, 0);
    for (uint32_t i = 0; i < nf; ++i) {
        const uint64_t n = fresh[i]->req.n;
        const uint64_t work = fresh[i]->classic ? 0  // classic DIC counts items in the stops
                              : vert ? (uint64_t)fresh[i]->req.m *
                                           (((n + 63) / 64 + FPV_WORDS - 1) / FPV_WORDS)
                                     : (n + FP_ROWS - 1) / FP_ROWS;
        pre_host_[i + 1] = pre_host_[i] + work;
    }
    plan_aux_.njobs = nf;
    HIP_TRY(hipMemcpyAsync(table_aux_, aux_host_.data(), sizeof(Job) * nf,
                           hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(d_plan_aux_, &plan_aux_, sizeof(Plan), hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(plan_aux_.pre_fp, pre_host_.data(), 8ull * (nf + 1),
                           hipMemcpyHostToDevice, s_));
    const bool prof = profiling();
    if (prof) {
        while (events_.size() < 2) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            events_.push_back(e);
        }
        HIP_TRY(hipEventRecord(events_[0], s_));
    }
    if (vert)
        launch_first_pass_vert((const Job *)table_aux_, d_plan_aux_, pre_host_[nf], s_);
    else
        launch_first_pass((const Job *)table_aux_, d_plan_aux_, pre_host_[nf], s_);
    if (prof)
        HIP_TRY(hipEventRecord(events_[1], s_));
    launch_l1_and_pairs_prepare((const Job *)table_aux_, d_plan_aux_, nf, s_);
    HIP_TRY(hipGetLastError());
    if ((rc = read_states()))
        return rc;
    if (prof) {
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, events_[0], events_[1]));
        for (ActiveJob *a : fresh)
            a->first_pass_ms = t;
    }

    // ---- candidate pools sized from the frequent-item count
    for (uint32_t i = 0; i < nf; ++i) {
        ActiveJob *a = fresh[i];
        Job &J = a->job;
        a->nL1 = st_[a->slot].nL1;
        const uint64_t cap = pool_cap_for(a->nL1, a->mult);
        if (cap > 0x7FFFFFFFull) {
            set_error("candidate pool would exceed 2^31 itemsets");
            return DIC_E_NOMEM;
        }
        a->cap = (uint32_t)cap;
        const PoolLayout L(cap, a->W);
        a->pool = dev_alloc(L.bytes);
        if (!a->pool) {
            set_error("device allocation failed (candidate pool)");
            return DIC_E_NOMEM;
        }
        if (const int pb = poison())
            HIP_TRY(hipMemsetAsync(a->pool, pb, L.bytes, s_));
        pool_assign(J, L, (char *)a->pool, a->cap);
        // the counts read item rows by frequent-item index: gather those rows
        // unless every item is frequent (classic start: all items, in order)
        J.fvert = (uint64_t *)a->req.vert;
        if (a->layout == LAYOUT_VERTICAL && a->nL1 < a->req.m && a->nL1 >= 2) {
            if (!a->fvert)
                a->fvert = dev_alloc(8ull * a->nL1 * J.nw);
            if (!a->fvert) {
                set_error("device allocation failed (frequent-item bitsets)");
                return DIC_E_NOMEM;
            }
            if (const int pb = poison())
                HIP_TRY(hipMemsetAsync(a->fvert, pb, 8ull * a->nL1 * J.nw, s_));
            J.fvert = (uint64_t *)a->fvert;
        }
        HIP_TRY(hipMemsetAsync(J.slots, 0xFF, L.hslots * 8, s_));
        HIP_TRY(hipMemsetAsync(J.pcnt, 0, (size_t)cap * 8, s_));
        HIP_TRY(hipMemsetAsync(J.ctrs, 0, CTR_TOTAL * 4, s_));
        aux_host_[i] = J;
    }
    // first candidates: pairs of frequent items (nL1 x nL1 work), or every
    // 1-itemset in classic mode (nL1 = m)
    for (uint32_t i = 0; i < nf; ++i)
        pre_host_[i + 1] = pre_host_[i] + (fresh[i]->classic
                                               ? (unsigned long long)fresh[i]->nL1
                                               : (unsigned long long)fresh[i]->nL1 * fresh[i]->nL1);
    HIP_TRY(hipMemcpyAsync(table_aux_, aux_host_.data(), sizeof(Job) * nf,
                           hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(plan_aux_.pre_cg, pre_host_.data(), 8ull * (nf + 1),
                           hipMemcpyHostToDevice, s_));
    if (pre_host_[nf])
        launch_init_pairs((const Job *)table_aux_, d_plan_aux_, pre_host_[nf], s_);
    // frequent items' bitsets (the first pass is done with pre_fp)
    fp_host_.assign(nf + 1, 0);
    for (uint32_t i = 0; i < nf; ++i)
        fp_host_[i + 1] = fp_host_[i] + (aux_host_[i].fvert != aux_host_[i].vert
                                             ? (unsigned long long)fresh[i]->nL1 * aux_host_[i].nw
                                             : 0ull);
    if (fp_host_[nf]) {
        HIP_TRY(hipMemcpyAsync(plan_aux_.pre_fp, fp_host_.data(), 8ull * (nf + 1),
                               hipMemcpyHostToDevice, s_));
        launch_gather_vert((const Job *)table_aux_, d_plan_aux_, fp_host_[nf], s_);
    }
    HIP_TRY(hipGetLastError());
    // the host buffers above must outlive the copies: settle before returning
    HIP_TRY(hipStreamSynchronize(s_));
    for (ActiveJob *a : fresh)
        a->in_loop = true;
    table_dirty_ = true;
    return DIC_OK;
}

bool Engine::knobs_changed() const
{
    const Knobs k = knobs();
    return k.vt_target != plan_step_.vt_target || k.vt_wave_k != plan_step_.vt_wave_k ||
           k.vt_tile_words != plan_step_.vt_tile_words ||
           k.count_target != plan_step_.count_target ||
           std::memcmp(k.cell_mode, plan_step_.cell_mode, sizeof(k.cell_mode)) != 0 ||
           std::memcmp(k.cell_target, plan_step_.cell_target, sizeof(k.cell_target)) != 0;
}

int Engine::upload_table()
{
    const Knobs k = knobs();
    plan_step_.vt_target = k.vt_target;
    plan_step_.vt_wave_k = k.vt_wave_k;
    plan_step_.vt_tile_words = k.vt_tile_words;
    plan_step_.count_target = k.count_target;
    std::memcpy(plan_step_.cell_mode, k.cell_mode, sizeof(k.cell_mode));
    std::memcpy(plan_step_.cell_target, k.cell_target, sizeof(k.cell_target));
    table_host_.clear();
    for (ActiveJob *a : jobs_)
        if (a->in_loop)
            table_host_.push_back(a->job);
    plan_step_.njobs = (uint32_t)table_host_.size();
    if (!table_host_.empty())
        HIP_TRY(hipMemcpyAsync(table_, table_host_.data(), sizeof(Job) * table_host_.size(),
                               hipMemcpyHostToDevice, s_));
    HIP_TRY(hipMemcpyAsync(d_plan_step_, &plan_step_, sizeof(Plan), hipMemcpyHostToDevice, s_));
    table_dirty_ = false;
    return DIC_OK;
}

int Engine::ensure_trace(uint32_t steps)
{
    for (ActiveJob *a : jobs_) {
        if (!a->in_loop)
            continue;
        const uint32_t epoch = st_[a->slot].epoch;
        if (epoch + steps <= a->trace_cap)
            continue;
        // no run takes more stops than trace_bound: the kernels write no
        // entry at or beyond trace_cap, and collection checks the count
        const uint64_t most = std::max<uint64_t>(
            TRACE_INIT, trace_bound(a->req.n, a->req.M, a->cap ? a->cap : pool_cap_for(a->nL1, a->mult)));
        if (a->trace_cap >= most)
            continue;
        uint64_t nc = a->trace_cap;
        while (nc < epoch + steps)
            nc *= 2;
        nc = std::min(nc, most);
        void *nb = dev_alloc(sizeof(dic_stop_trace) * nc);
        if (!nb) {
            set_error("device allocation failed (trace)");
            return DIC_E_NOMEM;
        }
        if (const int pb = poison())
            HIP_TRY(hipMemsetAsync(nb, pb, sizeof(dic_stop_trace) * nc, s_));
        HIP_TRY(hipMemcpyAsync(nb, a->trace, sizeof(dic_stop_trace) * a->trace_cap,
                               hipMemcpyDeviceToDevice, s_));
        HIP_TRY(hipStreamSynchronize(s_));
        dev_free(a->trace);
        a->trace = nb;
        a->trace_cap = (uint32_t)nc;
        a->job.trace = (dic_stop_trace *)nb;
        a->job.trace_cap = (uint32_t)nc;
        table_dirty_ = true;
    }
    return DIC_OK;
}

int Engine::advance(uint32_t max_steps)
{
    if (!running())
        return DIC_OK;
    // stops that the next live set certainly needs: the survivors' remaining
    // stops, or a full pass for candidates created at the last stop
    uint32_t S = 1;
    for (ActiveJob *a : jobs_) {
        const JobState &s = st_[a->slot];
        if (a->in_loop && job_running(s, a->cap))
            S = std::max(S, job_need(s, a->cap, a->stop_max));
    }
    S = std::min(S, std::max(1u, max_steps));
    // graph replays run whole multiples of GRAPH_STEPS stops
    const bool prof = profiling();
    const uint32_t S_run = (use_graphs() && own_stream_ && !prof)
                               ? (S + GRAPH_STEPS - 1) / GRAPH_STEPS * GRAPH_STEPS
                               : S;
    // a pending job also begins its first stop, and the last stop of the
    // chunk begins the next one: up to S_run + 1 new trace entries
    int rc = ensure_trace(S_run + 1);
    if (rc)
        return rc;
    if ((table_dirty_ || knobs_changed()) && (rc = upload_table()))
        return rc;
    bool any_rows = false, any_vert = false;
    for (const Job &J : table_host_) {
        any_rows |= J.layout == LAYOUT_ROWS;
        any_vert |= J.layout == LAYOUT_VERTICAL;
    }
    double ms = 0;
    uint32_t done = 0;
    // trace index of each job's stop at the chunk's first launch (a pending
    // job begins its first stop in it)
    std::vector<uint32_t> first_idx;
    if (prof)
        for (ActiveJob *a : jobs_) {
            const JobState &s = st_[a->slot];
            first_idx.push_back(s.pending ? 0u : (s.epoch ? s.epoch - 1u : 0u));
        }
    if ((rc = launch_steps(S, any_rows, any_vert, prof, &ms, &done)))
        return rc;
    if ((rc = read_states()))
        return rc;
    if (prof) {
        for (size_t i = 0; i < jobs_.size(); ++i) {
            ActiveJob *a = jobs_[i];
            if (!a->in_loop)
                continue;
            for (size_t k = 0; k < launch_ms_.size(); ++k) {
                const size_t e = first_idx[i] + k;
                if (e >= a->stop_ns.size())
                    a->stop_ns.resize(e + 1, 0u);
                a->stop_ns[e] = (uint32_t)std::min(4.0e9, launch_ms_[k] * 1e6);
            }
        }
        for (ActiveJob *a : jobs_)
            if (a->in_loop) {
                a->count_ms += ms;
                a->count_launches += done;
            }
    }
    return DIC_OK;
}

int Engine::collect(std::vector<ActiveJob *> &fin,
                    std::vector<std::pair<uint64_t, MineOutput>> &out)
{
    const uint32_t nf = (uint32_t)fin.size();
    JobState *states = (JobState *)slab_;
    uint32_t *outn_d = (uint32_t *)(states + max_jobs_);
    aux_host_.assign(nf, Job{});
    for (uint32_t i = 0; i < nf; ++i) {
        aux_host_[i] = fin[i]->job;
        HIP_TRY(hipMemsetAsync(outn_d + fin[i]->slot, 0, 4, s_));
    }
    HIP_TRY(hipMemcpyAsync(table_aux_, aux_host_.data(), sizeof(Job) * nf, hipMemcpyHostToDevice,
                           s_));
    launch_collect((const Job *)table_aux_, d_plan_aux_, nf, s_);
    HIP_TRY(hipGetLastError());
    std::vector<uint32_t> outn(max_jobs_);
    HIP_TRY(hipMemcpyAsync(outn.data(), outn_d, 4ull * max_jobs_, hipMemcpyDeviceToHost, s_));
    HIP_TRY(hipStreamSynchronize(s_));

    // every finished job's boxes (masks, counts, sort keys), item counts and
    // trace, staged in pinned host memory by one copy each
    struct Part {
        size_t mask, cnt, key, icnt, trace;
        uint32_t q, ntr;
    };
    std::vector<Part> part(nf);
    size_t total = 0;
    auto take = [&total](size_t bytes) {
        const size_t at = total;
        total += (bytes + 255) & ~(size_t)255;
        return at;
    };
    for (uint32_t i = 0; i < nf; ++i) {
        ActiveJob *a = fin[i];
        Part &P = part[i];
        P.q = outn[a->slot];
        P.ntr = std::min(st_[a->slot].stops, a->trace_cap);
        P.mask = take(8ull * P.q * a->W);
        P.cnt = take(4ull * P.q);
        P.key = take(16ull * P.q);
        P.icnt = take(4ull * a->req.m);
        P.trace = take(sizeof(dic_stop_trace) * P.ntr);
    }
    if (total > pinned_cap_) {
        if (pinned_)
            (void)hipHostFree(pinned_);
        pinned_ = nullptr;
        pinned_cap_ = 0;
        if (hipHostMalloc(&pinned_, total, hipHostMallocDefault) == hipSuccess) {
            pinned_cap_ = total;
        } else {
            (void)hipGetLastError();  // pageable staging instead: slower copies, same results
            pinned_ = nullptr;
        }
    }
    std::vector<char> pageable;
    if (!pinned_)
        pageable.resize(total);
    char *pin = pinned_ ? (char *)pinned_ : pageable.data();
    for (uint32_t i = 0; i < nf; ++i) {
        ActiveJob *a = fin[i];
        const Part &P = part[i];
        if (P.q) {
            HIP_TRY(hipMemcpyAsync(pin + P.mask, a->job.out_mask, 8ull * P.q * a->W,
                                   hipMemcpyDeviceToHost, s_));
            HIP_TRY(hipMemcpyAsync(pin + P.cnt, a->job.out_cnt, 4ull * P.q, hipMemcpyDeviceToHost,
                                   s_));
            HIP_TRY(hipMemcpyAsync(pin + P.key, a->job.out_key, 16ull * P.q,
                                   hipMemcpyDeviceToHost, s_));
        }
        HIP_TRY(hipMemcpyAsync(pin + P.icnt, a->job.item_cnt, 4ull * a->req.m,
                               hipMemcpyDeviceToHost, s_));
        if (P.ntr)
            HIP_TRY(hipMemcpyAsync(pin + P.trace, a->trace, sizeof(dic_stop_trace) * P.ntr,
                                   hipMemcpyDeviceToHost, s_));
    }
    HIP_TRY(hipStreamSynchronize(s_));
    const auto now = std::chrono::steady_clock::now();

    std::vector<MineOutput> res(nf);
    for (uint32_t i = 0; i < nf; ++i) {
        ActiveJob *a = fin[i];
        const JobState &s = st_[a->slot];
        const Part &P = part[i];
        MineOutput &o = res[i];
        const uint32_t W = a->W;
        const uint64_t *bm = (const uint64_t *)(pin + P.mask);
        const uint32_t *bc = (const uint32_t *)(pin + P.cnt);
        const unsigned long long *bk = (const unsigned long long *)(pin + P.key);
        const uint32_t *ic = (const uint32_t *)(pin + P.icnt);
        o.trace.assign((const dic_stop_trace *)(pin + P.trace),
                       (const dic_stop_trace *)(pin + P.trace) + P.ntr);
        for (size_t e = 0; e < o.trace.size() && e < a->stop_ns.size(); ++e)
            o.trace[e].launch_ns = a->stop_ns[e];
        // L = the frequent items (src < 0) and the collected boxes (src >= 0),
        // in canonical order: by key, then in full where keys tie
        struct Entry {
            unsigned long long hi, lo;
            int64_t src;
        };
        std::vector<Entry> e;
        e.reserve(P.q + 64);
        for (uint32_t it = 0; it < a->req.m; ++it)
            if (ic[it] >= a->tau)
                e.push_back({(1ull << 59) | ((unsigned long long)it << 47), 0ull, -1 - (int64_t)it});
        for (uint32_t t = 0; t < P.q; ++t)
            e.push_back({bk[2 * (size_t)t], bk[2 * (size_t)t + 1], (int64_t)t});
        auto size_of = [&](const uint64_t *m) {
            uint32_t c = 0;
            for (uint32_t w = 0; w < W; ++w)
                c += (uint32_t)__builtin_popcountll(m[w]);
            return c;
        };
        // stable LSD radix sort on hi, one byte per pass (a pass whose byte is
        // the same for every entry is skipped), then each run of equal hi by
        // (lo, the full comparison)
        {
            std::vector<Entry> tmp(e.size());
            for (int d = 0; d < 8; ++d) {
                const int sh = 8 * d;
                size_t cnt[257] = {0};
                for (const Entry &x : e)
                    ++cnt[((x.hi >> sh) & 255u) + 1];
                if (*std::max_element(cnt + 1, cnt + 257) == e.size())
                    continue;
                for (int b = 0; b < 256; ++b)
                    cnt[b + 1] += cnt[b];
                for (const Entry &x : e)
                    tmp[cnt[(x.hi >> sh) & 255u]++] = x;
                e.swap(tmp);
            }
        }
        for (size_t r0 = 0; r0 < e.size();) {
            size_t r1 = r0 + 1;
            while (r1 < e.size() && e[r1].hi == e[r0].hi)
                ++r1;
            if (r1 - r0 > 1)
                std::sort(e.begin() + r0, e.begin() + r1, [&](const Entry &x, const Entry &y) {
                    if (x.lo != y.lo)
                        return x.lo < y.lo;
                    if (x.src < 0 || y.src < 0)  // single items never tie
                        return false;
                    const uint64_t *mx = bm + (size_t)x.src * W, *my = bm + (size_t)y.src * W;
                    return canon_less(mx, my, W, size_of(mx), size_of(my));
                });
            r0 = r1;
        }
        const size_t q = e.size();
        o.masks.assign(q * W, 0ull);
        o.counts.resize(q);
        uint64_t kmax = 0;
        for (size_t t = 0; t < q; ++t) {
            const Entry &x = e[t];
            uint64_t *dst = &o.masks[t * W];
            if (x.src < 0) {
                const uint32_t it = (uint32_t)(-1 - x.src);
                dst[it >> 6] = 1ull << (it & 63);
                o.counts[t] = ic[it];
            } else {
                std::memcpy(dst, bm + (size_t)x.src * W, 8 * W);
                o.counts[t] = bc[x.src];
            }
        }
        if (q) {
            // sizes ascend: the last itemset is a largest one
            const unsigned long long kf = e[q - 1].hi >> 59;
            kmax = kf < 31 ? kf : size_of(&o.masks[(q - 1) * W]);
            if (kf == 31)  // 31 or more: any of the trailing ones may be larger
                for (size_t t = q; t-- > 0 && (e[t].hi >> 59) == 31;)
                    kmax = std::max<uint64_t>(kmax, size_of(&o.masks[t * W]));
        }
        dic_stats &S = o.stats;
        S.tau = a->tau;
        S.block = a->Mp;
        S.stop_max = a->stop_max;
        S.stops = s.stops;
        S.tests = s.tests;
        S.peak_live = s.peak_K;
        S.n_frequent = q;
        S.k_max = kmax;
        // itemsets ever created: the 1-itemsets are pool entries in classic mode
        S.known = (a->classic ? 0ull : (uint64_t)a->req.m) + std::min(s.pool_n, a->cap);
        S.restarts = a->restarts;
        S.mine_ms = std::chrono::duration<double, std::milli>(now - a->t0).count();
        S.count_ms = a->count_ms;
        S.count_launches = a->count_launches;
        S.first_pass_ms = a->first_pass_ms;
        o.status = s.asserts ? DIC_E_DEVICE : DIC_OK;
        if (s.stops > a->trace_cap) {
            o.status = DIC_E_DEVICE;
            set_error("the run took more stops than its trace can hold");
        }
        out.emplace_back(a->id, std::move(o));
    }
    return DIC_OK;
}

int Engine::harvest(std::vector<std::pair<uint64_t, MineOutput>> &done)
{
    std::vector<ActiveJob *> fin, over, keep;
    for (ActiveJob *a : jobs_) {
        const JobState &s = st_[a->slot];
        if (!a->in_loop) {
            keep.push_back(a);
        } else if (s.overflow) {
            over.push_back(a);
        } else if (!job_running(s, a->cap)) {
            fin.push_back(a);
        } else {
            keep.push_back(a);
        }
    }
    if (fin.empty() && over.empty())
        return DIC_OK;
    int rc = DIC_OK;
    if (!fin.empty())
        rc = collect(fin, done);
    for (ActiveJob *a : fin) {
        free_slots_.push_back(a->slot);
        delete a;
    }
    jobs_.swap(keep);
    table_dirty_ = true;
    if (rc) {
        for (ActiveJob *a : over)
            delete a;
        return rc;
    }
    // rerun overflowed jobs with POOL_GROWTH times the candidate room (requeue
    // mode: hand them back to be added again once the room is granted)
    std::vector<ActiveJob *> again;
    for (ActiveJob *a : over) {
        free_slots_.push_back(a->slot);
        if (requeue_ && a->restarts < MAX_RESTARTS) {
            MineOutput o;
            o.requeue = true;
            o.again = a->req;
            o.again.mult = a->mult * POOL_GROWTH;
            o.again.restarts = a->restarts + 1;
            o.again.count_ms = a->count_ms;
            o.again.count_launches = a->count_launches;
            done.emplace_back(a->id, std::move(o));
            delete a;
            continue;
        }
        if (a->restarts >= MAX_RESTARTS) {
            MineOutput o;
            o.status = DIC_E_NOMEM;
            set_error("candidate pool kept overflowing");
            done.emplace_back(a->id, std::move(o));
            delete a;
            continue;
        }
        ActiveJob *b = new ActiveJob;
        b->id = a->id;
        b->req = a->req;
        b->t0 = a->t0;
        b->mult = a->mult * POOL_GROWTH;
        b->layout = a->layout;
        b->classic = a->classic;
        b->restarts = a->restarts + 1;
        b->count_ms = a->count_ms;
        b->count_launches = a->count_launches;
        delete a;
        again.push_back(b);
    }
    std::vector<uint64_t> again_ids;
    for (ActiveJob *b : again)
        again_ids.push_back(b->id);
    const int arc = add_internal(again);
    if (arc)
        for (uint64_t id : again_ids) {
            MineOutput o;
            o.status = arc;
            done.emplace_back(id, std::move(o));
        }
    return DIC_OK;
}

// ---------------------------------------------------------------------------
// run a fixed set of jobs to completion
// ---------------------------------------------------------------------------

namespace {
std::mutex g_pool_mu;
std::vector<Engine *> g_pool;  // idle engines, each with its own stream and graphs

struct PooledEngine {
    Engine *e;
    PooledEngine()
    {
        std::lock_guard<std::mutex> g(g_pool_mu);
        if (g_pool.empty()) {
            e = new Engine(nullptr, MAX_JOBS);
        } else {
            e = g_pool.back();
            g_pool.pop_back();
        }
    }
    ~PooledEngine()
    {
        if (e->size() == 0) {
            std::lock_guard<std::mutex> g(g_pool_mu);
            g_pool.push_back(e);
        } else {
            delete e;  // left jobs behind after an error: do not reuse
        }
    }
};
}  // namespace

int run_jobs(const std::vector<MineRequest> &reqs, std::vector<MineOutput> &outs,
             hipStream_t stream)
{
    outs.assign(reqs.size(), MineOutput{});
    if (reqs.empty())
        return DIC_OK;
    PooledEngine pe;
    Engine &eng = *pe.e;
    const uint32_t cap = MAX_JOBS;
    std::vector<uint64_t> ids(reqs.size());
    std::iota(ids.begin(), ids.end(), 0ull);
    size_t next = 0;
    std::vector<std::pair<uint64_t, MineOutput>> done;
    int rc = DIC_OK;
    while (next < reqs.size() || eng.size() > 0) {
        // keep the engine full: add as many pending jobs as it has room for
        const size_t room = cap - eng.size();
        if (next < reqs.size() && room > 0) {
            const size_t take = std::min(room, reqs.size() - next);
            std::vector<MineRequest> r(reqs.begin() + next, reqs.begin() + next + take);
            std::vector<uint64_t> id(ids.begin() + next, ids.begin() + next + take);
            if ((rc = eng.add(r, id)))
                break;
            next += take;
        }
        if ((rc = eng.advance(1024)))
            break;
        if ((rc = eng.harvest(done)))
            break;
    }
    if (rc) {
        for (auto &o : outs)
            o.status = rc;
        return rc;
    }
    for (auto &d : done)
        outs[d.first] = std::move(d.second);
    (void)stream;  // every result is on the host already: the run is complete
    return DIC_OK;
}

}  // namespace dic
