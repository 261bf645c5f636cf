// dic_mine_noalloc: mining one database with no allocation at call time.
//
// The same kernels as dic_mine (FirstPass, the pair candidates, the stop
// kernels of Algorithms 3-5 with MakeCandidates, the collection of solid
// boxes) run for one job whose working buffers -- job state, job record,
// plans, arrival counters, item counts, candidate pool, frequent-item
// bitsets -- are carved from `scratch`, one static device array per GPU,
// instead of being allocated.  Results go to host arrays the caller owns and
// are put in canonical order there, in place.  Buffers that must start at
// zero (or empty) are cleared with a fill kernel, never with a memset node.
//
// `scratch` is a host-side stand-in in host code: its device address is
// taken once per device with hipGetSymbolAddress (first call on that device)
// and only that address is used afterwards.  Every call on a device shares
// that device's array; calls from one process are serialised by a lock.
#include <chrono>
#include <cstring>
#include <mutex>
#include <utility>

#include "dic_internal.h"

static __device__ __align__(256) unsigned char scratch[DIC_NOALLOC_SCRATCH_BYTES];

namespace dic {
const uint64_t *db_rows(dic_db *db);
const uint64_t *db_vert(dic_db *db);
uint64_t db_n(dic_db *db);
uint32_t db_m(dic_db *db);
uint32_t db_W(dic_db *db);
std::mutex &db_mutex(dic_db *db);
}  // namespace dic

using namespace dic;

namespace {

constexpr int MAX_DEVICES = 64;
constexpr uint32_t MAX_STEPS = 1024;  // stops enqueued between two state readbacks
constexpr uint32_t MAX_MULT = 4096;   // pool growth after overflows, at most

std::mutex g_dev_mu[MAX_DEVICES];
char *g_ptr[MAX_DEVICES];          // device address of `scratch` on each device
hipStream_t g_stream[MAX_DEVICES];  // the stream the calls on that device run on

#define NA_TRY(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            set_error(std::string(#x) + " failed: " + hipGetErrorString(e_));            \
            return DIC_E_DEVICE;                                                         \
        }                                                                                \
    } while (0)

// Once per device, with that device current: the address of its copy of
// `scratch`, and a stream.
int setup(int dev)
{
    if (g_ptr[dev])
        return DIC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("dic_mine_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                  hipGetErrorString(e));
        return DIC_E_DEVICE;
    }
    hipStream_t s = nullptr;
    NA_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g_stream[dev] = s;
    g_ptr[dev] = (char *)p;
    return DIC_OK;
}

// Canonical order of two itemsets (size, then ascending item lists).
bool canon_before(const uint64_t *A, const uint64_t *B, uint32_t W)
{
    uint32_t ka = 0, kb = 0;
    for (uint32_t w = 0; w < W; ++w) {
        ka += (uint32_t)__builtin_popcountll(A[w]);
        kb += (uint32_t)__builtin_popcountll(B[w]);
    }
    if (ka != kb)
        return ka < kb;
    for (uint32_t w = 0; w < W; ++w) {
        const uint64_t x = A[w] ^ B[w];
        if (x)
            return (A[w] & (x & (~x + 1))) != 0;  // A holds the smallest differing item
    }
    return false;
}

// In-place heapsort of q (mask, count) records into canonical order.
void sort_records(uint64_t *masks, uint32_t *counts, uint64_t q, uint32_t W)
{
    auto less = [&](uint64_t a, uint64_t b) { return canon_before(masks + a * W, masks + b * W, W); };
    auto swap_rec = [&](uint64_t a, uint64_t b) {
        for (uint32_t w = 0; w < W; ++w)
            std::swap(masks[a * W + w], masks[b * W + w]);
        std::swap(counts[a], counts[b]);
    };
    auto sift = [&](uint64_t root, uint64_t end) {
        for (;;) {
            uint64_t c = 2 * root + 1;
            if (c >= end)
                return;
            if (c + 1 < end && less(c, c + 1))
                ++c;
            if (!less(root, c))
                return;
            swap_rec(root, c);
            root = c;
        }
    };
    for (uint64_t i = q / 2; i-- > 0;)
        sift(i, q);
    for (uint64_t end = q; end > 1; --end) {
        swap_rec(0, end - 1);
        sift(0, end - 1);
    }
}

// Host side of one call: everything the kernels read is copied from here,
// so it lives until the call's last synchronisation.
struct Run {
    Job J;
    Plan aux, step;
    JobState st;
    unsigned long long pre_fp[2], pre_cg[2];
    uint32_t zero_u32[2];
    uint32_t ic[MAX_ITEMS];
};

constexpr int OVERFLOWED = 1;

// One attempt with candidate capacity pool_cap_for(nL1, mult).  Returns
// DIC_OK, OVERFLOWED (the pool filled up) or an error.
int mine_once(char *base, hipStream_t s, const MineRequest &req, uint32_t layout, uint32_t classic,
              uint32_t mult, Run &R, uint64_t *masks, uint32_t *counts, uint64_t capacity,
              uint64_t *size, dic_stats *stats)
{
    const uint32_t n = req.n, m = req.m, W = (m + 63u) / 64u, nw = (n + 63u) / 64u;
    uint64_t tau = 0;
    threshold(req.minsup, n, &tau);
    const uint32_t Mp = (uint32_t)(req.M < n ? req.M : n);
    const uint32_t stop_max = (n + Mp - 1u) / Mp;

    // fixed part of the scratch layout
    Carver c;
    const size_t o_st = c.take(sizeof(JobState) + 4);  // state, then the collected count
    const size_t o_job = c.take(sizeof(Job));
    const size_t o_aux = c.take(sizeof(Plan)), o_step = c.take(sizeof(Plan));
    const size_t o_a_fp = c.take(16), o_a_cg = c.take(16);
    const size_t o_s_count = c.take(8), o_s_countv = c.take(8);
    const size_t o_s_cg = c.take(16), o_s_fp = c.take(16);
    const size_t o_tk = c.take(4ull * TICKET_WORDS);
    const size_t m4 = align_up(4ull * m, 256);
    const size_t o_small = c.take(3 * m4);
    JobState *d_st = (JobState *)(base + o_st);
    uint32_t *d_outn = (uint32_t *)(base + o_st + sizeof(JobState));
    Job *d_job = (Job *)(base + o_job);
    Plan *d_aux = (Plan *)(base + o_aux), *d_step = (Plan *)(base + o_step);
    uint32_t *tickets = (uint32_t *)(base + o_tk);

    launch_fill32((uint32_t *)d_st, 0u, (sizeof(JobState) + 4) / 4, s);
    launch_fill32(tickets, 0u, TICKET_WORDS, s);
    launch_fill32((uint32_t *)(base + o_small), 0u, m, s);  // item counts

    Job &J = R.J;
    std::memset(&J, 0, sizeof(Job));
    J.rows = req.rows;
    J.vert = req.vert;
    J.fvert = (uint64_t *)req.vert;
    J.nw = nw;
    J.layout = layout;
    J.classic = classic;
    J.n = n;
    J.m = m;
    J.W = W;
    J.Mp = Mp;
    J.stop_max = stop_max;
    J.tau = (uint32_t)tau;
    J.item_cnt = (uint32_t *)(base + o_small);
    J.l1 = (uint32_t *)(base + o_small + m4);
    J.l1pos = (uint32_t *)(base + o_small + 2 * m4);
    J.st = d_st;
    J.out_n = d_outn;
    J.trace = nullptr;  // no per-stop trace: its fields are only ever written
    J.trace_cap = 0;

    std::memset(&R.aux, 0, sizeof(Plan));
    R.aux.njobs = 1;
    R.aux.pre_fp = (unsigned long long *)(base + o_a_fp);
    R.aux.pre_cg = (unsigned long long *)(base + o_a_cg);
    R.aux.tickets = tickets;
    const bool vert = layout == LAYOUT_VERTICAL;
    R.pre_fp[0] = 0;
    R.pre_fp[1] = classic ? 0ull
                  : vert  ? (unsigned long long)m * ((nw + 4095ull) / 4096ull)
                          : (n + 4095ull) / 4096ull;
    NA_TRY(hipMemcpyAsync(d_job, &J, sizeof(Job), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(d_aux, &R.aux, sizeof(Plan), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(R.aux.pre_fp, R.pre_fp, 16, hipMemcpyHostToDevice, s));
    if (R.pre_fp[1]) {
        if (vert)
            launch_first_pass_vert(d_job, d_aux, R.pre_fp[1], s);
        else
            launch_first_pass(d_job, d_aux, R.pre_fp[1], s);
    }
    launch_l1_and_pairs_prepare(d_job, d_aux, 1, s);
    NA_TRY(hipGetLastError());
    NA_TRY(hipMemcpyAsync(&R.st, d_st, sizeof(JobState), hipMemcpyDeviceToHost, s));
    NA_TRY(hipStreamSynchronize(s));

    // the candidate pool (and the frequent items' bitsets) after the fixed part
    const uint32_t nL1 = R.st.nL1;
    const uint64_t cap = pool_cap_for(nL1, mult);
    const PoolLayout L(cap < 0x7FFFFFFFull ? cap : 1, W);
    const bool gather = vert && nL1 < m && nL1 >= 2;
    const size_t o_pool = c.take(L.bytes);
    const size_t o_fvert = gather ? c.take(8ull * nL1 * nw) : c.off;
    if (cap >= 0x7FFFFFFFull || c.off > DIC_NOALLOC_SCRATCH_BYTES) {
        set_error("dic_mine_noalloc: this mine needs " + std::to_string(c.off) +
                  " bytes of working memory; the scratch array holds " +
                  std::to_string((unsigned long long)DIC_NOALLOC_SCRATCH_BYTES));
        return DIC_E_CAPACITY;
    }
    pool_assign(J, L, base + o_pool, (uint32_t)cap);
    if (gather)
        J.fvert = (uint64_t *)(base + o_fvert);
    launch_fill32((uint32_t *)J.slots, 0xFFFFFFFFu, 2 * L.hslots, s);
    launch_fill32((uint32_t *)J.pcnt, 0u, 2 * cap, s);
    launch_fill32(J.ctrs, 0u, CTR_TOTAL, s);
    NA_TRY(hipMemcpyAsync(d_job, &J, sizeof(Job), hipMemcpyHostToDevice, s));
    R.pre_cg[0] = 0;
    R.pre_cg[1] = classic ? (unsigned long long)nL1 : (unsigned long long)nL1 * nL1;
    NA_TRY(hipMemcpyAsync(R.aux.pre_cg, R.pre_cg, 16, hipMemcpyHostToDevice, s));
    if (R.pre_cg[1])
        launch_init_pairs(d_job, d_aux, R.pre_cg[1], s);
    if (gather) {
        R.pre_fp[1] = (unsigned long long)nL1 * nw;
        NA_TRY(hipMemcpyAsync(R.aux.pre_fp, R.pre_fp, 16, hipMemcpyHostToDevice, s));
        launch_gather_vert(d_job, d_aux, R.pre_fp[1], s);
    }
    const Knobs k = knobs();
    std::memset(&R.step, 0, sizeof(Plan));
    R.step.njobs = 1;
    R.step.pre_count = (uint32_t *)(base + o_s_count);
    R.step.pre_countv = (uint32_t *)(base + o_s_countv);
    R.step.pre_cg = (unsigned long long *)(base + o_s_cg);
    R.step.pre_fp = (unsigned long long *)(base + o_s_fp);
    R.step.vt_target = k.vt_target;
    R.step.vt_wave_k = k.vt_wave_k;
    R.step.vt_tile_words = k.vt_tile_words;
    R.step.count_target = k.count_target;
    std::memcpy(R.step.cell_mode, k.cell_mode, sizeof(k.cell_mode));
    std::memcpy(R.step.cell_target, k.cell_target, sizeof(k.cell_target));
    R.step.tickets = tickets;
    NA_TRY(hipMemcpyAsync(d_step, &R.step, sizeof(Plan), hipMemcpyHostToDevice, s));
    NA_TRY(hipGetLastError());
    NA_TRY(hipStreamSynchronize(s));

    // stops, S at a time, until no candidate is live
    for (;;) {
        NA_TRY(hipMemcpyAsync(&R.st, d_st, sizeof(JobState), hipMemcpyDeviceToHost, s));
        NA_TRY(hipStreamSynchronize(s));
        if (!job_running(R.st, (uint32_t)cap))
            break;
        uint32_t S = job_need(R.st, (uint32_t)cap, stop_max);
        S = S < 1u ? 1u : (S > MAX_STEPS ? MAX_STEPS : S);
        launch_begin(d_job, d_step, s);
        for (uint32_t t = 0; t < S; ++t)
            launch_step(d_job, d_step, s, !vert, vert, k.count_grid);
        NA_TRY(hipGetLastError());
    }
    if (R.st.overflow)
        return OVERFLOWED;

    // L: the frequent items, then the collected solid boxes, sorted in place
    launch_fill32(d_outn, 0u, 1, s);
    launch_collect(d_job, d_aux, 1, s);
    NA_TRY(hipGetLastError());
    NA_TRY(hipMemcpyAsync(R.zero_u32, d_outn, 4, hipMemcpyDeviceToHost, s));
    NA_TRY(hipMemcpyAsync(R.ic, J.item_cnt, 4ull * m, hipMemcpyDeviceToHost, s));
    NA_TRY(hipStreamSynchronize(s));
    const uint64_t q = R.zero_u32[0];
    uint64_t nf1 = 0;
    for (uint32_t i = 0; i < m; ++i)
        nf1 += R.ic[i] >= tau;
    *size = nf1 + q;
    if (nf1 + q > capacity) {
        set_error("dic_mine_noalloc: the result has " + std::to_string(nf1 + q) +
                  " itemsets; the output arrays hold " + std::to_string(capacity));
        return DIC_E_CAPACITY;
    }
    if (q) {
        NA_TRY(hipMemcpyAsync(masks + nf1 * W, J.out_mask, 8ull * q * W, hipMemcpyDeviceToHost, s));
        NA_TRY(hipMemcpyAsync(counts + nf1, J.out_cnt, 4ull * q, hipMemcpyDeviceToHost, s));
    }
    uint64_t t = 0;
    for (uint32_t i = 0; i < m; ++i)
        if (R.ic[i] >= tau) {
            std::memset(masks + t * W, 0, 8ull * W);
            masks[t * W + (i >> 6)] = 1ull << (i & 63u);
            counts[t] = R.ic[i];
            ++t;
        }
    NA_TRY(hipStreamSynchronize(s));
    sort_records(masks + nf1 * W, counts + nf1, q, W);
    if (stats) {
        std::memset(stats, 0, sizeof(dic_stats));
        stats->tau = tau;
        stats->block = Mp;
        stats->stop_max = stop_max;
        stats->stops = R.st.stops;
        stats->tests = R.st.tests;
        stats->peak_live = R.st.peak_K;
        stats->n_frequent = nf1 + q;
        uint32_t kmax = 0;
        if (nf1 + q) {
            const uint64_t *last = masks + (nf1 + q - 1) * W;
            for (uint32_t w = 0; w < W; ++w)
                kmax += (uint32_t)__builtin_popcountll(last[w]);
        }
        stats->k_max = kmax;
        const uint32_t pn = R.st.pool_n < (uint32_t)cap ? R.st.pool_n : (uint32_t)cap;
        stats->known = (classic ? 0ull : (uint64_t)m) + pn;
    }
    return R.st.asserts ? DIC_E_DEVICE : DIC_OK;
}

}  // namespace

extern "C" {

int dic_mine_noalloc(dic_db *db, double minsup, uint64_t M, uint64_t *masks, uint32_t *counts,
                     uint64_t capacity, uint64_t *size, dic_stats *stats)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!db || !size || (capacity && (!masks || !counts))) {
        set_error("dic_mine_noalloc: NULL argument");
        return DIC_E_INVAL;
    }
    *size = 0;
    if (!(minsup > 0.0) || M == 0) {
        set_error("dic_mine_noalloc: minsup must be > 0 (not NaN) and M >= 1");
        return DIC_E_INVAL;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        set_error("dic_mine_noalloc: no usable current device");
        return DIC_E_DEVICE;
    }
    std::lock_guard<std::mutex> gd(g_dev_mu[dev]);
    int rc = setup(dev);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> gdb(db_mutex(db));
    const MineRequest req{db_rows(db), db_vert(db), (uint32_t)db_n(db), db_m(db), minsup, M};
    const uint32_t layout = count_layout(), classic = init_mode();
    static thread_local Run R;  // host copies of the device records (no heap use per call)
    uint32_t restarts = 0;
    for (uint32_t mult = 1;; mult *= 4, ++restarts) {
        rc = mine_once(g_ptr[dev], g_stream[dev], req, layout, classic, mult, R, masks, counts,
                       capacity, size, stats);
        if (rc != OVERFLOWED)
            break;
        if (mult >= MAX_MULT) {
            set_error("dic_mine_noalloc: candidate pool kept overflowing");
            return DIC_E_CAPACITY;
        }
    }
    if (rc == DIC_OK && stats) {
        stats->restarts = restarts;
        stats->mine_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
    }
    return rc;
}

}  // extern "C"
