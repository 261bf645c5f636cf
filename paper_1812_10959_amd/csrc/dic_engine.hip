// Host engine: drives the per-stop kernels for a table of jobs.
//
// A run has three phases:
//   1. FirstPass on every job (item supports, frequent items), one readback
//      to learn each job's frequent-item count and size its candidate pool;
//   2. the stop loop: the host enqueues S stops at a time without looking at
//      the device (every kernel reads its job's state from device memory and
//      does nothing once the job is done), then reads back the small job
//      states once; S is the number of stops the live candidates still
//      certainly need, so no enqueued stop is idle;
//   3. collection of the solid boxes and the canonical sort.
// A job whose candidate pool overflowed is rerun with four times the room.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
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

constexpr uint32_t FP_ROWS = 4096;  // must match the first-pass kernel
constexpr uint32_t TRACE_INIT = 512;
constexpr uint32_t MAX_STEPS_PER_SYNC = 1024;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// splitmix64 (Steele, Lea & Flood's SplitMix generator in Vigna's 64-bit
// form): fills the per-item random words of the Zobrist itemset hash.
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::mutex g_zob_mu;
const unsigned long long *g_zob[64] = {};

const unsigned long long *zobrist(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return nullptr;
    std::lock_guard<std::mutex> g(g_zob_mu);
    if (g_zob[dev])
        return g_zob[dev];
    std::vector<unsigned long long> h(MAX_ITEMS);
    uint64_t seed = 0x5EED1812109590ull;
    for (auto &v : h)
        v = splitmix64(seed);
    void *d = nullptr;
    if (hipMalloc(&d, h.size() * 8) != hipSuccess)  // kept for the process lifetime
        return nullptr;
    if (hipMemcpyAsync(d, h.data(), h.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    g_zob[dev] = (const unsigned long long *)d;
    return g_zob[dev];
}

// A device buffer carved into aligned pieces.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    }
};

struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { if (p) dev_free(p); }
    bool alloc(size_t bytes) { p = dev_alloc(bytes ? bytes : 256); return p != nullptr; }
    char *at(size_t off) const { return (char *)p + off; }
};

struct JobPlanHost {
    uint32_t W, Mp, stop_max, tau;
    uint64_t n;
    uint32_t m;
    uint32_t cap = 0;
    uint32_t nL1 = 0;
    uint32_t trace_cap = TRACE_INIT;
    size_t a_cnt, a_l1;
    void *trace_buf = nullptr;
};

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

}  // namespace

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

uint64_t job_bytes(uint32_t n, uint32_t m, uint32_t cap, uint32_t trace_cap)
{
    (void)n;
    const uint64_t W = (m + 63u) / 64u;
    const uint64_t H = next_pow2(2ull * cap);
    uint64_t b = 0;
    b += sizeof(JobState) + 2ull * m * 4 + (uint64_t)trace_cap * sizeof(dic_stop_trace) + 1024;
    b += (uint64_t)cap * W * 8 * 2;         // pool masks + collected masks
    b += (uint64_t)cap * (8 + 8 + 5 * 4);   // hash, nonzero map, u32 fields
    b += (uint64_t)cap * 4 * 4;             // live0, live1, newbox, collected counts
    b += H * 8;                             // slots
    return b + 16 * 256;
}

static int run_once(const std::vector<MineRequest> &reqs, std::vector<MineOutput> &outs,
                    const std::vector<uint32_t> &cap_mult, std::vector<char> &overflowed,
                    hipStream_t s)
{
    const uint32_t njobs = (uint32_t)reqs.size();
    std::vector<JobPlanHost> H(njobs);
    const unsigned long long *zob = zobrist(s);
    if (!zob) {
        set_error("could not create the itemset hash table on the device");
        return DIC_E_DEVICE;
    }

    // ---- stage A: states, item counts, frequent items, traces, plan
    Carver ca;
    const size_t a_jobs = ca.take(sizeof(Job) * njobs);
    const size_t a_plan = ca.take(sizeof(Plan));
    const size_t a_pre_count = ca.take(4ull * (njobs + 1));
    const size_t a_pre_epi = ca.take(4ull * (njobs + 1));
    const size_t a_pre_cg = ca.take(8ull * (njobs + 1));
    const size_t a_pre_fp = ca.take(8ull * (njobs + 1));
    const size_t a_states = ca.take(sizeof(JobState) * njobs);
    const size_t a_outn = ca.take(4ull * njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        const MineRequest &r = reqs[j];
        JobPlanHost &h = H[j];
        uint64_t tau;
        threshold(r.minsup, r.n, &tau);  // validated by the caller
        h.n = r.n;
        h.m = r.m;
        h.W = (r.m + 63u) / 64u;
        h.Mp = (uint32_t)std::min<uint64_t>(r.M, r.n);
        h.stop_max = (uint32_t)((r.n + h.Mp - 1) / h.Mp);
        h.tau = (uint32_t)tau;
        h.a_cnt = ca.take(4ull * r.m);
        h.a_l1 = ca.take(4ull * r.m);
    }
    DevBuf A;
    if (!A.alloc(ca.off)) {
        set_error("device allocation failed (job states)");
        return DIC_E_NOMEM;
    }
    HIP_TRY(hipMemsetAsync(A.p, 0, ca.off, s));

    std::vector<Job> jobs(njobs);
    std::vector<DevBuf> traces(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        JobPlanHost &h = H[j];
        Job &J = jobs[j];
        std::memset(&J, 0, sizeof(Job));
        J.rows = reqs[j].rows;
        J.n = (uint32_t)h.n;
        J.m = h.m;
        J.W = h.W;
        J.Mp = h.Mp;
        J.stop_max = h.stop_max;
        J.tau = h.tau;
        J.st = (JobState *)A.at(a_states) + j;
        J.item_cnt = (uint32_t *)A.at(h.a_cnt);
        J.l1 = (uint32_t *)A.at(h.a_l1);
        J.out_n = (uint32_t *)A.at(a_outn) + j;
        if (!traces[j].alloc(sizeof(dic_stop_trace) * h.trace_cap)) {
            set_error("device allocation failed (trace)");
            return DIC_E_NOMEM;
        }
        J.trace = (dic_stop_trace *)traces[j].p;
        J.trace_cap = h.trace_cap;
    }
    Job *d_jobs = (Job *)A.at(a_jobs);
    Plan *d_plan = (Plan *)A.at(a_plan);
    Plan plan{};
    plan.njobs = njobs;
    plan.pre_count = (uint32_t *)A.at(a_pre_count);
    plan.pre_epi = (uint32_t *)A.at(a_pre_epi);
    plan.pre_cg = (unsigned long long *)A.at(a_pre_cg);
    plan.pre_fp = (unsigned long long *)A.at(a_pre_fp);
    plan.zobrist = zob;

    std::vector<unsigned long long> pre(njobs + 1, 0);
    for (uint32_t j = 0; j < njobs; ++j)
        pre[j + 1] = pre[j] + (H[j].n + FP_ROWS - 1) / FP_ROWS;
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(Job) * njobs, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_plan, &plan, sizeof(Plan), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(plan.pre_fp, pre.data(), 8ull * (njobs + 1), hipMemcpyHostToDevice, s));
    launch_first_pass(d_jobs, d_plan, pre[njobs], s);
    launch_l1_and_pairs_prepare(d_jobs, d_plan, njobs, s);
    HIP_TRY(hipGetLastError());

    std::vector<JobState> st(njobs);
    auto read_states = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(st.data(), A.at(a_states), sizeof(JobState) * njobs,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return DIC_OK;
    };
    int rc = read_states();
    if (rc)
        return rc;

    // ---- stage B: candidate pools sized from the pair count
    Carver cb;
    std::vector<size_t> b_off(njobs);
    std::vector<uint64_t> hslots(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        JobPlanHost &h = H[j];
        h.nL1 = st[j].nL1;
        const uint64_t nC2 = (uint64_t)h.nL1 * (h.nL1 ? h.nL1 - 1 : 0) / 2;
        uint64_t cap = std::max<uint64_t>(16384, 4 * nC2 + 16384) * cap_mult[j];
        if (cap > 0x7FFFFFFFull) {
            set_error("candidate pool would exceed 2^31 itemsets");
            return DIC_E_NOMEM;
        }
        h.cap = (uint32_t)cap;
        hslots[j] = next_pow2(2 * cap);
        b_off[j] = cb.off;
        cb.take(cap * h.W * 8);   // pmask
        cb.take(cap * 8);         // phash
        cb.take(cap * 8);         // pnz
        for (int f = 0; f < 5; ++f)
            cb.take(cap * 4);     // psupp pstop pstate ppromo pk
        cb.take(hslots[j] * 8);   // slots
        for (int f = 0; f < 3; ++f)
            cb.take(cap * 4);     // live0 live1 newbox
        cb.take(cap * h.W * 8);   // out_mask
        cb.take(cap * 4);         // out_cnt
    }
    DevBuf B;
    if (!B.alloc(cb.off)) {
        set_error("device allocation failed (candidate pools)");
        return DIC_E_NOMEM;
    }
    for (uint32_t j = 0; j < njobs; ++j) {
        JobPlanHost &h = H[j];
        Job &J = jobs[j];
        Carver c;
        c.off = b_off[j];
        const uint64_t cap = h.cap;
        J.cap = h.cap;
        J.hmask = (uint32_t)(hslots[j] - 1);
        J.pmask = (uint64_t *)B.at(c.take(cap * h.W * 8));
        J.phash = (unsigned long long *)B.at(c.take(cap * 8));
        J.pnz = (uint64_t *)B.at(c.take(cap * 8));
        J.psupp = (uint32_t *)B.at(c.take(cap * 4));
        J.pstop = (uint32_t *)B.at(c.take(cap * 4));
        J.pstate = (uint32_t *)B.at(c.take(cap * 4));
        J.ppromo = (uint32_t *)B.at(c.take(cap * 4));
        J.pk = (uint32_t *)B.at(c.take(cap * 4));
        J.slots = (unsigned long long *)B.at(c.take(hslots[j] * 8));
        J.live0 = (uint32_t *)B.at(c.take(cap * 4));
        J.live1 = (uint32_t *)B.at(c.take(cap * 4));
        J.newbox = (uint32_t *)B.at(c.take(cap * 4));
        J.out_mask = (uint64_t *)B.at(c.take(cap * h.W * 8));
        J.out_cnt = (uint32_t *)B.at(c.take(cap * 4));
        HIP_TRY(hipMemsetAsync(J.slots, 0xFF, hslots[j] * 8, s));
    }
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(Job) * njobs, hipMemcpyHostToDevice, s));
    for (uint32_t j = 0; j < njobs; ++j)
        pre[j + 1] = pre[j] + (unsigned long long)H[j].nL1 * H[j].nL1;
    HIP_TRY(hipMemcpyAsync(plan.pre_cg, pre.data(), 8ull * (njobs + 1), hipMemcpyHostToDevice, s));
    if (pre[njobs])
        launch_init_pairs(d_jobs, d_plan, pre[njobs], s);
    HIP_TRY(hipGetLastError());

    // ---- stop loop
    uint32_t steps = 0;
    for (uint32_t j = 0; j < njobs; ++j)
        steps = std::max(steps, st[j].max_rem);
    for (;;) {
        bool running = false;
        for (uint32_t j = 0; j < njobs; ++j)
            running |= !st[j].done && !st[j].overflow && st[j].k_next > 0;
        if (!running)
            break;
        uint32_t S = std::min(std::max(steps, 1u), MAX_STEPS_PER_SYNC);
        // every stop writes one trace entry: make room for S more
        bool table_dirty = false;
        for (uint32_t j = 0; j < njobs; ++j) {
            if (st[j].epoch + S <= H[j].trace_cap)
                continue;
            uint32_t nc = H[j].trace_cap;
            while (nc < st[j].epoch + S)
                nc *= 2;
            DevBuf nb;
            if (!nb.alloc(sizeof(dic_stop_trace) * nc)) {
                set_error("device allocation failed (trace)");
                return DIC_E_NOMEM;
            }
            HIP_TRY(hipMemcpyAsync(nb.p, traces[j].p, sizeof(dic_stop_trace) * H[j].trace_cap,
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            std::swap(nb.p, traces[j].p);
            H[j].trace_cap = nc;
            jobs[j].trace = (dic_stop_trace *)traces[j].p;
            jobs[j].trace_cap = nc;
            table_dirty = true;
        }
        if (table_dirty)
            HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(Job) * njobs, hipMemcpyHostToDevice,
                                   s));
        for (uint32_t k = 0; k < S; ++k)
            launch_step(d_jobs, d_plan, njobs, s);
        HIP_TRY(hipGetLastError());
        if ((rc = read_states()))
            return rc;
        steps = 0;
        for (uint32_t j = 0; j < njobs; ++j)
            if (!st[j].done && !st[j].overflow && st[j].k_next > 0)
                steps = std::max(steps, st[j].max_rem);
    }

    // ---- collect
    launch_collect(d_jobs, d_plan, njobs, s);
    HIP_TRY(hipGetLastError());
    std::vector<uint32_t> outn(njobs);
    HIP_TRY(hipMemcpyAsync(outn.data(), A.at(a_outn), 4ull * njobs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<std::vector<uint64_t>> om(njobs);
    std::vector<std::vector<uint32_t>> oc(njobs), icnt(njobs);
    for (uint32_t j = 0; j < njobs; ++j) {
        MineOutput &o = outs[j];
        overflowed[j] = st[j].overflow != 0;
        if (overflowed[j])
            continue;
        const uint32_t W = H[j].W;
        om[j].resize((size_t)outn[j] * W);
        oc[j].resize(outn[j]);
        icnt[j].resize(H[j].m);
        if (outn[j]) {
            HIP_TRY(hipMemcpyAsync(om[j].data(), jobs[j].out_mask, 8ull * outn[j] * W,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(oc[j].data(), jobs[j].out_cnt, 4ull * outn[j],
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipMemcpyAsync(icnt[j].data(), jobs[j].item_cnt, 4ull * H[j].m,
                               hipMemcpyDeviceToHost, s));
        const uint32_t ntr = std::min(st[j].epoch, H[j].trace_cap);
        o.trace.resize(ntr);
        if (ntr)
            HIP_TRY(hipMemcpyAsync(o.trace.data(), jobs[j].trace, sizeof(dic_stop_trace) * ntr,
                                   hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));

    for (uint32_t j = 0; j < njobs; ++j) {
        if (overflowed[j])
            continue;
        MineOutput &o = outs[j];
        const uint32_t W = H[j].W;
        // L = frequent items followed by the collected solid boxes
        std::vector<uint64_t> masks;
        std::vector<uint32_t> counts;
        for (uint32_t i = 0; i < H[j].m; ++i)
            if (icnt[j][i] >= H[j].tau) {
                size_t b = masks.size();
                masks.resize(b + W, 0);
                masks[b + (i >> 6)] = 1ull << (i & 63);
                counts.push_back(icnt[j][i]);
            }
        masks.insert(masks.end(), om[j].begin(), om[j].end());
        counts.insert(counts.end(), oc[j].begin(), oc[j].end());
        const size_t q = counts.size();
        std::vector<uint32_t> k(q), idx(q);
        for (size_t t = 0; t < q; ++t) {
            uint32_t c = 0;
            for (uint32_t w = 0; w < W; ++w)
                c += (uint32_t)__builtin_popcountll(masks[t * W + w]);
            k[t] = c;
        }
        std::iota(idx.begin(), idx.end(), 0u);
        std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
            return canon_less(&masks[(size_t)a * W], &masks[(size_t)b * W], W, k[a], k[b]);
        });
        o.masks.resize(q * W);
        o.counts.resize(q);
        uint64_t kmax = 0;
        for (size_t t = 0; t < q; ++t) {
            std::memcpy(&o.masks[t * W], &masks[(size_t)idx[t] * W], 8 * W);
            o.counts[t] = counts[idx[t]];
            kmax = std::max<uint64_t>(kmax, k[idx[t]]);
        }
        dic_stats &S = o.stats;
        S.tau = H[j].tau;
        S.block = H[j].Mp;
        S.stop_max = H[j].stop_max;
        S.stops = st[j].epoch;
        S.tests = st[j].tests;
        S.peak_live = st[j].peak_K;
        S.n_frequent = q;
        S.k_max = kmax;
        S.known = (uint64_t)H[j].m + std::min(st[j].pool_n, H[j].cap);
        o.status = st[j].asserts ? DIC_E_DEVICE : DIC_OK;
    }
    return DIC_OK;
}

int run_jobs(const std::vector<MineRequest> &reqs, std::vector<MineOutput> &outs,
             hipStream_t stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    outs.assign(reqs.size(), MineOutput{});
    std::vector<uint32_t> idx(reqs.size());
    std::iota(idx.begin(), idx.end(), 0u);
    std::vector<uint32_t> mult(reqs.size(), 1u);
    std::vector<uint32_t> restarts(reqs.size(), 0u);
    for (int attempt = 0; !idx.empty(); ++attempt) {
        if (attempt > 6) {
            set_error("candidate pool kept overflowing");
            for (uint32_t i : idx)
                outs[i].status = DIC_E_NOMEM;
            break;
        }
        std::vector<MineRequest> sub;
        std::vector<uint32_t> m;
        for (uint32_t i : idx) {
            sub.push_back(reqs[i]);
            m.push_back(mult[i]);
        }
        std::vector<MineOutput> so(sub.size());
        std::vector<char> ov(sub.size(), 0);
        int rc = run_once(sub, so, m, ov, stream);
        if (rc) {
            for (uint32_t i : idx)
                outs[i].status = rc;
            return rc;
        }
        std::vector<uint32_t> again;
        for (size_t t = 0; t < idx.size(); ++t) {
            const uint32_t i = idx[t];
            if (ov[t]) {
                mult[i] *= 4;
                restarts[i]++;
                again.push_back(i);
            } else {
                outs[i] = std::move(so[t]);
            }
        }
        idx.swap(again);
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t i = 0; i < outs.size(); ++i) {
        outs[i].stats.restarts = restarts[i];
        outs[i].stats.mine_ms = ms;
    }
    return DIC_OK;
}

}  // namespace dic
