// Internal declarations of the GPU library: device-visible job records, the
// per-stop work plan, kernel launchers and the host engine.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dic.h"

namespace dic {

// ---------------------------------------------------------------------------
// Itemset standing.  DIC keeps four sets (Section 3): dashed/solid x
// circle/box; pruned itemsets (Algorithm 4) stay known so they are never
// generated again.
// ---------------------------------------------------------------------------
enum : uint32_t {
    ST_DASHED_CIRCLE = 0,
    ST_DASHED_BOX = 1,
    ST_PRUNED = 2,
    ST_SOLID_CIRCLE = 3,
    ST_SOLID_BOX = 4,
};

constexpr unsigned long long SLOT_EMPTY = ~0ull;
constexpr uint32_t MAX_ITEMS = 4096;  // W <= 64, so a 64-bit map covers the words
constexpr int WG = 256;               // threads per workgroup in every kernel
constexpr uint32_t MAX_JOBS = 4096;   // jobs in one engine (one step launch) at most
constexpr int CW = 16;                // candidates per wave in the count kernel
constexpr int CAND_PER_WG = CW * (WG / 64);
constexpr int LDS_DWORDS = 8192;      // count kernel row tile (32 KiB)
constexpr int MAX_GROUPS = 16;        // 64-row groups per row tile (1024 rows)
constexpr int VT_WORDS = 6144;        // vertical tile: 64-bit words in LDS (48 KiB)
constexpr int VT_MAXW = 16;           // vertical tile: words per item (1024 rows)

enum : uint32_t { LAYOUT_ROWS = 0, LAYOUT_VERTICAL = 1 };

// Words per frequent item in a vertical tile (the tile holds every frequent
// item's bitset over those words) and the odd row stride that spreads the
// items' words over the LDS banks.  A power of two (16, 8, 4, 2 or 1): the
// count reads 16-, 8- and 4-word rows whole, without a condition per word.
__host__ __device__ inline uint32_t vert_tile_words(uint32_t nL1, uint32_t max_words,
                                                    uint32_t capacity = VT_WORDS)
{
    uint32_t t = nL1 ? capacity / nL1 : (uint32_t)VT_MAXW + 1u;
    t = t > 1u ? t - 1u : 1u;
    const uint32_t cap = max_words < (uint32_t)VT_MAXW ? max_words : (uint32_t)VT_MAXW;
    t = t > cap ? cap : t;
    uint32_t p = 1u;
    while (2u * p <= t)
        p *= 2u;
    return p;
}

// Tuning knobs of the count planning and launch (set by dic_set_option or
// the autotuner; every setting gives the same results).
// Per-shape planning of the bitset count: a cell per (band of the block's
// 64-row words, band of the survivors counted at the stop).  A cell's mode
// is 0 (fall back to vt_wave_k / vt_target), 1 (one wave per candidate) or
// 2 (LDS tiles with `target` workgroups aimed at; 0: vt_target).
constexpr uint32_t TUNE_BB = 5;  // block words: <= 4, <= 16, <= 64, <= 256, more
constexpr uint32_t TUNE_KB = 5;  // survivors: < 256, < 1024, < 4096, < 16384, more
constexpr uint32_t TUNE_CELLS = TUNE_BB * TUNE_KB;
__host__ __device__ inline uint32_t tune_cell(uint32_t block_words, uint32_t K)
{
    const uint32_t b = block_words <= 4u ? 0u : block_words <= 16u ? 1u : block_words <= 64u ? 2u
                       : block_words <= 256u ? 3u : 4u;
    const uint32_t k = K < 256u ? 0u : K < 1024u ? 1u : K < 4096u ? 2u : K < 16384u ? 3u : 4u;
    return b * TUNE_KB + k;
}

struct Knobs {
    uint32_t vt_target = 768;      // bitset count: workgroups aimed at per job per stop
    uint32_t vt_wave_k = 2048;     // bitset count: one wave per candidate below this
    uint32_t vt_tile_words = 16;   // bitset count: 64-row words per LDS tile at most
    uint32_t count_grid = 2048;    // workgroups launched for the count kernels
    uint32_t count_target = 2048;  // row-bitmap count: work items aimed at per job
    uint16_t cell_mode[TUNE_CELLS] = {};    // per-shape cells (see tune_cell)
    uint16_t cell_target[TUNE_CELLS] = {};
};
Knobs knobs();
int set_knob(const char *name, int64_t value);
__host__ __device__ inline uint32_t vert_tile_stride(uint32_t tw) { return tw | 1u; }

// Sort key of an itemset for the canonical result order (size, then the
// ascending item list, compared item by item): the size (31 standing for 31
// or more) in the top 5 bits of hi, then its first nine items, 12 bits each
// (items < MAX_ITEMS), four in hi and five in lo.  Keys compare as (hi, lo);
// two different itemsets with equal keys have 31 or more items or agree on
// their first nine, and need the full comparison.
__host__ __device__ inline void canon_key(const uint64_t *mask, uint32_t W, uint32_t k,
                                          unsigned long long *hi, unsigned long long *lo)
{
    unsigned long long h = (unsigned long long)(k < 31u ? k : 31u) << 59, l = 0;
    uint32_t n = 0;
    for (uint32_t w = 0; w < W && n < 9u; ++w) {
        uint64_t b = mask[w];
        while (b && n < 9u) {
            const unsigned long long item = w * 64u + (uint32_t)__builtin_ctzll(b);
            b &= b - 1;
            if (n < 4u)
                h |= item << (47u - 12u * n);
            else
                l |= item << (52u - 12u * (n - 4u));
            ++n;
        }
    }
    *hi = h;
    *lo = l;
}
static_assert(MAX_ITEMS <= 4096, "canon_key holds an item in 12 bits");
// a tile of capacity c holds nL1 rows of stride vert_tile_stride(vert_tile_words(nL1, ., c))
// whenever nL1 <= c: the count kernels' tile therefore covers any frequent-item count
static_assert(VT_WORDS >= MAX_ITEMS, "the count tile must hold one word of every item");

__host__ __device__ inline uint32_t row_tile_rows(uint32_t W)
{
    // rows staged per tile: 2W dword planes of r rows each
    uint32_t r = (uint32_t)(LDS_DWORDS / (2u * W));
    r = (r / 64u) * 64u;
    if (r > 64u * MAX_GROUPS)
        r = 64u * MAX_GROUPS;
    return r < 64u ? 64u : r;
}

// Standing of a pool itemset in one 32-bit word: its state in the low three
// bits and, above them, the index (epoch) of the stop that promoted it to a
// box (PROMO_NONE while it is a circle).  One word, so a reader in the same
// launch sees the state and its promotion stop together.
constexpr uint32_t PROMO_NONE = 0x1FFFFFFFu;
__host__ __device__ inline uint32_t standing(uint32_t state, uint32_t promo)
{
    return state | (promo << 3);
}
__host__ __device__ inline uint32_t standing_state(uint32_t w) { return w & 7u; }
__host__ __device__ inline uint32_t standing_promo(uint32_t w) { return w >> 3; }

// Mutable state of one mining run, updated only by kernels during a run.
// Stop e (epoch e, counted from 1) is one launch: it counts the survivors
// of stop e-1 (the current list) and the candidates made for stop e-1's new
// boxes on block e, prunes them, and appends its own survivors to the next
// list and its promotions to the next new-box list.
struct JobState {
    uint32_t done;      // no candidate left
    uint32_t overflow;  // candidate pool capacity exceeded
    uint32_t stop;      // block index 1..stop_max of the current stop (0 before the first)
    uint32_t epoch;     // index of the current stop (from 1); promotions are tagged with it
    uint32_t spare0, spare1;
    uint32_t k_cur;     // survivors of the last stop: the current list, counted at this one
    uint32_t pool_n;    // itemsets in the pool after the last stop (> cap: overflow)
    uint32_t nL1;       // frequent items
    uint32_t spare;
    uint32_t parity;    // 1: current list live1, last stop's new boxes newbox1; 0: the others
    uint32_t first;     // block [first, last) of this stop
    uint32_t last;
    uint32_t n_ct;      // count plan: candidate groups
    uint32_t n_ri;      //             row or tile chunks per group
    uint32_t rpi;       //             rows (row bitmaps) or tiles (bitsets) per chunk
    uint32_t peak_K;
    uint32_t asserts;   // invariant violations (must stay 0)
    unsigned long long tests;
    uint32_t fw, lw;    // bitsets: 64-row words [fw, lw] hold the block
    uint32_t tw;        // bitsets: words per tile
    uint32_t cpt;       // bitsets: candidates per thread
    uint32_t cmode;     // bitsets: 0 LDS tiles, 1 one wave per candidate
    uint32_t pool_base; // pool size when this stop began: entries at or above it
                        // were made at this stop for the last stop's new boxes
    uint32_t pending;   // added, its first stop not begun
    uint32_t need;      // stops the live set certainly still needs after this one
    uint32_t n_prev;    // boxes promoted at the last stop (extended at this one)
    uint32_t stops;     // stops completed
    uint32_t pad[2];
};
static_assert(sizeof(JobState) == 128, "JobState is read back as 128-byte records");

// Between chunks of stops a job is either pending (added, its first stop
// not begun; it runs if it has first candidates) or begun on its next stop.
inline bool job_running(const JobState &s, uint32_t)
{
    if (s.done || s.overflow)
        return false;
    return s.pending ? s.pool_n > 0 : true;
}
// Stops the job's live set certainly still needs.
inline uint32_t job_need(const JobState &s, uint32_t, uint32_t stop_max)
{
    return s.pending ? stop_max : s.need;
}

constexpr int KD = 16;  // frequent-item indices stored per candidate (larger: decode the mask)

// A live candidate travels between stops as a record in the live lists, so
// that a stop reads everything it needs of a candidate with one load: its
// pool entry, its support and the stops it has been counted on so far, its
// size and whether it is a box already, and (size <= KR) its frequent-item
// indices (larger itemsets' lists are read from the pool).  LREC uint4
// words: {p, supp, sc, k | box << 16}, then KR 16-bit items.
constexpr uint32_t LREC = 2;
constexpr int KR = 8;

// The counters that the workgroups of a stop's launch update with atomics
// live in lines of their own, 128 bytes apart, away from the job state that
// every work item reads (an atomic on a line holds up the reads of that
// line).  The stop's statistics are summed into CTR_LINES lines, each
// workgroup into the line of its index modulo CTR_LINES, so that no line
// takes the atomics of every workgroup; two more lines hold the list
// appends and the pool growth.  The serial part of the launch reads and
// clears them all.  Words of a statistics line:
constexpr uint32_t CTR_LINES = 8;
constexpr uint32_t CTR_STRIDE = 32;  // words between lines
// records appended to the next live list (low word) and to the next
// new-box list (high word) at this stop: one 64-bit word, so that a
// workgroup reserves both with one atomic
constexpr uint32_t CTR_APPEND = CTR_LINES * CTR_STRIDE;
// pool entries made at this stop (they follow pool_base)
constexpr uint32_t CTR_GEN = (CTR_LINES + 1) * CTR_STRIDE;
constexpr uint32_t CTR_TOTAL = (CTR_LINES + 2) * CTR_STRIDE;  // words
enum : uint32_t {
    CTR_WORDS = 0,   // nonzero mask dwords of the counted candidates (row bitmaps)
    CTR_ITEMS,       // items of the counted candidates
    CTR_PROMOTED,    // dashed circles promoted to boxes
    CTR_PRUNED,      // dashed circles erased by the upper bound
    CTR_SOLID,       // candidates that finished a full pass
    CTR_MAX_REM,     // most stops a kept candidate still needs (maximum)
    CTR_FIELDS
};

// Random word of item a for the Zobrist hash of an itemset, the XOR of its
// items' words (mining keys items by frequent-item index): output a + 1
// of the SplitMix64 generator (Steele, Lea & Flood, in Vigna's 64-bit form)
// from a fixed seed.  Computed in registers instead of read from a table.
__device__ __forceinline__ unsigned long long zob(uint32_t a)
{
    unsigned long long z = 0x5EED1812109590ull + (unsigned long long)(a + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Hash slot key: pool index in the high half, a 24-bit fingerprint and the
// itemset size (mod 256) in the low half.  Lookups of k-itemsets never match
// a slot of a (k+1)-itemset being inserted concurrently.
__device__ __forceinline__ uint32_t slot_tag(unsigned long long h, uint32_t k)
{
    return (uint32_t)(((h >> 40) & 0xFFFFFFull) << 8) | (k & 0xFFu);
}

// Read-only description of one mining run (device copy in a job table).
struct Job {
    const uint64_t *rows;  // n * W, row-major
    const uint64_t *vert;  // m * nw: bit r of vert[i * nw + g] = item i in row 64g + r
    uint64_t *fvert;       // nL1 * nw: the frequent items' rows of vert, in frequent-item
                           // order (vert itself when every item is frequent)
    uint32_t nw;           // 64-row words per item
    uint32_t layout;       // LAYOUT_ROWS or LAYOUT_VERTICAL counting
    uint32_t *l1pos;       // m: index of an item among the frequent items (or ~0)
    uint32_t n, m, W, Mp;
    uint32_t stop_max, tau;
    uint32_t cap;    // pool capacity (itemsets)
    uint32_t hmask;  // hash slots - 1
    uint64_t *pmask;  // cap * W
    uint16_t *pitems; // cap * KD: frequent-item indices of each itemset (size <= KD)
    unsigned long long *phash;  // Zobrist hash of each itemset
    uint64_t *pnz;    // bitmap of nonzero words
    uint32_t *psupp, *pk;
    uint32_t *pstate;           // standing word (state, promotion stop) of each itemset
    unsigned long long *slots;  // open addressing: idx<<32 | fp24<<8 | k8
    uint4 *live0, *live1;       // cap records each (LREC uint4 words per record)
    unsigned long long *pcnt;   // cap: count | arrivals << 32 of a split group (zero between stops)
    uint32_t *ctrs;             // CTR_TOTAL: the stop's counters (zero between stops)
    uint32_t *newbox0, *newbox1;  // cap each: boxes promoted at a stop (by parity)
    uint32_t *l1;               // m
    uint32_t *item_cnt;         // m
    dic_stop_trace *trace;
    uint32_t trace_cap;
    uint32_t classic;  // classic DIC start (Algorithm 1): 1-itemsets are pool entries 0..m-1
    JobState *st;
    uint64_t *out_mask;   // collect: cap * W
    uint32_t *out_cnt;    // cap
    unsigned long long *out_key;  // cap * 2: canon_key of each collected itemset
    uint32_t *out_n;      // 1
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Bump carving of one buffer into 256-byte aligned parts.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    }
};

// Candidate capacity of a job's pool: four times the pairs of its frequent
// items plus room for larger itemsets, times mult after overflows.
inline uint64_t pool_cap_for(uint32_t nL1, uint32_t mult)
{
    const uint64_t nC2 = (uint64_t)nL1 * (nL1 ? nL1 - 1u : 0u) / 2u;
    const uint64_t c = 4 * nC2 + 16384;
    return (c > 16384 ? c : 16384) * mult;
}

// Layout of a job's candidate pool buffer (byte offsets of its arrays).
struct PoolLayout {
    size_t mask, items, hash, nz, supp, state, k, slots, live0, live1, pcnt, ctrs, newbox0,
        newbox1, omask, ocnt, okey;
    size_t bytes;
    uint64_t hslots;
    PoolLayout(uint64_t cap, uint32_t W)
    {
        hslots = next_pow2(2 * cap);
        Carver c;
        mask = c.take(cap * W * 8);
        items = c.take(cap * KD * 2);
        hash = c.take(cap * 8);
        nz = c.take(cap * 8);
        supp = c.take(cap * 4);
        state = c.take(cap * 4);
        k = c.take(cap * 4);
        slots = c.take(hslots * 8);
        live0 = c.take(cap * LREC * 16);
        live1 = c.take(cap * LREC * 16);
        pcnt = c.take(cap * 8);
        ctrs = c.take(CTR_TOTAL * 4);
        newbox0 = c.take(cap * 4);
        newbox1 = c.take(cap * 4);
        omask = c.take(cap * W * 8);
        ocnt = c.take(cap * 4);
        okey = c.take(cap * 16);
        bytes = c.off;
    }
};

// Work plan of one step across all jobs (prefix sums, njobs + 1 entries).
struct Plan {
    uint32_t njobs;
    uint32_t total_v;               // pre_countv[njobs]: survivors' work items of the stop kernel
    unsigned long long total_cg;    // pre_cg[njobs]: MakeCandidates chunks
    uint32_t *pre_count;   // row-bitmap count work items (k_count)
    uint32_t *pre_countv;  // survivors' work items of the stop kernel
    unsigned long long *pre_cg;
    unsigned long long *pre_fp;  // first pass row chunks
    uint32_t vt_target, vt_wave_k, vt_tile_words, count_target;  // see Knobs
    uint32_t *tickets;  // arrival counters of candidate generation (zero between launches)
    uint16_t cell_mode[TUNE_CELLS], cell_target[TUNE_CELLS];  // see Knobs
};
// arrival counters: a root and TICKET_GROUPS group counters, TICKET_STRIDE
// words apart so that no two share a cache line
constexpr uint32_t TICKET_GROUPS = 32;
constexpr uint32_t TICKET_STRIDE = 64;
constexpr uint32_t TICKET_WORDS = (TICKET_GROUPS + 1) * TICKET_STRIDE;

// Point job J's pool arrays into base (laid out by L, capacity cap).
inline void pool_assign(Job &J, const PoolLayout &L, char *b, uint32_t cap)
{
    J.cap = cap;
    J.hmask = (uint32_t)(L.hslots - 1);
    J.pmask = (uint64_t *)(b + L.mask);
    J.pitems = (uint16_t *)(b + L.items);
    J.phash = (unsigned long long *)(b + L.hash);
    J.pnz = (uint64_t *)(b + L.nz);
    J.psupp = (uint32_t *)(b + L.supp);
    J.pstate = (uint32_t *)(b + L.state);
    J.pk = (uint32_t *)(b + L.k);
    J.slots = (unsigned long long *)(b + L.slots);
    J.live0 = (uint4 *)(b + L.live0);
    J.live1 = (uint4 *)(b + L.live1);
    J.pcnt = (unsigned long long *)(b + L.pcnt);
    J.ctrs = (uint32_t *)(b + L.ctrs);
    J.newbox0 = (uint32_t *)(b + L.newbox0);
    J.newbox1 = (uint32_t *)(b + L.newbox1);
    J.out_mask = (uint64_t *)(b + L.omask);
    J.out_cnt = (uint32_t *)(b + L.ocnt);
    J.out_key = (unsigned long long *)(b + L.okey);
}

// kernel launchers (dic_kernels.hip)
void launch_first_pass(const Job *jobs, const Plan *plan, unsigned long long total_chunks,
                       hipStream_t s);
void launch_first_pass_vert(const Job *jobs, const Plan *plan, unsigned long long total_chunks,
                            hipStream_t s);
void launch_transpose(const uint64_t *rows, uint64_t n, uint32_t m, uint64_t *vert, uint32_t nw,
                      hipStream_t s);
void launch_l1_and_pairs_prepare(const Job *jobs, const Plan *plan, uint32_t njobs, hipStream_t s);
void launch_init_pairs(const Job *jobs, const Plan *plan, unsigned long long total, hipStream_t s);
void launch_gather_vert(const Job *jobs, const Plan *plan, unsigned long long total, hipStream_t s);
// Begin the next stop for newly added jobs and plan every job's work (once
// per chunk of stops; later stops are begun by candidate generation).
void launch_begin(const Job *jobs, Plan *plan, hipStream_t s);
// One stop for every job in the table; when given, the two events bracket
// the CountSupport launch on stream s.
void launch_step(const Job *jobs, const Plan *plan, hipStream_t s, bool rows, bool vert,
                 uint32_t count_grid, hipEvent_t before = nullptr, hipEvent_t after = nullptr);
void launch_collect(const Job *jobs, const Plan *plan, uint32_t njobs, hipStream_t s);
void launch_fill32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s);
void launch_pack_lists(const uint32_t *items, const uint64_t *offsets, uint64_t n, uint32_t W,
                       uint64_t *rows, hipStream_t s);
void launch_check_padding(const uint64_t *rows, uint64_t n, uint32_t m, uint32_t *bad,
                          hipStream_t s);

// ---------------------------------------------------------------------------
// host side (dic_engine.hip / dic_api.hip)
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

void *dev_alloc(size_t bytes);
void dev_free(void *p);
hipStream_t lib_stream();

struct MineRequest {
    const uint64_t *rows;  // device, row-major
    const uint64_t *vert;  // device, item bitsets (m * ceil(n/64) words)
    uint32_t n, m;
    double minsup;
    uint64_t M;
    // a rerun after candidate-pool overflows: the pool multiplier, the
    // restarts so far and the count time of the earlier attempts
    uint32_t mult = 1, restarts = 0;
    double count_ms = 0;
    uint64_t count_launches = 0;
};

struct MineOutput {
    int status = 0;
    std::vector<uint64_t> masks;
    std::vector<uint32_t> counts;
    std::vector<dic_stop_trace> trace;
    dic_stats stats{};
    // an engine in requeue mode hands an overflowed job back instead of
    // rerunning it: `again` is the request to add once its memory is granted
    bool requeue = false;
    MineRequest again{};
};

// Compute tau from minsup; returns false on invalid minsup.
bool threshold(double minsup, uint64_t n, uint64_t *tau);

// Mine every request together (one launch per kernel per stop) on a pooled
// engine; stream is made to wait for the run's completion (nullptr: none).
int run_jobs(const std::vector<MineRequest> &reqs, std::vector<MineOutput> &outs,
             hipStream_t stream);
bool use_graphs();
void set_use_graphs(bool on);
// Test aid: when nonzero, every job buffer (pool, per-item records,
// frequent-item bitsets, trace) is filled with this byte value on
// allocation, so that a read of memory the run has not written yet gives a
// value from the fill instead of from whatever a previous job left there.
int poison();
void set_poison(int byte);

// Bytes the library's allocator sets aside for a request of b bytes.
inline uint64_t alloc_bytes(uint64_t b)
{
    if (b <= (1u << 20))
        return (b + 4095) & ~(uint64_t)4095;
    return (b + (2u << 20) - 1) & ~(uint64_t)((2u << 20) - 1);
}
// Most stops a run can take: a candidate is counted for one full pass
// (stop_max stops); a candidate of size k+1 is made at the latest one stop
// after its last k-subset ends its pass, so size-k candidates are done
// within k * (stop_max + 1) stops; and a candidate of size k has all its
// 2^k - 2 proper nonempty subsets frequent, those of size >= 2 (all of them
// in the classic start) in the pool with it, so k <= log2(cap) + 1.
uint64_t trace_bound(uint64_t n, uint64_t M, uint64_t cap);
// Upper bound of a job's device memory before its first pass (every item
// frequent), for a pool of pool_cap_for(m, mult): the pool, the per-item
// records, the frequent items' bitsets and the trace at its largest (twice:
// the old and new buffer while it grows), each as the allocator rounds it.
uint64_t job_bytes_bound(uint32_t m, uint64_t n, uint64_t M, uint32_t mult);

bool profiling();
void set_profiling(int on);
uint32_t count_layout();
void set_count_layout(uint32_t layout);
uint32_t init_mode();
void set_init_mode(uint32_t mode);

struct ActiveJob;

// A set of jobs mined together on one stream.  Jobs can be added between
// step chunks (their first pass runs at once); every advance() runs up to
// max_steps stops for all unfinished jobs with one launch per kernel per
// stop; harvest() hands back finished jobs and releases their memory.  A
// job whose candidate pool overflowed is restarted with 16 times the room
// (or handed back for that, in requeue mode).
// Not thread-safe: one owner thread.
class Engine {
  public:
    // s: the stream to run on; nullptr makes a private one (needed for
    // graph capture, which must not see other threads' work).
    Engine(hipStream_t s, uint32_t max_jobs);
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;

    int add(const std::vector<MineRequest> &reqs, const std::vector<uint64_t> &ids);
    int advance(uint32_t max_steps);
    int harvest(std::vector<std::pair<uint64_t, MineOutput>> &done);
    size_t size() const { return jobs_.size(); }
    bool running() const;
    // Requeue mode (serving): harvest hands an overflowed job back with
    // MineOutput::requeue set instead of rerunning it with a larger pool,
    // so that its owner can grant the larger memory first.
    void set_requeue(bool on) { requeue_ = on; }

  private:
    int add_internal(std::vector<ActiveJob *> &fresh);
    int add_impl(std::vector<ActiveJob *> &fresh);
    int read_states();
    int upload_table();
    bool knobs_changed() const;
    int ensure_trace(uint32_t steps);
    int collect(std::vector<ActiveJob *> &fin, std::vector<std::pair<uint64_t, MineOutput>> &out);
    int launch_steps(uint32_t S, bool rows, bool vert, bool prof, double *count_ms,
                     uint32_t *steps_done);

    hipStream_t s_;
    bool own_stream_ = false;
    hipGraphExec_t graphs_[2][2] = {};  // [rows][vert]
    uint32_t graph_grid_[2][2] = {};    // count grid each graph was captured with
    uint32_t max_jobs_;
    std::vector<ActiveJob *> jobs_;
    std::vector<int> free_slots_;
    void *slab_ = nullptr;       // JobState[max_jobs] + out_n[max_jobs]
    void *table_ = nullptr;      // Job[max_jobs] for the step kernels
    void *table_aux_ = nullptr;  // Job[max_jobs] for first pass / collection
    void *plan_buf_ = nullptr;   // two Plans and their prefix arrays
    Plan *d_plan_step_ = nullptr, *d_plan_aux_ = nullptr;
    Plan plan_step_{}, plan_aux_{};
    std::vector<JobState> st_;   // host copy of the slab
    std::vector<Job> table_host_, aux_host_;
    std::vector<unsigned long long> pre_host_;
    std::vector<unsigned long long> fp_host_;  // prefix of the frequent-item bitset gather
    void *pinned_ = nullptr;  // pinned host staging of finished jobs' outputs
    size_t pinned_cap_ = 0;
    bool table_dirty_ = true;
    bool requeue_ = false;
    std::vector<hipEvent_t> events_;
    std::vector<float> launch_ms_;  // per launch of the last profiled chunk
};

}  // namespace dic

struct dic_result {
    uint32_t W;
    std::vector<uint64_t> masks;
    std::vector<uint32_t> counts;
    std::vector<dic_stop_trace> trace;
    dic_stats stats;
};
