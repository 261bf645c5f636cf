// Association rules from frequent itemsets, on the device.
//
// Rule generation is the second subtask of association rule mining named in
// Section 1; the rule X => I \ X and its confidence supp(I) / supp(X) follow
// the paper's reference [1].  For every itemset I with |I| >= 2 every
// nonempty proper subset X is a candidate antecedent; X is frequent by
// downward closure, so its support is a lookup in the itemset table.
//
// Work is split into chunks of WG subset codes of one itemset (bit t of a
// code selects the t-th smallest item of I).  Two passes over the same
// chunks: the first counts the kept rules per chunk, the host turns the
// counts into offsets, the second writes every kept rule at its offset, so
// the output is in (itemset, code) order without a sort.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dic_internal.h"

struct dic_rules_result {
    uint32_t W = 0;
    std::vector<uint32_t> itemset, code, supp_x;
    std::vector<uint64_t> ante, cons;
    dic_rules_stats stats{};
};

namespace dic {

namespace {

constexpr uint32_t RULES_KMAX = DIC_RULES_KMAX;

struct RulesArgs {
    const uint64_t *masks;            // q * W
    const uint32_t *counts;           // q
    uint16_t *items;                  // q * RULES_KMAX: ascending item indices
    uint32_t *k;                      // q: itemset sizes
    unsigned long long *slots;        // open addressing: idx<<32 | fp24<<8 | k8
    uint32_t hmask;
    uint32_t W;
    uint64_t q;
    const unsigned long long *pre;    // q + 1: prefix of chunks per itemset
    unsigned long long chunks;        // pre[q]
    uint32_t *chunk_kept;             // chunks: kept rules (first pass)
    const unsigned long long *chunk_off;  // chunks: output offsets (second pass)
    uint32_t *missing;                // set when a subset is not among the itemsets
    double minconf;
    uint32_t *o_itemset, *o_code, *o_supp;
    uint64_t *o_ante, *o_cons;        // R * W each
};

__device__ __forceinline__ uint32_t find_itemset(const unsigned long long *pre, uint64_t q,
                                                 unsigned long long x)
{
    uint64_t lo = 0, hi = q;  // largest i with pre[i] <= x
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (pre[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

// Item lists, sizes and the hash table of all itemsets.  One thread per
// itemset.
__global__ __launch_bounds__(WG) void k_rules_index(RulesArgs a)
{
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= a.q)
        return;
    const uint64_t *I = a.masks + i * a.W;
    uint16_t *it = a.items + i * RULES_KMAX;
    uint32_t k = 0;
    unsigned long long h = 0;
    for (uint32_t w = 0; w < a.W; ++w) {
        uint64_t bits = I[w];
        while (bits) {
            const uint32_t p = w * 64u + (uint32_t)__builtin_ctzll(bits);
            bits &= bits - 1;
            if (k < RULES_KMAX)
                it[k] = (uint16_t)p;
            ++k;
            h ^= zob(p);
        }
    }
    a.k[i] = k;
    const unsigned long long v = ((unsigned long long)i << 32) | slot_tag(h, k);
    uint32_t s = (uint32_t)h & a.hmask;
    for (;;) {
        if (atomicCAS(a.slots + s, SLOT_EMPTY, v) == SLOT_EMPTY)
            return;
        s = (s + 1u) & a.hmask;
    }
}

// Support of the subset of itemset i selected by code, or NONE_U32 when it is
// not an itemset of the table.  An entry matches when its size equals the
// subset's and it holds every selected item.
constexpr uint32_t NONE_U32 = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t subset_support(const RulesArgs &a, const uint16_t *it,
                                                   uint32_t k, uint32_t code)
{
    unsigned long long h = 0;
    uint32_t kx = 0;
    for (uint32_t t = 0; t < k; ++t)
        if ((code >> t) & 1u) {
            h ^= zob(it[t]);
            ++kx;
        }
    const uint32_t tag = slot_tag(h, kx);
    uint32_t s = (uint32_t)h & a.hmask;
    for (;;) {
        const unsigned long long v = a.slots[s];
        if (v == SLOT_EMPTY)
            return NONE_U32;
        if ((uint32_t)v == tag) {
            const uint32_t idx = (uint32_t)(v >> 32);
            const uint64_t *E = a.masks + (uint64_t)idx * a.W;
            bool all = true;
            for (uint32_t t = 0; t < k && all; ++t)
                if ((code >> t) & 1u)
                    all = (E[it[t] >> 6] >> (it[t] & 63u)) & 1ull;
            if (all)
                return a.counts[idx];
        }
        s = (s + 1u) & a.hmask;
    }
}

// One chunk of one itemset: this thread's split and whether its rule is kept.
struct Split {
    uint32_t i, k, code, sx;
    bool kept;
};

__device__ __forceinline__ Split split_of(const RulesArgs &a, unsigned long long chunk)
{
    Split r;
    r.i = find_itemset(a.pre, a.q, chunk);
    r.k = a.k[r.i];
    const unsigned long long c = (chunk - a.pre[r.i]) * WG + threadIdx.x + 1ull;
    const unsigned long long full = (1ull << r.k) - 1ull;
    r.code = (uint32_t)c;
    r.sx = 0;
    r.kept = false;
    if (c < full) {
        r.sx = subset_support(a, a.items + (uint64_t)r.i * RULES_KMAX, r.k, r.code);
        if (r.sx == NONE_U32)
            atomicOr(a.missing, 1u);
        else
            r.kept = (double)a.counts[r.i] >= a.minconf * (double)r.sx;
    }
    return r;
}

// First pass: kept rules per chunk.
__global__ __launch_bounds__(WG) void k_rules_count(RulesArgs a)
{
    __shared__ uint32_t sh[WG / 64];
    for (unsigned long long ch = blockIdx.x; ch < a.chunks; ch += gridDim.x) {
        const Split r = split_of(a, ch);
        const uint32_t n = (uint32_t)__popcll(__ballot(r.kept));
        if ((threadIdx.x & 63u) == 0)
            sh[threadIdx.x >> 6] = n;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < WG / 64; ++w)
                t += sh[w];
            a.chunk_kept[ch] = t;
        }
        __syncthreads();
    }
}

// Second pass: every kept rule at its offset (chunk offset + rank in chunk).
__global__ __launch_bounds__(WG) void k_rules_write(RulesArgs a)
{
    __shared__ uint32_t sh[WG / 64];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (unsigned long long ch = blockIdx.x; ch < a.chunks; ch += gridDim.x) {
        const Split r = split_of(a, ch);
        const unsigned long long b = __ballot(r.kept);
        if (lane == 0)
            sh[wave] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t before = 0;
        for (uint32_t w = 0; w < wave; ++w)
            before += sh[w];
        __syncthreads();
        if (r.kept) {
            const uint64_t lanes_below = lane ? (~0ull >> (64u - lane)) : 0ull;
            const unsigned long long o =
                a.chunk_off[ch] + before + (uint32_t)__popcll(b & lanes_below);
            a.o_itemset[o] = r.i;
            a.o_code[o] = r.code;
            a.o_supp[o] = r.sx;
            const uint16_t *it = a.items + (uint64_t)r.i * RULES_KMAX;
            const uint64_t *I = a.masks + (uint64_t)r.i * a.W;
            for (uint32_t w = 0; w < a.W; ++w) {
                uint64_t x = 0;
                for (uint32_t t = 0; t < r.k; ++t)
                    if (((r.code >> t) & 1u) && (it[t] >> 6) == w)
                        x |= 1ull << (it[t] & 63u);
                a.o_ante[o * a.W + w] = x;
                a.o_cons[o * a.W + w] = I[w] & ~x;
            }
        }
    }
}

// Device buffers of one call, released together.
struct Buffers {
    std::vector<void *> p;
    void *get(size_t bytes)
    {
        void *x = dev_alloc(bytes ? bytes : 8);
        if (x)
            p.push_back(x);
        return x;
    }
    ~Buffers()
    {
        for (void *x : p)
            dev_free(x);
    }
};

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t v = 1;
    while (v < x)
        v <<= 1;
    return v;
}

#define RULES_TRY(x)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            set_error(std::string(#x) + " failed: " + hipGetErrorString(e_));             \
            return DIC_E_DEVICE;                                                          \
        }                                                                                 \
    } while (0)

int rules_run(const uint64_t *masks, const uint32_t *counts, uint64_t q, uint32_t W,
              double minconf, dic_rules_result *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    out->W = W;
    out->stats.itemsets = q;
    if (q == 0)
        return DIC_OK;
    // sizes, split counts and chunk prefix on the host
    std::vector<unsigned long long> pre(q + 1, 0);
    uint64_t splits = 0;
    for (uint64_t i = 0; i < q; ++i) {
        uint32_t k = 0;
        for (uint32_t w = 0; w < W; ++w)
            k += (uint32_t)__builtin_popcountll(masks[i * W + w]);
        if (k > RULES_KMAX) {
            set_error("dic_rules: itemset " + std::to_string(i) + " has " + std::to_string(k) +
                      " items (more than " + std::to_string(RULES_KMAX) + ")");
            return DIC_E_INVAL;
        }
        const uint64_t s = k >= 2 ? (1ull << k) - 2ull : 0ull;
        splits += s;
        pre[i + 1] = pre[i] + (s + WG - 1) / WG;
    }
    out->stats.splits = splits;
    const unsigned long long chunks = pre[q];
    hipStream_t st = lib_stream();
    Buffers B;
    RulesArgs a{};
    a.W = W;
    a.q = q;
    a.minconf = minconf;
    a.chunks = chunks;
    const uint64_t hslots = pow2_at_least(2 * q);
    a.hmask = (uint32_t)(hslots - 1);
    auto *d_masks = (uint64_t *)B.get(8ull * q * W);
    auto *d_counts = (uint32_t *)B.get(4ull * q);
    a.items = (uint16_t *)B.get(2ull * q * RULES_KMAX);
    a.k = (uint32_t *)B.get(4ull * q);
    a.slots = (unsigned long long *)B.get(8ull * hslots);
    auto *d_pre = (unsigned long long *)B.get(8ull * (q + 1));
    a.chunk_kept = (uint32_t *)B.get(4ull * chunks);
    auto *d_off = (unsigned long long *)B.get(8ull * chunks);
    a.missing = (uint32_t *)B.get(4);
    if (!d_masks || !d_counts || !a.items || !a.k || !a.slots || !d_pre || !a.chunk_kept ||
        !d_off || !a.missing) {
        set_error("dic_rules: device allocation failed");
        return DIC_E_NOMEM;
    }
    a.masks = d_masks;
    a.counts = d_counts;
    a.pre = d_pre;
    a.chunk_off = d_off;
    RULES_TRY(hipMemcpyAsync(d_masks, masks, 8ull * q * W, hipMemcpyHostToDevice, st));
    RULES_TRY(hipMemcpyAsync(d_counts, counts, 4ull * q, hipMemcpyHostToDevice, st));
    RULES_TRY(hipMemcpyAsync(d_pre, pre.data(), 8ull * (q + 1), hipMemcpyHostToDevice, st));
    RULES_TRY(hipMemsetAsync(a.slots, 0xFF, 8ull * hslots, st));
    RULES_TRY(hipMemsetAsync(a.missing, 0, 4, st));
    struct Events {
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t x : e)
                if (x)
                    (void)hipEventDestroy(x);
        }
    } ev;
    for (hipEvent_t &x : ev.e)
        RULES_TRY(hipEventCreate(&x));
    hipEvent_t e0 = ev.e[0], e1 = ev.e[1], e2 = ev.e[2], e3 = ev.e[3];
    const uint32_t grid_q = (uint32_t)((q + WG - 1) / WG);
    const uint32_t grid_c = (uint32_t)std::min<unsigned long long>(chunks ? chunks : 1, 65536);
    RULES_TRY(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_rules_index, dim3(grid_q), dim3(WG), 0, st, a);
    if (chunks)
        hipLaunchKernelGGL(k_rules_count, dim3(grid_c), dim3(WG), 0, st, a);
    RULES_TRY(hipGetLastError());
    RULES_TRY(hipEventRecord(e1, st));
    std::vector<uint32_t> kept(chunks);
    uint32_t missing = 0;
    if (chunks)
        RULES_TRY(hipMemcpyAsync(kept.data(), a.chunk_kept, 4ull * chunks, hipMemcpyDeviceToHost,
                                 st));
    RULES_TRY(hipMemcpyAsync(&missing, a.missing, 4, hipMemcpyDeviceToHost, st));
    RULES_TRY(hipStreamSynchronize(st));
    if (missing) {
        set_error("dic_rules: a subset of an itemset is not among the itemsets (input is not "
                  "downward closed)");
        return DIC_E_INVAL;
    }
    std::vector<unsigned long long> off(chunks);
    unsigned long long R = 0;
    for (unsigned long long c = 0; c < chunks; ++c) {
        off[c] = R;
        R += kept[c];
    }
    out->stats.rules = R;
    float ms1 = 0, ms2 = 0;
    RULES_TRY(hipEventElapsedTime(&ms1, e0, e1));
    if (R) {
        a.o_itemset = (uint32_t *)B.get(4ull * R);
        a.o_code = (uint32_t *)B.get(4ull * R);
        a.o_supp = (uint32_t *)B.get(4ull * R);
        a.o_ante = (uint64_t *)B.get(8ull * R * W);
        a.o_cons = (uint64_t *)B.get(8ull * R * W);
        if (!a.o_itemset || !a.o_code || !a.o_supp || !a.o_ante || !a.o_cons) {
            set_error("dic_rules: device allocation failed (output)");
            return DIC_E_NOMEM;
        }
        out->itemset.resize(R);
        out->code.resize(R);
        out->supp_x.resize(R);
        out->ante.resize(R * W);
        out->cons.resize(R * W);
        RULES_TRY(hipMemcpyAsync(d_off, off.data(), 8ull * chunks, hipMemcpyHostToDevice, st));
        RULES_TRY(hipEventRecord(e2, st));
        hipLaunchKernelGGL(k_rules_write, dim3(grid_c), dim3(WG), 0, st, a);
        RULES_TRY(hipGetLastError());
        RULES_TRY(hipEventRecord(e3, st));
        RULES_TRY(hipMemcpyAsync(out->itemset.data(), a.o_itemset, 4ull * R,
                                 hipMemcpyDeviceToHost, st));
        RULES_TRY(hipMemcpyAsync(out->code.data(), a.o_code, 4ull * R, hipMemcpyDeviceToHost, st));
        RULES_TRY(hipMemcpyAsync(out->supp_x.data(), a.o_supp, 4ull * R, hipMemcpyDeviceToHost,
                                 st));
        RULES_TRY(hipMemcpyAsync(out->ante.data(), a.o_ante, 8ull * R * W, hipMemcpyDeviceToHost,
                                 st));
        RULES_TRY(hipMemcpyAsync(out->cons.data(), a.o_cons, 8ull * R * W, hipMemcpyDeviceToHost,
                                 st));
        RULES_TRY(hipStreamSynchronize(st));
        RULES_TRY(hipEventElapsedTime(&ms2, e2, e3));
    }
    out->stats.kernel_ms = (double)ms1 + (double)ms2;
    out->stats.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return DIC_OK;
}

}  // namespace

}  // namespace dic

using namespace dic;

extern "C" {

int dic_rules_from_arrays(const uint64_t *masks, const uint32_t *counts, uint64_t q, uint32_t W,
                          double minconf, dic_rules_result **out)
{
    if (!out) {
        set_error("dic_rules: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    if (W == 0 || W > MAX_ITEMS / 64 || (q && (!masks || !counts)) || minconf != minconf) {
        set_error("dic_rules: need 1 <= W <= 64, itemset arrays, and a minconf that is a number");
        return DIC_E_INVAL;
    }
    if (q > 0xFFFFFFFFull) {
        set_error("dic_rules: more than 2^32 - 1 itemsets");
        return DIC_E_INVAL;
    }
    auto *r = new (std::nothrow) dic_rules_result;
    if (!r) {
        set_error("dic_rules: host allocation failed");
        return DIC_E_NOMEM;
    }
    const int rc = rules_run(masks, counts, q, W, minconf, r);
    if (rc) {
        delete r;
        return rc;
    }
    *out = r;
    return DIC_OK;
}

int dic_rules(const dic_result *res, double minconf, dic_rules_result **out)
{
    if (!res) {
        if (out)
            *out = nullptr;
        set_error("dic_rules: result is NULL");
        return DIC_E_INVAL;
    }
    return dic_rules_from_arrays(res->masks.empty() ? nullptr : res->masks.data(),
                                 res->counts.empty() ? nullptr : res->counts.data(),
                                 res->counts.size(), res->W, minconf, out);
}

uint64_t dic_rules_size(const dic_rules_result *r) { return r ? r->itemset.size() : 0; }
uint32_t dic_rules_words(const dic_rules_result *r) { return r ? r->W : 0; }
const uint32_t *dic_rules_itemset(const dic_rules_result *r)
{
    return r && !r->itemset.empty() ? r->itemset.data() : nullptr;
}
const uint32_t *dic_rules_code(const dic_rules_result *r)
{
    return r && !r->code.empty() ? r->code.data() : nullptr;
}
const uint32_t *dic_rules_supp_x(const dic_rules_result *r)
{
    return r && !r->supp_x.empty() ? r->supp_x.data() : nullptr;
}
const uint64_t *dic_rules_antecedent(const dic_rules_result *r)
{
    return r && !r->ante.empty() ? r->ante.data() : nullptr;
}
const uint64_t *dic_rules_consequent(const dic_rules_result *r)
{
    return r && !r->cons.empty() ? r->cons.data() : nullptr;
}
int dic_rules_stats_of(const dic_rules_result *r, dic_rules_stats *s)
{
    if (!r || !s) {
        set_error("dic_rules_stats_of: NULL argument");
        return DIC_E_INVAL;
    }
    *s = r->stats;
    return DIC_OK;
}
void dic_rules_free(dic_rules_result *r) { delete r; }

}  // extern "C"
