// HIP kernels for Dynamic Itemset Counting on gfx950.
//
// Every kernel works on a table of jobs (one job = one database being mined)
// so that the single-database path and the batched path are the same code:
// a step launches each kernel once for all jobs, and each workgroup or wave
// locates its job by binary search over per-job prefix sums of work.
//
// Per stop (the loop body of Algorithm 2, Section 4.2), one launch:
//   k_stop      MakeCandidates for the last stop's new boxes, with the new
//               candidates' CountSupport (Algorithm 3) on this stop's block
//               and their Prune (Algorithm 4) and CheckFullPass (Algorithm 5)
//               in the workgroup that made them; in other workgroups the
//               last stop's survivors are counted on the block and pruned
//               (k_count counts row-bitmap jobs just before); the last
//               workgroup completes the stop and begins the next one
// k_begin starts a chunk of stops: newly added jobs move to their first
// block, and every job is planned for the current job table.
// Before the loop: k_first_pass and k_l1 (FirstPass: item supports, the
// frequent items), k_init_pairs (pairs of frequent items as candidates),
// k_gather_vert (the frequent items' bitsets in frequent-item order).
// After it: k_collect gathers the solid boxes with their sort keys.
#include "dic_internal.h"

namespace dic {

namespace {

constexpr uint32_t FP_ROWS = 4096;       // first pass rows per workgroup item
constexpr uint32_t FPV_WORDS = 4096;     // first pass (bitsets): words per work item
static_assert(FPV_WORDS % WG == 0, "first-pass chunks are whole loads per thread");
constexpr int VT_CPT = 4;                // bitset count: candidates per thread at most
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int ZP = 2;                    // row-bitmap survivors pruned per thread

// s_waitcnt operand (gfx9 encoding) that waits for every outstanding vector
// memory operation of the wave -- loads, stores and atomics -- and for
// nothing else: vmcnt 0, expcnt 7, lgkmcnt 15.
constexpr int WAIT_VM0 = 0x0F70;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ unsigned long long lanemask_lt()
{
    uint32_t l = lane_id();
    return l ? (~0ull >> (64u - l)) : 0ull;
}

// Largest j with pre[j] <= x, given pre[0] <= x < pre[njobs].
template <typename T>
__device__ __forceinline__ uint32_t find_job(const T *pre, uint32_t njobs, T x)
{
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1u) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Wave-aggregated counter increment: one atomic per wave when every lane
// targets the same counter, per-lane atomics otherwise.  All lanes call.
__device__ __forceinline__ uint32_t wave_append(uint32_t *ctr, bool pred, bool uniform)
{
    if (uniform) {
        unsigned long long b = __ballot(pred);
        uint32_t base = 0;
        if (b) {
            int leader = __ffsll((long long)b) - 1;
            if ((int)lane_id() == leader)
                base = atomicAdd(ctr, (uint32_t)__popcll(b));
            base = (uint32_t)__shfl((int)base, leader);
        }
        return base + (uint32_t)__popcll(b & lanemask_lt());
    }
    return pred ? atomicAdd(ctr, 1u) : 0u;
}

// A candidate's frequent-item indices (ascending, KD x u16) as 8 words.
__device__ __forceinline__ void load_items(const uint16_t *pi, uint32_t w[KD / 2])
{
    const uint4 *q = (const uint4 *)pi;
    const uint4 h0 = q[0], h1 = q[1];
    w[0] = h0.x; w[1] = h0.y; w[2] = h0.z; w[3] = h0.w;
    w[4] = h1.x; w[5] = h1.y; w[6] = h1.z; w[7] = h1.w;
}
// Item t of such a list (t must be a compile-time constant after unrolling,
// so the list stays in registers).
__device__ __forceinline__ uint32_t item_at(const uint32_t w[KD / 2], int t)
{
    return (w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
}

// Read a hash slot.  Slots are filled by device-scope atomics, possibly
// from another XCD, so the read is a device-scope atomic too (a plain load
// may be served by a stale copy in this XCD's L2).
__device__ __forceinline__ unsigned long long slot_read(const Job *J, uint32_t s)
{
    return __hip_atomic_load(J->slots + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void hash_insert(const Job *J, unsigned long long h, uint32_t k,
                                            uint32_t idx)
{
    unsigned long long v = ((unsigned long long)idx << 32) | slot_tag(h, k);
    uint32_t s = (uint32_t)h & J->hmask;
    for (;;) {
        unsigned long long old = atomicCAS(J->slots + s, SLOT_EMPTY, v);
        if (old == SLOT_EMPTY)
            return;
        s = (s + 1u) & J->hmask;
    }
}

// Pool index of the itemset (S | {i}) \ {x} with hash h and size k, or NONE.
// Only itemsets that existed when the stop began (index < base) are
// considered: one created by this stop's candidate generation is a fresh
// circle, never the box being looked for, and its pool entry may still be
// in flight from another workgroup, so it is skipped without being read.
__device__ __forceinline__ uint32_t hash_find_sub(const Job *J, unsigned long long h, uint32_t k,
                                                  const uint64_t *S, uint32_t i, uint32_t x,
                                                  uint32_t base)
{
    const uint32_t tag = slot_tag(h, k);
    const uint32_t W = J->W;
    uint32_t s = (uint32_t)h & J->hmask;
    for (;;) {
        const unsigned long long v = slot_read(J, s);
        if (v == SLOT_EMPTY)
            return NONE;
        if ((uint32_t)v == tag && (uint32_t)(v >> 32) < base) {
            uint32_t idx = (uint32_t)(v >> 32);
            const uint64_t *P = J->pmask + (uint64_t)idx * W;
            bool eq = true;
            for (uint32_t w = 0; w < W && eq; ++w) {
                uint64_t e = S[w];
                if (w == (i >> 6))
                    e |= 1ull << (i & 63u);
                if (w == (x >> 6))
                    e &= ~(1ull << (x & 63u));
                eq = P[w] == e;
            }
            if (eq)
                return idx;
        }
        s = (s + 1u) & J->hmask;
    }
}

// Inclusive block scan of one value per thread (WG threads); *total gets
// the sum over the block.  sh must hold WG elements.
template <typename T>
__device__ __forceinline__ T block_scan_incl(T v, T *sh, T *total)
{
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint32_t off = 1; off < 64u; off <<= 1) {
        const T t = __shfl_up(v, off);
        if (lane >= off)
            v += t;
    }
    if (lane == 63u)
        sh[wave] = v;
    __syncthreads();
    T before = 0, all = 0;
    for (uint32_t w = 0; w < WG / 64; ++w) {
        const T x = sh[w];
        before += w < wave ? x : (T)0;
        all += x;
    }
    __syncthreads();
    *total = all;
    return v + before;
}

// Inclusive prefix sums of NV values per thread over the workgroup, in one
// pass: shuffles within each wave, then the wave totals through LDS.  tot
// receives the workgroup totals.  sh holds NV * (WG/64) words.
template <int NV>
__device__ __forceinline__ void block_scan_n(uint32_t (&v)[NV], uint32_t *sh, uint32_t (&tot)[NV])
{
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint32_t off = 1; off < 64u; off <<= 1)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const uint32_t t = (uint32_t)__shfl_up((int)v[c], off);
            if (lane >= off)
                v[c] += t;
        }
    if (lane == 63u)
#pragma unroll
        for (int c = 0; c < NV; ++c)
            sh[NV * wave + c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        uint32_t before = 0, all = 0;
        for (uint32_t w = 0; w < WG / 64; ++w) {
            const uint32_t x = sh[NV * w + c];
            before += w < wave ? x : 0u;
            all += x;
        }
        v[c] += before;
        tot[c] = all;
    }
    __syncthreads();
}

// Sum of one value per thread over the workgroup (result in every thread).
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *sh)
{
    for (int off = 32; off > 0; off >>= 1)
        v += (uint32_t)__shfl_xor((int)v, off);
    if (lane_id() == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < WG / 64; ++w)
        t += sh[w];
    __syncthreads();
    return t;
}

// NQ rounds of two workgroup-aggregated appends (ctr points at a pair of
// adjacent u32 counters, low word first; pa / pb receive the slots of
// threads whose a / b is true), in round order, with one 64-bit atomic for
// the workgroup; and, in the same exchange, the workgroup's sums of NS
// statistics and maximum of one more (st, per thread), which thread 0 adds
// to counter line `line` right after the append atomic.  Each wave reduces
// its statistics with shuffles before the one barrier that the appends
// need anyway (a separate reduction cost a barrier and an LDS pass more).
// sh holds 2 * NQ * (WG/64) + 2 + (NS + 1) * (WG/64) words.
template <int NQ, int NS>
__device__ __forceinline__ void block_append2_stats(uint32_t *ctr, const bool (&a)[NQ],
                                                    const bool (&b)[NQ], uint32_t (&st)[NS + 1],
                                                    uint32_t *line, uint32_t *sh,
                                                    uint32_t (&pa)[NQ], uint32_t (&pb)[NQ])
{
    constexpr int NW = WG / 64;
    uint32_t *shs = sh + 2 * NQ * NW + 2;
    const uint32_t wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i <= NS; ++i)
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)st[i], off);
            st[i] = i < NS ? st[i] + o : (o > st[i] ? o : st[i]);
        }
    unsigned long long ba[NQ], bb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        ba[q] = __ballot(a[q]);
        bb[q] = __ballot(b[q]);
        if (lane_id() == 0) {
            sh[q * NW + wave] = (uint32_t)__popcll(ba[q]);
            sh[(NQ + q) * NW + wave] = (uint32_t)__popcll(bb[q]);
        }
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int i = 0; i <= NS; ++i)
            shs[i * NW + wave] = st[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ta = 0, tb = 0;
        for (int i = 0; i < NQ * NW; ++i) {
            const uint32_t ca = sh[i], cb = sh[NQ * NW + i];
            sh[i] = ta;
            sh[NQ * NW + i] = tb;
            ta += ca;
            tb += cb;
        }
        // the statistics, then the append; both are complete before the
        // positions are handed out, so that the workgroup can arrive
        // without waiting for its stores
#pragma unroll
        for (int i = 0; i <= NS; ++i) {
            uint32_t x = shs[i * NW];
            for (int w = 1; w < NW; ++w) {
                const uint32_t o = shs[i * NW + w];
                x = i < NS ? x + o : (o > x ? o : x);
            }
            if (x)
                i < NS ? (void)atomicAdd(line + i, x) : (void)atomicMax(line + i, x);
        }
        unsigned long long old = 0;
        if (ta | tb)
            old = atomicAdd((unsigned long long *)ctr,
                            ((unsigned long long)tb << 32) | (unsigned long long)ta);
        __builtin_amdgcn_s_waitcnt(WAIT_VM0);
        sh[2 * NQ * NW] = (uint32_t)old;
        sh[2 * NQ * NW + 1] = (uint32_t)(old >> 32);
    }
    __syncthreads();
    const unsigned long long lt = lanemask_lt();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        pa[q] = sh[2 * NQ * NW] + sh[q * NW + wave] + (uint32_t)__popcll(ba[q] & lt);
        pb[q] = sh[2 * NQ * NW + 1] + sh[(NQ + q) * NW + wave] + (uint32_t)__popcll(bb[q] & lt);
    }
    __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------
// Item bitsets from rows: bit r of vert[i * nw + g] is set when row 64g + r
// holds item i.
//
// 64 x 64 bit transposition in one wave: lane r holds a 64-bit row, and after
// six exchange steps lane c holds column c.  The step of width j swaps the
// off-diagonal j x j blocks of every 2j x 2j block: lane r trades with lane
// r ^ j, the lower lane taking its partner's low-column half into its high
// columns and the upper lane the partner's high half into its low columns
// (a transpose is a block swap at every scale).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t transpose64(uint64_t x, uint32_t lane)
{
    constexpr uint64_t HI[6] = {0xFFFFFFFF00000000ull, 0xFFFF0000FFFF0000ull,
                                0xFF00FF00FF00FF00ull, 0xF0F0F0F0F0F0F0F0ull,
                                0xCCCCCCCCCCCCCCCCull, 0xAAAAAAAAAAAAAAAAull};
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = 32 >> s;
        const uint64_t y = __shfl_xor(x, j, 64);
        x = (lane & (uint32_t)j) ? ((x & HI[s]) | ((y >> j) & ~HI[s]))
                                 : ((x & ~HI[s]) | ((y << j) & HI[s]));
    }
    return x;
}

// A workgroup transposes one tile: TR_G consecutive row words (64 rows each)
// by the 64 * TR_W items of TR_W row-bitmap words.  Per row word, each wave
// loads the tile's words of its 64 rows (lane r: row 64g + r), transposes
// each 64 x 64 block and puts item i's word for g in LDS at (i, g).  The tile
// then leaves as runs of TR_G consecutive words per item (128 contiguous
// bytes), not one scattered word per lane.
//
// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so the
// k-th workgroup of XCD x takes unit x * P + k of the (tile, word chunk)
// units, chunk fastest: each XCD walks a contiguous range of rows, and the
// workgroups that read the same rows (one per chunk) share its L2.
constexpr uint32_t TR_G = 16;               // row words per tile
constexpr uint32_t TR_W = 4;                // row-bitmap words per tile (x 64 items)
constexpr uint32_t TR_STRIDE = TR_G + 1;    // LDS words per item (odd: spreads banks)
constexpr uint32_t N_XCD = 8;

__global__ __launch_bounds__(WG) void k_transpose(const uint64_t *__restrict__ rows, uint64_t n,
                                                  uint32_t m, uint32_t W, uint64_t *vert,
                                                  uint32_t nw, uint32_t per_xcd)
{
    __shared__ uint64_t T[TR_W * 64 * TR_STRIDE];
    const uint32_t chunks = (W + TR_W - 1u) / TR_W;
    const uint32_t tiles = (nw + TR_G - 1u) / TR_G;
    const uint64_t units = (uint64_t)tiles * chunks;
    const uint64_t u = (uint64_t)(blockIdx.x % N_XCD) * per_xcd + blockIdx.x / N_XCD;
    if (blockIdx.x / N_XCD >= per_xcd || u >= units)
        return;
    const uint32_t tile = (uint32_t)(u / chunks), c = (uint32_t)(u - (uint64_t)tile * chunks);
    const uint32_t g0 = tile * TR_G, w0 = c * TR_W;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    constexpr uint32_t PER_WAVE = TR_G / (WG / 64);
    // every load of the wave's row words before the first exchange
    uint64_t x[PER_WAVE][TR_W];
#pragma unroll
    for (uint32_t t = 0; t < PER_WAVE; ++t) {
        const uint64_t r = (uint64_t)(g0 + wave + t * (WG / 64)) * 64u + lane;
#pragma unroll
        for (uint32_t i = 0; i < TR_W; ++i)
            x[t][i] = r < n && w0 + i < W ? rows[r * W + w0 + i] : 0ull;
    }
#pragma unroll
    for (uint32_t t = 0; t < PER_WAVE; ++t)
#pragma unroll
        for (uint32_t i = 0; i < TR_W; ++i)
            T[(i * 64u + lane) * TR_STRIDE + wave + t * (WG / 64)] = transpose64(x[t][i], lane);
    __syncthreads();
    const uint32_t gl = threadIdx.x % TR_G;
    const uint32_t g = g0 + gl;
    for (uint32_t it = threadIdx.x / TR_G; it < TR_W * 64u; it += WG / TR_G) {
        const uint32_t item = w0 * 64u + it;
        if (item < m && g < nw)
            vert[(uint64_t)item * nw + g] = T[it * TR_STRIDE + gl];
    }
}

// FirstPass on item bitsets: supp(i) is the popcount of item i's bitset.
// Work item = (job, item, FPV_WORDS-word chunk).
__global__ __launch_bounds__(WG) void k_first_pass_vert(const Job *__restrict__ jobs,
                                                        const Plan *__restrict__ plan,
                                                        unsigned long long total)
{
    __shared__ uint32_t sh[WG / 64];
    for (unsigned long long it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t j = find_job(plan->pre_fp, plan->njobs, it);
        const Job *J = jobs + j;
        const uint32_t cpi = (J->nw + FPV_WORDS - 1u) / FPV_WORDS;
        const uint32_t local = (uint32_t)(it - plan->pre_fp[j]);
        const uint32_t item = local / cpi, ch = local - item * cpi;
        const uint32_t w0 = ch * FPV_WORDS;
        const uint32_t w1 = w0 + FPV_WORDS < J->nw ? w0 + FPV_WORDS : J->nw;
        const uint64_t *v = J->vert + (uint64_t)item * J->nw;
        // all of the thread's words in flight at once (FPV_WORDS / WG loads)
        constexpr uint32_t PER = FPV_WORDS / WG;
        uint64_t x[PER];
#pragma unroll
        for (uint32_t k = 0; k < PER; ++k) {
            const uint32_t w = w0 + threadIdx.x + k * WG;
            x[k] = v[w < w1 ? w : w0];
        }
        uint32_t c = 0;
#pragma unroll
        for (uint32_t k = 0; k < PER; ++k)
            c += w0 + threadIdx.x + k * WG < w1 ? (uint32_t)__popcll(x[k]) : 0u;
        c = block_sum(c, sh);
        if (threadIdx.x == 0 && c)
            atomicAdd(&J->item_cnt[item], c);
    }
}

// ---------------------------------------------------------------------------
// FirstPass: support of every item over all rows (column popcount).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_first_pass(const Job *__restrict__ jobs,
                                                   const Plan *__restrict__ plan,
                                                   unsigned long long total)
{
    __shared__ uint32_t hist[MAX_ITEMS];
    for (unsigned long long it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t j = find_job(plan->pre_fp, plan->njobs, it);
        const Job *J = jobs + j;
        const uint32_t W = J->W, m = J->m;
        const uint64_t chunk = it - plan->pre_fp[j];
        const uint64_t r0 = chunk * FP_ROWS;
        const uint64_t r1 = r0 + FP_ROWS < J->n ? r0 + FP_ROWS : J->n;
        for (uint32_t i = threadIdx.x; i < m; i += WG)
            hist[i] = 0;
        __syncthreads();
        const uint64_t *rows = J->rows;
        for (uint64_t e = r0 * W + threadIdx.x; e < r1 * W; e += WG) {
            uint64_t x = rows[e];
            const uint32_t base = (uint32_t)(e % W) * 64u;
            while (x) {
                atomicAdd(&hist[base + (uint32_t)__builtin_ctzll(x)], 1u);
                x &= x - 1;
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += WG)
            if (hist[i])
                atomicAdd(&J->item_cnt[i], hist[i]);
        __syncthreads();
    }
}

// Frequent items (ascending) and the size of the pair candidate set.
// One workgroup per job.
__global__ __launch_bounds__(WG) void k_l1(const Job *__restrict__ jobs)
{
    __shared__ uint32_t sh[WG];
    const Job *J = jobs + blockIdx.x;
    JobState *st = J->st;
    if (J->classic) {
        // classic DIC: every item may extend a box, and every 1-itemset is a
        // first candidate (pool entries 0..m-1)
        for (uint32_t i = threadIdx.x; i < J->m; i += WG) {
            J->l1[i] = i;
            J->l1pos[i] = i;
        }
        if (threadIdx.x == 0) {
            st->nL1 = J->m;
            st->pending = 1;
            st->pool_base = 0;
            st->pool_n = J->m;
        }
        return;
    }
    uint32_t carry = 0;
    for (uint32_t b = 0; b < J->m; b += WG) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t f = (i < J->m && J->item_cnt[i] >= J->tau) ? 1u : 0u;
        uint32_t tot;
        const uint32_t incl = block_scan_incl<uint32_t>(f, sh, &tot);
        if (f)
            J->l1[carry + incl - 1u] = i;
        if (i < J->m)
            J->l1pos[i] = f ? carry + incl - 1u : NONE;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        const uint32_t nL1 = carry;
        const uint64_t nC2 = (uint64_t)nL1 * (nL1 ? nL1 - 1u : 0u) / 2u;
        st->nL1 = nL1;
        st->pending = 1;
        st->pool_base = 0;
        st->pool_n = (uint32_t)nC2;
    }
}

// First candidates, written as pool entries and as the first live list:
// the bitwise OR of every pair of frequent items (entries 0..nC2-1), or in
// classic mode every 1-itemset (entries 0..m-1).
__global__ __launch_bounds__(WG) void k_init_pairs(const Job *__restrict__ jobs,
                                                   const Plan *__restrict__ plan,
                                                   unsigned long long total)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * WG;
    for (unsigned long long x = (unsigned long long)blockIdx.x * WG + threadIdx.x; x < total;
         x += stride) {
        const uint32_t j = find_job(plan->pre_cg, plan->njobs, x);
        const Job *J = jobs + j;
        const uint32_t nL1 = J->st->nL1;
        const unsigned long long local = x - plan->pre_cg[j];
        if (J->classic) {
            // 1-itemset {a} at pool entry a
            const uint32_t a = (uint32_t)local, W = J->W;
            uint64_t *mk = J->pmask + (uint64_t)a * W;
            for (uint32_t w = 0; w < W; ++w)
                mk[w] = 0;
            mk[a >> 6] = 1ull << (a & 63u);
            J->phash[a] = zob(a);
            J->pnz[a] = 1ull << (a >> 6);
            J->pk[a] = 1;
            J->pitems[(uint64_t)a * KD] = (uint16_t)a;
            J->psupp[a] = 0;
            J->pstate[a] = standing(ST_DASHED_CIRCLE, PROMO_NONE);
            uint4 *r = J->live1 + (uint64_t)a * LREC;  // the first stop's current list
            r[0] = make_uint4(a, 0u, 0u, 1u);
            r[1] = make_uint4(a, 0u, 0u, 0u);
            hash_insert(J, zob(a), 1, a);
            continue;
        }
        const uint32_t a = (uint32_t)(local / nL1), b = (uint32_t)(local % nL1);
        if (a >= b)
            continue;
        const uint32_t p = a * nL1 - a * (a + 1u) / 2u + (b - a - 1u);
        const uint32_t ia = J->l1[a], ib = J->l1[b];
        const uint32_t W = J->W;
        uint64_t *mk = J->pmask + (uint64_t)p * W;
        for (uint32_t w = 0; w < W; ++w)
            mk[w] = 0;
        mk[ia >> 6] |= 1ull << (ia & 63u);
        mk[ib >> 6] |= 1ull << (ib & 63u);
        const unsigned long long h = zob(a) ^ zob(b);
        J->phash[p] = h;
        J->pnz[p] = (1ull << (ia >> 6)) | (1ull << (ib >> 6));
        J->pk[p] = 2;
        J->pitems[(uint64_t)p * KD] = (uint16_t)a;
        J->pitems[(uint64_t)p * KD + 1] = (uint16_t)b;
        J->psupp[p] = 0;
        J->pstate[p] = standing(ST_DASHED_CIRCLE, PROMO_NONE);
        uint4 *r = J->live1 + (uint64_t)p * LREC;  // the first stop's current list
        r[0] = make_uint4(p, 0u, 0u, 2u);
        r[1] = make_uint4(a | (b << 16), 0u, 0u, 0u);
        // no hash entry: outside the classic start a pair is only ever looked
        // up by its index (MakeCandidates' 2-subsets); larger itemsets and
        // the classic start's pairs go through the hash table
    }
}

// ---------------------------------------------------------------------------
// One stop per launch.
// ---------------------------------------------------------------------------
//
// Stop e (epoch e) is one launch of k_stop (k_count counts the row-bitmap
// jobs' survivors just before it).  Its work items do not depend on each
// other:
//   * MakeCandidates for the boxes promoted at stop e-1: C = S | {a} for a
//     new box S and a frequent item a.  Each C admitted is counted on block
//     e by the workgroup that made it (CountSupport, Algorithm 3) and pruned
//     there at once (Algorithm 4, with CheckFullPass, Algorithm 5);
//   * CountSupport of the survivors of stop e-1 on block e, then Prune and
//     CheckFullPass of each (by the last chunk of a candidate group when the
//     group's block is split over several work items).
// The last workgroup to finish completes stop e for every job and begins
// stop e+1: the block advance with the rewind of Algorithm 2, the swap of
// the live and new-box lists, the plan of the next launch.
//
// MakeCandidates for stop e-1 runs while stop e's Prune changes the standing
// of other itemsets.  It must see each itemset as it stood at the end of
// stop e-1, and the standing word gives exactly that: an itemset is a box
// for it only if it was promoted at a stop before e.  The itemsets, counts
// and per-stop trace are those of the paper's order (at every stop: Count,
// Prune, MakeCandidates, CheckFullPass).

// Begin the job's next stop: the next block (stop <- stop + 1, back to the
// first block after the last), the next epoch and its zeroed trace entry.
__device__ __forceinline__ void begin_stop(const Job *J, JobState *st)
{
    // the next block, rewinding after the last (stop is 0 before the first)
    const uint32_t stop = st->stop >= J->stop_max ? 1u : st->stop + 1u;
    st->stop = stop;
    const uint64_t first = (uint64_t)(stop - 1u) * J->Mp;
    const uint64_t end = (uint64_t)stop * J->Mp;
    st->first = (uint32_t)first;
    st->last = (uint32_t)(end < J->n ? end : J->n);
    st->fw = st->first >> 6;  // the block's 64-row words, for the bitset counts
    st->lw = (st->last - 1u) >> 6;
    st->epoch += 1u;
    if (st->epoch - 1u < J->trace_cap) {
        dic_stop_trace t{};
        J->trace[st->epoch - 1u] = t;
    }
}

// The planning knobs, copied from the Plan into LDS by the serial part of a
// launch before any job is planned, so that a job's plan reads its cell
// without a dependent global load.
struct PlanTune {
    uint32_t cell[TUNE_CELLS];  // mode << 16 | target
    uint32_t vt_target, vt_wave_k, vt_tile_words, count_target;
};

// Every thread calls; the caller's barrier makes the copy visible.
__device__ __forceinline__ void load_tune(const Plan *plan, PlanTune *t)
{
    const uint32_t i = threadIdx.x;
    if (i < TUNE_CELLS)
        t->cell[i] = ((uint32_t)plan->cell_mode[i] << 16) | plan->cell_target[i];
    else if (i == TUNE_CELLS)
        t->vt_target = plan->vt_target;
    else if (i == TUNE_CELLS + 1)
        t->vt_wave_k = plan->vt_wave_k;
    else if (i == TUNE_CELLS + 2)
        t->vt_tile_words = plan->vt_tile_words;
    else if (i == TUNE_CELLS + 3)
        t->count_target = plan->count_target;
}

// Work of one job in the next launch, from its state s: chunks of
// MakeCandidates (WG (new box, frequent item) pairs each), the survivors'
// work items by layout, and the row-bitmap count's work items (k_count).
// The count plan is stored in s.
__device__ __forceinline__ void plan_stop(const Job *J, JobState &s, const PlanTune *tune,
                                          uint32_t *items_rows, uint32_t *items_stop,
                                          unsigned long long *chunks)
{
    *items_rows = *items_stop = 0;
    *chunks = 0;
    if (s.done || s.overflow || s.pending)
        return;
    *chunks = ((unsigned long long)s.n_prev * s.nL1 + WG - 1u) / WG;
    const uint32_t K = s.k_cur;
    if (K == 0)
        return;
    const uint32_t rows = s.last - s.first;
    // per-shape cell of this stop, else the global choice
    const uint32_t cell = tune->cell[tune_cell(s.lw - s.fw + 1u, K)];
    const uint32_t cmode = cell >> 16, ctarget = cell & 0xFFFFu;
    const bool wave = cmode ? cmode == 1u : K < tune->vt_wave_k;
    if (J->layout == LAYOUT_VERTICAL && wave) {
        // few candidates: one wave per candidate, no tile
        s.cmode = 1;
        *items_stop = (K + WG / 64 - 1u) / (WG / 64);
    } else if (J->layout == LAYOUT_VERTICAL) {
        // (candidate groups of WG * cpt) x (chunks of tiles of tw words)
        s.cmode = 0;
        const uint32_t tw = vert_tile_words(s.nL1, tune->vt_tile_words);
        const uint32_t ntile = (s.lw - s.fw + tw) / tw;
        // candidates per thread: spend the parallelism beyond vt_target
        // workgroups on fewer tile loads
        const uint64_t vt_target = ctarget ? ctarget : tune->vt_target;
        // (32-bit division when the work fits: a 64-bit one is far longer)
        const uint64_t work = (uint64_t)K * ntile, per = (uint64_t)WG * vt_target;
        uint64_t cpt = work + per <= 0xFFFFFFFFull
                           ? (uint64_t)(((uint32_t)work + (uint32_t)per - 1u) / (uint32_t)per)
                           : (work + per - 1u) / per;
        cpt = cpt < 1u ? 1u : (cpt > (uint64_t)VT_CPT ? (uint64_t)VT_CPT : cpt);
        s.cpt = (uint32_t)cpt;
        const uint32_t n_cg = (K + WG * (uint32_t)cpt - 1u) / (WG * (uint32_t)cpt);
        uint32_t want = ((uint32_t)vt_target + n_cg - 1u) / n_cg;
        want = want < 1u ? 1u : (want > ntile ? ntile : want);
        const uint32_t tpc = (ntile + want - 1u) / want;
        s.tw = tw;
        s.n_ct = n_cg;
        s.rpi = tpc;
        s.n_ri = (ntile + tpc - 1u) / tpc;
        *items_stop = n_cg * s.n_ri;
    } else {
        // k_count counts (row range x candidate group); the stop kernel then
        // prunes ZP * WG survivors per work item
        const uint32_t rt = row_tile_rows(J->W);
        const uint32_t n_ct = (K + CAND_PER_WG - 1u) / CAND_PER_WG;
        const uint32_t tiles = (rows + rt - 1u) / rt;
        uint32_t want = (tune->count_target + n_ct - 1u) / n_ct;
        want = want < 1u ? 1u : (want > tiles ? tiles : want);
        const uint32_t rpi = ((tiles + want - 1u) / want) * rt;
        s.n_ct = n_ct;
        s.rpi = rpi;
        s.n_ri = (rows + rpi - 1u) / rpi;
        *items_rows = n_ct * s.n_ri;
        *items_stop = (K + ZP * WG - 1u) / (ZP * WG);
    }
}

// One job's turn in the serial part of a launch: complete stop e (finish:
// after every work item of the stop kernel) or begin the first stop of a
// job added since the last chunk (begin: in k_begin), then plan the next
// launch.  The state is read once into registers, updated there and
// written back whole.  Completing stop e takes the candidates made at this
// launch for stop e-1's new boxes (the pool's growth), writes the trace,
// and either ends the run or begins stop e+1.  Counters that other
// workgroups of the launch updated with atomics are read with device-scope
// atomic loads.
// What settle_job reads from memory: the state, and the counters other
// workgroups of the launch updated with atomics (device-scope atomic loads).
// Loaded ahead of the knobs' copy, so that both are in flight together.
struct SettleIn {
    JobState s;
    uint32_t pn, asserts;
    uint32_t ctr[CTR_FIELDS];  // the counter lines added up (CTR_MAX_REM: their maximum)
    bool lines_done;           // the lines are cleared already
    unsigned long long kn_nn;
};

__device__ __forceinline__ void settle_load(const Job *J, bool finish, SettleIn &in)
{
    JobState *stp = J->st;
    __builtin_memcpy(&in.s, stp, sizeof(JobState));
    in.lines_done = false;
    if (finish) {
        in.pn = in.s.pool_base + __hip_atomic_load(J->ctrs + CTR_GEN, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        in.kn_nn = __hip_atomic_load((const unsigned long long *)(J->ctrs + CTR_APPEND),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        in.asserts = __hip_atomic_load(&stp->asserts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t c[CTR_LINES][CTR_FIELDS];
#pragma unroll
        for (uint32_t l = 0; l < CTR_LINES; ++l)
#pragma unroll
            for (uint32_t f = 0; f < CTR_FIELDS; ++f)
                c[l][f] = __hip_atomic_load(J->ctrs + l * CTR_STRIDE + f, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (uint32_t f = 0; f < CTR_FIELDS; ++f) {
            uint32_t t = c[0][f];
#pragma unroll
            for (uint32_t l = 1; l < CTR_LINES; ++l)
                t = f == CTR_MAX_REM ? (c[l][f] > t ? c[l][f] : t) : t + c[l][f];
            in.ctr[f] = t;
        }
    }
}

// The finishing form of settle_load for one job, by every lane of one wave:
// lane l < CTR_LINES reads statistics line l and clears it, and the lines
// are added up with shuffles.
__device__ __forceinline__ void settle_load_wave(const Job *J, SettleIn &in)
{
    JobState *stp = J->st;
    __builtin_memcpy(&in.s, stp, sizeof(JobState));
    in.pn = in.s.pool_base + __hip_atomic_load(J->ctrs + CTR_GEN, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    in.kn_nn = __hip_atomic_load((const unsigned long long *)(J->ctrs + CTR_APPEND),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    in.asserts = __hip_atomic_load(&stp->asserts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t lane = lane_id();
    uint32_t v[CTR_FIELDS];
#pragma unroll
    for (uint32_t f = 0; f < CTR_FIELDS; ++f)
        v[f] = 0u;
    if (lane < CTR_LINES) {
#pragma unroll
        for (uint32_t f = 0; f < CTR_FIELDS; ++f)
            v[f] = __hip_atomic_load(J->ctrs + lane * CTR_STRIDE + f, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
    // every counter starts the next stop at zero (read by its launch); the
    // loads above have returned before the lines are cleared
    __builtin_amdgcn_s_waitcnt(WAIT_VM0);
    if (lane < CTR_LINES) {
        uint4 *line = (uint4 *)(J->ctrs + lane * CTR_STRIDE);
        line[0] = line[1] = make_uint4(0u, 0u, 0u, 0u);  // words 0..7
    } else if (lane == CTR_LINES) {
        *(unsigned long long *)(J->ctrs + CTR_APPEND) = 0ull;
        J->ctrs[CTR_GEN] = 0u;
    }
    // totals over lanes 0..CTR_LINES-1 (the other lanes hold zeros)
#pragma unroll
    for (int off = 1; off < (int)CTR_LINES; off <<= 1)
#pragma unroll
        for (uint32_t f = 0; f < CTR_FIELDS; ++f) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v[f], off);
            v[f] = f == CTR_MAX_REM ? (o > v[f] ? o : v[f]) : v[f] + o;
        }
#pragma unroll
    for (uint32_t f = 0; f < CTR_FIELDS; ++f)
        in.ctr[f] = __builtin_amdgcn_readfirstlane(v[f]);
    in.lines_done = true;
}

__device__ __forceinline__ void settle_job(const Job *J, const SettleIn &in, bool finish,
                                           bool begin, const PlanTune *tune, uint32_t *items_rows,
                                           uint32_t *items_stop, unsigned long long *chunks)
{
    JobState *stp = J->st;
    JobState s = in.s;
    bool write = false;
    if (finish && !s.done && !s.overflow && !s.pending) {
        write = true;
        const uint32_t pn = in.pn;
        const unsigned long long kn_nn = in.kn_nn;
        const uint32_t mr = in.ctr[CTR_MAX_REM];
        s.asserts = in.asserts;
        if (!in.lines_done) {
            // the counters start the next stop at zero (read by its launch)
#pragma unroll
            for (uint32_t l = 0; l < CTR_LINES; ++l)
#pragma unroll
                for (uint32_t f = 0; f < CTR_FIELDS; ++f)
                    J->ctrs[l * CTR_STRIDE + f] = 0u;
            *(unsigned long long *)(J->ctrs + CTR_APPEND) = 0ull;
            J->ctrs[CTR_GEN] = 0u;
        }
        const uint32_t kn = (uint32_t)kn_nn, nn = (uint32_t)(kn_nn >> 32);
        const uint32_t E = s.epoch;
        s.pool_n = pn;
        if (pn > J->cap) {  // MakeCandidates ran out of pool room
            s.overflow = 1;
        } else {
            const uint32_t gen = pn - s.pool_base;
            if (E >= 2u && E - 2u < J->trace_cap)
                J->trace[E - 2u].generated = gen;
            const uint32_t live = s.k_cur + gen;
            if (live == 0u) {  // nothing was live at this stop: the run ended with the last one
                s.done = 1;
                s.need = 0;
                s.stops = E - 1u;
            } else {
                const uint32_t rows = s.last - s.first;
                s.stops = E;
                s.tests += (unsigned long long)live * rows;
                if (live > s.peak_K)
                    s.peak_K = live;
                if (E - 1u < J->trace_cap) {
                    dic_stop_trace *t = J->trace + (E - 1u);
                    t->stop = s.stop;
                    t->rows = rows;
                    t->live = live;
                    t->words = in.ctr[CTR_WORDS];
                    t->items = in.ctr[CTR_ITEMS];
                    t->promoted = in.ctr[CTR_PROMOTED];
                    t->pruned = in.ctr[CTR_PRUNED];
                    t->solidified = in.ctr[CTR_SOLID];
                }
                if (kn == 0u && nn == 0u) {  // no survivor and no new box: DASHED stays empty
                    s.done = 1;
                    s.need = 0;
                } else {
                    s.k_cur = kn;
                    s.n_prev = nn;
                    s.pool_base = pn;
                    s.parity ^= 1u;
                    // stops certainly still needed: the kept candidates'
                    // remaining stops, and one for the new boxes' extensions
                    s.need = mr > (nn ? 1u : 0u) ? mr : (nn ? 1u : 0u);
                    begin_stop(J, &s);
                }
            }
        }
    } else if (begin && s.pending && !s.done && !s.overflow) {
        // first stop: the first candidates (pool entries 0..pn-1, already in
        // live1) are the current list, counted like survivors
        write = true;
        const uint32_t pn = s.pool_n < J->cap ? s.pool_n : J->cap;
        s.k_cur = pn;
        s.n_prev = 0;
        s.pool_base = pn;
        s.parity = 1;
        s.stop = 0;
        s.epoch = 0;
        s.need = J->stop_max;  // a first candidate needs a full pass
        s.pending = 0;
        begin_stop(J, &s);
    }
    plan_stop(J, s, tune, items_rows, items_stop, chunks);
    if (write || (!s.done && !s.overflow && !s.pending))
        __builtin_memcpy(stp, &s, sizeof(JobState));
}

// Arrival counter of a launch, called by one thread per workgroup after the
// workgroup's work: true for the workgroup that arrives last.  Only the
// first n workgroups arrive (n = min(grid, work items), at least 1: the
// others had no work item); the rest return false at once.  Up to
// TICKET_GROUPS arrivals share one counter; more go through two levels
// (workgroups of a group, then the groups) so that no counter sees many
// atomics.  The last arrival clears the counters it used.
__device__ __forceinline__ bool arrive_last(uint32_t *tickets, uint32_t n)
{
    if (blockIdx.x >= n)
        return false;
    const uint32_t G = TICKET_GROUPS;
    if (n <= G) {
        if (atomicAdd(&tickets[0], 1u) != n - 1u)
            return false;
        __hip_atomic_store(&tickets[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    const uint32_t g = blockIdx.x % G;
    const uint32_t members = n / G + (g < n % G ? 1u : 0u);
    if (atomicAdd(&tickets[(g + 1u) * TICKET_STRIDE], 1u) != members - 1u)
        return false;
    if (atomicAdd(&tickets[0], 1u) != G - 1u)
        return false;
    for (uint32_t x = 0; x <= G; ++x)
        __hip_atomic_store(&tickets[x * TICKET_STRIDE], 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// The serial part of a launch for every job (one workgroup, every thread
// calls): settle_job per job, then per-job prefix sums of the next launch's
// work (row-bitmap count items, stop-kernel survivor items, MakeCandidates
// chunks) and their totals.  sh holds 2 * (WG/64) words.  Up to 64 jobs
// the sums are one wave's (no barrier); more use the workgroup's scans.
__device__ __forceinline__ void settle_and_plan(const Job *__restrict__ jobs, Plan *plan, bool finish, bool begin,
                                uint32_t *sh, unsigned long long *shc, PlanTune *tune)
{
    const uint32_t njobs = plan->njobs;
    if (threadIdx.x == 0) {
        plan->pre_count[0] = 0;
        plan->pre_countv[0] = 0;
        plan->pre_cg[0] = 0;
        if (njobs == 0u) {
            plan->total_v = 0;
            plan->total_cg = 0;
        }
    }
    if (njobs == 0u)
        return;
    if (njobs == 1u) {
        // One job: its serial part runs wave-uniform in wave 0, so the
        // compiler keeps it in scalar registers on the scalar ALU instead of
        // one lane's chain of vector instructions.
        const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        SettleIn in;
        if (wave == 0u) {
            if (finish)
                settle_load_wave(jobs, in);
            else
                settle_load(jobs, false, in);
        }
        load_tune(plan, tune);
        __syncthreads();
        if (wave != 0u)
            return;
        uint32_t items = 0, itemsv = 0;
        unsigned long long chunks = 0;
        settle_job(jobs, in, finish, begin, tune, &items, &itemsv, &chunks);
        if (threadIdx.x == 0) {
            plan->pre_count[1] = items;
            plan->pre_countv[1] = itemsv;
            plan->pre_cg[1] = chunks;
            plan->total_v = itemsv;
            plan->total_cg = chunks;
        }
        return;
    }
    if (njobs <= 64u) {
        SettleIn in;
        const uint32_t j = threadIdx.x;
        if (j < njobs)
            settle_load(jobs + j, finish, in);
        load_tune(plan, tune);
        __syncthreads();
        if (threadIdx.x >= 64u)
            return;
        uint32_t items = 0, itemsv = 0;
        unsigned long long chunks = 0;
        if (j < njobs)
            settle_job(jobs + j, in, finish, begin, tune, &items, &itemsv, &chunks);
        // inclusive sums over the wave's lanes
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t a = __shfl_up(items, off, 64), b = __shfl_up(itemsv, off, 64);
            const unsigned long long c = __shfl_up(chunks, off, 64);
            if ((int)j >= off) {
                items += a;
                itemsv += b;
                chunks += c;
            }
        }
        if (j < njobs) {
            plan->pre_count[j + 1] = items;
            plan->pre_countv[j + 1] = itemsv;
            plan->pre_cg[j + 1] = chunks;
        }
        if (j == njobs - 1u) {
            plan->total_v = itemsv;
            plan->total_cg = chunks;
        }
        return;
    }
    load_tune(plan, tune);
    __syncthreads();
    uint32_t carry_c = 0, carry_v = 0;
    unsigned long long carry_g = 0;
    for (uint32_t b = 0; b < njobs; b += WG) {
        const uint32_t j = b + threadIdx.x;
        uint32_t items = 0, itemsv = 0;
        unsigned long long chunks = 0;
        if (j < njobs) {
            SettleIn in;
            settle_load(jobs + j, finish, in);
            settle_job(jobs + j, in, finish, begin, tune, &items, &itemsv, &chunks);
        }
        uint32_t v[2] = {items, itemsv}, t[2];
        block_scan_n<2>(v, sh, t);
        unsigned long long tg;
        const unsigned long long g = block_scan_incl<unsigned long long>(chunks, shc, &tg);
        if (j < njobs) {
            plan->pre_count[j + 1] = carry_c + v[0];
            plan->pre_countv[j + 1] = carry_v + v[1];
            plan->pre_cg[j + 1] = carry_g + g;
        }
        carry_c += t[0];
        carry_v += t[1];
        carry_g += tg;
    }
    if (threadIdx.x == 0) {
        plan->total_v = carry_v;
        plan->total_cg = carry_g;
    }
}

// The frequent items' bitsets in frequent-item order (item-bitset jobs with
// some infrequent item): fvert[a * nw + g] = vert[l1[a] * nw + g].  The counts
// then index an item's row by its frequent-item index, one dependent load
// fewer per tile and per wave.  Work: every (job, a, g), by prefix sums.
__global__ __launch_bounds__(WG) void k_gather_vert(const Job *__restrict__ jobs,
                                                    const Plan *__restrict__ plan,
                                                    unsigned long long total)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * WG;
    for (unsigned long long x = (unsigned long long)blockIdx.x * WG + threadIdx.x; x < total;
         x += stride) {
        const uint32_t j = find_job(plan->pre_fp, plan->njobs, x);
        const Job *J = jobs + j;
        const unsigned long long local = x - plan->pre_fp[j];
        const uint32_t a = (uint32_t)(local / J->nw);
        const uint32_t g = (uint32_t)(local - (unsigned long long)a * J->nw);
        J->fvert[local] = J->vert[(uint64_t)J->l1[a] * J->nw + g];
    }
}

// Start of a chunk of stops (one workgroup).  A job added since the last
// chunk begins its first stop; every job is then planned against the
// current job table.
__global__ __launch_bounds__(WG) void k_begin(const Job *__restrict__ jobs, Plan *plan)
{
    __shared__ uint32_t sh[2 * (WG / 64)];
    __shared__ unsigned long long shc[WG / 64];
    __shared__ PlanTune tune;
    settle_and_plan(jobs, plan, false, true, sh, shc, &tune);
}

// CountSupport (Algorithm 3) on row bitmaps, ahead of the stop kernel.  Work
// item = (row range, group of CAND_PER_WG survivors).  The workgroup stages
// the complemented rows of a tile in LDS as 32-bit planes (plane d holds
// dword d of every row), each wave takes CW candidates, and for every
// candidate each lane holds one row per 64-row group: acc = OR over the
// candidate's nonzero dwords of (c_d AND NOT t_d); the row contains the
// candidate iff acc == 0.  The 64 answers of a group are counted with a
// wave ballot and a popcount.
__global__ __launch_bounds__(WG) void k_count(const Job *__restrict__ jobs,
                                              const Plan *__restrict__ plan)
{
    __shared__ uint32_t tile[LDS_DWORDS];
    const uint32_t total = plan->pre_count[plan->njobs];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = lane_id();
    for (uint32_t it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t j = find_job(plan->pre_count, plan->njobs, it);
        const Job *J = jobs + j;
        const JobState *st = J->st;
        const uint32_t local = it - plan->pre_count[j];
        const uint32_t n_ct = st->n_ct;
        const uint32_t ri = local / n_ct;
        const uint32_t ct = local - ri * n_ct;
        const uint32_t W = J->W;
        const uint32_t rt = row_tile_rows(W);
        const uint32_t r_begin = st->first + ri * st->rpi;
        const uint32_t r_lim = r_begin + st->rpi;
        const uint32_t r_end = r_lim < st->last ? r_lim : st->last;
        const uint32_t K = st->k_cur;  // the last stop's survivors, in the current list
        const uint4 *live = st->parity ? J->live1 : J->live0;
        const uint32_t c0 = ct * CAND_PER_WG + wave * CW;

        uint32_t pidx[CW];
        uint32_t cnt[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
            pidx[q] = (c0 + (uint32_t)q < K) ? live[(uint64_t)(c0 + q) * LREC].x : NONE;
            cnt[q] = 0;
        }

        for (uint64_t s0 = r_begin; s0 < r_end; s0 += rt) {
            const uint32_t nr = (uint32_t)((r_end - s0) < rt ? (r_end - s0) : rt);
            __syncthreads();
            for (uint32_t r = threadIdx.x; r < rt; r += WG) {
                if (r < nr) {
                    const uint64_t *src = J->rows + (uint64_t)(s0 + r) * W;
                    for (uint32_t w = 0; w < W; ++w) {
                        const uint64_t v = ~src[w];
                        tile[(2u * w) * rt + r] = (uint32_t)v;
                        tile[(2u * w + 1u) * rt + r] = (uint32_t)(v >> 32);
                    }
                } else {
                    for (uint32_t w = 0; w < 2u * W; ++w)
                        tile[w * rt + r] = ~0u;  // never contains a nonempty itemset
                }
            }
            __syncthreads();
            const uint32_t G = (nr + 63u) >> 6;
#pragma unroll
            for (int q = 0; q < CW; ++q) {
                const uint32_t p = pidx[q];
                if (p == NONE)
                    break;
                uint32_t acc[MAX_GROUPS];
#pragma unroll
                for (int g = 0; g < MAX_GROUPS; ++g)
                    acc[g] = 0;
                uint64_t nz = J->pnz[p];
                const uint64_t *cm = J->pmask + (uint64_t)p * W;
                while (nz) {
                    const uint32_t wd = (uint32_t)__builtin_ctzll(nz);
                    nz &= nz - 1;
                    const uint64_t v = cm[wd];
                    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
                    if (lo) {
                        const uint32_t *pl = tile + (2u * wd) * rt + lane;
#pragma unroll
                        for (int g = 0; g < MAX_GROUPS; ++g)
                            if ((uint32_t)g < G)
                                acc[g] |= lo & pl[g * 64];
                    }
                    if (hi) {
                        const uint32_t *pl = tile + (2u * wd + 1u) * rt + lane;
#pragma unroll
                        for (int g = 0; g < MAX_GROUPS; ++g)
                            if ((uint32_t)g < G)
                                acc[g] |= hi & pl[g * 64];
                    }
                }
                uint32_t s = 0;
#pragma unroll
                for (int g = 0; g < MAX_GROUPS; ++g)
                    if ((uint32_t)g < G)
                        s += (uint32_t)__popcll(__ballot(acc[g] == 0u));
                cnt[q] += s;
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < CW; ++q)
                if (pidx[q] != NONE && cnt[q])
                    atomicAdd(J->psupp + pidx[q], cnt[q]);
        }
    }
}

// What the bitset counts need of a candidate: its size and, with at most KD
// items, its frequent-item indices (16 x u16, ascending).  A larger one is
// counted from a pool entry's mask (wide) plus at most one extra frequent
// item (a candidate made at this stop from its generating box).
struct CandItems {
    uint32_t k;
    uint32_t pk32[KD / 2];
    uint32_t wide;   // pool entry whose mask holds the items (k > KD)
    uint32_t extra;  // frequent-item index added to it, or NONE
};

__device__ __forceinline__ CandItems cand_items(const Job *J, uint32_t p)
{
    CandItems ci;
    ci.k = J->pk[p];
    ci.wide = p;
    ci.extra = NONE;
    if (ci.k <= (uint32_t)KD) {
        const uint4 *ip = (const uint4 *)(J->pitems + (uint64_t)p * KD);
        const uint4 h0 = ip[0], h1 = ip[1];
        ci.pk32[0] = h0.x; ci.pk32[1] = h0.y; ci.pk32[2] = h0.z; ci.pk32[3] = h0.w;
        ci.pk32[4] = h1.x; ci.pk32[5] = h1.y; ci.pk32[6] = h1.z; ci.pk32[7] = h1.w;
    } else {
#pragma unroll
        for (int t = 0; t < KD / 2; ++t)
            ci.pk32[t] = 0u;
    }
    return ci;
}

// A live record (see LREC) in registers.
struct LRec {
    uint32_t p, supp, sc, kb;  // kb: size | box << 16
    uint32_t it[KR / 2];
};

__device__ __forceinline__ LRec load_rec(const uint4 *list, uint32_t c)
{
    const uint4 *r = list + (uint64_t)c * LREC;
    const uint4 a = r[0], b = r[1];
    LRec x;
    x.p = a.x; x.supp = a.y; x.sc = a.z; x.kb = a.w;
    x.it[0] = b.x; x.it[1] = b.y; x.it[2] = b.z; x.it[3] = b.w;
    return x;
}

__device__ __forceinline__ void store_rec(uint4 *list, uint32_t c, const LRec &x)
{
    uint4 *r = list + (uint64_t)c * LREC;
    r[0] = make_uint4(x.p, x.supp, x.sc, x.kb);
    r[1] = make_uint4(x.it[0], x.it[1], x.it[2], x.it[3]);
}

// A record's item list: from the record up to KR items, from the pool up
// to KD, none (the mask is decoded instead) above.
__device__ __forceinline__ CandItems rec_items(const Job *J, const LRec &x)
{
    CandItems ci;
    ci.k = x.kb & 0xFFFFu;
    ci.wide = x.p;
    ci.extra = NONE;
#pragma unroll
    for (int t = 0; t < KD / 2; ++t)
        ci.pk32[t] = t < KR / 2 ? x.it[t] : 0u;
    if (ci.k > (uint32_t)KR && ci.k <= (uint32_t)KD) {
        const uint4 *ip = (const uint4 *)(J->pitems + (uint64_t)x.p * KD);
        const uint4 h0 = ip[0], h1 = ip[1];
        ci.pk32[0] = h0.x; ci.pk32[1] = h0.y; ci.pk32[2] = h0.z; ci.pk32[3] = h0.w;
        ci.pk32[4] = h1.x; ci.pk32[5] = h1.y; ci.pk32[6] = h1.z; ci.pk32[7] = h1.w;
    }
    return ci;
}

// CountSupport of one candidate by one wave over every 64-row word of the
// current block, straight from the item bitsets (no tile).  Returns the
// count in every lane.
__device__ __forceinline__ uint32_t count_wave_bitsets(const Job *J, const JobState *st,
                                                       const CandItems &ci)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lo_mask = ~0ull << (st->first & 63u);
    const uint64_t hi_mask =
        (st->last & 63u) ? ((1ull << (st->last & 63u)) - 1ull) : ~0ull;
    const uint64_t nw = J->nw;
    const uint64_t *__restrict__ fv = J->fvert;
    const uint32_t fw = st->fw, lw = st->lw;
    uint32_t cnt = 0;
    if (ci.k <= (uint32_t)KD) {
        // items four at a time, 3 words per lane per pass: the twelve loads of a
        // group carry no condition (past the list: the first item again, past
        // the block: the last word, both masked out) and issue together
        for (uint32_t w0 = fw + lane; w0 <= lw; w0 += 192u) {
            uint64_t acc[3];
            uint32_t wc[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const uint32_t w = w0 + 64u * u;
                wc[u] = w <= lw ? w : lw;
                acc[u] = w <= lw ? (w == fw ? lo_mask : ~0ull) & (w == lw ? hi_mask : ~0ull) : 0ull;
            }
            uint32_t qv[KD / 2];
#pragma unroll
            for (int u = 0; u < KD / 2; ++u)
                qv[u] = ci.pk32[u];
            const uint32_t first = qv[0] & 0xFFFFu;
#pragma unroll 1
            for (uint32_t t0 = 0; t0 < ci.k; t0 += 4u) {
                uint32_t row[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    row[t] = t0 + t < ci.k ? qv[0] & 0xFFFFu : first;
#pragma unroll
                    for (int u = 0; u < KD / 2; ++u)
                        qv[u] = (qv[u] >> 16) | (u + 1 < KD / 2 ? qv[u + 1] << 16 : 0u);
                }
                uint64_t v[4][3];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int u = 0; u < 3; ++u)
                        v[t][u] = fv[(uint64_t)row[t] * nw + wc[u]];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int u = 0; u < 3; ++u)
                        acc[u] &= v[t][u];
            }
#pragma unroll
            for (int u = 0; u < 3; ++u)
                cnt += (uint32_t)__popcll(acc[u]);
        }
    } else {
        const uint64_t nz = J->pnz[ci.wide];
        const uint64_t *cm = J->pmask + (uint64_t)ci.wide * J->W;
        for (uint32_t w = st->fw + lane; w <= st->lw; w += 64) {
            uint64_t acc =
                (w == st->fw ? lo_mask : ~0ull) & (w == st->lw ? hi_mask : ~0ull);
            if (ci.extra != NONE)
                acc &= J->fvert[(uint64_t)ci.extra * nw + w];
            uint64_t nzw = nz;
            while (nzw) {
                const uint32_t wd = (uint32_t)__builtin_ctzll(nzw);
                nzw &= nzw - 1;
                uint64_t bits = cm[wd];
                while (bits) {
                    const uint32_t item = wd * 64u + (uint32_t)__builtin_ctzll(bits);
                    bits &= bits - 1;
                    acc &= J->fvert[(uint64_t)J->l1pos[item] * nw + w];
                }
            }
            cnt += (uint32_t)__popcll(acc);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        cnt += (uint32_t)__shfl_xor((int)cnt, off);
    return cnt;
}

// CountSupport of one candidate by one wave over the current block in row
// bitmaps: lanes take rows, each testing (row & I) == I on I's nonzero
// words.  I is pool entry p's mask plus item `extra` (NONE: none).
__device__ __forceinline__ uint32_t count_wave_rows(const Job *J, const JobState *st, uint32_t p, uint32_t extra)
{
    const uint32_t W = J->W, lane = threadIdx.x & 63u;
    const uint64_t *I = J->pmask + (uint64_t)p * W;
    const uint32_t xw = extra != NONE ? extra >> 6 : 0xFFFFFFFFu;
    const uint64_t xb = extra != NONE ? 1ull << (extra & 63u) : 0ull;
    const uint64_t nz = J->pnz[p] | (extra != NONE ? 1ull << xw : 0ull);
    uint32_t cnt = 0;
    for (uint32_t r = st->first + lane; r < st->last; r += 64u) {
        const uint64_t *row = J->rows + (uint64_t)r * W;
        bool in = true;
        uint64_t nzw = nz;
        while (nzw && in) {
            const uint32_t w = (uint32_t)__builtin_ctzll(nzw);
            nzw &= nzw - 1;
            const uint64_t iw = I[w] | (w == xw ? xb : 0ull);
            in = (row[w] & iw) == iw;
        }
        cnt += in ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1)
        cnt += (uint32_t)__shfl_xor((int)cnt, off);
    return cnt;
}

// Stage the tile of words [w0, w0 + tw) of the current block: for every
// frequent item a, its bitset words at tile[a * ts ...], edge words masked
// to the block and words past the block's last word zero (so a tile is
// always ANDed whole).  Every thread of the workgroup calls; the barriers on
// both sides keep the previous tile's readers and this tile's readers apart.
__device__ __forceinline__ void stage_tile(const Job *J, const JobState *st, uint32_t w0,
                                           uint32_t tw, uint32_t ts, uint64_t *tile)
{
    const uint32_t fw = st->fw, lw = st->lw, nL1 = st->nL1;
    const uint64_t lo_mask = ~0ull << (st->first & 63u);
    const uint64_t hi_mask = (st->last & 63u) ? ((1ull << (st->last & 63u)) - 1ull) : ~0ull;
    // the job's fields in registers before the loop: a field read inside the
    // predicated loads would be re-read (and waited for) before every load
    const uint64_t *__restrict__ fv = J->fvert;
    const uint64_t nw = J->nw;
    __syncthreads();
    // thread (q, r) loads word r of items q, q + per, q + 2 per, ...
    const uint32_t per = WG / tw;
    const uint32_t q = threadIdx.x / tw, r = threadIdx.x - q * tw;
    if (q < per) {
        const uint32_t g = w0 + r;
        const uint64_t mask = g > lw ? 0ull
                                     : (g == fw ? lo_mask : ~0ull) & (g == lw ? hi_mask : ~0ull);
        const uint64_t *src = fv + (g < lw ? g : lw);  // in bounds; masked to 0 past the block
        // 12 loads in flight per batch: every address is valid (clamped to the
        // last item), so the loads carry no condition and issue together
        for (uint32_t a = q; a < nL1; a += 12u * per) {
            uint64_t v[12];
#pragma unroll
            for (int u = 0; u < 12; ++u) {
                const uint32_t it = a + u * per < nL1 ? a + u * per : nL1 - 1u;
                v[u] = src[(uint64_t)it * nw];
            }
#pragma unroll
            for (int u = 0; u < 12; ++u)
                if (a + u * per < nL1)
                    tile[(a + u * per) * ts + r] = v[u] & mask;
        }
    }
    __syncthreads();
}

// Transactions of a staged tile (tw words, words past the block zero) that
// contain the candidate: the AND of its items' tile rows, popcounted.
// The whole-row form for NW = 16, 8 or 4 words, in passes of at most eight
// words: the first item's words start the AND, and each further item's
// eight words are read together (all in flight, one wait) before they are
// ANDed.  (One accumulator per word of the whole row left room for only one
// read in flight, and a row cost eight LDS round trips.)  The item loop is
// not unrolled; the item list is a queue of 16-bit entries shifted by one
// item per iteration.
template <int NW>
__device__ __forceinline__ uint32_t and_tile_rows(const CandItems &ci, const uint64_t *tile,
                                                  uint32_t ts)
{
    constexpr int H = NW < 8 ? NW : 8;
    uint32_t sum = 0;
#pragma unroll
    for (int h = 0; h < NW; h += H) {
        uint32_t qv[KD / 2];
#pragma unroll
        for (int u = 0; u < KD / 2; ++u)
            qv[u] = ci.pk32[u];
        uint64_t acc[H];
        {
            const uint64_t *row = tile + (qv[0] & 0xFFFFu) * ts + h;
#pragma unroll
            for (int w = 0; w < H; ++w)
                acc[w] = row[w];
        }
#pragma unroll 1
        for (uint32_t t = 1; t < ci.k; ++t) {
#pragma unroll
            for (int u = 0; u < KD / 2; ++u)
                qv[u] = (qv[u] >> 16) | (u + 1 < KD / 2 ? qv[u + 1] << 16 : 0u);
            const uint64_t *row = tile + (qv[0] & 0xFFFFu) * ts + h;
            uint64_t v[H];
#pragma unroll
            for (int w = 0; w < H; ++w)
                v[w] = row[w];
#pragma unroll
            for (int w = 0; w < H; ++w)
                acc[w] &= v[w];
        }
#pragma unroll
        for (int w = 0; w < H; ++w)
            sum += (uint32_t)__popcll(acc[w]);
    }
    return sum;
}

// Any tile: the whole-row forms when the candidate has an item list and the
// tile a power-of-two width of at least 4 words; otherwise word by word.
__device__ __forceinline__ uint32_t and_tile_items(const Job *J, const CandItems &ci,
                                                   const uint64_t *tile, uint32_t ts, uint32_t nwt)
{
    if (ci.k <= (uint32_t)KD) {
        if (nwt == 16u)
            return and_tile_rows<16>(ci, tile, ts);
        if (nwt == 8u)
            return and_tile_rows<8>(ci, tile, ts);
        if (nwt == 4u)
            return and_tile_rows<4>(ci, tile, ts);
    }
    uint64_t acc[VT_MAXW];
#pragma unroll
    for (int w = 0; w < VT_MAXW; ++w)
        acc[w] = ~0ull;
    if (ci.k <= (uint32_t)KD) {
        uint32_t qv[KD / 2];
#pragma unroll
        for (int u = 0; u < KD / 2; ++u)
            qv[u] = ci.pk32[u];
#pragma unroll 1
        for (uint32_t t = 0; t < ci.k; ++t) {
            const uint64_t *row = tile + (qv[0] & 0xFFFFu) * ts;
#pragma unroll
            for (int u = 0; u < KD / 2; ++u)
                qv[u] = (qv[u] >> 16) | (u + 1 < KD / 2 ? qv[u + 1] << 16 : 0u);
#pragma unroll
            for (int w = 0; w < VT_MAXW; ++w)
                if ((uint32_t)w < nwt)
                    acc[w] &= row[w];
        }
    } else {
        if (ci.extra != NONE) {
            const uint64_t *row = tile + ci.extra * ts;
#pragma unroll
            for (int w = 0; w < VT_MAXW; ++w)
                if ((uint32_t)w < nwt)
                    acc[w] &= row[w];
        }
        uint64_t nzw = J->pnz[ci.wide];
        const uint64_t *cm = J->pmask + (uint64_t)ci.wide * J->W;
        while (nzw) {
            const uint32_t wd = (uint32_t)__builtin_ctzll(nzw);
            nzw &= nzw - 1;
            uint64_t bits = cm[wd];
            while (bits) {
                const uint32_t item = wd * 64u + (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1;
                const uint64_t *row = tile + J->l1pos[item] * ts;
#pragma unroll
                for (int w = 0; w < VT_MAXW; ++w)
                    if ((uint32_t)w < nwt)
                        acc[w] &= row[w];
            }
        }
    }
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < VT_MAXW; ++w)
        if ((uint32_t)w < nwt)
            sum += (uint32_t)__popcll(acc[w]);
    return sum;
}

// Nonzero 32-bit words of a pool entry's mask (the row-bitmap count's AND
// work per transaction, for the trace), with an optional extra item.
__device__ __forceinline__ uint32_t mask_dwords(const Job *J, uint32_t p, uint32_t extra)
{
    uint32_t words = 0;
    const uint64_t *cm = J->pmask + (uint64_t)p * J->W;
    uint64_t nzw = J->pnz[p] | (extra != NONE ? 1ull << (extra >> 6) : 0ull);
    while (nzw) {
        const uint32_t w = (uint32_t)__builtin_ctzll(nzw);
        nzw &= nzw - 1;
        const uint64_t v = cm[w] | (extra != NONE && w == (extra >> 6) ? 1ull << (extra & 63u) : 0ull);
        words += ((uint32_t)v != 0u) + ((uint32_t)(v >> 32) != 0u);
    }
    return words;
}

// Prune (Algorithm 4) and CheckFullPass (Algorithm 5) of NQ candidates per
// thread at this stop.  Record q (when valid) holds the candidate's support
// after this stop's count and the stops it has been counted on now
// (Algorithm 3's stop_I + 1).  A dashed circle with supp >= tau becomes a
// box (promoted at this epoch); otherwise, if supp + M * (stop_max - sc) <
// tau it is pruned (kept as known, never output or generated again).  One
// that has seen every block becomes solid; a box keeps its standing word
// then (the collection takes dashed and solid boxes alike: none is dashed
// once the run ends).  Survivors' records go to the next live list and new
// boxes to the next new-box list, with one append atomic per workgroup;
// the stop's statistics are summed over the workgroup.  words: nonzero
// mask dwords (row bitmaps' trace figure).  Every thread of the workgroup
// calls.
template <int NQ>
__device__ __forceinline__ void prune_core(const Job *J, JobState *st, LRec (&r)[NQ],
                                           const bool (&valid)[NQ], const uint32_t (&words)[NQ],
                                           uint32_t *sh_app)
{
    const uint32_t E = st->epoch;
    bool keep[NQ], promoted[NQ];
    uint32_t nwords = 0, nitems = 0, npro = 0, npru = 0, nsol = 0, rem = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        keep[q] = promoted[q] = false;
        if (!valid[q])
            continue;
        const uint32_t p = r[q].p, supp = r[q].supp, sc = r[q].sc;
        bool box = ((r[q].kb >> 16) & 1u) != 0u;
        nwords += words[q];
        nitems += r[q].kb & 0xFFFFu;
        bool pruned = false;
        if (!box) {
            if (supp >= J->tau) {
                box = true;
                promoted[q] = true;
                ++npro;
                r[q].kb |= 1u << 16;
                J->pstate[p] = standing(ST_DASHED_BOX, E);
            } else if ((uint64_t)supp + (uint64_t)J->Mp * (uint64_t)(J->stop_max - sc) <
                       (uint64_t)J->tau) {
                pruned = true;
                ++npru;
                J->pstate[p] = standing(ST_PRUNED, PROMO_NONE);
            }
        }
        if (!pruned) {
            if (sc == J->stop_max) {
                ++nsol;
                if (box)
                    J->psupp[p] = supp;  // its final count, for the collection
                else
                    J->pstate[p] = standing(ST_SOLID_CIRCLE, PROMO_NONE);
            } else {
                keep[q] = true;
                const uint32_t rm = J->stop_max - sc;
                rem = rm > rem ? rm : rem;
            }
        }
    }
    uint4 *next = st->parity ? J->live0 : J->live1;
    uint32_t *nbox = st->parity ? J->newbox0 : J->newbox1;
    uint32_t pos[NQ], npos[NQ];
    uint32_t v[6] = {nwords, nitems, npro, npru, nsol, rem};  // in CTR_* order
    block_append2_stats<NQ, 5>(J->ctrs + CTR_APPEND, keep, promoted, v,
                               J->ctrs + (blockIdx.x & (CTR_LINES - 1u)) * CTR_STRIDE, sh_app,
                               pos, npos);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (keep[q])
            store_rec(next, pos[q], r[q]);
        if (promoted[q])
            nbox[npos[q]] = r[q].p;
    }
}

// Work item of the survivors of the last stop (the current list) at this
// stop; each candidate's record is read once.  Bitsets, wave mode: WG/64
// candidates, one wave each, counted over the whole block, then pruned.
// Bitsets, tile mode: (group of WG * cpt candidates) x (chunk of tiles);
// each thread ANDs the tile rows of its candidates' items word by word and
// popcounts, so a 64-bit AND tests 64 transactions.  With one chunk per
// group the work item prunes its group; otherwise each chunk adds its
// partial count and one arrival to a word per candidate (list position),
// and the chunk that finds every other chunk's arrival there prunes that
// candidate with the total.  Row bitmaps: k_count has added the block's
// counts to the pool; ZP * WG survivors are pruned.  Every thread calls.
__device__ __forceinline__ void survivors_stop(const Job *J, uint32_t local, uint64_t *tile,
                                               uint32_t *sh_app)
{
    JobState *st = J->st;
    const uint4 *cur = st->parity ? J->live1 : J->live0;
    const uint32_t K = st->k_cur;
    if (J->layout == LAYOUT_ROWS) {
        LRec r[ZP];
        bool valid[ZP];
        uint32_t words[ZP];
#pragma unroll
        for (int q = 0; q < ZP; ++q) {
            const uint32_t c = local * (ZP * WG) + (uint32_t)q * WG + threadIdx.x;
            valid[q] = c < K;
            r[q] = valid[q] ? load_rec(cur, c) : LRec{};
        }
#pragma unroll
        for (int q = 0; q < ZP; ++q) {
            r[q].supp = valid[q] ? J->psupp[r[q].p] : 0u;  // k_count's running total
            r[q].sc += 1u;
            words[q] = valid[q] ? mask_dwords(J, r[q].p, NONE) : 0u;
        }
        prune_core<ZP>(J, st, r, valid, words, sh_app);
        return;
    }
    if (st->cmode == 1) {
        const uint32_t c = local * (WG / 64) + (threadIdx.x >> 6);
        LRec r[1];
        bool valid[1] = {false};
        uint32_t words[1] = {0u};
        r[0] = LRec{};
        if (c < K) {
            r[0] = load_rec(cur, __builtin_amdgcn_readfirstlane(c));
            const uint32_t cnt = count_wave_bitsets(J, st, rec_items(J, r[0]));
            r[0].supp += cnt;
            r[0].sc += 1u;
            valid[0] = (threadIdx.x & 63u) == 0u;  // the wave's first lane prunes it
        }
        prune_core<1>(J, st, r, valid, words, sh_app);
        return;
    }
    const uint32_t n_cg = st->n_ct;
    const uint32_t rc = local / n_cg;
    const uint32_t cg = local - rc * n_cg;
    const uint32_t tw = st->tw, ts = vert_tile_stride(tw);
    const uint32_t fw = st->fw, lw = st->lw;
    const uint32_t ntile = (lw - fw + tw) / tw;
    const uint32_t t0 = rc * st->rpi;
    const uint32_t t1 = t0 + st->rpi < ntile ? t0 + st->rpi : ntile;
    const uint32_t cpt = st->cpt;
    LRec r[VT_CPT];
    bool valid[VT_CPT];
    uint32_t cnt[VT_CPT];
    const uint32_t cpos0 = cg * cpt * WG + threadIdx.x;  // list position of candidate q: + q * WG
#pragma unroll
    for (int q = 0; q < VT_CPT; ++q) {
        const uint32_t c = cpos0 + (uint32_t)q * WG;
        valid[q] = (uint32_t)q < cpt && c < K;
        r[q] = valid[q] ? load_rec(cur, c) : LRec{};
        cnt[q] = 0;
    }
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t w0 = fw + t * tw;
        stage_tile(J, st, w0, tw, ts, tile);
        // one candidate at a time (the loop is not unrolled, so the compiler
        // decodes one candidate's item rows at a time): the head record is
        // counted, then the records rotate; VT_CPT rotations restore them
#pragma unroll 1
        for (int q = 0; q < VT_CPT; ++q) {
            if (valid[0])
                cnt[0] += and_tile_items(J, rec_items(J, r[0]), tile, ts, tw);
            const LRec r0 = r[0];
            const bool v0 = valid[0];
            const uint32_t c0 = cnt[0];
#pragma unroll
            for (int u = 0; u + 1 < VT_CPT; ++u) {
                r[u] = r[u + 1];
                valid[u] = valid[u + 1];
                cnt[u] = cnt[u + 1];
            }
            r[VT_CPT - 1] = r0;
            valid[VT_CPT - 1] = v0;
            cnt[VT_CPT - 1] = c0;
        }
    }
    if (st->n_ri > 1u) {
        // every chunk adds its count plus one arrival (2^32) to the
        // candidate's word; the chunk that finds the others' n_ri - 1
        // arrivals there is the last for that candidate: it has the total,
        // clears the word and prunes the candidate
        const unsigned long long last_arrivals = (unsigned long long)(st->n_ri - 1u) << 32;
#pragma unroll
        for (int q = 0; q < VT_CPT; ++q) {
            if (!valid[q])
                continue;
            unsigned long long *wq = J->pcnt + cpos0 + q * WG;
            const unsigned long long old = atomicAdd(wq, (1ull << 32) | cnt[q]);
            if ((old & ~0xFFFFFFFFull) == last_arrivals) {
                cnt[q] += (uint32_t)old;
                __hip_atomic_store(wq, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                valid[q] = false;  // a later chunk prunes it
            }
        }
    }
#pragma unroll
    for (int q = 0; q < VT_CPT; ++q) {
        if (valid[q] && (uint64_t)r[q].supp + cnt[q] > J->n) {  // a support never exceeds n
            atomicAdd(&st->asserts, 1u);
            __builtin_amdgcn_s_waitcnt(WAIT_VM0);  // complete before the arrival
        }
        r[q].supp += cnt[q];
        r[q].sc += 1u;
    }
    const uint32_t words[VT_CPT] = {};  // a figure of the row-bitmap count only
    prune_core<VT_CPT>(J, st, r, valid, words, sh_app);
}

// Copy W 64-bit words (the loads of a group of eight are issued together).
__device__ __forceinline__ void copy_words(uint64_t *dst, const uint64_t *src, uint32_t W)
{
    for (uint32_t w = 0; w < W; w += 8u) {
        uint64_t r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            r[u] = w + u < W ? src[w + u] : 0ull;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (w + u < W)
                dst[w + u] = r[u];
    }
}

// Item v of C = S | {a} in ascending order, given S's ascending list sw and
// a's place pos in C (v a compile-time constant after unrolling).
__device__ __forceinline__ uint32_t c_item(const uint32_t sw[KD / 2], uint32_t pos, uint32_t a,
                                           int v)
{
    const uint32_t lo = v < KD ? item_at(sw, v) : 0u;
    const uint32_t hi = v > 0 ? item_at(sw, v - 1) : 0u;
    return (uint32_t)v < pos ? lo : ((uint32_t)v == pos ? a : hi);
}

// Whether the k-item list pw equals C's ascending list (k + 1 items) without
// its element at position ct.
__device__ __forceinline__ bool list_equals(const uint32_t pw[KD / 2], const uint32_t sw[KD / 2],
                                            uint32_t pos, uint32_t a, uint32_t ct, uint32_t k)
{
    bool eq = true;
#pragma unroll
    for (int u = 0; u < KD; ++u)
        if ((uint32_t)u < k)
            eq &= item_at(pw, u) ==
                  ((uint32_t)u < ct ? c_item(sw, pos, a, u) : c_item(sw, pos, a, u + 1));
    return eq;
}

// Continue the linear probe for the k-itemset "C without position ct"
// (hash h) after slot s.  Only itemsets that existed when the stop began
// (index < base) are considered: one created at this stop is a fresh
// circle, never the box being looked for, and its pool entry may still be
// in flight from another workgroup, so it is skipped without being read.
__device__ __forceinline__ uint32_t probe_list(const Job *J, unsigned long long h, uint32_t k,
                                               const uint32_t sw[KD / 2], uint32_t pos, uint32_t a,
                                               uint32_t ct, uint32_t s, uint32_t base)
{
    const uint32_t tag = slot_tag(h, k);
    for (;;) {
        s = (s + 1u) & J->hmask;
        const unsigned long long v = slot_read(J, s);
        if (v == SLOT_EMPTY)
            return NONE;
        if ((uint32_t)v == tag && (uint32_t)(v >> 32) < base) {
            const uint32_t idx = (uint32_t)(v >> 32);
            uint32_t pw[KD / 2];
            load_items(J->pitems + (uint64_t)idx * KD, pw);
            if (list_equals(pw, sw, pos, a, ct, k))
                return idx;
        }
    }
}

// Whether standing word w is a box as of the end of the last stop (epoch
// E - 1): a dashed or solid box promoted before epoch E.  Prune at epoch E
// may be changing the word in this very launch; either value read answers
// the same.
__device__ __forceinline__ bool box_before(uint32_t w, uint32_t E)
{
    const uint32_t s = standing_state(w);
    return (s == ST_DASHED_BOX || s == ST_SOLID_BOX) && standing_promo(w) < E;
}

// MakeCandidates' admission test for C = S | {a}, |S| = k with k <= KD:
// every maximal subset (S \ {s_t}) | {a} other than S must have been a box
// at the end of the last stop, and none that drops an item larger than a
// may have been promoted at that stop (that subset generates C).  sw: S's
// ascending list; pos: a's place in C.  Subsets are checked in groups of
// SUBG whose hash-slot, item-list and standing loads are issued together.
constexpr int SUBG = 2;
__device__ __forceinline__ bool subsets_are_boxes(const Job *J, const uint32_t sw[KD / 2],
                                                  uint32_t k, uint32_t a, uint32_t pos,
                                                  unsigned long long hC, uint32_t base, uint32_t E)
{
    bool ok = true;
#pragma unroll
    for (int g = 0; g < KD; g += SUBG) {
        if (!ok || (uint32_t)g >= k)
            continue;
        unsigned long long h[SUBG], v[SUBG];
        uint32_t slot[SUBG];
#pragma unroll
        for (int u = 0; u < SUBG; ++u) {
            h[u] = hC ^ zob(item_at(sw, g + u));
            slot[u] = (uint32_t)h[u] & J->hmask;
            v[u] = (uint32_t)(g + u) < k ? slot_read(J, slot[u]) : SLOT_EMPTY;
        }
        uint32_t idx[SUBG], pw[SUBG][KD / 2], sst[SUBG];
#pragma unroll
        for (int u = 0; u < SUBG; ++u) {
            const bool hit = v[u] != SLOT_EMPTY && (uint32_t)v[u] == slot_tag(h[u], k) &&
                             (uint32_t)(v[u] >> 32) < base;
            idx[u] = hit ? (uint32_t)(v[u] >> 32) : NONE;
            if (hit) {
                load_items(J->pitems + (uint64_t)idx[u] * KD, pw[u]);
                sst[u] = J->pstate[idx[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < SUBG; ++u) {
            const int t = g + u;
            if ((uint32_t)t >= k)
                continue;
            const uint32_t drop = item_at(sw, t);
            const uint32_t ct = (uint32_t)t < pos ? (uint32_t)t : (uint32_t)t + 1u;
            uint32_t sub = idx[u], s2 = 0;
            if (sub != NONE && list_equals(pw[u], sw, pos, a, ct, k)) {
                s2 = sst[u];
            } else if (v[u] == SLOT_EMPTY) {
                sub = NONE;
            } else {
                sub = probe_list(J, h[u], k, sw, pos, a, ct, slot[u], base);
                if (sub != NONE)
                    s2 = J->pstate[sub];
            }
            if (sub == NONE || !box_before(s2, E))
                ok = false;
            else if (drop > a && standing_promo(s2) == E - 1u)
                ok = false;
        }
    }
    return ok;
}

// The same test for |S| = k > KD (no item list): S's items come from its
// bit mask and subsets are compared by mask.
__device__ __forceinline__ bool subsets_are_boxes_wide(const Job *J, uint32_t p, uint32_t k, uint32_t a,
                                       unsigned long long hC, uint32_t base, uint32_t E)
{
    const uint32_t W = J->W;
    const uint32_t i = J->l1[a];
    const uint64_t *S = J->pmask + (uint64_t)p * W;
    if ((S[i >> 6] >> (i & 63u)) & 1ull)
        return false;
    uint64_t nzw = J->pnz[p];
    while (nzw) {
        const uint32_t wd = (uint32_t)__builtin_ctzll(nzw);
        nzw &= nzw - 1;
        uint64_t bits = S[wd];
        while (bits) {
            const uint32_t xj = wd * 64u + (uint32_t)__builtin_ctzll(bits);
            bits &= bits - 1;
            const uint32_t sub = hash_find_sub(J, hC ^ zob(J->l1pos[xj]), k, S, i, xj, base);
            if (sub == NONE)
                return false;
            const uint32_t s2 = J->pstate[sub];
            if (!box_before(s2, E))
                return false;
            if (xj > i && standing_promo(s2) == E - 1u)
                return false;  // a subset dropping a larger item generates C
        }
    }
    return true;
}

// Workgroup-aggregated append that also reports each thread's rank among
// the workgroup's appends and their total: one atomic on ctr per workgroup.
// Every thread of the workgroup calls.  sh holds WG/64 + 2 words.
__device__ __forceinline__ void block_append_rank(uint32_t *ctr, bool pred, uint32_t *sh, uint32_t *base,
                                  uint32_t *rank, uint32_t *total)
{
    const unsigned long long b = __ballot(pred);
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 0)
        sh[wave] = (uint32_t)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < WG / 64; ++w) {
            const uint32_t c = sh[w];
            sh[w] = t;
            t += c;
        }
        sh[WG / 64] = t ? atomicAdd(ctr, t) : 0u;
        sh[WG / 64 + 1] = t;
    }
    __syncthreads();
    *rank = sh[wave] + (uint32_t)__popcll(b & lanemask_lt());
    *base = sh[WG / 64];
    *total = sh[WG / 64 + 1];
    __syncthreads();
}

// Counts of a candidate made at this stop, one wave each: its record in
// LDS (REC words: generating pool entry, added frequent item, size, a pad,
// then the item list when the size is at most KD).
constexpr uint32_t REC = 12;

// MakeCandidates for one chunk of WG (new box, frequent item) pairs of job J,
// then CountSupport, Prune and CheckFullPass of what it made.  For each
// itemset S promoted at the last stop and each frequent item a not in S,
// C = S | {a} is admitted when every maximal proper subset of C was a box
// at the end of that stop.  C is produced by exactly one of its subsets
// C \ {i} promoted at that stop: the one with the largest i, so no
// candidate is generated twice and no set of already-known itemsets is
// needed (an itemset whose subsets were all boxes before was generated
// earlier).  C is counted on this stop's block at once, by the waves of the
// workgroup (few candidates: one wave each, records in LDS) or by its
// threads over LDS tiles of the block (many), and pruned as a dashed circle
// seen on one block.  Every thread of the workgroup calls.
__device__ __forceinline__ void candgen_stop(const Job *J, unsigned long long chunk, uint64_t *lds, uint32_t *sh_app,
                             uint32_t *sh_cnt)
{
    JobState *st = J->st;
    const uint32_t W = J->W;
    const uint32_t nL1 = st->nL1;
    const uint32_t base = st->pool_base;
    const uint32_t E = st->epoch;
    const uint32_t *nb_last = st->parity ? J->newbox1 : J->newbox0;
    const unsigned long long x = chunk * WG + threadIdx.x;
    const bool valid = x < (unsigned long long)st->n_prev * nL1;
    bool gen = false;
    uint32_t p = 0, a = 0, k = 0;
    unsigned long long hC = 0;
    uint32_t sw[KD / 2];  // S's frequent-item indices, ascending (k <= KD)
    uint32_t pos = 0;     // a's place in C = S | {a}
#pragma unroll
    for (int t = 0; t < KD / 2; ++t)
        sw[t] = 0u;
    if (valid) {
        // (32-bit division whenever the index fits: a 64-bit one is far longer)
        const uint32_t q = x <= 0xFFFFFFFFull ? (uint32_t)x / nL1 : (uint32_t)(x / nL1);
        a = (uint32_t)x - q * nL1;  // the new item, as a frequent-item index
        p = nb_last[q];
        k = J->pk[p];
        const unsigned long long hS = J->phash[p];
        if (k <= (uint32_t)KD) {
            load_items(J->pitems + (uint64_t)p * KD, sw);
            // a's place in S's ascending list; a already in S: no extension
            bool in = false;
#pragma unroll
            for (int t = 0; t < KD; ++t)
                if ((uint32_t)t < k) {
                    const uint32_t v = item_at(sw, t);
                    pos += v < a ? 1u : 0u;
                    in |= v == a;
                }
            hC = hS ^ zob(a);
            if (!in && k == 2u && !J->classic) {
                // C's other maximal subsets {s0, a} and {s1, a} are pair
                // candidates found at their lexicographic index (pairs
                // are created up front, except in classic mode)
                const uint32_t s0 = item_at(sw, 0), s1 = item_at(sw, 1);
                const uint32_t lo0 = s0 < a ? s0 : a, hi0 = s0 < a ? a : s0;
                const uint32_t lo1 = s1 < a ? s1 : a, hi1 = s1 < a ? a : s1;
                const uint32_t sub0 = lo0 * nL1 - lo0 * (lo0 + 1u) / 2u + (hi0 - lo0 - 1u);
                const uint32_t sub1 = lo1 * nL1 - lo1 * (lo1 + 1u) / 2u + (hi1 - lo1 - 1u);
                const uint32_t w0 = J->pstate[sub0], w1 = J->pstate[sub1];
                gen = box_before(w0, E) && box_before(w1, E) &&
                      // a subset dropping a larger item than a, promoted
                      // at the last stop, generates C instead
                      !(s1 > a && standing_promo(w0) == E - 1u) &&
                      !(s0 > a && standing_promo(w1) == E - 1u);
            } else if (!in) {
                gen = subsets_are_boxes(J, sw, k, a, pos, hC, base, E);
            }
        } else {
            hC = hS ^ zob(a);
            gen = subsets_are_boxes_wide(J, p, k, a, hC, base, E);
        }
    }
    // New entries are pool slots from pool_base on, counted in the stop's
    // pool-growth counter.  Lookups in this launch never read them (see
    // probe_list), so no fence is needed before publishing them in the hash
    // table.
    uint32_t wg_base, rank, g;
    block_append_rank(J->ctrs + CTR_GEN, gen, sh_app, &wg_base, &rank, &g);
    wg_base += base;
    const uint32_t np = wg_base + rank;
    const bool stored = gen && np < J->cap;
    const uint32_t kc = k + 1u;
    uint32_t cw[KD / 2];  // C's frequent-item indices, ascending (kc <= KD)
#pragma unroll
    for (int u = 0; u < KD / 2; ++u)
        cw[u] = 0u;
    if (stored) {
#pragma unroll
        for (int u = 0; u < KD / 2; ++u)
            cw[u] = ((uint32_t)(2 * u) <= k ? c_item(sw, pos, a, 2 * u) : 0u) |
                    (((uint32_t)(2 * u + 1) <= k ? c_item(sw, pos, a, 2 * u + 1) : 0u) << 16);
        const uint32_t i = J->l1[a];
        copy_words(J->pmask + (uint64_t)np * W, J->pmask + (uint64_t)p * W, W);
        J->pmask[(uint64_t)np * W + (i >> 6)] |= 1ull << (i & 63u);
        J->phash[np] = hC;
        J->pnz[np] = J->pnz[p] | (1ull << (i >> 6));
        J->pk[np] = kc;
        J->pstate[np] = standing(ST_DASHED_CIRCLE, PROMO_NONE);  // Prune below may change it
        if (kc <= (uint32_t)KD) {
            uint4 *ci = (uint4 *)(J->pitems + (uint64_t)np * KD);
            ci[0] = make_uint4(cw[0], cw[1], cw[2], cw[3]);
            ci[1] = make_uint4(cw[4], cw[5], cw[6], cw[7]);
        }
        hash_insert(J, hC, kc, np);
    }
    // candidates of this workgroup stored in the pool (ranks 0 .. gs-1)
    const uint32_t gs = wg_base >= J->cap ? 0u : (g < J->cap - wg_base ? g : J->cap - wg_base);
    if (gs == 0u)
        return;
    // CountSupport of the new candidates on this stop's block
    uint32_t cnt = 0;
    const uint32_t nwords = st->lw - st->fw + 1u;
    const bool vert = J->layout == LAYOUT_VERTICAL;
    const uint32_t tw = vert_tile_words(nL1, VT_MAXW);
    const uint32_t ntile = (nwords + tw - 1u) / tw;
    const uint32_t wave_passes = (gs + WG / 64 - 1u) / (WG / 64) * ((nwords + 191u) / 192u);
    if (vert && 2u * ntile < wave_passes) {
        // many: each thread ANDs its own candidate's rows over LDS tiles
        CandItems ci{};
        ci.k = kc;
        ci.wide = p;
        ci.extra = kc > (uint32_t)KD ? a : NONE;
#pragma unroll
        for (int u = 0; u < KD / 2; ++u)
            ci.pk32[u] = cw[u];
        const uint32_t ts = vert_tile_stride(tw);
        for (uint32_t t = 0; t < ntile; ++t) {
            const uint32_t w0 = st->fw + t * tw;
            stage_tile(J, st, w0, tw, ts, lds);
            if (stored)
                cnt += and_tile_items(J, ci, lds, ts, tw);
        }
    } else {
        // few: one wave per candidate, the candidates' records in LDS
        uint32_t *rec = (uint32_t *)lds;
        if (stored) {
            uint32_t *r = rec + rank * REC;
            r[0] = p;
            r[1] = a;
            r[2] = kc;
            r[3] = 0u;
#pragma unroll
            for (int u = 0; u < KD / 2; ++u)
                r[4 + u] = cw[u];
        }
        __syncthreads();
        for (uint32_t r0 = threadIdx.x >> 6; r0 < gs; r0 += WG / 64) {
            const uint32_t *r = rec + r0 * REC;
            uint32_t c;
            if (vert) {
                CandItems ci;
                ci.wide = r[0];
                ci.k = r[2];
                ci.extra = ci.k > (uint32_t)KD ? r[1] : NONE;
#pragma unroll
                for (int u = 0; u < KD / 2; ++u)
                    ci.pk32[u] = r[4 + u];
                c = count_wave_bitsets(J, st, ci);
            } else {
                c = count_wave_rows(J, st, r[0], J->l1[r[1]]);
            }
            if ((threadIdx.x & 63u) == 0)
                sh_cnt[r0] = c;
        }
        __syncthreads();
        cnt = stored ? sh_cnt[rank] : 0u;
    }
    // Prune and CheckFullPass: a dashed circle counted on one block
    LRec r[1];
    r[0].p = np;
    r[0].supp = cnt;
    r[0].sc = 1u;
    r[0].kb = kc;
#pragma unroll
    for (int u = 0; u < KR / 2; ++u)
        r[0].it[u] = cw[u];  // larger itemsets' lists are read from the pool
    bool ok[1] = {stored};
    uint32_t words[1] = {stored && !vert ? mask_dwords(J, p, J->l1[a]) : 0u};
    if (stored && !vert)
        J->psupp[np] = cnt;  // row bitmaps keep the running total in the pool
    prune_core<1>(J, st, r, ok, words, sh_app);
}

// One stop for every job in the table: MakeCandidates chunks (with the new
// candidates' count and prune) of every job first, then the survivors' work
// items of every job.  The last workgroup to finish completes the stop for
// every job, begins its next one and plans the next launch.  Three waves per
// SIMD (what the LDS tile allows).
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_stop(
    const Job *__restrict__ jobs, Plan *plan)
{
    __shared__ uint64_t tile[VT_WORDS];
    __shared__ uint32_t sh_app[2 * VT_CPT * (WG / 64) + 2 + 6 * (WG / 64)];
    __shared__ uint32_t sh_cnt[WG];
    __shared__ unsigned long long shc[WG / 64];
    __shared__ uint32_t sh_flag;
    const uint32_t njobs = plan->njobs;
    const unsigned long long ncg = plan->total_cg;
    const unsigned long long total = ncg + plan->total_v;
    for (unsigned long long it = blockIdx.x; it < total; it += gridDim.x) {
        if (it < ncg) {
            const uint32_t j = find_job(plan->pre_cg, njobs, it);
            // job 0's prefix is 0: no load (and no wait for it) on a single job
            candgen_stop(jobs + j, j ? it - plan->pre_cg[j] : it, tile, sh_app, sh_cnt);
        } else {
            const uint32_t v = (uint32_t)(it - ncg);
            const uint32_t j = find_job(plan->pre_countv, njobs, v);
            survivors_stop(jobs + j, j ? v - plan->pre_countv[j] : v, tile, sh_app);
        }
    }
    // Everything the serial part reads from this launch's other workgroups
    // is a device-scope atomic (the counter lines: pool growth, list
    // appends, statistics; asserts) and is read with device-scope atomic
    // loads.  Each is complete before its workgroup passes the barrier below:
    // the returning ones because their results were used, the no-return
    // ones (Prune's statistics, asserts) because the thread that issued them
    // waited for them (s_waitcnt vmcnt(0): a workgroup barrier alone does
    // not wait for memory operations).  Plain stores of this launch
    // (records, standings, counts) are read only by later launches, so the
    // workgroup arrives without waiting for them.  A device-scope release
    // would also write back this XCD's L2, which costs tens of microseconds
    // per launch.
    __syncthreads();
    if (threadIdx.x == 0)
        sh_flag = arrive_last(plan->tickets, total < gridDim.x ? (total ? (uint32_t)total : 1u)
                                                              : gridDim.x);
    __syncthreads();
    if (sh_flag)
        settle_and_plan(jobs, plan, true, false, (uint32_t *)tile, shc,
                        (PlanTune *)(tile + VT_WORDS / 2));
}

// Gather solid boxes (the output L without its 1-itemsets), each with its
// canonical sort key.
__global__ __launch_bounds__(WG) void k_collect(const Job *__restrict__ jobs)
{
    const Job *J = jobs + blockIdx.y;
    const uint32_t pool_n = J->st->pool_n < J->cap ? J->st->pool_n : J->cap;
    const uint32_t W = J->W;
    for (uint32_t b = blockIdx.x * WG; b < pool_n; b += gridDim.x * WG) {
        const uint32_t p = b + threadIdx.x;
        // a box keeps its dashed standing word when it becomes solid; the run
        // has ended, so every box is solid
        const uint32_t sw = p < pool_n ? standing_state(J->pstate[p]) : ST_PRUNED;
        const bool box = sw == ST_SOLID_BOX || sw == ST_DASHED_BOX;
        const uint32_t pos = wave_append(J->out_n, box, true);
        if (box) {
            const uint64_t *pm = J->pmask + (uint64_t)p * W;
            for (uint32_t w = 0; w < W; ++w)
                J->out_mask[(uint64_t)pos * W + w] = pm[w];
            J->out_cnt[pos] = J->psupp[p];
            unsigned long long hi, lo;
            canon_key(pm, W, J->pk[p], &hi, &lo);
            J->out_key[2 * (uint64_t)pos] = hi;
            J->out_key[2 * (uint64_t)pos + 1] = lo;
        }
    }
}

// Fill n 32-bit words with v (a kernel instead of a memset node, so that a
// caller may capture the work into a graph).
__global__ __launch_bounds__(WG) void k_fill32(uint32_t *__restrict__ p, uint32_t v, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * WG)
        p[i] = v;
}

// Item lists (CSR) to bit rows, one thread per row.
__global__ __launch_bounds__(WG) void k_pack_lists(const uint32_t *__restrict__ items,
                                                   const uint64_t *__restrict__ offsets,
                                                   uint64_t n, uint32_t W, uint64_t *rows)
{
    for (uint64_t r = (uint64_t)blockIdx.x * WG + threadIdx.x; r < n;
         r += (uint64_t)gridDim.x * WG) {
        uint64_t *row = rows + r * W;
        for (uint32_t w = 0; w < W; ++w)
            row[w] = 0;
        for (uint64_t e = offsets[r]; e < offsets[r + 1]; ++e) {
            const uint32_t it = items[e];
            row[it >> 6] |= 1ull << (it & 63u);
        }
    }
}

__global__ __launch_bounds__(WG) void k_check_padding(const uint64_t *__restrict__ rows,
                                                      uint64_t n, uint32_t m, uint32_t *bad)
{
    const uint32_t W = (m + 63u) / 64u;
    const uint64_t pad = ~((1ull << (m & 63u)) - 1ull);
    for (uint64_t r = (uint64_t)blockIdx.x * WG + threadIdx.x; r < n;
         r += (uint64_t)gridDim.x * WG)
        if (rows[r * W + W - 1] & pad)
            atomicOr(bad, 1u);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

uint32_t grid_for(unsigned long long work, uint32_t per, uint32_t cap)
{
    unsigned long long g = (work + per - 1) / per;
    if (g < 1)
        g = 1;
    return (uint32_t)(g < cap ? g : cap);
}
}  // namespace

void launch_first_pass(const Job *jobs, const Plan *plan, unsigned long long total_chunks,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_first_pass, dim3(grid_for(total_chunks, 1, 4096)), dim3(WG), 0, s, jobs,
                       plan, total_chunks);
}

void launch_first_pass_vert(const Job *jobs, const Plan *plan, unsigned long long total_chunks,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_first_pass_vert, dim3(grid_for(total_chunks, 1, 8192)), dim3(WG), 0, s,
                       jobs, plan, total_chunks);
}

void launch_transpose(const uint64_t *rows, uint64_t n, uint32_t m, uint64_t *vert, uint32_t nw,
                      hipStream_t s)
{
    const uint32_t W = (m + 63u) / 64u;
    const uint64_t units = (uint64_t)((nw + TR_G - 1u) / TR_G) * ((W + TR_W - 1u) / TR_W);
    const uint32_t per_xcd = (uint32_t)((units + N_XCD - 1) / N_XCD);
    if (units == 0)
        return;
    hipLaunchKernelGGL(k_transpose, dim3(per_xcd * N_XCD), dim3(WG), 0, s, rows, n, m, W, vert,
                       nw, per_xcd);
}

void launch_l1_and_pairs_prepare(const Job *jobs, const Plan *, uint32_t njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_l1, dim3(njobs), dim3(WG), 0, s, jobs);
}

void launch_init_pairs(const Job *jobs, const Plan *plan, unsigned long long total, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_pairs, dim3(grid_for(total, WG, 8192)), dim3(WG), 0, s, jobs, plan,
                       total);
}

void launch_gather_vert(const Job *jobs, const Plan *plan, unsigned long long total, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_vert, dim3(grid_for(total, WG, 16384)), dim3(WG), 0, s, jobs,
                       plan, total);
}

void launch_begin(const Job *jobs, Plan *plan, hipStream_t s)
{
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(WG), 0, s, jobs, plan);
}

void launch_step(const Job *jobs, const Plan *plan, hipStream_t s, bool rows, bool vert,
                 uint32_t count_grid, hipEvent_t before, hipEvent_t after)
{
    Plan *pl = const_cast<Plan *>(plan);
    (void)vert;  // the bitset count is part of the stop kernel
    if (before)
        (void)hipEventRecord(before, s);
    if (rows)
        hipLaunchKernelGGL(k_count, dim3(count_grid), dim3(WG), 0, s, jobs, plan);
    hipLaunchKernelGGL(k_stop, dim3(count_grid), dim3(WG), 0, s, jobs, pl);
    if (after)
        (void)hipEventRecord(after, s);
}

void launch_collect(const Job *jobs, const Plan *, uint32_t njobs, hipStream_t s)
{
    hipLaunchKernelGGL(k_collect, dim3(64, njobs), dim3(WG), 0, s, jobs);
}

void launch_fill32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s)
{
    if (n)
        hipLaunchKernelGGL(k_fill32, dim3(grid_for(n, WG, 4096)), dim3(WG), 0, s, p, v, n);
}

void launch_pack_lists(const uint32_t *items, const uint64_t *offsets, uint64_t n, uint32_t W,
                       uint64_t *rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_lists, dim3(grid_for(n, WG, 16384)), dim3(WG), 0, s, items, offsets,
                       n, W, rows);
}

void launch_check_padding(const uint64_t *rows, uint64_t n, uint32_t m, uint32_t *bad,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_check_padding, dim3(grid_for(n, WG, 16384)), dim3(WG), 0, s, rows, n, m,
                       bad);
}

}  // namespace dic
