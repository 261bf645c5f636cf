/*
 * dic_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain serial CPU reference for frequent itemset mining (Zymbler, "Parallel
 * Algorithm for Frequent Itemset Mining on Intel Many-core Systems").  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * use it.  It shares no code with the GPU library.
 *
 * What each function follows:
 *   oracle_tau          -- Section 1: support is a fraction of transactions;
 *                          the integer threshold is the smallest count that
 *                          reaches it (reading: ceil with a near-integer guard).
 *   oracle_dic          -- Section 4.2: Algorithm 2 (driver), FirstPass (full
 *                          first pass, pairs of frequent items), Algorithm 3
 *                          (CountSupport), Algorithm 4 (Prune), MakeCandidates
 *                          (join of boxes by bitwise OR, no pseudocode in the
 *                          paper) and Algorithm 5 (CheckFullPass), in that
 *                          order at every stop; Section 3 for the four sets
 *                          and the stop/rewind schedule.
 *   oracle_apriori      -- Section 3: level-wise Apriori (join, a-priori
 *                          prune, count), an independent cross-check.
 *   oracle_bruteforce / oracle_tidlist -- the problem statement of Section 1
 *                          written out (every itemset, or a depth-first walk
 *                          that stops where support falls below threshold,
 *                          which is exact because support is anti-monotone).
 *
 * Everything is integer except minsup, which becomes the integer threshold
 * once.  No blocking, no layout tricks.  Built plainly it is serial; built
 * with OpenMP (the benchmark's CPU baseline) the one loop the paper runs in
 * parallel -- each live candidate's count over a block, Algorithm 3 --
 * is shared among threads, with identical results.
 */
#include "dic_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_result {
    uint32_t W;
    uint64_t size;
    uint64_t *masks;  /* size * W */
    uint32_t *counts; /* size */
    or_stats stats;
    or_stop *trace;
    uint64_t trace_len;
};

/* ------------------------------------------------------------------------ */
/* threshold                                                                 */
/* ------------------------------------------------------------------------ */

int oracle_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

int oracle_tau(double minsup, uint64_t n, uint64_t *tau)
{
    if (!tau || n == 0 || !(minsup > 0.0)) /* NaN fails the comparison too */
        return OR_E_INVAL;
    double x = minsup * (double)n;
    uint64_t t;
    if (!(x < 9007199254740992.0)) { /* 2^53 and beyond, or +inf */
        t = n + 1;
    } else {
        double r = nearbyint(x);
        double scale = x > 1.0 ? x : 1.0;
        if (fabs(x - r) <= 1e-9 * scale)
            t = (uint64_t)r;
        else
            t = (uint64_t)ceil(x);
    }
    if (t > n + 1)
        t = n + 1; /* nothing can reach it; keep the value bounded */
    if (t < 1)
        t = 1;
    *tau = t;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* itemset helpers                                                           */
/* ------------------------------------------------------------------------ */

/* I is contained in T: BitMask(I) AND BitMask(T) = BitMask(I) (Section 4.1). */
static int is_subset(const uint64_t *I, const uint64_t *T, uint32_t W)
{
    for (uint32_t w = 0; w < W; ++w)
        if ((I[w] & T[w]) != I[w])
            return 0;
    return 1;
}

static uint32_t n_items(const uint64_t *I, uint32_t W)
{
    uint32_t k = 0;
    for (uint32_t w = 0; w < W; ++w)
        k += (uint32_t)__builtin_popcountll(I[w]);
    return k;
}

static int has_item(const uint64_t *I, uint32_t p) { return (int)((I[p >> 6] >> (p & 63)) & 1u); }

/* Canonical order: size ascending, then ascending item lists lexicographic. */
static int mask_cmp(const uint64_t *A, const uint64_t *B, uint32_t W)
{
    uint32_t ka = n_items(A, W), kb = n_items(B, W);
    if (ka != kb)
        return ka < kb ? -1 : 1;
    /* walk both item lists in ascending order; first difference decides */
    uint32_t wa = 0, wb = 0;
    uint64_t xa = A[0], xb = B[0];
    for (uint32_t i = 0; i < ka; ++i) {
        while (xa == 0) xa = A[++wa];
        while (xb == 0) xb = B[++wb];
        uint32_t ia = wa * 64u + (uint32_t)__builtin_ctzll(xa);
        uint32_t ib = wb * 64u + (uint32_t)__builtin_ctzll(xb);
        if (ia != ib)
            return ia < ib ? -1 : 1;
        xa &= xa - 1;
        xb &= xb - 1;
    }
    return 0;
}

static uint32_t canon_W;
static const uint64_t *canon_masks;
static int canon_cmp(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return mask_cmp(canon_masks + a * canon_W, canon_masks + b * canon_W, canon_W);
}

/* Build a result from q itemsets (masks q*W, counts q), sorting canonically. */
static int make_result(uint32_t W, uint64_t q, const uint64_t *masks, const uint32_t *counts,
                       or_result **out)
{
    or_result *r = (or_result *)calloc(1, sizeof(*r));
    if (!r)
        return OR_E_NOMEM;
    r->W = W;
    r->size = q;
    r->masks = (uint64_t *)malloc((q ? q : 1) * W * sizeof(uint64_t));
    r->counts = (uint32_t *)malloc((q ? q : 1) * sizeof(uint32_t));
    uint64_t *perm = (uint64_t *)malloc((q ? q : 1) * sizeof(uint64_t));
    if (!r->masks || !r->counts || !perm) {
        free(perm);
        oracle_result_free(r);
        return OR_E_NOMEM;
    }
    for (uint64_t i = 0; i < q; ++i)
        perm[i] = i;
    canon_W = W;
    canon_masks = masks;
    qsort(perm, q, sizeof(uint64_t), canon_cmp);
    uint64_t kmax = 0;
    for (uint64_t i = 0; i < q; ++i) {
        memcpy(r->masks + i * W, masks + perm[i] * W, W * sizeof(uint64_t));
        r->counts[i] = counts[perm[i]];
        uint64_t k = n_items(masks + perm[i] * W, W);
        if (k > kmax)
            kmax = k;
    }
    free(perm);
    r->stats.n_frequent = q;
    r->stats.k_max = kmax;
    *out = r;
    return OR_OK;
}

static int check_db(const uint64_t *rows, uint64_t n, uint32_t m)
{
    if (!rows || n == 0 || m == 0 || n >= 0xFFFFFFFFull)
        return OR_E_INVAL;
    uint32_t W = (m + 63u) / 64u;
    uint32_t tail = m & 63u;
    if (tail) {
        uint64_t pad = ~((1ull << tail) - 1ull);
        for (uint64_t r = 0; r < n; ++r)
            if (rows[r * W + W - 1] & pad)
                return OR_E_INVAL;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* growable arrays                                                           */
/* ------------------------------------------------------------------------ */

static int grow(void **p, uint64_t *cap, uint64_t need, size_t elem)
{
    if (need <= *cap)
        return 1;
    uint64_t c = *cap ? *cap : 64;
    while (c < need)
        c *= 2;
    void *q = realloc(*p, c * elem);
    if (!q)
        return 0;
    *p = q;
    *cap = c;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* KNOWN: every itemset ever created, with its current standing              */
/* ------------------------------------------------------------------------ */

enum { K_EMPTY = 0, K_CIRCLE = 1, K_BOX = 2, K_INFREQUENT = 3 };

typedef struct {
    uint32_t W;
    uint64_t cap, used;
    uint64_t *keys;
    uint8_t *state;
} known_map;

static uint64_t fnv1a(const uint64_t *key, uint32_t W)
{
    uint64_t h = 1469598103934665603ull;
    for (uint32_t w = 0; w < W; ++w)
        for (int b = 0; b < 8; ++b) {
            h ^= (key[w] >> (8 * b)) & 0xFFu;
            h *= 1099511628211ull;
        }
    return h;
}

static int known_init(known_map *k, uint32_t W, uint64_t cap)
{
    uint64_t c = 1024;
    while (c < cap)
        c *= 2;
    k->W = W;
    k->cap = c;
    k->used = 0;
    k->keys = (uint64_t *)calloc(c * W, sizeof(uint64_t));
    k->state = (uint8_t *)calloc(c, 1);
    return k->keys && k->state;
}

static void known_free(known_map *k)
{
    free(k->keys);
    free(k->state);
}

static uint64_t known_slot(const known_map *k, const uint64_t *key)
{
    uint64_t s = fnv1a(key, k->W) & (k->cap - 1);
    while (k->state[s] != K_EMPTY && memcmp(k->keys + s * k->W, key, k->W * sizeof(uint64_t)))
        s = (s + 1) & (k->cap - 1);
    return s;
}

static int known_get(const known_map *k, const uint64_t *key)
{
    return k->state[known_slot(k, key)];
}

static int known_set(known_map *k, const uint64_t *key, int st)
{
    if (2 * (k->used + 1) > k->cap) {
        known_map bigger;
        if (!known_init(&bigger, k->W, 2 * k->cap))
            return 0;
        for (uint64_t s = 0; s < k->cap; ++s)
            if (k->state[s] != K_EMPTY) {
                uint64_t t = known_slot(&bigger, k->keys + s * k->W);
                memcpy(bigger.keys + t * k->W, k->keys + s * k->W, k->W * sizeof(uint64_t));
                bigger.state[t] = k->state[s];
                bigger.used++;
            }
        known_free(k);
        *k = bigger;
    }
    uint64_t s = known_slot(k, key);
    if (k->state[s] == K_EMPTY) {
        memcpy(k->keys + s * k->W, key, k->W * sizeof(uint64_t));
        k->used++;
    }
    k->state[s] = (uint8_t)st;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Dynamic Itemset Counting                                                  */
/* ------------------------------------------------------------------------ */

/* A candidate under count (Section 3's dashed itemsets) or a finished one
 * (solid): where its mask sits in the arena, its size, how many blocks it has
 * been counted on, how many transactions of those blocks contain it, and its
 * standing.  A candidate is erased by setting gone. */
typedef struct {
    uint64_t at;
    uint32_t size;
    uint64_t blocks;
    uint64_t hits;
    uint8_t reached; /* its count reached the threshold (a box) */
    uint8_t gone;
} cand;

typedef struct {
    uint32_t W;
    uint64_t *arena; /* every mask ever created, W words each */
    uint64_t arena_n, arena_cap;
    cand *live; /* candidates still counted block by block */
    uint64_t nlive, caplive;
    cand *done; /* counted over a full pass (and the first pass's 1-itemsets) */
    uint64_t ndone, capdone;
    known_map seen; /* every itemset ever created, with its standing */
    uint64_t *fresh; /* arena offsets of the candidates that reached the threshold at this stop */
    uint64_t nfresh, capfresh;
} miner;

static const uint64_t *mask_of(const miner *S, const cand *c) { return S->arena + c->at; }

static int arena_put(miner *S, const uint64_t *mask, uint64_t *at)
{
    if (!grow((void **)&S->arena, &S->arena_cap, S->arena_n + S->W, sizeof(uint64_t)))
        return 0;
    memcpy(S->arena + S->arena_n, mask, S->W * sizeof(uint64_t));
    *at = S->arena_n;
    S->arena_n += S->W;
    return 1;
}

static int cand_push(cand **v, uint64_t *n, uint64_t *cap, cand c)
{
    if (!grow((void **)v, cap, *n + 1, sizeof(cand)))
        return 0;
    (*v)[(*n)++] = c;
    return 1;
}

/* A new candidate: counted on no block yet, known as not (yet) frequent. */
static int start_candidate(miner *S, const uint64_t *mask, uint32_t size)
{
    cand c;
    memset(&c, 0, sizeof(c));
    c.size = size;
    if (!arena_put(S, mask, &c.at) || !cand_push(&S->live, &S->nlive, &S->caplive, c))
        return 0;
    return known_set(&S->seen, mask, K_CIRCLE);
}

/* Drop the erased candidates from the live list, keeping the others' order. */
static void sweep_live(miner *S)
{
    uint64_t j = 0;
    for (uint64_t i = 0; i < S->nlive; ++i)
        if (!S->live[i].gone)
            S->live[j++] = S->live[i];
    S->nlive = j;
}

/* Each maximal proper subset of C (C minus one item) is known as frequent. */
static int maximal_subsets_frequent(const miner *S, const uint64_t *C, uint64_t *scratch)
{
    for (uint32_t w = 0; w < S->W; ++w)
        for (uint64_t rest = C[w]; rest; rest &= rest - 1) {
            memcpy(scratch, C, S->W * sizeof(uint64_t));
            scratch[w] &= ~(rest & (~rest + 1));
            if (known_get(&S->seen, scratch) != K_BOX)
                return 0;
        }
    return 1;
}

/* Algorithm 3: every live candidate is counted on the block [lo, hi): one
 * more block seen, plus the block's transactions that contain it.  Each
 * candidate's count is its own, so the candidates may be shared among
 * threads (the loop the paper parallelises; built without OpenMP it runs
 * serially). */
static void count_block_phase(miner *S, const uint64_t *rows, uint64_t lo, uint64_t hi)
{
    const uint32_t W = S->W;
    const int64_t nl = (int64_t)S->nlive;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t i = 0; i < nl; ++i) {
        cand *c = &S->live[i];
        const uint64_t *mask = mask_of(S, c);
        uint64_t h = 0;
        for (uint64_t t = lo; t < hi; ++t)
            h += (uint64_t)is_subset(mask, rows + t * W, W);
        c->blocks += 1;
        c->hits += h;
    }
}

/* Algorithm 4 on the live circles, in list order.  One whose count reached
 * tau becomes a box and is noted as fresh.  One that cannot reach tau any
 * more is erased (and known as infrequent): even if every transaction of
 * the blocks it has not been counted on held it -- at most Mp per block,
 * nblk blocks in a pass -- it would fall short.  Every live circle that
 * strictly contains an erased one goes with it. */
static int threshold_phase(miner *S, uint64_t tau, uint64_t Mp, uint64_t nblk, or_stop *tr,
                           or_stats *st)
{
    const uint32_t W = S->W;
    S->nfresh = 0;
    uint32_t widest = 0; /* no circle of this size or less has a proper superset */
    for (uint64_t i = 0; i < S->nlive; ++i)
        if (!S->live[i].reached && S->live[i].size > widest)
            widest = S->live[i].size;
    for (uint64_t i = 0; i < S->nlive; ++i) {
        cand *c = &S->live[i];
        if (c->reached || c->gone)
            continue;
        if (c->hits >= tau) {
            c->reached = 1;
            tr->promoted++;
            if (!known_set(&S->seen, mask_of(S, c), K_BOX) ||
                !grow((void **)&S->fresh, &S->capfresh, S->nfresh + 1, sizeof(uint64_t)))
                return 0;
            S->fresh[S->nfresh++] = c->at;
            continue;
        }
        const uint64_t best = c->hits + Mp * (nblk - c->blocks);
        if (best >= tau)
            continue;
        c->gone = 1;
        tr->pruned++;
        if (!known_set(&S->seen, mask_of(S, c), K_INFREQUENT))
            return 0;
        for (uint64_t j = 0; c->size < widest && j < S->nlive; ++j) {
            cand *d = &S->live[j];
            if (j == i || d->reached || d->gone || d->size <= c->size ||
                !is_subset(mask_of(S, c), mask_of(S, d), W))
                continue;
            d->gone = 1;
            st->superset_prunes++;
            tr->pruned++;
            if (!known_set(&S->seen, mask_of(S, d), K_INFREQUENT))
                return 0;
        }
    }
    sweep_live(S);
    return 1;
}

/* MakeCandidates, reading 0: each box that reached tau at this stop, grown
 * by each frequent item it lacks, is a new candidate when that itemset is new
 * and all its maximal proper subsets are frequent. */
static int extend_fresh_phase(miner *S, const uint32_t *freq, uint64_t nfreq, uint64_t *C,
                              uint64_t *scratch, or_stop *tr)
{
    const uint32_t W = S->W;
    for (uint64_t f = 0; f < S->nfresh; ++f) {
        /* the arena may move as candidates are added: address it afresh */
        const uint32_t size = n_items(S->arena + S->fresh[f], W) + 1u;
        for (uint64_t a = 0; a < nfreq; ++a) {
            const uint64_t *base = S->arena + S->fresh[f];
            const uint32_t it = freq[a];
            if (has_item(base, it))
                continue;
            memcpy(C, base, W * sizeof(uint64_t));
            C[it >> 6] |= 1ull << (it & 63);
            if (known_get(&S->seen, C) != K_EMPTY || !maximal_subsets_frequent(S, C, scratch))
                continue;
            if (!start_candidate(S, C, size))
                return 0;
            tr->generated++;
        }
    }
    return 1;
}

/* MakeCandidates, reading 1 (the paper's wording taken literally): the OR of
 * every two boxes of one size that has exactly one more item, when new and
 * with all maximal proper subsets frequent.  Finished boxes come first, then
 * live ones, each in list order. */
static int extend_pairs_phase(miner *S, uint64_t *C, uint64_t *scratch, or_stop *tr)
{
    const uint32_t W = S->W;
    uint64_t *boxes = NULL, nb = 0, capb = 0;
    int ok = 1;
    for (uint64_t pass = 0; pass < 2 && ok; ++pass) {
        const cand *v = pass ? S->live : S->done;
        const uint64_t nv = pass ? S->nlive : S->ndone;
        for (uint64_t i = 0; i < nv && ok; ++i)
            if (v[i].reached) {
                ok = grow((void **)&boxes, &capb, nb + 1, sizeof(uint64_t));
                if (ok)
                    boxes[nb++] = v[i].at;
            }
    }
    for (uint64_t x = 0; x < nb && ok; ++x) {
        const uint32_t ka = n_items(S->arena + boxes[x], W);
        for (uint64_t y = x + 1; y < nb && ok; ++y) {
            /* the arena may move as candidates are added: address it afresh */
            const uint64_t *A = S->arena + boxes[x], *B = S->arena + boxes[y];
            if (n_items(B, W) != ka)
                continue;
            for (uint32_t w = 0; w < W; ++w)
                C[w] = A[w] | B[w];
            if (n_items(C, W) != ka + 1u || known_get(&S->seen, C) != K_EMPTY ||
                !maximal_subsets_frequent(S, C, scratch))
                continue;
            ok = start_candidate(S, C, ka + 1u);
            if (ok)
                tr->generated++;
        }
    }
    free(boxes);
    return ok;
}

/* Algorithm 5: a candidate counted on every block of a pass is finished --
 * frequent iff its count reached tau (a circle that reaches it only here is
 * counted in the statistics; Prune promotes first, so it never happens). */
static int retire_phase(miner *S, uint64_t tau, uint64_t nblk, or_stop *tr, or_stats *st)
{
    for (uint64_t i = 0; i < S->nlive; ++i) {
        cand *c = &S->live[i];
        if (c->blocks != nblk)
            continue;
        if (c->hits >= tau && !c->reached) {
            st->fullpass_promotions++;
            c->reached = 1;
            if (!known_set(&S->seen, mask_of(S, c), K_BOX))
                return 0;
        }
        if (!cand_push(&S->done, &S->ndone, &S->capdone, *c))
            return 0;
        c->gone = 1;
        tr->solidified++;
    }
    sweep_live(S);
    return 1;
}

static void miner_free(miner *S)
{
    free(S->arena);
    free(S->live);
    free(S->done);
    free(S->fresh);
    known_free(&S->seen);
}

/* The first candidates.  init_mode 0 (FirstPass, Section 4.1): one pass
 * counts every item; each 1-itemset is finished (frequent or not) and every
 * pair of frequent items is a candidate.  init_mode 1 (Algorithm 1): every
 * 1-itemset is a candidate and every item may extend a box.  freq receives
 * the items that may extend boxes, ascending. */
static int first_candidates(miner *S, const uint64_t *rows, uint64_t n, uint32_t m,
                            uint64_t tau, uint64_t nblk, int init_mode, uint32_t *freq,
                            uint64_t *nfreq, uint64_t *C)
{
    const uint32_t W = S->W;
    *nfreq = 0;
    if (init_mode == 1) {
        for (uint32_t i = 0; i < m; ++i) {
            memset(C, 0, W * sizeof(uint64_t));
            C[i >> 6] = 1ull << (i & 63);
            if (!start_candidate(S, C, 1))
                return 0;
            freq[(*nfreq)++] = i;
        }
        return 1;
    }
    uint64_t *item_hits = (uint64_t *)calloc(m, sizeof(uint64_t));
    if (!item_hits)
        return 0;
    for (uint64_t t = 0; t < n; ++t)
        for (uint32_t i = 0; i < m; ++i)
            item_hits[i] += (uint64_t)has_item(rows + t * W, i);
    int ok = 1;
    for (uint32_t i = 0; i < m && ok; ++i) {
        memset(C, 0, W * sizeof(uint64_t));
        C[i >> 6] = 1ull << (i & 63);
        cand c;
        memset(&c, 0, sizeof(c));
        c.size = 1;
        c.blocks = nblk;
        c.hits = item_hits[i];
        c.reached = item_hits[i] >= tau;
        ok = arena_put(S, C, &c.at) && cand_push(&S->done, &S->ndone, &S->capdone, c) &&
             known_set(&S->seen, C, c.reached ? K_BOX : K_CIRCLE);
        if (ok && c.reached)
            freq[(*nfreq)++] = i;
    }
    free(item_hits);
    for (uint64_t a = 0; a < *nfreq && ok; ++a)
        for (uint64_t b = a + 1; b < *nfreq && ok; ++b) {
            memset(C, 0, W * sizeof(uint64_t));
            C[freq[a] >> 6] |= 1ull << (freq[a] & 63);
            C[freq[b] >> 6] |= 1ull << (freq[b] & 63);
            ok = start_candidate(S, C, 2);
        }
    return ok;
}

int oracle_dic(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, uint64_t M,
               int candgen_mode, or_result **out)
{
    return oracle_dic_init(rows, n, m, minsup, M, candgen_mode, 0, out);
}

/* Section 4.2 (Algorithm 2): after the first candidates, the database is
 * read block after block -- block b holds transactions [(b-1)Mp, min(b Mp,
 * n)), Mp = min(M, n), nblk = ceil(n / Mp) blocks, the first again after the
 * last -- and at each stop the live candidates are counted (Algorithm 3),
 * promoted or erased (Algorithm 4), extended (MakeCandidates) and retired
 * after a full pass (Algorithm 5), until none is live.  The result is the
 * finished itemsets that reached tau. */
int oracle_dic_init(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, uint64_t M,
                    int candgen_mode, int init_mode, or_result **out)
{
    if (!out)
        return OR_E_INVAL;
    *out = NULL;
    int rc = check_db(rows, n, m);
    if (rc)
        return rc;
    if (M == 0 || (candgen_mode != 0 && candgen_mode != 1) || (init_mode != 0 && init_mode != 1))
        return OR_E_INVAL;
    uint64_t tau;
    if ((rc = oracle_tau(minsup, n, &tau)))
        return rc;

    const uint32_t W = (m + 63u) / 64u;
    const uint64_t Mp = M < n ? M : n;
    const uint64_t nblk = (n + Mp - 1) / Mp;

    miner S;
    memset(&S, 0, sizeof(S));
    S.W = W;
    or_stats st;
    memset(&st, 0, sizeof(st));
    or_stop *trace = NULL;
    uint64_t ntrace = 0, captrace = 0;
    uint32_t *freq = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint64_t nfreq = 0;
    uint64_t *C = (uint64_t *)calloc(W, sizeof(uint64_t));
    uint64_t *scratch = (uint64_t *)calloc(W, sizeof(uint64_t));
    rc = OR_E_NOMEM;
    if (!freq || !C || !scratch || !known_init(&S.seen, W, 4096) ||
        !first_candidates(&S, rows, n, m, tau, nblk, init_mode, freq, &nfreq, C))
        goto done;

    for (uint64_t b = 0; S.nlive > 0;) {
        b = b % nblk + 1; /* the next block, the first again after the last */
        const uint64_t lo = (b - 1) * Mp;
        const uint64_t hi = b * Mp < n ? b * Mp : n;
        or_stop tr;
        memset(&tr, 0, sizeof(tr));
        tr.stop = (uint32_t)b;
        tr.rows = (uint32_t)(hi - lo);
        tr.live = S.nlive;
        st.stops++;
        st.tests += S.nlive * (hi - lo);
        if (S.nlive > st.peak_live)
            st.peak_live = S.nlive;
        count_block_phase(&S, rows, lo, hi);
        if (!threshold_phase(&S, tau, Mp, nblk, &tr, &st))
            goto done;
        if (!(candgen_mode == 0 ? extend_fresh_phase(&S, freq, nfreq, C, scratch, &tr)
                                : extend_pairs_phase(&S, C, scratch, &tr)))
            goto done;
        if (!retire_phase(&S, tau, nblk, &tr, &st))
            goto done;
        if (!grow((void **)&trace, &captrace, ntrace + 1, sizeof(or_stop)))
            goto done;
        trace[ntrace++] = tr;
    }

    /* the result: the finished itemsets that reached tau */
    {
        uint64_t q = 0;
        for (uint64_t i = 0; i < S.ndone; ++i)
            q += S.done[i].reached;
        uint64_t *masks = (uint64_t *)malloc((q ? q : 1) * W * sizeof(uint64_t));
        uint32_t *counts = (uint32_t *)malloc((q ? q : 1) * sizeof(uint32_t));
        if (!masks || !counts) {
            free(masks);
            free(counts);
            goto done;
        }
        q = 0;
        for (uint64_t i = 0; i < S.ndone; ++i)
            if (S.done[i].reached) {
                memcpy(masks + q * W, mask_of(&S, &S.done[i]), W * sizeof(uint64_t));
                counts[q] = (uint32_t)S.done[i].hits;
                q++;
            }
        or_result *r = NULL;
        rc = make_result(W, q, masks, counts, &r);
        free(masks);
        free(counts);
        if (rc)
            goto done;
        st.n_frequent = r->stats.n_frequent;
        st.k_max = r->stats.k_max;
        st.tau = tau;
        st.block = Mp;
        st.stop_max = nblk;
        st.known = S.seen.used;
        r->stats = st;
        r->trace = trace;
        r->trace_len = ntrace;
        trace = NULL;
        *out = r;
        rc = OR_OK;
    }

done:
    free(trace);
    free(freq);
    free(C);
    free(scratch);
    miner_free(&S);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Apriori (independent cross-check)                                         */
/* ------------------------------------------------------------------------ */

/* itemsets of one level as sorted item arrays, row-major [count][k] */
typedef struct {
    uint32_t k;
    uint64_t count, cap;
    uint32_t *items;
    uint64_t *supp;
} level;

static int level_push(level *L, const uint32_t *items)
{
    if (L->count == L->cap) {
        uint64_t c = L->cap ? 2 * L->cap : 256;
        uint32_t *it = (uint32_t *)realloc(L->items, c * L->k * sizeof(uint32_t));
        if (!it)
            return 0;
        L->items = it;
        uint64_t *sp = (uint64_t *)realloc(L->supp, c * sizeof(uint64_t));
        if (!sp)
            return 0;
        L->supp = sp;
        L->cap = c;
    }
    memcpy(L->items + L->count * L->k, items, L->k * sizeof(uint32_t));
    L->supp[L->count] = 0;
    L->count++;
    return 1;
}

static int lex_cmp(const uint32_t *a, const uint32_t *b, uint32_t k)
{
    for (uint32_t i = 0; i < k; ++i)
        if (a[i] != b[i])
            return a[i] < b[i] ? -1 : 1;
    return 0;
}

static int level_contains(const level *L, const uint32_t *items)
{
    uint64_t lo = 0, hi = L->count;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        int c = lex_cmp(L->items + mid * L->k, items, L->k);
        if (c == 0)
            return 1;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return 0;
}

int oracle_apriori(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, or_result **out)
{
    if (!out)
        return OR_E_INVAL;
    *out = NULL;
    int rc = check_db(rows, n, m);
    if (rc)
        return rc;
    uint64_t tau;
    if ((rc = oracle_tau(minsup, n, &tau)))
        return rc;
    const uint32_t W = (m + 63u) / 64u;
    rc = OR_E_NOMEM;

    unsigned char *present = (unsigned char *)calloc(m, 1);
    uint32_t *buf = (uint32_t *)malloc((m + 1) * sizeof(uint32_t));
    uint64_t *all_masks = NULL, nall = 0, capm = 0;
    uint32_t *all_counts = NULL;
    uint64_t capc = 0;
    level prev = {1, 0, 0, NULL, NULL}, cur = {0, 0, 0, NULL, NULL};
    if (!present || !buf)
        goto done;

    /* level 1 */
    {
        uint64_t *cnt = (uint64_t *)calloc(m, sizeof(uint64_t));
        if (!cnt)
            goto done;
        for (uint64_t t = 0; t < n; ++t)
            for (uint32_t i = 0; i < m; ++i)
                if ((rows[t * W + (i >> 6)] >> (i & 63)) & 1u)
                    cnt[i]++;
        for (uint32_t i = 0; i < m; ++i)
            if (cnt[i] >= tau) {
                if (!level_push(&prev, &i)) {
                    free(cnt);
                    goto done;
                }
                prev.supp[prev.count - 1] = cnt[i];
            }
        free(cnt);
    }

    for (;;) {
        /* emit the frequent itemsets of this level */
        for (uint64_t c = 0; c < prev.count; ++c) {
            if (!grow((void **)&all_masks, &capm, (nall + 1) * W, sizeof(uint64_t)) ||
                !grow((void **)&all_counts, &capc, nall + 1, sizeof(uint32_t)))
                goto done;
            uint64_t *mk = all_masks + nall * W;
            memset(mk, 0, W * sizeof(uint64_t));
            for (uint32_t j = 0; j < prev.k; ++j) {
                uint32_t it = prev.items[c * prev.k + j];
                mk[it >> 6] |= 1ull << (it & 63);
            }
            all_counts[nall++] = (uint32_t)prev.supp[c];
        }
        if (prev.count < 2)
            break;
        /* join: itemsets that share their first k-1 items */
        uint32_t k = prev.k + 1;
        cur.k = k;
        cur.count = 0;
        for (uint64_t a = 0; a < prev.count; ++a) {
            const uint32_t *A = prev.items + a * prev.k;
            for (uint64_t b = a + 1; b < prev.count; ++b) {
                const uint32_t *B = prev.items + b * prev.k;
                if (lex_cmp(A, B, prev.k - 1) != 0)
                    break; /* sorted: the shared-prefix group has ended */
                memcpy(buf, A, prev.k * sizeof(uint32_t));
                buf[prev.k] = B[prev.k - 1];
                /* a-priori prune: every (k-1)-subset must be frequent */
                int ok = 1;
                uint32_t sub[64 + 1];
                uint32_t *s = k - 1 <= 64 ? sub : NULL;
                uint32_t *heap = NULL;
                if (!s) {
                    heap = (uint32_t *)malloc((k - 1) * sizeof(uint32_t));
                    if (!heap)
                        goto done;
                    s = heap;
                }
                for (uint32_t drop = 0; drop + 2 < k && ok; ++drop) {
                    uint32_t q = 0;
                    for (uint32_t j = 0; j < k; ++j)
                        if (j != drop)
                            s[q++] = buf[j];
                    ok = level_contains(&prev, s);
                }
                free(heap);
                if (ok && !level_push(&cur, buf))
                    goto done;
            }
        }
        if (cur.count == 0)
            break;
        /* count: for each transaction, mark its items and test every candidate */
        for (uint64_t t = 0; t < n; ++t) {
            for (uint32_t i = 0; i < m; ++i)
                present[i] = (unsigned char)((rows[t * W + (i >> 6)] >> (i & 63)) & 1u);
            for (uint64_t c = 0; c < cur.count; ++c) {
                const uint32_t *it = cur.items + c * k;
                uint32_t j = 0;
                while (j < k && present[it[j]])
                    ++j;
                if (j == k)
                    cur.supp[c]++;
            }
        }
        /* keep the frequent ones (order is preserved: still lexicographic) */
        level next = {k, 0, 0, NULL, NULL};
        for (uint64_t c = 0; c < cur.count; ++c)
            if (cur.supp[c] >= tau) {
                if (!level_push(&next, cur.items + c * k)) {
                    free(next.items);
                    free(next.supp);
                    goto done;
                }
                next.supp[next.count - 1] = cur.supp[c];
            }
        free(prev.items);
        free(prev.supp);
        prev = next;
        if (prev.count == 0)
            break;
    }

    {
        or_result *r = NULL;
        rc = make_result(W, nall, all_masks, all_counts, &r);
        if (rc)
            goto done;
        r->stats.tau = tau;
        *out = r;
        rc = OR_OK;
    }
done:
    free(present);
    free(buf);
    free(all_masks);
    free(all_counts);
    free(prev.items);
    free(prev.supp);
    free(cur.items);
    free(cur.supp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* exact enumeration                                                         */
/* ------------------------------------------------------------------------ */

int oracle_bruteforce(const uint64_t *rows, uint64_t n, uint32_t m, double minsup,
                      or_result **out)
{
    if (!out)
        return OR_E_INVAL;
    *out = NULL;
    int rc = check_db(rows, n, m);
    if (rc)
        return rc;
    if (m > 20)
        return OR_E_RANGE;
    uint64_t tau;
    if ((rc = oracle_tau(minsup, n, &tau)))
        return rc;
    uint64_t total = (1ull << m) - 1;
    uint64_t *masks = (uint64_t *)malloc(total * sizeof(uint64_t));
    uint32_t *counts = (uint32_t *)malloc(total * sizeof(uint32_t));
    if (!masks || !counts) {
        free(masks);
        free(counts);
        return OR_E_NOMEM;
    }
    uint64_t q = 0;
    for (uint64_t s = 1; s <= total; ++s) {
        uint64_t c = 0;
        for (uint64_t t = 0; t < n; ++t)
            if ((rows[t] & s) == s) /* m <= 20: one word per row */
                c++;
        if (c >= tau) {
            masks[q] = s;
            counts[q] = (uint32_t)c;
            q++;
        }
    }
    or_result *r = NULL;
    rc = make_result(1, q, masks, counts, &r);
    free(masks);
    free(counts);
    if (rc)
        return rc;
    r->stats.tau = tau;
    *out = r;
    return OR_OK;
}

typedef struct {
    uint32_t m, W;
    uint64_t tau;
    uint32_t **tids; /* per item: ascending row ids containing it */
    uint64_t *ntid;
    uint64_t *masks, nout, capm;
    uint32_t *counts;
    uint64_t capc;
    uint64_t *cur; /* current itemset mask */
    int fail;
} tid_walk;

static void tid_dfs(tid_walk *T, const uint32_t *tl, uint64_t ntl, uint32_t start)
{
    for (uint32_t i = start; i < T->m && !T->fail; ++i) {
        /* intersect the current row list with item i's */
        uint32_t *nx = (uint32_t *)malloc((ntl ? ntl : 1) * sizeof(uint32_t));
        if (!nx) {
            T->fail = 1;
            return;
        }
        uint64_t a = 0, b = 0, c = 0;
        const uint32_t *L = T->tids[i];
        while (a < ntl && b < T->ntid[i]) {
            if (tl[a] == L[b]) {
                nx[c++] = tl[a];
                a++;
                b++;
            } else if (tl[a] < L[b]) {
                a++;
            } else {
                b++;
            }
        }
        if (c >= T->tau) {
            T->cur[i >> 6] |= 1ull << (i & 63);
            if (!grow((void **)&T->masks, &T->capm, (T->nout + 1) * T->W, sizeof(uint64_t)) ||
                !grow((void **)&T->counts, &T->capc, T->nout + 1, sizeof(uint32_t))) {
                T->fail = 1;
                free(nx);
                return;
            }
            memcpy(T->masks + T->nout * T->W, T->cur, T->W * sizeof(uint64_t));
            T->counts[T->nout++] = (uint32_t)c;
            tid_dfs(T, nx, c, i + 1);
            T->cur[i >> 6] &= ~(1ull << (i & 63));
        }
        free(nx);
    }
}

int oracle_tidlist(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, or_result **out)
{
    if (!out)
        return OR_E_INVAL;
    *out = NULL;
    int rc = check_db(rows, n, m);
    if (rc)
        return rc;
    tid_walk T;
    memset(&T, 0, sizeof(T));
    if ((rc = oracle_tau(minsup, n, &T.tau)))
        return rc;
    T.m = m;
    T.W = (m + 63u) / 64u;
    rc = OR_E_NOMEM;
    uint32_t *all = NULL;
    T.tids = (uint32_t **)calloc(m, sizeof(uint32_t *));
    T.ntid = (uint64_t *)calloc(m, sizeof(uint64_t));
    T.cur = (uint64_t *)calloc(T.W, sizeof(uint64_t));
    if (!T.tids || !T.ntid || !T.cur)
        goto done;
    for (uint64_t t = 0; t < n; ++t)
        for (uint32_t i = 0; i < m; ++i)
            if ((rows[t * T.W + (i >> 6)] >> (i & 63)) & 1u)
                T.ntid[i]++;
    for (uint32_t i = 0; i < m; ++i) {
        T.tids[i] = (uint32_t *)malloc((T.ntid[i] ? T.ntid[i] : 1) * sizeof(uint32_t));
        if (!T.tids[i])
            goto done;
        T.ntid[i] = 0;
    }
    for (uint64_t t = 0; t < n; ++t)
        for (uint32_t i = 0; i < m; ++i)
            if ((rows[t * T.W + (i >> 6)] >> (i & 63)) & 1u)
                T.tids[i][T.ntid[i]++] = (uint32_t)t;
    all = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!all)
        goto done;
    for (uint64_t t = 0; t < n; ++t)
        all[t] = (uint32_t)t;
    tid_dfs(&T, all, n, 0);
    if (T.fail)
        goto done;
    {
        or_result *r = NULL;
        rc = make_result(T.W, T.nout, T.masks, T.counts, &r);
        if (rc)
            goto done;
        r->stats.tau = T.tau;
        *out = r;
        rc = OR_OK;
    }
done:
    free(all);
    if (T.tids)
        for (uint32_t i = 0; i < m; ++i)
            free(T.tids[i]);
    free(T.tids);
    free(T.ntid);
    free(T.cur);
    free(T.masks);
    free(T.counts);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* single-step references                                                    */
/* ------------------------------------------------------------------------ */

int oracle_item_counts(const uint64_t *rows, uint64_t n, uint32_t m, uint32_t *counts)
{
    int rc = check_db(rows, n, m);
    if (rc || !counts)
        return rc ? rc : OR_E_INVAL;
    const uint32_t W = (m + 63u) / 64u;
    for (uint32_t i = 0; i < m; ++i)
        counts[i] = 0;
    for (uint64_t t = 0; t < n; ++t)
        for (uint32_t i = 0; i < m; ++i)
            if (has_item(rows + t * W, i))
                counts[i]++;
    return OR_OK;
}

int oracle_count_block(const uint64_t *rows, uint64_t n, uint32_t m, const uint64_t *masks,
                       uint64_t q, uint64_t first, uint64_t last, uint32_t *counts)
{
    int rc = check_db(rows, n, m);
    if (rc || (!masks && q) || (!counts && q) || first > last || last > n)
        return rc ? rc : OR_E_INVAL;
    const uint32_t W = (m + 63u) / 64u;
    for (uint64_t c = 0; c < q; ++c) {
        uint32_t s = 0;
        for (uint64_t t = first; t < last; ++t)
            if (is_subset(masks + c * W, rows + t * W, W))
                s++;
        counts[c] = s;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* association rules                                                         */
/* ------------------------------------------------------------------------ */

struct or_rules {
    uint64_t size, cap;
    uint32_t *itemset, *code, *supp_x;
};

static int rules_push(or_rules *R, uint32_t i, uint32_t code, uint32_t sx)
{
    if (R->size == R->cap) {
        uint64_t nc = R->cap ? 2 * R->cap : 1024;
        uint32_t *a = (uint32_t *)realloc(R->itemset, nc * sizeof(uint32_t));
        if (!a)
            return OR_E_NOMEM;
        R->itemset = a;
        uint32_t *b = (uint32_t *)realloc(R->code, nc * sizeof(uint32_t));
        if (!b)
            return OR_E_NOMEM;
        R->code = b;
        uint32_t *c = (uint32_t *)realloc(R->supp_x, nc * sizeof(uint32_t));
        if (!c)
            return OR_E_NOMEM;
        R->supp_x = c;
        R->cap = nc;
    }
    R->itemset[R->size] = i;
    R->code[R->size] = code;
    R->supp_x[R->size] = sx;
    R->size++;
    return OR_OK;
}

void oracle_rules_free(or_rules *R)
{
    if (!R)
        return;
    free(R->itemset);
    free(R->code);
    free(R->supp_x);
    free(R);
}

int oracle_rules(const uint64_t *masks, const uint32_t *counts, uint64_t q, uint32_t W,
                 double minconf, or_rules **out)
{
    if (!out || W == 0 || (q && (!masks || !counts)) || minconf != minconf)
        return OR_E_INVAL;
    *out = NULL;
    for (uint64_t i = 0; i < q; ++i)
        if (n_items(masks + i * W, W) > OR_RULES_KMAX)
            return OR_E_RANGE;
    or_rules *R = (or_rules *)calloc(1, sizeof(*R));
    uint64_t *perm = (uint64_t *)malloc((q ? q : 1) * sizeof(uint64_t));
    uint64_t *X = (uint64_t *)malloc(W * sizeof(uint64_t));
    if (!R || !perm || !X) {
        free(perm);
        free(X);
        oracle_rules_free(R);
        return OR_E_NOMEM;
    }
    /* itemsets in canonical order, so supp(X) is found by binary search */
    for (uint64_t i = 0; i < q; ++i)
        perm[i] = i;
    canon_W = W;
    canon_masks = masks;
    qsort(perm, q, sizeof(uint64_t), canon_cmp);
    int rc = OR_OK;
    uint32_t items[OR_RULES_KMAX];
    for (uint64_t i = 0; i < q && rc == OR_OK; ++i) {
        const uint64_t *I = masks + i * W;
        uint32_t k = 0;
        for (uint32_t p = 0; p < 64u * W; ++p)
            if (has_item(I, p))
                items[k++] = p;
        if (k < 2)
            continue;
        const uint32_t full = (1u << k) - 1u;
        for (uint32_t code = 1; code < full && rc == OR_OK; ++code) {
            /* X: the items of I selected by the bits of code */
            memset(X, 0, W * sizeof(uint64_t));
            for (uint32_t t = 0; t < k; ++t)
                if ((code >> t) & 1u)
                    X[items[t] >> 6] |= 1ull << (items[t] & 63u);
            uint64_t lo = 0, hi = q;
            int found = 0;
            while (lo < hi) {
                uint64_t mid = lo + (hi - lo) / 2;
                int c = mask_cmp(X, masks + perm[mid] * W, W);
                if (c == 0) {
                    lo = mid;
                    found = 1;
                    break;
                }
                if (c < 0)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            if (!found) {
                rc = OR_E_INVAL; /* a subset of a frequent itemset is missing */
                break;
            }
            const uint32_t sx = counts[perm[lo]];
            if ((double)counts[i] >= minconf * (double)sx)
                rc = rules_push(R, (uint32_t)i, code, sx);
        }
    }
    free(perm);
    free(X);
    if (rc) {
        oracle_rules_free(R);
        return rc;
    }
    *out = R;
    return OR_OK;
}

uint64_t oracle_rules_size(const or_rules *R) { return R ? R->size : 0; }
const uint32_t *oracle_rules_itemset(const or_rules *R) { return R ? R->itemset : NULL; }
const uint32_t *oracle_rules_code(const or_rules *R) { return R ? R->code : NULL; }
const uint32_t *oracle_rules_supp_x(const or_rules *R) { return R ? R->supp_x : NULL; }

/* ------------------------------------------------------------------------ */
/* result accessors                                                          */
/* ------------------------------------------------------------------------ */

uint64_t oracle_result_size(const or_result *r) { return r ? r->size : 0; }
uint32_t oracle_result_words(const or_result *r) { return r ? r->W : 0; }
const uint64_t *oracle_result_masks(const or_result *r) { return r ? r->masks : NULL; }
const uint32_t *oracle_result_counts(const or_result *r) { return r ? r->counts : NULL; }
uint64_t oracle_result_trace_len(const or_result *r) { return r ? r->trace_len : 0; }
const or_stop *oracle_result_trace(const or_result *r) { return r ? r->trace : NULL; }

int oracle_result_stats(const or_result *r, or_stats *s)
{
    if (!r || !s)
        return OR_E_INVAL;
    *s = r->stats;
    return OR_OK;
}

void oracle_result_free(or_result *r)
{
    if (!r)
        return;
    free(r->masks);
    free(r->counts);
    free(r->trace);
    free(r);
}
