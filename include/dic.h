/*
 * dic.h -- frequent itemset mining by Dynamic Itemset Counting on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Zymbler, "Parallel Algorithm for Frequent Itemset Mining on Intel
 * Many-core Systems".  Given a transaction database D = (T_1..T_n) over items
 * 0..m-1 and a minimum support fraction minsup, the library returns every
 * itemset contained in at least tau transactions together with its exact
 * count (the problem statement of Section 1).  It gets there the way the
 * paper's ParallelDIC does (Algorithm 2): a full first pass finds the
 * frequent items and seeds all their pairs as candidates; then the database
 * is scanned in blocks of M transactions, rewinding after the last block,
 * and at every stop each live candidate's support is counted over the block
 * (Algorithm 3), candidates that reached tau are promoted and hopeless ones
 * pruned (Algorithm 4), supersets of new frequent itemsets whose maximal
 * subsets are all frequent are added (MakeCandidates), and candidates that
 * have seen every transaction once become final (Algorithm 5).  Every step
 * runs in HIP kernels on the GPU; counts are exact 32-bit integers.
 *
 * Threshold: tau = max(1, ceil(minsup * n)), except that when minsup * n is
 * within 1e-9 (relative, at least absolute 1e-9) of an integer that integer
 * is used, and when minsup * n exceeds n the threshold is n + 1 (nothing is
 * frequent).  minsup must be > 0 and not NaN.
 *
 * Bit layout (Section 4.1, one 64-bit word generalised to W words): a row
 * is W = ceil(m / 64) uint64 words; item p is bit (p & 63) of word (p >> 6);
 * bits at or above m must be zero.  A transaction T contains an itemset I
 * exactly when (T[w] & I[w]) == I[w] for every word w.
 *
 * Limits: 1 <= m <= 4096 items, 1 <= n < 2^32 - 1 transactions.
 *
 * Errors: every call returns 0 on success or a negative DIC_E_* code and
 * sets a thread-local message readable with dic_last_error().  No C++
 * exception crosses this interface.  On error every out-pointer is set to
 * NULL (or left untouched where documented) and nothing is leaked.
 *
 * Threads: calls on different databases may run concurrently from different
 * host threads.  Calls on the same database are serialised internally.
 */
#ifndef DIC_H
#define DIC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define DIC_API __attribute__((visibility("default")))
#else
#define DIC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define DIC_OK 0
#define DIC_E_INVAL (-1)    /* a bad argument                                   */
#define DIC_E_NOMEM (-2)    /* device or host allocation failed                 */
#define DIC_E_CAPACITY (-3) /* request can never fit the server's memory budget */
#define DIC_E_BUSY (-4)     /* database still referenced by queued/running work */
#define DIC_E_PENDING (-5)  /* result not ready yet                             */
#define DIC_E_DEVICE (-6)   /* a HIP runtime error                              */
#define DIC_E_TIMEOUT (-7)  /* wait timed out                                   */
#define DIC_E_NOTFOUND (-8) /* unknown ticket                                   */

typedef struct dic_db dic_db;
typedef struct dic_result dic_result;
typedef struct dic_server dic_server;

/* Per-stop record of one mining run (the loop body of Algorithm 2). */
typedef struct dic_stop_trace {
    uint32_t stop;       /* block index 1..stop_max counted at this stop      */
    uint32_t rows;       /* transactions in that block                         */
    uint32_t live;       /* candidates counted (|DASHED| at CountSupport)      */
    uint32_t promoted;   /* dashed circles that reached tau (Prune)            */
    uint32_t pruned;     /* dashed circles erased by the upper bound (Prune)   */
    uint32_t generated;  /* new candidates (MakeCandidates)                    */
    uint32_t solidified; /* candidates that finished a full pass (CheckFullPass) */
    uint32_t words;      /* nonzero 32-bit words over the live candidates' masks:
                            the AND work per transaction at this stop      */
    uint32_t items;      /* items over the live candidates (sum of sizes)   */
    uint32_t launch_ns;  /* with the "profile" option: the stop's launch time in
                            ns (HIP events; in a batch the launch is shared) */
} dic_stop_trace;

typedef struct dic_stats {
    uint64_t tau;        /* integer support threshold                          */
    uint64_t block;      /* M' = min(M, n)                                     */
    uint64_t stop_max;   /* ceil(n / M')                                       */
    uint64_t stops;      /* stops executed                                     */
    uint64_t tests;      /* subset tests: sum over stops of live * rows        */
    uint64_t peak_live;  /* largest live candidate set                         */
    uint64_t n_frequent; /* |L|                                                */
    uint64_t k_max;      /* size of the largest frequent itemset               */
    uint64_t known;      /* itemsets ever created (1-itemsets included)        */
    uint64_t restarts;   /* runs repeated after growing the candidate capacity */
    double mine_ms;      /* wall time from submission to result                */
    double count_ms;     /* CountSupport kernel time (HIP events; 0 unless the
                            "profile" option is on)                           */
    uint64_t count_launches; /* CountSupport launches timed into count_ms      */
    double first_pass_ms; /* FirstPass kernel time (HIP events; 0 unless the
                             "profile" option is on; a batch's jobs share it) */
} dic_stats;

/*
 * Copy a database to the device.  rows: host pointer to n*W uint64 words,
 * row-major (layout above).  The library copies the data; the caller keeps
 * ownership of rows.  DIC_E_INVAL if rows is NULL, n == 0, n >= 2^32-1,
 * m == 0, m > 4096, or any bit at or above m is set.  *out is NULL on error.
 */
DIC_API int dic_load_db(const uint64_t *rows, uint64_t n, uint32_t m, dic_db **out);

/*
 * Same, from a database already in device memory (rows is a device pointer
 * to n*W words, e.g. a framework tensor).  The data is copied device to
 * device on the library's stream; the padding-bit check runs on the GPU.
 */
DIC_API int dic_load_db_device(const uint64_t *rows, uint64_t n, uint32_t m, dic_db **out);

/*
 * Build a database from item lists in CSR form: transaction t holds
 * items[offsets[t] .. offsets[t+1]) (host pointers; offsets has n+1
 * entries, offsets[0] == 0, non-decreasing).  Duplicate items are
 * harmless.  The bit rows are packed on the GPU.  DIC_E_INVAL if an item
 * is >= m or the offsets are malformed.
 */
DIC_API int dic_load_db_lists(const uint32_t *items, const uint64_t *offsets, uint64_t n, uint32_t m,
                      dic_db **out);

/* n, m of a loaded database (NULL-safe: 0). */
DIC_API uint64_t dic_db_rows(const dic_db *db);
DIC_API uint32_t dic_db_items(const dic_db *db);

/*
 * Free a database.  NULL gives DIC_OK.  DIC_E_BUSY (and nothing is freed)
 * while a server request that references it is queued or running.
 */
DIC_API int dic_free_db(dic_db *db);

/*
 * Mine one database: every itemset with support >= tau and its exact count.
 * minsup > 0 (values above 1 give an empty result), M >= 1 (clamped to n).
 * Synchronous.  *out is owned by the caller (dic_result_free).
 */
DIC_API int dic_mine(dic_db *db, double minsup, uint64_t M, dic_result **out);

/*
 * Mine many databases at once: one launch per kernel per stop covers every
 * database still running.  outs[i] receives database i's result, identical
 * to what dic_mine would return; status[i] (may be NULL) its own code.
 * Returns DIC_OK if every element succeeded, else the first failing
 * element's code (failed elements have outs[i] == NULL).
 */
DIC_API int dic_batch(dic_db *const *dbs, const double *minsup, const uint64_t *M, uint32_t count,
              dic_result **outs, int *status);

/*
 * Mine one database like dic_mine, allocating nothing: for callers that
 * cannot allocate device memory (work captured into HIP graphs, tight
 * serving loops, harnesses that forbid hipMalloc).  The working memory of
 * the mine (job state, plans, counters, item counts, candidate pool,
 * frequent-item bitsets) comes from one static device array of
 * DIC_NOALLOC_SCRATCH_BYTES per GPU, held by the process from the first
 * call on that GPU until it ends; its contents are cleared by each call
 * where they must start empty.
 *   masks  host array of capacity * W words (W = ceil(m / 64)), caller-owned
 *   counts host array of capacity entries, caller-owned
 *   *size  receives |L|, also when it exceeds capacity
 *   stats  may be NULL; the per-stop trace is not kept (no trace accessor),
 *          count_ms is 0
 * On success masks/counts hold L in canonical order with the counts
 * dic_mine returns, bit for bit.  DIC_E_CAPACITY if |L| > capacity
 * (nothing is written to the arrays) or if the mine needs more working
 * memory than the array holds (the message gives the bytes); DIC_E_INVAL for NULL db/size, NULL arrays with a
 * nonzero capacity, minsup <= 0 or NaN, M == 0; DIC_E_DEVICE on a runtime
 * error.  Runs on the current device.  Calls on one device from one
 * process are serialised by a lock; work of two processes never shares an
 * array.  A caller that captures the call's stream work into graphs must
 * not replay two such graphs concurrently on one device: they share the
 * array and would race.
 */
#define DIC_NOALLOC_SCRATCH_BYTES (64ull << 20)
DIC_API int dic_mine_noalloc(dic_db *db, double minsup, uint64_t M, uint64_t *masks,
                             uint32_t *counts, uint64_t capacity, uint64_t *size,
                             dic_stats *stats);

/* Result accessors; pointers stay valid until dic_result_free. */
DIC_API uint64_t dic_result_size(const dic_result *r);
DIC_API uint32_t dic_result_words(const dic_result *r);
/* size*W words, canonical order: size ascending, then item lists ascending */
DIC_API const uint64_t *dic_result_masks(const dic_result *r);
DIC_API const uint32_t *dic_result_counts(const dic_result *r);
DIC_API int dic_result_stats(const dic_result *r, dic_stats *s);
/* per-stop records, *n_stops entries (NULL-safe) */
DIC_API const dic_stop_trace *dic_result_trace(const dic_result *r, uint64_t *n_stops);
DIC_API void dic_result_free(dic_result *r);

/* ---------------------------------------------------------------------------
 * Association rules (the second subtask of association rule mining named in
 * Section 1; rule X => Y and its confidence supp(X u Y) / supp(X) as defined
 * in the paper's reference [1]; the paper does not define them itself).
 *
 * For every itemset I of a mining result with |I| >= 2 and every nonempty
 * proper subset X of I, the rule X => I \ X is kept when
 *     (double)supp(I) >= minconf * (double)supp(X)
 * in IEEE double arithmetic.  supp(X) is the count of X in the same result
 * (X is frequent whenever I is).  Rules are ordered by I's position in the
 * result, then by X's subset code: bit t of the code selects the t-th
 * smallest item of I.  Computed on the device (itemset hash table, every
 * split looked up in parallel); the result lives in host memory.
 *
 * Errors: DIC_E_INVAL for NULL out, a NaN minconf, W outside [1, 64], an
 * itemset of more than DIC_RULES_KMAX items, or itemsets that are not
 * downward closed (a subset of some I missing); DIC_E_NOMEM; DIC_E_DEVICE.
 * minconf <= 0 keeps every split, minconf > 1 keeps none.
 * ------------------------------------------------------------------------- */
#define DIC_RULES_KMAX 24
typedef struct dic_rules_result dic_rules_result;
typedef struct dic_rules_stats {
    uint64_t itemsets;  /* itemsets of the input                                */
    uint64_t splits;    /* (I, X) pairs examined: sum over |I| >= 2 of 2^|I| - 2 */
    uint64_t rules;     /* rules kept                                           */
    double kernel_ms;   /* device time of the two passes                        */
    double total_ms;    /* the whole call, transfers included                   */
} dic_rules_stats;

/* Rules of a result from dic_mine / dic_batch / the server.  *out is owned by
 * the caller (dic_rules_free). */
DIC_API int dic_rules(const dic_result *r, double minconf, dic_rules_result **out);
/* The same from host arrays: q itemsets as masks (q * W words, item p at bit
 * p & 63 of word p >> 6) with their counts.  The arrays are read during the
 * call only. */
DIC_API int dic_rules_from_arrays(const uint64_t *masks, const uint32_t *counts, uint64_t q,
                                  uint32_t W, double minconf, dic_rules_result **out);
/* Rule accessors; pointers stay valid until dic_rules_free (NULL when empty). */
DIC_API uint64_t dic_rules_size(const dic_rules_result *r);
DIC_API uint32_t dic_rules_words(const dic_rules_result *r);
DIC_API const uint32_t *dic_rules_itemset(const dic_rules_result *r); /* index of I        */
DIC_API const uint32_t *dic_rules_code(const dic_rules_result *r);    /* subset code of X  */
DIC_API const uint32_t *dic_rules_supp_x(const dic_rules_result *r);  /* supp(X)           */
DIC_API const uint64_t *dic_rules_antecedent(const dic_rules_result *r); /* X, size * W    */
DIC_API const uint64_t *dic_rules_consequent(const dic_rules_result *r); /* I \ X, size * W */
DIC_API int dic_rules_stats_of(const dic_rules_result *r, dic_rules_stats *s);
DIC_API void dic_rules_free(dic_rules_result *r);

/*
 * Serving: a request loop that keeps databases and candidate tables on the
 * device and runs admitted requests together (continuous batching: a
 * request that arrives while others are running joins at the next stop
 * once its memory fits the budget).
 */
typedef struct dic_serve_opts {
    uint32_t max_active;   /* requests mined together at most (0: 64)        */
    uint32_t reserved;
} dic_serve_opts;

DIC_API int dic_serve_create(uint64_t hbm_budget_bytes, const dic_serve_opts *opts, dic_server **out);
/* Queue a request.  DIC_E_CAPACITY at once if its footprint estimate can
 * never fit the budget.  *ticket identifies it for poll/wait. */
DIC_API int dic_serve_submit(dic_server *srv, dic_db *db, double minsup, uint64_t M, uint64_t *ticket);
/* DIC_E_PENDING while queued or running; otherwise hands over the result
 * (or the request's error code) and forgets the ticket. */
DIC_API int dic_serve_poll(dic_server *srv, uint64_t ticket, dic_result **out);
/* Like poll but blocks up to timeout_ms (negative: forever). */
DIC_API int dic_serve_wait(dic_server *srv, uint64_t ticket, int64_t timeout_ms, dic_result **out);
/* Latency percentiles (submit to completion, ms) and completed requests/s. */
DIC_API int dic_serve_stats(dic_server *srv, double *p50_ms, double *p99_ms, double *throughput_rps);
/* Device memory charged against the budget now, the most ever charged, and
 * the budget itself (any pointer may be NULL).  The charge is each admitted
 * request's bound plus, once, each database an admitted request uses; a
 * request whose candidate pool overflows is charged its larger bound before
 * it runs again, so *peak never exceeds *budget. */
DIC_API int dic_serve_usage(dic_server *srv, uint64_t *used, uint64_t *peak, uint64_t *budget);
/* Waits for running work, drops queued requests, frees the server. */
DIC_API int dic_serve_destroy(dic_server *srv);

/*
 * Route the library's device allocations through the caller's allocator:
 * alloc(size, stream) returns device memory or NULL, free(ptr, stream)
 * releases a block; both are given `stream` (a hipStream_t, or NULL) as
 * passed here, so an allocator may tie its blocks to it.  A NULL from alloc
 * fails the call that needed the memory with DIC_E_NOMEM, after it has
 * released what it had taken.  Every block goes back to the functions that
 * allocated it, also after they have been replaced.  Pass NULL functions to
 * return to the library's own hipMalloc-backed cache.
 *
 * Streams: database loads (dic_load_db*) and dic_rules run on `stream` when
 * it is not NULL (else on a library stream).  Mining (dic_mine, dic_batch,
 * serving) runs on streams private to the library's engines -- a stop chunk
 * is captured into a HIP graph, which needs a stream no other thread uses --
 * and every call that hands back results has completed its device work, so
 * no block is freed while a kernel may still use it.
 */
DIC_API int dic_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *),
                      void *stream);

/*
 * Library options (process-wide):
 *   "profile"  0/1: time every CountSupport launch with HIP events recorded
 *              on the stream it runs on; reported as dic_stats.count_ms.
 *              Profiled runs launch their kernels directly (no graphs).
 *   "layout"   counting layout of runs started from now on: 1 (default)
 *              per-item bitsets over 64-row words (a candidate's support in
 *              a word is the popcount of the AND of its items' words), 0 the
 *              row bitmaps themselves (one AND/compare per row and nonzero
 *              word).  Both give identical results.
 *   "init"     start of runs started from now on: 0 (default) the paper's
 *              FirstPass (Section 4.1: one full pass counts the 1-itemsets,
 *              pairs of frequent items are the first candidates); 1 classic
 *              DIC (Algorithm 1, Section 3): every 1-itemset starts as a
 *              dashed circle and is counted block by block like any other
 *              candidate.  Both give identical itemsets and counts; the
 *              per-stop trace differs.  With M >= n either is level-wise
 *              Apriori (one block per pass).
 *   "graphs"   1 (default): stops run as replays of a captured HIP graph of
 *              a few stops on the engine's own stream; 0: direct launches.
 *   Count planning (results never depend on them; chosen by the autotuner):
 *   "vt_target"     workgroups aimed at per job per stop (bitsets), 64..65536
 *   "vt_wave_k"     below this many live candidates one wave counts each
 *                   candidate over the whole block (bitsets), 0..2^30
 *   "vt_tile_words" 64-row words per LDS tile at most (bitsets), 1..16
 *   "count_grid"    workgroups launched for the count kernels, 64..65536
 *   "count_target"  work items aimed at per job per stop (rows), 64..65536
 */
DIC_API int dic_set_option(const char *name, int64_t value);

/* Thread-local message for the last error on this thread ("" if none). */
DIC_API const char *dic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
