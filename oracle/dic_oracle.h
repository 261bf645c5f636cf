/*
 * dic_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference for frequent itemset mining by
 * Dynamic Itemset Counting (Zymbler, "Parallel Algorithm for Frequent Itemset
 * Mining on Intel Many-core Systems"), plus two independent cross-checks
 * (level-wise Apriori and exhaustive / depth-first exact enumeration).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may call this library.  It shares no code, header, table or helper with the
 * GPU library; the two are built separately and neither includes the other.
 *
 * Data layout (Section 4.1, direct bit representation, widened to W words):
 * a database is row-major uint64[n * W], W = ceil(m / 64); item p is bit
 * (p & 63) of word (p >> 6).  Bits at or above m must be zero.
 *
 * Results are in canonical order: itemset size ascending, then the ascending
 * item-index list compared lexicographically.  Counts are exact uint32.
 */
#ifndef DIC_ORACLE_H
#define DIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_NOMEM (-2)
#define OR_E_RANGE (-3) /* brute force asked for more items than it enumerates */

typedef struct or_stop {
    uint32_t stop;        /* stop index 1..stop_max of this iteration        */
    uint32_t rows;        /* rows in the block counted at this stop (B_s)    */
    uint64_t live;        /* |DASHED| when counting started (K_s)            */
    uint64_t promoted;    /* dashed circles that became boxes in Prune       */
    uint64_t pruned;      /* dashed circles erased by Prune                  */
    uint64_t generated;   /* candidates inserted by MakeCandidates           */
    uint64_t solidified;  /* itemsets moved to SOLID by CheckFullPass        */
} or_stop;

typedef struct or_stats {
    uint64_t tau;             /* integer support threshold                  */
    uint64_t block;           /* M' = min(M, n)                             */
    uint64_t stop_max;        /* ceil(n / M')                               */
    uint64_t stops;           /* iterations of the main loop                */
    uint64_t tests;           /* sum over stops of K_s * B_s                */
    uint64_t peak_live;       /* max K_s                                    */
    uint64_t n_frequent;      /* |L|                                        */
    uint64_t k_max;           /* size of the largest frequent itemset       */
    uint64_t known;           /* itemsets ever created (1-itemsets too)     */
    uint64_t superset_prunes; /* supersets erased by Prune's superset loop  */
    uint64_t fullpass_promotions; /* circles promoted by CheckFullPass      */
} or_stats;

typedef struct or_result or_result;

/* Integer threshold from a fractional minsup (see oracle_dic). */
int oracle_tau(double minsup, uint64_t n, uint64_t *tau);

/* Threads of the count loop when built with OpenMP (threads <= 0: keep the
 * current setting); returns the number in use (1 in a serial build). */
int oracle_threads(int threads);

/*
 * Dynamic Itemset Counting, ParallelDIC driver (Algorithm 2) run serially.
 * candgen_mode 0: candidates are S + {i} for each newly promoted box S and
 *                 each frequent item i not in S;
 * candgen_mode 1: candidates are the OR of every pair of equal-size boxes
 *                 that differ in one item (the literal bitwise-OR join).
 * Both admit a candidate only if it is new and all its maximal proper
 * subsets are boxes; they must give identical traces and results.
 */
int oracle_dic(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, uint64_t M,
               int candgen_mode, or_result **out);

/*
 * The same with a choice of initialisation.  init_mode 0 is the paper's
 * FirstPass (Section 4.1): one full pass counts the 1-itemsets, the frequent
 * ones are solid boxes and their pairs the first candidates.  init_mode 1 is
 * classic DIC (Algorithm 1, Section 3): every 1-itemset starts as a dashed
 * circle and is counted, promoted, pruned and solidified like any other
 * candidate; pairs appear when their two items are boxes.  Both give the
 * same frequent itemsets; the trace differs.
 */
int oracle_dic_init(const uint64_t *rows, uint64_t n, uint32_t m, double minsup, uint64_t M,
                    int candgen_mode, int init_mode, or_result **out);

/* Level-wise Apriori over sorted item arrays; counts by item-presence lookup. */
int oracle_apriori(const uint64_t *rows, uint64_t n, uint32_t m, double minsup,
                   or_result **out);

/* Every nonempty itemset over m <= 20 items, each counted by a full scan. */
int oracle_bruteforce(const uint64_t *rows, uint64_t n, uint32_t m, double minsup,
                      or_result **out);

/* Depth-first exact enumeration with transaction-id lists (any m). */
int oracle_tidlist(const uint64_t *rows, uint64_t n, uint32_t m, double minsup,
                   or_result **out);

/* Support of each first-pass item over all rows: counts[m]. */
int oracle_item_counts(const uint64_t *rows, uint64_t n, uint32_t m, uint32_t *counts);

/* Rows of [first, last) containing each of q itemsets (masks q*W words). */
int oracle_count_block(const uint64_t *rows, uint64_t n, uint32_t m, const uint64_t *masks,
                       uint64_t q, uint64_t first, uint64_t last, uint32_t *counts);

/*
 * Association rules, the second subtask of association rule mining named in
 * Section 1 (rule and confidence as defined by Agrawal et al., the paper's
 * reference [1]).  Input: q frequent itemsets (masks q*W) with exact counts.
 * For every itemset I with |I| >= 2 and every nonempty proper subset X of I,
 * the rule X => I \ X has confidence supp(I) / supp(X); it is kept when
 * (double)supp(I) >= minconf * (double)supp(X) in IEEE double arithmetic.
 * Rules are ordered by I's position in the input, then by the subset code of
 * X: bit t of the code selects the t-th smallest item of I.  supp(X) is
 * looked up among the input itemsets; a missing subset (input not downward
 * closed) gives OR_E_INVAL, an itemset of more than OR_RULES_KMAX items
 * gives OR_E_RANGE.
 */
#define OR_RULES_KMAX 24u
typedef struct or_rules or_rules;
int oracle_rules(const uint64_t *masks, const uint32_t *counts, uint64_t q, uint32_t W,
                 double minconf, or_rules **out);
uint64_t oracle_rules_size(const or_rules *R);
const uint32_t *oracle_rules_itemset(const or_rules *R); /* index of I in the input  */
const uint32_t *oracle_rules_code(const or_rules *R);    /* subset code of X over I   */
const uint32_t *oracle_rules_supp_x(const or_rules *R);  /* supp(X)                   */
void oracle_rules_free(or_rules *R);

uint64_t oracle_result_size(const or_result *r);
uint32_t oracle_result_words(const or_result *r);
const uint64_t *oracle_result_masks(const or_result *r);
const uint32_t *oracle_result_counts(const or_result *r);
int oracle_result_stats(const or_result *r, or_stats *s);
uint64_t oracle_result_trace_len(const or_result *r);
const or_stop *oracle_result_trace(const or_result *r);
void oracle_result_free(or_result *r);

#ifdef __cplusplus
}
#endif
#endif
