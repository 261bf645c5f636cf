// The C ABI of include/dic.h: argument checks, database objects, results,
// the device-memory hook and the library stream.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "dic_internal.h"

struct dic_db {
    uint64_t *rows = nullptr;  // device, n * W, row-major
    uint64_t *vert = nullptr;  // device, m * nw: per-item bitsets over 64-row words
    uint64_t n = 0;
    uint32_t m = 0, W = 0, nw = 0;
    std::mutex mu;             // one mining call at a time on this database
    std::atomic<int> refs{0};  // server requests queued or running on it
};

namespace dic {

const uint64_t *db_rows(dic_db *db) { return db->rows; }
const uint64_t *db_vert(dic_db *db) { return db->vert; }
uint64_t db_n(dic_db *db) { return db->n; }
uint32_t db_m(dic_db *db) { return db->m; }
uint32_t db_W(dic_db *db) { return db->W; }
void db_ref(dic_db *db, int delta) { db->refs += delta; }
uint64_t db_bytes(dic_db *db)
{
    return alloc_bytes(8ull * db->n * db->W) + alloc_bytes(8ull * db->m * db->nw);
}
std::mutex &db_mutex(dic_db *db) { return db->mu; }

namespace {

thread_local std::string t_err;

std::mutex g_cfg_mu;
void *(*g_alloc)(size_t, void *) = nullptr;
void (*g_free)(void *, void *) = nullptr;
void *g_user_stream = nullptr;
hipStream_t g_stream = nullptr;
// Blocks from a caller's allocator, each with the free function and stream
// it came with: a block goes back to the allocator that made it even after
// the allocator was changed (engines are pooled and outlive such changes).
struct UserBlock {
    void (*free_fn)(void *, void *);
    void *stream;
};
std::map<void *, UserBlock> g_user_blocks;

// Small caching allocator over hipMalloc: freed blocks are kept by size and
// handed out again to requests that fit (a mining run allocates and frees
// the same few sizes over and over).
std::mutex g_cache_mu;
std::multimap<size_t, void *> g_cache;
std::map<void *, size_t> g_sizes;
size_t g_cached_bytes = 0;
constexpr size_t CACHE_LIMIT = 32ull << 30;

size_t round_size(size_t b) { return (size_t)alloc_bytes(b); }

}  // namespace

void set_error(const std::string &msg) { t_err = msg; }

void *dev_alloc(size_t bytes)
{
    void *(*alloc)(size_t, void *) = nullptr;
    UserBlock ub{};
    {
        std::lock_guard<std::mutex> g(g_cfg_mu);
        alloc = g_alloc;
        ub = UserBlock{g_free, g_user_stream};
    }
    if (alloc) {  // the caller's functions run without the library's locks held
        void *p = alloc(bytes, ub.stream);
        if (p) {
            std::lock_guard<std::mutex> g(g_cfg_mu);
            g_user_blocks[p] = ub;
        }
        return p;
    }
    const size_t r = round_size(bytes);
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_cache.lower_bound(r);
        if (it != g_cache.end() && it->first <= 2 * r + (8u << 20)) {
            void *p = it->second;
            g_cached_bytes -= it->first;
            g_cache.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, r) != hipSuccess) {
        (void)hipGetLastError();
        // give the cache back to the runtime and try once more
        std::lock_guard<std::mutex> g(g_cache_mu);
        for (auto &kv : g_cache) {
            (void)hipFree(kv.second);
            g_sizes.erase(kv.second);
        }
        g_cache.clear();
        g_cached_bytes = 0;
        if (hipMalloc(&p, r) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_sizes[p] = r;
    return p;
}

void dev_free(void *p)
{
    if (!p)
        return;
    UserBlock ub{};
    {
        std::lock_guard<std::mutex> g(g_cfg_mu);
        auto u = g_user_blocks.find(p);
        if (u != g_user_blocks.end()) {
            ub = u->second;
            g_user_blocks.erase(u);
        }
    }
    if (ub.free_fn) {
        ub.free_fn(p, ub.stream);
        return;
    }
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto it = g_sizes.find(p);
    if (it == g_sizes.end())
        return;  // not ours
    if (g_cached_bytes + it->second > CACHE_LIMIT) {
        (void)hipFree(p);
        g_sizes.erase(it);
        return;
    }
    g_cache.emplace(it->second, p);
    g_cached_bytes += it->second;
}

hipStream_t lib_stream()
{
    std::lock_guard<std::mutex> g(g_cfg_mu);
    if (g_user_stream)
        return (hipStream_t)g_user_stream;
    if (!g_stream) {
        if (hipStreamCreateWithFlags(&g_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            g_stream = nullptr;
        }
    }
    return g_stream;
}

}  // namespace dic

using namespace dic;

#define API_TRY(x)                                                                      \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#x) + " failed: " + hipGetErrorString(e_));           \
            return DIC_E_DEVICE;                                                        \
        }                                                                               \
    } while (0)

extern "C" {

const char *dic_last_error(void) { return t_err.c_str(); }

int dic_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *),
                      void *stream)
{
    if ((alloc == nullptr) != (free_fn == nullptr)) {
        set_error("dic_set_allocator: give both functions or neither");
        return DIC_E_INVAL;
    }
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_alloc = alloc;
    g_free = free_fn;
    g_user_stream = stream;
    return DIC_OK;
}

int dic_set_option(const char *name, int64_t value)
{
    if (name && std::strcmp(name, "profile") == 0 && (value == 0 || value == 1)) {
        set_profiling((int)value);
        return DIC_OK;
    }
    if (name && std::strcmp(name, "graphs") == 0 && (value == 0 || value == 1)) {
        set_use_graphs(value != 0);
        return DIC_OK;
    }
    if (name && std::strcmp(name, "init") == 0 && (value == 0 || value == 1)) {
        set_init_mode((uint32_t)value);
        return DIC_OK;
    }
    if (name && std::strcmp(name, "poison") == 0 && value >= 0 && value <= 255) {
        set_poison((int)value);
        return DIC_OK;
    }
    if (name && std::strcmp(name, "layout") == 0 && (value == 0 || value == 1)) {
        set_count_layout(value ? LAYOUT_VERTICAL : LAYOUT_ROWS);
        return DIC_OK;
    }
    if (name && set_knob(name, value) == DIC_OK)
        return DIC_OK;
    set_error(std::string("dic_set_option: unknown option or value ") + (name ? name : "(null)"));
    return DIC_E_INVAL;
}

static int check_shape(uint64_t n, uint32_t m)
{
    if (n == 0 || n >= 0xFFFFFFFFull) {
        set_error("n must be in [1, 2^32 - 2]");
        return DIC_E_INVAL;
    }
    if (m == 0 || m > MAX_ITEMS) {
        set_error("m must be in [1, 4096]");
        return DIC_E_INVAL;
    }
    return DIC_OK;
}

static int new_db(uint64_t n, uint32_t m, dic_db **out)
{
    dic_db *db = new (std::nothrow) dic_db;
    if (!db) {
        set_error("host allocation failed");
        return DIC_E_NOMEM;
    }
    db->n = n;
    db->m = m;
    db->W = (m + 63u) / 64u;
    db->nw = (uint32_t)((n + 63u) / 64u);
    db->rows = (uint64_t *)dev_alloc(8ull * n * db->W);
    db->vert = (uint64_t *)dev_alloc(8ull * m * db->nw);
    if (!db->rows || !db->vert) {
        dev_free(db->rows);
        dev_free(db->vert);
        delete db;
        set_error("device allocation failed for the database");
        return DIC_E_NOMEM;
    }
    *out = db;
    return DIC_OK;
}

static void delete_db(dic_db *db)
{
    dev_free(db->rows);
    dev_free(db->vert);
    delete db;
}

// The per-item bitset copy of a database whose rows are on the device
// (the layout counted by default); enqueued on s.
static void build_vertical(dic_db *db, hipStream_t s)
{
    launch_transpose(db->rows, db->n, db->m, db->vert, db->nw, s);
}

int dic_load_db(const uint64_t *rows, uint64_t n, uint32_t m, dic_db **out)
{
    if (!out) {
        set_error("dic_load_db: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    if (!rows) {
        set_error("dic_load_db: rows is NULL");
        return DIC_E_INVAL;
    }
    int rc = check_shape(n, m);
    if (rc)
        return rc;
    const uint32_t W = (m + 63u) / 64u;
    if (m & 63u) {
        const uint64_t pad = ~((1ull << (m & 63u)) - 1ull);
        for (uint64_t r = 0; r < n; ++r)
            if (rows[r * W + W - 1] & pad) {
                set_error("dic_load_db: row " + std::to_string(r) + " has a bit at or above m set");
                return DIC_E_INVAL;
            }
    }
    dic_db *db = nullptr;
    if ((rc = new_db(n, m, &db)))
        return rc;
    hipStream_t s = lib_stream();
    bool ok = hipMemcpyAsync(db->rows, rows, 8ull * n * W, hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok)
        build_vertical(db, s);
    if (!ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("dic_load_db: copy to device failed");
        delete_db(db);
        return DIC_E_DEVICE;
    }
    *out = db;
    return DIC_OK;
}

int dic_load_db_device(const uint64_t *rows, uint64_t n, uint32_t m, dic_db **out)
{
    if (!out) {
        set_error("dic_load_db_device: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    if (!rows) {
        set_error("dic_load_db_device: rows is NULL");
        return DIC_E_INVAL;
    }
    int rc = check_shape(n, m);
    if (rc)
        return rc;
    dic_db *db = nullptr;
    if ((rc = new_db(n, m, &db)))
        return rc;
    hipStream_t s = lib_stream();
    uint32_t *bad = (uint32_t *)dev_alloc(4);
    uint32_t hbad = 0;
    bool ok = bad && hipMemsetAsync(bad, 0, 4, s) == hipSuccess &&
              hipMemcpyAsync(db->rows, rows, 8ull * n * db->W, hipMemcpyDeviceToDevice, s) ==
                  hipSuccess;
    if (ok && (m & 63u))
        launch_check_padding(db->rows, n, m, bad, s);
    if (ok)
        build_vertical(db, s);
    ok = ok && hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    dev_free(bad);
    if (!ok) {
        set_error("dic_load_db_device: device copy failed");
        delete_db(db);
        return DIC_E_DEVICE;
    }
    if (hbad) {
        set_error("dic_load_db_device: a row has a bit at or above m set");
        delete_db(db);
        return DIC_E_INVAL;
    }
    *out = db;
    return DIC_OK;
}

int dic_load_db_lists(const uint32_t *items, const uint64_t *offsets, uint64_t n, uint32_t m,
                      dic_db **out)
{
    if (!out) {
        set_error("dic_load_db_lists: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    int rc = check_shape(n, m);
    if (rc)
        return rc;
    if (!offsets || offsets[0] != 0) {
        set_error("dic_load_db_lists: offsets must start at 0");
        return DIC_E_INVAL;
    }
    for (uint64_t t = 0; t < n; ++t)
        if (offsets[t + 1] < offsets[t]) {
            set_error("dic_load_db_lists: offsets must not decrease");
            return DIC_E_INVAL;
        }
    const uint64_t nnz = offsets[n];
    if (nnz && !items) {
        set_error("dic_load_db_lists: items is NULL");
        return DIC_E_INVAL;
    }
    for (uint64_t e = 0; e < nnz; ++e)
        if (items[e] >= m) {
            set_error("dic_load_db_lists: item " + std::to_string(items[e]) + " >= m");
            return DIC_E_INVAL;
        }
    dic_db *db = nullptr;
    if ((rc = new_db(n, m, &db)))
        return rc;
    hipStream_t s = lib_stream();
    uint32_t *d_items = (uint32_t *)dev_alloc(4 * (nnz ? nnz : 1));
    uint64_t *d_off = (uint64_t *)dev_alloc(8 * (n + 1));
    bool ok = d_items && d_off &&
              (nnz == 0 ||
               hipMemcpyAsync(d_items, items, 4 * nnz, hipMemcpyHostToDevice, s) == hipSuccess) &&
              hipMemcpyAsync(d_off, offsets, 8 * (n + 1), hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok) {
        launch_pack_lists(d_items, d_off, n, db->W, db->rows, s);
        build_vertical(db, s);
    }
    ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
    dev_free(d_items);
    dev_free(d_off);
    if (!ok) {
        set_error("dic_load_db_lists: device work failed");
        delete_db(db);
        return DIC_E_DEVICE;
    }
    *out = db;
    return DIC_OK;
}

uint64_t dic_db_rows(const dic_db *db) { return db ? db->n : 0; }
uint32_t dic_db_items(const dic_db *db) { return db ? db->m : 0; }

int dic_free_db(dic_db *db)
{
    if (!db)
        return DIC_OK;
    if (db->refs.load() > 0) {
        set_error("dic_free_db: database is referenced by queued or running requests");
        return DIC_E_BUSY;
    }
    {
        std::lock_guard<std::mutex> g(db->mu);  // wait for a running dic_mine
    }
    delete_db(db);
    return DIC_OK;
}

static int check_mine_args(const dic_db *db, double minsup, uint64_t M)
{
    if (!db) {
        set_error("database is NULL");
        return DIC_E_INVAL;
    }
    if (!(minsup > 0.0)) {
        set_error("minsup must be > 0 (and not NaN)");
        return DIC_E_INVAL;
    }
    if (M == 0) {
        set_error("M must be >= 1");
        return DIC_E_INVAL;
    }
    return DIC_OK;
}

static int to_result(MineOutput &o, uint32_t W, dic_result **out)
{
    dic_result *r = new (std::nothrow) dic_result;
    if (!r) {
        set_error("host allocation failed");
        return DIC_E_NOMEM;
    }
    r->W = W;
    r->masks = std::move(o.masks);
    r->counts = std::move(o.counts);
    r->trace = std::move(o.trace);
    r->stats = o.stats;
    *out = r;
    return DIC_OK;
}

int dic_mine(dic_db *db, double minsup, uint64_t M, dic_result **out)
{
    if (!out) {
        set_error("dic_mine: out is NULL");
        return DIC_E_INVAL;
    }
    *out = nullptr;
    int rc = check_mine_args(db, minsup, M);
    if (rc)
        return rc;
    std::lock_guard<std::mutex> g(db->mu);
    std::vector<MineRequest> reqs{{db->rows, db->vert, (uint32_t)db->n, db->m, minsup, M}};
    std::vector<MineOutput> outs;
    rc = run_jobs(reqs, outs, lib_stream());
    if (rc)
        return rc;
    if (outs[0].status)
        return outs[0].status;
    return to_result(outs[0], db->W, out);
}

int dic_batch(dic_db *const *dbs, const double *minsup, const uint64_t *M, uint32_t count,
              dic_result **outs, int *status)
{
    if (!outs || (count && (!dbs || !minsup || !M))) {
        set_error("dic_batch: NULL argument");
        return DIC_E_INVAL;
    }
    for (uint32_t i = 0; i < count; ++i) {
        outs[i] = nullptr;
        if (status)
            status[i] = DIC_OK;
    }
    std::vector<MineRequest> reqs;
    std::vector<uint32_t> where;
    int first_rc = DIC_OK;
    for (uint32_t i = 0; i < count; ++i) {
        int rc = check_mine_args(dbs[i], minsup[i], M[i]);
        if (rc) {
            if (status)
                status[i] = rc;
            if (!first_rc)
                first_rc = rc;
            continue;
        }
        reqs.push_back({dbs[i]->rows, dbs[i]->vert, (uint32_t)dbs[i]->n, dbs[i]->m, minsup[i],
                        M[i]});
        where.push_back(i);
    }
    if (reqs.empty())
        return first_rc;
    // lock each distinct database once, in address order
    std::vector<dic_db *> locks;
    for (uint32_t i : where)
        locks.push_back(dbs[i]);
    std::sort(locks.begin(), locks.end());
    locks.erase(std::unique(locks.begin(), locks.end()), locks.end());
    for (dic_db *d : locks)
        d->mu.lock();
    std::vector<MineOutput> res;
    int rc = run_jobs(reqs, res, lib_stream());
    for (dic_db *d : locks)
        d->mu.unlock();
    if (rc) {
        for (uint32_t i : where)
            if (status)
                status[i] = rc;
        return rc;
    }
    for (size_t t = 0; t < where.size(); ++t) {
        const uint32_t i = where[t];
        int e = res[t].status;
        if (!e)
            e = to_result(res[t], dbs[i]->W, &outs[i]);
        if (status)
            status[i] = e;
        if (e && !first_rc)
            first_rc = e;
    }
    return first_rc;
}

uint64_t dic_result_size(const dic_result *r) { return r ? r->counts.size() : 0; }
uint32_t dic_result_words(const dic_result *r) { return r ? r->W : 0; }
const uint64_t *dic_result_masks(const dic_result *r)
{
    return r && !r->masks.empty() ? r->masks.data() : nullptr;
}
const uint32_t *dic_result_counts(const dic_result *r)
{
    return r && !r->counts.empty() ? r->counts.data() : nullptr;
}

int dic_result_stats(const dic_result *r, dic_stats *s)
{
    if (!r || !s) {
        set_error("dic_result_stats: NULL argument");
        return DIC_E_INVAL;
    }
    *s = r->stats;
    return DIC_OK;
}

const dic_stop_trace *dic_result_trace(const dic_result *r, uint64_t *n_stops)
{
    if (n_stops)
        *n_stops = r ? r->trace.size() : 0;
    return r && !r->trace.empty() ? r->trace.data() : nullptr;
}

void dic_result_free(dic_result *r) { delete r; }

}  // extern "C"
