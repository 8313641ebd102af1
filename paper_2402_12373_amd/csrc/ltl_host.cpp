// Host runtime of the LTL learner: the C-ABI of include/ltl.h.
//
// Per job it lays out the specification as characteristic-matrix rows, carves
// the caller's workspace into fixed tables (row metadata, atom matrices, the
// language-cache hash table, recipes) and the level arena, and drives the
// level loop of Sec. 3 (enum): for each cost level, build the canonical block
// list (connective x split), run the evaluation kernel, read back 64 bytes of
// counters, compact the representatives, write the new entries and verify
// every presumed duplicate in full.  All matrix work runs in the kernels of
// ltl_kernels.hip; the host only plans, launches and reads counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ltl.h"
#include "ltl_internal.h"

using namespace ltl;

namespace {

constexpr int ORDER[7] = {LTL_F, LTL_U, LTL_G, LTL_X, LTL_AND, LTL_OR, LTL_NOT};   // Sec. 3 listing
constexpr uint32_t MAX_GRID = 8192;
// Row-split levels: the number of waves their row chunks aim for.
#ifndef LTL_TARGET_WAVES
#define LTL_TARGET_WAVES 8192
#endif
constexpr uint64_t TARGET_WAVES = LTL_TARGET_WAVES;
// Levels with fewer tiles than this are row-split (waves take chunks of row
// blocks), so that small levels are not one long chain of dependent row-block
// loads per wave (a tuning constant; ltl_ctx_opts.split_tiles overrides it).
constexpr uint64_t SPLIT_TILES = 8192;
constexpr uint64_t MIN_CHUNK = 4;        // row blocks per work item at least (per-item fixed cost)
// Whole-row levels: the waves the verification and the write pass aim for (a tuning constant;
// with jobs in flight on several streams, 32768 beat 65536 by 1-2% and matched it on one stream)
#ifndef LTL_PASS_WAVES
#define LTL_PASS_WAVES 32768
#endif
constexpr uint64_t PASS_WAVES = LTL_PASS_WAVES;
constexpr uint32_t RUC_SPLIT_MIN_BLOCKS = 64;   // scale (32 row blocks): whole-row 2.47e8 vs row-split 2.02e8
                                                // candidates/s; long (650): row-split 1.09e7 vs whole-row 0.62e7
constexpr uint64_t PASS_MIN_CHUNK = 16;  // row blocks per chunk at least (per-item owner and claim lookups)
// per-level upload, one copy: [counters init (256 B) | canonical blocks | blocks by
// class | all blocks, one tile numbering]
constexpr uint64_t UPLOAD_BYTES = 256 + 3 * sizeof(Block) * MAX_BLOCKS;
// the level's "cannot be kept" flag, a cache line away from the counters in the upload area
constexpr uint64_t FULL_FLAG_OFF = 128;
static_assert(sizeof(Counters) <= FULL_FLAG_OFF, "the counters precede the flag");
// pinned staging: the upload image, then 256 B for the counters read back
constexpr uint64_t PINNED_BYTES = UPLOAD_BYTES + 256;

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

bool is_unary(int op) { return op == LTL_NOT || op == LTL_X || op == LTL_F || op == LTL_G; }

}  // namespace

// Whole-row levels run the U class (VALU-bound) on a second stream, beside the
// unary and AND/OR classes (HBM-bound), joined before the compaction (a tuning switch).
#ifndef LTL_FORK_U
#define LTL_FORK_U 1
#endif
#ifndef LTL_ANDOR_EVAL_AUX
#define LTL_ANDOR_EVAL_AUX 1
#endif

struct ltl_ctx {
    ltl_ctx_opts o;
    hipStream_t s = nullptr;
    hipStream_t aux = nullptr;       // second stream of the context (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::mutex *big_mu = nullptr;    // batch lanes with LTL_BATCH_BIG_ALONE: one whole-row level at a time
    std::vector<hipEvent_t> events;  // timing events, kept across jobs (created on first use)
    bool busy = false;
    char *pinned = nullptr;          // page-locked host staging: two block tables + counters
    char *jpin = nullptr;            // page-locked staging of a job's row tables (grown on demand)
    uint64_t jpin_bytes = 0;
    uint32_t table_clean_log2 = 0;   // the hash table at the start of the workspace is empty (this size)
    // batch lanes with a shared budget: the lane's own hash table and entry tables (24
    // bytes a slot), kept clean across jobs, outside the job regions
    char *cache = nullptr;
    uint32_t cache_slots_log2 = 0;
    uint64_t pool_total = 0;         // ... and the pool their regions come from
    std::vector<uint32_t> fp_keys;   // the fingerprint keys' sequence, as far as jobs have needed it
    // allocation-free contexts (ltl_learn_noalloc): host staging in ordinary memory instead
    // of page-locked buffers
    bool noalloc = false;
    std::vector<char> heap_pinned, heap_jpin;
};

struct LevelInfo {
    bool evaluated = false;
    bool stored = false;
    uint32_t n = 0;            // entries (distinct new languages)
    uint32_t gid_base = 0;     // global id of the first entry
    uint64_t cands = 0;
    uint64_t first = LTL_NO_SOLUTION;
    uint64_t colliders = 0;
    uint64_t alg_bytes = 0;    // one matrix per candidate (none written if not stored) + children once per tile
    double ms = 0.0;
    std::vector<Block> blocks;
    std::vector<int> a_level, b_level;   // child levels per block (host decode)
};

struct TimedLaunch {
    int kind;
    hipEvent_t e0, e1;
};

struct ltl_job {
    ltl_ctx *ctx = nullptr;
    hipStream_t s = nullptr;
    uint32_t A = 0, T = 0, npos = 0, nneg = 0;
    std::vector<uint64_t> off;     // host copy of offsets
    uint64_t TB = 0;
    ltl_opset ops{};
    uint32_t bound = 0;
    uint32_t wbits = 32;
    bool mw = false;
    uint32_t R = 0, NB = 0, ksteps = 0, maxw = 1;
    uint64_t wbytes = 4, cm_bytes = 0;
    std::vector<uint32_t> row0, nwords;   // per trace: first row, words
    // workspace
    char *ws = nullptr;
    uint64_t wsb = 0, used = 0;
    Counters *ctr = nullptr;
    void *valid = nullptr, *sepm = nullptr, *sepw = nullptr, *atoms = nullptr;
    uint64_t *nxt = nullptr, *tfp = nullptr, *offsets_d = nullptr;
    uint32_t *key = nullptr;
    uint32_t *ruc_meta = nullptr;            // relaxed check: key metadata per row half
    unsigned long long *entry_key = nullptr; // relaxed check: key per global entry
    bool ruc_pack = false;                   // keys in pack form (FKP, or matrices of <= 126 bits)
    uint32_t *row_trace = nullptr, *row_word = nullptr, *letters_d = nullptr;
    Block *blocks_d = nullptr;       // canonical order (candidate decode)
    Block *blocks_cls_d = nullptr;   // grouped by connective class, class-local tiles
    unsigned long long *tkey = nullptr;
    uint32_t *tval = nullptr;
    uint32_t slots_log2 = 0;
    uint32_t *recipe = nullptr;
    uint32_t *entry_slot = nullptr;  // per global entry: its hash slot (to empty the table afterwards)
    uint32_t *store = nullptr;       // per global entry: arena position of its matrix
    std::vector<uint32_t> recipe_h;  // host copy of recipe[0 .. size) (formula reconstruction)
    uint64_t recipe_cap = 0, max_entries = 0;
    bool table_consistent = true;    // every claimed slot belongs to a finalized entry
    char *arena = nullptr;
    uint64_t arena_region = 0;     // bytes from arena to the end of the workspace
    uint64_t total_entries = 0;    // entries in the arena
    uint64_t stored_entries = 0;   // entries of stored levels
    std::vector<LevelInfo> L;
    uint32_t levels_done = 0;
    int status = LTL_NOT_FOUND;
    bool searching = true;
    uint32_t sol_level = 0;
    uint64_t sol_index = LTL_NO_SOLUTION;
    uint64_t colliders = 0;
    bool timing = false;
    bool timing_level = false;       // one event pair per level only
    double span_ms = 0.0;            // level spans collected (timing_level)
    std::vector<TimedLaunch> pending;
    std::vector<Block> grouped;
    Counters ctr_init{};
    std::vector<hipEvent_t> event_pool;
    double kernel_ms[LTL_K_KINDS] = {0};
    uint32_t kernel_launches[LTL_K_KINDS] = {0};
    // why the job ran out of memory: 0 not, 1 tables or level scratch did not fit (or the
    // hash table overflowed), 2 a level's new entries did not fit the arena (oom_new of
    // them), 3 the stored entries exceeded the entry cap
    int oom_kind = 0;
    uint64_t oom_new = 0;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return LTL_E_DEVICE;            \
    } while (0)
#define HIP_TRY_E(expr)                                       \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return e_;                      \
    } while (0)

static void *ws_take(ltl_job *j, uint64_t bytes) {
    uint64_t at = align_up(j->used, 256);
    if (at + bytes > j->wsb) return nullptr;
    j->used = at + bytes;
    return j->ws + at;
}

static hipEvent_t pool_event(ltl_job *j) {
    if (!j->event_pool.empty()) {
        hipEvent_t e = j->event_pool.back();
        j->event_pool.pop_back();
        return e;
    }
    if (!j->ctx->events.empty()) {       // the context's events, kept across jobs
        hipEvent_t e = j->ctx->events.back();
        j->ctx->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records events around a launch when timing is on.
struct Timer {
    ltl_job *j;
    TimedLaunch t{};
    bool on = false;
    // counts `dispatches` kernel launches for the kind (rocprofv3 counts dispatches too)
    Timer(ltl_job *job, int kind, uint32_t dispatches = 1) : j(job) {
        j->kernel_launches[kind] += dispatches;
        if (!j->timing) return;
        t.kind = kind;
        t.e0 = pool_event(j);
        t.e1 = pool_event(j);
        if (t.e0 && t.e1) {
            (void)hipEventRecord(t.e0, j->s);
            on = true;
        }
    }
    ~Timer() {
        if (on) {
            (void)hipEventRecord(t.e1, j->s);
            j->pending.push_back(t);
        }
    }
};

// One event pair around a whole level, from its first to its last kernel
// (LTL_CTX_TIMING_LEVEL: two events per level instead of two per kernel group).
struct LevelSpan {
    ltl_job *j;
    TimedLaunch t{};
    bool on = false;
    explicit LevelSpan(ltl_job *job) : j(job) {
        if (!j->timing_level) return;
        t.kind = -1;
        t.e0 = pool_event(j);
        t.e1 = pool_event(j);
        if (t.e0 && t.e1 && hipEventRecord(t.e0, j->s) == hipSuccess) {
            on = true;
        } else {
            if (t.e0) j->event_pool.push_back(t.e0);
            if (t.e1) j->event_pool.push_back(t.e1);
        }
    }
    void end() {
        if (!on) return;
        (void)hipEventRecord(t.e1, j->s);
        j->pending.push_back(t);
        on = false;
    }
    ~LevelSpan() { end(); }
};

// Adds the elapsed times of completed launches; returns their sum.
static double collect_times(ltl_job *j) {
    double tot = 0.0;
    for (auto &t : j->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.e0, t.e1) == hipSuccess) {
            if (t.kind >= 0) j->kernel_ms[t.kind] += ms;
            else j->span_ms += ms;                  // a whole level (timing_level)
            tot += ms;
        }
        j->event_pool.push_back(t.e0);
        j->event_pool.push_back(t.e1);
    }
    j->pending.clear();
    return tot;
}

static int sync_read_counters(ltl_job *j, Counters *host) {
    Counters *pin = (Counters *)(j->ctx->pinned + UPLOAD_BYTES);
    HIP_TRY(hipMemcpyAsync(pin, j->ctr, sizeof(Counters), hipMemcpyDeviceToHost, j->s));
    HIP_TRY(hipStreamSynchronize(j->s));
    *host = *pin;
    return LTL_OK;
}

template <typename T>
static Rows<T> make_rows(const ltl_job *j) {
    Rows<T> r;
    r.valid = (const T *)j->valid;
    r.sepm = (const T *)j->sepm;
    r.sepw = (const T *)j->sepw;
    r.nxt = j->nxt;
    r.key = j->key;
    r.R = j->R;
    r.NB = j->NB;
    r.ksteps = j->ksteps;
    r.maxw = j->maxw;
    return r;
}

// ---------------------------------------------------------------------------
// ABI: context
// ---------------------------------------------------------------------------
extern "C" int ltl_ctx_create(const ltl_ctx_opts *opts, ltl_ctx **out) {
    if (!opts || !out || !opts->workspace || opts->workspace_bytes < LTL_MIN_WORKSPACE) return LTL_E_INVAL;
    if (((uintptr_t)opts->workspace) & 255u) return LTL_E_INVAL;
    if (opts->fp_bits > 64 || opts->ruc_key_bits > 125) return LTL_E_INVAL;
    if (opts->word_bits != 0 && opts->word_bits != 32 && opts->word_bits != 64) return LTL_E_INVAL;
    if (opts->hash_slots_log2 != 0 && (opts->hash_slots_log2 < 8 || opts->hash_slots_log2 > 31)) return LTL_E_INVAL;
    if (hipSetDevice(opts->device) != hipSuccess) return LTL_E_DEVICE;
    ltl_ctx *c = new (std::nothrow) ltl_ctx;
    if (!c) return LTL_E_INVAL;
    c->o = *opts;
    c->s = (hipStream_t)opts->stream;
    if (hipHostMalloc((void **)&c->pinned, PINNED_BYTES, hipHostMallocDefault) != hipSuccess ||
        (LTL_FORK_U && !(opts->flags & LTL_CTX_ONE_STREAM) &&
         (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess))) {
        ltl_ctx_destroy(c);
        return LTL_E_DEVICE;
    }
    *out = c;
    return LTL_OK;
}

extern "C" void ltl_ctx_destroy(ltl_ctx *ctx) {
    if (!ctx) return;
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    for (auto e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->jpin) (void)hipHostFree(ctx->jpin);
    delete ctx;
}

extern "C" const char *ltl_status_str(int st) {
    switch (st) {
    case LTL_OK: return "ok";
    case LTL_NOT_FOUND: return "no separating formula within the cost bound";
    case LTL_E_INVAL: return "invalid argument";
    case LTL_E_INCONSISTENT: return "a trace is both positive and negative";
    case LTL_E_TOO_LONG: return "trace too long";
    case LTL_E_OOM: return "out of workspace or entry cap";
    case LTL_E_DEVICE: return "HIP device error";
    case LTL_E_STATE: return "call out of order";
    case LTL_E_BUFFER: return "output buffer too small";
    default: return "unknown status";
    }
}

// ---------------------------------------------------------------------------
// Job creation: validation, row layout, workspace carve, atom packing
// ---------------------------------------------------------------------------
static int job_setup(ltl_job *j, const ltl_spec *spec) {
    ltl_ctx *c = j->ctx;
    j->ws = (char *)c->o.workspace;
    j->wsb = c->o.workspace_bytes;
    j->used = 0;
    j->s = c->s;
    j->timing = (c->o.flags & LTL_CTX_TIMING) != 0;
    j->timing_level = !j->timing && (c->o.flags & LTL_CTX_TIMING_LEVEL) != 0;
    const uint32_t T = j->T;

    // offsets on the host (device specs: copy them back; the letters stay on the device)
    j->off.resize((size_t)T + 1);
    if (spec->flags & LTL_SPEC_DEVICE) {
        // on the job's own stream, not the null stream (no wait behind other streams' work)
        HIP_TRY(hipMemcpyAsync(j->off.data(), spec->offsets, sizeof(uint64_t) * ((size_t)T + 1),
                               hipMemcpyDeviceToHost, j->s));
        HIP_TRY(hipStreamSynchronize(j->s));
    } else {
        memcpy(j->off.data(), spec->offsets, sizeof(uint64_t) * ((size_t)T + 1));
    }
    if (j->off[0] != 0) return LTL_E_INVAL;
    uint64_t maxlen = 0;
    for (uint32_t t = 0; t < T; ++t) {
        if (j->off[t + 1] <= j->off[t]) return LTL_E_INVAL;          // empty trace (or decreasing)
        maxlen = std::max<uint64_t>(maxlen, j->off[t + 1] - j->off[t]);
    }
    if (maxlen > LTL_MAX_TRACE_LEN) return LTL_E_TOO_LONG;
    j->TB = j->off[T];

    // word size and row layout
    uint32_t wb = c->o.word_bits ? c->o.word_bits : (maxlen <= 32 ? 32u : 64u);
    if (wb == 32 && maxlen > 32) return LTL_E_TOO_LONG;
    j->wbits = wb;
    j->wbytes = wb / 8;
    j->row0.resize(T);
    j->nwords.resize(T);
    uint64_t r = 0;
    uint32_t maxw = 1;
    for (uint32_t t = 0; t < T; ++t) {
        const uint64_t len = j->off[t + 1] - j->off[t];
        const uint32_t w = (uint32_t)((len + wb - 1) / wb);
        if ((r & 63u) + w > 64u) r = align_up(r, 64);                 // no trace straddles a row block
        j->row0[t] = (uint32_t)r;
        j->nwords[t] = w;
        r += w;
        maxw = std::max(maxw, w);
    }
    const uint64_t R = align_up(std::max<uint64_t>(r, 1), 64);
    if (R > 0x7FFFFFFFull) return LTL_E_TOO_LONG;
    j->R = (uint32_t)R;
    j->NB = (uint32_t)(R / 64);
    j->maxw = maxw;
    j->mw = (wb == 64 && maxw > 1);     // words of one trace exchange bits across lanes
    uint32_t k = 0;
    while ((1ull << k) < maxlen) ++k;
    j->ksteps = k;
    j->cm_bytes = R * j->wbytes;
    // kernels address rows of a matrix (and of the row tables) with 32-bit byte offsets
    if (j->cm_bytes >= (1ull << 31) || R * 8ull >= (1ull << 31)) return LTL_E_TOO_LONG;

    // host row metadata, written straight into one page-locked image of the device
    // row tables: [valid | sepm | sepw (R words each) | nxt (R x 8 B) | keys (R x 4 B per
    // 32-bit half) | row_trace | row_word (R x 4 B each)], then room for the trace
    // fingerprints read back
    const uint64_t W = wb;
    const uint32_t nkeys = (wb == 64) ? 2u : 1u;
    const uint64_t o_valid = 0, o_sepm = R * j->wbytes, o_sepw = 2 * R * j->wbytes, o_nxt = 3 * R * j->wbytes;
    const uint64_t o_key = o_nxt + R * 8, o_rtr = o_key + R * 4 * nkeys, o_rwd = o_rtr + R * 4;
    // relaxed check: two words per 32-bit half of a row (the key metadata)
    const bool ruc = (c->o.flags & LTL_CTX_RUC) != 0;
    const uint64_t o_ruc = o_rwd + R * 4;
    const uint64_t tables_bytes = o_ruc + (ruc ? R * 8 * nkeys : 0);
    if (ruc && R * 8 * nkeys >= (1ull << 31)) return LTL_E_TOO_LONG;
    const uint64_t o_tfp = align_up(tables_bytes, 256);
    const uint64_t jpin_need = o_tfp + (uint64_t)T * 8;
    if (c->noalloc) {
        if (c->heap_jpin.size() < jpin_need) c->heap_jpin.resize(jpin_need);
        c->jpin = c->heap_jpin.data();
        c->jpin_bytes = c->heap_jpin.size();
    } else if (c->jpin_bytes < jpin_need) {
        if (c->jpin) (void)hipHostFree(c->jpin);
        c->jpin = nullptr;
        c->jpin_bytes = 0;
        if (hipHostMalloc((void **)&c->jpin, jpin_need, hipHostMallocDefault) != hipSuccess) return LTL_E_DEVICE;
        c->jpin_bytes = jpin_need;
    }
    char *img = c->jpin;
    memset(img, 0, tables_bytes);
    uint32_t *row_trace = (uint32_t *)(img + o_rtr);
    uint32_t *row_word = (uint32_t *)(img + o_rwd);
    uint64_t *nxt = (uint64_t *)(img + o_nxt);
    for (uint64_t rr = 0; rr < R; ++rr) row_trace[rr] = 0xFFFFFFFFu;
    auto put = [&](uint64_t off, uint64_t row, uint64_t v) {
        if (wb == 64) ((uint64_t *)(img + off))[row] = v;
        else ((uint32_t *)(img + off))[row] = (uint32_t)v;
    };
    const uint64_t full = (wb == 64) ? ~0ull : 0xFFFFFFFFull;
    const uint64_t msb = 1ull << (wb - 1);
    for (uint32_t t = 0; t < T; ++t) {
        const uint64_t len = j->off[t + 1] - j->off[t];
        for (uint32_t w = 0; w < j->nwords[t]; ++w) {
            const uint64_t row = j->row0[t] + w;
            const uint64_t n = std::min<uint64_t>(W, len - (uint64_t)w * W);
            put(o_valid, row, (n == W) ? full : ((full << (W - n)) & full));
            put(o_sepm, row, (w == 0) ? msb : 0);
            put(o_sepw, row, (w == 0 && t < j->npos) ? msb : 0);
            const uint32_t later = j->nwords[t] - 1 - w;
            const uint32_t lane = (uint32_t)(row & 63u);
            nxt[row] = later ? (((later == 64 ? 0ull : (1ull << later)) - 1ull) << (lane + 1)) : 0ull;
            row_trace[row] = t;
            row_word[row] = w;
        }
    }
    {   // the fingerprint keys: one fixed sequence, generated once per context and copied
        if (c->fp_keys.size() < R * nkeys) {
            uint64_t seed = 0x5eed1e55c0ffee11ull;
            c->fp_keys.resize(R * nkeys);
            for (uint64_t q = 0; q < R * nkeys; ++q) c->fp_keys[q] = (uint32_t)(splitmix64(seed) >> 32) | 1u;
        }
        memcpy(img + o_key, c->fp_keys.data(), R * nkeys * 4);
    }
    if (ruc) {
        // Key metadata of the relaxed check (Sec. 5; FKP, Sec. 7), per 32-bit half of a row
        // (chunk j of trace t: positions 32j..32j+31), top half first:
        //   pack form (FKP, or every matrix of at most 126 bits): the first m_t positions of
        //   each trace, in trace order, fill the key from bit 0 and stop at 126 bits; a half
        //   gets (mask of its kept positions, key bit of its first position);
        //   keyed sums: the odd keys (a, b), top halves of SplitMix64 draws 2i and 2i + 1
        //   of the seed's sequence, i = t * 2^32 + j.
        // Halves past the end of their trace get (0, 0) and add nothing.
        const uint32_t kb = 126;
        std::vector<uint64_t> m(T);
        for (uint32_t t = 0; t < T; ++t) m[t] = j->off[t + 1] - j->off[t];
        j->ruc_pack = (c->o.flags & LTL_CTX_RUC_FKP) || j->TB <= kb;
        if ((c->o.flags & LTL_CTX_RUC_FKP) && j->TB > kb) {
            uint32_t best = 1;
            uint64_t best_d = ~0ull;
            for (uint32_t k = 1; k <= 100; ++k) {
                uint64_t tot = 0;
                for (uint32_t t = 0; t < T; ++t) tot += (m[t] * k + 50) / 100;
                const uint64_t d = tot > kb ? tot - kb : kb - tot;
                if (d < best_d) { best_d = d; best = k; }
            }
            for (uint32_t t = 0; t < T; ++t) m[t] = (m[t] * best + 50) / 100;
        }
        uint32_t *meta = (uint32_t *)(img + o_ruc);     // zeroed with the image
        const uint32_t halves = nkeys;
        uint64_t keyoff = 0;                            // key bit of the current trace's first position
        for (uint32_t t = 0; t < T; ++t) {
            const uint64_t len = j->off[t + 1] - j->off[t];
            for (uint32_t w = 0; w < j->nwords[t]; ++w) {
                const uint64_t row = j->row0[t] + w;
                for (uint32_t hh = 0; hh < halves; ++hh) {
                    const uint64_t jc = (uint64_t)w * halves + hh;      // chunk of the trace
                    if (32 * jc >= len) continue;
                    uint32_t *e = meta + (row * halves + hh) * 2;
                    if (j->ruc_pack) {
                        const uint64_t start = keyoff + 32 * jc;
                        if (32 * jc >= m[t] || start >= kb) continue;
                        const uint64_t kept = std::min<uint64_t>({32, m[t] - 32 * jc, kb - start});
                        e[0] = (uint32_t)(0xFFFFFFFFull << (32 - kept));
                        e[1] = (uint32_t)start;
                    } else {
                        const uint64_t ci = ((uint64_t)t << 32) | jc;
                        // draw i is the mix of seed + (i + 1) gamma; splitmix64 adds gamma first
                        uint64_t st = c->o.ruc_seed + (2 * ci) * 0x9e3779b97f4a7c15ull;
                        e[0] = (uint32_t)(splitmix64(st) >> 32) | 1u;
                        e[1] = (uint32_t)(splitmix64(st) >> 32) | 1u;
                    }
                }
            }
            keyoff += m[t];
        }
    }

    // workspace carve: the language-cache hash table first (12 bytes per slot), at
    // a fixed place so that a context can hand an emptied table to its next job
    uint32_t sl = c->cache ? c->cache_slots_log2 : c->o.hash_slots_log2;
    if (!sl) {
        sl = 26;
        while (sl > 10 && (24ull << sl) > j->wsb / 4) --sl;
    }
    j->slots_log2 = sl;
    const uint64_t nslots = 1ull << sl;
    j->max_entries = c->o.max_entries ? c->o.max_entries : nslots / 2;
    j->recipe_cap = nslots;
    if (c->cache) {       // the context's own language cache (batch lanes with a shared budget)
        j->tkey = (unsigned long long *)c->cache;
        j->tval = (uint32_t *)(c->cache + nslots * 8);
        j->recipe = j->tval + nslots;
        j->entry_slot = j->recipe + nslots;
        j->store = j->entry_slot + nslots;
    } else {
        j->tkey = (unsigned long long *)ws_take(j, nslots * 8);
        j->tval = (uint32_t *)ws_take(j, nslots * 4);
        j->recipe = (uint32_t *)ws_take(j, nslots * 4);
        j->entry_slot = (uint32_t *)ws_take(j, nslots * 4);
        j->store = (uint32_t *)ws_take(j, nslots * 4);
    }
    if (!j->tkey || !j->tval || !j->recipe || !j->entry_slot || !j->store) return LTL_E_OOM;

    char *upload = (char *)ws_take(j, UPLOAD_BYTES);   // counters, then the level's block tables
    j->ctr = (Counters *)upload;
    char *tables = (char *)ws_take(j, tables_bytes);
    if (tables) {
        j->valid = tables + o_valid;
        j->sepm = tables + o_sepm;
        j->sepw = tables + o_sepw;
        j->nxt = (uint64_t *)(tables + o_nxt);
        j->key = (uint32_t *)(tables + o_key);
        j->row_trace = (uint32_t *)(tables + o_rtr);
        j->row_word = (uint32_t *)(tables + o_rwd);
        j->ruc_meta = ruc ? (uint32_t *)(tables + o_ruc) : nullptr;
    }
    if (ruc) {
        j->entry_key = (unsigned long long *)ws_take(j, nslots * 16);
        if (!j->entry_key) return LTL_E_OOM;
    }
    j->atoms = ws_take(j, (uint64_t)j->A * R * j->wbytes);
    j->tfp = (uint64_t *)ws_take(j, (uint64_t)T * 8);
    j->blocks_d = upload ? (Block *)(upload + 256) : nullptr;
    j->blocks_cls_d = j->blocks_d;   // placed after the canonical blocks of each level
    if (!(spec->flags & LTL_SPEC_DEVICE)) {
        j->letters_d = (uint32_t *)ws_take(j, j->TB * 4);
        j->offsets_d = (uint64_t *)ws_take(j, ((uint64_t)T + 1) * 8);
    } else {
        j->letters_d = (uint32_t *)spec->letters;
        j->offsets_d = (uint64_t *)spec->offsets;
    }
    if (!j->ctr || !j->valid || !j->sepm || !j->sepw || !j->nxt || !j->key || !j->row_trace || !j->row_word ||
        !j->atoms || !j->tfp || !j->blocks_d || !j->blocks_cls_d || !j->letters_d || !j->offsets_d)
        return LTL_E_OOM;
    j->arena = j->ws + align_up(j->used, 256);
    if ((uint64_t)(j->arena - j->ws) >= j->wsb) return LTL_E_OOM;
    j->arena_region = j->wsb - (uint64_t)(j->arena - j->ws);

    // uploads: the row tables in one copy
    HIP_TRY(hipMemcpyAsync(tables, img, tables_bytes, hipMemcpyHostToDevice, j->s));
    if (!(spec->flags & LTL_SPEC_DEVICE)) {
        HIP_TRY(hipMemcpyAsync(j->letters_d, spec->letters, j->TB * 4, hipMemcpyHostToDevice, j->s));
        HIP_TRY(hipMemcpyAsync(j->offsets_d, spec->offsets, ((uint64_t)T + 1) * 8, hipMemcpyHostToDevice, j->s));
    }
    static_assert(sizeof(Counters) % 4 == 0, "counters are cleared as words");
    HIP_TRY(launch_zero2((uint32_t *)j->ctr, sizeof(Counters) / 4, nullptr, 0, j->s));
    {
        Timer tm(j, LTL_K_INTAKE, c->table_clean_log2 != sl ? 3u : 2u);
        if (c->table_clean_log2 != sl) HIP_TRY(launch_table_init(j->tkey, j->tval, nslots, j->s));
        c->table_clean_log2 = 0;   // dirty until the job empties its slots again
        if (wb == 64)
            HIP_TRY(Launch<uint64_t>::pack(j->letters_d, j->offsets_d, j->row_trace, j->row_word, j->R, j->A,
                                           (uint64_t *)j->atoms, j->ctr, j->s));
        else
            HIP_TRY(Launch<uint32_t>::pack(j->letters_d, j->offsets_d, j->row_trace, j->row_word, j->R, j->A,
                                           (uint32_t *)j->atoms, j->ctr, j->s));
        HIP_TRY(launch_trace_fp(j->letters_d, j->offsets_d, T, j->tfp, j->s));
    }
    const uint64_t *tf = (const uint64_t *)(img + o_tfp);
    HIP_TRY(hipMemcpyAsync((void *)tf, j->tfp, (uint64_t)T * 8, hipMemcpyDeviceToHost, j->s));
    Counters hc;
    if (int e = sync_read_counters(j, &hc)) return e;     // also waits for the fingerprints
    collect_times(j);
    if (j->A < 32 && (hc.letter_or >> j->A)) return LTL_E_INVAL;      // a letter names a missing proposition

    // P and N must be disjoint (Sec. 2): equal fingerprints are compared exactly (the
    // positives' fingerprints sorted, each negative's looked up by binary search)
    std::vector<std::pair<uint64_t, uint32_t>> pos(j->npos);
    for (uint32_t t = 0; t < j->npos; ++t) pos[t] = {tf[t], t};
    std::sort(pos.begin(), pos.end());
    for (uint32_t t = j->npos; t < T; ++t) {
        auto lo = std::lower_bound(pos.begin(), pos.end(), std::make_pair(tf[t], 0u));
        for (auto it = lo; it != pos.end() && it->first == tf[t]; ++it) {
            const uint32_t p = it->second;
            const uint64_t lp = j->off[p + 1] - j->off[p], ln = j->off[t + 1] - j->off[t];
            if (lp != ln) continue;
            std::vector<uint32_t> a(lp), b(ln);
            if (spec->flags & LTL_SPEC_DEVICE) {
                HIP_TRY(hipMemcpy(a.data(), spec->letters + j->off[p], lp * 4, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(b.data(), spec->letters + j->off[t], ln * 4, hipMemcpyDeviceToHost));
            } else {
                memcpy(a.data(), spec->letters + j->off[p], lp * 4);
                memcpy(b.data(), spec->letters + j->off[t], ln * 4);
            }
            if (a == b) return LTL_E_INCONSISTENT;
        }
    }
    j->L.assign((size_t)j->bound + 1, LevelInfo());
    return LTL_OK;
}

extern "C" int ltl_job_create(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
                              ltl_job **out) {
    if (!ctx || !spec || !ops || !out) return LTL_E_INVAL;
    if (ctx->busy) return LTL_E_STATE;
    if (spec->num_props < 1 || spec->num_props > 32) return LTL_E_INVAL;
    const uint64_t T = (uint64_t)spec->num_pos + spec->num_neg;
    if (T < 1 || T > 0x7FFFFFFFull || !spec->letters || !spec->offsets) return LTL_E_INVAL;
    if (cost_bound < 1 || cost_bound >= LTL_MAX_LEVELS) return LTL_E_INVAL;
    if (!(ops->op_mask & 1u) || (ops->op_mask & ~(0xFFu | LTL_OPS_NNF))) return LTL_E_INVAL;
    for (int k = 0; k < 8; ++k)
        if ((ops->op_mask >> k) & 1u)
            if (ops->cost[k] < 1 || ops->cost[k] >= LTL_MAX_LEVELS) return LTL_E_INVAL;
    if (hipSetDevice(ctx->o.device) != hipSuccess) return LTL_E_DEVICE;
    ltl_job *j = new (std::nothrow) ltl_job;
    if (!j) return LTL_E_INVAL;
    j->ctx = ctx;
    j->A = spec->num_props;
    j->T = (uint32_t)T;
    j->npos = spec->num_pos;
    j->nneg = spec->num_neg;
    j->ops = *ops;
    j->bound = cost_bound;
    int st = job_setup(j, spec);
    if (st != LTL_OK) {
        for (auto &t : j->pending) { (void)hipEventDestroy(t.e0); (void)hipEventDestroy(t.e1); }
        for (auto e : j->event_pool) (void)hipEventDestroy(e);
        delete j;
        return st;
    }
    ctx->busy = true;
    *out = j;
    return LTL_OK;
}

extern "C" void ltl_job_destroy(ltl_job *j) {
    if (!j) return;
    if (j->ctx && j->table_consistent && j->tkey &&
        launch_clear_slots(j->entry_slot, (uint32_t)j->total_entries, j->tkey, j->tval, j->s) == hipSuccess)
        j->ctx->table_clean_log2 = j->slots_log2;
    if (j->s) (void)hipStreamSynchronize(j->s); else (void)hipDeviceSynchronize();
    if (j->ctx) {      // events go back to the context for its next job
        for (auto &t : j->pending) { j->ctx->events.push_back(t.e0); j->ctx->events.push_back(t.e1); }
        for (auto e : j->event_pool) j->ctx->events.push_back(e);
    }
    if (j->ctx) j->ctx->busy = false;
    delete j;
}

// ---------------------------------------------------------------------------
// Levels
// ---------------------------------------------------------------------------
static void add_block(LevelInfo &lv, int op, int la, int lb, const ltl_job *j, bool tri, uint32_t &cand,
                      uint32_t &tile) {
    Block b{};
    b.op = (uint32_t)op;
    b.tri = tri ? 1u : 0u;
    const uint64_t R = j->R;
    if (op == LTL_ATOM) {
        b.na = j->A;
        b.nb = 0;
        b.a_gid = 0;
        b.a_ptr = (uint64_t)(uintptr_t)j->atoms;
        b.ind = 0;
    } else {
        // children are stored entries, found through store[] (claim order within a level)
        const LevelInfo &A = j->L[la];
        b.na = A.n;
        b.a_gid = A.gid_base;
        b.ind = 1;
        if (lb >= 0) {
            const LevelInfo &B = j->L[lb];
            b.nb = B.n;
            b.b_gid = B.gid_base;
            b.ind |= 2;
        }
    }
    (void)R;
    uint64_t nc, nt;
    if (b.nb == 0) {
        nc = b.na;
        b.nti = (b.na + TILE - 1) / TILE;
        b.ntj = 1;
        nt = b.nti;
    } else if (!tri) {
        nc = (uint64_t)b.na * b.nb;
        b.nti = (b.na + TILE - 1) / TILE;
        b.ntj = (b.nb + TILE - 1) / TILE;
        nt = (uint64_t)b.nti * b.ntj;
    } else {
        nc = (uint64_t)b.na * (b.na - 1) / 2;
        b.nti = b.ntj = (b.na + TILE - 1) / TILE;
        nt = (uint64_t)b.nti * (b.nti + 1) / 2;
    }
    if (nc == 0) return;
    b.cand_base = cand;
    b.ncand = (uint32_t)std::min<uint64_t>(nc, 0xFFFFFFFFull);
    b.tile_base = tile;
    b.ntile = (uint32_t)std::min<uint64_t>(nt, 0xFFFFFFFFull);
    // overflow of the 31-bit candidate space is checked by the caller on the u64 totals
    cand = (uint32_t)std::min<uint64_t>((uint64_t)cand + nc, 0xFFFFFFFFull);
    tile = (uint32_t)std::min<uint64_t>((uint64_t)tile + nt, 0xFFFFFFFFull);
    lv.blocks.push_back(b);
    lv.a_level.push_back(la);
    lv.b_level.push_back(lb);
}

// Canonical block order of level c (Sec. 3 listing: ops F, U, G, X, And, Or, Not).
static uint64_t build_blocks(ltl_job *j, uint32_t c, LevelInfo &lv, uint64_t &ntiles) {
    lv.blocks.clear();
    lv.a_level.clear();
    lv.b_level.clear();
    uint32_t cand = 0, tile = 0;
    uint64_t total = 0, tiles = 0;
    auto has = [&](int x) { return x >= 1 && (uint32_t)x < c && j->L[x].evaluated && j->L[x].n > 0; };
    if (c == j->ops.cost[LTL_ATOM]) {
        add_block(lv, LTL_ATOM, -1, -1, j, false, cand, tile);
        total = j->A;
        tiles = (j->A + TILE - 1) / TILE;
    } else {
        for (int op : ORDER) {
            if (!((j->ops.op_mask >> op) & 1u)) continue;
            const int x = (int)c - (int)j->ops.cost[op];
            if (x < 1) continue;
            // negation normal form: negations of atoms only
            if (op == LTL_NOT && (j->ops.op_mask & LTL_OPS_NNF) && x != (int)j->ops.cost[LTL_ATOM]) continue;
            if (is_unary(op)) {
                if (!has(x)) continue;
                total += j->L[x].n;
                tiles += (j->L[x].n + TILE - 1) / TILE;
                add_block(lv, op, x, -1, j, false, cand, tile);
            } else if (op == LTL_U) {
                for (int a = 1; a < x; ++a) {
                    const int b = x - a;
                    if (!has(a) || !has(b)) continue;
                    total += (uint64_t)j->L[a].n * j->L[b].n;
                    tiles += (uint64_t)((j->L[a].n + TILE - 1) / TILE) * ((j->L[b].n + TILE - 1) / TILE);
                    add_block(lv, op, a, b, j, false, cand, tile);
                }
            } else {
                for (int a = 1; a <= x - a; ++a) {
                    const int b = x - a;
                    if (!has(a) || !has(b)) continue;
                    if (a < b) {
                        total += (uint64_t)j->L[a].n * j->L[b].n;
                        tiles += (uint64_t)((j->L[a].n + TILE - 1) / TILE) * ((j->L[b].n + TILE - 1) / TILE);
                        add_block(lv, op, a, b, j, false, cand, tile);
                    } else {
                        const uint64_t n = j->L[a].n;
                        if (n < 2) continue;
                        total += n * (n - 1) / 2;
                        const uint64_t nt = (n + TILE - 1) / TILE;
                        tiles += nt * (nt + 1) / 2;
                        add_block(lv, op, a, a, j, true, cand, tile);
                    }
                }
            }
        }
    }
    ntiles = tiles;
    return total;
}

template <typename T>
static int eval_level_t(ltl_job *j, uint32_t c, LevelInfo &lv) {
    uint64_t ntiles = 0;
    const uint64_t C = build_blocks(j, c, lv, ntiles);
    lv.cands = C;
    lv.gid_base = (uint32_t)j->total_entries;
    if (C == 0) {
        lv.n = 0;
        return LTL_OK;
    }
    if (C >= 0x7FFFFFFFull || lv.blocks.size() > (size_t)MAX_BLOCKS || ntiles >= 0xFFFFFFFFull) return LTL_E_OOM;
    const uint32_t nc = (uint32_t)C;
    const uint32_t nw = (nc + 31) / 32;
    const uint32_t nchunks = (nw + SCAN_CHUNK_WORDS - 1) / SCAN_CHUNK_WORDS;
    const uint64_t nslots = 1ull << j->slots_log2;
    const uint32_t new_cap = (uint32_t)std::min<uint64_t>(C, nslots);

    // per-level scratch at the top of the workspace
    uint64_t top = j->wsb;
    auto take_top = [&](uint64_t bytes) -> char * {
        if (bytes + 256 > top) return nullptr;
        top = (top - bytes) & ~255ull;
        return j->ws + top;
    };
    const uint64_t nwa = align_up(nw, 64);                 // words, so the bitmaps stay aligned
    const bool ruc = (j->ctx->o.flags & LTL_CTX_RUC) != 0;
    // the relaxed check writes its entries in a pass of its own, so the row-split kernels pay
    // only where a tile's rows are long (one wave per tile would walk many row blocks):
    // by default it keeps the whole-row kernels below RUC_SPLIT_MIN_BLOCKS row blocks
    const bool split = ntiles < (j->ctx->o.split_tiles ? (uint64_t)j->ctx->o.split_tiles : SPLIT_TILES) &&
                       (!ruc || j->ctx->o.split_tiles || j->NB >= RUC_SPLIT_MIN_BLOCKS);
    // batch lanes that take turns for whole-row levels: held until the level's work is done
    std::unique_lock<std::mutex> big_turn;
    if (!split && j->ctx->big_mu) big_turn = std::unique_lock<std::mutex>(*j->ctx->big_mu);
    // bitmap | coll_bits | fb_bits, cleared at once
    // bitmap | coll_bits | fb_bits | cand_viol | cand_fp (row-split levels whose tiles
    // span several workgroups); cleared at once
    uint64_t clear_bytes = nwa * 4 * 3;
    // (the relaxed check's second sums follow cand_fp)
    const uint64_t fp_words = split ? (uint64_t)nc * (ruc ? 2 : 1) : 0;
    uint32_t *bits3 = (uint32_t *)take_top(align_up(nwa * 4 * 4 + fp_words * 8, 256));
    uint32_t *cand_slot = (uint32_t *)take_top((uint64_t)nc * 4);
    uint32_t *wordpre = (uint32_t *)take_top((uint64_t)nw * 4);
    uint32_t *chunks = (uint32_t *)take_top((uint64_t)std::max<uint32_t>(nchunks, 1) * 4);
    uint32_t *new_slots = (uint32_t *)take_top((uint64_t)new_cap * 4);
    uint32_t *claimer = (uint32_t *)take_top((uint64_t)new_cap * 4);
    uint32_t *new_owner = (uint32_t *)take_top((uint64_t)new_cap * 4);
    // whole-row levels (and relaxed-check levels, whose write pass is always a pass of its
    // own): claim number per candidate, and the claims other candidates joined
    const bool write_pass = !split || ruc;
    uint32_t *cand_claim = write_pass ? (uint32_t *)take_top((uint64_t)nc * 4) : nullptr;
    uint32_t *has_member = write_pass ? (uint32_t *)take_top(align_up((uint64_t)new_cap * 4, 256)) : nullptr;
    T *stage = (T *)take_top((uint64_t)j->R * sizeof(T));
    unsigned long long *cand_key = ruc ? (unsigned long long *)take_top((uint64_t)nc * 16) : nullptr;
    const uint64_t arena_off = (uint64_t)(j->arena - j->ws);
    const uint64_t arena_used = j->total_entries * j->cm_bytes;
    if (!bits3 || !cand_slot || !wordpre || !chunks || !new_slots || !claimer || !new_owner || !stage ||
        (write_pass && (!cand_claim || !has_member)) || (ruc && !cand_key) ||
        arena_off + arena_used > top)
        return LTL_E_OOM;
    uint32_t *bitmap = bits3, *coll_bits = bits3 + nwa, *fb_bits = bits3 + 2 * nwa, *cand_viol = bits3 + 3 * nwa;
    unsigned long long *cand_fp = (unsigned long long *)(bits3 + 4 * nwa);
    const uint64_t arena_free = top - (arena_off + arena_used);
    const uint32_t arena_cap = (uint32_t)std::min<uint64_t>(
        {arena_free / j->cm_bytes, j->recipe_cap - j->total_entries, (uint64_t)new_cap});

    Counters *pin_ctr = (Counters *)j->ctx->pinned;
    Block *pin_blocks = (Block *)(j->ctx->pinned + 256);
    Block *pin_grouped = pin_blocks + lv.blocks.size();
    memcpy(pin_blocks, lv.blocks.data(), sizeof(Block) * lv.blocks.size());
    // the same blocks grouped by connective class, each class with its own tile numbering
    // U by the carry adder (one add, one xor and one bit-select per half-word, a scalar
    // prefix across the words of a trace): faster than the App. B doubling on every row
    // layout measured (2x on multi-word rows, where each doubling step moves words across
    // lanes; 5% on one-word rows); the doubling can be forced
    const uint32_t fl = j->ctx->o.flags;
    const bool ucarry = (fl & LTL_CTX_U_CARRY) != 0 || !(fl & LTL_CTX_U_DOUBLING);
    auto cls_of = [&](uint32_t op) {
        if (op == LTL_AND || op == LTL_OR) return 1;
        if (op == LTL_U) return ucarry ? 3 : 2;
        return 0;
    };
    std::vector<Block> &grouped = j->grouped;
    grouped.clear();
    uint32_t cls_first[5] = {0}, cls_tiles[4] = {0};
    // F, G, X and NOT over the same child level are evaluated as one fused block
    int fuse_idx[4] = {-1, -1, -1, -1};
    {
        const uint32_t fops[4] = {LTL_F, LTL_G, LTL_X, LTL_NOT};
        for (size_t bi = 0; bi < lv.blocks.size(); ++bi)
            for (int q = 0; q < 4; ++q)
                if (lv.blocks[bi].op == fops[q]) fuse_idx[q] = (int)bi;
        for (int q = 0; q < 4; ++q)
            if (fuse_idx[q] < 0 || lv.blocks[fuse_idx[q]].a_gid != lv.blocks[fuse_idx[0] < 0 ? 0 : fuse_idx[0]].a_gid ||
                lv.blocks[fuse_idx[q]].na != lv.blocks[fuse_idx[0] < 0 ? 0 : fuse_idx[0]].na)
                fuse_idx[0] = -1;
    }
    const bool fuse = fuse_idx[0] >= 0;
    for (int k = 0; k < 4; ++k) {
        cls_first[k] = (uint32_t)grouped.size();
        uint32_t tb = 0;
        for (size_t bi = 0; bi < lv.blocks.size(); ++bi) {
            const Block &b = lv.blocks[bi];
            if (cls_of(b.op) != k) continue;
            if (fuse && (int)bi == fuse_idx[1]) continue;      // folded into the fused block
            if (fuse && (int)bi == fuse_idx[2]) continue;
            if (fuse && (int)bi == fuse_idx[3]) continue;
            Block g = b;
            if (fuse && (int)bi == fuse_idx[0]) {
                g.op = OP_FUSED4;
                for (int q = 0; q < 4; ++q) g.fcb[q] = lv.blocks[fuse_idx[q]].cand_base;
            }
            g.tile_base = tb;
            tb += g.ntile;
            grouped.push_back(g);
        }
        cls_tiles[k] = tb;
    }
    cls_first[4] = (uint32_t)grouped.size();
    // whole-row binary classes with LTL_CTX_LDS_TILES stage their child operands in LDS:
    // groups of 2 x 2 tiles (8 x 8 pairs), numbered per class like the tiles
    const bool staged = !split && !ruc && (j->ctx->o.flags & LTL_CTX_LDS_TILES);
    uint32_t cls_groups[4] = {0, 0, 0, 0};
    if (staged) {
        for (int k = 1; k < 4; ++k) {
            uint32_t gb = 0;
            for (uint32_t q = cls_first[k]; q < cls_first[k + 1]; ++q) {
                Block &g = grouped[q];
                const uint32_t ngi = (g.nti + 1) / 2, ngj = (g.ntj + 1) / 2;
                g.st_base = gb;
                g.nst = g.tri ? ngi * (ngi + 1) / 2 : ngi * ngj;
                gb += g.nst;
            }
            cls_groups[k] = gb;
        }
    }
    {   // algorithmic bytes: every candidate's matrix written or compared once, each child
        // matrix read once per tile (tiles of TILE children a side; fused unary tiles read a
        // child once for its four connectives)
        uint64_t child_reads = 0;
        for (const Block &g : grouped) {
            if (g.nb == 0) {
                child_reads += g.na;
            } else if (!g.tri) {
                child_reads += (uint64_t)g.ntj * g.na + (uint64_t)g.nti * g.nb;
            } else {
                for (uint32_t it = 0; it < g.nti; ++it) {
                    const uint64_t rows = std::min<uint64_t>(TILE, g.na - (uint64_t)it * TILE);
                    child_reads += (uint64_t)(g.nti - it) * rows + (uint64_t)(it + 1) * rows;
                }
            }
        }
        lv.alg_bytes = (C + child_reads) * j->cm_bytes;   // new entries written: a stored level
    }
    memcpy(pin_grouped, grouped.data(), sizeof(Block) * grouped.size());
    // row-split levels evaluate (and verify) every class in one dispatch: one tile numbering over the grouped blocks
    const bool merged_eval = split;
    Block *pin_all = pin_grouped + grouped.size();
    uint32_t all_tiles = 0;
    if (merged_eval) {
        for (size_t k = 0; k < grouped.size(); ++k) {
            pin_all[k] = grouped[k];
            pin_all[k].tile_base = all_tiles;
            all_tiles += grouped[k].ntile;
        }
    }
    // row-split levels: workgroups per tile, enough for the wave target when rows are long
    uint32_t wg_split = 1;
    if (merged_eval) {
        const uint64_t need = std::max<uint64_t>(
            1, std::min<uint64_t>((j->NB + MIN_CHUNK - 1) / MIN_CHUNK, TARGET_WAVES / std::max(1u, all_tiles)));
        const uint32_t wgw = Launch<T>::waves_per_wg(j->mw);
        wg_split = (uint32_t)((need + wgw - 1) / wgw);
        if (wg_split > 1) clear_bytes = nwa * 4 * 4 + fp_words * 8;
    }
    *pin_ctr = Counters{};
    pin_ctr->first_sol = ~0ull;
    *(uint32_t *)(j->ctx->pinned + FULL_FLAG_OFF) = 0;     // uploaded with the counters
    Block *grouped_d = j->blocks_d + lv.blocks.size();
    Block *all_d = grouped_d + grouped.size();
    HIP_TRY(hipMemcpyAsync(j->ctr, j->ctx->pinned,
                           256 + sizeof(Block) * (lv.blocks.size() + grouped.size() * (merged_eval ? 2 : 1)),
                           hipMemcpyHostToDevice, j->s));
    HIP_TRY(launch_zero2(bits3, clear_bytes / 4, has_member, has_member ? (uint64_t)new_cap : 0, j->s));

    LevelArgs<T> A{};
    A.rows = make_rows<T>(j);
    A.blocks = j->blocks_d;
    A.nblocks = (uint32_t)lv.blocks.size();
    A.tkey = j->tkey;
    A.tval = j->tval;
    A.slot_mask = (uint32_t)(nslots - 1);
    const uint32_t fb = j->ctx->o.fp_bits;
    A.fp_mask = (fb == 0 || fb >= 64) ? ~0ull : ((1ull << fb) - 1ull);
    A.ctr = j->ctr;
    A.full = (uint32_t *)((char *)j->ctr + FULL_FLAG_OFF);
    {   // the evaluation stops once the claims pass abort_cap: the arena's capacity, or for a
        // batch lane of a shared budget what would not fit the whole pool either (so that a
        // level that fits the pool but not the region is counted in full, and its re-run
        // sized from the count)
        uint64_t cap = arena_cap;
        if (j->ctx->pool_total) {
            const uint64_t fit = j->ctx->pool_total / j->cm_bytes;
            cap = std::max<uint64_t>(cap, fit > j->total_entries ? fit - j->total_entries : 0);
        }
        A.abort_cap = (uint32_t)std::min<uint64_t>(cap, new_cap);
    }
    A.cand_slot = cand_slot;
    A.new_slots = new_slots;
    A.claimer = claimer;
    A.new_owner = new_owner;
    A.new_cap = new_cap;
    A.bitmap = bitmap;
    A.wordpre = wordpre;
    A.coll_bits = coll_bits;
    A.fb_bits = fb_bits;
    A.arena = (T *)j->arena;
    A.level_base = lv.gid_base;
    A.recipe = j->recipe;
    A.store = j->store;
    // row-split levels write the claimers' matrices in the evaluation dispatch (each wave its
    // rows); whole-row levels in a write pass after the compaction, which keeps only what the
    // verification reads when the level will not be stored
    A.cw = split ? 1u : 0u;
    A.cand_claim = cand_claim;
    A.has_member = has_member;
    A.bound_level = (c == j->bound) ? 1u : 0u;
    A.verify_rep = 0;
    A.stage = stage;
    A.arena_cap = arena_cap;
    A.ucarry = ucarry ? 1 : 0;
    A.wg_split = wg_split;
    A.cand_fp = cand_fp;
    A.cand_viol = cand_viol;
    A.ruc_meta = j->ruc_meta;
    A.cand_key = cand_key;
    A.entry_key = j->entry_key;
    A.ruc_pack = j->ruc_pack ? 1u : 0u;
    A.ruc_bits = j->ctx->o.ruc_key_bits;
    A.ruc_fpb_off = nc;
    {   // materialize work items: entries x row chunks (sized on the candidate count, an upper bound)
        const uint64_t per = std::max<uint64_t>(
            1, std::min<uint64_t>((j->NB + MIN_CHUNK - 1) / MIN_CHUNK, TARGET_WAVES / std::max<uint64_t>(1, new_cap)));
        A.mat_chunk = (uint32_t)((j->NB + per - 1) / per);
    }
    auto launch_level = [&](bool verify, bool write = false) -> hipError_t {
        if (merged_eval && !write) {
            if (!verify) {
                const uint64_t items = (uint64_t)all_tiles * wg_split;
                HIP_TRY_E(Launch<T>::level_wg(A, j->mw, all_d, (uint32_t)grouped.size(), all_tiles,
                                              (uint32_t)std::min<uint64_t>(items, MAX_GRID), j->s, ruc));
                if (wg_split > 1) return ruc ? Launch<T>::ruc_finish(A, nc, j->s) : Launch<T>::probe(A, nc, j->s);
                return hipSuccess;
            }
            const uint64_t per = std::max<uint64_t>(
                1, std::min<uint64_t>((j->NB + MIN_CHUNK - 1) / MIN_CHUNK, TARGET_WAVES / std::max(1u, all_tiles)));
            const uint32_t chunk = (uint32_t)((j->NB + per - 1) / per);
            const uint64_t nchunk = (j->NB + chunk - 1) / chunk;
            const uint32_t grid = (uint32_t)std::min<uint64_t>(((uint64_t)all_tiles * nchunk + 3) / 4, MAX_GRID);
            return Launch<T>::verify_all(A, j->mw, all_d, (uint32_t)grouped.size(), all_tiles, chunk, grid, j->s);
        }
        // whole-row tiles, one dispatch per connective class; the U class (VALU-bound)
        // on the context's second stream when other classes (HBM-bound) run beside it
        const int ucls = ucarry ? 3 : 2;
        const bool fork = j->ctx->aux && cls_tiles[ucls] && (cls_tiles[0] || cls_tiles[1]);
        if (fork) {
            HIP_TRY_E(hipEventRecord(j->ctx->ev_fork, j->s));
            HIP_TRY_E(hipStreamWaitEvent(j->ctx->aux, j->ctx->ev_fork, 0));
        }
        const int order[4] = {ucls, 0, 1, ucls == 2 ? 3 : 2};
        for (int q = 0; q < 4; ++q) {
            const int k = order[q];
            if (!cls_tiles[k]) continue;
            // the evaluation needs a tile's whole rows (its fingerprints); verification and
            // the write pass treat row blocks independently, so they take chunks of a tile's
            // rows, enough for PASS_WAVES waves (one wave per tile leaves most SIMDs with one
            // or two waves on long rows, too few to keep the owners' loads in flight)
            // binary classes staged in LDS: work items are groups of 4 tiles, one workgroup each
            const bool stg = staged && k != 0;
            const uint64_t units = stg ? (uint64_t)cls_groups[k] : (uint64_t)cls_tiles[k];
            const uint64_t waves_per_unit = stg ? 4 : 1;
            uint32_t chunk = j->NB;
            if (verify || write) {
                const uint64_t per = std::max<uint64_t>(
                    1, std::min<uint64_t>(j->NB / PASS_MIN_CHUNK, PASS_WAVES / (units * waves_per_unit)));
                chunk = (uint32_t)((j->NB + per - 1) / per);
            }
            const uint64_t items = units * ((j->NB + chunk - 1) / chunk);
            const uint32_t grid = (uint32_t)std::min<uint64_t>(stg ? items : (items + 3) / 4, MAX_GRID);
            // the evaluation's and/or class follows U on the second stream (the unary class,
            // the longest, keeps the first to itself); verification and write pass keep U alone
            const bool on_aux = fork && (k == ucls || (LTL_ANDOR_EVAL_AUX && k == 1 && !verify && !write));
            hipStream_t st = on_aux ? j->ctx->aux : j->s;
            const Block *cb = grouped_d + cls_first[k];
            const uint32_t nb = cls_first[k + 1] - cls_first[k];
            hipError_t e;
            if (ruc && !verify && !write)
                e = Launch<T>::level_ruc(A, j->mw, k, cb, nb, cls_tiles[k], grid, st);
            else if (stg)
                e = Launch<T>::level_staged(A, j->mw, write ? 2 : (verify ? 1 : 0), k, cb, nb, cls_groups[k], chunk,
                                            grid, st);
            else if (write)
                e = Launch<T>::write_pass(A, j->mw, k, cb, nb, cls_tiles[k], chunk, grid, st);
            else
                e = Launch<T>::level(A, j->mw, verify, k, cb, nb, cls_tiles[k], chunk, grid, st);
            if (e != hipSuccess) return e;
        }
        if (fork) {
            HIP_TRY_E(hipEventRecord(j->ctx->ev_join, j->ctx->aux));
            HIP_TRY_E(hipStreamWaitEvent(j->s, j->ctx->ev_join, 0));
        }
        return hipSuccess;
    };
    // kernels after the evaluation read the level's new-entry count on the device
    const uint32_t grid_new = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((new_cap + 255) / 256, 2048));
    const uint64_t mat_items = (uint64_t)new_cap * ((j->NB + A.mat_chunk - 1) / A.mat_chunk);
    const uint32_t grid_mat = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((mat_items + 3) / 4, MAX_GRID));
    j->table_consistent = false;
    uint32_t ncls = 0;
    for (int k = 0; k < 4; ++k) ncls += cls_tiles[k] ? 1u : 0u;
    LevelSpan span(j);
    {
        Timer tm(j, LTL_K_EVAL, merged_eval ? (wg_split > 1 ? 2u : 1u) : ncls);
        HIP_TRY(launch_level(false));
    }
    if (ruc) {              // relaxed check: the claims of new keys
        Timer tm(j, LTL_K_COMPACT);
        HIP_TRY(Launch<T>::ruc_claim(A, nc, j->s));
    }
    if (wg_split > 1 && !ruc) {     // claimers' matrices (their rows were spread over workgroups)
        Timer tm(j, LTL_K_MATERIALIZE);
        HIP_TRY(Launch<T>::materialize(A, j->mw, 0u, grid_mat, j->s));
    }
    {
        Timer tm(j, LTL_K_COMPACT, nw <= SMALL_COMPACT_WORDS ? 1u : 5u);
        if (nw <= SMALL_COMPACT_WORDS) {
            HIP_TRY(launch_compact_small(new_slots, j->ctr, arena_cap, j->tval, bitmap, nw, wordpre, j->recipe,
                                         lv.gid_base, j->entry_slot, new_owner, j->store, j->s));
        } else {
            HIP_TRY(launch_mark(new_slots, j->ctr, arena_cap, j->tval, bitmap, grid_new, j->s));
            HIP_TRY(launch_scan(bitmap, nw, chunks, wordpre, j->s));
            HIP_TRY(launch_scatter(new_slots, j->ctr, arena_cap, j->tval, bitmap, wordpre, j->recipe, lv.gid_base,
                                   j->entry_slot, new_owner, j->store, false, grid_new, j->s));
        }
    }
    if (ruc) {
        // relaxed check: nothing is compared.  If the level will be stored (decided on the
        // device), each entry gets its representative's key and, in the write pass, its
        // representative's matrix (a level that is not stored writes nothing: no member
        // flags are set)
        Timer tm(j, LTL_K_MATERIALIZE, ncls + 1);
        HIP_TRY(Launch<T>::ruc_entry_keys(A, j->s));
        HIP_TRY(launch_level(false, true));
    } else if (write_pass) {
        Timer tm(j, LTL_K_MATERIALIZE, ncls + 1);
        HIP_TRY(Launch<T>::mark_members(A, nc, j->s));
        HIP_TRY(launch_level(false, true));
    }
    if (!ruc) {
        Timer tm(j, LTL_K_VERIFY, merged_eval ? 1u : ncls);
        HIP_TRY(launch_level(true));
    }
    span.end();
    Counters hc;
    if (int e = sync_read_counters(j, &hc)) return e;
    if (hc.overflow || hc.n_new > arena_cap) {
        j->oom_kind = hc.overflow ? 1 : 2;
        j->oom_new = hc.n_new;
        return LTL_E_OOM;
    }
    lv.first = (hc.first_sol == ~0ull) ? LTL_NO_SOLUTION : (uint64_t)hc.first_sol;
    lv.stored = lv.first == LTL_NO_SOLUTION && c < j->bound;
    uint32_t n_new = hc.n_new;
    // a level that is not stored need not write its new entries (check-only)
    if (!lv.stored) lv.alg_bytes -= (uint64_t)std::min<uint64_t>(n_new, C) * j->cm_bytes;
    // relaxed check: the candidates that joined a cached language are not compared
    if (ruc) lv.alg_bytes -= (C - std::min<uint64_t>(n_new, C)) * j->cm_bytes;
    lv.colliders = 0;
    if (hc.n_coll) {
        // A fingerprint group held two different matrices.  Exact re-check: every
        // entry gets the matrix of its representative (the canonical-first member),
        // every other candidate is compared with it, and the ones that differ go to
        // the sequential fallback in canonical order.
        HIP_TRY(launch_zero2(coll_bits, nwa, &j->ctr->n_coll, 1, j->s));
        A.verify_rep = 1;
        {
            Timer tm(j, LTL_K_MATERIALIZE);
            HIP_TRY(Launch<T>::materialize(A, j->mw, 1u, grid_mat, j->s));
        }
        {
            Timer tm(j, LTL_K_VERIFY, merged_eval ? 1u : ncls);
            HIP_TRY(launch_level(true));
        }
        if (int e = sync_read_counters(j, &hc)) return e;
        lv.colliders = hc.n_coll;
    }
    if (hc.n_coll) {
        {
            Timer tm(j, LTL_K_FALLBACK);
            HIP_TRY(Launch<T>::fallback(A, j->mw, nw, nc, j->s));
        }
        if (int e = sync_read_counters(j, &hc)) return e;
        if (hc.overflow || hc.n_new > arena_cap) return LTL_E_OOM;
        n_new = hc.n_new;
        {
            Timer tm(j, LTL_K_COMPACT, 5);
            HIP_TRY(launch_or_bits(bitmap, fb_bits, nw, j->s));
            HIP_TRY(launch_scan(bitmap, nw, chunks, wordpre, j->s));
            HIP_TRY(launch_scatter(new_slots, j->ctr, arena_cap, j->tval, bitmap, wordpre, j->recipe, lv.gid_base,
                                   j->entry_slot, new_owner, j->store, true, grid_new, j->s));
        }
        {
            Timer tm(j, LTL_K_MATERIALIZE);
            HIP_TRY(Launch<T>::materialize(A, j->mw, 1u, grid_mat, j->s));
        }
    }
    j->table_consistent = true;
    lv.n = n_new;
    j->total_entries += n_new;
    return LTL_OK;
}

extern "C" int ltl_eval_level(ltl_job *j, uint32_t c, ltl_level_stats *stats) {
    if (!j) return LTL_E_INVAL;
    if (!j->searching || c != j->levels_done + 1 || c > j->bound) return LTL_E_STATE;
    if (hipSetDevice(j->ctx->o.device) != hipSuccess) return LTL_E_DEVICE;
    LevelInfo &lv = j->L[c];
    lv = LevelInfo();
    const double before = [&] { double s = j->span_ms; for (double v : j->kernel_ms) s += v; return s; }();
    int st = LTL_OK;
    if (c >= j->ops.cost[LTL_ATOM]) st = (j->wbits == 64) ? eval_level_t<uint64_t>(j, c, lv) : eval_level_t<uint32_t>(j, c, lv);
    else lv.gid_base = (uint32_t)j->total_entries;
    collect_times(j);
    double after = j->span_ms;
    for (double v : j->kernel_ms) after += v;
    lv.ms = after - before;
    if (st != LTL_OK) {
        j->status = st;
        j->searching = false;
        return st;
    }
    lv.evaluated = true;
    j->levels_done = c;
    j->colliders += lv.colliders;
    if (stats) {
        stats->cost = c;
        stats->stored = lv.stored ? 1u : 0u;
        stats->candidates = lv.cands;
        stats->new_entries = lv.n;
        stats->first_solution = lv.first;
        stats->colliders = lv.colliders;
        stats->kernel_ms = lv.ms;
        stats->alg_bytes = lv.alg_bytes;
    }
    if (lv.first != LTL_NO_SOLUTION) {
        j->status = LTL_OK;
        j->searching = false;
        j->sol_level = c;
        j->sol_index = lv.first;
        return LTL_OK;
    }
    if (c == j->bound) {
        j->status = LTL_NOT_FOUND;
        j->searching = false;
        return LTL_OK;
    }
    lv.stored = true;
    j->stored_entries += lv.n;
    if (j->stored_entries > j->max_entries) {
        j->status = LTL_E_OOM;
        j->searching = false;
        j->oom_kind = 3;
        return LTL_E_OOM;
    }
    return LTL_OK;
}

// ---------------------------------------------------------------------------
// Formula reconstruction from recipes (host decode of the canonical order)
// ---------------------------------------------------------------------------
static void host_cand_decode(const Block &b, uint32_t l, uint32_t &i, uint32_t &j) {
    if (b.nb == 0) { i = l; j = 0; return; }
    if (!b.tri) { i = l / b.nb; j = l % b.nb; return; }
    const uint64_t n = b.na;
    auto Tt = [&](uint64_t ii) -> uint64_t { return ii * n - ii * (ii + 1) / 2; };
    uint64_t ii = 0;
    uint64_t lo = 0, hi = n - 1;           // largest ii with Tt(ii) <= l
    while (lo < hi) {
        uint64_t mid = (lo + hi + 1) / 2;
        if (Tt(mid) <= l) lo = mid; else hi = mid - 1;
    }
    ii = lo;
    i = (uint32_t)ii;
    j = (uint32_t)(l - Tt(ii) + ii + 1);
}

static int emit_candidate(ltl_job *j, uint32_t level, uint32_t x, ltl_node *buf, uint32_t cap, uint32_t &n,
                          uint32_t &root);

// Host copy of the recipes of entries [0, upto), extended by one bulk copy.
static int host_recipes(ltl_job *j, uint64_t upto) {
    const uint64_t have = j->recipe_h.size();
    if (upto <= have) return LTL_OK;
    j->recipe_h.resize(upto);
    HIP_TRY(hipMemcpyAsync(j->recipe_h.data() + have, j->recipe + have, (upto - have) * 4, hipMemcpyDeviceToHost,
                           j->s));
    HIP_TRY(hipStreamSynchronize(j->s));
    return LTL_OK;
}

static int emit_entry(ltl_job *j, uint32_t level, uint32_t e, ltl_node *buf, uint32_t cap, uint32_t &n,
                      uint32_t &root) {
    const LevelInfo &lv = j->L[level];
    if (e >= lv.n) return LTL_E_INVAL;
    if (int st = host_recipes(j, (uint64_t)lv.gid_base + lv.n)) return st;
    return emit_candidate(j, level, j->recipe_h[lv.gid_base + e], buf, cap, n, root);
}

static int emit_candidate(ltl_job *j, uint32_t level, uint32_t x, ltl_node *buf, uint32_t cap, uint32_t &n,
                          uint32_t &root) {
    const LevelInfo &lv = j->L[level];
    size_t bi = 0;
    for (size_t k = 0; k < lv.blocks.size(); ++k)
        if (lv.blocks[k].cand_base <= x) bi = k;
    const Block &b = lv.blocks[bi];
    if (x - b.cand_base >= b.ncand) return LTL_E_INVAL;
    uint32_t i, jj;
    host_cand_decode(b, x - b.cand_base, i, jj);
    if (b.op == LTL_ATOM) {
        if (n >= cap) return LTL_E_INVAL;
        buf[n] = ltl_node{LTL_ATOM, i, 0};
        root = n++;
        return LTL_OK;
    }
    uint32_t ra = 0, rb = 0;
    int st = emit_entry(j, (uint32_t)lv.a_level[bi], i, buf, cap, n, ra);
    if (st) return st;
    if (b.nb) {
        st = emit_entry(j, (uint32_t)lv.b_level[bi], jj, buf, cap, n, rb);
        if (st) return st;
    }
    if (n >= cap) return LTL_E_INVAL;
    buf[n] = ltl_node{b.op, ra, b.nb ? rb : 0u};
    root = n++;
    return LTL_OK;
}

// The overfitting formula (Sec. 2), built position by position from the end of each
// trace of P; nodes are counted even when buf is full, so the caller learns the size.
extern "C" int ltl_overfit(const ltl_spec *spec, const ltl_opset *ops, ltl_node *buf, uint32_t cap,
                           uint32_t *num_nodes, uint64_t *cost) {
    if (!spec || !ops || !num_nodes || !cost || (!buf && cap)) return LTL_E_INVAL;
    if (spec->flags & LTL_SPEC_DEVICE) return LTL_E_INVAL;
    if (!spec->letters || !spec->offsets || spec->num_pos < 1) return LTL_E_INVAL;
    if (spec->num_props < 1 || spec->num_props > 32) return LTL_E_INVAL;
    const uint32_t need_ops = (1u << LTL_ATOM) | (1u << LTL_NOT) | (1u << LTL_AND) | (1u << LTL_OR) | (1u << LTL_X);
    if ((ops->op_mask & need_ops) != need_ops || (ops->op_mask & LTL_OPS_NNF)) return LTL_E_INVAL;
    if (ops->op_mask & ~(0xFFu | LTL_OPS_NNF)) return LTL_E_INVAL;
    for (int k = 0; k < 8; ++k)
        if (((ops->op_mask >> k) & 1u) && ops->cost[k] < 1) return LTL_E_INVAL;
    const uint32_t A = spec->num_props;
    uint32_t n = 0;
    uint64_t c = 0;
    auto node = [&](uint32_t op, uint32_t a, uint32_t b) -> uint32_t {
        if (n < cap) buf[n] = ltl_node{op, a, b};
        c += ops->cost[op];
        return n++;
    };
    uint32_t disj = 0;
    for (uint32_t t = 0; t < spec->num_pos; ++t) {
        const uint64_t o0 = spec->offsets[t], o1 = spec->offsets[t + 1];
        if (o1 <= o0) return LTL_E_INVAL;                    // empty trace
        // not X true: the last position
        const uint32_t p0 = node(LTL_ATOM, 0, 0);
        const uint32_t np0 = node(LTL_NOT, node(LTL_ATOM, 0, 0), 0);
        const uint32_t tru = node(LTL_OR, p0, np0);
        const uint32_t xt = node(LTL_X, tru, 0);
        uint32_t rest = node(LTL_NOT, xt, 0);
        for (uint64_t q = o1; q-- > o0;) {
            const uint32_t letter = spec->letters[q];
            if (A < 32 && (letter >> A)) return LTL_E_INVAL;
            uint32_t conj = 0;
            for (uint32_t k = 0; k < A; ++k) {
                uint32_t lit = node(LTL_ATOM, k, 0);
                if (!((letter >> k) & 1u)) lit = node(LTL_NOT, lit, 0);
                conj = k ? node(LTL_AND, conj, lit) : lit;
            }
            rest = node(LTL_AND, conj, rest);
            if (q > o0) rest = node(LTL_X, rest, 0);
        }
        disj = t ? node(LTL_OR, disj, rest) : rest;
    }
    *num_nodes = n;
    *cost = c;
    return n <= cap ? LTL_OK : LTL_E_OOM;
}

extern "C" int ltl_job_formula(ltl_job *j, uint32_t cost, uint64_t entry, ltl_node *buf, uint32_t cap,
                               uint32_t *num_nodes) {
    if (!j || !buf || !num_nodes || cost > j->levels_done || cost >= j->L.size()) return LTL_E_INVAL;
    if (!j->L[cost].evaluated || entry >= j->L[cost].n) return LTL_E_INVAL;
    uint32_t n = 0, root = 0;
    int st = emit_entry(j, cost, (uint32_t)entry, buf, cap, n, root);
    if (st) return st;
    *num_nodes = n;
    return LTL_OK;
}

extern "C" int ltl_job_dump_cm(ltl_job *j, uint32_t cost, uint64_t entry, uint8_t *pos_bits, uint64_t cap) {
    if (!j || !pos_bits || cost > j->levels_done || cost >= j->L.size()) return LTL_E_INVAL;
    const LevelInfo &lv = j->L[cost];
    if (!lv.evaluated || entry >= lv.n || cap < j->TB) return LTL_E_INVAL;
    if (!lv.stored) return LTL_E_STATE;      // matrices of a level that is not stored may be partial
    std::vector<uint64_t> words(j->R);
    uint32_t pos = 0;
    HIP_TRY(hipMemcpy(&pos, j->store + lv.gid_base + entry, 4, hipMemcpyDeviceToHost));
    const char *src = j->arena + (uint64_t)pos * j->cm_bytes;
    if (j->wbits == 64) {
        HIP_TRY(hipMemcpy(words.data(), src, j->cm_bytes, hipMemcpyDeviceToHost));
    } else {
        std::vector<uint32_t> w32(j->R);
        HIP_TRY(hipMemcpy(w32.data(), src, j->cm_bytes, hipMemcpyDeviceToHost));
        for (uint32_t r = 0; r < j->R; ++r) words[r] = w32[r];
    }
    const uint64_t W = j->wbits;
    uint64_t q = 0;
    for (uint32_t t = 0; t < j->T; ++t) {
        const uint64_t len = j->off[t + 1] - j->off[t];
        for (uint64_t i = 0; i < len; ++i) {
            const uint64_t w = words[j->row0[t] + i / W];
            pos_bits[q++] = (uint8_t)((w >> (W - 1 - (i % W))) & 1ull);
        }
    }
    return LTL_OK;
}

extern "C" int ltl_job_get_info(ltl_job *j, ltl_job_info *out) {
    if (!j || !out) return LTL_E_INVAL;
    out->word_bits = j->wbits;
    out->rows = j->R;
    out->cm_bytes = j->cm_bytes;
    out->total_positions = j->TB;
    out->hash_slots_log2 = j->slots_log2;
    out->doubling_steps = j->ksteps;
    out->arena_bytes = j->arena_region;
    out->max_entries = j->max_entries;
    return LTL_OK;
}

extern "C" int ltl_job_result(ltl_job *j, ltl_result *out) {
    if (!j || !out) return LTL_E_INVAL;
    memset(out, 0, sizeof(*out));
    out->status = j->searching ? LTL_NOT_FOUND : j->status;
    out->levels_done = j->levels_done;
    out->solution_index = LTL_NO_SOLUTION;
    for (uint32_t c = 1; c <= j->levels_done && c < LTL_MAX_LEVELS; ++c) {
        out->level_new[c] = j->L[c].n;
        out->level_candidates[c] = j->L[c].cands;
        out->level_ms[c] = j->L[c].ms;
        out->level_bytes[c] = j->L[c].alg_bytes;
    }
    out->colliders = j->colliders;
    for (int k = 0; k < LTL_K_KINDS; ++k) {
        out->kernel_ms[k] = j->kernel_ms[k];
        out->kernel_launches[k] = j->kernel_launches[k];
    }
    if (!j->searching && j->status == LTL_OK) {
        out->cost = j->sol_level;
        out->solution_index = j->sol_index;
        uint32_t n = 0, root = 0;
        int st = emit_candidate(j, j->sol_level, (uint32_t)j->sol_index, out->nodes, LTL_MAX_NODES, n, root);
        if (st) return st;
        out->num_nodes = n;
    }
    return out->status;
}

// The whole learner on one job; *oom_kind / *oom_new tell why it ran out of memory
// (see ltl_job::oom_kind; 1 when the job could not even be laid out).
static int learn_job(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
                     ltl_result *out, int *oom_kind, uint64_t *oom_new) {
    if (!out) return LTL_E_INVAL;
    memset(out, 0, sizeof(*out));
    out->solution_index = LTL_NO_SOLUTION;
    *oom_kind = 0;
    *oom_new = 0;
    ltl_job *j = nullptr;
    int st = ltl_job_create(ctx, spec, ops, cost_bound, &j);
    if (st != LTL_OK) {
        out->status = st;
        if (st == LTL_E_OOM) *oom_kind = 1;
        return st;
    }
    for (uint32_t c = 1; c <= cost_bound; ++c) {
        st = ltl_eval_level(j, c, nullptr);
        if (st != LTL_OK || !j->searching) break;
    }
    st = ltl_job_result(j, out);
    if (st == LTL_E_OOM) {
        *oom_kind = j->oom_kind ? j->oom_kind : 1;
        *oom_new = j->oom_new;
    }
    ltl_job_destroy(j);
    return st;
}

extern "C" int ltl_learn(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
                         ltl_result *out) {
    int kind = 0;
    uint64_t nn = 0;
    return learn_job(ctx, spec, ops, cost_bound, out, &kind, &nn);
}

// ---------------------------------------------------------------------------
// Autotuner: tile shape and level schedule of a workload, by timing whole jobs
// ---------------------------------------------------------------------------
extern "C" int ltl_autotune(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
                            ltl_tuning *out) {
    if (!ctx || !spec || !ops || !out) return LTL_E_INVAL;
    if (ctx->busy) return LTL_E_STATE;
    memset(out, 0, sizeof(*out));
    // candidate configurations: binary tiles in registers (4 x 4) or staged in LDS (8 x 8),
    // and the level size (in tiles) from which levels run the whole-row kernels
    static const uint32_t kFlags[LTL_TUNE_CONFIGS] = {0, LTL_CTX_LDS_TILES, 0, 0, LTL_CTX_LDS_TILES};
    static const uint32_t kSplit[LTL_TUNE_CONFIGS] = {8192, 8192, 2048, 32768, 32768};
    const ltl_ctx_opts saved = ctx->o;
    const uint32_t keep = LTL_CTX_U_CARRY | LTL_CTX_U_DOUBLING | LTL_CTX_RUC | LTL_CTX_RUC_FKP;
    ltl_result ref{}, r{};
    int status = LTL_OK;
    // an untimed warm-up run, then TUNE_ROUNDS rounds over the configurations (the
    // fastest run of each counts: short jobs vary by more than the configurations do)
    constexpr int TUNE_ROUNDS = 3;
    for (int k = -1; k < TUNE_ROUNDS * LTL_TUNE_CONFIGS && status == LTL_OK; ++k) {
        const int q = k < 0 ? 0 : k % LTL_TUNE_CONFIGS;
        ctx->o.flags = (saved.flags & keep) | kFlags[q];
        ctx->o.split_tiles = kSplit[q];
        const auto t0 = std::chrono::steady_clock::now();
        const int st = ltl_learn(ctx, spec, ops, cost_bound, &r);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (st < 0 && st != LTL_E_OOM) { status = st; break; }
        if (k < 0) { ref = r; continue; }
        // every configuration must give the same result
        bool same = r.status == ref.status && r.cost == ref.cost && r.levels_done == ref.levels_done &&
                    r.solution_index == ref.solution_index && r.num_nodes == ref.num_nodes;
        for (uint32_t c = 0; same && c <= r.levels_done && c < LTL_MAX_LEVELS; ++c)
            same = r.level_new[c] == ref.level_new[c] && r.level_candidates[c] == ref.level_candidates[c];
        if (!same) { status = LTL_E_STATE; break; }
        if (k < LTL_TUNE_CONFIGS) {
            out->ms[q] = ms;
            out->flags[q] = kFlags[q];
            out->split_tiles[q] = kSplit[q];
            ++out->tried;
        } else {
            out->ms[q] = std::min(out->ms[q], ms);
        }
    }
    for (uint32_t q = 0; q < out->tried; ++q)
        if (out->ms[q] < out->ms[out->best]) out->best = q;
    ctx->o = saved;
    return status;
}

// ---------------------------------------------------------------------------
// Learning without allocation: the library's static device scratch as workspace
// ---------------------------------------------------------------------------
namespace ltl {
void *noalloc_scratch(int device, hipError_t *err);
std::mutex &noalloc_lock(int device);
}  // namespace ltl

extern "C" int ltl_learn_noalloc(int32_t device, void *stream, const ltl_spec *spec, const ltl_opset *ops,
                                 uint32_t cost_bound, ltl_result *out) {
    if (!out) return LTL_E_INVAL;
    memset(out, 0, sizeof(*out));
    out->solution_index = LTL_NO_SOLUTION;
    if (device < 0 || device >= 64) return out->status = LTL_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return out->status = LTL_E_DEVICE;
    std::lock_guard<std::mutex> turn(noalloc_lock(device));
    hipError_t err = hipSuccess;
    void *ws = noalloc_scratch(device, &err);
    if (!ws) return out->status = LTL_E_DEVICE;
    ltl_ctx c;
    c.o = ltl_ctx_opts{};
    c.o.device = device;
    c.o.workspace = ws;
    c.o.workspace_bytes = LTL_NOALLOC_SCRATCH_BYTES;
    c.o.stream = stream;
    c.o.hash_slots_log2 = LTL_NOALLOC_SLOTS_LOG2;
    c.s = (hipStream_t)stream;
    c.noalloc = true;
    c.heap_pinned.resize(PINNED_BYTES);
    c.pinned = c.heap_pinned.data();
    // table_clean_log2 = 0: the job initialises the hash table (the array holds the last
    // call's contents)
    const int st = ltl_learn(&c, spec, ops, cost_bound, out);
    if (c.s) (void)hipStreamSynchronize(c.s); else (void)hipDeviceSynchronize();
    return st;
}

// ---------------------------------------------------------------------------
// Formula evaluation: tr |= phi (Sec. 2) for every trace of a specification
// ---------------------------------------------------------------------------
template <typename T>
static int holds_t(ltl_job *j, const ltl_node *nodes, uint32_t n, uint8_t *out) {
    // node matrices in the arena (atoms are the packed atom matrices), then the answer bytes
    const uint64_t cmb = j->cm_bytes;
    const uint64_t need = (uint64_t)n * cmb + align_up(j->T, 256) + 256;
    if (need > j->arena_region) return LTL_E_OOM;
    std::vector<const T *> cm(n);
    Rows<T> rw = make_rows<T>(j);
    for (uint32_t k = 0; k < n; ++k) {
        const ltl_node &v = nodes[k];
        if (v.op == LTL_ATOM) {
            cm[k] = (const T *)j->atoms + (uint64_t)v.a * j->R;
            continue;
        }
        T *dst = (T *)(j->arena + (uint64_t)k * cmb);
        const bool bin = v.op == LTL_AND || v.op == LTL_OR || v.op == LTL_U;
        HIP_TRY(Launch<T>::formula_node(rw, j->mw, (int)v.op, cm[v.a], bin ? cm[v.b] : nullptr, dst, j->s));
        cm[k] = dst;
    }
    uint8_t *bits_d = (uint8_t *)(j->arena + align_up((uint64_t)n * cmb, 256));
    HIP_TRY(Launch<T>::first_bits(cm[n - 1], j->row_trace, j->row_word, j->R, bits_d, j->s));
    HIP_TRY(hipMemcpyAsync(out, bits_d, j->T, hipMemcpyDeviceToHost, j->s));
    HIP_TRY(hipStreamSynchronize(j->s));
    return LTL_OK;
}

extern "C" int ltl_holds(ltl_ctx *ctx, const ltl_spec *spec, const ltl_node *nodes, uint32_t num_nodes,
                         uint8_t *out) {
    if (!ctx || !spec || !nodes || !out || num_nodes < 1) return LTL_E_INVAL;
    if ((uint64_t)spec->num_pos + spec->num_neg > 0x7FFFFFFFull) return LTL_E_INVAL;
    for (uint32_t k = 0; k < num_nodes; ++k) {
        const ltl_node &v = nodes[k];
        if (v.op > LTL_U) return LTL_E_INVAL;
        if (v.op == LTL_ATOM) {
            if (v.a >= spec->num_props) return LTL_E_INVAL;
        } else {
            const bool bin = v.op == LTL_AND || v.op == LTL_OR || v.op == LTL_U;
            if (v.a >= k || (bin && v.b >= k)) return LTL_E_INVAL;
        }
    }
    // every trace in one class: the classes play no part here (and need not be disjoint)
    ltl_spec all = *spec;
    all.num_pos = spec->num_pos + spec->num_neg;
    all.num_neg = 0;
    ltl_opset ops{};
    ops.op_mask = 1u;
    ops.cost[LTL_ATOM] = 1;
    ltl_job *j = nullptr;
    int st = ltl_job_create(ctx, &all, &ops, 1, &j);
    if (st != LTL_OK) return st;
    st = (j->wbits == 64) ? holds_t<uint64_t>(j, nodes, num_nodes, out) : holds_t<uint32_t>(j, nodes, num_nodes, out);
    ltl_job_destroy(j);
    return st;
}

// ---------------------------------------------------------------------------
// Batched learning: lanes of (stream, workspace slice, context), jobs taken in order
// ---------------------------------------------------------------------------
// A batch executor: `lanes` contexts (stream, workspace slice, hash table) and
// lanes-1 worker threads that sleep between runs.  The calling thread works as
// lane 0 of each run.
// Language-cache footprint of a job: the fixed tables of its row layout, the bytes per
// matrix, and an estimate of the workspace region it needs.
struct Footprint {
    uint64_t fixed = 0;    // row tables, atom matrices, letters, counters
    uint64_t cmb = 0;      // bytes per characteristic matrix
    uint64_t request = 0;  // region to start with
};

struct ltl_batch {
    ltl_batch_opts o{};
    std::mutex big_mu;                     // LTL_BATCH_BIG_ALONE: turns for whole-row levels
    std::vector<hipStream_t> streams;
    std::vector<ltl_ctx *> ctxs;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_start, cv_done;
    std::atomic<uint64_t> generation{0};   // bumped once per run (under mu)
    std::atomic<uint32_t> lanes_busy{0};   // worker lanes still in the current run
    std::atomic<bool> quit{false};
    std::atomic<bool> running{false};
    // the current run
    const ltl_batch_job *jobs = nullptr;
    uint32_t njobs = 0;
    ltl_result *results = nullptr;
    double *job_ms = nullptr;
    const double *arrival_ms = nullptr;    // serving: job i may start arrival_ms[i] after t0
    std::atomic<uint32_t> next{0};
    std::chrono::steady_clock::time_point t0;
    // LTL_BATCH_SHARED_BUDGET: regions of the whole workspace, sized per job
    bool shared = false;
    uint64_t pool_base = 0, pool_bytes = 0;    // the regions' pool after the lanes' caches
    std::mutex pool_mu;
    std::condition_variable pool_cv;
    std::map<uint64_t, uint64_t> free_regions;    // offset -> size, coalesced
    uint64_t in_use = 0;
    std::deque<std::pair<uint32_t, uint64_t>> queue;   // (job, region bytes requested), arrival order
    uint32_t jobs_left = 0;
    uint32_t in_flight = 0;
    uint32_t head_bypassed = 0;            // admissions that passed over the job at the queue's head
    std::vector<Footprint> foot;           // per job of the run
    ltl_batch_stats stats{};
};

// ---------------------------------------------------------------------------
// Shared budget: first-fit regions of the batch workspace
// ---------------------------------------------------------------------------
static bool pool_alloc(ltl_batch *b, uint64_t size, uint64_t &off) {
    for (auto it = b->free_regions.begin(); it != b->free_regions.end(); ++it) {
        if (it->second < size) continue;
        off = it->first;
        const uint64_t rest = it->second - size;
        b->free_regions.erase(it);
        if (rest) b->free_regions[off + size] = rest;
        b->in_use += size;
        b->stats.peak_bytes = std::max(b->stats.peak_bytes, b->in_use);
        return true;
    }
    return false;
}

static void pool_release(ltl_batch *b, uint64_t off, uint64_t size) {
    b->in_use -= size;
    auto it = b->free_regions.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != b->free_regions.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_regions.erase(nx);
    }
    if (it != b->free_regions.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_regions.erase(it);
        }
    }
}

// Region bytes for `entries` stored matrices plus `cands` candidates of the level being
// evaluated (the language cache's hash and entry tables are the lane's own).
static uint64_t region_for(const Footprint &f, uint64_t entries, uint64_t cands) {
    const uint64_t body = f.fixed + entries * f.cmb + cands * 40;
    return std::max<uint64_t>(LTL_MIN_WORKSPACE, align_up(body + body / 8 + (8u << 20), 1u << 20));
}

// First estimate: the stored levels up to cost 5 (or the bound) with level sizes modelled
// as A * 5^(c-1) (about the growth of the workloads' first levels).  Too small an estimate
// costs a re-run in a larger region, never a different result.
static Footprint footprint_estimate(const ltl_batch_job &jb) {
    Footprint f;
    const ltl_spec &sp = jb.spec;
    const uint32_t T = sp.num_pos + sp.num_neg;
    std::vector<uint64_t> off((size_t)T + 1, 0);
    if (sp.flags & LTL_SPEC_DEVICE) {
        if (hipMemcpy(off.data(), sp.offsets, off.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            f.request = LTL_MIN_WORKSPACE;
            return f;
        }
    } else {
        memcpy(off.data(), sp.offsets, off.size() * 8);
    }
    uint64_t maxlen = 1;
    for (uint32_t t = 0; t < T; ++t) maxlen = std::max<uint64_t>(maxlen, off[t + 1] - off[t]);
    const uint64_t W = maxlen <= 32 ? 32 : 64;
    uint64_t r = 0;
    for (uint32_t t = 0; t < T; ++t) {
        const uint64_t w = (off[t + 1] - off[t] + W - 1) / W;
        if ((r & 63u) + w > 64u) r = align_up(r, 64);
        r += w;
    }
    const uint64_t R = align_up(std::max<uint64_t>(r, 1), 64);
    f.cmb = R * (W / 8);
    f.fixed = R * 64 + (uint64_t)sp.num_props * f.cmb + off[T] * 4 + (uint64_t)T * 16 + (4u << 20);
    uint64_t entries = 0, e = sp.num_props;
    for (uint32_t c = 1; c < std::min<uint32_t>(jb.cost_bound, 6); ++c, e *= 5) entries += e;
    f.request = region_for(f, entries, e);
    return f;
}

// Region for the next attempt of a job that ran out of memory: what its completed levels
// hold, plus one more level grown by the last growth factor (2..10), and at least four
// times the last region.
static uint64_t regrow(const Footprint &f, const ltl_result &res, uint64_t last) {
    const uint32_t d = std::min<uint32_t>(res.levels_done, LTL_MAX_LEVELS - 1);
    uint64_t stored = 0;
    for (uint32_t c = 1; c <= d; ++c) stored += res.level_new[c];
    const uint64_t en = d ? res.level_new[d] : 1, ep = d > 1 ? res.level_new[d - 1] : 1;
    const double g = std::min(10.0, std::max(2.0, (double)en / (double)std::max<uint64_t>(ep, 1)));
    const uint64_t cn = d ? res.level_candidates[d] : 1;
    const uint64_t need = region_for(f, stored + (uint64_t)(g * (double)en), (uint64_t)(g * (double)cn));
    return std::max<uint64_t>(last * 4, need);
}

static void batch_lane_jobs(ltl_batch *b, uint32_t lane) {
    for (;;) {
        const uint32_t i = b->next.fetch_add(1);
        if (i >= b->njobs) break;
        if (b->arrival_ms && b->arrival_ms[i] > 0.0)      // not admitted before it arrives
            std::this_thread::sleep_until(b->t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                                      std::chrono::duration<double, std::milli>(b->arrival_ms[i])));
        const auto a = std::chrono::steady_clock::now();
        ltl_learn(b->ctxs[lane], &b->jobs[i].spec, &b->jobs[i].ops, b->jobs[i].cost_bound, &b->results[i]);
        const auto e = std::chrono::steady_clock::now();
        if (b->job_ms) {
            b->job_ms[2 * (size_t)i] = std::chrono::duration<double, std::milli>(e - a).count();
            b->job_ms[2 * (size_t)i + 1] = std::chrono::duration<double, std::milli>(e - b->t0).count();
        }
    }
}

// Slots of the hash table a context sizes for a workspace of `bytes` (as job_setup does
// when hash_slots_log2 is 0).
static uint32_t auto_slots_log2(uint64_t bytes) {
    uint32_t sl = 26;
    while (sl > 10 && (24ull << sl) > bytes / 4) --sl;
    return sl;
}

// A job that ran out of memory would also run out, at the same level and with the same
// counts, in the whole pool `total`: its stored entries exceeded the entry cap (the
// lane's hash table does not depend on the region), or the new entries of its failing
// level alone exceed the pool.  Then the result of this run is final.
static bool oom_at_any_size(const Footprint &f, const ltl_result &res, int kind, uint64_t oom_new, uint64_t total) {
    if (kind == 3) return true;
    if (kind == 2 && f.cmb) {
        uint64_t stored = 0;
        for (uint32_t c = 1; c <= res.levels_done && c < LTL_MAX_LEVELS; ++c) stored += res.level_new[c];
        return (stored + oom_new) * f.cmb > total;
    }
    return false;
}

// Shared-budget lanes: each lane takes the first arrived job (in arrival order) whose
// requested region fits the free workspace, binds its context to that region and runs
// it; a job that runs out of memory in a region smaller than the whole workspace goes
// back to the head of the queue with a region four times larger.  To keep a large job
// at the head from waiting forever, at most 4 * lanes admissions may pass over it.
static void batch_lane_shared(ltl_batch *b, uint32_t lane) {
    ltl_ctx *c = b->ctxs[lane];
    const uint64_t total = b->pool_bytes;
    for (;;) {
        uint32_t i = 0;
        uint64_t req = 0, off = 0;
        {
            std::unique_lock<std::mutex> lk(b->pool_mu);
            for (;;) {
                if (b->jobs_left == 0) return;
                const double now_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - b->t0).count();
                bool found = false;
                double next_arrival = -1.0;
                size_t k = 0;
                for (auto it = b->queue.begin(); it != b->queue.end(); ++it, ++k) {
                    const double arr = b->arrival_ms ? b->arrival_ms[it->first] : 0.0;
                    if (arr > now_ms) {
                        next_arrival = arr;
                        break;
                    }
                    if (k > 0 && b->head_bypassed >= 4 * b->o.lanes) break;   // the head job's turn
                    if (pool_alloc(b, it->second, off)) {
                        i = it->first;
                        req = it->second;
                        b->head_bypassed = (k > 0) ? b->head_bypassed + 1 : 0;
                        b->queue.erase(it);
                        found = true;
                        break;
                    }
                }
                if (found) break;
                // a finished job notifies; otherwise the next arrival is the next event
                if (next_arrival >= 0.0)
                    b->pool_cv.wait_until(lk, b->t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                                          std::chrono::duration<double, std::milli>(next_arrival)));
                else
                    b->pool_cv.wait(lk);
            }
            ++b->in_flight;
            b->stats.max_in_flight = std::max(b->stats.max_in_flight, b->in_flight);
            ++b->stats.admissions;
        }
        // the lane's context on the job's region; its language cache (hash and entry tables)
        // is the lane's own, emptied by each job, so no job initialises a table
        c->o.workspace = (char *)b->o.workspace + b->pool_base + off;
        c->o.workspace_bytes = req;
        c->pool_total = total;
        const auto a = std::chrono::steady_clock::now();
        ltl_result &res = b->results[i];
        int kind = 0;
        uint64_t oom_new = 0;
        const int st = learn_job(c, &b->jobs[i].spec, &b->jobs[i].ops, b->jobs[i].cost_bound, &res, &kind, &oom_new);
        const auto e = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(b->pool_mu);
        pool_release(b, off, req);
        --b->in_flight;
        if (b->job_ms) b->job_ms[2 * (size_t)i] += std::chrono::duration<double, std::milli>(e - a).count();
        if (st == LTL_E_OOM && req < total && !oom_at_any_size(b->foot[i], res, kind, oom_new, total)) {
            b->queue.emplace_front(i, std::min<uint64_t>(total, regrow(b->foot[i], res, req)));
            ++b->stats.reruns;
        } else {
            if (b->job_ms) b->job_ms[2 * (size_t)i + 1] = std::chrono::duration<double, std::milli>(e - b->t0).count();
            b->stats.region_bytes_total += req;
            --b->jobs_left;
        }
        b->pool_cv.notify_all();
    }
}

// Waits up to `us` microseconds, polling, for pred(); true if it became true.  Runs
// come back to back, and a sleeping thread can take milliseconds to be woken.
template <typename Pred>
static bool spin_for(Pred pred, int us) {
    const auto t0 = std::chrono::steady_clock::now();
    while (!pred()) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(us)) return false;
        std::this_thread::yield();
    }
    return true;
}

constexpr int BATCH_SPIN_US = 5000;

static void batch_worker(ltl_batch *b, uint32_t lane) {
    (void)hipSetDevice(b->o.device);
    uint64_t seen = 0;
    for (;;) {
        if (!spin_for([&] { return b->quit.load() || b->generation.load() != seen; }, BATCH_SPIN_US)) {
            std::unique_lock<std::mutex> lk(b->mu);
            b->cv_start.wait(lk, [&] { return b->quit.load() || b->generation.load() != seen; });
        }
        if (b->quit.load()) return;
        seen = b->generation.load();
        if (b->shared) batch_lane_shared(b, lane);
        else batch_lane_jobs(b, lane);
        {
            std::lock_guard<std::mutex> lk(b->mu);
            if (b->lanes_busy.fetch_sub(1) == 1) b->cv_done.notify_all();
        }
    }
}

extern "C" void ltl_batch_destroy(ltl_batch *b) {
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->quit.store(true);
    }
    b->cv_start.notify_all();
    for (auto &t : b->workers) t.join();
    for (size_t l = 0; l < b->ctxs.size(); ++l)
        if (b->ctxs[l]) ltl_ctx_destroy(b->ctxs[l]);
    for (size_t l = 0; l < b->streams.size(); ++l)
        if (b->streams[l]) {
            (void)hipStreamSynchronize(b->streams[l]);
            (void)hipStreamDestroy(b->streams[l]);
        }
    delete b;
}

extern "C" int ltl_batch_create(const ltl_batch_opts *o, ltl_batch **out) {
    if (!out) return LTL_E_INVAL;
    *out = nullptr;
    if (!o || !o->workspace) return LTL_E_INVAL;
    if (o->lanes < 1 || o->lanes > 64) return LTL_E_INVAL;
    const bool shared = (o->flags & LTL_BATCH_SHARED_BUDGET) != 0;
    const uint64_t slice = (o->workspace_bytes / o->lanes) & ~255ull;
    if (shared ? o->workspace_bytes < LTL_MIN_WORKSPACE : slice < LTL_MIN_WORKSPACE) return LTL_E_INVAL;
    if (((uintptr_t)o->workspace) & 255u) return LTL_E_INVAL;
    if (shared && (o->hash_slots_log2 || o->max_entries)) return LTL_E_INVAL;   // sized per region
    if (hipSetDevice(o->device) != hipSuccess) return LTL_E_DEVICE;
    ltl_batch *b = new (std::nothrow) ltl_batch();
    if (!b) return LTL_E_INVAL;
    b->o = *o;
    b->shared = shared;
    // shared budget: each lane's language cache (hash and entry tables, 24 bytes a slot) at
    // the start of the workspace, as large as the hash table a context of the whole
    // workspace would have, or smaller until the lanes' caches take at most half of it;
    // the rest is the pool of job regions
    uint32_t cache_sl = auto_slots_log2(o->workspace_bytes);
    while (cache_sl > 10 && (uint64_t)o->lanes * (24ull << cache_sl) > o->workspace_bytes / 2) --cache_sl;
    const uint64_t cache_one = align_up(24ull << cache_sl, 256);
    const uint64_t cache_all = shared ? cache_one * o->lanes : 0;
    b->pool_base = cache_all;
    b->pool_bytes = shared ? ((o->workspace_bytes - cache_all) & ~255ull) : 0;
    if (shared && b->pool_bytes < LTL_MIN_WORKSPACE) {
        delete b;
        return LTL_E_INVAL;
    }
    const uint32_t lanes = o->lanes;
    b->streams.assign(lanes, nullptr);
    b->ctxs.assign(lanes, nullptr);
    int st = LTL_OK;
    for (uint32_t l = 0; l < lanes && st == LTL_OK; ++l) {
        if (hipStreamCreateWithFlags(&b->streams[l], hipStreamNonBlocking) != hipSuccess) {
            st = LTL_E_DEVICE;
            break;
        }
        ltl_ctx_opts co{};
        co.device = o->device;
        co.flags = o->flags & ~(LTL_BATCH_BIG_ALONE | LTL_BATCH_SHARED_BUDGET);
        // shared budget: a lane's context is bound to a region per job (set when the job
        // is admitted); until then it names the start of the workspace
        co.workspace = (char *)o->workspace + (shared ? cache_all : (uint64_t)l * slice);
        co.workspace_bytes = shared ? LTL_MIN_WORKSPACE : slice;
        co.stream = b->streams[l];
        co.hash_slots_log2 = o->hash_slots_log2;
        co.word_bits = o->word_bits;
        co.fp_bits = o->fp_bits;
        co.max_entries = o->max_entries;
        co.split_tiles = o->split_tiles;
        st = ltl_ctx_create(&co, &b->ctxs[l]);
        if (st == LTL_OK && (o->flags & LTL_BATCH_BIG_ALONE)) b->ctxs[l]->big_mu = &b->big_mu;
        if (st == LTL_OK && shared) {
            b->ctxs[l]->cache = (char *)o->workspace + (uint64_t)l * cache_one;
            b->ctxs[l]->cache_slots_log2 = cache_sl;
        }
    }
    if (st != LTL_OK) {
        ltl_batch_destroy(b);
        return st;
    }
    for (uint32_t l = 1; l < lanes; ++l) b->workers.emplace_back(batch_worker, b, l);
    *out = b;
    return LTL_OK;
}

static int batch_go(ltl_batch *b, const ltl_batch_job *jobs, uint32_t njobs, const double *arrival_ms,
                    ltl_result *results, double *job_ms);

extern "C" int ltl_batch_run(ltl_batch *b, const ltl_batch_job *jobs, uint32_t njobs, ltl_result *results,
                             double *job_ms) {
    return batch_go(b, jobs, njobs, nullptr, results, job_ms);
}

extern "C" int ltl_batch_serve(ltl_batch *b, const ltl_batch_job *jobs, uint32_t njobs, const double *arrival_ms,
                               ltl_result *results, double *job_ms) {
    if (!arrival_ms && njobs) return LTL_E_INVAL;
    for (uint32_t i = 0; i < njobs; ++i)
        if (!(arrival_ms[i] >= 0.0) || (i && arrival_ms[i] < arrival_ms[i - 1])) return LTL_E_INVAL;
    return batch_go(b, jobs, njobs, arrival_ms, results, job_ms);
}

static int batch_go(ltl_batch *b, const ltl_batch_job *jobs, uint32_t njobs, const double *arrival_ms,
                    ltl_result *results, double *job_ms) {
    if (!b || (!jobs && njobs) || (!results && njobs)) return LTL_E_INVAL;
    if (b->running.exchange(true)) return LTL_E_STATE;
    if (hipSetDevice(b->o.device) != hipSuccess) {
        b->running = false;
        return LTL_E_DEVICE;
    }
    b->jobs = jobs;
    b->njobs = njobs;
    b->results = results;
    b->job_ms = job_ms;
    b->arrival_ms = arrival_ms;
    b->next = 0;
    if (b->shared) {      // every job starts with its footprint estimate
        b->stats = ltl_batch_stats{};
        b->stats.budget_bytes = b->pool_bytes;
        b->free_regions.clear();
        b->free_regions[0] = b->pool_bytes;
        b->in_use = 0;
        b->queue.clear();
        b->foot.resize(njobs);
        // a first region of at least a third of a lane's even share: the lanes' first
        // regions take at most a third of the budget, and most jobs then fit at once
        // (each re-run repeats the levels before its failure)
        const uint64_t floor = align_up(b->stats.budget_bytes / (3ull * b->o.lanes), 1u << 20) & ~255ull;
        for (uint32_t i = 0; i < njobs; ++i) {
            b->foot[i] = footprint_estimate(jobs[i]);
            b->queue.emplace_back(i, std::min<uint64_t>(b->stats.budget_bytes,
                                                        std::max<uint64_t>(floor, b->foot[i].request)));
        }
        b->jobs_left = njobs;
        b->in_flight = 0;
        b->head_bypassed = 0;
        if (job_ms)
            for (uint32_t i = 0; i < 2 * njobs; ++i) job_ms[i] = 0.0;
    }
    b->t0 = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->lanes_busy = (uint32_t)b->workers.size();
        b->generation.fetch_add(1);
    }
    b->cv_start.notify_all();
    if (b->shared) batch_lane_shared(b, 0);
    else batch_lane_jobs(b, 0);
    if (!spin_for([&] { return b->lanes_busy.load() == 0; }, BATCH_SPIN_US)) {
        std::unique_lock<std::mutex> lk(b->mu);
        b->cv_done.wait(lk, [&] { return b->lanes_busy.load() == 0; });
    }
    b->running = false;
    return LTL_OK;
}

extern "C" int ltl_batch_get_stats(ltl_batch *b, ltl_batch_stats *out) {
    if (!b || !out) return LTL_E_INVAL;
    std::lock_guard<std::mutex> lk(b->pool_mu);
    *out = b->stats;
    return LTL_OK;
}

extern "C" int ltl_learn_batch(const ltl_batch_opts *o, const ltl_batch_job *jobs, uint32_t njobs,
                               ltl_result *results, double *job_ms) {
    if (!o || (!jobs && njobs) || (!results && njobs)) return LTL_E_INVAL;
    ltl_batch_opts oo = *o;
    if (oo.lanes >= 1 && oo.lanes <= 64) oo.lanes = std::min<uint32_t>(oo.lanes, std::max<uint32_t>(njobs, 1u));
    // the slice size is that of the requested lane count, so results do not depend on njobs
    if (o->lanes >= 1 && o->lanes <= 64 && !(o->flags & LTL_BATCH_SHARED_BUDGET))
        oo.workspace_bytes = ((o->workspace_bytes / o->lanes) & ~255ull) * oo.lanes;
    ltl_batch *b = nullptr;
    int st = ltl_batch_create(&oo, &b);
    if (st != LTL_OK) return st;
    st = ltl_batch_run(b, jobs, njobs, results, job_ms);
    ltl_batch_destroy(b);
    return st;
}
