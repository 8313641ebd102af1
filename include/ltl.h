/*
 * ltl.h -- C-ABI of the MI355X (gfx950) enumerative LTL learner.
 *
 * The library learns a minimal-cost LTL formula separating positive traces P
 * from negative traces N (the "LTL learning problem" of Sec. 2 of "LTL
 * learning on GPUs", arXiv 2402.12373): bottom-up, cost-ordered enumeration
 * (Sec. 3, enum / handleOp), every candidate represented by its characteristic
 * matrix over all positions of all traces (Sec. 4), computed from its
 * children's matrices by branch-free word-parallel operators (Sec. 4 and
 * App. B), deduplicated exactly by observational equivalence modulo the
 * suffix-closure of P and N (Sec. 4; the exhaustive case of Sec. 5), and
 * checked against the separation predicate of Sec. 4 at position 0.
 *
 * Conventions common to all calls
 *   - Traces are numbered P first (in the given order), then N (Sec. 4 fixes a
 *     total order on P and N).
 *   - Functions return LTL_OK (0), LTL_NOT_FOUND (1, not an error) or a
 *     negative error code; nothing is thrown and nothing aborts.
 *   - Device memory: the library allocates none.  All device buffers live in
 *     the caller-provided workspace (ltl_ctx_opts.workspace); host-side state
 *     is ordinary malloc'd memory owned by the context / job.
 *   - A context runs one job at a time; calls on one context are not
 *     thread-safe.  Different contexts may share a device if their workspaces
 *     are disjoint.
 */
#ifndef LTL_H
#define LTL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define LTL_OK              0    /* success; for learning: a separating formula was found     */
#define LTL_NOT_FOUND       1    /* no separating formula of cost <= bound; counts are valid   */
#define LTL_E_INVAL        (-1)  /* null pointer, bad size, bad letter, empty trace, bad costs */
#define LTL_E_INCONSISTENT (-2)  /* a trace occurs in both P and N (Sec. 2 requires P, N disjoint) */
#define LTL_E_TOO_LONG     (-3)  /* a trace is longer than LTL_MAX_TRACE_LEN positions         */
#define LTL_E_OOM          (-4)  /* a level that must be stored exceeds the workspace or the
                                    entry cap; counts of the completed levels stay valid       */
#define LTL_E_DEVICE       (-5)  /* a HIP runtime error                                        */
#define LTL_E_STATE        (-6)  /* call out of order (e.g. levels not evaluated in order)     */
#define LTL_E_BUFFER       (-7)  /* an output buffer is too small; the size needed is reported */

#define LTL_MAX_TRACE_LEN  4096  /* positions per trace (64 words of 64 bits)                  */
#define LTL_MAX_LEVELS     64    /* cost levels 0..63                                          */
#define LTL_MAX_NODES      64    /* nodes of a returned formula                                */
#define LTL_NO_SOLUTION    UINT64_MAX

/* ---------------------------------------------------------------- connectives (Sec. 2 grammar) */
enum {
    LTL_ATOM = 0,   /* atomic proposition p                                     */
    LTL_NOT  = 1,   /* negation                                                 */
    LTL_AND  = 2,   /* conjunction                                              */
    LTL_OR   = 3,   /* disjunction                                              */
    LTL_X    = 4,   /* next (strong: false at the last position)                */
    LTL_F    = 5,   /* eventually                                               */
    LTL_G    = 6,   /* always (until the end of the trace)                      */
    LTL_U    = 7    /* until                                                    */
};

/* ---------------------------------------------------------------- context */
typedef struct ltl_ctx ltl_ctx;
typedef struct ltl_job ltl_job;

#define LTL_CTX_U_CARRY   0x1u   /* compute U by a carry-propagating add (one add per word and
                                    a prefix over the words of a trace) instead of the log2(n)
                                    shift-doubling of App. B; both give identical matrices.
                                    This is the default (it was faster on every row layout
                                    measured); LTL_CTX_U_DOUBLING selects the doubling         */
#define LTL_CTX_LDS_TILES 0x20u  /* binary connectives of whole-row levels stage their child
                                    operands in LDS: a workgroup of 4 waves loads the words of
                                    8 + 8 children once per row block for an 8 x 8 group of
                                    pairs, instead of each wave reading its 4 + 4 children
                                    into registers for a 4 x 4 tile (the default); a tile
                                    shape for ltl_autotune, results are identical               */
#define LTL_CTX_U_DOUBLING 0x10u /* compute U by the shift-doubling of App. B at every level
                                    instead of the carry adder (LTL_CTX_U_CARRY wins if both
                                    are set)                                                   */
#define LTL_CTX_ONE_STREAM 0x80u /* run every kernel on the context's stream: the U class of a
                                    whole-row level is not forked onto a second stream beside
                                    the other classes (batch lanes, whose jobs already overlap) */
#define LTL_CTX_TIMING    0x2u   /* record GPU time per kernel kind and per level (HIP events
                                    around each kernel group)                                  */
#define LTL_CTX_TIMING_LEVEL 0x4u /* record only the GPU time of each level: one event pair from
                                    its first to its last kernel (level_ms; kernel_ms stays 0) */
#define LTL_CTX_RUC       0x8u   /* relaxed uniqueness check (Sec. 5): a candidate is cached iff
                                    its 126-bit key is new; matrices are never compared (no
                                    verification pass).  The key of a matrix of at most 126 bits
                                    is the matrix itself (trace by trace, P then N), so the check
                                    is exact there.  A larger matrix is hashed: two keyed sums
                                    over its 32-position chunks (chunk j of trace t: positions
                                    32j..32j+31, first position in the top bit),
                                        A = sum premix(v, a) * a,  B = sum premix(v, b) * b
                                    (mod 2^64), premix(v, k) = y ^ (y >> 16) with
                                    y = (v ^ (v >> 8)) + k (mod 2^32); a and b are the top halves,
                                    low bit set, of draws 2i and 2i + 1 of the SplitMix64
                                    sequence of ltl_ctx_opts.ruc_seed, i = t * 2^32 + j; the key
                                    is the top 63 bits of A, then of B.  False positives drop
                                    languages (the formula found separates but may cost more
                                    than the minimum); level counts count new keys.  The entry
                                    kept for a key is its canonical-first candidate.  Levels run
                                    the whole-row kernels                                        */
#define LTL_CTX_RUC_FKP   0x40u  /* with LTL_CTX_RUC: keys by first-k-percent (Sec. 7) instead
                                    of hashing: the first m_t = round(k |tr_t| / 100) positions
                                    (halves rounded up) of each trace, concatenated in trace
                                    order and cut after 126 bits, k in 1..100 the smallest whose
                                    total is nearest to 126 bits                                 */

typedef struct {
    int32_t  device;            /* HIP device ordinal used by every call of this context        */
    uint32_t flags;             /* LTL_CTX_*                                                    */
    void    *workspace;         /* device pointer, caller-owned, 256-byte aligned, valid until
                                   ltl_ctx_destroy; the library writes only inside it           */
    uint64_t workspace_bytes;   /* its size                                                     */
    void    *stream;            /* hipStream_t for all work; NULL = the null stream             */
    uint32_t hash_slots_log2;   /* language-cache hash table size; 0 = automatic                */
    uint32_t word_bits;         /* 0 = automatic (32 if every trace has <= 32 positions, else 64),
                                   or 32 / 64                                                   */
    uint32_t fp_bits;           /* debug: keep only this many fingerprint bits (1..64), forcing
                                   collisions that the exact compare must resolve; 0 = 64       */
    uint32_t split_tiles;       /* a level of fewer than this many tiles (4 children a side) runs
                                   the row-split kernels (several waves per tile), a larger one
                                   the whole-row kernels (one wave per tile, one dispatch per
                                   connective class); 0 = the library's default (8192).  1 forces
                                   the whole-row kernels and 0xFFFFFFFF the row-split kernels at
                                   every level; results do not depend on it                     */
    uint64_t max_entries;       /* cap on stored language-cache entries; 0 = derived from the
                                   hash table (half its slots)                                  */
    uint64_t ruc_seed;          /* LTL_CTX_RUC: seed of the keyed sums' keys                    */
    uint32_t ruc_key_bits;      /* LTL_CTX_RUC, debug: keep only the first ruc_key_bits bits
                                   (1..125) of every key, forcing false positives; 0 = 126      */
    uint32_t reserved;          /* 0                                                            */
} ltl_ctx_opts;

/* Create a context on opts->device.  Returns LTL_E_INVAL for a null/unaligned
 * workspace or size < LTL_MIN_WORKSPACE, LTL_E_DEVICE if the device cannot be
 * selected.  *out is set only on success. */
#define LTL_MIN_WORKSPACE (16ull << 20)
int  ltl_ctx_create(const ltl_ctx_opts *opts, ltl_ctx **out);
void ltl_ctx_destroy(ltl_ctx *ctx);

/* ---------------------------------------------------------------- specification */
#define LTL_SPEC_DEVICE 0x1u    /* letters and offsets are device pointers (already in HBM) */

typedef struct {
    uint32_t num_props;         /* |Sigma|, 1..32; a letter is a bitmask of true propositions */
    uint32_t num_pos;           /* |P|: traces 0 .. num_pos-1                                 */
    uint32_t num_neg;           /* |N|: traces num_pos .. num_pos+num_neg-1                   */
    uint32_t flags;             /* LTL_SPEC_*                                                 */
    const uint32_t *letters;    /* offsets[num_pos+num_neg] letters, trace after trace;
                                   read during the call only (copied to the device)           */
    const uint64_t *offsets;    /* num_pos+num_neg+1 prefix offsets, offsets[0] = 0           */
} ltl_spec;

/* Cost-homomorphism restricted to an operator set (Sec. 2): cost(op phi psi) =
 * cost[op] + cost(phi) + cost(psi).  Disabled connectives are never used. */
typedef struct {
    uint32_t op_mask;           /* bit k enables connective k; bit LTL_ATOM must be set;
                                   LTL_OPS_NNF may be added; other bits are an error (INVAL)  */
    uint32_t cost[8];           /* cost of each enabled connective, >= 1                       */
} ltl_opset;

/* op_mask flag: negation normal form, i.e. negation applies to atoms only (the
 * formulae of the experiments of Sec. 7 are learned U-free and in this form; a
 * U-free set simply leaves bit LTL_U clear).  The cache keeps each language at its
 * least cost, so the children of a negation are exactly the entries of the atom
 * level (cost[LTL_ATOM]); the canonical order is otherwise unchanged. */
#define LTL_OPS_NNF (1u << 8)

/* Kernel kinds for per-kind GPU time (LTL_CTX_TIMING). */
enum {
    LTL_K_EVAL = 0,          /* level evaluation: matrices, fingerprints, separation, cache claims */
    LTL_K_VERIFY = 1,        /* full compare of every presumed duplicate with its owner            */
    LTL_K_MATERIALIZE = 2,   /* writing the new entries of a level                                  */
    LTL_K_COMPACT = 3,       /* representative bits, prefix scan, recipes, slot settlement          */
    LTL_K_FALLBACK = 4,      /* exact resolution of fingerprint collisions                          */
    LTL_K_INTAKE = 5,        /* specification intake: packing, table init, validation               */
    LTL_K_KINDS = 6
};

/* Formula as postfix nodes; children are earlier node indices. */
typedef struct {
    uint32_t op;                /* LTL_ATOM .. LTL_U                                           */
    uint32_t a;                 /* ATOM: proposition index; otherwise first child node         */
    uint32_t b;                 /* second child node for AND, OR, U; else 0                    */
} ltl_node;

typedef struct {
    int32_t  status;                           /* LTL_OK / LTL_NOT_FOUND / error           */
    uint32_t cost;                             /* minimal cost when status == LTL_OK        */
    uint32_t levels_done;                      /* highest cost level fully evaluated        */
    uint32_t num_nodes;                        /* nodes of the solution                     */
    ltl_node nodes[LTL_MAX_NODES];             /* the solution (root = last node)           */
    uint64_t solution_index;                   /* canonical index of the solution in its
                                                  level, or LTL_NO_SOLUTION                 */
    uint64_t level_new[LTL_MAX_LEVELS];        /* distinct new languages per cost level     */
    uint64_t level_candidates[LTL_MAX_LEVELS]; /* candidates evaluated per cost level       */
    double   level_ms[LTL_MAX_LEVELS];         /* GPU time per level (LTL_CTX_TIMING or
                                                  LTL_CTX_TIMING_LEVEL)                     */
    uint64_t colliders;                        /* fingerprint collisions resolved exactly   */
    double   kernel_ms[LTL_K_KINDS];           /* GPU time per kernel kind (LTL_CTX_TIMING) */
    uint32_t kernel_launches[LTL_K_KINDS];     /* launches per kernel kind                  */
    uint32_t pad;
    uint64_t level_bytes[LTL_MAX_LEVELS];      /* algorithmic HBM bytes per level (see
                                                  ltl_level_stats.alg_bytes)                */
} ltl_result;

/* ---------------------------------------------------------------- learning */

/* Learn a sound and minimal formula for (P, N) under the cost-homomorphism
 * (Sec. 2 "LTL learning problem"), searching costs up to cost_bound inclusive.
 * Returns the status also stored in out->status: LTL_OK with the solution, or
 * LTL_NOT_FOUND (no separating formula of cost <= cost_bound), or an error.
 * Per-level counts in *out are valid for levels 1..levels_done in every case.
 * Deterministic: the same inputs give the same result, whatever the launch
 * configuration. */
int ltl_learn(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
              ltl_result *out);

/* ---------------------------------------------------------------- autotuning */

/* The project's autotuner for tile shapes and level schedules: runs the job (spec,
 * ops, cost_bound) on ctx once untimed, then once per configuration, timing each whole
 * job on the host clock, and reports the configurations, their times and the fastest
 * (index `best`).  A configuration is a binary tile shape (child operands read into
 * registers for 4 x 4 pairs, flags 0, or staged in LDS for 8 x 8 pairs,
 * LTL_CTX_LDS_TILES) and the level size in tiles from which levels run the
 * whole-row kernels (ltl_ctx_opts.split_tiles).  The caller applies the choice to its
 * contexts or batches; ctx's options are restored.  Every configuration must give the
 * same result (status, counts, solution): LTL_E_STATE if one does not.  Errors as
 * ltl_learn (a job that runs out of memory is timed like any other). */
#define LTL_TUNE_CONFIGS 5
typedef struct {
    uint32_t tried;                          /* configurations timed                     */
    uint32_t best;                           /* index of the fastest                      */
    uint32_t flags[LTL_TUNE_CONFIGS];        /* LTL_CTX_LDS_TILES or 0                    */
    uint32_t split_tiles[LTL_TUNE_CONFIGS];  /* ltl_ctx_opts.split_tiles                  */
    double   ms[LTL_TUNE_CONFIGS];           /* wall time of the job, the fastest of three
                                                runs (milliseconds)                       */
} ltl_tuning;
int ltl_autotune(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound, ltl_tuning *out);

/* ---------------------------------------------------------------- learning without allocation */

/* For callers that cannot allocate device memory or call allocating HIP routines
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): ltl_learn on the library's own fixed device scratch array of
 * LTL_NOALLOC_SCRATCH_BYTES per GPU (a static device array of the library's code
 * object, held by each GPU the library runs on until the process ends) instead
 * of a caller workspace.  No hipMalloc, hipHostMalloc, hipFree, stream or event
 * is created; the caller passes the device, a stream (NULL = the null stream),
 * the inputs and *out.  The hash table is 2^LTL_NOALLOC_SLOTS_LOG2 slots; U by
 * the carry adder; no timing.  A specification or a level that does not fit the array
 * returns LTL_E_OOM (nothing is allocated instead).  Calls on one GPU share its
 * array, which keeps the last call's contents (the call clears what must start at
 * zero); overlapping calls on one GPU would race, so the library runs them one at
 * a time (the call returns when its work on the stream has ended).  Results
 * equal ltl_learn's on a context with the same hash table size.  Errors as
 * ltl_learn, and LTL_E_DEVICE if the array's address cannot be found. */
#define LTL_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define LTL_NOALLOC_SLOTS_LOG2    18
int ltl_learn_noalloc(int32_t device, void *stream, const ltl_spec *spec, const ltl_opset *ops,
                      uint32_t cost_bound, ltl_result *out);

/* ---------------------------------------------------------------- batched learning */

/* Many independent learning jobs of uneven sizes, run `lanes` at a time.  Each
 * lane has its own HIP stream, its own slice of the workspace (workspace_bytes /
 * lanes, 256-byte aligned) and its own context, so the levels of different jobs
 * overlap on the device; every job's result equals that of ltl_learn on a
 * context with the same options and a workspace of the slice's size. */
/* Batch flag: the whole-row levels (the device-filling ones) of different lanes run
 * one at a time; smaller levels still overlap.  For mixes dominated by large jobs,
 * whose big levels slow each other down when they share the device. */
#define LTL_BATCH_BIG_ALONE 0x100u
/* Batch flag: one shared device-memory budget (the whole workspace) instead of equal
 * slices.  Each job is admitted with a region of the workspace sized by its estimated
 * language-cache footprint (fixed tables plus the modelled matrices of its first
 * levels, at least a quarter of workspace / lanes); free lanes take arrived jobs in
 * arrival order, the first one whose region fits the free memory (a job passed over
 * 4 * lanes times is admitted next).  A job that runs out of memory in a region smaller
 * than the workspace is run again, at the head of the queue, in a region sized from its
 * completed levels (at least four times larger), so its result equals that of ltl_learn
 * on a context with enough memory (or with the whole workspace).  Each lane keeps its
 * own language-cache tables (hash table and entry tables, 24 bytes a slot) at the start
 * of the workspace, emptied by every job, with the slots a context of the whole
 * workspace would have (fewer if the lanes' tables would take more than half of it;
 * hash_slots_log2 and max_entries must be 0); the rest is the pool of regions, whose use
 * never exceeds it (ltl_batch_get_stats reports the pool and the peak). */
#define LTL_BATCH_SHARED_BUDGET 0x200u

typedef struct {
    int32_t  device;
    uint32_t flags;              /* LTL_CTX_* for every job, and LTL_BATCH_BIG_ALONE        */
    void    *workspace;          /* device pointer, caller-owned, split evenly among lanes   */
    uint64_t workspace_bytes;
    uint32_t lanes;              /* jobs in flight at once, 1..64                            */
    uint32_t hash_slots_log2;    /* per lane; 0 = automatic                                  */
    uint32_t word_bits;          /* as in ltl_ctx_opts                                       */
    uint32_t fp_bits;
    uint64_t max_entries;        /* per job; 0 = derived from the lane's hash table          */
    uint32_t split_tiles;        /* as in ltl_ctx_opts (e.g. from ltl_autotune)              */
    uint32_t reserved;
} ltl_batch_opts;

typedef struct {
    ltl_spec  spec;              /* host or device buffers (LTL_SPEC_DEVICE)                 */
    ltl_opset ops;
    uint32_t  cost_bound;
    uint32_t  reserved;
} ltl_batch_job;

/* Runs jobs[0..njobs-1] (taken in order by free lanes).  results[i] receives job
 * i's result; if job_ms is not NULL, job_ms[2*i] is its duration and
 * job_ms[2*i+1] its completion time since the call began (milliseconds, host
 * clock).  Returns LTL_OK if every job ran (each job's own status is in its
 * result), LTL_E_INVAL for bad options, LTL_E_DEVICE if a lane could not start. */
int ltl_learn_batch(const ltl_batch_opts *opts, const ltl_batch_job *jobs, uint32_t njobs, ltl_result *results,
                    double *job_ms);

/* The same lanes kept for many calls: a batch executor owns `lanes` contexts
 * (each with its stream, its workspace slice and its hash table, initialised
 * once) and lanes-1 host worker threads.  ltl_batch_run has the semantics of
 * ltl_learn_batch with the executor's options; consecutive runs reuse the
 * tables (each job empties the slots it used).  One run at a time per executor
 * (LTL_E_STATE if a run is already in progress).  The caller keeps the
 * workspace alive until ltl_batch_destroy, which waits for the lanes' streams.
 * Errors of ltl_batch_create: LTL_E_INVAL (options), LTL_E_DEVICE. */
typedef struct ltl_batch ltl_batch;
int ltl_batch_create(const ltl_batch_opts *opts, ltl_batch **out);
int ltl_batch_run(ltl_batch *batch, const ltl_batch_job *jobs, uint32_t njobs, ltl_result *results,
                  double *job_ms);

/* Serving: as ltl_batch_run, but job i arrives arrival_ms[i] milliseconds after the
 * call begins (non-decreasing, >= 0) and no lane starts it before then; free lanes
 * take arrived jobs in arrival order, each within its lane's workspace slice (its share
 * of device memory).  job_ms as in ltl_learn_batch (completion times count from the call's
 * start, so a job's latency is job_ms[2*i+1] - arrival_ms[i]).  Each job's result equals
 * that of ltl_learn on a lane's context.  Errors: LTL_E_INVAL (arrival times missing,
 * negative or decreasing), else as ltl_batch_run. */
int ltl_batch_serve(ltl_batch *batch, const ltl_batch_job *jobs, uint32_t njobs, const double *arrival_ms,
                    ltl_result *results, double *job_ms);
void ltl_batch_destroy(ltl_batch *batch);

/* Memory accounting of the last run of a shared-budget batch (LTL_BATCH_SHARED_BUDGET):
 * the pool of job regions, the peak bytes of regions in use at once, admissions (runs started,
 * re-runs included), re-runs after out-of-memory, the most jobs in flight at once and
 * the summed region bytes of the finished jobs.  Zero for a batch with slices. */
typedef struct {
    uint64_t budget_bytes;
    uint64_t peak_bytes;
    uint32_t admissions;
    uint32_t reruns;
    uint32_t max_in_flight;
    uint32_t pad;
    uint64_t region_bytes_total;
} ltl_batch_stats;
int ltl_batch_get_stats(ltl_batch *batch, ltl_batch_stats *out);

/* ---------------------------------------------------------------- level-by-level interface */

/* Start a learning job (Sec. 3 enum, before its first level): validate the
 * specification (Sec. 2: finite non-empty traces, P and N disjoint) and pack it
 * into the context's workspace (row layout and the atom matrices, i.e. the
 * characteristic matrices of the atomic propositions of Sec. 4); the job is then
 * driven one cost level at a time by ltl_eval_level.  cost_bound (inclusive,
 * 1..63) is the last level.  The job owns host state until ltl_job_destroy and
 * uses the context exclusively (LTL_E_STATE while another job is open).
 * Errors: LTL_E_INVAL, LTL_E_INCONSISTENT, LTL_E_TOO_LONG, LTL_E_OOM (workspace
 * too small for the fixed tables), LTL_E_DEVICE, LTL_E_STATE. */
int ltl_job_create(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t cost_bound,
                   ltl_job **out);

typedef struct {
    uint32_t cost;               /* the level evaluated                                   */
    uint32_t stored;             /* 1 if its matrices were kept for later levels          */
    uint64_t candidates;         /* candidates of this level in the canonical order       */
    uint64_t new_entries;        /* distinct languages first reached at this cost         */
    uint64_t first_solution;     /* smallest separating canonical index, or LTL_NO_SOLUTION */
    uint64_t colliders;          /* fingerprint matches whose full compare failed         */
    double   kernel_ms;          /* GPU time of the level (LTL_CTX_TIMING[_LEVEL]), else 0 */
    uint64_t alg_bytes;          /* algorithmic HBM bytes of the level: one matrix per
                                    candidate (written if new, else compared with the
                                    stored one; a level that is not stored writes none)
                                    plus each child matrix read once per tile (4 children
                                    a side); re-reads are not counted                     */
} ltl_level_stats;

/* Evaluate exactly one cost level: every candidate of cost `cost` built from the
 * stored levels by one connective (Sec. 3 handleOp), in the canonical order
 * (op in F, U, G, X, AND, OR, NOT; splits a ascending; pairs row-major; AND/OR
 * with a <= b and i < j on the diagonal), with the separation check and exact
 * dedup.  Levels must be evaluated in order 1, 2, ... (LTL_E_STATE otherwise,
 * and after a solution was found, after LTL_E_OOM, or beyond the job's bound).
 * Returns LTL_OK or an error; stats may be NULL. */
int ltl_eval_level(ltl_job *job, uint32_t cost, ltl_level_stats *stats);

/* Result so far (status LTL_OK once a level has a separating candidate,
 * LTL_NOT_FOUND while none has, or the error that stopped the job). */
int ltl_job_result(ltl_job *job, ltl_result *out);

/* The overfitting formula of (P, N) (Sec. 2): the disjunction, over the traces of
 * P in order, of tr's description, in which each position's letter is the
 * conjunction of every proposition (in index order), negated when it is absent,
 * chained to the next position by X, and the last letter conjoined with not X true
 * (the last position; true = p0 or not p0).  Its language is exactly P, so it
 * separates (P, N); the learner of Sec. 3 enumerates below its cost and returns it
 * when nothing cheaper separates.  Host-only (no device call): reads the spec's host
 * buffers.  Writes the postfix nodes (root last, no shared subformulas) into
 * buf[0..cap) and their cost under `ops` into *cost.  Errors: LTL_E_INVAL (null
 * pointer, device spec, invalid spec or letters, an operator set without NOT, AND,
 * OR or X, or with LTL_OPS_NNF: not X true negates a compound formula), LTL_E_OOM
 * (more than cap nodes; *num_nodes then holds the number needed). */
int ltl_overfit(const ltl_spec *spec, const ltl_opset *ops, ltl_node *buf, uint32_t cap, uint32_t *num_nodes,
                uint64_t *cost);

/* ---------------------------------------------------------------- formulas on traces, splitting */

/* tr |= phi for every trace of a specification (Sec. 2: phi holds at position 0
 * of tr under the finite-trace semantics: strong X, nothing holds past the end).
 * nodes[0 .. num_nodes) is a postfix formula (children before parents, root
 * last).  The formula's characteristic matrix is computed node by node on the
 * device with the learner's own connective kernels, in the context's workspace
 * (num_nodes matrices); out[t] = 1 if trace t (P first, then N; the classes play
 * no other part and may overlap) satisfies it, else 0.  The caller owns out
 * (num_pos + num_neg bytes).  Uses the context like a job (LTL_E_STATE while one
 * is open).  Errors: LTL_E_INVAL (null pointer, a node naming a later node or a
 * missing proposition, a bad spec), LTL_E_TOO_LONG, LTL_E_OOM (the matrices do
 * not fit the workspace), LTL_E_DEVICE. */
int ltl_holds(ltl_ctx *ctx, const ltl_spec *spec, const ltl_node *nodes, uint32_t num_nodes, uint8_t *out);

/* Deterministic splitting (Sec. 6, detSplit): a specification of at most `win`
 * traces (or of at most one trace per class) goes to the learner of Sec. 3
 * (ltl_learn below the cost of the overfitting formula, else that formula; see
 * ltl_overfit).  A larger one is split into halves P1 | P2 and N1 | N2 (in the
 * given order, first floor(n/2) traces) and learned as
 *   phi11 = split(P1, N1),  phi12 = split(P1, N2 accepted by phi11),
 *   phi21 = split(P2 - L, N1),  phi22 = split(P2 - L, N2 accepted by phi21),
 *   (phi11 and phi12) or (phi21 and phi22),
 * with L the P2 traces that phi11 and phi12 both accept (the traces the first
 * disjunct accepts; the paper's union would drop traces the conjunction rejects,
 * making the result unsound).  A part with no positive trace contributes no
 * disjunct; a conjunct with no negative trace left is dropped.  If any part runs
 * out of memory, the whole call is repeated with win / 2.  The result is sound
 * (accepts P, rejects N), not necessarily minimal.  The spec must be host
 * buffers with at least one trace per class; the leaves run on ctx.  The formula
 * goes to buf[0 .. cap) as postfix nodes, its size to *num_nodes.  Errors:
 * LTL_E_INVAL, LTL_E_OOM (out of memory even at a window of 1),
 * LTL_E_BUFFER (more than cap nodes; *num_nodes holds the size), and the
 * learner's errors. */
int ltl_det_split(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t win, ltl_node *buf,
                  uint32_t cap, uint32_t *num_nodes);

/* Random splitting (Sec. 6, randSplit): phi11 = the learner of Sec. 3 on a
 * random sub-specification (P0, N0) of at most w traces, as large as possible
 * and with the classes as equal in size as possible (|P0| = min(|P|,
 * ceil(t/2)), |N0| = min(|N|, t - |P0|), then |P0| = min(|P|, t - |N0|), with
 * t = min(w, |P| + |N|)), starting at w = win and halving w while the learner
 * runs out of memory (a specification that fits is drawn whole); then, with
 * A the traces phi11 accepts,
 *   phi12 = split(P in A, N in A), phi21 = split(P - A, N - A), phi22 = split(P - A, N in A),
 *   (phi11 and phi12) or (phi21 and phi22)
 * (a part with no positive trace is false and drops its disjunct; a part with no
 * negative trace is true and drops out of its conjunction).  The random subsets:
 * the q-th draw of the recursion (q = 0, 1, ... in call order) takes the P0
 * indices from stream 2q and the N0 indices from stream 2q + 1, where stream c
 * is the SplitMix64 sequence (Steele, Lea and Flood, OOPSLA 2014) started at
 * state seed * 2^32 + c: index i gets the output mix(state + (i + 1) * gamma),
 * and the k indices with the smallest outputs are taken.  seed < 2^32.  Output,
 * requirements and errors as ltl_det_split (LTL_E_OOM: a window below 2). */
int ltl_rand_split(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t win, uint64_t seed,
                   ltl_node *buf, uint32_t cap, uint32_t *num_nodes);

/* Formula of stored entry `entry` of level `cost`: the recipe of the entry's
 * representative (the first candidate of its language in the canonical order of
 * Sec. 3's enumeration), expanded into its children's recipes down to the atoms
 * (postfix nodes into buf, at most cap).  Errors: LTL_E_INVAL (no such entry, cap
 * too small). */
int ltl_job_formula(ltl_job *job, uint32_t cost, uint64_t entry, ltl_node *buf, uint32_t cap,
                    uint32_t *num_nodes);

/* Characteristic matrix (Sec. 4: the characteristic sequences of all traces, in
 * the order P then N) of stored entry `entry` of level `cost`, one byte (0/1)
 * per position, traces in order P then N, positions 0..|tr|-1 of each.  cap must
 * be >= the total number of positions.  Only stored levels keep their matrices
 * (a level with a solution, or at the cost bound, is not stored): LTL_E_STATE
 * otherwise.  For tests and debugging. */
int ltl_job_dump_cm(ltl_job *job, uint32_t cost, uint64_t entry, uint8_t *pos_bits, uint64_t cap);

typedef struct {
    uint32_t word_bits;          /* 32 or 64                                               */
    uint32_t rows;               /* machine words per characteristic matrix                */
    uint64_t cm_bytes;           /* bytes per stored matrix                                */
    uint64_t total_positions;    /* sum of trace lengths                                   */
    uint32_t hash_slots_log2;
    uint32_t doubling_steps;     /* ceil(log2(longest trace)) steps of U doubling          */
    uint64_t arena_bytes;        /* workspace bytes available for stored matrices          */
    uint64_t max_entries;
} ltl_job_info;

int  ltl_job_get_info(ltl_job *job, ltl_job_info *out);
void ltl_job_destroy(ltl_job *job);

/* Static description of a status code. */
const char *ltl_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* LTL_H */
