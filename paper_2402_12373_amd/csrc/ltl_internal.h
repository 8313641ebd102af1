// Internal structures shared by the host runtime and the gfx950 kernels of the
// LTL learner.  Not part of the public C-ABI (include/ltl.h).
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace ltl {

// Language-cache hash table slot values (tval[]).  Keys (tkey[]) are 64-bit
// fingerprints of a characteristic matrix; 0 marks an empty slot.
constexpr uint32_t VAL_OPEN = 0x7FFFFFFFu;     // empty slot / group not yet elected
constexpr uint32_t VAL_SETTLED = 0x80000000u;  // tag: low 31 bits = global entry id
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;
constexpr uint32_t MAX_PROBES = 1u << 16;
constexpr int MAX_BLOCKS = 512;                // op x split blocks per level
constexpr int TILE = 4;                        // children per tile side

// One block of the canonical candidate order of a level: one connective and,
// for binary connectives, one split (a, b) of the remaining cost.
struct Block {
    uint32_t op;          // LTL_ATOM .. LTL_U
    uint32_t tri;         // AND/OR with a == b: pairs (i, j) with i < j of one level
    uint32_t na, nb;      // entries of the child levels (nb = 0 for unary)
    uint32_t cand_base;   // canonical index of the block's first candidate
    uint32_t ncand;       // candidates in the block
    uint32_t tile_base;   // first tile of the block in the level's tile list
    uint32_t ntile;       // tiles of the block
    uint32_t nti, ntj;    // tile grid (rows of a-tiles, columns of b-tiles)
    uint32_t a_gid, b_gid;   // global entry id of the first a / b entry (ATOM: prop 0)
    uint64_t a_ptr;       // ATOM: device address of the first atom matrix
    uint32_t st_base;     // LDS-staged binary blocks: first 8 x 8 group of tiles in the class list
    uint32_t nst;         // ... and the block's groups
    uint32_t fcb[4];      // OP_FUSED4 blocks: canonical base of F, G, X, NOT over the same children
    uint32_t ind;         // bit 0 / bit 1: a / b children are stored entries, found through store[]
    uint32_t pad;
};

// Evaluation-only block: F, G, X and NOT over the same child level in one tile
// (each child is read once for its four candidates).
constexpr uint32_t OP_FUSED4 = 16;

struct Counters {
    unsigned long long first_sol;   // smallest separating canonical index (atomicMin)
    uint32_t n_new;                 // new fingerprint groups claimed this level
    uint32_t overflow;              // hash table or list capacity exceeded
    uint32_t n_coll;                // candidates whose full compare failed
    uint32_t letter_or;             // OR of the letters that name a missing proposition (validation)
    uint32_t n_fallback_new;        // representatives added by the exact fallback
    uint32_t pad[9];
};

template <typename T>
struct Rows {
    const T *valid;          // valid position bits of each word
    const T *sepm;           // top bit for the first word of a live trace, else 0
    const T *sepw;           // expected value of that bit: set for P traces
    const uint64_t *nxt;     // lanes (in the row block) holding later words of the same trace
    const uint32_t *key;     // fingerprint keys (odd, 32-bit): 1 (W=32) or 2 (W=64) per row
    uint32_t R, NB;          // words per matrix, 64-word row blocks
    uint32_t ksteps;         // U doubling steps = ceil(log2(longest trace))
    uint32_t maxw;           // longest trace in words
};

template <typename T>
struct LevelArgs {
    Rows<T> rows;
    const Block *blocks;     // canonical order (for decoding a candidate index)
    uint32_t nblocks;
    unsigned long long *tkey;
    uint32_t *tval;
    uint32_t slot_mask;
    uint64_t fp_mask;
    Counters *ctr;
    uint32_t *cand_slot;     // per candidate: its hash slot (or NO_SLOT)
    uint32_t *new_slots;     // slots claimed this level, in claim order
    uint32_t *claimer;       // per claim: the candidate that claimed the slot (its matrix is stored)
    uint32_t *new_owner;     // owner (canonical index) of each claimed slot, recorded at settlement
    uint32_t new_cap;
    uint32_t *bitmap;        // per candidate: group representative bit
    uint32_t *wordpre;       // exclusive prefix of popcounts of bitmap words
    uint32_t *coll_bits;     // per candidate: full compare failed
    uint32_t *fb_bits;       // per candidate: representative found by the exact fallback
    T *arena;
    uint32_t level_base;     // global id of the level's first entry
    uint32_t *recipe;        // per global entry: canonical candidate index in its level
    uint32_t *store;         // per global entry: arena position of its matrix (claim order
                             // within the level: position level_base + claim number)
    uint32_t cw;             // the evaluation pass writes each claimer's matrix
    // Whole-row levels write the claimers' matrices in a pass of their own, after the
    // evaluation: if the level turns out not to be stored (a solution was found, or it
    // is the bound level), only the claimers whose group other candidates joined
    // (has_member) are written, for the verification to compare with.
    uint32_t *cand_claim;    // per candidate: its claim number, or 0xFFFFFFFF
    uint32_t *has_member;    // per claim: another candidate of the level joined its group
    uint32_t bound_level;    // the level is the cost bound (never stored)
    uint32_t verify_rep;     // verify against the representative (exact re-check) instead of
                             // against the claimer
    T *stage;                // R words of scratch for the fallback
    uint32_t arena_cap;      // new entries the arena can take this level
    int ucarry;
    uint32_t mat_chunk;            // row blocks per materialize work item
    // Row-split tiles spread over wg_split workgroups (long rows, few tiles): each
    // workgroup adds its partial fingerprint and separation flags per candidate;
    // k_probe claims the slots and k_materialize writes the claimers afterwards.
    uint32_t wg_split;
    unsigned long long *cand_fp;   // per candidate: sum of partial fingerprints
    uint32_t *cand_viol;           // per candidate: separation violated (bit)
    uint32_t *full;                // set once the level's claims pass abort_cap (own cache line)
    uint32_t abort_cap;            // claims after which the level is known to end out of memory
    // Relaxed uniqueness check: the evaluation writes each candidate's 126-bit key, a
    // claim pass caches the new keys, and the level's entries get their representative's
    // key and, in the write pass, its matrix.
    const uint32_t *ruc_meta;      // per row: per 32-bit half (top half first), the keyed sums'
                                   // odd keys (a, b), or in pack form (kept-position mask, key offset)
    unsigned long long *cand_key;  // per candidate: its key (2 words)
    unsigned long long *entry_key; // per global entry: its key
    uint32_t ruc_pack;             // keys in pack form (prefix bits) instead of keyed sums
    uint32_t ruc_bits;             // keep the first ruc_bits bits of each key (0: all 126)
    uint32_t ruc_fpb_off;          // row-split tiles over workgroups: second sums at cand_fp + this
};


template <typename T>
struct Launch {
    // cls: 0 unary, 1 and/or, 2 until (doubling), 3 until (carry adder)
    static hipError_t level(const LevelArgs<T> &A, bool mw, bool verify, int cls, const Block *blocks,
                            uint32_t nblocks, uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s);
    // whole-row binary classes with child operands staged in LDS: one workgroup of 4 waves
    // per 8 x 8 group of tiles (pass 0 evaluation, 1 verification, 2 write pass)
    static hipError_t level_staged(const LevelArgs<T> &A, bool mw, int pass, int cls, const Block *blocks,
                                   uint32_t nblocks, uint32_t ngroups, uint32_t chunk, uint32_t grid, hipStream_t s);
    // row-split levels, every connective class in one dispatch: evaluation with one
    // workgroup per tile (claims and claimers' matrices included) ...
    static hipError_t level_wg(const LevelArgs<T> &A, bool mw, const Block *blocks, uint32_t nblocks,
                               uint32_t ntiles, uint32_t grid, hipStream_t s, bool ruc = false);
    // relaxed check, row-split tiles spread over workgroups: added partial sums -> keys
    static hipError_t ruc_finish(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s);
    // relaxed check: evaluation writing each candidate's key (whole-row tiles, one class) ...
    static hipError_t level_ruc(const LevelArgs<T> &A, bool mw, int cls, const Block *blocks, uint32_t nblocks,
                                uint32_t ntiles, uint32_t grid, hipStream_t s);
    // ... the claims of new keys, and the keys of the level's entries after the compaction
    static hipError_t ruc_claim(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s);
    static hipError_t ruc_entry_keys(const LevelArgs<T> &A, hipStream_t s);
    // claims for tiles spread over several workgroups (A.wg_split > 1)
    static hipError_t probe(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s);
    // whole-row levels: groups joined by other candidates, then the write pass per class
    static hipError_t mark_members(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s);
    static hipError_t write_pass(const LevelArgs<T> &A, bool mw, int cls, const Block *blocks, uint32_t nblocks,
                                 uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s);
    static constexpr uint32_t waves_per_wg(bool mw) { return mw ? 4u : 8u; }
    // ... and verification with one wave per (tile, row chunk)
    static hipError_t verify_all(const LevelArgs<T> &A, bool mw, const Block *blocks, uint32_t nblocks,
                                 uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s);
    // rep_mode 0: claim order, matrix of each claimer at level_base + claim number;
    // rep_mode 1: matrix of each entry's representative at store[entry]
    static hipError_t materialize(const LevelArgs<T> &A, bool mw, uint32_t rep_mode, uint32_t grid, hipStream_t s);
    static hipError_t fallback(const LevelArgs<T> &A, bool mw, uint32_t nwords, uint32_t ncand, hipStream_t s);
    static hipError_t pack(const uint32_t *letters, const uint64_t *offsets, const uint32_t *row_trace,
                           const uint32_t *row_word, uint32_t R, uint32_t nprops, T *atoms, Counters *ctr,
                           hipStream_t s);
    // formula evaluation: one node's matrix from its children's (op NOT .. U)
    static hipError_t formula_node(const Rows<T> &rw, bool mw, int op, const T *pa, const T *pb, T *dst,
                                   hipStream_t s);
    // position 0 of every trace of a matrix, one byte per trace
    static hipError_t first_bits(const T *cm, const uint32_t *row_trace, const uint32_t *row_word, uint32_t R,
                                 uint8_t *out, hipStream_t s);
};

hipError_t launch_scan(const uint32_t *bits, uint32_t nw, uint32_t *chunk_sums, uint32_t *wordpre, hipStream_t s);
hipError_t launch_mark(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, const uint32_t *tval,
                       uint32_t *bitmap, uint32_t grid, hipStream_t s);
hipError_t launch_or_bits(uint32_t *dst, const uint32_t *src, uint32_t nw, hipStream_t s);
// mark + scan + scatter in one workgroup, for levels with at most SMALL_COMPACT_WORDS bitmap words
constexpr uint32_t SMALL_COMPACT_WORDS = 128;
hipError_t launch_compact_small(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, uint32_t *tval,
                                uint32_t *bitmap, uint32_t nw, uint32_t *wordpre, uint32_t *recipe,
                                uint32_t level_base, uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store,
                                hipStream_t s);
// recipes + slot settlement (+ entry -> slot); repass re-reads the recorded owners
hipError_t launch_scatter(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, uint32_t *tval,
                          const uint32_t *bitmap, const uint32_t *wordpre, uint32_t *recipe, uint32_t level_base,
                          uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store, bool repass, uint32_t grid,
                          hipStream_t s);
// zero words [0, na) of a and [0, nb) of b (either may be null) in one kernel
hipError_t launch_zero2(uint32_t *a, uint64_t na, uint32_t *b, uint64_t nb, hipStream_t s);
hipError_t launch_clear_slots(const uint32_t *entry_slot, uint32_t n, unsigned long long *tkey, uint32_t *tval,
                              hipStream_t s);
hipError_t launch_table_init(unsigned long long *tkey, uint32_t *tval, uint64_t nslots, hipStream_t s);
hipError_t launch_trace_fp(const uint32_t *letters, const uint64_t *offsets, uint32_t ntr, uint64_t *out,
                           hipStream_t s);
constexpr uint32_t SCAN_CHUNK_WORDS = 2048;   // bitmap words per scan block

}  // namespace ltl
