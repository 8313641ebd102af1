/*
 * ltl_oracle.c -- CPU oracle for the enumerative LTL learner.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU path (paper_2402_12373_amd/csrc).
 *
 * What it computes (paper "LTL learning on GPUs", arXiv 2402.12373):
 *   - finite-trace LTL satisfaction, by the textbook clauses of Sec. 2
 *     ("Formal preliminaries"): X, F, U clauses as given there, G as
 *     "for all later positions", and tr,i |= phi is false whenever i >= |tr|;
 *   - the characteristic sequence / matrix of a formula (Sec. 4): one truth
 *     value per (trace, position) over the fixed trace order P then N;
 *   - the bottom-up, cost-ordered enumeration of Sec. 3 (enum / handleOp /
 *     relaxedCheckAndCache), with the relaxed uniqueness check replaced by an
 *     exact one: a candidate is cached iff its whole characteristic matrix is
 *     not yet in the language cache (the exhaustive case of Sec. 5);
 *   - the separation predicate (dagger) of Sec. 4: every positive trace
 *     satisfies phi at position 0 and no negative trace does;
 *   - optionally the relaxed uniqueness check of Sec. 5 itself: a candidate is
 *     cached iff its 126-bit key is new, the key being the matrix itself when it
 *     has at most 126 bits, else a keyed hash of it (our stand-in for the hash the
 *     paper names) or the first-k-percent map (FKP) of Sec. 7 (oracle_run_relaxed).
 *
 * Two evaluation modes for the temporal operators, cross-checked by tests:
 *   MODE_QUANT  : the clauses literally (O(n^2) per trace for F, G, U);
 *   MODE_EXPAND : backward expansion laws  F p = p | X F p,  G p = p & (end | X G p),
 *                 p U q = q | (p & X(p U q))  (Sec. 4's disjunction reading).
 *
 * Canonical enumeration order (binding on both implementations):
 *   for op in (F, U, G, X, AND, OR, NOT) restricted to the operator set   [Sec. 3 listing]
 *     x = c - cost(op)
 *     unary  : for e in level x                    -> op(L_x[e])
 *     U      : for a = 1.. (b = x-a):  for i in L_a: for j in L_b   -> L_a[i] U L_b[j]
 *     AND/OR : for a = 1.. with a <= b = x-a:
 *                a <  b : for i in L_a: for j in L_b            -> L_a[i] op L_b[j]
 *                a == b : for i in L_a: for j > i in L_a        -> L_a[i] op L_a[j]
 *   A level's entries are kept in order of first occurrence.  The first solution is
 *   the separating candidate of smallest canonical index at the minimal cost; the
 *   whole level is evaluated (its new-language count is reported in full).
 *
 * Parity pins: see tests/test_oracle_*.py (paper worked examples of Sec. 4 and
 * App. A, exhaustive brute force over syntax trees, identities).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O_ATOM = 0, O_NOT = 1, O_AND = 2, O_OR = 3, O_X = 4, O_F = 5, O_G = 6, O_U = 7 };
#define O_NNF (1u << 8)   /* op_mask flag: negation of atoms only */
enum { MODE_QUANT = 0, MODE_EXPAND = 1 };
enum { ST_OK = 0, ST_NOT_FOUND = 1, ST_EINVAL = -1, ST_EOOM = -4, ST_EINCONS = -2 };

typedef struct {
    int32_t num_props;
    int32_t num_pos;
    int32_t num_neg;
    int32_t pad_;
    const uint32_t *letters;   /* all letters, P traces then N traces */
    const uint64_t *offsets;   /* num_pos+num_neg+1 */
} o_spec;

typedef struct { int32_t op, a, b; } o_node;   /* postfix; ATOM: a = proposition */

/* ------------------------------------------------------------------------ */
/* Textbook satisfaction (Sec. 2).                                          */
/* ------------------------------------------------------------------------ */

static int64_t trace_len(const o_spec *s, int t) {
    return (int64_t)(s->offsets[t + 1] - s->offsets[t]);
}

static int holds_node(const o_spec *s, int t, int64_t i, const o_node *f, int k) {
    int64_t len = trace_len(s, t);
    if (i >= len) return 0;                 /* out of range: always false */
    switch (f[k].op) {
    case O_ATOM: return (int)((s->letters[s->offsets[t] + i] >> f[k].a) & 1u);
    case O_NOT:  return !holds_node(s, t, i, f, f[k].a);
    case O_AND:  return holds_node(s, t, i, f, f[k].a) && holds_node(s, t, i, f, f[k].b);
    case O_OR:   return holds_node(s, t, i, f, f[k].a) || holds_node(s, t, i, f, f[k].b);
    case O_X:    return holds_node(s, t, i + 1, f, f[k].a);
    case O_F:
        for (int64_t j = i; j < len; ++j)
            if (holds_node(s, t, j, f, f[k].a)) return 1;
        return 0;
    case O_G:
        for (int64_t j = i; j < len; ++j)
            if (!holds_node(s, t, j, f, f[k].a)) return 0;
        return 1;
    case O_U:
        for (int64_t j = i; j < len; ++j) {
            if (!holds_node(s, t, j, f, f[k].b)) continue;
            int ok = 1;
            for (int64_t m = i; m < j && ok; ++m)
                if (!holds_node(s, t, m, f, f[k].a)) ok = 0;
            if (ok) return 1;
        }
        return 0;
    }
    return 0;
}

int oracle_holds(const o_spec *s, int t, int64_t i, const o_node *f, int n) {
    if (!s || !f || n <= 0) return -1;
    return holds_node(s, t, i, f, n - 1);
}

/* ------------------------------------------------------------------------ */
/* Characteristic matrices: one byte per (trace, position), trace-major in   */
/* the fixed order P then N (Sec. 4).                                       */
/* ------------------------------------------------------------------------ */

static int64_t total_positions(const o_spec *s) {
    return (int64_t)s->offsets[s->num_pos + s->num_neg];
}

static void cm_atom(const o_spec *s, int p, uint8_t *out) {
    int64_t tb = total_positions(s);
    for (int64_t q = 0; q < tb; ++q) out[q] = (uint8_t)((s->letters[q] >> p) & 1u);
}

/* Apply one connective to children matrices a (and b), position by position. */
static void cm_apply(const o_spec *s, int op, const uint8_t *a, const uint8_t *b, int mode, uint8_t *out) {
    int T = s->num_pos + s->num_neg;
    for (int t = 0; t < T; ++t) {
        int64_t o = (int64_t)s->offsets[t];
        int64_t len = trace_len(s, t);
        const uint8_t *A = a + o;
        const uint8_t *B = b ? b + o : NULL;
        uint8_t *R = out + o;
        switch (op) {
        case O_NOT: for (int64_t i = 0; i < len; ++i) R[i] = !A[i]; break;
        case O_AND: for (int64_t i = 0; i < len; ++i) R[i] = A[i] && B[i]; break;
        case O_OR:  for (int64_t i = 0; i < len; ++i) R[i] = A[i] || B[i]; break;
        case O_X:   for (int64_t i = 0; i < len; ++i) R[i] = (i + 1 < len) ? A[i + 1] : 0; break;
        case O_F:
            if (mode == MODE_QUANT) {
                for (int64_t i = 0; i < len; ++i) {
                    int v = 0;
                    for (int64_t j = i; j < len; ++j) if (A[j]) { v = 1; break; }
                    R[i] = (uint8_t)v;
                }
            } else {
                int nxt = 0;                                   /* F at |tr| is false */
                for (int64_t i = len - 1; i >= 0; --i) { nxt = A[i] || nxt; R[i] = (uint8_t)nxt; }
            }
            break;
        case O_G:
            if (mode == MODE_QUANT) {
                for (int64_t i = 0; i < len; ++i) {
                    int v = 1;
                    for (int64_t j = i; j < len; ++j) if (!A[j]) { v = 0; break; }
                    R[i] = (uint8_t)v;
                }
            } else {
                int nxt = 1;                /* base: nothing left to violate G past the end */
                for (int64_t i = len - 1; i >= 0; --i) { nxt = A[i] && nxt; R[i] = (uint8_t)nxt; }
            }
            break;
        case O_U:
            if (mode == MODE_QUANT) {
                for (int64_t i = 0; i < len; ++i) {
                    int v = 0;
                    for (int64_t j = i; j < len && !v; ++j) {
                        if (!B[j]) continue;
                        int ok = 1;
                        for (int64_t m = i; m < j; ++m) if (!A[m]) { ok = 0; break; }
                        if (ok) v = 1;
                    }
                    R[i] = (uint8_t)v;
                }
            } else {
                int nxt = 0;                                   /* U at |tr| is false */
                for (int64_t i = len - 1; i >= 0; --i) { nxt = B[i] || (A[i] && nxt); R[i] = (uint8_t)nxt; }
            }
            break;
        default: break;
        }
    }
}

int oracle_apply(const o_spec *s, int op, const uint8_t *a, const uint8_t *b, int mode, uint8_t *out) {
    if (!s || !a || !out || op <= O_ATOM || op > O_U) return -1;
    if ((op == O_AND || op == O_OR || op == O_U) && !b) return -1;
    cm_apply(s, op, a, b, mode, out);
    return 0;
}

/* Matrix of a whole formula, bottom-up over its postfix nodes. */
int oracle_eval_formula(const o_spec *s, const o_node *f, int n, int mode, uint8_t *out) {
    if (!s || !f || n <= 0 || !out) return -1;
    int64_t tb = total_positions(s);
    uint8_t *buf = (uint8_t *)malloc((size_t)tb * (size_t)n);
    if (!buf) return -1;
    for (int k = 0; k < n; ++k) {
        uint8_t *dst = buf + (size_t)k * tb;
        if (f[k].op == O_ATOM) cm_atom(s, f[k].a, dst);
        else cm_apply(s, f[k].op, buf + (size_t)f[k].a * tb,
                      (f[k].op == O_AND || f[k].op == O_OR || f[k].op == O_U) ? buf + (size_t)f[k].b * tb : NULL,
                      mode, dst);
    }
    memcpy(out, buf + (size_t)(n - 1) * tb, (size_t)tb);
    free(buf);
    return 0;
}

/* Separation predicate (dagger), Sec. 4: truth at position 0 of every trace. */
static int separates(const o_spec *s, const uint8_t *cm) {
    int T = s->num_pos + s->num_neg;
    for (int t = 0; t < T; ++t) {
        int v = cm[s->offsets[t]];
        if (t < s->num_pos ? !v : v) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Language cache: levels of distinct matrices, stored one bit per position */
/* (packing is for storage and comparison only), with an exact hash map.     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t op;          /* connective that produced the entry (ATOM for level cost(ATOM)) */
    int32_t la, lb;      /* child levels (-1 if none) */
    int64_t ia, ib;      /* child indices within those levels; ATOM: ia = proposition */
} o_recipe;

typedef struct {
    int64_t n, cap;
    uint8_t *bits;       /* n * pbytes */
    o_recipe *rec;
} o_level;

typedef struct {
    uint64_t *h;         /* stored hash per slot (0 = empty) */
    int32_t *lev;
    int64_t *idx;
    uint64_t *key;       /* relaxed mode: the entry's 126-bit key (2 words per slot) */
    int64_t cap, n;
} o_map;

struct o_run {
    o_spec spec;
    int32_t cost[8];
    uint32_t op_mask;
    int bound, mode, threads;
    int64_t tb, pbytes;
    o_level *L;          /* L[0..bound] */
    o_map map;
    int status, found_cost, levels_done;
    int64_t *E, *C;      /* per level: new languages, candidates */
    double *secs;        /* per level wall time */
    int64_t first;       /* canonical index of first solution (-1 none) */
    o_recipe sol;        /* the solution candidate */
    int ruc;             /* RUC_NONE (exact), RUC_HASH, RUC_FKP */
    uint64_t ruc_seed;   /* RUC_HASH: SplitMix64 seed of the per-chunk keys */
    int ruc_bits;        /* keep the first ruc_bits bits of each key (1..125); 0 = all 126 */
    int64_t *ruc_m;      /* per trace: positions that enter the packed key (pack form) */
    int ruc_pack;        /* key = packed prefix bits (FKP, or any matrix of <= 126 bits) */
};
typedef struct o_run o_run;

static uint64_t fnv1a(const uint8_t *p, int64_t n) {
    /* Fowler-Noll-Vo FNV-1a, 64-bit */
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ull; }
    return h ? h : 1;
}

/* ------------------------------------------------------------------------ */
/* Relaxed uniqueness check (Sec. 5): 126-bit keys.                          */
/*                                                                           */
/* The key is a string of 126 bits, held in two words (bit 0 of the string = */
/* the top bit of the first word; the last two bits of the second word are   */
/* zero).                                                                    */
/*  - Pack form: the characteristic sequences' first m_t positions, trace by  */
/*    trace in the order P then N, cut after 126 bits and padded with zeros.  */
/*    A matrix of at most 126 bits is its own key (m_t = |tr_t|): the check   */
/*    is then exact.  FKP (Sec. 7) keeps the first k percent of each sequence */
/*    (m_t = |tr_t| k / 100 rounded half up), k in 1..100 the smallest whose  */
/*    total is nearest to 126 bits.                                          */
/*  - Hash form (RUC_HASH on a matrix of more than 126 bits): two keyed sums  */
/*    over 32-position chunks, chunk j of trace t holding positions          */
/*    32j .. 32j+31 (position 32j in the top bit, zeros past the end):        */
/*        A = sum premix(v, a) * a,  B = sum premix(v, b) * b   (mod 2^64)    */
/*    with premix(v, k) = y ^ (y >> 16), y = (v ^ (v >> 8)) + k (mod 2^32),   */
/*    and the odd 32-bit keys a, b = top halves of draws 2i and 2i + 1 of the */
/*    SplitMix64 sequence (Steele, Lea, Flood, OOPSLA 2014) of the seed, with */
/*    i = t * 2^32 + j, low bit set.  The string is A's top 63 bits, then B's. */
/* ------------------------------------------------------------------------ */
enum { RUC_NONE = 0, RUC_HASH = 1, RUC_FKP = 2 };
#define RUC_KEY_BITS 126

static uint64_t splitmix64_draw(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint32_t ruc_premix(uint32_t v, uint32_t k) {
    uint32_t y = (v ^ (v >> 8)) + k;
    return y ^ (y >> 16);
}

/* FKP's k for the traces of s (0 if the whole matrix fits 126 bits); fills m[t]. */
static int ruc_prefixes(const o_spec *s, int kind, int64_t *m) {
    int T = s->num_pos + s->num_neg;
    if (total_positions(s) <= RUC_KEY_BITS || kind != RUC_FKP) {
        for (int t = 0; t < T; ++t) m[t] = trace_len(s, t);
        return 0;
    }
    int best = 1;
    int64_t best_d = -1;
    for (int k = 1; k <= 100; ++k) {
        int64_t tot = 0;
        for (int t = 0; t < T; ++t) tot += (trace_len(s, t) * k + 50) / 100;
        int64_t d = tot > RUC_KEY_BITS ? tot - RUC_KEY_BITS : RUC_KEY_BITS - tot;
        if (best_d < 0 || d < best_d) { best_d = d; best = k; }
    }
    for (int t = 0; t < T; ++t) m[t] = (trace_len(s, t) * best + 50) / 100;
    return best;
}

static void ruc_key_of(const o_spec *s, int pack, const int64_t *m, uint64_t seed, int bits, const uint8_t *cm,
                       uint64_t key[2]) {
    int T = s->num_pos + s->num_neg;
    uint64_t k0 = 0, k1 = 0;
    if (pack) {
        int64_t q = 0;
        for (int t = 0; t < T && q < RUC_KEY_BITS; ++t) {
            const uint8_t *row = cm + s->offsets[t];
            for (int64_t i = 0; i < m[t] && q < RUC_KEY_BITS; ++i, ++q) {
                if (!row[i]) continue;
                if (q < 64) k0 |= 1ull << (63 - q);
                else k1 |= 1ull << (63 - (q - 64));
            }
        }
    } else {
        uint64_t A = 0, B = 0;
        for (int t = 0; t < T; ++t) {
            const uint8_t *row = cm + s->offsets[t];
            int64_t n = trace_len(s, t);
            for (int64_t j = 0; 32 * j < n; ++j) {
                uint32_t v = 0;
                for (int i = 0; i < 32 && 32 * j + i < n; ++i)
                    if (row[32 * j + i]) v |= 1u << (31 - i);
                uint64_t ci = ((uint64_t)t << 32) | (uint64_t)j;
                uint32_t a = (uint32_t)(splitmix64_draw(seed, 2 * ci) >> 32) | 1u;
                uint32_t b = (uint32_t)(splitmix64_draw(seed, 2 * ci + 1) >> 32) | 1u;
                A += (uint64_t)ruc_premix(v, a) * a;
                B += (uint64_t)ruc_premix(v, b) * b;
            }
        }
        k0 = (A & ~1ull) | (B >> 63);
        k1 = (B << 1) & ~3ull;
    }
    if (bits > 0 && bits < RUC_KEY_BITS) {
        if (bits <= 64) { k0 &= bits == 64 ? ~0ull : ~(~0ull >> bits); k1 = 0; }
        else k1 &= ~(~0ull >> (bits - 64));
    }
    key[0] = k0;
    key[1] = k1;
}

/* Test hooks: the key of one matrix, and FKP's k. */
int oracle_ruc_key(const o_spec *s, const uint8_t *cm, int kind, uint64_t seed, int bits, uint64_t *out) {
    if (!s || !cm || !out || (kind != RUC_HASH && kind != RUC_FKP)) return -1;
    int T = s->num_pos + s->num_neg;
    int64_t *m = (int64_t *)malloc((size_t)(T > 0 ? T : 1) * sizeof(int64_t));
    if (!m) return -1;
    ruc_prefixes(s, kind, m);
    int pack = kind == RUC_FKP || total_positions(s) <= RUC_KEY_BITS;
    ruc_key_of(s, pack, m, seed, bits, cm, out);
    free(m);
    return 0;
}

int oracle_fkp_k(const o_spec *s, int64_t *m_out) {
    if (!s) return -1;
    int T = s->num_pos + s->num_neg;
    int64_t *m = (int64_t *)malloc((size_t)(T > 0 ? T : 1) * sizeof(int64_t));
    if (!m) return -1;
    int k = ruc_prefixes(s, RUC_FKP, m);
    if (m_out) memcpy(m_out, m, (size_t)T * sizeof(int64_t));
    free(m);
    return k;
}

static uint64_t key_hash(const uint64_t key[2]) {
    return fnv1a((const uint8_t *)key, 16);
}

static void pack_bits(const uint8_t *cm, int64_t tb, uint8_t *dst, int64_t pbytes) {
    memset(dst, 0, (size_t)pbytes);
    for (int64_t q = 0; q < tb; ++q) if (cm[q]) dst[q >> 3] |= (uint8_t)(1u << (q & 7));
}

static void unpack_bits(const uint8_t *src, int64_t tb, uint8_t *cm) {
    for (int64_t q = 0; q < tb; ++q) cm[q] = (uint8_t)((src[q >> 3] >> (q & 7)) & 1u);
}

static const uint8_t *entry_bits(o_run *r, int lev, int64_t i) {
    return r->L[lev].bits + (size_t)i * (size_t)r->pbytes;
}

static int map_grow(o_run *r) {
    o_map *m = &r->map;
    int64_t ncap = m->cap ? m->cap * 2 : 1024;
    uint64_t *h = (uint64_t *)calloc((size_t)ncap, sizeof(uint64_t));
    int32_t *lev = (int32_t *)malloc((size_t)ncap * sizeof(int32_t));
    int64_t *idx = (int64_t *)malloc((size_t)ncap * sizeof(int64_t));
    uint64_t *key = (uint64_t *)malloc((size_t)ncap * 2 * sizeof(uint64_t));
    if (!h || !lev || !idx || !key) { free(h); free(lev); free(idx); free(key); return -1; }
    for (int64_t k = 0; k < m->cap; ++k) {
        if (!m->h[k]) continue;
        int64_t pos = (int64_t)(m->h[k] & (uint64_t)(ncap - 1));
        while (h[pos]) pos = (pos + 1) & (ncap - 1);
        h[pos] = m->h[k]; lev[pos] = m->lev[k]; idx[pos] = m->idx[k];
        key[2 * pos] = m->key[2 * k]; key[2 * pos + 1] = m->key[2 * k + 1];
    }
    free(m->h); free(m->lev); free(m->idx); free(m->key);
    m->h = h; m->lev = lev; m->idx = idx; m->key = key; m->cap = ncap;
    return 0;
}

/* Returns 1 if the language is already cached, else 0: exact mode compares the
 * matrices `bits`, relaxed mode the 126-bit keys `key` (hash hv of either). */
static int map_contains(o_run *r, const uint8_t *bits, const uint64_t *key, uint64_t hv) {
    o_map *m = &r->map;
    if (!m->cap) return 0;
    int64_t pos = (int64_t)(hv & (uint64_t)(m->cap - 1));
    while (m->h[pos]) {
        if (m->h[pos] == hv) {
            if (r->ruc ? (m->key[2 * pos] == key[0] && m->key[2 * pos + 1] == key[1])
                       : memcmp(entry_bits(r, m->lev[pos], m->idx[pos]), bits, (size_t)r->pbytes) == 0)
                return 1;
        }
        pos = (pos + 1) & (m->cap - 1);
    }
    return 0;
}

static int map_insert(o_run *r, uint64_t hv, const uint64_t *key, int lev, int64_t idx) {
    o_map *m = &r->map;
    if ((m->n + 1) * 2 > m->cap && map_grow(r)) return -1;
    int64_t pos = (int64_t)(hv & (uint64_t)(m->cap - 1));
    while (m->h[pos]) pos = (pos + 1) & (m->cap - 1);
    m->h[pos] = hv; m->lev[pos] = lev; m->idx[pos] = idx;
    m->key[2 * pos] = key ? key[0] : 0; m->key[2 * pos + 1] = key ? key[1] : 0;
    m->n++;
    return 0;
}

static int level_push(o_run *r, int lev, const uint8_t *bits, o_recipe rc) {
    o_level *L = &r->L[lev];
    if (L->n == L->cap) {
        int64_t nc = L->cap ? L->cap * 2 : 64;
        uint8_t *nb = (uint8_t *)realloc(L->bits, (size_t)nc * (size_t)r->pbytes);
        if (!nb) return -1;
        L->bits = nb;
        o_recipe *nr = (o_recipe *)realloc(L->rec, (size_t)nc * sizeof(o_recipe));
        if (!nr) return -1;
        L->rec = nr;
        L->cap = nc;
    }
    memcpy(L->bits + (size_t)L->n * (size_t)r->pbytes, bits, (size_t)r->pbytes);
    L->rec[L->n] = rc;
    L->n++;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Candidate batches: candidates are generated in canonical order, their      */
/* matrices computed (possibly in parallel), then merged strictly in order.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    o_run *r;
    int level;
    int64_t cap, n;
    o_recipe *rc;
    uint8_t *cm;        /* n * tb scratch (unpacked result) */
    uint8_t *ca, *cb;   /* per-thread child scratch: threads * tb */
    uint8_t *pk;        /* n * pbytes */
    uint64_t *hv;
    uint64_t *key;      /* relaxed mode: n * 2 words */
    uint8_t *sep;
    int64_t next_index; /* canonical index of rc[0] */
    int64_t first;      /* -1 none */
    int err;
} o_batch;

static void batch_flush(o_batch *B) {
    o_run *r = B->r;
    int64_t tb = r->tb;
    int64_t n = B->n;
    if (n == 0) return;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(r->threads)
#endif
    for (int64_t k = 0; k < n; ++k) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint8_t *ca = B->ca + (size_t)tid * tb;
        uint8_t *cb = B->cb + (size_t)tid * tb;
        o_recipe rc = B->rc[k];
        uint8_t *out = B->cm + (size_t)k * tb;
        unpack_bits(entry_bits(r, rc.la, rc.ia), tb, ca);
        if (rc.lb >= 0) unpack_bits(entry_bits(r, rc.lb, rc.ib), tb, cb);
        cm_apply(&r->spec, rc.op, ca, rc.lb >= 0 ? cb : NULL, r->mode, out);
        B->sep[k] = (uint8_t)separates(&r->spec, out);
        pack_bits(out, tb, B->pk + (size_t)k * r->pbytes, r->pbytes);
        if (r->ruc) {
            ruc_key_of(&r->spec, r->ruc_pack, r->ruc_m, r->ruc_seed, r->ruc_bits, out, B->key + 2 * k);
            B->hv[k] = key_hash(B->key + 2 * k);
        } else {
            B->hv[k] = fnv1a(B->pk + (size_t)k * r->pbytes, r->pbytes);
        }
    }
    /* sequential merge in canonical order */
    for (int64_t k = 0; k < n && !B->err; ++k) {
        int64_t ci = B->next_index + k;
        if (B->sep[k] && B->first < 0) { B->first = ci; r->sol = B->rc[k]; }
        const uint8_t *pk = B->pk + (size_t)k * r->pbytes;
        const uint64_t *key = B->key + 2 * k;
        if (!map_contains(r, pk, key, B->hv[k])) {
            if (level_push(r, B->level, pk, B->rc[k]) ||
                map_insert(r, B->hv[k], key, B->level, r->L[B->level].n - 1))
                B->err = 1;
        }
    }
    B->next_index += n;
    B->n = 0;
}

static void batch_emit(o_batch *B, int op, int la, int64_t ia, int lb, int64_t ib) {
    o_recipe rc = { op, la, lb, ia, ib };
    B->rc[B->n++] = rc;
    if (B->n == B->cap) batch_flush(B);
}

static int level_exists(o_run *r, int c) { return c >= 1 && c <= r->bound && r->L[c].n > 0; }

/* One cost level in canonical order. */
static int run_level(o_run *r, int c, o_batch *B) {
    static const int order[7] = { O_F, O_U, O_G, O_X, O_AND, O_OR, O_NOT };
    B->level = c; B->n = 0; B->next_index = 0; B->first = -1; B->err = 0;
    for (int oi = 0; oi < 7; ++oi) {
        int op = order[oi];
        if (!(r->op_mask & (1u << op))) continue;
        int x = c - r->cost[op];
        if (x < 1) continue;
        /* negation normal form (op_mask bit 8, the U-free NNF formulae of Sec. 7):
         * negation of atoms only, i.e. of the entries of the atom level */
        if (op == O_NOT && (r->op_mask & O_NNF) && x != r->cost[O_ATOM]) continue;
        if (op == O_NOT || op == O_X || op == O_F || op == O_G) {
            if (!level_exists(r, x)) continue;
            for (int64_t e = 0; e < r->L[x].n; ++e) batch_emit(B, op, x, e, -1, 0);
        } else if (op == O_U) {
            for (int a = 1; a < x; ++a) {
                int b = x - a;
                if (!level_exists(r, a) || !level_exists(r, b)) continue;
                for (int64_t i = 0; i < r->L[a].n; ++i)
                    for (int64_t j = 0; j < r->L[b].n; ++j) batch_emit(B, op, a, i, b, j);
            }
        } else {   /* AND, OR: commutative, a <= b, and i < j on the diagonal */
            for (int a = 1; a <= x - a; ++a) {
                int b = x - a;
                if (!level_exists(r, a) || !level_exists(r, b)) continue;
                if (a < b) {
                    for (int64_t i = 0; i < r->L[a].n; ++i)
                        for (int64_t j = 0; j < r->L[b].n; ++j) batch_emit(B, op, a, i, b, j);
                } else {
                    for (int64_t i = 0; i < r->L[a].n; ++i)
                        for (int64_t j = i + 1; j < r->L[a].n; ++j) batch_emit(B, op, a, i, a, j);
                }
            }
        }
    }
    batch_flush(B);
    r->C[c] = B->next_index;
    r->E[c] = r->L[c].n;
    return B->err ? -1 : 0;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Runs the learner.  cost[ATOM..U] >= 1; op_mask bit k enables connective k
 * (bit 8, O_NNF: negation of atoms only)
 * (ATOM must be enabled).  bound is inclusive.  max_entries caps the number of
 * stored entries (0 = none); a level must be stored iff it has no solution and
 * it is below the bound; if storing it would exceed the cap, the run stops with
 * ST_EOOM at that level (its counts are still reported).
 * ruc: RUC_NONE for the exact check, else the relaxed check of Sec. 5 with the
 * key form RUC_HASH (seed ruc_seed) or RUC_FKP; ruc_bits > 0 keeps only the
 * first ruc_bits bits of every key.  The entry kept for a key is the
 * canonical-first candidate that has it; new-language counts count new keys.
 */
o_run *oracle_run_relaxed(const o_spec *s, const int32_t *cost, uint32_t op_mask, int bound, int mode,
                          int threads, int64_t max_entries, int ruc, uint64_t ruc_seed, int ruc_bits) {
    o_run *r = (o_run *)calloc(1, sizeof(o_run));
    if (!r) return NULL;
    r->spec = *s;
    r->ruc = ruc; r->ruc_seed = ruc_seed; r->ruc_bits = ruc_bits;
    memcpy(r->cost, cost, sizeof(r->cost));
    r->op_mask = op_mask; r->bound = bound; r->mode = mode;
    r->threads = threads > 0 ? threads : 1;
    r->first = -1; r->found_cost = -1; r->levels_done = 0;
    r->status = ST_EINVAL;
    int T = s->num_pos + s->num_neg;
    if (bound < 1 || s->num_props < 1 || s->num_props > 32 || T < 1 || !(op_mask & 1u) ||
        (op_mask & ~(0xFFu | O_NNF))) return r;
    for (int k = 0; k < 8; ++k) if ((op_mask & (1u << k)) && cost[k] < 1) return r;
    for (int t = 0; t < T; ++t) if (trace_len(s, t) < 1) return r;
    for (int64_t q = 0; q < total_positions(s); ++q)
        if (s->num_props < 32 && (s->letters[q] >> s->num_props)) return r;
    /* a trace in both classes makes the specification inconsistent (P and N disjoint) */
    for (int i = 0; i < s->num_pos; ++i)
        for (int j = s->num_pos; j < T; ++j) {
            if (trace_len(s, i) != trace_len(s, j)) continue;
            if (!memcmp(s->letters + s->offsets[i], s->letters + s->offsets[j],
                        (size_t)trace_len(s, i) * sizeof(uint32_t))) { r->status = ST_EINCONS; return r; }
        }
    if (ruc < RUC_NONE || ruc > RUC_FKP || ruc_bits < 0) return r;
    r->tb = total_positions(s);
    r->pbytes = (r->tb + 7) / 8;
    if (ruc) {
        r->ruc_m = (int64_t *)malloc((size_t)T * sizeof(int64_t));
        if (!r->ruc_m) return r;
        ruc_prefixes(s, ruc, r->ruc_m);
        r->ruc_pack = ruc == RUC_FKP || r->tb <= RUC_KEY_BITS;
    }
    r->L = (o_level *)calloc((size_t)bound + 1, sizeof(o_level));
    r->E = (int64_t *)calloc((size_t)bound + 1, sizeof(int64_t));
    r->C = (int64_t *)calloc((size_t)bound + 1, sizeof(int64_t));
    r->secs = (double *)calloc((size_t)bound + 1, sizeof(double));
    if (!r->L || !r->E || !r->C || !r->secs) return r;

    o_batch B;
    memset(&B, 0, sizeof(B));
    B.r = r;
    int64_t cap = (64ll << 20) / (r->tb > 0 ? r->tb : 1);
    if (cap < 1) cap = 1;
    if (cap > 65536) cap = 65536;
    B.cap = cap;
    B.rc = (o_recipe *)malloc((size_t)cap * sizeof(o_recipe));
    B.cm = (uint8_t *)malloc((size_t)cap * (size_t)r->tb);
    B.ca = (uint8_t *)malloc((size_t)r->threads * (size_t)r->tb);
    B.cb = (uint8_t *)malloc((size_t)r->threads * (size_t)r->tb);
    B.pk = (uint8_t *)malloc((size_t)cap * (size_t)r->pbytes);
    B.hv = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
    B.key = (uint64_t *)calloc((size_t)cap * 2, sizeof(uint64_t));
    B.sep = (uint8_t *)malloc((size_t)cap);
    uint8_t *tmp = (uint8_t *)malloc((size_t)r->tb);
    uint8_t *pk = (uint8_t *)malloc((size_t)r->pbytes);
    int64_t stored = 0;
    uint64_t akey[2] = {0, 0};
    if (!B.rc || !B.cm || !B.ca || !B.cb || !B.pk || !B.hv || !B.key || !B.sep || !tmp || !pk) goto fail;

    /* Atom level (Sec. 3 listing: atom check, then the cache starts with the atoms). */
    {
        int c0 = cost[O_ATOM];
        double t0 = now_s();
        if (c0 > bound) { r->status = ST_NOT_FOUND; goto done; }
        for (int p = 0; p < s->num_props; ++p) {
            cm_atom(s, p, tmp);
            if (separates(s, tmp) && r->first < 0) {
                r->first = p;
                r->sol.op = O_ATOM; r->sol.la = -1; r->sol.lb = -1; r->sol.ia = p; r->sol.ib = 0;
            }
            pack_bits(tmp, r->tb, pk, r->pbytes);
            uint64_t hv;
            if (r->ruc) {
                ruc_key_of(s, r->ruc_pack, r->ruc_m, r->ruc_seed, r->ruc_bits, tmp, akey);
                hv = key_hash(akey);
            } else {
                hv = fnv1a(pk, r->pbytes);
            }
            if (!map_contains(r, pk, akey, hv)) {
                o_recipe rc = { O_ATOM, -1, -1, p, 0 };
                if (level_push(r, c0, pk, rc) || map_insert(r, hv, akey, c0, r->L[c0].n - 1)) goto fail;
            }
        }
        r->C[c0] = s->num_props;
        r->E[c0] = r->L[c0].n;
        r->secs[c0] = now_s() - t0;
        r->levels_done = c0;
        if (r->first >= 0) { r->found_cost = c0; r->status = ST_OK; goto done; }
        stored += r->E[c0];
        if (c0 < bound && max_entries > 0 && stored > max_entries) { r->status = ST_EOOM; goto done; }
    }
    for (int c = cost[O_ATOM] + 1; c <= bound; ++c) {
        double t0 = now_s();
        if (run_level(r, c, &B)) goto fail;
        r->secs[c] = now_s() - t0;
        r->levels_done = c;
        if (B.first >= 0) { r->first = B.first; r->found_cost = c; r->status = ST_OK; goto done; }
        if (c == bound) { r->status = ST_NOT_FOUND; goto done; }
        stored += r->E[c];
        if (max_entries > 0 && stored > max_entries) { r->status = ST_EOOM; goto done; }
    }
    r->status = ST_NOT_FOUND;
    goto done;
fail:
    r->status = ST_EOOM;
done:
    free(B.rc); free(B.cm); free(B.ca); free(B.cb); free(B.pk); free(B.hv); free(B.key); free(B.sep);
    free(tmp); free(pk);
    return r;
}

o_run *oracle_run(const o_spec *s, const int32_t *cost, uint32_t op_mask, int bound, int mode,
                  int threads, int64_t max_entries) {
    return oracle_run_relaxed(s, cost, op_mask, bound, mode, threads, max_entries, RUC_NONE, 0, 0);
}

void oracle_free(o_run *r) {
    if (!r) return;
    if (r->L) for (int c = 0; c <= r->bound; ++c) { free(r->L[c].bits); free(r->L[c].rec); }
    free(r->L); free(r->E); free(r->C); free(r->secs);
    free(r->map.h); free(r->map.lev); free(r->map.idx); free(r->map.key); free(r->ruc_m);
    free(r);
}

int oracle_status(const o_run *r) { return r->status; }
int oracle_found_cost(const o_run *r) { return r->found_cost; }
int oracle_levels_done(const o_run *r) { return r->levels_done; }
int64_t oracle_level_new(const o_run *r, int c) { return (c >= 0 && c <= r->bound && r->E) ? r->E[c] : -1; }
int64_t oracle_level_candidates(const o_run *r, int c) { return (c >= 0 && c <= r->bound && r->C) ? r->C[c] : -1; }
double oracle_level_seconds(const o_run *r, int c) { return (c >= 0 && c <= r->bound && r->secs) ? r->secs[c] : -1.0; }
int64_t oracle_first_index(const o_run *r) { return r->first; }

/* Formula of a recipe, as postfix nodes; returns node count or -1 if cap too small. */
static int emit_formula(const o_run *r, o_recipe rc, o_node *buf, int cap, int *n) {
    int ka = -1, kb = -1;
    if (rc.op == O_ATOM) {
        if (*n >= cap) return -1;
        buf[*n].op = O_ATOM; buf[*n].a = (int32_t)rc.ia; buf[*n].b = 0;
        return (*n)++;
    }
    ka = emit_formula(r, r->L[rc.la].rec[rc.ia], buf, cap, n);
    if (ka < 0) return -1;
    if (rc.lb >= 0) { kb = emit_formula(r, r->L[rc.lb].rec[rc.ib], buf, cap, n); if (kb < 0) return -1; }
    if (*n >= cap) return -1;
    buf[*n].op = rc.op; buf[*n].a = ka; buf[*n].b = kb < 0 ? 0 : kb;
    return (*n)++;
}

int oracle_entry_formula(const o_run *r, int c, int64_t i, o_node *buf, int cap) {
    if (!r->L || c < 0 || c > r->bound || i < 0 || i >= r->L[c].n) return -1;
    int n = 0;
    return emit_formula(r, r->L[c].rec[i], buf, cap, &n) < 0 ? -1 : n;
}

int oracle_solution_formula(const o_run *r, o_node *buf, int cap) {
    if (r->first < 0) return -1;
    int n = 0;
    return emit_formula(r, r->sol, buf, cap, &n) < 0 ? -1 : n;
}

int oracle_entry_cm(const o_run *r, int c, int64_t i, uint8_t *out) {
    if (!r->L || c < 0 || c > r->bound || i < 0 || i >= r->L[c].n) return -1;
    unpack_bits(r->L[c].bits + (size_t)i * (size_t)r->pbytes, r->tb, out);
    return 0;
}
