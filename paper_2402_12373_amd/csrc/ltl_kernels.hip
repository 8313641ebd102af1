// gfx950 kernels of the enumerative LTL learner.
//
// Data layout (all inside the caller's workspace):
//   * A characteristic matrix (CM, Sec. 4) is R machine words, contiguous: the
//     characteristic sequences of all traces in the fixed order P then N.  A
//     trace of n positions takes ceil(n / W) consecutive words (W = 32 or 64),
//     position 0 in the most significant bit of its first word (the paper's
//     pictures: X is a left shift).  Bits past the end of a trace are 0.
//     Traces never straddle a 64-word row block, so the words of one trace sit
//     in consecutive lanes of one wave.
//   * Stored levels live in one arena: entry g (global id) at arena + g * R.
//   * Waves work with lanes across the words of a matrix ("rows"): a wave
//     evaluates a tile of up to 4 x 4 candidates, streaming row blocks of 64
//     words, so every load and store of a matrix is a coalesced 256/512-byte
//     access, whether it reads a child, a stored owner or writes a new entry.
//
// Connectives as branch-free word operations (Sec. 4, App. B), lane = word:
//   NOT  : ~w & valid
//   AND/OR: bitwise
//   X    : w << 1, with the next word's top bit carried in (wave ballot)
//   F    : w | -w (the "round up to a power of two minus one" reading of the
//          footnote in Sec. 4, MSB-first), or all-valid if a later word of the
//          trace is non-zero (wave ballot)
//   G    : valid & ~F(valid & ~w)   (always = not eventually not, within the trace)
//   U    : log2(n) shift-by-power-of-two doubling of App. B:
//             cs2 |= cs1 & (cs2 << s);  cs1 &= cs1 << s;   s = 1, 2, 4, ...
//          with cross-word shifts through lane shuffles; optionally a
//          carry-propagating add (psi | phi) + psi whose carry vector is the
//          until-chain psi_i | (phi_i & U_{i+1}).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ltl.h"
#include "ltl_internal.h"

namespace ltl {

#ifndef LTL_UC_ADD_PREFIX
#define LTL_UC_ADD_PREFIX 1      // carries between the words of a trace by one add (else Kogge-Stone)
#endif
constexpr int OP_UC = 8;   // U computed by the carry-chain adder

// Row blocks of operands in flight per evaluation wave, for one-word rows and for
// multi-word rows (tuning constants: multi-word tiles hold more registers per row block)
#ifndef LTL_EVAL_PIPE
#define LTL_EVAL_PIPE 2
#endif
#ifndef LTL_EVAL_PIPE_MW
#define LTL_EVAL_PIPE_MW 1
#endif
// Waves per SIMD the 64-bit level kernels are register-allocated for (tuning constants)
#ifndef LTL_WAVES_U64
#define LTL_WAVES_U64 2
#endif
#ifndef LTL_WAVES_U64_WG
#define LTL_WAVES_U64_WG 1
#endif

template <typename T> struct Word;
template <> struct Word<uint32_t> { static constexpr int BITS = 32; };
template <> struct Word<uint64_t> { static constexpr int BITS = 64; };

// ---------------------------------------------------------------------------
// Row metadata and kernel arguments
// ---------------------------------------------------------------------------
template <typename T>
struct RowMeta {
    T v, sm, sw;
    uint64_t nx, hn;
    uint64_t hnr;      // multi-word rows: hn bit-reversed, shifted down by one (carry prefix)
    uint32_t k0, k1;
    uint32_t cont;     // multi-word rows: all ones if the next lane holds the next word of this
                       // lane's trace, else 0
};

// Global-address-space views: loads through them become global_load with a
// scalar base and a 32-bit lane offset (no flat addressing).
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ gptr<T> as_global(uint64_t p) {
    return (gptr<T>)(uintptr_t)p;
}

// Element idx of a global array, addressed as a scalar base plus a 32-bit byte
// offset (one global_load with saddr, no 64-bit address arithmetic per lane).
// Every array read this way is below 2 GiB (checked when a job is laid out).
template <typename T>
__device__ __forceinline__ T ldg(gptr<T> base, uint32_t idx) {
    return *(gptr<T>)((const __attribute__((address_space(1))) char *)base + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T *base, uint32_t idx, T v) {
    *(__attribute__((address_space(1))) T *)((__attribute__((address_space(1))) char *)(uintptr_t)base +
                                             idx * (uint32_t)sizeof(T)) = v;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// FULL: everything the evaluation pass needs (separation bits, fingerprint keys);
// LIGHT: valid bits and the trace-continuation mask only (verify, materialize).
template <typename T, bool MW, bool FULL>
__device__ __forceinline__ RowMeta<T> load_meta(const Rows<T> &rw, uint32_t r, int lane) {
    RowMeta<T> m;
    m.v = ldg(as_global(rw.valid), r);
    if constexpr (FULL) {
        m.sw = ldg(as_global(rw.sepw), r);
        if constexpr (MW || sizeof(T) == 8) m.sm = ldg(as_global(rw.sepm), r);
        else m.sm = m.v & (T)0x80000000u;     // one word per trace: every live row is a first word
        if constexpr (sizeof(T) == 8) {       // two 32-bit halves, two keys per row
            const uint64_t kk = ldg(as_global((const uint64_t *)rw.key), r);
            m.k0 = (uint32_t)kk;
            m.k1 = (uint32_t)(kk >> 32);
        } else {
            m.k0 = ldg(as_global(rw.key), r);
            m.k1 = 0;
        }
    } else {
        m.sm = m.sw = 0;
        m.k0 = m.k1 = 0;
    }
    if constexpr (MW) {
        m.nx = ldg(as_global(rw.nxt), r);
    } else {
        m.nx = 0;
    }
    m.hn = 0;
    m.hnr = 0;
    m.cont = 0;
    return m;
}

// Wave-uniform part of the metadata, computed once the loads have landed.
template <typename T, bool MW>
__device__ __forceinline__ void finish_meta(RowMeta<T> &m, int lane) {
    if constexpr (MW) {
        const bool c = (m.nx & (2ull << lane)) != 0ull;
        m.hn = __ballot(c);
        m.hnr = __builtin_bitreverse64(m.hn) >> 1;
        m.cont = c ? ~0u : 0u;
    }
}

// ---------------------------------------------------------------------------
// Connectives
// ---------------------------------------------------------------------------

// 32-bit half of the next lane (lane 63 reads 0): one DPP whole-wave move.
__device__ __forceinline__ uint32_t next_lane32(uint32_t x) {
    constexpr int WAVE_SHL1 = 0x130;
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, WAVE_SHL1, 0xF, 0xF, true);
}

// Shift toward earlier positions by s within each trace: bits of later words of
// the same trace move in; nothing crosses into another trace.  Below 64 positions
// the word is a pair of 32-bit halves and each half of the result is one funnel
// shift (v_alignbit) of two neighbouring halves of this word and the next one
// (only the halves that reach the result are moved across lanes); the next word's
// halves are masked to 0 where the trace ends at this lane.
template <typename T, bool MW>
__device__ __forceinline__ T shl_pos(T x, uint32_t s, const RowMeta<T> &m, int lane) {
    if constexpr (!MW) {
        return x << s;
    } else {
        const uint32_t hi = (uint32_t)(x >> 32), lo = (uint32_t)x;
        if (s < 32) {
            // the moves run in every lane; lanes whose trace ends here drop the value
            const uint32_t nhi = next_lane32(hi) & m.cont;
            const uint32_t sh = 32u - s;
            return ((uint64_t)__builtin_amdgcn_alignbit(hi, lo, sh) << 32) | __builtin_amdgcn_alignbit(lo, nhi, sh);
        } else if (s == 32) {
            const uint32_t nhi = next_lane32(hi) & m.cont;
            return ((uint64_t)lo << 32) | nhi;
        } else if (s <= 64) {
            const uint32_t nhi = next_lane32(hi) & m.cont;
            const uint32_t nlo = next_lane32(lo) & m.cont;
            if (s == 64) return ((uint64_t)nhi << 32) | nlo;
            const uint32_t sh = 64u - s;
            return ((uint64_t)__builtin_amdgcn_alignbit(lo, nhi, sh) << 32) | __builtin_amdgcn_alignbit(nhi, nlo, sh);
        } else {
            uint32_t q = s >> 6;
            uint32_t src = (uint32_t)lane + q;
            uint64_t v = __shfl((unsigned long long)x, (int)(src & 63u));
            bool in = src < 64u && ((m.nx >> (src & 63u)) & 1ull);
            return in ? (T)v : (T)0;
        }
    }
}

template <typename T, bool MW>
__device__ __forceinline__ T op_F(T x, const RowMeta<T> &m) {
    T f = x | (T)((T)0 - x);
    if constexpr (MW) {
        uint64_t nz = __ballot(x != 0);
        if (nz & m.nx) f = m.v;
    }
    return f;
}

template <typename T, bool MW>
__device__ __forceinline__ T op_X(T x, const RowMeta<T> &m, int lane) {
    if constexpr (!MW) {
        return x << 1;
    } else {
        uint64_t top = __ballot((x >> 63) != 0);
        T cin = (top & m.nx & (2ull << lane)) ? (T)1 : (T)0;
        return (x << 1) | cin;
    }
}

template <typename T, bool MW>
__device__ __forceinline__ T op_U(T phi, T psi, const RowMeta<T> &m, uint32_t k, int lane) {
    T c1 = phi, c2 = psi;
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t s = 1u << i;
        c2 |= c1 & shl_pos<T, MW>(c2, s, m, lane);
        if (i + 1 < k) c1 &= shl_pos<T, MW>(c1, s, m, lane);
    }
    return c2;
}

// U as a carry chain.  Read a word MSB-first (bit 63 = its first position) as an
// unsigned integer: with A = phi | psi and B = psi, the carry out of each bit of A + B is
// psi | (phi & carry in), which is the recurrence of phi U psi toward earlier positions.
// Per bit that is psi where psi holds, else phi & carry in; since S ^ psi = A ^ carry in
// for the sum S, the result is bit-select(S ^ psi, psi, A) (a v_bfi per 32-bit half).
template <typename T>
__device__ __forceinline__ T uc_select(T S, T psi, T A) {
    const T t = S ^ psi;
    return (t & psi) | (~t & A);
}

template <typename T, bool MW>
__device__ __forceinline__ T op_UC(T phi, T psi, const RowMeta<T> &m, uint32_t maxw, int lane) {
    const T A = phi | psi;
    if constexpr (!MW) {
        return uc_select<T>((T)(A + psi), psi, A);
    } else {
        const uint64_t S = A + psi;
        // lanes whose word carries out without a carry in (G), and iff one comes in (P);
        // the carry into each lane from the later words of its trace is a prefix over the
        // lanes, from the last word of a trace toward its first; Pm is cut where a trace ends
        uint64_t Gm = __builtin_amdgcn_ballot_w64(S < A);
        uint64_t Pm = __builtin_amdgcn_ballot_w64(S == ~0ull) & m.hn;
#if LTL_UC_ADD_PREFIX
        // the prefix as one 64-bit add: in reversed lane order a later word is a lower
        // bit, and with generate G and propagate P (disjoint) the carry into each bit of
        // (G | P) + G is g | (p & carry) of the bit below; the bits below a lane whose next
        // lane starts another trace are cleared first (m.hnr), so no carry crosses traces
        (void)maxw;
        const uint64_t Gr = __builtin_bitreverse64(Gm) & m.hnr, Pr = __builtin_bitreverse64(Pm) & m.hnr;
        const uint64_t X = Gr | Pr;
        const uint64_t Cm = __builtin_bitreverse64((X + Gr) ^ X ^ Gr);
#else
        for (uint32_t d = 1; d < maxw; d <<= 1) {
            Gm |= Pm & (Gm >> d);
            Pm &= Pm >> d;
        }
        const uint64_t Cm = (Gm >> 1) & m.hn;
#endif
        (void)lane;
        const uint64_t cin = __builtin_amdgcn_inverse_ballot_w64(Cm) ? 1ull : 0ull;
        return uc_select<uint64_t>(S + cin, psi, A);
    }
}

template <typename T, bool MW, int OP>
__device__ __forceinline__ T apply(T a, T b, const RowMeta<T> &m, const Rows<T> &rw, int lane) {
    if constexpr (OP == LTL_ATOM) return a;
    else if constexpr (OP == LTL_NOT) return ~a & m.v;
    else if constexpr (OP == LTL_AND) return a & b;
    else if constexpr (OP == LTL_OR) return a | b;
    else if constexpr (OP == LTL_X) return op_X<T, MW>(a, m, lane);
    else if constexpr (OP == LTL_F) return op_F<T, MW>(a, m);
    else if constexpr (OP == LTL_G) return m.v & ~op_F<T, MW>((T)(m.v & ~a), m);
    else if constexpr (OP == LTL_U) return op_U<T, MW>(a, b, m, rw.ksteps, lane);
    else return op_UC<T, MW>(a, b, m, rw.maxw, lane);
}

// ---------------------------------------------------------------------------
// Fingerprint: fp = sum over 32-bit halves h of premix(h, key) * key (mod 2^64),
// keys random odd 32-bit numbers per half-word (one 32x32->64 multiply-add
// each).  premix is the bijection y = w ^ w>>8; y += key; y ^ y>>16.
// - Two matrices that differ in one half-word never collide (a nonzero 33-bit
//   difference times an odd 32-bit key is nonzero below 2^64).
// - The shifts keep the 2-adic valuation of any difference below 8, so that
//   differences confined to the top bits (the position-0 bits) still spread over
//   the sum.
// - The key added between the two shift stages makes the value table of each
//   row its own (the carries depend on the row).  Without it a short trace,
//   whose word takes few values, contributes one of a few multiples of a shared
//   constant times its key, and two matrices collide whenever the keys satisfy a
//   small integer relation over the rows they differ in: 37 pairs of distinct
//   languages shared a fingerprint among the 6.9 M of a length-4 Hamming
//   specification, none with the added key.
// Only a function of the matrix matters: every match is confirmed by a full
// compare.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t premix(uint32_t w, uint32_t key) {
    uint32_t y = (w ^ (w >> 8)) + key;
    return y ^ (y >> 16);
}

template <typename T>
__device__ __forceinline__ void fp_add(uint64_t &acc, T w, const RowMeta<T> &m) {
    if constexpr (sizeof(T) == 4) {
        acc += (uint64_t)premix((uint32_t)w, m.k0) * (uint64_t)m.k0;
    } else {
        acc += (uint64_t)premix((uint32_t)w, m.k0) * (uint64_t)m.k0;
        acc += (uint64_t)premix((uint32_t)(w >> 32), m.k1) * (uint64_t)m.k1;
    }
}

// Relaxed uniqueness check (Sec. 5), one 32-bit half h of a row (positions 32j..32j+31 of
// a trace, first position in the top bit) with its metadata (a, b):
//   keyed sums: A += premix(h, a) * a, B += premix(h, b) * b (odd keys a, b; dead halves 0);
//   pack form : the kept positions h & a, top-aligned, land at bit b of the 128-bit key
//               (bit 0 = the top bit of A); the host keeps every key bit below 126, so the
//               halves' contributions never overlap and their sum is their union.
__device__ __forceinline__ void ruc_half(uint64_t &ka, uint64_t &kb, uint32_t h, uint32_t a, uint32_t b, bool pack) {
    if (pack) {
        const uint64_t x = (uint64_t)(h & a) << 32;
        if (b < 64) {
            ka += x >> b;
            kb += b ? (x << (64 - b)) : 0ull;
        } else {
            kb += x >> (b - 64);
        }
    } else {
        ka += (uint64_t)premix(h, a) * (uint64_t)a;
        kb += (uint64_t)premix(h, b) * (uint64_t)b;
    }
}

template <typename T>
__device__ __forceinline__ void ruc_add(uint64_t &ka, uint64_t &kb, T w, const uint4 &mk, bool pack) {
    if constexpr (sizeof(T) == 8) {
        ruc_half(ka, kb, (uint32_t)(w >> 32), mk.x, mk.y, pack);
        ruc_half(ka, kb, (uint32_t)w, mk.z, mk.w, pack);
    } else {
        ruc_half(ka, kb, (uint32_t)w, mk.x, mk.y, pack);
    }
}

template <typename T>
__device__ __forceinline__ uint4 load_ruc_meta(const uint32_t *meta, uint32_t r) {
    const gptr<uint64_t> m = as_global((const uint64_t *)meta);
    if constexpr (sizeof(T) == 8) {
        const uint64_t top = ldg(m, 2 * r), low = ldg(m, 2 * r + 1);
        return make_uint4((uint32_t)top, (uint32_t)(top >> 32), (uint32_t)low, (uint32_t)(low >> 32));
    }
    const uint64_t v = ldg(m, r);
    return make_uint4((uint32_t)v, (uint32_t)(v >> 32), 0u, 0u);
}

// The 126-bit key from the two sums: pack form as summed; keyed sums: A's top 63 bits,
// then B's.  Then only the first `bits` bits are kept (debug truncation).
__device__ __forceinline__ void ruc_key(uint64_t sa, uint64_t sb, bool pack, uint32_t bits, uint64_t &k0,
                                        uint64_t &k1) {
    if (pack) {
        k0 = sa;
        k1 = sb;
    } else {
        k0 = (sa & ~1ull) | (sb >> 63);
        k1 = (sb << 1) & ~3ull;
    }
    if (bits > 0 && bits < 126) {
        if (bits <= 64) {
            k0 &= (bits == 64) ? ~0ull : ~(~0ull >> bits);
            k1 = 0;
        } else {
            k1 &= ~(~0ull >> (bits - 64));
        }
    }
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor((unsigned long long)x, o);
    return x;
}

// Lane-group swaps of gfx950: with lo = what the lower partner keeps and hi = what
// the upper partner keeps, the swap leaves the partner's copy of the kept value in
// the other register, so one swap and one add per 32-bit half do a halving step
// without selecting by lane.  O = 32: lanes l and l + 32; O = 16: lanes l and
// l + 16 within each 32-lane half.
template <int O>
__device__ __forceinline__ uint32_t swap_add_u32(uint32_t lo, uint32_t hi, uint32_t &carry_src) {
    if constexpr (O == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        carry_src = r[1];
        return r[0];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(lo, hi, false, false);
        carry_src = r[1];
        return r[0];
    }
}

template <int O>
__device__ __forceinline__ uint64_t swap_add_u64(uint64_t lo, uint64_t hi) {
    uint32_t b0, b1;
    const uint32_t a0 = swap_add_u32<O>((uint32_t)lo, (uint32_t)hi, b0);
    const uint32_t a1 = swap_add_u32<O>((uint32_t)(lo >> 32), (uint32_t)(hi >> 32), b1);
    return (((uint64_t)a1 << 32) | a0) + (((uint64_t)b1 << 32) | b0);
}

// One halving step of wave_sums: H sums held, the partner at xor distance O
// gets half of them; the kept half absorbs what the partner hands over.
template <int H, int O, int NP>
__device__ __forceinline__ void halve_sums(uint64_t (&v)[NP], int lane) {
    if constexpr (H > 1) {
        if constexpr (O >= 16) {
#pragma unroll
            for (int k = 0; k < H / 2; ++k) v[k] = swap_add_u64<O>(v[k], v[k + H / 2]);
        } else {
            const bool up = (lane & O) != 0;
#pragma unroll
            for (int k = 0; k < H / 2; ++k) {
                const uint64_t send = up ? v[k] : v[k + H / 2];
                const uint64_t keep = up ? v[k + H / 2] : v[k];
                v[k] = keep + (uint64_t)__shfl_xor((unsigned long long)send, O);
            }
        }
        halve_sums<H / 2, O / 2, NP>(v, lane);
    }
}

// NP wave sums at once (NP a power of two, at most 64): lane p < NP receives
// the sum of v[p] over the wave.  Each xor step hands the partner half of the
// sums still held and adds the half it receives (NP/2 + NP/4 + ... exchanges
// instead of 6 per sum); afterwards lane l holds sum l / (64/NP), partial over
// the lanes that agree in the higher bits, which the remaining steps complete.
template <int NP>
__device__ __forceinline__ uint64_t wave_sums(uint64_t (&v)[NP], int lane) {
    static_assert(NP >= 1 && NP <= 64 && (NP & (NP - 1)) == 0, "NP must be a power of two");
    constexpr int STRIDE = 64 / NP;
    halve_sums<NP, 32, NP>(v, lane);
    uint64_t x = v[0];
#pragma unroll
    for (int o = STRIDE / 2; o > 0; o >>= 1) x += (uint64_t)__shfl_xor((unsigned long long)x, o);
    return (uint64_t)__shfl((unsigned long long)x, (lane % NP) * STRIDE);
}

// Stafford's "Mix13" 64-bit finalizer (as used by SplitMix64).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t finish_fp(uint64_t s, uint64_t mask) {
    s &= mask;
    return s ? s : 1ull;
}

// ---------------------------------------------------------------------------
// Canonical order: blocks, tiles, candidate indices
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_block_tile(const Block *B, int nb, uint32_t t) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_block_cand(const Block *B, int nb, uint32_t x) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B[mid].cand_base <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void decode_tile(const Block &b, uint32_t lt, uint32_t &i0, uint32_t &j0) {
    if (b.nb == 0) { i0 = lt * TILE; j0 = 0; return; }
    if (!b.tri) { i0 = (lt / b.ntj) * TILE; j0 = (lt % b.ntj) * TILE; return; }
    const uint64_t n = b.nti;
    // row it holds n - it tiles; start(it) = it*n - it*(it-1)/2
    double nn = 2.0 * (double)n + 1.0;
    double disc = nn * nn - 8.0 * (double)lt;
    uint64_t it = (uint64_t)((nn - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (it >= n) it = n - 1;
    auto start = [&](uint64_t i) -> uint64_t { return i * n - (i * (i ? i - 1 : 0)) / 2; };
    while (it > 0 && start(it) > lt) --it;
    while (it + 1 < n && start(it + 1) <= lt) ++it;
    uint64_t jt = it + (lt - start(it));
    i0 = (uint32_t)it * TILE;
    j0 = (uint32_t)jt * TILE;
}

__host__ __device__ __forceinline__ uint32_t cand_index(const Block &b, uint32_t i, uint32_t j) {
    if (b.nb == 0) return b.cand_base + i;
    if (!b.tri) return b.cand_base + (uint32_t)((uint64_t)i * b.nb + j);
    uint64_t n = b.na;
    return b.cand_base + (uint32_t)((uint64_t)i * n - (uint64_t)i * (i + 1) / 2 + (j - i - 1));
}

// Inverse of cand_index within a block: local index l -> (i, j).
__host__ __device__ __forceinline__ void cand_decode(const Block &b, uint32_t l, uint32_t &i, uint32_t &j) {
    if (b.nb == 0) { i = l; j = 0; return; }
    if (!b.tri) { i = l / b.nb; j = l % b.nb; return; }
    const uint64_t n = b.na;
    auto T = [&](uint64_t ii) -> uint64_t { return ii * n - ii * (ii + 1) / 2; };
    double nn = 2.0 * (double)n - 1.0;
    double disc = nn * nn - 8.0 * (double)l;
    uint64_t ii = (uint64_t)((nn - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (ii >= n) ii = n - 1;
    while (ii > 0 && T(ii) > l) --ii;
    while (ii + 1 < n && T(ii + 1) <= l) ++ii;
    i = (uint32_t)ii;
    j = (uint32_t)(l - T(ii) + ii + 1);
}

__device__ __forceinline__ uint32_t rank_of(const uint32_t *bitmap, const uint32_t *wordpre, uint32_t x) {
    uint32_t w = bitmap[x >> 5];
    uint32_t below = (x & 31u) ? (w & ((1u << (x & 31u)) - 1u)) : 0u;
    return wordpre[x >> 5] + (uint32_t)__popc(below);
}

// ---------------------------------------------------------------------------
// Language-cache probe (one lane per candidate).  A slot whose key equals the
// fingerprint is either a settled entry of an earlier level (the candidate is a
// presumed duplicate of it, confirmed by the verify pass) or the group of this
// level (the smallest canonical index wins by atomicMin).
// ---------------------------------------------------------------------------
// The next claim numbers of a level, one atomic per group of lanes that claim together
// (the active lanes of the caller): the level's claim counter is one address that every
// new language of the level increments.
__device__ __forceinline__ uint32_t claim_number(Counters *ctr) {
    const uint64_t m = __ballot(1);
    const uint32_t lane = (uint32_t)__lane_id();
    const uint32_t lead = (uint32_t)__builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(&ctr->n_new, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, (int)lead);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

template <typename T>
__device__ uint32_t probe_claim(const LevelArgs<T> &A, uint64_t fp, uint32_t idx, uint32_t &claim) {
    claim = 0xFFFFFFFFu;
    uint32_t h = (uint32_t)(mix64(fp) >> 32) & A.slot_mask;
    for (uint32_t n = 0; n < MAX_PROBES; ++n) {
        unsigned long long k = __hip_atomic_load(&A.tkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == 0ull) {
            unsigned long long prev = atomicCAS(&A.tkey[h], 0ull, (unsigned long long)fp);
            if (prev == 0ull) {
                atomicMin(&A.tval[h], idx);
                const uint32_t pos = claim_number(A.ctr);
                if (pos == A.abort_cap || pos == A.new_cap) atomicOr(A.full, 1u);   // the level cannot be kept
                if (pos < A.new_cap) {
                    A.new_slots[pos] = h;
                    A.claimer[pos] = idx;
                    claim = pos;
                } else {
                    atomicOr(&A.ctr->overflow, 1u);
                }
                return h;
            }
            k = prev;
        }
        if (k == (unsigned long long)fp) {
            uint32_t v = __hip_atomic_load(&A.tval[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!(v & VAL_SETTLED)) atomicMin(&A.tval[h], idx);
            return h;
        }
        h = (h + 1) & A.slot_mask;
    }
    atomicOr(&A.ctr->overflow, 1u);
    return NO_SLOT;
}

// ---------------------------------------------------------------------------
// Level evaluation tile: TI x TJ candidates of one block (TJ = 1 for unary).
// EVAL   : fingerprint + separation, probe/claim in the language cache; with
//          A.cw, a second pass writes the matrix of every candidate that
//          claimed a new slot (its children are still in cache).
// VERIFY : recompute, compare in full with the stored matrix of the owner.
// ---------------------------------------------------------------------------
// F, G, X, NOT of one child, selected by a compile-time index (fused unary tiles)
template <typename T, bool MW>
__device__ __forceinline__ T apply_fused(int k, T a, const RowMeta<T> &m, const Rows<T> &rw, int lane) {
    if (k == 0) return apply<T, MW, LTL_F>(a, (T)0, m, rw, lane);
    if (k == 1) return apply<T, MW, LTL_G>(a, (T)0, m, rw, lane);
    if (k == 2) return apply<T, MW, LTL_X>(a, (T)0, m, rw, lane);
    return apply<T, MW, LTL_NOT>(a, (T)0, m, rw, lane);
}

// The words of one row block of every candidate of a tile.  For U, the App. B
// update cs1 <- cs1 & (cs1 << s) depends on phi (the a side) only: its chain is
// computed once per a-child and shared by the TJ pairs of that child.
// `need` (wave-uniform, bit p = pair p) names the pairs whose words are used.
// With GUARD and several words per trace (where one step of one pair costs
// lane moves and 64-bit shifts), the U chains of the other pairs, and of
// a-children none of whose pairs is needed, are skipped and their words left
// unspecified; the carry adder skips the other pairs too.  With one word per trace a step is two instructions, less than
// the branches that would skip it, so every pair is computed.
template <typename T, bool MW, int OP, int TI, int TJ, bool GUARD = false>
__device__ __forceinline__ void tile_words(const T (&av)[TI], const T (&bv)[TJ], const RowMeta<T> &m,
                                           const Rows<T> &rw, int lane, T (&w)[TI * TJ],
                                           uint32_t need = ~0u) {
    if constexpr (OP == LTL_U) {
        constexpr uint32_t ROW = (1u << TJ) - 1u;
        T c1[TI];
#pragma unroll
        for (int ii = 0; ii < TI; ++ii) {
            c1[ii] = av[ii];
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) w[ii * TJ + jj] = bv[jj];
        }
        constexpr bool G = GUARD && MW;
        const uint32_t k = rw.ksteps;
        for (uint32_t i = 0; i < k; ++i) {
            const uint32_t sh = 1u << i;
#pragma unroll
            for (int ii = 0; ii < TI; ++ii) {
                if (G && !((need >> (ii * TJ)) & ROW)) continue;
#pragma unroll
                for (int jj = 0; jj < TJ; ++jj) {
                    if (G && !((need >> (ii * TJ + jj)) & 1u)) continue;
                    T &c2 = w[ii * TJ + jj];
                    c2 |= c1[ii] & shl_pos<T, MW>(c2, sh, m, lane);
                }
            }
            if (i + 1 < k) {
#pragma unroll
                for (int ii = 0; ii < TI; ++ii) {
                    if (G && !((need >> (ii * TJ)) & ROW)) continue;
                    c1[ii] &= shl_pos<T, MW>(c1[ii], sh, m, lane);
                }
            }
        }
    } else if constexpr (OP == (int)OP_FUSED4) {
#pragma unroll
        for (int ii = 0; ii < TI; ++ii)
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) w[ii * TJ + jj] = apply_fused<T, MW>(jj, av[ii], m, rw, lane);
    } else {
        // the carry adder on several words per trace costs two ballots and a prefix over
        // the wave's masks per pair: with GUARD, pairs outside `need` are skipped (left 0)
        constexpr bool G = GUARD && MW && OP == OP_UC;
#pragma unroll
        for (int ii = 0; ii < TI; ++ii)
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) {
                if (G && !((need >> (ii * TJ + jj)) & 1u)) {
                    w[ii * TJ + jj] = 0;
                    continue;
                }
                w[ii * TJ + jj] = apply<T, MW, OP>(av[ii], bv[jj], m, rw, lane);
            }
    }
}

// Scalar address of child i on side `which` (0: a, 1: b) of a block: stored
// entries are found through store[] (claim order within their level), atoms
// directly.
template <typename T>
__device__ __forceinline__ uint64_t child_addr(const LevelArgs<T> &A, const Block &b, int which, uint32_t i) {
    const uint64_t cmb = (uint64_t)A.rows.R * sizeof(T);
    if (b.ind & (which ? 2u : 1u)) {
        const uint32_t pos = uniform(A.store[(which ? b.b_gid : b.a_gid) + i]);
        return (uint64_t)(uintptr_t)A.arena + (uint64_t)pos * cmb;
    }
    return b.a_ptr + (uint64_t)i * cmb;      // atoms (a side only: ATOM blocks are unary)
}

template <typename T>
__device__ __forceinline__ uint64_t arena_addr(const LevelArgs<T> &A, uint32_t pos) {
    return (uint64_t)(uintptr_t)A.arena + (uint64_t)pos * A.rows.R * sizeof(T);
}

// Row-split tiles (small levels): the waves of one workgroup take the row chunks
// of one tile and combine their partial fingerprints and separation flags here.
constexpr int WG_WAVES = 8;
struct WgShare {
    unsigned long long fp[WG_WAVES][16];
    unsigned long long fpb[WG_WAVES][16];   // relaxed check: the second keyed sum
    uint32_t bad[WG_WAVES][16];
    uint32_t claim[16];
};

// EVAL with WG: rows [rb0, rb1) are this wave's chunk of the tile; wave 0 of the
// workgroup claims the slots, then every wave writes its chunk of each claimer.
// WONLY: the write pass of a whole-row level (no evaluation): the claimers of the
// tile, known from cand_claim, get their matrices written.
template <typename T, bool MW, int OP, int TI, int TJ, bool VERIFY, bool CW = true, bool WG = false,
          bool WONLY = false, bool RK = false>
__device__ __forceinline__ void run_tile(const LevelArgs<T> &A, const Block &b, uint32_t i0, uint32_t j0, int lane,
                                         uint32_t rb0, uint32_t rb1, WgShare *sh = nullptr, uint32_t wv = 0,
                                         uint32_t nwv = 1) {
    constexpr int NP = TI * TJ;
    constexpr bool BIN = (OP == LTL_AND || OP == LTL_OR || OP == LTL_U || OP == OP_UC);
    constexpr bool FUSED = (OP == (int)OP_FUSED4);
    const uint32_t nbj = b.tri ? b.na : b.nb;
    // child matrices of the tile (clamped; results of out-of-range pairs are dropped)
    gptr<T> ap[TI];
    gptr<T> bp[TJ];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii) ap[ii] = as_global<T>(child_addr<T>(A, b, 0, min(i0 + ii, b.na - 1)));
#pragma unroll
    for (int jj = 0; jj < TJ; ++jj)
        bp[jj] = BIN ? as_global<T>(child_addr<T>(A, b, 1, min(j0 + jj, nbj - 1))) : (gptr<T>)nullptr;
    // canonical index of each pair, 0xFFFFFFFF if the pair is outside the block
    uint32_t idx[NP];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) {
            const uint32_t i = i0 + ii, j = j0 + jj;
            bool v = i < b.na;
            if constexpr (BIN) v = v && (b.tri ? (j < b.na && j > i) : (j < b.nb));
            if constexpr (FUSED) idx[ii * TJ + jj] = uniform(v ? b.fcb[jj] + i : 0xFFFFFFFFu);
            else idx[ii * TJ + jj] = uniform(v ? cand_index(b, i, j) : 0xFFFFFFFFu);
        }

    // one row block of operands (and, for VERIFY, of the owners), loaded one block ahead
    struct Rowset {
        RowMeta<T> m;
        T av[TI], bv[TJ];
        T tv[VERIFY ? NP : 1];
        uint4 rk[RK ? 1 : 0];       // relaxed check: key metadata of the row
    };
    gptr<T> tp[VERIFY ? NP : 1];      // VERIFY: stored matrix to compare with, or null
    if constexpr (VERIFY) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            uint32_t g = 0xFFFFFFFFu;
            if (idx[p] != 0xFFFFFFFFu) {
                const uint32_t h = uniform(A.cand_slot[idx[p]]);
                if (h != NO_SLOT) {
                    const uint32_t v = uniform(A.tval[h]);
                    if (v & VAL_SETTLED) {
                        g = v & ~VAL_SETTLED;
                        // the candidate whose matrix is stored is not compared with itself
                        if (g >= A.level_base) {
                            const uint32_t src = A.verify_rep
                                ? uniform(A.recipe[g])
                                : uniform(A.claimer[uniform(A.store[g]) - A.level_base]);
                            if (src == idx[p]) g = 0xFFFFFFFFu;
                        }
                    } else if (v != idx[p]) {
                        g = A.level_base + uniform(rank_of(A.bitmap, A.wordpre, v));
                    }
                }
            }
            tp[p] = (g != 0xFFFFFFFFu) ? as_global<T>(arena_addr<T>(A, uniform(A.store[g]))) : (gptr<T>)nullptr;
        }
    }
    auto load = [&](uint32_t blk, Rowset &L) {
        const uint32_t r = blk * 64u + (uint32_t)lane;
        L.m = load_meta<T, MW, !VERIFY>(A.rows, r, lane);
        if constexpr (RK) L.rk[0] = load_ruc_meta<T>(A.ruc_meta, r);
#pragma unroll
        for (int ii = 0; ii < TI; ++ii) L.av[ii] = ldg(ap[ii], r);
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) L.bv[jj] = BIN ? ldg(bp[jj], r) : (T)0;
        if constexpr (VERIFY) {
#pragma unroll
            for (int p = 0; p < NP; ++p) L.tv[p] = tp[p] ? ldg(tp[p], r) : (T)0;
        }
    };

    // row blocks are streamed PIPE at a time, the next PIPE loaded while the current
    // ones are computed
    constexpr int PIPE = (VERIFY || WG) ? 1 : (MW ? LTL_EVAL_PIPE_MW : LTL_EVAL_PIPE);
    auto load_group = [&](uint32_t blk, Rowset (&L)[PIPE]) {
#pragma unroll
        for (int u = 0; u < PIPE; ++u)
            if (blk + u < rb1) load(blk + u, L[u]);
    };

    if constexpr (!VERIFY) {
      uint32_t my_claim = 0xFFFFFFFFu;
      if constexpr (WONLY) {
        // a level that will not be stored keeps only the matrices the verification reads
        const bool keep_all = !A.bound_level && uniform64(A.ctr->first_sol) == ~0ull;
        if (lane < NP) {
            uint32_t idx_l = 0xFFFFFFFFu;
#pragma unroll
            for (int p = 0; p < NP; ++p)
                if (lane == p) idx_l = idx[p];
            if (idx_l != 0xFFFFFFFFu) {
                const uint32_t q = A.cand_claim[idx_l];
                if (q < A.arena_cap && (keep_all || A.has_member[q])) my_claim = q;
            }
        }
      } else {
        uint64_t acc[NP];
        uint64_t acc_b[RK ? NP : 1];      // relaxed check: the second keyed sum
        const bool rpack = RK && A.ruc_pack;
        // separation violations: only the position-0 bit (the top bit of a trace's first
        // word) counts, so 64-bit rows keep the top halves alone
        uint32_t viol[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) { acc[p] = 0; viol[p] = 0; }
#pragma unroll
        for (int p = 0; p < (RK ? NP : 1); ++p) acc_b[p] = 0;
        Rowset cur[PIPE], nxt[PIPE];
        load_group(rb0, cur);
        for (uint32_t blk = rb0; blk < rb1; blk += PIPE) {
            if (blk + PIPE < rb1) load_group(blk + PIPE, nxt);
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                if (blk + u < rb1) {
                    finish_meta<T, MW>(cur[u].m, lane);
                    T w[NP];
                    tile_words<T, MW, OP, TI, TJ>(cur[u].av, cur[u].bv, cur[u].m, A.rows, lane, w);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        // one word per trace (32-bit layout): every live row is a first word and
                        // dead rows are zero, so the position-0 bit is masked once, after the loop
                        if constexpr (!MW && sizeof(T) == 4) viol[p] |= (uint32_t)(w[p] ^ cur[u].m.sw);
                        else viol[p] |= (uint32_t)((w[p] ^ cur[u].m.sw) >> (8 * sizeof(T) - 32)) &
                                        (uint32_t)(cur[u].m.sm >> (8 * sizeof(T) - 32));
                        if constexpr (RK) ruc_add<T>(acc[p], acc_b[RK ? p : 0], w[p], cur[u].rk[0], rpack);
                        else fp_add<T>(acc[p], w[p], cur[u].m);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < PIPE; ++u) cur[u] = nxt[u];
        }
        const uint64_t my_fp = wave_sums<NP>(acc, lane);   // valid in lanes < NP
        uint64_t my_fp_b = 0;
        if constexpr (RK) my_fp_b = wave_sums<NP>(acc_b, lane);
        uint32_t my_idx = 0xFFFFFFFFu;
        bool my_bad = false;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if constexpr (!MW && sizeof(T) == 4) viol[p] &= 0x80000000u;
            const bool bad = __ballot(viol[p] != 0) != 0ull;
            if (lane == p) { my_idx = idx[p]; my_bad = bad; }
        }
        if constexpr (RK && WG) {
            // relaxed check, a tile's row chunks over the waves of a workgroup (and maybe over
            // several workgroups): partial sums combined in LDS, then the key or, for a tile
            // spread over workgroups, the partial sums added per candidate (k_ruc_finish)
            if (lane < NP) {
                sh->fp[wv][lane] = my_fp;
                sh->fpb[wv][lane] = my_fp_b;
                sh->bad[wv][lane] = my_bad ? 1u : 0u;
            }
            __syncthreads();
            if (wv == 0 && lane < NP && my_idx != 0xFFFFFFFFu) {
                uint64_t fa = 0, fb = 0;
                uint32_t bad = 0;
                for (uint32_t w = 0; w < nwv; ++w) {
                    fa += sh->fp[w][lane];
                    fb += sh->fpb[w][lane];
                    bad |= sh->bad[w][lane];
                }
                if (A.wg_split > 1) {
                    atomicAdd(&A.cand_fp[my_idx], (unsigned long long)fa);
                    atomicAdd(&A.cand_fp[A.ruc_fpb_off + my_idx], (unsigned long long)fb);
                    if (bad) atomicOr(&A.cand_viol[my_idx >> 5], 1u << (my_idx & 31u));
                } else {
                    if (!bad) atomicMin(&A.ctr->first_sol, (unsigned long long)my_idx);
                    uint64_t k0, k1;
                    ruc_key(fa, fb, rpack, A.ruc_bits, k0, k1);
                    A.cand_key[2 * (uint64_t)my_idx] = k0;
                    A.cand_key[2 * (uint64_t)my_idx + 1] = k1;
                    A.cand_claim[my_idx] = 0xFFFFFFFFu;
                }
            }
            __syncthreads();   // the shared block is free for the next tile
            return;
        } else if constexpr (RK) {
            // relaxed check: the key is written; the claims are a pass of their own
            if (my_idx != 0xFFFFFFFFu) {
                if (!my_bad) atomicMin(&A.ctr->first_sol, (unsigned long long)my_idx);
                uint64_t k0, k1;
                ruc_key(my_fp, my_fp_b, rpack, A.ruc_bits, k0, k1);
                A.cand_key[2 * (uint64_t)my_idx] = k0;
                A.cand_key[2 * (uint64_t)my_idx + 1] = k1;
                A.cand_claim[my_idx] = 0xFFFFFFFFu;     // representatives are marked after the compaction
            }
            return;
        } else if constexpr (WG) {
            // partial results of this wave's row chunk -> wave 0 claims for the tile
            if (lane < NP) {
                sh->fp[wv][lane] = my_fp;
                sh->bad[wv][lane] = my_bad ? 1u : 0u;
            }
            __syncthreads();
            if (wv == 0 && lane < NP) {
                uint32_t claim = 0xFFFFFFFFu;
                if (my_idx != 0xFFFFFFFFu) {
                    uint64_t fp = 0;
                    uint32_t bad = 0;
                    for (uint32_t w = 0; w < nwv; ++w) {
                        fp += sh->fp[w][lane];
                        bad |= sh->bad[w][lane];
                    }
                    if (A.wg_split > 1) {      // one of several workgroups of the tile: partial sums
                        atomicAdd(&A.cand_fp[my_idx], (unsigned long long)fp);
                        if (bad) atomicOr(&A.cand_viol[my_idx >> 5], 1u << (my_idx & 31u));
                    } else {
                        if (!bad) atomicMin(&A.ctr->first_sol, (unsigned long long)my_idx);
                        A.cand_slot[my_idx] = probe_claim<T>(A, finish_fp(fp, A.fp_mask), my_idx, claim);
                    }
                }
                sh->claim[lane] = claim;
            }
            __syncthreads();
            if (lane < NP) my_claim = sh->claim[lane];
            __syncthreads();   // the shared block is free for the next tile
        } else if (my_idx != 0xFFFFFFFFu) {
            if (!my_bad) atomicMin(&A.ctr->first_sol, (unsigned long long)my_idx);
            A.cand_slot[my_idx] = probe_claim<T>(A, finish_fp(my_fp, A.fp_mask), my_idx, my_claim);
            if (A.cand_claim) A.cand_claim[my_idx] = my_claim;
        }
      }
        // claimers' matrices (in the evaluation pass the children are still in cache)
        if (CW && (WG || WONLY || A.cw) && __ballot(my_claim < A.arena_cap) != 0ull) {
            gptr<T> dp[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const uint32_t cp = (uint32_t)__builtin_amdgcn_readlane((int)my_claim, p);
                dp[p] = (cp < A.arena_cap) ? as_global<T>(arena_addr<T>(A, A.level_base + cp)) : (gptr<T>)nullptr;
            }
            uint32_t wneed = 0;     // the pairs whose matrices are written
#pragma unroll
            for (int p = 0; p < NP; ++p)
                if (dp[p]) wneed |= 1u << p;
            wneed = uniform(wneed);
            // a memory-bound pass (children re-read, new matrices written): several row
            // blocks of loads in flight per wave
            constexpr int UNR = 4;
            struct RowsetW {
                RowMeta<T> m;
                T av[TI], bv[TJ];
            };
            for (uint32_t blk = rb0; blk < rb1; blk += UNR) {
                RowsetW L[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    if (blk + u < rb1) {
                        const uint32_t r = (blk + u) * 64u + (uint32_t)lane;
                        L[u].m = load_meta<T, MW, false>(A.rows, r, lane);
#pragma unroll
                        for (int ii = 0; ii < TI; ++ii) L[u].av[ii] = ldg(ap[ii], r);
#pragma unroll
                        for (int jj = 0; jj < TJ; ++jj) L[u].bv[jj] = BIN ? ldg(bp[jj], r) : (T)0;
                    }
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    if (blk + u < rb1) {
                        finish_meta<T, MW>(L[u].m, lane);
                        T w[NP];
                        tile_words<T, MW, OP, TI, TJ, true>(L[u].av, L[u].bv, L[u].m, A.rows, lane, w, wneed);
                        const uint32_t r = (blk + u) * 64u + (uint32_t)lane;
#pragma unroll
                        for (int p = 0; p < NP; ++p)
                            if (dp[p]) stg((T *)(uintptr_t)dp[p], r, w[p]);
                    }
                }
            }
        }
    } else {
        uint32_t vneed = 0;     // the pairs compared with a stored matrix
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (tp[p]) vneed |= 1u << p;
        vneed = uniform(vneed);
        if (!vneed) return;
        T diff[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) diff[p] = 0;
        Rowset cur[PIPE], nxt[PIPE];
        load_group(rb0, cur);
        for (uint32_t blk = rb0; blk < rb1; blk += PIPE) {
            if (blk + PIPE < rb1) load_group(blk + PIPE, nxt);
#pragma unroll
            for (int u = 0; u < PIPE; ++u) {
                if (blk + u < rb1) {
                    finish_meta<T, MW>(cur[u].m, lane);
                    T w[NP];
                    tile_words<T, MW, OP, TI, TJ, true>(cur[u].av, cur[u].bv, cur[u].m, A.rows, lane, w, vneed);
#pragma unroll
                    for (int p = 0; p < NP; ++p) diff[p] |= w[p] ^ cur[u].tv[p];
                }
            }
#pragma unroll
            for (int u = 0; u < PIPE; ++u) cur[u] = nxt[u];
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (!tp[p]) continue;
            const bool mism = __ballot(diff[p] != 0) != 0ull;
            if (mism && lane == 0) {
                const uint32_t bit = 1u << (idx[p] & 31u);
                if (!(atomicOr(&A.coll_bits[idx[p] >> 5], bit) & bit)) atomicAdd(&A.ctr->n_coll, 1u);
            }
        }
    }
}

__device__ __forceinline__ Block uniform_block(const Block &in) {
    Block b;
    const uint32_t *src = (const uint32_t *)&in;
    uint32_t *dst = (uint32_t *)&b;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(Block) / 4); ++k) dst[k] = uniform(src[k]);
    return b;
}

// ---------------------------------------------------------------------------
// LDS staging of child operand tiles (binary connectives, whole-row levels).  A
// workgroup of 4 waves takes an 8 x 8 group of pairs (2 x 2 tiles of 4 x 4): per row
// block each wave loads 4 of the 16 child words (waves 0-1 the 8 a-children, waves
// 2-3 the 8 b-children) into LDS, and every wave reads the 4 + 4 words of its own
// tile from there, so each child row block is fetched once per 8 x 8 group instead of
// once per 4 x 4 tile.  The LDS buffer is double-buffered: one barrier per row block.
// ---------------------------------------------------------------------------
enum { CLS_UNARY = 0, CLS_ANDOR = 1, CLS_U = 2, CLS_UC = 3 };
constexpr int STG_SIDE = 2 * TILE;            // children per side of a group
template <typename T>
struct StageBuf {
    T w[2][2 * STG_SIDE][64];
};

template <typename T, bool MW, int OP, bool VERIFY, bool WONLY>
__device__ __forceinline__ void run_tile_staged(const LevelArgs<T> &A, const Block &b, uint32_t ia0, uint32_t jb0,
                                                int lane, uint32_t wv, uint32_t rb0, uint32_t rb1, StageBuf<T> *sb) {
    constexpr int TI = TILE, TJ = TILE, NP = TI * TJ;
    constexpr bool EVAL = !VERIFY && !WONLY;
    const uint32_t nbj = b.tri ? b.na : b.nb;
    const uint32_t di = TI * (wv >> 1), dj = TJ * (wv & 1);
    const uint32_t i0 = ia0 + di, j0 = jb0 + dj;
    uint32_t idx[NP];
#pragma unroll
    for (int ii = 0; ii < TI; ++ii)
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) {
            const uint32_t i = i0 + ii, j = j0 + jj;
            const bool v = i < b.na && (b.tri ? (j < b.na && j > i) : (j < b.nb));
            idx[ii * TJ + jj] = uniform(v ? cand_index(b, i, j) : 0xFFFFFFFFu);
        }
    // the 4 children this wave stages
    const uint32_t side = wv >> 1, part = wv & 1;
    gptr<T> sp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t c = (side ? jb0 : ia0) + 4u * part + (uint32_t)k;
        sp[k] = as_global<T>(child_addr<T>(A, b, (int)side, min(c, (side ? nbj : b.na) - 1)));
    }
    // what this wave does with its pairs
    uint32_t need = 0;
    gptr<T> tp[VERIFY ? NP : 1];      // VERIFY: stored matrix to compare with, or null
    gptr<T> dp[WONLY ? NP : 1];       // WONLY: arena place of the claimer's matrix, or null
    if constexpr (VERIFY) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            uint32_t g = 0xFFFFFFFFu;
            if (idx[p] != 0xFFFFFFFFu) {
                const uint32_t h = uniform(A.cand_slot[idx[p]]);
                if (h != NO_SLOT) {
                    const uint32_t v = uniform(A.tval[h]);
                    if (v & VAL_SETTLED) {
                        g = v & ~VAL_SETTLED;
                        if (g >= A.level_base) {
                            const uint32_t src = A.verify_rep
                                ? uniform(A.recipe[g])
                                : uniform(A.claimer[uniform(A.store[g]) - A.level_base]);
                            if (src == idx[p]) g = 0xFFFFFFFFu;
                        }
                    } else if (v != idx[p]) {
                        g = A.level_base + uniform(rank_of(A.bitmap, A.wordpre, v));
                    }
                }
            }
            tp[p] = (g != 0xFFFFFFFFu) ? as_global<T>(arena_addr<T>(A, uniform(A.store[g]))) : (gptr<T>)nullptr;
            if (tp[p]) need |= 1u << p;
        }
    } else if constexpr (WONLY) {
        const bool keep_all = !A.bound_level && uniform64(A.ctr->first_sol) == ~0ull;
        uint32_t my_claim = 0xFFFFFFFFu;
        if (lane < NP) {
            uint32_t idx_l = 0xFFFFFFFFu;
#pragma unroll
            for (int p = 0; p < NP; ++p)
                if (lane == p) idx_l = idx[p];
            if (idx_l != 0xFFFFFFFFu) {
                const uint32_t q = A.cand_claim[idx_l];
                if (q < A.arena_cap && (keep_all || A.has_member[q])) my_claim = q;
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const uint32_t cp = (uint32_t)__builtin_amdgcn_readlane((int)my_claim, p);
            dp[p] = (cp < A.arena_cap) ? as_global<T>(arena_addr<T>(A, A.level_base + cp)) : (gptr<T>)nullptr;
            if (dp[p]) need |= 1u << p;
        }
    } else {
        need = ~0u;
    }
    need = uniform(need);
    // the group is skipped only if none of its waves has work (every wave stages)
    if (!__syncthreads_or(need != 0u)) return;

    uint64_t acc[EVAL ? NP : 1];
    uint32_t viol[EVAL ? NP : 1];
    T diff[VERIFY ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if constexpr (EVAL) { acc[p] = 0; viol[p] = 0; }
        if constexpr (VERIFY) diff[p] = 0;
    }
    const uint32_t slot0 = side * STG_SIDE + 4u * part;
    T nxt[4];
    if (rb0 < rb1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) nxt[k] = ldg(sp[k], rb0 * 64u + (uint32_t)lane);
    }
    uint32_t buf = 0;
    for (uint32_t blk = rb0; blk < rb1; ++blk) {
        const uint32_t r = blk * 64u + (uint32_t)lane;
        T cur[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
        if (blk + 1 < rb1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nxt[k] = ldg(sp[k], r + 64u);
        }
        RowMeta<T> m = load_meta<T, MW, EVAL>(A.rows, r, lane);
        T tv[VERIFY ? NP : 1];
        if constexpr (VERIFY) {
#pragma unroll
            for (int p = 0; p < NP; ++p) tv[p] = tp[p] ? ldg(tp[p], r) : (T)0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) sb->w[buf][slot0 + k][lane] = cur[k];
        __syncthreads();
        if (need) {
            T av[TI], bv[TJ];
#pragma unroll
            for (int ii = 0; ii < TI; ++ii) av[ii] = sb->w[buf][di + ii][lane];
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) bv[jj] = sb->w[buf][STG_SIDE + dj + jj][lane];
            finish_meta<T, MW>(m, lane);
            T w[NP];
            tile_words<T, MW, OP, TI, TJ, !EVAL>(av, bv, m, A.rows, lane, w, need);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if constexpr (EVAL) {
                    if constexpr (!MW && sizeof(T) == 4) viol[p] |= (uint32_t)(w[p] ^ m.sw);
                    else viol[p] |= (uint32_t)((w[p] ^ m.sw) >> (8 * sizeof(T) - 32)) &
                                    (uint32_t)(m.sm >> (8 * sizeof(T) - 32));
                    fp_add<T>(acc[p], w[p], m);
                } else if constexpr (VERIFY) {
                    diff[p] |= w[p] ^ tv[p];
                } else {
                    if (dp[p]) stg((T *)(uintptr_t)dp[p], r, w[p]);
                }
            }
        }
        buf ^= 1u;
    }
    if constexpr (EVAL) {
        const uint64_t my_fp = wave_sums<NP>(acc, lane);   // valid in lanes < NP
        uint32_t my_idx = 0xFFFFFFFFu;
        bool my_bad = false;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if constexpr (!MW && sizeof(T) == 4) viol[p] &= 0x80000000u;
            const bool bad = __ballot(viol[p] != 0) != 0ull;
            if (lane == p) { my_idx = idx[p]; my_bad = bad; }
        }
        if (my_idx != 0xFFFFFFFFu) {
            uint32_t my_claim;
            if (!my_bad) atomicMin(&A.ctr->first_sol, (unsigned long long)my_idx);
            A.cand_slot[my_idx] = probe_claim<T>(A, finish_fp(my_fp, A.fp_mask), my_idx, my_claim);
            if (A.cand_claim) A.cand_claim[my_idx] = my_claim;
        }
    } else if constexpr (VERIFY) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (!tp[p]) continue;
            const bool mism = __ballot(diff[p] != 0) != 0ull;
            if (mism && lane == 0) {
                const uint32_t bit = 1u << (idx[p] & 31u);
                if (!(atomicOr(&A.coll_bits[idx[p] >> 5], bit) & bit)) atomicAdd(&A.ctr->n_coll, 1u);
            }
        }
    }
}

__device__ __forceinline__ int find_block_group(const Block *B, int nb, uint32_t s) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B[mid].st_base <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Local group index -> first a and b child of the 8 x 8 group (row-major over the
// block's group grid; the upper triangle for AND/OR of one level with itself).
__device__ __forceinline__ void decode_group(const Block &b, uint32_t ls, uint32_t &ia0, uint32_t &jb0) {
    const uint32_t ngi = (b.nti + 1) / 2;
    if (!b.tri) {
        const uint32_t ngj = (b.ntj + 1) / 2;
        ia0 = (ls / ngj) * STG_SIDE;
        jb0 = (ls % ngj) * STG_SIDE;
        return;
    }
    const uint64_t n = ngi;
    double nn = 2.0 * (double)n + 1.0;
    double disc = nn * nn - 8.0 * (double)ls;
    uint64_t it = (uint64_t)((nn - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (it >= n) it = n - 1;
    auto start = [&](uint64_t i) -> uint64_t { return i * n - (i * (i ? i - 1 : 0)) / 2; };
    while (it > 0 && start(it) > ls) --it;
    while (it + 1 < n && start(it + 1) <= ls) ++it;
    const uint64_t jt = it + (ls - start(it));
    ia0 = (uint32_t)it * STG_SIDE;
    jb0 = (uint32_t)jt * STG_SIDE;
}

// PASS 0 evaluation, 1 verification, 2 write pass; one workgroup of 4 waves per
// (group, row chunk) work item.
template <typename T, bool MW, int PASS, int CLS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : LTL_WAVES_U64)))
void k_level_stg(LevelArgs<T> A, const Block *blocks, uint32_t nblocks, uint32_t ngroups, uint32_t chunk) {
    __shared__ StageBuf<T> sb;
    constexpr bool VERIFY = PASS == 1, WONLY = PASS == 2;
    const int lane = (int)__lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    if constexpr (VERIFY || WONLY) {
        if (uniform(A.ctr->overflow) || uniform(A.ctr->n_new) > A.arena_cap) return;
    }
    const uint32_t NB = A.rows.NB;
    const uint32_t nchunk = (NB + chunk - 1) / chunk;
    const uint32_t nwork = ngroups * nchunk;
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint32_t s = w / nchunk, q = w - s * nchunk;
        const uint32_t rb0 = q * chunk, rb1 = min(NB, rb0 + chunk);
        const int bi = (int)uniform((uint32_t)find_block_group(blocks, (int)nblocks, s));
        const Block b = uniform_block(blocks[bi]);
        uint32_t ia0, jb0;
        decode_group(b, s - b.st_base, ia0, jb0);
        ia0 = uniform(ia0);
        jb0 = uniform(jb0);
        if constexpr (CLS == CLS_ANDOR) {
            if (b.op == LTL_AND) run_tile_staged<T, MW, LTL_AND, VERIFY, WONLY>(A, b, ia0, jb0, lane, wv, rb0, rb1, &sb);
            else run_tile_staged<T, MW, LTL_OR, VERIFY, WONLY>(A, b, ia0, jb0, lane, wv, rb0, rb1, &sb);
        } else if constexpr (CLS == CLS_U) {
            run_tile_staged<T, MW, LTL_U, VERIFY, WONLY>(A, b, ia0, jb0, lane, wv, rb0, rb1, &sb);
        } else {
            run_tile_staged<T, MW, OP_UC, VERIFY, WONLY>(A, b, ia0, jb0, lane, wv, rb0, rb1, &sb);
        }
        __syncthreads();    // the LDS buffers are free for the next work item
    }
}

// Connective classes get kernels of their own, so that each is register-
// allocated for its own tile loop: CLS_UNARY (ATOM, NOT, X, F, G; 4 children
// per tile), CLS_ANDOR (4 x 4 pairs), CLS_U (4 x 4 pairs, doubling) and
// CLS_UC (4 x 4 pairs, carry adder).  Blocks of a class are listed in
// A.cls_blocks with class-local tile numbering.


// (the relaxed check's key pass holds two sums per pair: register-allocated for two waves
// per SIMD, as the 64-bit kernels)
template <typename T, bool MW, bool VERIFY, int CLS, bool WONLY = false, bool RK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !RK ? 4 : LTL_WAVES_U64))) void k_level(LevelArgs<T> A, const Block *blocks, uint32_t nblocks,
                                               uint32_t ntiles, uint32_t chunk) {
    const int lane = (int)__lane_id();
    if constexpr (VERIFY || WONLY) {
        if (uniform(A.ctr->overflow) || uniform(A.ctr->n_new) > A.arena_cap) return;
    }
    const uint32_t NB = A.rows.NB;
    const uint32_t nchunk = (NB + chunk - 1) / chunk;          // row chunks per tile
    const uint32_t nwork = ntiles * nchunk;
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t w = wave; w < nwork; w += nwaves) {
        if constexpr (!VERIFY && !WONLY) {
            // once the level's new groups outgrow the arena (or the slot list) the level ends
            // in LTL_E_OOM whatever else it finds: the remaining tiles are not evaluated (a batch
            // lane of a shared budget goes on up to what the whole pool could hold).  The flag
            // has a cache line of its own (the claim counter's line is busy with atomics)
            if (uniform(__hip_atomic_load(A.full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) break;
        }
        const uint32_t t = w / nchunk, q = w - t * nchunk;
        const uint32_t rb0 = q * chunk, rb1 = min(NB, rb0 + chunk);
        const int bi = (int)uniform((uint32_t)find_block_tile(blocks, (int)nblocks, t));
        const Block b = uniform_block(blocks[bi]);
        uint32_t i0, j0;
        decode_tile(b, t - b.tile_base, i0, j0);
        i0 = uniform(i0);
        j0 = uniform(j0);
        if constexpr (CLS == CLS_UNARY) {
            switch (b.op) {
            case LTL_ATOM: run_tile<T, MW, LTL_ATOM, TILE, 1, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            case LTL_NOT:  run_tile<T, MW, LTL_NOT, TILE, 1, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            case LTL_X:    run_tile<T, MW, LTL_X, TILE, 1, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            case LTL_F:    run_tile<T, MW, LTL_F, TILE, 1, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            case LTL_G:    run_tile<T, MW, LTL_G, TILE, 1, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            default:       run_tile<T, MW, (int)OP_FUSED4, TILE, 4, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1); break;
            }
        } else if constexpr (CLS == CLS_ANDOR) {
            if (b.op == LTL_AND) run_tile<T, MW, LTL_AND, TILE, TILE, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1);
            else run_tile<T, MW, LTL_OR, TILE, TILE, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1);
        } else if constexpr (CLS == CLS_U) {
            run_tile<T, MW, LTL_U, TILE, TILE, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1);
        } else {
            run_tile<T, MW, OP_UC, TILE, TILE, VERIFY, true, false, WONLY, RK>(A, b, i0, j0, lane, rb0, rb1);
        }
    }
}

// Verification of a row-split level, all connective classes in one dispatch
// (small levels, where the number of dispatches, not occupancy, bounds the
// level): blocks of every class, one tile numbering, one row chunk per wave.
template <typename T, bool MW, bool VERIFY>
__global__ __launch_bounds__(256) void k_level_all(LevelArgs<T> A, const Block *blocks, uint32_t nblocks,
                                                   uint32_t ntiles, uint32_t chunk) {
    const int lane = (int)__lane_id();
    if constexpr (VERIFY) {
        if (uniform(A.ctr->overflow) || uniform(A.ctr->n_new) > A.arena_cap) return;
    }
    const uint32_t NB = A.rows.NB;
    const uint32_t nchunk = (NB + chunk - 1) / chunk;
    const uint32_t nwork = ntiles * nchunk;
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t w = wave; w < nwork; w += nwaves) {
        const uint32_t t = w / nchunk, q = w - t * nchunk;
        const uint32_t rb0 = q * chunk, rb1 = min(NB, rb0 + chunk);
        const int bi = (int)uniform((uint32_t)find_block_tile(blocks, (int)nblocks, t));
        const Block b = uniform_block(blocks[bi]);
        uint32_t i0, j0;
        decode_tile(b, t - b.tile_base, i0, j0);
        i0 = uniform(i0);
        j0 = uniform(j0);
        switch (b.op) {
        case LTL_ATOM: run_tile<T, MW, LTL_ATOM, TILE, 1, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_NOT:  run_tile<T, MW, LTL_NOT, TILE, 1, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_X:    run_tile<T, MW, LTL_X, TILE, 1, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_F:    run_tile<T, MW, LTL_F, TILE, 1, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_G:    run_tile<T, MW, LTL_G, TILE, 1, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_AND:  run_tile<T, MW, LTL_AND, TILE, TILE, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_OR:   run_tile<T, MW, LTL_OR, TILE, TILE, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        case LTL_U:
            if (A.ucarry) run_tile<T, MW, OP_UC, TILE, TILE, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1);
            else run_tile<T, MW, LTL_U, TILE, TILE, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1);
            break;
        default:       run_tile<T, MW, (int)OP_FUSED4, TILE, 4, VERIFY, false>(A, b, i0, j0, lane, rb0, rb1); break;
        }
    }
}

// Row-split levels, every connective class in one dispatch: one workgroup of
// WG_WAVES waves per tile, each wave a chunk of the row blocks; the tile's slots
// are claimed and its claimers' matrices written in the same dispatch.  Tiles of
// long rows may be spread over A.wg_split workgroups, each a range of row blocks
// (then k_probe claims and k_materialize writes).  Multi-word rows need more
// registers per wave: half as many waves per workgroup.
template <bool MW> constexpr int wg_waves() { return MW ? WG_WAVES / 2 : WG_WAVES; }

template <typename T, bool MW, bool RK = false>
__global__ __launch_bounds__(64 * wg_waves<MW>())
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !RK ? 4 : LTL_WAVES_U64_WG)))
void k_level_wg(LevelArgs<T> A, const Block *blocks, uint32_t nblocks, uint32_t ntiles) {
    __shared__ WgShare sh;
    const int lane = (int)__lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    const uint32_t nwv = blockDim.x >> 6;
    const uint32_t NB = A.rows.NB;
    const uint32_t G = A.wg_split;
    const uint32_t gchunk = (NB + G - 1) / G;               // row blocks per workgroup of a tile
    const uint32_t nwork = ntiles * G;
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint32_t t = w / G, g = w - t * G;
        const uint32_t g0 = min(NB, g * gchunk), g1 = min(NB, g0 + gchunk);
        const uint32_t chunk = (g1 - g0 + nwv - 1) / nwv;
        const uint32_t rb0 = min(g1, g0 + wv * chunk), rb1 = min(g1, rb0 + chunk);
        const int bi = (int)uniform((uint32_t)find_block_tile(blocks, (int)nblocks, t));
        const Block b = uniform_block(blocks[bi]);
        uint32_t i0, j0;
        decode_tile(b, t - b.tile_base, i0, j0);
        i0 = uniform(i0);
        j0 = uniform(j0);
        switch (b.op) {
        case LTL_ATOM: run_tile<T, MW, LTL_ATOM, TILE, 1, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_NOT:  run_tile<T, MW, LTL_NOT, TILE, 1, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_X:    run_tile<T, MW, LTL_X, TILE, 1, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_F:    run_tile<T, MW, LTL_F, TILE, 1, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_G:    run_tile<T, MW, LTL_G, TILE, 1, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_AND:  run_tile<T, MW, LTL_AND, TILE, TILE, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_OR:   run_tile<T, MW, LTL_OR, TILE, TILE, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        case LTL_U:
            if (A.ucarry) run_tile<T, MW, OP_UC, TILE, TILE, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv);
            else run_tile<T, MW, LTL_U, TILE, TILE, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv);
            break;
        default:       run_tile<T, MW, (int)OP_FUSED4, TILE, 4, false, true, true, false, RK>(A, b, i0, j0, lane, rb0, rb1, &sh, wv, nwv); break;
        }
    }
}

// Whole-row levels: claims whose group another candidate of the level joined
// (after compaction: the candidate's slot holds an entry of this level that it did
// not claim).  Only needed when the level will not be stored.
template <typename T>
__global__ __launch_bounds__(256) void k_mark_members(LevelArgs<T> A, uint32_t ncand) {
    if (!A.bound_level && uniform64(A.ctr->first_sol) == ~0ull) return;
    if (uniform(A.ctr->overflow) || uniform(A.ctr->n_new) > A.arena_cap) return;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < ncand; x += gridDim.x * blockDim.x) {
        const uint32_t h = A.cand_slot[x];
        if (h == NO_SLOT) continue;
        const uint32_t v = A.tval[h];
        if (!(v & VAL_SETTLED)) continue;
        const uint32_t g = v & ~VAL_SETTLED;
        if (g < A.level_base) continue;
        const uint32_t q = A.store[g] - A.level_base;
        if (A.claimer[q] != x) A.has_member[q] = 1u;
    }
}

// Tiles spread over several workgroups: combined partial results -> claims.
template <typename T>
__global__ __launch_bounds__(256) void k_probe(LevelArgs<T> A, uint32_t ncand) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < ncand; x += gridDim.x * blockDim.x) {
        const bool bad = (A.cand_viol[x >> 5] >> (x & 31u)) & 1u;
        if (!bad) atomicMin(&A.ctr->first_sol, (unsigned long long)x);
        uint32_t claim;
        A.cand_slot[x] = probe_claim<T>(A, finish_fp(A.cand_fp[x], A.fp_mask), x, claim);
        if (A.cand_claim) A.cand_claim[x] = claim;
    }
}

// ---------------------------------------------------------------------------
// One candidate's matrix, by canonical index (materialize, fallback)
// ---------------------------------------------------------------------------
template <typename T, bool MW, int OP>
__device__ __forceinline__ T cand_word(const LevelArgs<T> &A, const T *pa, const T *pb, uint32_t r, int lane,
                                       const RowMeta<T> &m) {
    constexpr bool BIN = (OP == LTL_AND || OP == LTL_OR || OP == LTL_U || OP == OP_UC);
    return apply<T, MW, OP>(pa[r], BIN ? pb[r] : (T)0, m, A.rows, lane);
}

template <typename T>
__device__ __forceinline__ void cand_children(const LevelArgs<T> &A, uint32_t x, int &op, const T *&pa,
                                              const T *&pb) {
    const int bi = find_block_cand(A.blocks, (int)A.nblocks, x);
    const Block &b = A.blocks[bi];
    uint32_t i, j;
    cand_decode(b, x - b.cand_base, i, j);
    op = (int)b.op;
    if (op == LTL_U && A.ucarry) op = OP_UC;
    pa = (const T *)(uintptr_t)child_addr<T>(A, b, 0, i);
    pb = b.nb ? (const T *)(uintptr_t)child_addr<T>(A, b, 1, j) : pa;
}

// Writes (or compares) one candidate's matrix, one row block at a time.  The
// whole wave must call it (connectives use wave ballots and shuffles).
template <typename T, bool MW, int OP>
__device__ void cand_rowblock(const LevelArgs<T> &A, const T *pa, const T *pb, uint32_t blk, int lane,
                              T *dst) {
    const uint32_t r = blk * 64u + (uint32_t)lane;
    RowMeta<T> m = load_meta<T, MW, false>(A.rows, r, lane);
    finish_meta<T, MW>(m, lane);
    dst[r] = cand_word<T, MW, OP>(A, pa, pb, r, lane, m);
}

template <typename T, bool MW>
__device__ void cand_write_block(const LevelArgs<T> &A, int op, const T *pa, const T *pb, uint32_t blk, int lane,
                                 T *dst) {
    switch (op) {
    case LTL_ATOM: cand_rowblock<T, MW, LTL_ATOM>(A, pa, pb, blk, lane, dst); break;
    case LTL_NOT:  cand_rowblock<T, MW, LTL_NOT>(A, pa, pb, blk, lane, dst); break;
    case LTL_X:    cand_rowblock<T, MW, LTL_X>(A, pa, pb, blk, lane, dst); break;
    case LTL_F:    cand_rowblock<T, MW, LTL_F>(A, pa, pb, blk, lane, dst); break;
    case LTL_G:    cand_rowblock<T, MW, LTL_G>(A, pa, pb, blk, lane, dst); break;
    case LTL_AND:  cand_rowblock<T, MW, LTL_AND>(A, pa, pb, blk, lane, dst); break;
    case LTL_OR:   cand_rowblock<T, MW, LTL_OR>(A, pa, pb, blk, lane, dst); break;
    case LTL_U:    cand_rowblock<T, MW, LTL_U>(A, pa, pb, blk, lane, dst); break;
    default:       cand_rowblock<T, MW, OP_UC>(A, pa, pb, blk, lane, dst); break;
    }
}

// One candidate's whole matrix into dst, four row blocks per iteration so that
// every wave keeps several loads in flight.
template <typename T, bool MW, int OP>
__device__ void write_matrix(const LevelArgs<T> &A, const T *pa, const T *pb, T *dst, int lane, uint32_t rb0,
                             uint32_t NB) {
    constexpr int UNR = 4;
    constexpr bool BIN = (OP == LTL_AND || OP == LTL_OR || OP == LTL_U || OP == OP_UC);
    gptr<T> a = as_global<T>(pa);
    gptr<T> b = as_global<T>(pb);
    for (uint32_t blk = rb0; blk < NB; blk += UNR) {
        RowMeta<T> m[UNR];
        T av[UNR], bv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (blk + u < NB) {
                const uint32_t r = (blk + u) * 64u + (uint32_t)lane;
                m[u] = load_meta<T, MW, false>(A.rows, r, lane);
                av[u] = ldg(a, r);
                bv[u] = BIN ? ldg(b, r) : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (blk + u < NB) {
                const uint32_t r = (blk + u) * 64u + (uint32_t)lane;
                finish_meta<T, MW>(m[u], lane);
                stg(dst, r, apply<T, MW, OP>(av[u], bv[u], m[u], A.rows, lane));
            }
        }
    }
}

// New entries of the level.  Claim order (rep_mode 0): claim q stores the matrix
// of its claimer at level_base + q.  Representative order (rep_mode 1, the exact
// re-check after a failed compare): entry e stores the matrix of its
// representative recipe[base + e] at store[base + e].  A work item is one chunk
// of A.mat_chunk row blocks of one entry.
// ---------------------------------------------------------------------------
// Relaxed check: claims of new keys (one thread per candidate).  A slot word holds
// a tag of the key's slot hash and the claiming candidate; a candidate whose tag
// matches compares its whole key with the claimer's (a slot of this level) or with
// the entry's (a settled slot), so equal keys always meet and different keys never
// merge, whatever the slot hash (fp_mask truncates it in tests).  The smallest
// canonical index of a key's candidates wins (atomicMin), as in the exact check.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ruc_claim(LevelArgs<T> A, uint32_t ncand) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncand) return;
    const uint64_t k0 = A.cand_key[2 * (uint64_t)c], k1 = A.cand_key[2 * (uint64_t)c + 1];
    const uint64_t th = mix64(k0 ^ mix64(k1 ^ 0x9E3779B97F4A7C15ull)) & A.fp_mask;
    const uint32_t tag = (uint32_t)th | 0x80000000u;
    const unsigned long long word = ((unsigned long long)tag << 32) | c;
    uint32_t h = (uint32_t)(mix64(th) >> 32) & A.slot_mask;
    for (uint32_t n = 0; n < MAX_PROBES; ++n) {
        unsigned long long w = __hip_atomic_load(&A.tkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w == 0ull) {
            const unsigned long long prev = atomicCAS(&A.tkey[h], 0ull, word);
            if (prev == 0ull) {
                atomicMin(&A.tval[h], c);
                const uint32_t pos = claim_number(A.ctr);
                if (pos == A.abort_cap || pos == A.new_cap) atomicOr(A.full, 1u);   // the level cannot be kept
                if (pos < A.new_cap) {
                    A.new_slots[pos] = h;
                    A.claimer[pos] = c;
                } else {
                    atomicOr(&A.ctr->overflow, 1u);
                }
                A.cand_slot[c] = h;
                return;
            }
            w = prev;
        }
        if ((uint32_t)(w >> 32) == tag) {
            const uint32_t v = __hip_atomic_load(&A.tval[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long *o = (v & VAL_SETTLED) ? A.entry_key + 2 * (uint64_t)(v & ~VAL_SETTLED)
                                                             : A.cand_key + 2 * (uint64_t)(uint32_t)w;
            if (o[0] == k0 && o[1] == k1) {
                if (!(v & VAL_SETTLED)) atomicMin(&A.tval[h], c);
                A.cand_slot[c] = h;
                return;
            }
        }
        h = (h + 1) & A.slot_mask;
    }
    atomicOr(&A.ctr->overflow, 1u);
    A.cand_slot[c] = NO_SLOT;
}

// Relaxed check, tiles spread over several workgroups: the added partial sums -> keys.
template <typename T>
__global__ __launch_bounds__(256) void k_ruc_finish(LevelArgs<T> A, uint32_t ncand) {
    const bool pack = A.ruc_pack != 0;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < ncand; x += gridDim.x * blockDim.x) {
        const bool bad = (A.cand_viol[x >> 5] >> (x & 31u)) & 1u;
        if (!bad) atomicMin(&A.ctr->first_sol, (unsigned long long)x);
        uint64_t k0, k1;
        ruc_key(A.cand_fp[x], A.cand_fp[A.ruc_fpb_off + x], pack, A.ruc_bits, k0, k1);
        A.cand_key[2 * (uint64_t)x] = k0;
        A.cand_key[2 * (uint64_t)x + 1] = k1;
        A.cand_claim[x] = 0xFFFFFFFFu;
    }
}

// Relaxed check, after the compaction of a level that will be stored: each new entry
// keeps its representative's key (for later levels), and the representative is marked
// with the entry's arena slot (claim order) for the write pass, which then writes the
// representative's matrix (a claimer's may differ from it under the same key).
template <typename T>
__global__ __launch_bounds__(256) void k_ruc_entry_keys(LevelArgs<T> A) {
    if (A.bound_level || uniform64(A.ctr->first_sol) != ~0ull) return;
    const uint32_t n = level_new_count(A.ctr, A.arena_cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = A.level_base + i;
        const uint32_t x = A.recipe[g];
        A.entry_key[2 * (uint64_t)g] = A.cand_key[2 * (uint64_t)x];
        A.entry_key[2 * (uint64_t)g + 1] = A.cand_key[2 * (uint64_t)x + 1];
        A.cand_claim[x] = A.store[g] - A.level_base;
    }
}

template <typename T, bool MW>
__global__ __launch_bounds__(256) void k_materialize(LevelArgs<T> A, uint32_t rep_mode) {
    const int lane = (int)__lane_id();
    const uint32_t n_entries = uniform(level_new_count(A.ctr, A.arena_cap));
    const uint32_t NB = A.rows.NB;
    const uint32_t chunk = A.mat_chunk;
    const uint32_t nchunk = (NB + chunk - 1) / chunk;
    const uint32_t nwork = n_entries * nchunk;
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t w = wave; w < nwork; w += nwaves) {
        const uint32_t e = w / nchunk, q = w - e * nchunk;
        const uint32_t rb0 = q * chunk, rb1 = min(NB, rb0 + chunk);
        const uint32_t x = uniform(rep_mode ? A.recipe[A.level_base + e] : A.claimer[e]);
        const uint32_t pos = rep_mode ? uniform(A.store[A.level_base + e]) : A.level_base + e;
        int op;
        const T *pa, *pb;
        cand_children<T>(A, x, op, pa, pb);
        op = (int)uniform((uint32_t)op);
        pa = (const T *)uniform64((uint64_t)(uintptr_t)pa);
        pb = (const T *)uniform64((uint64_t)(uintptr_t)pb);
        T *dst = (T *)(uintptr_t)arena_addr<T>(A, pos);
        switch (op) {
        case LTL_ATOM: write_matrix<T, MW, LTL_ATOM>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_NOT:  write_matrix<T, MW, LTL_NOT>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_X:    write_matrix<T, MW, LTL_X>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_F:    write_matrix<T, MW, LTL_F>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_G:    write_matrix<T, MW, LTL_G>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_AND:  write_matrix<T, MW, LTL_AND>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_OR:   write_matrix<T, MW, LTL_OR>(A, pa, pb, dst, lane, rb0, rb1); break;
        case LTL_U:    write_matrix<T, MW, LTL_U>(A, pa, pb, dst, lane, rb0, rb1); break;
        default:       write_matrix<T, MW, OP_UC>(A, pa, pb, dst, lane, rb0, rb1); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Exact fallback for fingerprint collisions (rare; forced in tests by
// truncating fingerprints).  One workgroup handles the colliders strictly in
// canonical order: each is compared in full with every cached matrix of equal
// fingerprint along its probe sequence; if none is equal it becomes a new
// representative in the first empty slot.  Sequential, hence deterministic.
// ---------------------------------------------------------------------------
template <typename T, bool MW>
__device__ bool fb_equal(const LevelArgs<T> &A, const T *target, int t_op, const T *t_pa, const T *t_pb,
                         uint32_t *s_flag, int lane, int wv, int nw) {
    // compares A.stage with `target` (stored) or with the recomputation of (t_op, t_pa, t_pb)
    if (threadIdx.x == 0) *s_flag = 0;
    __syncthreads();
    for (uint32_t blk = (uint32_t)wv; blk < A.rows.NB; blk += (uint32_t)nw) {
        const uint32_t r = blk * 64u + (uint32_t)lane;
        T tw;
        if (target) {
            tw = target[r];
        } else {
            RowMeta<T> m = load_meta<T, MW, false>(A.rows, r, lane);
            finish_meta<T, MW>(m, lane);
            switch (t_op) {
            case LTL_ATOM: tw = cand_word<T, MW, LTL_ATOM>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_NOT:  tw = cand_word<T, MW, LTL_NOT>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_X:    tw = cand_word<T, MW, LTL_X>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_F:    tw = cand_word<T, MW, LTL_F>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_G:    tw = cand_word<T, MW, LTL_G>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_AND:  tw = cand_word<T, MW, LTL_AND>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_OR:   tw = cand_word<T, MW, LTL_OR>(A, t_pa, t_pb, r, lane, m); break;
            case LTL_U:    tw = cand_word<T, MW, LTL_U>(A, t_pa, t_pb, r, lane, m); break;
            default:       tw = cand_word<T, MW, OP_UC>(A, t_pa, t_pb, r, lane, m); break;
            }
        }
        if (__ballot(tw != A.stage[r]) != 0ull && lane == 0) atomicOr(s_flag, 1u);
    }
    __syncthreads();
    bool eq = (*s_flag == 0);
    __syncthreads();
    return eq;
}

template <typename T, bool MW>
__global__ __launch_bounds__(256) void k_fallback(LevelArgs<T> A, uint32_t nwords, uint32_t ncand) {
    __shared__ unsigned long long s_part[4];
    __shared__ uint32_t s_flag;
    __shared__ unsigned long long s_key;
    __shared__ uint32_t s_val;
    __shared__ uint32_t s_words[256];
    const int lane = (int)__lane_id();
    const int wv = (int)(threadIdx.x >> 6);
    const int nw = (int)(blockDim.x >> 6);
    // the collider bitmap is read a block-wide chunk at a time (one coalesced word per
    // thread); chunks without a collider are skipped, the others are walked word by word
    for (uint32_t base = 0; base < nwords; base += blockDim.x) {
        const uint32_t mine = (base + threadIdx.x < nwords) ? A.coll_bits[base + threadIdx.x] : 0u;
        if (!__syncthreads_or(mine != 0u)) continue;
        s_words[threadIdx.x] = mine;
        __syncthreads();
      for (uint32_t k = 0; k < blockDim.x && base + k < nwords; ++k) {
        const uint32_t wi = base + k;
        uint32_t bits = s_words[k];
        while (bits) {
            const uint32_t x = wi * 32u + (uint32_t)__ffs(bits) - 1u;
            bits &= bits - 1u;
            if (x >= ncand) break;
            int op;
            const T *pa, *pb;
            cand_children<T>(A, x, op, pa, pb);
            // stage the collider's matrix and its fingerprint
            uint64_t acc = 0;
            for (uint32_t blk = (uint32_t)wv; blk < A.rows.NB; blk += (uint32_t)nw) {
                cand_write_block<T, MW>(A, op, pa, pb, blk, lane, A.stage);
            }
            __syncthreads();
            for (uint32_t blk = (uint32_t)wv; blk < A.rows.NB; blk += (uint32_t)nw) {
                const uint32_t r = blk * 64u + (uint32_t)lane;
                RowMeta<T> m = load_meta<T, MW, true>(A.rows, r, lane);
                fp_add<T>(acc, A.stage[r], m);
            }
            acc = wave_sum(acc);
            if (lane == 0) s_part[wv] = acc;
            __syncthreads();
            uint64_t fp = 0;
            for (int k = 0; k < nw; ++k) fp += s_part[k];
            fp = finish_fp(fp, A.fp_mask);
            uint32_t h = (uint32_t)(mix64(fp) >> 32) & A.slot_mask;
            for (uint32_t n = 0; n < MAX_PROBES; ++n) {
                // thread 0 reads the slot; everyone acts on the same copy
                if (threadIdx.x == 0) { s_key = A.tkey[h]; s_val = A.tval[h]; }
                __syncthreads();
                const unsigned long long k = s_key;
                const uint32_t v = s_val;
                __syncthreads();
                if (k == 0ull) {
                    if (threadIdx.x == 0) {
                        A.tkey[h] = fp;
                        A.tval[h] = x;
                        A.fb_bits[x >> 5] |= 1u << (x & 31u);
                        const uint32_t pos = A.ctr->n_new;
                        A.ctr->n_new = pos + 1;
                        A.ctr->n_fallback_new += 1;
                        if (pos < A.new_cap) {
                            A.new_slots[pos] = h;
                            A.new_owner[pos] = x;
                        } else {
                            A.ctr->overflow = 1;
                        }
                    }
                    __syncthreads();
                    break;
                }
                if (k == (unsigned long long)fp) {
                    const T *target = nullptr;
                    int t_op = 0;
                    const T *t_pa = nullptr, *t_pb = nullptr;
                    if (v & VAL_SETTLED) {
                        target = (const T *)(uintptr_t)arena_addr<T>(A, A.store[v & ~VAL_SETTLED]);
                    } else if ((A.fb_bits[v >> 5] >> (v & 31u)) & 1u) {
                        cand_children<T>(A, v, t_op, t_pa, t_pb);
                    } else {
                        target = (const T *)(uintptr_t)arena_addr<T>(
                            A, A.store[A.level_base + rank_of(A.bitmap, A.wordpre, v)]);
                    }
                    if (fb_equal<T, MW>(A, target, t_op, t_pa, t_pb, &s_flag, lane, wv, nw)) break;
                }
                h = (h + 1) & A.slot_mask;
                if (n + 1 == MAX_PROBES && threadIdx.x == 0) A.ctr->overflow = 1;
            }
            __syncthreads();
        }
      }
        __syncthreads();     // s_words is rewritten by the next chunk
    }
}

// ---------------------------------------------------------------------------
// Compaction of representatives: bitmap -> word prefix -> entry ids
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t &total) {
    const int lane = (int)__lane_id();
    const int wv = (int)(threadIdx.x >> 6);
    const int nwv = (int)(blockDim.x >> 6);
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, (unsigned)o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_tmp[wv] = inc;
    __syncthreads();
    uint32_t wbase = 0;
    total = 0;
    for (int k = 0; k < nwv; ++k) {
        uint32_t t = s_tmp[k];
        if (k < wv) wbase += t;
        total += t;
    }
    __syncthreads();
    return wbase + inc - v;
}

constexpr int SCAN_WPT = 8;                       // bitmap words per thread
constexpr int SCAN_CHUNK = 256 * SCAN_WPT;        // bitmap words per block

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *bits, uint32_t nw, uint32_t *chunk_sums) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t base = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_WPT;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_WPT; ++k)
        if (base + k < nw) s += (uint32_t)__popc(bits[base + k]);
    uint32_t total;
    block_exclusive_scan(s, s_tmp, total);
    if (threadIdx.x == 0) chunk_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_chunks(uint32_t *chunk_sums, uint32_t nchunks) {
    __shared__ uint32_t s_tmp[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nchunks; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nchunks ? chunk_sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, s_tmp, total);
        if (i < nchunks) chunk_sums[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *bits, uint32_t nw, const uint32_t *chunk_sums,
                                                    uint32_t *wordpre) {
    __shared__ uint32_t s_tmp[4];
    const uint32_t base = blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_WPT;
    uint32_t c[SCAN_WPT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_WPT; ++k) {
        c[k] = (base + k < nw) ? (uint32_t)__popc(bits[base + k]) : 0u;
        s += c[k];
    }
    uint32_t total;
    uint32_t run = chunk_sums[blockIdx.x] + block_exclusive_scan(s, s_tmp, total);
#pragma unroll
    for (int k = 0; k < SCAN_WPT; ++k) {
        if (base + k < nw) wordpre[base + k] = run;
        run += c[k];
    }
}

// The number of new groups of the level is read on the device (no host round
// trip between the level's kernels); a level whose new entries would not fit
// the arena (or the slot list) is marked in ctr->overflow and left alone.
__device__ __forceinline__ uint32_t level_new_count(const Counters *ctr, uint32_t cap) {
    const uint32_t n = ctr->n_new;
    return (n <= cap && !ctr->overflow) ? n : 0u;
}

// representatives -> recipes (entry order = canonical order of the representative),
// and settlement of the level's slots: owner index -> global entry id.  The owner
// of each new slot is recorded (new_owner) for a re-pass after the exact fallback.
// The matrix of claim i sits at arena position level_base + i (store[]).
__device__ __forceinline__ void settle_slot(uint32_t i, const uint32_t *new_slots, uint32_t *tval,
                                            const uint32_t *bitmap, const uint32_t *wordpre, uint32_t *recipe,
                                            uint32_t level_base, uint32_t *entry_slot, uint32_t *new_owner,
                                            uint32_t *store, bool repass) {
    const uint32_t s = new_slots[i];
    const uint32_t x = repass ? new_owner[i] : tval[s];
    if (!repass) new_owner[i] = x;
    const uint32_t g = level_base + rank_of(bitmap, wordpre, x);
    recipe[g] = x;
    entry_slot[g] = s;
    store[g] = level_base + i;
    tval[s] = VAL_SETTLED | g;
}

// Small levels (at most SMALL_WORDS bitmap words): representative bits, their
// ordered prefix and the recipes in one workgroup of 1024 threads.
constexpr uint32_t SMALL_WPT = 8;
constexpr uint32_t SMALL_WORDS = 1024 * SMALL_WPT;

__global__ __launch_bounds__(1024) void k_compact_small(const uint32_t *new_slots, const Counters *ctr, uint32_t cap,
                                                        uint32_t *tval, uint32_t *bitmap, uint32_t nw,
                                                        uint32_t *wordpre, uint32_t *recipe, uint32_t level_base,
                                                        uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store) {
    __shared__ uint32_t s_tmp[16];
    const uint32_t n = level_new_count(ctr, cap);
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t x = tval[new_slots[i]];
        atomicOr(&bitmap[x >> 5], 1u << (x & 31u));
    }
    __syncthreads();
    const uint32_t base = threadIdx.x * SMALL_WPT;
    uint32_t c[SMALL_WPT];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < SMALL_WPT; ++k) {
        c[k] = (base + k < nw) ? (uint32_t)__popc(__hip_atomic_load(&bitmap[base + k], __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT)) : 0u;
        sum += c[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, s_tmp, total);
#pragma unroll
    for (uint32_t k = 0; k < SMALL_WPT; ++k) {
        if (base + k < nw) wordpre[base + k] = run;
        run += c[k];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        settle_slot(i, new_slots, tval, bitmap, wordpre, recipe, level_base, entry_slot, new_owner, store, false);
}

// slot owners -> representative bits
__global__ void k_mark(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, const uint32_t *tval,
                       uint32_t *bitmap) {
    const uint32_t n = level_new_count(ctr, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t x = tval[new_slots[i]];
        atomicOr(&bitmap[x >> 5], 1u << (x & 31u));
    }
}

__global__ void k_or_bits(uint32_t *dst, const uint32_t *src, uint32_t nw) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) dst[i] |= src[i];
}

__global__ void k_scatter(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, uint32_t *tval,
                          const uint32_t *bitmap, const uint32_t *wordpre, uint32_t *recipe, uint32_t level_base,
                          uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store, uint32_t repass) {
    const uint32_t n = level_new_count(ctr, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        settle_slot(i, new_slots, tval, bitmap, wordpre, recipe, level_base, entry_slot, new_owner, store,
                    repass != 0);
}

// Zero two word ranges in one launch (a level's bitmaps and its member flags).  A
// 16-byte-aligned range is cleared in 16-byte stores, its last n % 4 words one by one.
__device__ inline void zero_words(uint32_t *p, uint64_t n, uint64_t t, uint64_t stride) {
    uint64_t head = 0;
    if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        const uint64_t n4 = n >> 2;
        uint4 *q = reinterpret_cast<uint4 *>(p);
        for (uint64_t i = t; i < n4; i += stride) q[i] = make_uint4(0u, 0u, 0u, 0u);
        head = n4 << 2;
    }
    for (uint64_t i = head + t; i < n; i += stride) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_zero2(uint32_t *a, uint64_t na, uint32_t *b, uint64_t nb) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    zero_words(a, na, t, stride);
    zero_words(b, nb, t, stride);
}

// return the slots of a finished job to the empty state
__global__ void k_clear_slots(const uint32_t *entry_slot, uint32_t n, unsigned long long *tkey, uint32_t *tval) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t s = entry_slot[i];
        tkey[s] = 0ull;
        tval[s] = VAL_OPEN;
    }
}

// ---------------------------------------------------------------------------
// Specification intake
// ---------------------------------------------------------------------------
__global__ void k_table_init(unsigned long long *tkey, uint32_t *tval, uint64_t nslots) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
         i += (uint64_t)gridDim.x * blockDim.x) {
        tkey[i] = 0ull;
        tval[i] = VAL_OPEN;
    }
}

// Atom matrices: bit (W-1-i) of word w of trace t for proposition p is p in tr_t[w*W + i].
// One thread per (row, bit): the W threads of a row read W consecutive letters
// (coalesced), and each proposition's word is one wave ballot, bit-reversed so
// that position 0 lands in the most significant bit.  Dead rows get zero words.
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const uint32_t *letters, const uint64_t *offsets,
                                              const uint32_t *row_trace, const uint32_t *row_word, uint32_t R,
                                              uint32_t nprops, T *atoms, Counters *ctr) {
    constexpr uint32_t BITS = (uint32_t)Word<T>::BITS;
    const uint32_t lane = (uint32_t)__lane_id();
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = (uint32_t)(g / BITS);          // whole waves: R * BITS is a multiple of 64
    const uint32_t i = (uint32_t)(g % BITS);
    uint32_t lt = 0;
    if (r < R) {
        const uint32_t t = row_trace[r];
        if (t != 0xFFFFFFFFu) {
            const uint64_t off = offsets[t];
            const uint64_t len = offsets[t + 1] - off;
            const uint64_t pos = (uint64_t)row_word[r] * BITS + i;
            if (pos < len) lt = letters[off + pos];
        }
    }
    for (uint32_t p = 0; p < nprops; ++p) {
        const uint64_t m = __ballot((lt >> p) & 1u);
        if (r < R && i == 0) {
            T w;
            if constexpr (BITS == 32) w = (T)__builtin_bitreverse32((uint32_t)(m >> (lane & 32u)));
            else w = (T)__builtin_bitreverse64(m);
            atoms[(size_t)p * R + r] = w;
        }
    }
    // letters naming a missing proposition (validation): one atomic per wave that holds one
    uint32_t lor = nprops < 32 ? (lt >> nprops) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lor |= (uint32_t)__shfl_xor((int)lor, o);
    if (lane == 0 && lor) atomicOr(&ctr->letter_or, lor << nprops);
}

// Per-trace fingerprint (length and letters), for the P/N disjointness check (equal
// fingerprints are compared exactly on the host): one wave per trace, the sum of a mix of
// each (position, letter) pair plus a mix of the length.
__global__ __launch_bounds__(256) void k_trace_fp(const uint32_t *letters, const uint64_t *offsets, uint32_t ntr,
                                                  uint64_t *out) {
    const uint32_t t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;     // wave-uniform
    const uint32_t lane = (uint32_t)__lane_id();
    if (t >= ntr) return;
    const uint64_t off = offsets[t], len = offsets[t + 1] - off;
    uint64_t h = 0;
    for (uint64_t i = lane; i < len; i += 64) h += mix64((i << 32) ^ (uint64_t)letters[off + i] ^ 0x2545f4914f6cdd1dull);
    h = wave_sum(h);
    if (lane == 0) out[t] = h + mix64(len + 0x9e3779b97f4a7c15ull);
}

// ---------------------------------------------------------------------------
// Formula evaluation (position-0 truth of a given formula on every trace)
// ---------------------------------------------------------------------------
// One node of a formula: its whole matrix from its children's, one row block per
// wave (traces never straddle a row block, so the blocks are independent).
template <typename T, bool MW, int OP>
__device__ __forceinline__ void node_block(const Rows<T> &rw, const T *pa, const T *pb, T *dst, uint32_t blk,
                                           int lane) {
    constexpr bool BIN = (OP == LTL_AND || OP == LTL_OR || OP == LTL_U);
    const uint32_t r = blk * 64u + (uint32_t)lane;
    RowMeta<T> m = load_meta<T, MW, false>(rw, r, lane);
    finish_meta<T, MW>(m, lane);
    const T a = ldg(as_global<T>(pa), r);
    const T b = BIN ? ldg(as_global<T>(pb), r) : (T)0;
    stg(dst, r, apply<T, MW, OP>(a, b, m, rw, lane));
}

template <typename T, bool MW>
__global__ __launch_bounds__(256) void k_formula_node(Rows<T> rw, int op, const T *pa, const T *pb, T *dst) {
    const int lane = (int)__lane_id();
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t blk = wave; blk < rw.NB; blk += nwaves) {
        switch (op) {
        case LTL_NOT: node_block<T, MW, LTL_NOT>(rw, pa, pb, dst, blk, lane); break;
        case LTL_AND: node_block<T, MW, LTL_AND>(rw, pa, pb, dst, blk, lane); break;
        case LTL_OR:  node_block<T, MW, LTL_OR>(rw, pa, pb, dst, blk, lane); break;
        case LTL_X:   node_block<T, MW, LTL_X>(rw, pa, pb, dst, blk, lane); break;
        case LTL_F:   node_block<T, MW, LTL_F>(rw, pa, pb, dst, blk, lane); break;
        case LTL_G:   node_block<T, MW, LTL_G>(rw, pa, pb, dst, blk, lane); break;
        default:      node_block<T, MW, LTL_U>(rw, pa, pb, dst, blk, lane); break;
        }
    }
}

// Position 0 of each trace (the top bit of its first word) -> one byte per trace.
template <typename T>
__global__ void k_first_bits(const T *cm, const uint32_t *row_trace, const uint32_t *row_word, uint32_t R,
                             uint8_t *out) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint32_t t = row_trace[r];
    if (t == 0xFFFFFFFFu || row_word[r] != 0u) return;
    out[t] = (uint8_t)((cm[r] >> (Word<T>::BITS - 1)) & (T)1);
}

// ---------------------------------------------------------------------------
// Launchers (host side of this translation unit)
// ---------------------------------------------------------------------------
// Multi-word kernels (lanes of one trace exchange bits) exist for 64-bit words only.
template <typename T, bool MW, bool V>
static void launch_cls(const LevelArgs<T> &A, int cls, const Block *blocks, uint32_t nb, uint32_t nt, uint32_t ch,
                       uint32_t grid, hipStream_t s) {
    switch (cls) {
    case CLS_UNARY: hipLaunchKernelGGL((k_level<T, MW, V, CLS_UNARY>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_ANDOR: hipLaunchKernelGGL((k_level<T, MW, V, CLS_ANDOR>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_U:     hipLaunchKernelGGL((k_level<T, MW, V, CLS_U>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    default:        hipLaunchKernelGGL((k_level<T, MW, V, CLS_UC>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    }
}

// Multi-word kernels (lanes of one trace exchange bits) exist for 64-bit words only.
template <typename T>
hipError_t Launch<T>::level(const LevelArgs<T> &A, bool mw, bool verify, int cls, const Block *blocks,
                            uint32_t nblocks, uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            if (verify) launch_cls<T, true, true>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
            else launch_cls<T, true, false>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
            return hipGetLastError();
        }
    }
    if (verify) launch_cls<T, false, true>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
    else launch_cls<T, false, false>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
    return hipGetLastError();
}

template <typename T, bool MW>
static void launch_ruc_cls(const LevelArgs<T> &A, int cls, const Block *blocks, uint32_t nb, uint32_t nt,
                           uint32_t grid, hipStream_t s) {
    const uint32_t ch = A.rows.NB;
    switch (cls) {
    case CLS_UNARY: hipLaunchKernelGGL((k_level<T, MW, false, CLS_UNARY, false, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_ANDOR: hipLaunchKernelGGL((k_level<T, MW, false, CLS_ANDOR, false, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_U:     hipLaunchKernelGGL((k_level<T, MW, false, CLS_U, false, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    default:        hipLaunchKernelGGL((k_level<T, MW, false, CLS_UC, false, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    }
}

template <typename T>
hipError_t Launch<T>::level_ruc(const LevelArgs<T> &A, bool mw, int cls, const Block *blocks, uint32_t nblocks,
                                uint32_t ntiles, uint32_t grid, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            launch_ruc_cls<T, true>(A, cls, blocks, nblocks, ntiles, grid, s);
            return hipGetLastError();
        }
    }
    launch_ruc_cls<T, false>(A, cls, blocks, nblocks, ntiles, grid, s);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::ruc_claim(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, (ncand + 255) / 256);
    hipLaunchKernelGGL((k_ruc_claim<T>), dim3(grid), dim3(256), 0, s, A, ncand);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::ruc_entry_keys(const LevelArgs<T> &A, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((A.new_cap + 255) / 256, 2048));
    hipLaunchKernelGGL((k_ruc_entry_keys<T>), dim3(grid), dim3(256), 0, s, A);
    return hipGetLastError();
}

template <typename T, bool MW, int PASS>
static void launch_stg_cls(const LevelArgs<T> &A, int cls, const Block *blocks, uint32_t nb, uint32_t ng, uint32_t ch,
                           uint32_t grid, hipStream_t s) {
    switch (cls) {
    case CLS_ANDOR: hipLaunchKernelGGL((k_level_stg<T, MW, PASS, CLS_ANDOR>), dim3(grid), dim3(256), 0, s, A, blocks, nb, ng, ch); break;
    case CLS_U:     hipLaunchKernelGGL((k_level_stg<T, MW, PASS, CLS_U>), dim3(grid), dim3(256), 0, s, A, blocks, nb, ng, ch); break;
    default:        hipLaunchKernelGGL((k_level_stg<T, MW, PASS, CLS_UC>), dim3(grid), dim3(256), 0, s, A, blocks, nb, ng, ch); break;
    }
}

template <typename T, bool MW>
static void launch_stg(const LevelArgs<T> &A, int pass, int cls, const Block *blocks, uint32_t nb, uint32_t ng,
                       uint32_t ch, uint32_t grid, hipStream_t s) {
    if (pass == 0) launch_stg_cls<T, MW, 0>(A, cls, blocks, nb, ng, ch, grid, s);
    else if (pass == 1) launch_stg_cls<T, MW, 1>(A, cls, blocks, nb, ng, ch, grid, s);
    else launch_stg_cls<T, MW, 2>(A, cls, blocks, nb, ng, ch, grid, s);
}

template <typename T>
hipError_t Launch<T>::level_staged(const LevelArgs<T> &A, bool mw, int pass, int cls, const Block *blocks,
                                   uint32_t nblocks, uint32_t ngroups, uint32_t chunk, uint32_t grid, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            launch_stg<T, true>(A, pass, cls, blocks, nblocks, ngroups, chunk, grid, s);
            return hipGetLastError();
        }
    }
    launch_stg<T, false>(A, pass, cls, blocks, nblocks, ngroups, chunk, grid, s);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::mark_members(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((ncand + 255) / 256, 4096));
    hipLaunchKernelGGL((k_mark_members<T>), dim3(grid), dim3(256), 0, s, A, ncand);
    return hipGetLastError();
}

template <typename T, bool MW>
static void launch_write_cls(const LevelArgs<T> &A, int cls, const Block *blocks, uint32_t nb, uint32_t nt,
                             uint32_t ch, uint32_t grid, hipStream_t s) {
    switch (cls) {
    case CLS_UNARY: hipLaunchKernelGGL((k_level<T, MW, false, CLS_UNARY, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_ANDOR: hipLaunchKernelGGL((k_level<T, MW, false, CLS_ANDOR, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    case CLS_U:     hipLaunchKernelGGL((k_level<T, MW, false, CLS_U, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    default:        hipLaunchKernelGGL((k_level<T, MW, false, CLS_UC, true>), dim3(grid), dim3(256), 0, s, A, blocks, nb, nt, ch); break;
    }
}

template <typename T>
hipError_t Launch<T>::write_pass(const LevelArgs<T> &A, bool mw, int cls, const Block *blocks, uint32_t nblocks,
                                 uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            launch_write_cls<T, true>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
            return hipGetLastError();
        }
    }
    launch_write_cls<T, false>(A, cls, blocks, nblocks, ntiles, chunk, grid, s);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::probe(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((ncand + 255) / 256, 4096));
    hipLaunchKernelGGL((k_probe<T>), dim3(grid), dim3(256), 0, s, A, ncand);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::verify_all(const LevelArgs<T> &A, bool mw, const Block *blocks, uint32_t nblocks,
                                 uint32_t ntiles, uint32_t chunk, uint32_t grid, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            hipLaunchKernelGGL((k_level_all<T, true, true>), dim3(grid), dim3(256), 0, s, A, blocks, nblocks, ntiles, chunk);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_level_all<T, false, true>), dim3(grid), dim3(256), 0, s, A, blocks, nblocks, ntiles, chunk);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::level_wg(const LevelArgs<T> &A, bool mw, const Block *blocks, uint32_t nblocks,
                               uint32_t ntiles, uint32_t grid, hipStream_t s, bool ruc) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            if (ruc)
                hipLaunchKernelGGL((k_level_wg<T, true, true>), dim3(grid), dim3(64 * wg_waves<true>()), 0, s, A,
                                   blocks, nblocks, ntiles);
            else
                hipLaunchKernelGGL((k_level_wg<T, true>), dim3(grid), dim3(64 * wg_waves<true>()), 0, s, A, blocks,
                                   nblocks, ntiles);
            return hipGetLastError();
        }
    }
    if (ruc)
        hipLaunchKernelGGL((k_level_wg<T, false, true>), dim3(grid), dim3(64 * wg_waves<false>()), 0, s, A, blocks,
                           nblocks, ntiles);
    else
        hipLaunchKernelGGL((k_level_wg<T, false>), dim3(grid), dim3(64 * wg_waves<false>()), 0, s, A, blocks,
                           nblocks, ntiles);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::ruc_finish(const LevelArgs<T> &A, uint32_t ncand, hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((ncand + 255) / 256, 4096));
    hipLaunchKernelGGL((k_ruc_finish<T>), dim3(grid), dim3(256), 0, s, A, ncand);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::materialize(const LevelArgs<T> &A, bool mw, uint32_t rep_mode, uint32_t grid,
                                  hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            hipLaunchKernelGGL((k_materialize<T, true>), dim3(grid), dim3(256), 0, s, A, rep_mode);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_materialize<T, false>), dim3(grid), dim3(256), 0, s, A, rep_mode);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::fallback(const LevelArgs<T> &A, bool mw, uint32_t nwords, uint32_t ncand, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            hipLaunchKernelGGL((k_fallback<T, true>), dim3(1), dim3(256), 0, s, A, nwords, ncand);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_fallback<T, false>), dim3(1), dim3(256), 0, s, A, nwords, ncand);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::pack(const uint32_t *letters, const uint64_t *offsets, const uint32_t *row_trace,
                           const uint32_t *row_word, uint32_t R, uint32_t nprops, T *atoms, Counters *ctr,
                           hipStream_t s) {
    const uint64_t threads = (uint64_t)R * Word<T>::BITS;
    hipLaunchKernelGGL((k_pack<T>), dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, letters, offsets, row_trace,
                       row_word, R, nprops, atoms, ctr);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::formula_node(const Rows<T> &rw, bool mw, int op, const T *pa, const T *pb, T *dst,
                                   hipStream_t s) {
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((rw.NB + 3) / 4, 4096));
    if constexpr (sizeof(T) == 8) {
        if (mw) {
            hipLaunchKernelGGL((k_formula_node<T, true>), dim3(grid), dim3(256), 0, s, rw, op, pa, pb, dst);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_formula_node<T, false>), dim3(grid), dim3(256), 0, s, rw, op, pa, pb, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::first_bits(const T *cm, const uint32_t *row_trace, const uint32_t *row_word, uint32_t R,
                                 uint8_t *out, hipStream_t s) {
    hipLaunchKernelGGL((k_first_bits<T>), dim3((R + 255) / 256), dim3(256), 0, s, cm, row_trace, row_word, R, out);
    return hipGetLastError();
}

template struct Launch<uint32_t>;
template struct Launch<uint64_t>;

hipError_t launch_scan(const uint32_t *bits, uint32_t nw, uint32_t *chunk_sums, uint32_t *wordpre, hipStream_t s) {
    const uint32_t nchunks = (nw + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nchunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nchunks), dim3(256), 0, s, bits, nw, chunk_sums);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(256), 0, s, chunk_sums, nchunks);
    hipLaunchKernelGGL(k_scan_apply, dim3(nchunks), dim3(256), 0, s, bits, nw, chunk_sums, wordpre);
    return hipGetLastError();
}

hipError_t launch_mark(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, const uint32_t *tval,
                       uint32_t *bitmap, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_mark, dim3(grid), dim3(256), 0, s, new_slots, ctr, cap, tval, bitmap);
    return hipGetLastError();
}

hipError_t launch_compact_small(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, uint32_t *tval,
                                uint32_t *bitmap, uint32_t nw, uint32_t *wordpre, uint32_t *recipe,
                                uint32_t level_base, uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_compact_small, dim3(1), dim3(1024), 0, s, new_slots, ctr, cap, tval, bitmap, nw, wordpre,
                       recipe, level_base, entry_slot, new_owner, store);
    return hipGetLastError();
}

hipError_t launch_or_bits(uint32_t *dst, const uint32_t *src, uint32_t nw, hipStream_t s) {
    if (!nw) return hipSuccess;
    hipLaunchKernelGGL(k_or_bits, dim3((nw + 255) / 256), dim3(256), 0, s, dst, src, nw);
    return hipGetLastError();
}

hipError_t launch_scatter(const uint32_t *new_slots, const Counters *ctr, uint32_t cap, uint32_t *tval,
                          const uint32_t *bitmap, const uint32_t *wordpre, uint32_t *recipe, uint32_t level_base,
                          uint32_t *entry_slot, uint32_t *new_owner, uint32_t *store, bool repass, uint32_t grid,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, s, new_slots, ctr, cap, tval, bitmap, wordpre, recipe,
                       level_base, entry_slot, new_owner, store, repass ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_zero2(uint32_t *a, uint64_t na, uint32_t *b, uint64_t nb, hipStream_t s) {
    if (!a) na = 0;
    if (!b) nb = 0;
    const uint64_t n = std::max(na, nb);
    if (!n) return hipSuccess;
    const uint64_t g = std::min<uint64_t>((n / 4 + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(k_zero2, dim3((uint32_t)g), dim3(256), 0, s, a, na, b, nb);
    return hipGetLastError();
}

hipError_t launch_clear_slots(const uint32_t *entry_slot, uint32_t n, unsigned long long *tkey, uint32_t *tval,
                              hipStream_t s) {
    if (!n) return hipSuccess;
    const uint32_t g = std::min<uint32_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_clear_slots, dim3(g), dim3(256), 0, s, entry_slot, n, tkey, tval);
    return hipGetLastError();
}

hipError_t launch_table_init(unsigned long long *tkey, uint32_t *tval, uint64_t nslots, hipStream_t s) {
    uint64_t g = (nslots + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_table_init, dim3((uint32_t)g), dim3(256), 0, s, tkey, tval, nslots);
    return hipGetLastError();
}

hipError_t launch_trace_fp(const uint32_t *letters, const uint64_t *offsets, uint32_t ntr, uint64_t *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_trace_fp, dim3((ntr + 3) / 4), dim3(256), 0, s, letters, offsets, ntr, out);
    return hipGetLastError();
}

}  // namespace ltl
