// Divide and conquer (Sec. 6): deterministic and random splitting of a
// specification into sub-specifications small enough for the enumerator, and
// recombination of the learned formulas.  Host code over the public C-ABI: the
// leaves run the learner of Sec. 3 (ltl_learn below the cost of the overfitting
// formula, else that formula), and "the traces a formula accepts" is ltl_holds,
// the same kernels evaluating the formula on the device.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "ltl.h"

namespace {

using Trace = std::vector<uint32_t>;
using Traces = std::vector<const Trace *>;
using Formula = std::vector<ltl_node>;

struct Ctx {
    ltl_ctx *ctx;
    ltl_opset ops;
    uint32_t A;
};

// Host specification of (P, N) (flattened letters and offsets, P first).
struct HostSpec {
    std::vector<uint32_t> letters;
    std::vector<uint64_t> offsets;
    ltl_spec spec{};
    HostSpec(uint32_t A, const Traces &P, const Traces &N) {
        offsets.push_back(0);
        for (const Traces *cls : {&P, &N})
            for (const Trace *t : *cls) {
                letters.insert(letters.end(), t->begin(), t->end());
                offsets.push_back(letters.size());
            }
        spec.num_props = A;
        spec.num_pos = (uint32_t)P.size();
        spec.num_neg = (uint32_t)N.size();
        spec.flags = 0;
        spec.letters = letters.data();
        spec.offsets = offsets.data();
    }
};

// The learner of Sec. 3: enumerate the levels below the cost of the overfitting
// formula; if none of them separates, the overfitting formula (it does).
int learn_leaf(const Ctx &c, const Traces &P, const Traces &N, Formula &out) {
    HostSpec hs(c.A, P, N);
    uint32_t n = 0;
    uint64_t co = 0;
    int st = ltl_overfit(&hs.spec, &c.ops, nullptr, 0, &n, &co);
    if (st != LTL_OK && st != LTL_E_OOM) return st;
    Formula of(n);
    st = ltl_overfit(&hs.spec, &c.ops, of.data(), n, &n, &co);
    if (st != LTL_OK) return st;
    const uint64_t bound = std::min<uint64_t>(co - 1, LTL_MAX_LEVELS - 1);
    if (bound >= 1) {
        ltl_result r;
        st = ltl_learn(c.ctx, &hs.spec, &c.ops, (uint32_t)bound, &r);
        if (st == LTL_OK) {
            out.assign(r.nodes, r.nodes + r.num_nodes);
            return LTL_OK;
        }
        if (st != LTL_NOT_FOUND) return st;
    }
    out = of;
    return LTL_OK;
}

// Position-0 truth of f on each trace (on the device).
int accepted(const Ctx &c, const Formula &f, const Traces &ts, std::vector<uint8_t> &out) {
    out.assign(ts.size(), 0);
    if (ts.empty()) return LTL_OK;
    HostSpec hs(c.A, ts, Traces());
    return ltl_holds(c.ctx, &hs.spec, f.data(), (uint32_t)f.size(), out.data());
}

// f op g as one postfix list: g's child indices shifted past f.
Formula join(uint32_t op, const Formula &f, const Formula &g) {
    Formula r = f;
    const uint32_t k = (uint32_t)f.size();
    for (ltl_node v : g) {
        if (v.op != LTL_ATOM) {
            v.a += k;
            if (v.op == LTL_AND || v.op == LTL_OR || v.op == LTL_U) v.b += k;
        }
        r.push_back(v);
    }
    r.push_back(ltl_node{op, k - 1, k + (uint32_t)g.size() - 1});
    return r;
}

// ---------------------------------------------------------------- deterministic splitting
// A formula is "absent" (has_f false) when its part had no positive trace: it
// contributes no disjunct.
int det_split(const Ctx &c, const Traces &P, const Traces &N, uint32_t w, bool &has_f, Formula &f) {
    has_f = false;
    f.clear();
    if (P.empty()) return LTL_OK;
    if (P.size() + N.size() <= w || std::max(P.size(), N.size()) <= 1) {
        int st = learn_leaf(c, P, N, f);
        has_f = st == LTL_OK;
        return st;
    }
    const size_t hp = P.size() / 2, hn = N.size() / 2;
    const Traces P1(P.begin(), P.begin() + hp), P2(P.begin() + hp, P.end());
    const Traces N1(N.begin(), N.begin() + hn), N2(N.begin() + hn, N.end());
    // one pair: phi_a = split(Pp, N1), phi_b = split(Pp, N2 in L(phi_a)); conjunction
    auto pair = [&](const Traces &Pp, bool &has, Formula &g) -> int {
        bool ha = false, hb = false;
        Formula fa, fb;
        int st = det_split(c, Pp, N1, w, ha, fa);
        if (st != LTL_OK || !ha) { has = false; return st; }
        std::vector<uint8_t> in;
        if ((st = accepted(c, fa, N2, in)) != LTL_OK) return st;
        Traces left;
        for (size_t i = 0; i < N2.size(); ++i)
            if (in[i]) left.push_back(N2[i]);
        if (!left.empty()) {
            if ((st = det_split(c, Pp, left, w, hb, fb)) != LTL_OK) return st;
        }
        has = true;
        g = hb ? join(LTL_AND, fa, fb) : fa;
        return LTL_OK;
    };
    bool h1 = false, h2 = false;
    Formula first, second;
    int st = pair(P1, h1, first);
    if (st == LTL_OK) {
        // the second pair learns from the P2 traces the first conjunction rejects
        Traces P2r;
        if (h1) {
            std::vector<uint8_t> in;
            st = accepted(c, first, P2, in);
            for (size_t i = 0; st == LTL_OK && i < P2.size(); ++i)
                if (!in[i]) P2r.push_back(P2[i]);
        } else {
            P2r = P2;
        }
        if (st == LTL_OK) st = pair(P2r, h2, second);
    }
    if (st == LTL_E_OOM) {     // the whole call again with half the window
        if (w <= 1) return LTL_E_OOM;
        return det_split(c, P, N, w / 2, has_f, f);
    }
    if (st != LTL_OK) return st;
    if (!h1) { has_f = h2; f = second; return LTL_OK; }
    has_f = true;
    f = h2 ? join(LTL_OR, first, second) : first;
    return LTL_OK;
}

// ---------------------------------------------------------------- random splitting
// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): state s advances by gamma, output = mix(s).
constexpr uint64_t SM_GAMMA = 0x9e3779b97f4a7c15ull;
uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// k of the n indices: those with the k smallest outputs of the SplitMix64 stream
// started at state seed * 2^32 + stream (output i = mix(state + (i + 1) * gamma)),
// in increasing index order.  All n when k >= n.
std::vector<uint32_t> sample_subset(uint64_t seed, uint64_t stream, uint32_t n, uint32_t k) {
    std::vector<uint32_t> idx(n);
    for (uint32_t i = 0; i < n; ++i) idx[i] = i;
    if (k >= n) return idx;
    const uint64_t s0 = (seed << 32) + stream;
    std::vector<uint64_t> key(n);
    for (uint32_t i = 0; i < n; ++i) key[i] = sm_mix(s0 + (uint64_t)(i + 1) * SM_GAMMA);
    std::nth_element(idx.begin(), idx.begin() + k, idx.end(), [&](uint32_t a, uint32_t b) {
        return key[a] != key[b] ? key[a] < key[b] : a < b;
    });
    idx.resize(k);
    std::sort(idx.begin(), idx.end());
    return idx;
}

// Formula kinds of a random-splitting part: none (no positive trace: false), true
// (no negative trace left), or a formula.
enum Kind { NONE, TRUE_F, FORMULA };

struct RandSplit {
    const Ctx &c;
    uint32_t win;
    uint64_t seed;
    uint64_t calls = 0;   // sub-specifications drawn so far (two streams each)

    int split(const Traces &P, const Traces &N, Kind &kind, Formula &f) {
        f.clear();
        if (P.empty()) { kind = NONE; return LTL_OK; }
        if (N.empty()) { kind = TRUE_F; return LTL_OK; }
        // phi11: the learner on a random sub-specification of at most w traces, the
        // classes as equal in size as the window allows; w halved on out-of-memory
        // (the whole specification when it fits, since then every trace is drawn)
        Formula f11;
        int st = LTL_E_OOM;
        for (uint32_t w = win; st == LTL_E_OOM; w /= 2) {
            if (w < 2) return LTL_E_OOM;
            const uint64_t total = std::min<uint64_t>(w, P.size() + N.size());
            uint64_t kp = std::min<uint64_t>(P.size(), (total + 1) / 2);
            const uint64_t kn = std::min<uint64_t>(N.size(), total - kp);
            kp = std::min<uint64_t>(P.size(), total - kn);
            const uint64_t q = calls++;
            Traces P0, N0;
            for (uint32_t i : sample_subset(seed, 2 * q, (uint32_t)P.size(), (uint32_t)kp)) P0.push_back(P[i]);
            for (uint32_t i : sample_subset(seed, 2 * q + 1, (uint32_t)N.size(), (uint32_t)kn)) N0.push_back(N[i]);
            st = learn_leaf(c, P0, N0, f11);
        }
        if (st != LTL_OK) return st;
        std::vector<uint8_t> aP, aN;
        if ((st = accepted(c, f11, P, aP)) != LTL_OK) return st;
        if ((st = accepted(c, f11, N, aN)) != LTL_OK) return st;
        Traces Pin, Pout, Nin, Nout;
        for (size_t i = 0; i < P.size(); ++i) (aP[i] ? Pin : Pout).push_back(P[i]);
        for (size_t i = 0; i < N.size(); ++i) (aN[i] ? Nin : Nout).push_back(N[i]);
        Kind k12, k21, k22;
        Formula f12, f21, f22;
        if ((st = split(Pin, Nin, k12, f12)) != LTL_OK) return st;
        if ((st = split(Pout, Nout, k21, f21)) != LTL_OK) return st;
        if ((st = split(Pout, Nin, k22, f22)) != LTL_OK) return st;
        Kind k1, k2;
        Formula g1, g2;
        conj(FORMULA, f11, k12, f12, k1, g1);
        conj(k21, f21, k22, f22, k2, g2);
        if (k1 == NONE) { kind = k2; f = g2; }
        else if (k2 == NONE) { kind = k1; f = g1; }
        else { kind = FORMULA; f = join(LTL_OR, g1, g2); }   // both are formulas here
        return LTL_OK;
    }

    static void conj(Kind ka, const Formula &a, Kind kb, const Formula &b, Kind &k, Formula &r) {
        if (ka == NONE || kb == NONE) { k = NONE; r.clear(); return; }
        if (kb == TRUE_F) { k = ka; r = a; return; }
        if (ka == TRUE_F) { k = kb; r = b; return; }
        k = FORMULA;
        r = join(LTL_AND, a, b);
    }
};

int check_args(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t win, uint32_t *num_nodes) {
    if (!ctx || !spec || !ops || !num_nodes || win < 1) return LTL_E_INVAL;
    if (spec->flags & LTL_SPEC_DEVICE) return LTL_E_INVAL;
    if (!spec->letters || !spec->offsets || spec->num_props < 1 || spec->num_props > 32) return LTL_E_INVAL;
    if (spec->num_pos < 1 || spec->num_neg < 1) return LTL_E_INVAL;
    if ((uint64_t)spec->num_pos + spec->num_neg > 0x7FFFFFFFull) return LTL_E_INVAL;
    return LTL_OK;
}

void split_traces(const ltl_spec *spec, std::vector<Trace> &store, Traces &P, Traces &N) {
    const uint32_t T = spec->num_pos + spec->num_neg;
    store.resize(T);
    for (uint32_t t = 0; t < T; ++t) {
        store[t].assign(spec->letters + spec->offsets[t], spec->letters + spec->offsets[t + 1]);
        (t < spec->num_pos ? P : N).push_back(&store[t]);
    }
}

int emit(const Formula &f, bool has, ltl_node *buf, uint32_t cap, uint32_t *num_nodes) {
    if (!has) { *num_nodes = 0; return LTL_OK; }
    *num_nodes = (uint32_t)f.size();
    if (f.size() > cap || !buf) return LTL_E_BUFFER;
    std::memcpy(buf, f.data(), f.size() * sizeof(ltl_node));
    return LTL_OK;
}

}  // namespace

extern "C" int ltl_det_split(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t win,
                             ltl_node *buf, uint32_t cap, uint32_t *num_nodes) {
    if (int st = check_args(ctx, spec, ops, win, num_nodes)) return st;
    std::vector<Trace> store;
    Traces P, N;
    split_traces(spec, store, P, N);
    Ctx c{ctx, *ops, spec->num_props};
    bool has = false;
    Formula f;
    int st = det_split(c, P, N, win, has, f);
    if (st != LTL_OK) return st;
    return emit(f, has, buf, cap, num_nodes);
}

extern "C" int ltl_rand_split(ltl_ctx *ctx, const ltl_spec *spec, const ltl_opset *ops, uint32_t win,
                              uint64_t seed, ltl_node *buf, uint32_t cap, uint32_t *num_nodes) {
    if (int st = check_args(ctx, spec, ops, win, num_nodes)) return st;
    if (seed >> 32) return LTL_E_INVAL;
    std::vector<Trace> store;
    Traces P, N;
    split_traces(spec, store, P, N);
    Ctx c{ctx, *ops, spec->num_props};
    RandSplit r{c, win, seed};
    Kind k;
    Formula f;
    int st = r.split(P, N, k, f);
    if (st != LTL_OK) return st;
    return emit(f, k == FORMULA, buf, cap, num_nodes);
}
