// The device tree compiler's per-thread steps and its host-side glue, shared
// by the HIP kernels (devcompile.hip) and a CPU build that runs the same steps
// in arbitrary thread interleavings (tests/csrc/devcompile_emu.cpp).
//
// It produces, for a population of prefix trees (Section 3.1), exactly the
// programs of compile_tree (prep.cpp): the same stack needs and Ershov
// evaluation order (the larger operand first, a freedom Section 6.2 gives),
// the same terminal folding, chunk cuts, instruction words, chunk numbering
// and parent-cache records.  compile_tree's right-to-left pass fixes each
// function node's values from its two operands' values; here the same values
// are computed bottom-up: one thread per terminal walks towards the root, and
// at each function the second of its two operands to arrive computes it.
// Values one thread leaves for another go through the Mem policy (coherent
// stores and loads on the device; plain ones on the CPU), and the arrival
// counter orders them: the writer's stores complete before its increment,
// the reader loads after its increment returned.
#pragma once
#include <cstdint>

#include "prep.h"

#include <algorithm>
#include <unordered_map>
#include <vector>

#if defined(__HIPCC__)
#define GPE_HD __host__ __device__
#else
#define GPE_HD
#endif

namespace gpe {

// info word of a node: stack need (bits 0..5), roots a chunk (bit 6),
// instruction form (bits 8..12: mode | first operand is the right << 3 |
// folded operand is the left << 4, as compile_tree's form)
constexpr int32_t kDcCut = 64;

struct DcNodes {
    const uint8_t* ops;
    const int64_t* offsets;            // [n_trees + 1]
    int64_t n_trees;
    int64_t n;
    const int32_t* endl;               // tree-local subtree ends
    const int32_t* parl;               // tree-local parents, -1 at a root
    int32_t* info;
    int32_t* len;                      // words the subtree emits in its own chunk
    int32_t* open;                     // nodes not yet in a chunk below; during emission: code position
    int32_t* cnt;                      // operands arrived; then, at a chunk root: its chunk id
    uint8_t* slot;                     // emission: stack slot of the node's value
    const int32_t* rec;                // record id of a recorded function node, else -1 (may be null)
    int32_t* err;
    int boolean;
    int S;                             // stack slots
    int64_t C;                         // chunk size target (at least 2)
};

struct DcChunks {
    int64_t n;
    const int64_t* root;               // global node of each chunk's root
    const int64_t* tree_start;
    const int64_t* code_off;           // global word offset of its code
    const int64_t* in_off;             // its first LOAD input (write pass)
    uint32_t* code;
    int32_t* n_in;                     // count pass output
    int32_t* inputs;                   // global chunk ids, in LOAD order
    int32_t* parent;                   // global parent chunk id (set by the parent's thread)
    int64_t* nodes;
    int32_t* max_slot;
    uint8_t* stores;
};

// One ancestor on the path from a crossover point up to the root (listed
// nearest first): the ancestor a and its other operand sib (tree-local),
// f | (the path operand is the right one) << 2, and sib's opcode.
struct DcPathLevel {
    int32_t a, sib, fside, sib_op;
};

GPE_HD inline uint32_t dc_word(uint32_t f, uint32_t mode, uint32_t d, uint32_t payload)
{
    return f | (mode << 2) | (d << 5) | (payload << kPayloadShift);
}

GPE_HD inline int64_t dc_tree_of(const DcNodes& q, int64_t g)
{
    int64_t lo = 0, hi = q.n_trees;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (q.offsets[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

GPE_HD inline bool dc_foldable(const DcNodes& q, int64_t v)
{
    const uint8_t b = q.ops[v];
    return !(b & kFuncBit) && (q.boolean || b == 0);
}

GPE_HD inline int dc_max(int a, int b) { return a > b ? a : b; }

// A terminal: need 1, one open node, one PUSH word (when not folded).
template <class Mem> GPE_HD inline void dc_leaf(const DcNodes& q, int64_t g)
{
    Mem::st(q.info + g, 1);
    Mem::st(q.len + g, 1);
    Mem::st(q.open + g, 1);
}

// The function at global index g of the tree [s, e), both operands done.
template <class Mem> GPE_HD inline void dc_func(const DcNodes& q, int64_t g, int64_t s, int64_t e)
{
    const int64_t l = g + 1, r = s + q.endl[g + 1];
    if (r <= l || r >= e) {
        Mem::err(q.err, 1);
        return;
    }
    const int32_t il = Mem::ld(q.info + l), ir = Mem::ld(q.info + r);
    bool cl = (il & kDcCut) != 0, cr = (ir & kDcCut) != 0;
    const bool fol = dc_foldable(q, l), fo_r = dc_foldable(q, r);
    auto cost_l = [&]() { return cl ? 1 : (il & 63); };
    auto cost_r = [&]() { return cr ? 1 : (ir & 63); };
    auto need_of = [&]() {
        const bool fl = !cl && fol, fr = !cr && fo_r;
        if (fl && fr) return 1;
        if (fl) return cost_r();
        if (fr) return cost_l();
        const int nl = cost_l(), nr = cost_r();
        return nl >= nr ? dc_max(nl, nr + 1) : dc_max(nr, nl + 1);
    };
    int nd = need_of();
    if (nd > q.S) {
        // both operands need a full stack: the bigger one roots a chunk of its own
        if (cost_l() >= cost_r()) {
            cl = true;
            Mem::st(q.info + l, il | kDcCut);
        } else {
            cr = true;
            Mem::st(q.info + r, ir | kDcCut);
        }
        nd = need_of();
    }
    const bool fl = !cl && fol, fr = !cr && fo_r;
    int form, len;
    if (fl && fr) {
        form = M_XX;
        len = 1;
    } else if (fl || fr) {
        form = (q.boolean || fl ? M_XS : M_SX) | (fl ? 16 : 0);
        const bool ocut = fl ? cr : cl;
        len = (ocut ? 1 : Mem::ld(q.len + (fl ? r : l))) + 1;
    } else {
        const bool first_r = !(cost_l() >= cost_r());
        form = (!first_r || q.boolean ? M_SS : M_RS) | (first_r ? 8 : 0);
        len = (cl ? 1 : Mem::ld(q.len + l)) + (cr ? 1 : Mem::ld(q.len + r)) + 1;
    }
    const int64_t o = 1 + (cl ? 1 : (int64_t)Mem::ld(q.open + l)) + (cr ? 1 : (int64_t)Mem::ld(q.open + r));
    const bool cut = o >= q.C && g != s;
    Mem::st(q.len + g, len);
    Mem::st(q.open + g, (int32_t)(o < 0x7fffffff ? o : 0x7fffffff));
    Mem::st(q.info + g, nd | (cut ? kDcCut : 0) | (form << 8));
}

// One arrival: node v (global, done) of the tree [s, e) counts itself at its
// parent.  Returns the parent when this was the parent's second operand (the
// parent is then done too), else -1.
template <class Mem> GPE_HD inline int64_t dc_step(const DcNodes& q, int64_t s, int64_t e, int64_t v)
{
    const int32_t p = q.parl[v];
    if (p < 0) return -1;
    const int64_t pg = s + p;
    if (pg >= v || pg < s) {
        Mem::err(q.err, 2);
        return -1;
    }
    Mem::publish();                                 // v's values are stored before its arrival counts
    const int32_t old = Mem::fetch_add(q.cnt + pg, 1);
    Mem::after_count();
    if (old == 0) return -1;                        // the other operand is not done yet
    dc_func<Mem>(q, pg, s, e);
    return pg;
}

// Emission of chunk k (compile_tree's scan in prefix order: an instruction's
// first operand's code starts where its own code starts, the second's after
// it, the instruction's word follows both, a recorded node's STORE follows its
// word).  write = 0: only count the chunk's LOADs.
GPE_HD inline void dc_emit(const DcNodes& q, const DcChunks& c, int64_t k, int write)
{
    const int64_t R = c.root[k], s = c.tree_start[k];
    const int64_t end = s + q.endl[R];
    auto cutp = [&](int64_t v) { return (q.info[v] & kDcCut) != 0; };
    if (!write) {
        int32_t n_in = 0;
        for (int64_t v = R; v < end;) {
            if (v != R && cutp(v)) {
                v = s + q.endl[v];
                continue;
            }
            if (q.ops[v] & kFuncBit) {
                const int64_t l = v + 1, r = s + q.endl[v + 1];
                n_in += (cutp(l) ? 1 : 0) + (cutp(r) ? 1 : 0);
            }
            ++v;
        }
        c.n_in[k] = n_in;
        return;
    }
    uint32_t* code = c.code + c.code_off[k];
    int32_t* ins = c.inputs + c.in_off[k];
    int32_t n_in = 0, max_slot = 0;
    int64_t nodes = 0;
    uint8_t stores = 0;
    auto words = [&](int64_t v) { return cutp(v) ? 1 : q.len[v]; };
    auto place = [&](int64_t ch, int32_t at, int32_t d) {
        if (cutp(ch)) {
            const int32_t id = q.cnt[ch];
            c.parent[id] = (int32_t)k;
            code[at] = dc_word(0, M_LOAD, (uint32_t)d, (uint32_t)n_in);
            ins[n_in++] = id;
        } else {
            q.open[ch] = at;
            q.slot[ch] = (uint8_t)d;
        }
    };
    q.open[R] = 0;
    q.slot[R] = 0;
    for (int64_t v = R; v < end;) {
        if (v != R && cutp(v)) {                    // a chunk below: skip its subtree
            v = s + q.endl[v];
            continue;
        }
        const int32_t at = q.open[v];
        if (at < 0) {                               // folded into its parent
            ++v;
            continue;
        }
        const int32_t d = q.slot[v];
        max_slot = dc_max(max_slot, d);
        const uint8_t op = q.ops[v];
        if (!(op & kFuncBit)) {
            code[at] = dc_word(0, M_PUSH, (uint32_t)d, op);
            nodes += 1;
            ++v;
            continue;
        }
        const int64_t l = v + 1, r = s + q.endl[v + 1];
        const int form = (q.info[v] >> 8) & 31;
        const uint32_t m = (uint32_t)(form & 7);
        int32_t w;
        uint32_t payload = 0;
        if (m == M_XX) {
            q.open[l] = -1;
            q.open[r] = -1;
            if (q.boolean) payload = (uint32_t)q.ops[l] | ((uint32_t)q.ops[r] << 11);
            w = at;
            nodes += 3;
        } else if (m == M_XS || m == M_SX) {
            const bool left_folded = (form & 16) != 0;
            const int64_t folded = left_folded ? l : r, other = left_folded ? r : l;
            q.open[folded] = -1;
            if (q.boolean) payload = q.ops[folded];
            place(other, at, d);
            w = at + words(other);
            nodes += 2;
        } else {
            const bool first_r = (form & 8) != 0;
            const int64_t first = first_r ? r : l, second = first_r ? l : r;
            place(first, at, d);
            place(second, at + words(first), d + 1);
            w = at + words(first) + words(second);
            max_slot = dc_max(max_slot, d + 1);
            nodes += 1;
        }
        code[w] = dc_word(op & 3, m, (uint32_t)d, payload);
        if (q.rec && q.rec[v] >= 0) {
            code[w + 1] = dc_word(0, M_STORE, (uint32_t)d, (uint32_t)q.rec[v]);
            stores = 1;
        }
        ++v;
    }
    code[q.len[R]] = kEndWord;
    c.nodes[k] = nodes;
    c.max_slot[k] = max_slot;
    c.stores[k] = stores;
}

// ------------------------------------------------------------ host glue

// Chunk numbering, as compile_tree numbers a tree's chunks (by decreasing root
// index, the tree's root chunk last) and a population concatenates its trees.
// roots_asc: every chunk root (cut nodes and tree roots), ascending global
// indices.  Outputs per chunk id: root, tree start, tree; ids[j] = the id of
// roots_asc[j]; cbase[t] = tree t's first id (n_trees + 1 entries).
inline bool dc_number_chunks(const std::vector<int64_t>& roots_asc, const int64_t* offsets, int64_t n_trees,
                             std::vector<int64_t>* root, std::vector<int64_t>* tstart, std::vector<int32_t>* ctree,
                             std::vector<int32_t>* ids, std::vector<int64_t>* cbase)
{
    const int64_t nch = (int64_t)roots_asc.size();
    root->assign(nch, 0);
    tstart->assign(nch, 0);
    ctree->assign(nch, 0);
    ids->assign(nch, 0);
    cbase->assign(n_trees + 1, 0);
    int64_t j = 0;
    for (int64_t t = 0; t < n_trees; ++t) {
        int64_t j1 = j;
        while (j1 < nch && roots_asc[j1] < offsets[t + 1]) ++j1;
        if (j1 == j || roots_asc[j] != offsets[t]) return false;   // every tree has its root chunk
        const int64_t m = j1 - j;
        (*cbase)[t + 1] = (*cbase)[t] + m;
        for (int64_t i = 0; i < m; ++i) {
            const int64_t k = (*cbase)[t] + (m - 1 - i);
            (*root)[k] = roots_asc[j + i];
            (*tstart)[k] = offsets[t];
            (*ctree)[k] = (int32_t)t;
            (*ids)[j + i] = (int32_t)k;
        }
        j = j1;
    }
    return j == nch;
}

// A recorded function node: global index, record id (local to its tree),
// global parent (-1 at the root).
struct DcStored {
    int64_t node;
    int32_t rec;
    int64_t parent;
};

// Records of one tree, exactly as compile_tree assigns them: per point in
// order, the point, then per ancestor nearest first its other operand and the
// ancestor itself; a terminal stands for its input vector -(op + 1); a node
// seen before keeps its id.  Appends the tree's spines and its recorded
// function nodes; returns its record count.
inline int64_t dc_tree_records(int64_t s, int64_t n_points, const int64_t* points, const uint8_t* point_op,
                               const int32_t* point_end, const int64_t* lv_off, const DcPathLevel* lv,
                               std::vector<Spine>* spines, std::vector<DcStored>* stored)
{
    std::unordered_map<int64_t, int32_t> rec_of;
    auto rec = [&](int64_t v, uint8_t op, int64_t parent) -> int32_t {
        if (!(op & kFuncBit)) return -(int32_t)op - 1;
        auto it = rec_of.find(v);
        if (it != rec_of.end()) return it->second;
        const int32_t id = (int32_t)rec_of.size();
        rec_of.emplace(v, id);
        stored->push_back(DcStored{s + v, id, parent < 0 ? -1 : s + parent});
        return id;
    };
    for (int64_t p = 0; p < n_points; ++p) {
        const int64_t c = points[p];
        const DcPathLevel* L = lv + lv_off[p];
        const int64_t nl = lv_off[p + 1] - lv_off[p];
        Spine sp;
        sp.point = c;
        sp.at_point = rec(c, point_op[p], nl > 0 ? L[0].a : -1);
        sp.child_nodes_removed = point_end[p] - c;
        for (int64_t k = 0; k < nl; ++k) {
            SpineLevel x;
            x.fside = L[k].fside;
            x.sib = rec(L[k].sib, (uint8_t)L[k].sib_op, L[k].a);
            x.par = rec(L[k].a, kFuncBit, k + 1 < nl ? L[k + 1].a : -1);
            sp.levels.push_back(x);
        }
        spines->push_back(std::move(sp));
    }
    return (int64_t)rec_of.size();
}

// Words each recorded node adds to its own subtree's code in its chunk: its
// STORE, plus those of recorded operands that do not root a chunk of their
// own.  Every ancestor of a recorded node is recorded, so no other node's
// code grows.  cut[i] belongs to stored[i]; inc[i] is the result.
inline void dc_store_words(const std::vector<DcStored>& stored, const std::vector<uint8_t>& cut,
                           std::vector<int32_t>* inc)
{
    const size_t m = stored.size();
    std::vector<size_t> order(m);
    for (size_t i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return stored[a].node > stored[b].node; });
    std::unordered_map<int64_t, size_t> at;
    at.reserve(m * 2);
    for (size_t i = 0; i < m; ++i) at.emplace(stored[i].node, i);
    inc->assign(m, 1);
    for (size_t i : order) {
        if (cut[i] || stored[i].parent < 0) continue;
        auto it = at.find(stored[i].parent);
        if (it != at.end()) (*inc)[it->second] += (*inc)[i];
    }
}

}  // namespace gpe
