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
    uint64_t* slot64;                  // packed hand-off: the two operands' words of each function
    uint8_t* ncut;                     // 1: roots a chunk because its parent's operands both need a full stack
    uint8_t* big;                      // 1: a function whose subtree has at least big_min nodes (may be null)
    int64_t big_min;
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
    uint32_t* code;
    int32_t* n_in;                     // LOADs in its code
    int32_t* parent;                   // global parent chunk id (set by the parent's thread)
    int32_t* load_idx;                 // which LOAD of its parent reads it (set by the parent's thread)
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

// An operand as its parent sees it: roots a chunk of its own (then it is one
// LOAD word of one slot), or its stack need, code words and open nodes.
struct DcKid {
    bool cut;
    int need;
    int32_t len;
    int32_t open;
};

// The function at global index g of the tree starting at s, from its two
// operands (compile_tree's rules): its stack need, instruction form, code
// words and open nodes, whether it roots a chunk by size, and which operand
// (0 none, 1 left, 2 right) it makes root a chunk because both need a full
// stack.
struct DcNode {
    int need, form;
    int32_t len;
    int64_t open;
    bool cut;
    int cut_kid;
};

GPE_HD inline DcNode dc_combine(const DcNodes& q, int64_t g, int64_t s, int64_t l, int64_t r, DcKid L, DcKid R)
{
    const bool fol = dc_foldable(q, l), fo_r = dc_foldable(q, r);
    auto cost_l = [&]() { return L.cut ? 1 : L.need; };
    auto cost_r = [&]() { return R.cut ? 1 : R.need; };
    auto need_of = [&]() {
        const bool fl = !L.cut && fol, fr = !R.cut && fo_r;
        if (fl && fr) return 1;
        if (fl) return cost_r();
        if (fr) return cost_l();
        const int nl = cost_l(), nr = cost_r();
        return nl >= nr ? dc_max(nl, nr + 1) : dc_max(nr, nl + 1);
    };
    DcNode o;
    o.cut_kid = 0;
    o.need = need_of();
    if (o.need > q.S) {
        // both operands need a full stack: the bigger one roots a chunk of its own
        if (cost_l() >= cost_r()) {
            L.cut = true;
            o.cut_kid = 1;
        } else {
            R.cut = true;
            o.cut_kid = 2;
        }
        o.need = need_of();
    }
    const bool fl = !L.cut && fol, fr = !R.cut && fo_r;
    if (fl && fr) {
        o.form = M_XX;
        o.len = 1;
    } else if (fl || fr) {
        o.form = (q.boolean || fl ? M_XS : M_SX) | (fl ? 16 : 0);
        const DcKid& other = fl ? R : L;
        o.len = (other.cut ? 1 : other.len) + 1;
    } else {
        const bool first_r = !(cost_l() >= cost_r());
        o.form = (!first_r || q.boolean ? M_SS : M_RS) | (first_r ? 8 : 0);
        o.len = (L.cut ? 1 : L.len) + (R.cut ? 1 : R.len) + 1;
    }
    o.open = 1 + (L.cut ? 1 : (int64_t)L.open) + (R.cut ? 1 : (int64_t)R.open);
    o.cut = o.open >= q.C && g != s;
    return o;
}

// The outcome of a finished function node: its info and code words for the
// later passes; an operand cut by the stack rule in the per-node byte array
// ncut (its own thread has finished it; only this parent decides that).
template <class Mem>
GPE_HD inline void dc_store(const DcNodes& q, int64_t g, int64_t s, int64_t l, int64_t r, const DcNode& o)
{
    Mem::st(q.len + g, o.len);
    Mem::st(q.info + g, o.need | (o.cut ? kDcCut : 0) | (o.form << 8));
    if (o.cut_kid) q.ncut[o.cut_kid == 1 ? l : r] = 1;
    if (q.big) q.big[g] = s + q.endl[g] - g >= q.big_min ? 1 : 0;
}

GPE_HD inline bool dc_cut(const DcNodes& q, int64_t v) { return (q.info[v] & kDcCut) != 0 || q.ncut[v] != 0; }

// After the bottom-up pass: node g's cut in its info word alone (emission
// reads one word per node), and whether it roots a chunk (a cut or a root).
GPE_HD inline bool dc_finish(const DcNodes& q, int64_t g)
{
    const bool cut = dc_cut(q, g);
    if (cut) q.info[g] |= kDcCut;
    return cut || q.parl[g] < 0;
}

// ----- hand-off through memory (any chunk target)
// A terminal: need 1, one open node, one PUSH word (when not folded).
template <class Mem> GPE_HD inline void dc_leaf(const DcNodes& q, int64_t g)
{
    Mem::st(q.info + g, 1);
    Mem::st(q.len + g, 1);
    Mem::st(q.open + g, 1);
    if (q.big) q.big[g] = 0;
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
    const int64_t l = pg + 1, r = s + q.endl[pg + 1];
    if (r <= l || r >= e) {
        Mem::err(q.err, 1);
        return -1;
    }
    auto kid = [&](int64_t c) {
        const int32_t i = Mem::ld(q.info + c);
        DcKid k;
        k.cut = (i & kDcCut) != 0;
        k.need = i & 63;
        k.len = Mem::ld(q.len + c);
        k.open = Mem::ld(q.open + c);
        return k;
    };
    const DcNode o = dc_combine(q, pg, s, l, r, kid(l), kid(r));
    dc_store<Mem>(q, pg, s, l, r, o);
    Mem::st(q.open + pg, (int32_t)(o.open < 0x7fffffff ? o.open : 0x7fffffff));
    return pg;
}

// ----- hand-off through one 64-bit word per function (chunk targets up to
// kDcPackMaxC).  A node that does not root a chunk has fewer open nodes than
// the target (else it would root one) and no more code words than open
// nodes, so need - 1 (5 bits), words (13) and open nodes (14) fit in 32 bits;
// a chunk root is all ones.  Each operand ORs its word into its half of the
// parent's slot (left operand low, right high); the second to arrive gets the
// first's word back from the same atomic, so no other value crosses threads.
constexpr int64_t kDcPackMaxC = 8192;
constexpr uint32_t kDcPackCut = 0xffffffffu;

GPE_HD inline uint32_t dc_pack(int need, int32_t len, int64_t open)
{
    return (uint32_t)(need - 1) | ((uint32_t)len << 5) | ((uint32_t)open << 18);
}

GPE_HD inline DcKid dc_unpack(uint32_t w)
{
    DcKid k;
    k.cut = w == kDcPackCut;
    k.need = (int)(w & 31) + 1;
    k.len = (int32_t)((w >> 5) & 8191);
    k.open = (int32_t)(w >> 18);
    return k;
}

// A terminal's stores, and its word for its parent.
template <class Mem> GPE_HD inline uint32_t dc_leaf_packed(const DcNodes& q, int64_t g)
{
    Mem::st(q.info + g, 1);
    Mem::st(q.len + g, 1);
    if (q.big) q.big[g] = 0;
    return dc_pack(1, 1, 1);
}

// One arrival of node v (word w) at its parent; returns the parent (and its
// word in *w) when this was the parent's second operand, else -1.
template <class Mem>
GPE_HD inline int64_t dc_step_packed(const DcNodes& q, int64_t s, int64_t e, int64_t v, uint32_t* w)
{
    const int32_t p = q.parl[v];
    if (p < 0) return -1;
    const int64_t pg = s + p;
    if (pg >= v || pg < s) {
        Mem::err(q.err, 2);
        return -1;
    }
    const bool left = v == pg + 1;
    const uint64_t old = Mem::fetch_or64(q.slot64 + pg, left ? (uint64_t)*w : (uint64_t)*w << 32);
    if (old == 0) return -1;                        // the other operand is not done yet
    const uint32_t other = left ? (uint32_t)(old >> 32) : (uint32_t)old;
    const int64_t l = pg + 1, r = s + q.endl[pg + 1];
    if (r <= l || r >= e || (!left && r != v)) {
        Mem::err(q.err, 1);
        return -1;
    }
    const DcNode o = dc_combine(q, pg, s, l, r, dc_unpack(left ? *w : other), dc_unpack(left ? other : *w));
    dc_store<Mem>(q, pg, s, l, r, o);
    *w = o.cut ? kDcPackCut : dc_pack(o.need, o.len, o.open);
    return pg;
}

// Emission of one chunk by compile_tree's scan in prefix order (an
// instruction's first operand's code starts where its own code starts, the
// second's after it, the instruction's word follows both, a recorded node's
// STORE follows its word), one node per step so that a thread can take up
// another chunk as soon as one is done.  Reads cuts from the info words
// (dc_finish has run).  A chunk that roots a child chunk writes the child's
// parent and which of its LOADs reads it.
struct DcEmit {
    int64_t k, v, R, s, end;
    int64_t nodes;
    int32_t n_in, max_slot;
    uint8_t stores;
};

GPE_HD inline void dc_emit_begin(const DcNodes& q, const DcChunks& c, int64_t k, DcEmit& e)
{
    e.k = k;
    e.R = c.root[k];
    e.s = c.tree_start[k];
    e.end = e.s + q.endl[e.R];
    e.v = e.R;
    e.nodes = 0;
    e.n_in = 0;
    e.max_slot = 0;
    e.stores = 0;
    q.open[e.R] = 0;
    q.slot[e.R] = 0;
}

// One step; false once the chunk is complete (its END word and totals written).
GPE_HD inline bool dc_emit_step(const DcNodes& q, const DcChunks& c, DcEmit& e)
{
    const int64_t v = e.v;
    if (v >= e.end) {
        c.code[c.code_off[e.k] + q.len[e.R]] = kEndWord;
        c.nodes[e.k] = e.nodes;
        c.max_slot[e.k] = e.max_slot;
        c.stores[e.k] = e.stores;
        c.n_in[e.k] = e.n_in;
        return false;
    }
    const int32_t iv = q.info[v];
    if (v != e.R && (iv & kDcCut)) {            // a chunk below: skip its subtree
        e.v = e.s + q.endl[v];
        return true;
    }
    const int32_t at = q.open[v];
    e.v = v + 1;
    if (at < 0) return true;                    // folded into its parent
    uint32_t* code = c.code + c.code_off[e.k];
    const int32_t d = q.slot[v];
    e.max_slot = dc_max(e.max_slot, d);
    const uint8_t op = q.ops[v];
    if (!(op & kFuncBit)) {
        code[at] = dc_word(0, M_PUSH, (uint32_t)d, op);
        e.nodes += 1;
        return true;
    }
    const int64_t l = v + 1, r = e.s + q.endl[v + 1];
    const int32_t il = q.info[l], ir = q.info[r];
    auto words = [&](int64_t x, int32_t ix) { return (ix & kDcCut) ? 1 : q.len[x]; };
    auto place = [&](int64_t ch, int32_t ich, int32_t pos, int32_t dd) {
        if (ich & kDcCut) {
            const int32_t id = q.cnt[ch];
            c.parent[id] = (int32_t)e.k;
            c.load_idx[id] = e.n_in;
            code[pos] = dc_word(0, M_LOAD, (uint32_t)dd, (uint32_t)e.n_in);
            e.n_in += 1;
        } else {
            q.open[ch] = pos;
            q.slot[ch] = (uint8_t)dd;
        }
    };
    const int form = (iv >> 8) & 31;
    const uint32_t m = (uint32_t)(form & 7);
    int32_t w;
    uint32_t payload = 0;
    if (m == M_XX) {
        q.open[l] = -1;
        q.open[r] = -1;
        if (q.boolean) payload = (uint32_t)q.ops[l] | ((uint32_t)q.ops[r] << 11);
        w = at;
        e.nodes += 3;
    } else if (m == M_XS || m == M_SX) {
        const bool left_folded = (form & 16) != 0;
        const int64_t folded = left_folded ? l : r, other = left_folded ? r : l;
        const int32_t io = left_folded ? ir : il;
        q.open[folded] = -1;
        if (q.boolean) payload = q.ops[folded];
        place(other, io, at, d);
        w = at + words(other, io);
        e.nodes += 2;
    } else {
        const bool first_r = (form & 8) != 0;
        const int64_t first = first_r ? r : l, second = first_r ? l : r;
        const int32_t i1 = first_r ? ir : il, i2 = first_r ? il : ir;
        place(first, i1, at, d);
        const int32_t w1 = words(first, i1);
        place(second, i2, at + w1, d + 1);
        w = at + w1 + words(second, i2);
        e.max_slot = dc_max(e.max_slot, d + 1);
        e.nodes += 1;
    }
    code[w] = dc_word(op & 3, m, (uint32_t)d, payload);
    if (q.rec && q.rec[v] >= 0) {
        code[w + 1] = dc_word(0, M_STORE, (uint32_t)d, (uint32_t)q.rec[v]);
        e.stores = 1;
    }
    return true;
}

// ------------------------------------------------------------ host glue

// The LOAD lists of all chunks from each child's parent and LOAD index:
// in_off (nch + 1 entries) by prefix sums over n_in, inputs[in_off[p] + j] =
// the child that LOAD j of chunk p reads.  Chunks whose parent is -1 are
// roots.  False if the lists are inconsistent.
inline bool dc_scatter_inputs(int64_t nch, const int32_t* n_in, const int32_t* parent, const int32_t* load_idx,
                              std::vector<int64_t>* in_off, std::vector<int32_t>* inputs)
{
    in_off->assign(nch + 1, 0);
    for (int64_t k = 0; k < nch; ++k) {
        if (n_in[k] < 0 || n_in[k] > nch) return false;
        (*in_off)[k + 1] = (*in_off)[k] + n_in[k];
    }
    if ((*in_off)[nch] > nch) return false;     // each chunk is read by at most one LOAD
    inputs->assign((size_t)(*in_off)[nch], -1);
    for (int64_t k = 0; k < nch; ++k) {
        const int32_t p = parent[k];
        if (p < 0) continue;
        if (p >= nch || load_idx[k] < 0 || load_idx[k] >= n_in[p]) return false;
        int32_t& slot = (*inputs)[(size_t)((*in_off)[p] + load_idx[k])];
        if (slot >= 0) return false;
        slot = (int32_t)k;
    }
    for (int32_t x : *inputs)
        if (x < 0) return false;
    return true;
}

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
// code grows.  st[0 .. m): the recorded nodes of one tree, cut[i] whether
// st[i] roots a chunk; inc[i] receives the result for st[i].
inline void dc_store_words(const DcStored* st, const uint8_t* cut, size_t m, int32_t* inc)
{
    std::vector<size_t> order(m);
    for (size_t i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return st[a].node > st[b].node; });
    // parents precede their operands in prefix order: a parent's position in
    // `order` is found by binary search over the decreasing node indices
    std::vector<int64_t> node_desc(m);
    for (size_t i = 0; i < m; ++i) node_desc[i] = st[order[i]].node;
    for (size_t i = 0; i < m; ++i) inc[i] = 1;
    for (size_t k = 0; k < m; ++k) {
        const size_t i = order[k];
        if (cut[i] || st[i].parent < 0) continue;
        const auto it = std::lower_bound(node_desc.begin(), node_desc.end(), st[i].parent,
                                         [](int64_t a, int64_t b) { return a > b; });
        if (it != node_desc.end() && *it == st[i].parent) inc[order[it - node_desc.begin()]] += inc[i];
    }
}

}  // namespace gpe
