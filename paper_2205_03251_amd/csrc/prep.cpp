// Host-side tree compiler: see prep.h.
#include "prep.h"

#include <algorithm>
#include <climits>
#include <functional>
#include <memory>
#include <atomic>
#include <thread>
#include <unordered_map>

namespace gpe {

namespace {

inline bool is_func(uint8_t b) { return (b & kFuncBit) != 0; }

// compile_tree's state of one node, in one 16-byte record so that reading an
// operand touches one cache line: the end of its subtree, the words its
// subtree emits in its own chunk, the nodes not yet assigned to a chunk below
// it (during emission: where its code starts, -1 when folded into its
// parent), its stack need, whether it roots a chunk, its instruction form
// (mode | first operand is the right << 3 | folded operand is the left << 4)
// and, during emission, the stack slot of its value.
struct NodeRec {
    int32_t end;
    int32_t len;
    int32_t open;
    uint8_t need, cut, form, slot;
};
static_assert(sizeof(NodeRec) == 16, "one node record is 16 bytes");

// Per-node work arrays of compile_tree, grown to the largest tree seen.
struct CompileScratch {
    int64_t cap = 0;
    std::unique_ptr<NodeRec[]> node;
    std::unique_ptr<int32_t[]> st, chunk;
    void ensure(int64_t n)
    {
        if (n <= cap) return;
        cap = std::max<int64_t>(n, cap + cap / 2);
        node.reset(new NodeRec[cap + 1]);
        st.reset(new int32_t[cap + 1]);
        chunk.reset(new int32_t[cap + 1]);
    }
};


}  // namespace

bool validate_prefix(const uint8_t* ops, int64_t n, int n_inputs, std::string* why)
{
    if (n < 1) {
        if (why) *why = "empty tree";
        return false;
    }
    if (n > INT32_MAX) {
        if (why) *why = "tree longer than 2^31-1 nodes";
        return false;
    }
    {
        // Branch-free scan: valid iff the open child slots stay >= 1 before
        // the last byte and reach 0 at it, and no byte is out of range.  The
        // loop below only runs to say what is wrong.
        int64_t slots = 1, least = 1;
        uint32_t bad = 0;
        const uint32_t nin = (uint32_t)n_inputs;
        for (int64_t i = 0; i < n; ++i) {
            const uint32_t b = ops[i], f = b >> 7;
            slots += 2 * (int64_t)f - 1;
            least = std::min(least, i + 1 < n ? slots : least);
            bad |= (f & (uint32_t)((b & 0x7c) != 0)) | ((f ^ 1u) & (uint32_t)(b >= nin));
        }
        if (slots == 0 && least >= 1 && bad == 0) return true;
    }
    int64_t open = 1;   // child slots still to fill
    for (int64_t i = 0; i < n; ++i) {
        if (open == 0) {
            if (why) *why = "bytes after the end of the tree at index " + std::to_string(i);
            return false;
        }
        uint8_t b = ops[i];
        if (is_func(b)) {
            if ((b & 0x7f) > 3) {
                if (why) *why = "unknown function byte at index " + std::to_string(i);
                return false;
            }
            open += 1;
        } else {
            if (b >= n_inputs) {
                if (why) *why = "terminal index >= n_inputs at index " + std::to_string(i);
                return false;
            }
            open -= 1;
        }
    }
    if (open != 0) {
        if (why) *why = "tree ends with " + std::to_string(open) + " operand(s) missing";
        return false;
    }
    return true;
}

bool postfix_to_prefix(const uint8_t* post, int64_t n, int n_inputs, std::vector<uint8_t>* pre,
                       std::vector<int64_t>* post_to_pre, std::string* why)
{
    if (n < 1 || n > INT32_MAX) {
        if (why) *why = "bad tree length";
        return false;
    }
    // start[i]: first postfix index of the subtree ending at i.
    std::vector<int64_t> start(n);
    std::vector<int64_t> st;
    st.reserve(64);
    for (int64_t i = 0; i < n; ++i) {
        uint8_t b = post[i];
        if (is_func(b)) {
            if ((b & 0x7f) > 3 || st.size() < 2) {
                if (why) *why = "malformed postfix tree at index " + std::to_string(i);
                return false;
            }
            st.pop_back();                 // right operand
            start[i] = start[st.back()];   // left operand's start
            st.back() = i;
        } else {
            if (b >= n_inputs) {
                if (why) *why = "terminal index >= n_inputs at index " + std::to_string(i);
                return false;
            }
            start[i] = i;
            st.push_back(i);
        }
    }
    if (st.size() != 1) {
        if (why) *why = "postfix array is not exactly one tree";
        return false;
    }
    pre->resize(n);
    post_to_pre->resize(n);
    // Prefix order = node, left subtree, right subtree.  In postfix the right
    // operand of node v ends at v-1 and the left one ends just before the
    // right one starts.
    std::vector<int64_t> todo;
    todo.push_back(n - 1);
    int64_t k = 0;
    while (!todo.empty()) {
        int64_t v = todo.back();
        todo.pop_back();
        (*pre)[k] = post[v];
        (*post_to_pre)[v] = k;
        ++k;
        if (is_func(post[v])) {
            int64_t r = v - 1;
            int64_t l = start[r] - 1;
            todo.push_back(r);
            todo.push_back(l);
        }
    }
    return true;
}

bool compile_tree(const uint8_t* ops, int64_t n, const CompileOptions& opt, const int64_t* points,
                  int64_t n_points, TreeProg* out, std::string* why, const int32_t* ext, const Collapsed* col)
{
    const bool boolean = opt.vtype == 1;
    const int S = opt.stack_slots;
    const int64_t C = std::max<int64_t>(2, opt.chunk_nodes);
    if (S < 2 || S > kMaxStackSlots) {
        if (why) *why = "stack_slots out of range";
        return false;
    }
    // Float folds terminal 0 (kept in registers); Boolean folds any terminal
    // (read from the staged input words).
    auto external = [&](int64_t v) { return ext != nullptr && ext[v] >= 0; };
    auto opaque = [&](int64_t v) { return col != nullptr && col->opaque[v] >= 0; };
    auto foldable = [&](int64_t v) {
        return !is_func(ops[v]) && !external(v) && !opaque(v) && (boolean || ops[v] == 0);
    };
    auto full = [&](int64_t v) { return col != nullptr ? col->node_map[v] : v; };
    auto forced = [&](int64_t v) { return col != nullptr && col->cut_at != nullptr && col->cut_at[v] != 0; };
    const int32_t id_base = col != nullptr ? col->id_base : 0;
    if (col != nullptr && n_points > 0) {
        if (why) *why = "record points in a collapsed tree";
        return false;
    }

    // Per node, filled by the right-to-left pass; nodes are written before
    // they are read, so nothing needs clearing first.  The records are kept
    // per thread and reused: a load compiles many trees on each thread, and
    // fresh pages cost more than the pass itself.
    static thread_local CompileScratch ws;
    ws.ensure(n);
    NodeRec* nd = ws.node.get();
    const bool index = opt.index_min_size > 0;
    out->big_ends.clear();
    auto words = [&](int64_t c) -> int32_t { return nd[c].cut ? 1 : nd[c].len; };   // LOAD or the code
    std::vector<int64_t> roots;                 // the cut nodes

    // The pass: a node's values depend on its operands' only, so nodes can be
    // finished in any order that puts every node after the nodes above it in
    // index.  leaf(i) and func(i, l, r) do node i.
    auto leaf = [&](int64_t i) {
        NodeRec& x = nd[i];
        x.end = (int32_t)(i + 1);
        x.cut = opaque(i) ? 1 : 0;            // a compiled chunk: one LOAD
        x.need = 1;
        x.open = 1;
        x.len = 1;                            // PUSH, when not folded into its parent
    };
    auto func = [&](int64_t i, int32_t l, int32_t r, std::vector<int64_t>& cuts, std::vector<SubtreeEnd>& bigs) {
        NodeRec& x = nd[i];
        NodeRec& L = nd[l];
        NodeRec& R = nd[r];
        x.end = R.end;
        if (index && full(x.end) - full(i) >= opt.index_min_size)
            bigs.push_back({(int32_t)full(i), (int32_t)full(x.end)});
        x.cut = 0;
        const bool fol = foldable(l), fo_r = foldable(r);
        auto cost = [](const NodeRec& c) { return c.cut ? 1 : (int)c.need; };
        auto need_of = [&]() {
            bool fl = !L.cut && fol, fr = !R.cut && fo_r;
            if (fl && fr) return 1;
            if (fl) return cost(R);
            if (fr) return cost(L);
            int nl = cost(L), nr = cost(R);
            return nl >= nr ? std::max(nl, nr + 1) : std::max(nr, nl + 1);
        };
        int need = need_of();
        if (need > S) {
            // Both operands need a full stack: give the bigger one a chunk of
            // its own; its value then arrives by one LOAD (one slot).
            int32_t big = cost(L) >= cost(R) ? l : r;
            nd[big].cut = 1;
            cuts.push_back(big);
            need = need_of();
        }
        x.need = (uint8_t)need;
        // the instruction form, fixed now that the operands' cuts are final
        const bool fl = !L.cut && fol, fr = !R.cut && fo_r;
        if (fl && fr) {
            x.form = M_XX;
            x.len = 1;
        } else if (fl || fr) {
            x.form = (uint8_t)((boolean || fl ? M_XS : M_SX) | (fl ? 16 : 0));
            x.len = words(fl ? r : l) + 1;
        } else {
            const bool first_r = !(cost(L) >= cost(R));
            x.form = (uint8_t)((!first_r || boolean ? M_SS : M_RS) | (first_r ? 8 : 0));
            x.len = words(l) + words(r) + 1;
        }
        int64_t o = 1 + (L.cut ? 1 : L.open) + (R.cut ? 1 : R.open);
        x.open = (int32_t)std::min<int64_t>(o, INT32_MAX);
        if ((o >= C || forced(i)) && i != 0) {
            x.cut = 1;
            cuts.push_back(i);
        }
    };
    const int pth = (int)std::min<int64_t>(std::max(1, opt.threads), 64);
    if (pth > 1 && n >= 200000) {
        // Segments of the array in parallel, right to left, a node's right
        // operand found as the end of its left one; a node whose subtree runs
        // past its segment's end waits.  Then the waiting nodes, about the
        // tree's depth per segment, in decreasing index order.
        std::vector<std::vector<int64_t>> seg_cuts(pth), seg_wait(pth);
        std::vector<std::vector<SubtreeEnd>> seg_big(pth);
        std::vector<std::thread> th;
        auto seg = [&](int t) {
            const int64_t lo = n * t / pth, hi = n * (t + 1) / pth;
            for (int64_t i = hi - 1; i >= lo; --i) {
                if (!is_func(ops[i])) {
                    leaf(i);
                    continue;
                }
                const int32_t l = (int32_t)(i + 1);
                if (l >= hi || nd[l].end < 0 || nd[l].end >= hi || nd[nd[l].end].end < 0) {
                    nd[i].end = -1;           // an operand lies beyond this segment
                    seg_wait[t].push_back(i);
                    continue;
                }
                func(i, l, nd[l].end, seg_cuts[t], seg_big[t]);
            }
        };
        for (int t = 1; t < pth; ++t) th.emplace_back(seg, t);
        seg(0);
        for (auto& x : th) x.join();
        std::vector<SubtreeEnd> bigs;
        for (int t = pth - 1; t >= 0; --t)
            for (int64_t i : seg_wait[t]) func(i, (int32_t)(i + 1), nd[i + 1].end, roots, bigs);
        for (int t = 0; t < pth; ++t) {
            roots.insert(roots.end(), seg_cuts[t].begin(), seg_cuts[t].end());
            out->big_ends.insert(out->big_ends.end(), seg_big[t].begin(), seg_big[t].end());
        }
        out->big_ends.insert(out->big_ends.end(), bigs.begin(), bigs.end());
        std::sort(out->big_ends.begin(), out->big_ends.end());
    } else {
        // one pass with an operand stack (the right operand is the second entry)
        int32_t* st = ws.st.get();
        int64_t top = 0;
        for (int64_t i = n - 1; i >= 0; --i) {
            if (!is_func(ops[i])) {
                leaf(i);
                st[top++] = (int32_t)i;
                continue;
            }
            const int32_t l = st[--top];
            const int32_t r = st[top - 1];
            st[top - 1] = (int32_t)i;
            func(i, l, r, roots, out->big_ends);
        }
        std::reverse(out->big_ends.begin(), out->big_ends.end());   // found right to left
    }

    // Records requested by the crossover points: the mother's vector at the
    // point, at every ancestor, and at each ancestor's other operand.
    std::unordered_map<int64_t, int32_t> rec_of;
    auto rec = [&](int64_t v) -> int32_t {
        if (!is_func(ops[v])) return -(int32_t)ops[v] - 1;
        auto it = rec_of.find(v);
        if (it != rec_of.end()) return it->second;
        int32_t id = (int32_t)rec_of.size();
        rec_of.emplace(v, id);
        return id;
    };
    out->spines.clear();
    std::vector<int64_t> path;
    for (int64_t p = 0; p < n_points; ++p) {
        int64_t c = points[p];
        if (c < 0 || c >= n) {
            if (why) *why = "record point " + std::to_string(c) + " out of range";
            return false;
        }
        path.clear();
        int64_t v = 0;
        path.push_back(0);
        while (v != c) {
            int64_t l = v + 1, r = nd[l].end;
            v = (c < r) ? l : r;
            path.push_back(v);
        }
        Spine sp;
        sp.point = c;
        sp.at_point = rec(c);
        sp.child_nodes_removed = nd[c].end - c;
        for (int64_t k = (int64_t)path.size() - 2; k >= 0; --k) {
            int64_t a = path[k], below = path[k + 1];
            int64_t l = a + 1, r = nd[l].end;
            bool right = below != l;
            int64_t sib = right ? l : r;
            SpineLevel lv;
            lv.fside = (ops[a] & 3) | (right ? 4 : 0);
            lv.sib = rec(sib);
            lv.par = rec(a);
            sp.levels.push_back(lv);
        }
        out->spines.push_back(std::move(sp));
    }
    if (rec_of.size() > kMaxPayload) {
        if (why) *why = "too many parent-cache records in one tree";
        return false;
    }
    out->n_records = (int64_t)rec_of.size();
    // A recorded node's STORE follows its own word: recount the code lengths
    // of the recorded nodes, operands before parents.  Every ancestor of a
    // recorded node is recorded (the point's ancestors, and the siblings'
    // parents are on that path), so no other node's code grows.
    std::unique_ptr<uint8_t[]> stored;
    if (!rec_of.empty()) {
        stored.reset(new uint8_t[n]());
        std::vector<int64_t> recd;
        recd.reserve(rec_of.size());
        for (const auto& kv : rec_of) {
            stored[kv.first] = 1;
            recd.push_back(kv.first);
        }
        std::sort(recd.begin(), recd.end(), std::greater<int64_t>());
        for (int64_t i : recd) {
            const int64_t l = i + 1, r = nd[l].end;
            const uint32_t m = nd[i].form & 7;
            int32_t w = m == M_XX ? 1 : (m == M_XS || m == M_SX) ? words((nd[i].form & 16) ? r : l) + 1
                                                                  : words(l) + words(r) + 1;
            nd[i].len = w + 1;
        }
    }

    // Chunks: the root plus every cut node, numbered by descending prefix
    // index so that every chunk comes after the chunks it reads.
    std::sort(roots.begin(), roots.end(), std::greater<int64_t>());
    roots.push_back(0);
    const int64_t nch = (int64_t)roots.size();
    std::unordered_map<int64_t, int32_t> chunk_map;
    int32_t* chunk_dense = ws.chunk.get();
    const bool dense = nch > 64;
    if (dense) {
        for (int64_t k = 0; k < nch; ++k) chunk_dense[roots[k]] = (int32_t)k;
    } else {
        for (int64_t k = 0; k < nch; ++k) chunk_map[roots[k]] = (int32_t)k;
    }
    auto chunk_of = [&](int64_t v) { return dense ? chunk_dense[v] : chunk_map[v]; };

    // Chunk k's code: len[root] words, then kEndWord.  Each word's place is
    // known from the code lengths: an instruction's first operand's code
    // starts where the instruction's own code starts, the second's after
    // it, and the instruction's word follows both.  So every chunk's code
    // is written by one scan of its nodes in prefix order (parents before
    // their operands), independent of every other chunk's.
    out->chunks.assign(nch, Chunk());
    int64_t total = 0;
    for (int64_t k = 0; k < nch; ++k) {
        Chunk& ch = out->chunks[k];
        ch.code_off = total;
        ch.code_len = (int64_t)nd[roots[k]].len + 1;
        total += ch.code_len;
    }
    out->code.resize((size_t)total);
    // where each node's code starts in its chunk (in open, not read again)
    // and the slot it leaves its value in; -1: folded into its parent
    std::vector<int32_t> slot_hi(nch, 0);
    std::vector<uint8_t> too_many(nch, 0);
    auto emit = [&](int64_t k) {
        Chunk& ch = out->chunks[k];
        uint32_t* code = out->code.data() + ch.code_off;
        const int64_t root = roots[k], end = nd[root].end;
        int32_t max_slot = 0;
        ch.root_node = full(root);
        ch.end_node = index ? full(end) : -1;
        ch.nodes = 0;
        // place operand c's code at q, value in slot d: a LOAD if it roots a chunk
        auto place = [&](int64_t c, int32_t q, int32_t d) {
            if (nd[c].cut) {
                int32_t id;
                if (opaque(c)) {
                    id = col->opaque[c];
                } else {
                    id = chunk_of(c);
                    out->chunks[id].parent = id_base + (int32_t)k;
                    id += id_base;
                }
                code[q] = ins_word(0, M_LOAD, (uint32_t)d, (uint32_t)ch.inputs.size());
                ch.inputs.push_back(id);
            } else {
                nd[c].open = q;
                nd[c].slot = (uint8_t)d;
            }
        };
        nd[root].open = 0;
        nd[root].slot = 0;
        for (int64_t v = root; v < end;) {
            if (v != root && nd[v].cut) {       // a chunk below (or a collapsed one): skip its subtree
                v = nd[v].end;
                continue;
            }
            const int32_t q = nd[v].open;
            if (q < 0) {                        // folded into its parent
                ++v;
                continue;
            }
            const int32_t d = nd[v].slot;
            max_slot = std::max(max_slot, d);
            if (!is_func(ops[v])) {
                code[q] = ins_word(0, M_PUSH, (uint32_t)d, external(v) ? (uint32_t)ext[v] : ops[v]);
                ch.nodes += 1;
                ++v;
                continue;
            }
            const int64_t l = v + 1, r = nd[l].end;
            const uint32_t m = nd[v].form & 7;
            int32_t w;                          // the instruction's own word
            uint32_t payload = 0;
            if (m == M_XX) {
                nd[l].open = nd[r].open = -1;
                if (boolean) payload = (uint32_t)ops[l] | ((uint32_t)ops[r] << 11);
                w = q;
                ch.nodes += 3;
            } else if (m == M_XS || m == M_SX) {
                const bool left_folded = (nd[v].form & 16) != 0;
                const int64_t folded = left_folded ? l : r, other = left_folded ? r : l;
                nd[folded].open = -1;
                if (boolean) payload = ops[folded];
                place(other, q, d);
                w = q + words(other);
                ch.nodes += 2;
            } else {
                const bool first_r = (nd[v].form & 8) != 0;
                const int64_t first = first_r ? r : l, second = first_r ? l : r;
                place(first, q, d);
                place(second, q + words(first), d + 1);
                w = q + words(first) + words(second);
                max_slot = std::max(max_slot, d + 1);
                ch.nodes += 1;
            }
            code[w] = ins_word(ops[v] & 3, m, (uint32_t)d, payload);
            if (stored && stored[v]) {
                code[w + 1] = ins_word(0, M_STORE, (uint32_t)d, (uint32_t)rec_of.find(v)->second);
                ch.stores = true;
            }
            ++v;
        }
        code[ch.code_len - 1] = kEndWord;
        slot_hi[k] = max_slot;
        if (ch.inputs.size() > kMaxPayload) too_many[k] = 1;
    };
    const int nth = (int)std::min<int64_t>(std::max(1, opt.threads), nch / 2);
    if (nth > 1 && n >= 200000) {
        std::atomic<int64_t> next{0};
        auto work = [&]() {
            for (int64_t k; (k = next++) < nch;) emit(k);
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nth; ++t) th.emplace_back(work);
        work();
        for (auto& t : th) t.join();
    } else {
        for (int64_t k = 0; k < nch; ++k) emit(k);
    }
    int32_t max_slot = 0;
    for (int64_t k = 0; k < nch; ++k) {
        if (too_many[k]) {
            if (why) *why = "chunk reads too many child chunks";
            return false;
        }
        max_slot = std::max(max_slot, slot_hi[k]);
    }
    out->max_stack = max_slot + 1;
    if (out->max_stack > S) {
        if (why) *why = "internal error: stack bound exceeded";
        return false;
    }
    // Longest chain of chunk work from each chunk up to the tree root
    // (parents come after children, so walk backwards).
    for (int64_t k = col != nullptr ? -1 : (int64_t)out->chunks.size() - 1; k >= 0; --k) {
        Chunk& ch = out->chunks[k];
        ch.path_nodes = ch.nodes + (ch.parent >= 0 ? out->chunks[ch.parent].path_nodes : 0);
    }
    return true;
}

void big_subtree_ends(const uint8_t* ops, int64_t n, int64_t min_size,
                      std::vector<SubtreeEnd>* out)
{
    out->clear();
    std::vector<std::pair<int64_t, int32_t>> st;   // open function nodes: (node, operands started)
    st.reserve(256);
    for (int64_t i = 0; i < n; ++i) {
        if (!st.empty()) ++st.back().second;
        if (is_func(ops[i])) {
            st.push_back({i, 0});
            continue;
        }
        while (!st.empty() && st.back().second == 2) {
            const int64_t a = st.back().first;
            if (i + 1 - a >= min_size) out->push_back({(int32_t)a, (int32_t)(i + 1)});
            st.pop_back();
        }
    }
    std::sort(out->begin(), out->end());
}

int64_t subtree_end_indexed(const uint8_t* ops, int64_t n, int64_t x, const std::vector<SubtreeEnd>& big)
{
    if (!is_func(ops[x])) return x + 1;
    auto it = std::lower_bound(big.begin(), big.end(), SubtreeEnd{(int32_t)x, -1});
    if (it != big.end() && it->first == x) return it->second;
    int64_t o = 0;
    for (int64_t k = x; k < n; ++k) {
        o += is_func(ops[k]) ? 1 : -1;
        if (o < 0) return k + 1;
    }
    return n;
}

// From the root down: at each ancestor a of c the first operand starts at
// a + 1 and ends at end(a + 1), taken from the index or found by scanning that
// (small) subtree; c lies in whichever operand holds it, the other operand is
// the sibling, and the end of the next ancestor is end(a + 1) or end(a).
void path_to_root(const uint8_t* ops, int64_t n, int64_t c, const std::vector<SubtreeEnd>& big,
                  std::vector<PathLevel>* levels, int64_t* removed_end)
{
    levels->clear();
    *removed_end = -1;
    if (c < 0 || c >= n) return;
    auto end_of = [&](int64_t x) { return subtree_end_indexed(ops, n, x, big); };
    int64_t a = 0, end_a = n;
    while (a != c) {
        const int64_t l = a + 1, end_l = end_of(l);
        PathLevel lv;
        lv.node = a;
        lv.f = ops[a] & 3;
        if (c < end_l) {
            lv.right = 0;
            lv.sib_begin = end_l;
            lv.sib_end = end_a;
            end_a = end_l;
            a = l;
        } else {
            lv.right = 1;
            lv.sib_begin = l;
            lv.sib_end = end_l;
            a = end_l;
        }
        levels->push_back(lv);
    }
    *removed_end = end_a;
    std::reverse(levels->begin(), levels->end());   // nearest the point first
}

bool compose_child(const SrcTree& m, int64_t c, int64_t c_end, const SrcTree& f, int64_t d, int64_t d_end,
                   const uint8_t* child, int64_t n_child, const CompileOptions& opt, TreeProg* out,
                   std::string* why)
{
    const int64_t delta = (d_end - d) - (c_end - c);
    if (opt.index_min_size <= 0 || c < 0 || c_end > m.n || c >= c_end || d < 0 || d_end > f.n || d >= d_end ||
        n_child != m.n + delta) {
        if (why) *why = "compose_child: bad crossover";
        return false;
    }
    out->code.clear();
    out->chunks.clear();
    out->spines.clear();
    out->n_records = 0;
    out->big_ends.clear();
    out->max_stack = 1;
    // A reused chunk keeps its code, its node count and its inputs (renumbered);
    // the ones whose parent chunk is recompiled ("tops") become collapsed leaves.
    struct Top {
        int64_t root, end;               // in the child
        int64_t src_root, src_end;       // in the parent it comes from
        int32_t id;
        bool from_mother;
    };
    std::vector<Top> tops;
    std::vector<int32_t> mid(m.n_chunks, -1), fid(f.n_chunks, -1);
    auto take = [&](const SrcTree& t, int64_t k, std::vector<int32_t>& ids, int64_t root, int64_t end) {
        const Chunk& s = t.chunks[k];
        ids[k] = (int32_t)out->chunks.size();
        Chunk ch;
        ch.code_off = 0;
        ch.code_len = s.code_len;
        ch.dev_src = s.code_off;
        ch.src_vec = s.vec_slot;
        ch.root_node = root;
        ch.end_node = end;
        ch.nodes = s.nodes;
        ch.parent = -2;                  // set below
        ch.inputs.reserve(s.inputs.size());
        for (int32_t in : s.inputs) ch.inputs.push_back(ids[in]);   // children come first
        out->chunks.push_back(std::move(ch));
        out->max_stack = std::max(out->max_stack, t.max_stack);
    };
    // the mother's chunks off the path; ends at c stay (the removed subtree starts there)
    for (int64_t k = 0; k < m.n_chunks; ++k) {
        const int64_t r = m.chunks[k].root_node, e = m.chunks[k].end_node;
        if (r >= c && r < c_end) continue;       // inside the removed subtree
        if (r < c && c < e) continue;            // holds the point: recompiled
        if (m.chunks[k].stores) continue;        // the child records nothing: recompiled
        take(m, k, mid, r < c ? r : r + delta, e <= c ? e : e + delta);
    }
    // the father's chunks inside the donor subtree
    for (int64_t k = 0; k < f.n_chunks; ++k) {
        const int64_t r = f.chunks[k].root_node, e = f.chunks[k].end_node;
        if (r < d || r >= d_end || f.chunks[k].stores) continue;
        take(f, k, fid, r - d + c, e - d + c);
    }
    for (int side = 0; side < 2; ++side) {
        const SrcTree& t = side == 0 ? m : f;
        const std::vector<int32_t>& ids = side == 0 ? mid : fid;
        for (int64_t k = 0; k < t.n_chunks; ++k) {
            if (ids[k] < 0) continue;
            const int32_t p = t.chunks[k].parent;
            Chunk& ch = out->chunks[ids[k]];
            if (p >= 0 && ids[p] >= 0) {
                ch.parent = ids[p];
            } else {
                tops.push_back(Top{ch.root_node, ch.end_node, t.chunks[k].root_node, t.chunks[k].end_node, ids[k],
                                   side == 0});
            }
        }
    }
    std::sort(tops.begin(), tops.end(), [](const Top& a, const Top& b) { return a.root < b.root; });
    const int32_t n_reused = (int32_t)out->chunks.size();
    if (tops.size() == 1 && tops[0].root == 0 && tops[0].end == n_child) {
        // the donor's chunk is the whole child
        out->chunks[tops[0].id].parent = -1;
    } else {
        // the rest of the child, with every top collapsed to one leaf
        std::vector<uint8_t> gops;
        std::vector<int32_t> opq;
        std::vector<int64_t> nmap;
        size_t j = 0;
        for (int64_t p = 0; p < n_child;) {
            nmap.push_back(p);
            if (j < tops.size() && tops[j].root == p) {
                gops.push_back(0);
                opq.push_back(tops[j].id);
                p = tops[j].end;
                ++j;
            } else {
                gops.push_back(child[p]);
                opq.push_back(-1);
                ++p;
            }
        }
        nmap.push_back(n_child);
        if (j != tops.size()) {
            if (why) *why = "compose_child: overlapping chunks";
            return false;
        }
        // Only the path from the point to the root must be evaluated anew;
        // every subtree hanging off it that is not a reused chunk gets a chunk
        // of its own when it is not small, so those run side by side and the
        // chain of dependent chunks holds little more than the path itself.
        const int64_t G = (int64_t)gops.size();
        std::vector<int32_t> gend(G), gst;
        gst.reserve(64);
        for (int64_t v = G - 1; v >= 0; --v) {
            if (gops[v] & kFuncBit && opq[v] < 0) {
                gst.pop_back();
                gend[v] = gend[gst.back()];
                gst.pop_back();
            } else {
                gend[v] = (int32_t)(v + 1);
            }
            gst.push_back((int32_t)v);
        }
        std::vector<uint8_t> cut_at(G, 0);
        const int64_t gp = std::upper_bound(nmap.begin(), nmap.end() - 1, c) - nmap.begin() - 1;   // glue node at c
        for (int64_t v = 0; v != gp && v >= 0 && v < G && (gops[v] & kFuncBit) && opq[v] < 0;) {
            const int64_t l = v + 1, r = gend[l];
            const int64_t next = gp < r ? l : r, sib = next == l ? r : l;
            if (opq[sib] < 0 && (gops[sib] & kFuncBit) && gend[sib] - sib >= kPathSiblingChunk) cut_at[sib] = 1;
            v = next;
        }
        Collapsed col{opq.data(), nmap.data(), n_reused, cut_at.data()};
        TreeProg glue;
        if (!compile_tree(gops.data(), (int64_t)gops.size(), opt, nullptr, 0, &glue, why, nullptr, &col))
            return false;
        out->max_stack = std::max(out->max_stack, glue.max_stack);
        out->code.swap(glue.code);
        for (Chunk& ch : glue.chunks) {
            for (int32_t in : ch.inputs)
                if (in < n_reused) out->chunks[in].parent = n_reused + (int32_t)(&ch - glue.chunks.data());
            out->chunks.push_back(std::move(ch));
        }
        out->big_ends.swap(glue.big_ends);
    }
    // the chunk graph must be a tree listed children first, the root last
    const int64_t nc = (int64_t)out->chunks.size();
    for (int64_t k = 0; k < nc; ++k) {
        const Chunk& ch = out->chunks[k];
        bool ok = (k == nc - 1) ? ch.parent == -1 : (ch.parent > k && ch.parent < nc);
        for (int32_t in : ch.inputs) ok = ok && in >= 0 && in < k && out->chunks[in].parent == k;
        if (!ok) {
            if (why) *why = "compose_child: inconsistent chunk graph";
            return false;
        }
    }
    // index entries inside the reused chunks, from the parents' indexes: in
    // the order of the tops, so sorted, as the recompiled part's are; merged
    std::vector<SubtreeEnd> reused_big;
    for (const Top& tp : tops) {
        const std::vector<SubtreeEnd>& big = tp.from_mother ? *m.big : *f.big;
        auto it = std::lower_bound(big.begin(), big.end(), SubtreeEnd{(int32_t)tp.src_root, INT32_MIN});
        const int64_t shift = tp.root - tp.src_root;
        for (; it != big.end() && it->first < tp.src_end; ++it)
            reused_big.push_back({(int32_t)(it->first + shift), (int32_t)(it->second + shift)});
    }
    std::vector<SubtreeEnd> merged(out->big_ends.size() + reused_big.size());
    std::merge(out->big_ends.begin(), out->big_ends.end(), reused_big.begin(), reused_big.end(), merged.begin());
    out->big_ends.swap(merged);
    for (int64_t k = (int64_t)out->chunks.size() - 1; k >= 0; --k) {
        Chunk& ch = out->chunks[k];
        ch.path_nodes = ch.nodes + (ch.parent >= 0 ? out->chunks[ch.parent].path_nodes : 0);
    }
    return true;
}

}  // namespace gpe
