// CPU run of the device tree compiler's steps (paper_2205_03251_amd/csrc/
// devcompile_core.h), checked tree by tree against the host compiler
// (compile_tree in prep.cpp): every chunk's code words, parent, inputs, root,
// node counts, subtree end and STORE flag, the stack bound, the records and
// spines, the index of large subtrees.
//
// The bottom-up pass runs its terminal threads in a random interleaving, one
// arrival at a time (or each thread to its end, in a random order), so the
// "second operand to arrive computes the node" rule is exercised with every
// operand order; emission runs the chunks in a random order.
//
// Input (stdin, text): vtype n_inputs chunk_nodes index_min_size n_trees seed mode
// handoff (0: through per-node memory; 1: packed into one word per function)
// host_threads (the threads compile_tree may use for a large tree),
// then n_trees + 1 offsets, the ops bytes, n_trees + 1 record offsets and the
// record points.  Output: "ok chunks <n> words <w> records <r>", or a line
// naming the first difference (exit status 1).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2205_03251_amd/csrc/devcompile_core.h"

using namespace gpe;

namespace {

struct CpuMem {
    static int32_t ld(const int32_t* p) { return *p; }
    static void st(int32_t* p, int32_t v) { *p = v; }
    static int32_t fetch_add(int32_t* p, int32_t v)
    {
        const int32_t o = *p;
        *p = o + v;
        return o;
    }
    static uint64_t fetch_or64(uint64_t* p, uint64_t v)
    {
        const uint64_t o = *p;
        *p = o | v;
        return o;
    }
    static void publish() {}
    static void after_count() {}
    static void err(int32_t* p, int32_t v) { *p |= v; }
};

[[noreturn]] void fail(const std::string& what)
{
    std::printf("mismatch: %s\n", what.c_str());
    std::exit(1);
}

template <class T> T rd()
{
    long long v;
    if (std::scanf("%lld", &v) != 1) fail("short input");
    return (T)v;
}

}  // namespace

int main()
{
    const int vtype = rd<int>(), n_inputs = rd<int>();
    const int64_t chunk_nodes = rd<int64_t>(), index_min = rd<int64_t>(), n_trees = rd<int64_t>();
    const uint64_t seed = rd<uint64_t>();
    const int mode = rd<int>();
    const int handoff = rd<int>();
    const int host_threads = rd<int>();
    if (handoff == 1 && chunk_nodes > kDcPackMaxC) fail("the packed hand-off takes chunk targets up to 8192");
    std::vector<int64_t> off(n_trees + 1);
    for (auto& v : off) v = rd<int64_t>();
    const int64_t n = off[n_trees];
    std::vector<uint8_t> ops(n);
    for (auto& v : ops) v = rd<uint8_t>();
    std::vector<int64_t> roff(n_trees + 1);
    for (auto& v : roff) v = rd<int64_t>();
    std::vector<int64_t> pts(roff[n_trees]);
    for (auto& v : pts) v = rd<int64_t>();
    std::mt19937_64 rng(seed);
    const int S = 10;

    // the tree index (what the device index gives): subtree ends and parents
    std::vector<int32_t> endl(n), parl(n);
    for (int64_t t = 0; t < n_trees; ++t) {
        const int64_t s = off[t], m = off[t + 1] - s;
        std::string why;
        if (!validate_prefix(ops.data() + s, m, n_inputs, &why)) fail("invalid input tree: " + why);
        std::vector<int32_t> st;
        for (int64_t i = m - 1; i >= 0; --i) {
            if (ops[s + i] & kFuncBit) {
                const int32_t l = st.back();
                st.pop_back();
                const int32_t r = st.back();
                st.pop_back();
                endl[s + i] = endl[s + r];
                parl[s + l] = (int32_t)i;
                parl[s + r] = (int32_t)i;
                st.push_back((int32_t)i);
            } else {
                endl[s + i] = (int32_t)(i + 1);
                st.push_back((int32_t)i);
            }
        }
        parl[s] = -1;
    }

    std::vector<int32_t> info(n, -7), len(n, -7), open(n, -7), cnt(n, 0), rec;
    std::vector<uint8_t> slot(n, 0), ncut(n, 0), big(n, 7);
    std::vector<uint64_t> slot64(n, 0);
    int32_t err = 0;
    DcNodes q{};
    q.ops = ops.data();
    q.offsets = off.data();
    q.n_trees = n_trees;
    q.n = n;
    q.endl = endl.data();
    q.parl = parl.data();
    q.info = info.data();
    q.len = len.data();
    q.open = open.data();
    q.cnt = cnt.data();
    q.slot64 = slot64.data();
    q.ncut = ncut.data();
    q.big = index_min > 0 ? big.data() : nullptr;
    q.big_min = index_min;
    q.slot = slot.data();
    q.err = &err;
    q.boolean = vtype == 1;
    q.S = S;
    q.C = std::max<int64_t>(2, chunk_nodes);

    // bottom-up pass: threads = terminals
    struct Th {
        int64_t v, s, e;
        bool started;
        uint32_t w;
    };
    std::vector<Th> th;
    for (int64_t g = 0; g < n; ++g)
        if (!(ops[g] & kFuncBit)) {
            const int64_t t = dc_tree_of(q, g);
            th.push_back(Th{g, off[t], off[t + 1], false, 0});
        }
    // one step of a thread: its terminal, or one arrival; false when it ends
    auto step = [&](Th& x) {
        if (!x.started) {
            x.started = true;
            if (handoff) x.w = dc_leaf_packed<CpuMem>(q, x.v);
            else dc_leaf<CpuMem>(q, x.v);
            return true;
        }
        const int64_t nv = handoff ? dc_step_packed<CpuMem>(q, x.s, x.e, x.v, &x.w) : dc_step<CpuMem>(q, x.s, x.e, x.v);
        if (nv < 0) return false;
        x.v = nv;
        return true;
    };
    if (mode == 0) {
        std::shuffle(th.begin(), th.end(), rng);
        for (auto& x : th)
            while (step(x)) {
            }
    } else {
        while (!th.empty()) {
            const size_t i = (size_t)(rng() % th.size());
            if (!step(th[i])) {
                th[i] = th.back();
                th.pop_back();
            }
        }
    }
    if (err) fail("inconsistent index " + std::to_string(err));
    for (int64_t g = 0; g < n; ++g)
        if (info[g] < 0) fail("node " + std::to_string(g) + " never finished");

    // records: the paths, read as the device reads them
    std::vector<std::vector<Spine>> spines(n_trees);
    std::vector<int64_t> n_rec(n_trees, 0);
    std::vector<DcStored> stored;
    for (int64_t t = 0; t < n_trees; ++t) {
        const int64_t s = off[t], np = roff[t + 1] - roff[t];
        std::vector<int64_t> lv_off(np + 1, 0);
        std::vector<DcPathLevel> lv;
        std::vector<uint8_t> pop(np);
        std::vector<int32_t> pend(np);
        for (int64_t p = 0; p < np; ++p) {
            const int64_t c = pts[roff[t] + p];
            pop[p] = ops[s + c];
            pend[p] = endl[s + c];
            int32_t below = (int32_t)c;
            for (int32_t a = parl[s + c]; a >= 0; a = parl[s + a]) {
                const int32_t l = a + 1, r = endl[s + l];
                const bool right = below != l;
                const int32_t sib = right ? l : r;
                lv.push_back(DcPathLevel{a, sib, (ops[s + a] & 3) | (right ? 4 : 0), ops[s + sib]});
                below = a;
            }
            lv_off[p + 1] = (int64_t)lv.size();
        }
        n_rec[t] = dc_tree_records(s, np, pts.data() + roff[t], pop.data(), pend.data(), lv_off.data(), lv.data(),
                                   &spines[t], &stored);
    }
    if (!stored.empty()) {
        std::vector<uint8_t> cut(stored.size());
        for (size_t i = 0; i < stored.size(); ++i) cut[i] = dc_cut(q, stored[i].node) ? 1 : 0;
        std::vector<int32_t> inc(stored.size());
        dc_store_words(stored.data(), cut.data(), stored.size(), inc.data());
        rec.assign(n, -1);
        for (size_t i = 0; i < stored.size(); ++i) {
            len[stored[i].node] += inc[i];
            rec[stored[i].node] = stored[i].rec;
        }
        q.rec = rec.data();
    }

    // chunk roots and numbering
    std::vector<int64_t> roots_asc;
    for (int64_t g = 0; g < n; ++g)
        if (dc_finish(q, g)) roots_asc.push_back(g);
    std::vector<int64_t> root, tstart, cbase;
    std::vector<int32_t> ctree, ids;
    if (!dc_number_chunks(roots_asc, off.data(), n_trees, &root, &tstart, &ctree, &ids, &cbase))
        fail("a tree without its root chunk");
    const int64_t nch = (int64_t)root.size();
    for (int64_t j = 0; j < nch; ++j) cnt[roots_asc[j]] = ids[j];
    std::vector<int64_t> code_off(nch + 1, 0);
    for (int64_t k = 0; k < nch; ++k) code_off[k + 1] = code_off[k] + len[root[k]] + 1;
    std::vector<uint32_t> code(code_off[nch] + 1, 0xdeadbeefu);
    std::vector<int32_t> n_in(nch, -1), parent(nch, -1), load_idx(nch, -1), max_slot(nch, -1);
    std::vector<int64_t> nodes(nch, -1);
    std::vector<uint8_t> stores(nch, 9);
    DcChunks ck{};
    ck.n = nch;
    ck.root = root.data();
    ck.tree_start = tstart.data();
    ck.code_off = code_off.data();
    ck.code = code.data();
    ck.n_in = n_in.data();
    ck.parent = parent.data();
    ck.load_idx = load_idx.data();
    ck.nodes = nodes.data();
    ck.max_slot = max_slot.data();
    ck.stores = stores.data();
    // emission: chunks in random order, their steps interleaved at random
    {
        std::vector<int64_t> order(nch);
        for (int64_t k = 0; k < nch; ++k) order[k] = k;
        std::shuffle(order.begin(), order.end(), rng);
        std::vector<DcEmit> live;
        size_t next = 0;
        while (next < order.size() || !live.empty()) {
            while (live.size() < 8 && next < order.size()) {
                live.emplace_back();
                dc_emit_begin(q, ck, order[next++], live.back());
            }
            const size_t i = (size_t)(rng() % live.size());
            if (!dc_emit_step(q, ck, live[i])) {
                live[i] = live.back();
                live.pop_back();
            }
        }
    }
    std::vector<int64_t> in_off;
    std::vector<int32_t> inputs;
    if (!dc_scatter_inputs(nch, n_in.data(), parent.data(), load_idx.data(), &in_off, &inputs))
        fail("inconsistent LOAD lists");

    // against compile_tree, tree by tree
    CompileOptions opt;
    opt.vtype = vtype;
    opt.n_inputs = n_inputs;
    opt.chunk_nodes = chunk_nodes;
    opt.stack_slots = S;
    opt.index_min_size = index_min;
    opt.threads = host_threads;
    int64_t total_rec = 0;
    for (int64_t t = 0; t < n_trees; ++t) {
        const int64_t s = off[t], m = off[t + 1] - s, b = cbase[t], nc = cbase[t + 1] - b;
        TreeProg prog;
        std::string why;
        if (!compile_tree(ops.data() + s, m, opt, pts.data() + roff[t], roff[t + 1] - roff[t], &prog, &why))
            fail("compile_tree: " + why);
        const std::string T = "tree " + std::to_string(t) + ": ";
        if ((int64_t)prog.chunks.size() != nc)
            fail(T + "chunks " + std::to_string(nc) + " vs " + std::to_string(prog.chunks.size()));
        std::vector<int64_t> path(nc, 0);
        int32_t ms = 0;
        for (int64_t i = nc - 1; i >= 0; --i) {
            const int64_t k = b + i;
            const Chunk& h = prog.chunks[i];
            const std::string C = T + "chunk " + std::to_string(i) + ": ";
            const int32_t par = parent[k] >= 0 ? parent[k] - (int32_t)b : -1;
            if (par != h.parent) fail(C + "parent");
            path[i] = nodes[k] + (par >= 0 ? path[par] : 0);
            if (root[k] - s != h.root_node) fail(C + "root");
            if (nodes[k] != h.nodes) fail(C + "nodes");
            if (path[i] != h.path_nodes) fail(C + "path nodes");
            if ((index_min > 0 ? endl[root[k]] : -1) != h.end_node) fail(C + "end node");
            if ((stores[k] != 0) != h.stores) fail(C + "stores");
            if (code_off[k + 1] - code_off[k] != h.code_len) fail(C + "code length");
            for (int64_t w = 0; w < h.code_len; ++w)
                if (code[code_off[k] + w] != prog.code[h.code_off + w])
                    fail(C + "word " + std::to_string(w) + ": " + std::to_string(code[code_off[k] + w]) + " vs " +
                         std::to_string(prog.code[h.code_off + w]));
            if ((int64_t)h.inputs.size() != n_in[k]) fail(C + "input count");
            for (int32_t j = 0; j < n_in[k]; ++j)
                if (inputs[in_off[k] + j] - (int32_t)b != h.inputs[j]) fail(C + "input " + std::to_string(j));
            ms = std::max(ms, max_slot[k] + 1);
        }
        if (ms != prog.max_stack) fail(T + "max stack");
        if (n_rec[t] != prog.n_records) fail(T + "records");
        total_rec += n_rec[t];
        if (spines[t].size() != prog.spines.size()) fail(T + "spine count");
        for (size_t i = 0; i < spines[t].size(); ++i) {
            const Spine &a = spines[t][i], &h = prog.spines[i];
            if (a.point != h.point || a.at_point != h.at_point || a.child_nodes_removed != h.child_nodes_removed ||
                a.levels.size() != h.levels.size())
                fail(T + "spine " + std::to_string(i));
            for (size_t j = 0; j < a.levels.size(); ++j)
                if (a.levels[j].fside != h.levels[j].fside || a.levels[j].sib != h.levels[j].sib ||
                    a.levels[j].par != h.levels[j].par)
                    fail(T + "spine " + std::to_string(i) + " level " + std::to_string(j));
        }
        if (index_min > 0) {
            std::vector<SubtreeEnd> bl;
            for (int64_t i = 0; i < m; ++i) {
                if (big[s + i] > 1) fail(T + "large-subtree flag never written");
                if (big[s + i]) bl.push_back({(int32_t)i, endl[s + i]});
            }
            if (bl != prog.big_ends) fail(T + "large subtrees");
        }
    }
    std::printf("ok chunks %lld words %lld records %lld\n", (long long)nch, (long long)code_off[nch],
                (long long)total_rec);
    return 0;
}
