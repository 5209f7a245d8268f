// gpeval runtime: context, device memory under an HBM budget, population
// assembly, launch plans (one persistent batched launch captured in a
// hipGraph, or one launch per tree), incremental batches and the C ABI.
#include <algorithm>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <thread>

#include "runtime.h"

namespace gpe {

// ------------------------------------------------------------ errors
int set_err(Ctx* c, int code, const std::string& msg)
{
    if (c) {
        std::lock_guard<std::mutex> lk(c->err_mu);
        c->err = msg;
    }
    return code;
}

int hip_check(Ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return GP_OK;
    return set_err(c, GP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPC(c, x)                                        \
    do {                                                  \
        int rc__ = hip_check((c), (x), #x);               \
        if (rc__ != GP_OK) return rc__;                   \
    } while (0)

#define RC(x)                                             \
    do {                                                  \
        int rc__ = (x);                                   \
        if (rc__ != GP_OK) return rc__;                   \
    } while (0)

// ------------------------------------------------------------ memory
DevBuf::~DevBuf() { release(); }

void DevBuf::release()
{
    if (p && !borrowed) {
        (void)hipFree(p);
        if (ctx) ctx->used -= bytes;
    }
    p = nullptr;
    bytes = 0;
    borrowed = false;
}

int scratch_alloc(Ctx* c, DevArena* a, DevBuf& b, size_t bytes)
{
    if (!a) return dev_alloc(c, b, bytes);
    b.release();
    const size_t r = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    a->high = std::max(a->high, a->used + r);
    if (a->used + r > a->buf.bytes) return dev_alloc(c, b, bytes);   // the arena grows at its next reset
    b.p = (uint8_t*)a->buf.p + a->used;
    b.bytes = r;
    b.ctx = nullptr;
    b.borrowed = true;
    a->used += r;
    return GP_OK;
}

int arena_reset(Ctx* c, DevArena* a)
{
    a->used = 0;
    if (a->high > a->buf.bytes) {
        a->buf.release();
        RC(dev_alloc(c, a->buf, a->high + a->high / 4));
    }
    return GP_OK;
}

int dev_alloc(Ctx* c, DevBuf& b, size_t bytes)
{
    b.release();
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (c->used + bytes > c->budget)
        return set_err(c, GP_EBUDGET,
                       "device memory budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                           std::to_string(c->budget - std::min<uint64_t>(c->budget, c->used)) + " left");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(c, GP_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    b.ctx = c;
    b.p = p;
    b.bytes = bytes;
    c->used += bytes;
    return GP_OK;
}

static int upload(Ctx* c, DevBuf& b, const void* src, size_t bytes, hipStream_t s)
{
    RC(dev_alloc(c, b, bytes));
    if (bytes) HIPC(c, hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return GP_OK;
}

Plan::~Plan()
{
    if (graph) (void)hipGraphExecDestroy(graph);
}

// ---------------------------------------------------------- heuristics
// Programs are compiled for 10 stack slots, so every interpreter variant
// (10 or 16 slots) can run them; the rare subtree needing more becomes a
// chunk of its own.
int compile_stack_slots() { return 10; }

int64_t auto_chunk_nodes(int vtype, int64_t total_nodes, int64_t n_trees, int64_t T)
{
    (void)vtype;
    (void)n_trees;
    (void)T;
    // Small chunks keep the chain of dependent chunks in the largest trees
    // short; very small ones spend more on chunk hand-off than on work.
    if (total_nodes < 200000) return 256;
    return 1024;
}

static int64_t elems_of(int vtype, int64_t T) { return vtype == GP_BOOL ? (T + 63) / 64 : T; }

static int64_t pad_to(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

static int ilog2_ceil(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

static TuneKey tune_key(int vtype, const CaseSet* cs, const Pop* p)
{
    return TuneKey{vtype, ilog2_ceil(cs->T), ilog2_ceil(std::max<int64_t>(1, p->total_nodes / std::max<int64_t>(1, p->n_trees)))};
}

static int default_variant(int vtype, const CaseSet* cs, const Pop* p, int forced)
{
    Variant* vt = variant_table();
    auto ok = [&](int v) {
        return v >= 0 && v < variant_count() &&
               variant_fits(vt[v], vtype, p->max_stack, p->n_inputs, cs->n_elems, cs->stride,
                            vtype == GP_BOOL ? 8 : 4);
    };
    if (ok(forced)) return forced;
    int wantK = 1;
    if (vtype == GP_F32) wantK = cs->n_elems <= 64 ? 1 : cs->n_elems <= 128 ? 2 : 4;
    else wantK = cs->n_elems <= 64 ? 1 : 2;
    // prefer a table-dispatch interpreter when one fits
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v) && vt[v].K == wantK && vt[v].table) return v;
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v) && vt[v].K == wantK) return v;
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v)) return v;
    return -1;
}

Launch choose_launch(Ctx* c, int vtype, const CaseSet* cs, const Pop* p)
{
    Launch L;
    const int v = default_variant(vtype, cs, p, c->forced_variant);
    auto it = c->tuned.find(tune_key(vtype, cs, p));
    const bool tuned = it != c->tuned.end() &&
                       (c->forced_variant < 0 || it->second.variant == v) &&
                       default_variant(vtype, cs, p, it->second.variant) == it->second.variant;
    if (tuned && c->forced_variant < 0) L = it->second;
    else {
        L.variant = v;
        L.waves_per_cu = tuned ? it->second.waves_per_cu : 0;
    }
    if (c->forced_waves >= 0) L.waves_per_cu = c->forced_waves;
    return L;
}

int64_t resident_grid(const Ctx* c, const Variant& v, int waves_per_cu)
{
    int per_cu = std::max(1, v.max_blocks_per_cu);
    if (waves_per_cu > 0) per_cu = std::min(per_cu, waves_per_cu);
    return (int64_t)per_cu * std::max(1, c->n_cu);
}

// Subtrees of at least this many nodes are indexed for co-evaluation's path
// search (about 1.2 % of the nodes of a random tree, 8 bytes each).
static constexpr int64_t kBigSubtree = 4096;

// -------------------------------------------------- population assembly
int build_population(Ctx* c, int vtype, int layout, int n_inputs, int64_t n_trees, const uint8_t* ops,
                     const int64_t* offsets, const int64_t* rec_points, const int64_t* rec_offsets,
                     int64_t chunk_nodes, Pop* out, hipStream_t stream, bool index_subtrees,
                     const int32_t* ext_rows)
{
    if (vtype != GP_F32 && vtype != GP_BOOL) return set_err(c, GP_EINVAL, "unknown value type");
    if (layout != GP_PREFIX && layout != GP_POSTFIX) return set_err(c, GP_EINVAL, "unknown layout");
    if (n_inputs < 1 || n_inputs > kMaxInputs) return set_err(c, GP_EINVAL, "n_inputs must be 1..64");
    if (n_trees < 1 || !ops || !offsets) return set_err(c, GP_EINVAL, "empty population");
    if (n_trees > INT32_MAX / 2) return set_err(c, GP_EINVAL, "too many trees");
    if (offsets[0] != 0) return set_err(c, GP_EINVAL, "offsets[0] must be 0");
    int64_t total = 0;
    for (int64_t t = 0; t < n_trees; ++t) {
        if (offsets[t + 1] <= offsets[t]) return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + " is empty");
        total += offsets[t + 1] - offsets[t];
    }
    if (rec_points && !rec_offsets) return set_err(c, GP_EINVAL, "record_points needs record_offsets");
    if (rec_offsets && rec_offsets[0] != 0) return set_err(c, GP_EINVAL, "record_offsets[0] must be 0");
    if (chunk_nodes <= 0) chunk_nodes = auto_chunk_nodes(vtype, total, n_trees, 0);
    chunk_nodes = std::max<int64_t>(chunk_nodes, 16);

    CompileOptions opt;
    opt.vtype = vtype;
    opt.n_inputs = n_inputs;
    opt.chunk_nodes = chunk_nodes;
    opt.stack_slots = compile_stack_slots();
    opt.index_min_size = index_subtrees && layout == GP_PREFIX ? kBigSubtree : 0;

    std::vector<TreeProg> progs(n_trees);
    std::vector<std::string> errs(n_trees);
    std::vector<char> bad(n_trees, 0);
    std::vector<int64_t> order(n_trees), tree_nodes(n_trees);
    for (int64_t t = 0; t < n_trees; ++t) {
        order[t] = t;
        tree_nodes[t] = offsets[t + 1] - offsets[t];
    }
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return tree_nodes[x] > tree_nodes[y]; });
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        std::vector<uint8_t> pre;
        std::vector<int64_t> map, pts;
        for (;;) {
            int64_t k = next.fetch_add(1);
            if (k >= n_trees) return;
            int64_t t = order[k];
            const uint8_t* tops = ops + offsets[t];
            int64_t n = tree_nodes[t];
            const int64_t* p0 = rec_points ? rec_points + rec_offsets[t] : nullptr;
            int64_t np = rec_points ? rec_offsets[t + 1] - rec_offsets[t] : 0;
            if (np < 0) {
                bad[t] = 1;
                errs[t] = "record_offsets not increasing";
                continue;
            }
            const uint8_t* tree = tops;
            pts.assign(p0, p0 + np);
            if (layout == GP_POSTFIX) {
                if (!postfix_to_prefix(tops, n, n_inputs, &pre, &map, &errs[t])) {
                    bad[t] = 1;
                    continue;
                }
                for (auto& q : pts) {
                    if (q < 0 || q >= n) {
                        bad[t] = 1;
                        errs[t] = "record point out of range";
                        break;
                    }
                    q = map[q];
                }
                if (bad[t]) continue;
                tree = pre.data();
            } else if (!validate_prefix(tops, n, n_inputs, &errs[t])) {
                bad[t] = 1;
                continue;
            }
            const int32_t* ext = (ext_rows && layout == GP_PREFIX) ? ext_rows + offsets[t] : nullptr;
            if (!compile_tree(tree, n, opt, pts.data(), (int64_t)pts.size(), &progs[t], &errs[t], ext)) {
                bad[t] = 1;
                continue;
            }
            // spine keys use the caller's indices
            for (int64_t i = 0; i < np; ++i) progs[t].spines[i].point = p0[i];
        }
    };
    const int hw = (int)std::min<int64_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
    int nth = (int)std::min<int64_t>(hw, n_trees);
    if (total < 100000) nth = 1;
    // with fewer trees than threads, each tree emits its chunks on the rest
    if (total >= 100000 && n_trees < hw) opt.threads = std::max<int>(1, hw / (int)n_trees);
    std::vector<std::thread> th;
    for (int i = 1; i < nth; ++i) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
    for (int64_t t = 0; t < n_trees; ++t)
        if (bad[t]) return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + ": " + errs[t]);
    out->layout = layout;
    if (opt.index_min_size > 0) {
        out->big_ends.resize(n_trees);
        out->big_built.assign(n_trees, 1);
        for (int64_t t = 0; t < n_trees; ++t) out->big_ends[t].swap(progs[t].big_ends);
    }
    return assemble_population(c, vtype, n_inputs, progs, tree_nodes, chunk_nodes, out, stream);
}

int build_population_device(Ctx* c, int vtype, int n_inputs, int64_t n_trees, const uint8_t* host_ops,
                            const uint8_t* dev_ops, const int64_t* offsets, const int64_t* rec_points,
                            const int64_t* rec_offsets, int64_t chunk_nodes, Pop* out, DevBuf* ops_keep)
{
    if (vtype != GP_F32 && vtype != GP_BOOL) return set_err(c, GP_EINVAL, "unknown value type");
    if (n_inputs < 1 || n_inputs > kMaxInputs) return set_err(c, GP_EINVAL, "n_inputs must be 1..64");
    if (n_trees < 1 || (!host_ops && !dev_ops) || !offsets) return set_err(c, GP_EINVAL, "empty population");
    if (n_trees > INT32_MAX / 2) return set_err(c, GP_EINVAL, "too many trees");
    if (offsets[0] != 0) return set_err(c, GP_EINVAL, "offsets[0] must be 0");
    for (int64_t t = 0; t < n_trees; ++t)
        if (offsets[t + 1] <= offsets[t]) return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + " is empty");
    if (rec_points && !rec_offsets) return set_err(c, GP_EINVAL, "record_points needs record_offsets");
    if (rec_offsets && rec_offsets[0] != 0) return set_err(c, GP_EINVAL, "record_offsets[0] must be 0");
    const int64_t total = offsets[n_trees];
    if (chunk_nodes <= 0) chunk_nodes = auto_chunk_nodes(vtype, total, n_trees, 0);
    chunk_nodes = std::max<int64_t>(chunk_nodes, 16);
    hipStream_t s = c->stream;
    // the index reads the trees with 16-byte loads: a copy of our own unless
    // the caller's device array is aligned and need not be kept
    const bool trace = std::getenv("GPEVAL_TRACE_LOAD") != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    DevBuf ops_buf, offs;
    const uint8_t* dops = dev_ops;
    if (!dev_ops || ((uintptr_t)dev_ops & 15) != 0 || ops_keep) {
        RC(dev_alloc(c, ops_buf, (size_t)total + 32));
        HIPC(c, hipMemcpyAsync(ops_buf.p, host_ops ? host_ops : dev_ops, (size_t)total,
                               host_ops ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        dops = ops_buf.as<uint8_t>();
    }
    RC(upload(c, offs, offsets, (size_t)(n_trees + 1) * sizeof(int64_t), s));
    if (trace) {
        HIPC(c, hipStreamSynchronize(s));
        std::fprintf(stderr, "[devcompile] %-28s %9.2f ms\n", "trees to the device",
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    RC(device_compile_population(c, vtype, n_inputs, n_trees, dops, offs.as<int64_t>(), offsets, host_ops,
                                 rec_points, rec_offsets, nullptr, chunk_nodes, kBigSubtree, out, nullptr, nullptr,
                                 s));
    out->layout = GP_PREFIX;
    out->device_compiled = true;
    if (ops_keep) ops_keep->swap(ops_buf);
    return GP_OK;
}

// One copy for k_splice, cut into pieces that end on 64 KiB boundaries of
// the destination (one workgroup each).
static void add_splice_item(std::vector<SpliceItem>& items, const uint8_t* src, int64_t dst, int64_t len)
{
    while (len > 0) {
        const int64_t take = std::min<int64_t>(len, ((dst + 65536) & ~int64_t(15)) - dst);
        items.push_back(SpliceItem{src, dst, take});
        src += take;
        dst += take;
        len -= take;
    }
}

int assemble_population(Ctx* c, int vtype, int n_inputs, std::vector<TreeProg>& progs,
                        const std::vector<int64_t>& tree_nodes, int64_t chunk_nodes, Pop* out,
                        hipStream_t stream, const uint32_t* dev_code_src)
{
    const int64_t n_trees = (int64_t)progs.size();
    out->vtype = vtype;
    out->n_inputs = n_inputs;
    out->n_trees = n_trees;
    out->chunk_nodes = chunk_nodes;
    out->tree_nodes = tree_nodes;
    out->total_nodes = 0;
    for (int64_t v : tree_nodes) out->total_nodes += v;

    // Global numbering: tree t's root chunk writes vector slot t; every
    // other chunk gets a slot after the roots.
    // Chunks whose code is already on the device (dev_src, from
    // dev_code_src) are gathered after all host code.
    int64_t n_chunks = 0, n_code = 0, n_rec = 0, n_in = 0, n_lv = 0, n_dev = 0;
    bool promo = false;
    for (auto& pg : progs) {
        n_chunks += (int64_t)pg.chunks.size();
        n_code += (int64_t)pg.code.size();
        for (auto& ch : pg.chunks) {
            if (ch.dev_src >= 0) n_dev += ch.code_len;
            if (ch.src_vec >= 0) promo = true;
        }
        n_rec += pg.n_records;
        for (auto& ch : pg.chunks) n_in += (int64_t)ch.inputs.size();
        for (auto& sp : pg.spines) n_lv += (int64_t)sp.levels.size();
    }
    if (n_chunks > INT32_MAX / 2 || n_rec > INT32_MAX / 2 || n_in > INT32_MAX / 2)
        return set_err(c, GP_EINVAL, "population too large for one load");
    if (n_dev > 0 && !dev_code_src) return set_err(c, GP_EINVAL, "internal error: no source for reused chunks");
    std::vector<SpliceItem> gather;
    int64_t dev_at = n_code;
    const bool keep = n_trees > 0 && !progs[0].chunks.empty() && progs[0].chunks[0].end_node >= 0;
    out->kept_chunks.clear();
    out->kept_max_stack.clear();
    if (keep) {
        out->kept_chunks.resize(n_trees);
        out->kept_max_stack.assign(n_trees, 0);
    }
    std::vector<uint32_t> code;
    code.reserve(n_code + 64);
    std::vector<DevChunk> dch(n_chunks);
    std::vector<int32_t> chunk_in;
    chunk_in.reserve(n_in);
    std::vector<SpineLvl> levels;
    levels.reserve(n_lv);
    out->chunk_n_in.assign(n_chunks, 0);
    out->chunk_tree.assign(n_chunks, 0);
    out->promo_src.clear();
    out->promo_in.clear();
    out->promo_rows.clear();
    out->chunk_path.clear();
    if (promo) {
        out->promo_src.assign(n_chunks, -1);
        out->promo_in.assign(n_chunks, 0);
        out->chunk_path.assign(n_chunks, 0);
    }
    out->rec_base.assign(n_trees, 0);
    out->leaves.clear();
    out->spines.clear();
    out->spine_of.clear();
    out->cuts.clear();
    out->max_stack = 0;
    out->max_code_len = 0;
    int64_t cbase = 0, rbase = 0, next_slot = n_trees;
    std::vector<int32_t> slot;
    for (int64_t t = 0; t < n_trees; ++t) {
        TreeProg& pg = progs[t];
        out->rec_base[t] = rbase;
        out->max_stack = std::max(out->max_stack, pg.max_stack);
        const int64_t obase = (int64_t)code.size();
        code.insert(code.end(), pg.code.begin(), pg.code.end());
        const int64_t nc = (int64_t)pg.chunks.size();
        slot.assign(nc, 0);
        for (int64_t k = 0; k < nc; ++k) slot[k] = (k == nc - 1) ? (int32_t)t : (int32_t)(next_slot++);
        if (nc > 0 && progs[t].chunks[0].end_node >= 0) {
            if (out->cuts.size() != (size_t)n_trees) out->cuts.assign(n_trees, {});
            auto& cl = out->cuts[t];
            cl.reserve(nc);
            for (int64_t k = 0; k < nc; ++k)
                cl.push_back(Pop::CutSlot{(int32_t)progs[t].chunks[k].root_node, (int32_t)progs[t].chunks[k].end_node,
                                          slot[k]});
            std::sort(cl.begin(), cl.end(), [](const Pop::CutSlot& a, const Pop::CutSlot& b) { return a.node < b.node; });
        }
        for (int64_t k = 0; k < nc; ++k) {
            const Chunk& ch = pg.chunks[k];
            DevChunk& d = dch[cbase + k];
            if (ch.dev_src >= 0) {
                d.code_off = dev_at;
                add_splice_item(gather, (const uint8_t*)(dev_code_src + ch.dev_src), dev_at * 4, ch.code_len * 4);
                dev_at += ch.code_len;
            } else {
                d.code_off = obase + ch.code_off;
            }
            d.code_len = (int32_t)ch.code_len;
            out->max_code_len = std::max(out->max_code_len, ch.code_len);
            d.parent = ch.parent >= 0 ? (int32_t)(cbase + ch.parent) : -1;
            d.out_slot = slot[k];
            d.in_off = (int32_t)chunk_in.size();
            d.rec_base = (int32_t)rbase;
            d.n_in = (int32_t)ch.inputs.size();
            for (int32_t in : ch.inputs) chunk_in.push_back(slot[in]);
            out->chunk_n_in[cbase + k] = (int32_t)ch.inputs.size();
            out->chunk_tree[cbase + k] = (int32_t)t;
            if (promo) {
                out->promo_src[cbase + k] = ch.src_vec;
                out->chunk_path[cbase + k] = ch.path_nodes;
                for (int32_t in : ch.inputs) out->promo_in[cbase + k] += pg.chunks[in].src_vec >= 0 ? 1 : 0;
                if (ch.src_vec >= 0) {
                    out->promo_rows.push_back(slot[k]);
                    out->promo_rows.push_back(ch.src_vec);
                }
            }
            if (ch.inputs.empty()) out->leaves.emplace_back(ch.path_nodes, (int32_t)(cbase + k));
        }
        for (auto& sp : pg.spines) {
            uint64_t key = ((uint64_t)t << 32) | (uint32_t)sp.point;
            if (out->spine_of.count(key)) continue;
            SpineInfo si;
            si.tree = (int32_t)t;
            si.at_point = sp.at_point;
            si.level_off = (int64_t)levels.size();
            si.n_levels = (int32_t)sp.levels.size();
            si.removed_nodes = sp.child_nodes_removed;
            for (auto& lv : sp.levels) levels.push_back(SpineLvl{lv.fside, lv.sib, lv.par, 0});
            out->spine_of[key] = (int32_t)out->spines.size();
            out->spines.push_back(si);
        }
        if (keep) {
            // kept for building children: code offsets become the uploaded ones
            for (int64_t k = 0; k < nc; ++k) {
                pg.chunks[k].code_off = dch[cbase + k].code_off;
                pg.chunks[k].dev_src = -1;
                pg.chunks[k].vec_slot = slot[k];
                pg.chunks[k].src_vec = -1;
            }
            out->kept_chunks[t].swap(pg.chunks);
            out->kept_max_stack[t] = pg.max_stack;
        }
        cbase += nc;
        rbase += pg.n_records;
        std::vector<uint32_t>().swap(pg.code);
        std::vector<Chunk>().swap(pg.chunks);
    }
    // Longest remaining chain first.
    std::stable_sort(out->leaves.begin(), out->leaves.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                         return x.first > y.first;
                     });
    out->n_chunks = n_chunks;
    out->n_code = n_code + n_dev;
    out->n_records = n_rec;
    if (n_dev == 0) {
        code.push_back(0);                  // one word past the end for the fetch-ahead
        RC(upload(c, out->code, code.data(), code.size() * sizeof(uint32_t), stream));
    } else {
        static const uint32_t zero = 0;
        RC(dev_alloc(c, out->code, (size_t)(n_code + n_dev + 1) * sizeof(uint32_t)));
        uint32_t* dc = out->code.as<uint32_t>();
        if (n_code) HIPC(c, hipMemcpyAsync(dc, code.data(), (size_t)n_code * 4, hipMemcpyHostToDevice, stream));
        HIPC(c, hipMemcpyAsync(dc + n_code + n_dev, &zero, 4, hipMemcpyHostToDevice, stream));
        if ((int64_t)gather.size() > (int64_t(1) << 24)) return set_err(c, GP_EINVAL, "too many chunks to gather");
        DevBuf items;
        RC(upload(c, items, gather.data(), gather.size() * sizeof(SpliceItem), stream));
        HIPC(c, launch_splice(items.as<SpliceItem>(), (int64_t)gather.size(), (uint8_t*)dc, stream));
        HIPC(c, hipStreamSynchronize(stream));
    }
    RC(upload(c, out->chunks, dch.data(), dch.size() * sizeof(DevChunk), stream));
    RC(upload(c, out->chunk_in, chunk_in.data(), chunk_in.size() * sizeof(int32_t), stream));
    RC(upload(c, out->levels, levels.data(), levels.size() * sizeof(SpineLvl), stream));
    HIPC(c, hipStreamSynchronize(stream));
    return GP_OK;
}

int ensure_eval_buffers(Ctx* c, Pop* p, const CaseSet* cs)
{
    const size_t esz = p->vtype == GP_BOOL ? 8 : 4;
    if (p->stride == cs->stride && p->vecs.p && p->fit.p) return GP_OK;
    for (auto& kv : p->plans)
        if (kv.second->graph) {
            (void)hipGraphExecDestroy(kv.second->graph);
            kv.second->graph = nullptr;
        }
    p->vecs.release();
    p->recs.release();
    p->evaluated_with = 0;
    RC(dev_alloc(c, p->vecs, (size_t)p->n_chunks * cs->stride * esz));
    if (p->n_records) RC(dev_alloc(c, p->recs, (size_t)p->n_records * cs->stride * esz));
    RC(dev_alloc(c, p->fit, (size_t)p->n_trees * 8));
    p->stride = cs->stride;
    return GP_OK;
}

static int make_plan(Ctx* c, Pop* p, const CaseSet* cs, Launch L, bool per_tree, Plan** out,
                     hipStream_t stream)
{
    const int variant = L.variant;
    const Variant& v = variant_table()[variant];
    const int32_t n_slices = (int32_t)((cs->n_elems + kWave * v.K - 1) / (kWave * v.K));
    auto key = std::make_tuple(variant, std::max(0, L.waves_per_cu), per_tree ? 1 : 0);
    auto it = p->plans.find(key);
    if (it != p->plans.end() && it->second->n_slices == n_slices) {
        *out = it->second.get();
        return GP_OK;
    }
    auto pl = std::make_unique<Plan>();
    pl->variant = variant;
    pl->waves_per_cu = std::max(0, L.waves_per_cu);
    pl->per_tree = per_tree;
    pl->n_slices = n_slices;
    std::vector<int64_t> items;
    items.reserve(p->leaves.size() * n_slices);
    if (!per_tree) {
        for (auto& lf : p->leaves)
            for (int32_t s = 0; s < n_slices; ++s) items.push_back(((int64_t)lf.second << 16) | s);
    } else {
        std::vector<std::vector<int64_t>> by_tree(p->n_trees);
        for (auto& lf : p->leaves)
            for (int32_t s = 0; s < n_slices; ++s)
                by_tree[p->chunk_tree[lf.second]].push_back(((int64_t)lf.second << 16) | s);
        pl->tree_item_begin.resize(p->n_trees);
        pl->tree_item_count.resize(p->n_trees);
        for (int64_t t = 0; t < p->n_trees; ++t) {
            pl->tree_item_begin[t] = (int64_t)items.size();
            pl->tree_item_count[t] = (int64_t)by_tree[t].size();
            items.insert(items.end(), by_tree[t].begin(), by_tree[t].end());
        }
    }
    pl->n_items = (int64_t)items.size();
    std::vector<int32_t> pend((size_t)p->n_chunks * n_slices);
    for (int64_t k = 0; k < p->n_chunks; ++k)
        for (int32_t s = 0; s < n_slices; ++s) pend[(size_t)k * n_slices + s] = p->chunk_n_in[k];
    RC(upload(c, pl->items, items.data(), items.size() * sizeof(int64_t), stream));
    RC(upload(c, pl->pending_init, pend.data(), pend.size() * sizeof(int32_t), stream));
    RC(dev_alloc(c, pl->pending, pend.size() * sizeof(int32_t)));
    RC(dev_alloc(c, pl->cursor, (size_t)(per_tree ? p->n_trees : 1) * sizeof(unsigned int)));
    pl->grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident_grid(c, v, pl->waves_per_cu), pl->n_items));
    HIPC(c, hipStreamSynchronize(stream));
    p->plans[key] = std::move(pl);
    *out = p->plans[key].get();
    return GP_OK;
}

static EvalParams eval_params(Pop* p, const CaseSet* cs, Plan* pl)
{
    EvalParams e;
    e.code = p->code.as<uint32_t>();
    e.chunks = p->chunks.as<DevChunk>();
    e.chunk_in = p->chunk_in.as<int32_t>();
    e.items = pl->items.as<int64_t>();
    e.n_items = pl->n_items;
    e.pending = pl->pending.as<int32_t>();
    e.cursor = pl->cursor.as<unsigned int>();
    e.inputs = cs->inputs.p;
    e.vecs = p->vecs.p;
    e.recs = p->recs.p;
    e.stride = cs->stride;
    e.n_slices = pl->n_slices;
    e.n_inputs = cs->n_inputs;
    return e;
}

static FitParams fit_params(Pop* p, const CaseSet* cs)
{
    FitParams f;
    f.vecs = p->vecs.p;
    f.first_slot = 0;
    f.target = cs->target.p;
    f.fit_out = p->fit.p;
    f.stride = cs->stride;
    f.n_valid = cs->T;
    f.P = cs->P;
    return f;
}

// Everything one full evaluation enqueues: reset counters and cursors,
// evaluate, score.
static int enqueue_body(Ctx* c, Pop* p, const CaseSet* cs, Plan* pl, hipStream_t s, int64_t* launches,
                        bool time_kernel)
{
    const int64_t n_pend = p->n_chunks * pl->n_slices;
    HIPC(c, launch_init(pl->pending.as<int32_t>(), pl->pending_init.as<int32_t>(), n_pend,
                        pl->cursor.as<unsigned int>(), pl->per_tree ? (int)p->n_trees : 1, s));
    EvalParams e = eval_params(p, cs, pl);
    int64_t nl = 1;
    if (time_kernel) HIPC(c, hipEventRecord(c->kev0, s));
    if (!pl->per_tree) {
        HIPC(c, launch_eval(pl->variant, e, pl->grid, s));
        ++nl;
    } else {
        const int64_t full = resident_grid(c, variant_table()[pl->variant], pl->waves_per_cu);
        for (int64_t t = 0; t < p->n_trees; ++t) {
            EvalParams et = e;
            et.items = e.items + pl->tree_item_begin[t];
            et.n_items = pl->tree_item_count[t];
            et.cursor = e.cursor + t;
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(full, et.n_items));
            HIPC(c, launch_eval(pl->variant, et, grid, s));
            ++nl;
        }
    }
    if (time_kernel) HIPC(c, hipEventRecord(c->kev1, s));
    HIPC(c, launch_fitness(p->vtype, fit_params(p, cs), p->n_trees, s));
    ++nl;
    if (launches) *launches += nl;
    return GP_OK;
}

int enqueue_full(Ctx* c, Pop* p, gp_handle cases_h, const CaseSet* cs, Launch L, bool per_tree,
                 bool use_graph, hipStream_t s, int64_t* launches, bool time_kernel)
{
    RC(ensure_eval_buffers(c, p, cs));
    Plan* pl = nullptr;
    RC(make_plan(c, p, cs, L, per_tree, &pl, s));
    if (!use_graph) {
        RC(enqueue_body(c, p, cs, pl, s, launches, time_kernel));
    } else {
        if (!pl->graph || pl->graph_cases != cases_h) {
            if (pl->graph) {
                (void)hipGraphExecDestroy(pl->graph);
                pl->graph = nullptr;
            }
            hipGraph_t g = nullptr;
            HIPC(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            int64_t dummy = 0;
            int rc = enqueue_body(c, p, cs, pl, s, &dummy, false);
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (rc != GP_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            HIPC(c, e2);
            hipError_t e3 = hipGraphInstantiate(&pl->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPC(c, e3);
            pl->graph_cases = cases_h;
        }
        HIPC(c, hipGraphLaunch(pl->graph, s));
        if (launches) *launches += 1;
    }
    p->evaluated_with = cases_h;
    return GP_OK;
}

// Cache promotion for children built from their parents' chunks (Section 5,
// Figure 1): a reused chunk runs its parent chunk's code on the same inputs
// (its inputs are reused chunks too), so its values are that chunk's values
// from the parents' last full evaluation.  Those rows are moved over, and a
// plan of its own runs only the chunks compiled anew: a chunk whose inputs
// are all reused is a leaf work item, and every dependency counter counts
// only the inputs compiled anew.
int enqueue_promoted(Ctx* c, Pop* p, const Pop* src, gp_handle cases_h, const CaseSet* cs, Launch L,
                     hipStream_t s, int64_t* n_evaluated)
{
    if (p->promo_src.size() != (size_t)p->n_chunks || p->promo_in.size() != (size_t)p->n_chunks)
        return set_err(c, GP_EINVAL, "internal error: no record of reused chunks");
    if (src->evaluated_with != cases_h || src->stride != cs->stride || !src->vecs.p)
        return set_err(c, GP_EINVAL, "internal error: the parents hold no values for this case set");
    RC(ensure_eval_buffers(c, p, cs));
    const Variant& v = variant_table()[L.variant];
    Plan pl;
    pl.variant = L.variant;
    pl.waves_per_cu = std::max(0, L.waves_per_cu);
    pl.per_tree = false;
    pl.n_slices = (int32_t)((cs->n_elems + kWave * v.K - 1) / (kWave * v.K));
    std::vector<std::pair<int64_t, int32_t>> ready;
    std::vector<int32_t> pend((size_t)p->n_chunks * pl.n_slices, 0);
    int64_t n_eval = 0;
    for (int64_t k = 0; k < p->n_chunks; ++k) {
        if (p->promo_src[k] >= 0) continue;
        ++n_eval;
        const int32_t left = p->chunk_n_in[k] - p->promo_in[k];
        for (int32_t sl = 0; sl < pl.n_slices; ++sl) pend[(size_t)k * pl.n_slices + sl] = left;
        if (left == 0) ready.emplace_back(p->chunk_path[k], (int32_t)k);
    }
    std::stable_sort(ready.begin(), ready.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                         return x.first > y.first;
                     });
    std::vector<int64_t> items;
    items.reserve(ready.size() * pl.n_slices);
    for (auto& r : ready)
        for (int32_t sl = 0; sl < pl.n_slices; ++sl) items.push_back(((int64_t)r.second << 16) | sl);
    pl.n_items = (int64_t)items.size();
    const size_t esz = p->vtype == GP_BOOL ? 8 : 4;
    const int64_t n_rows = (int64_t)p->promo_rows.size() / 2;
    DevBuf rows;
    if (n_rows > 0) {
        RC(upload(c, rows, p->promo_rows.data(), p->promo_rows.size() * sizeof(int64_t), s));
        HIPC(c, launch_move_rows(src->vecs.p, rows.as<int64_t>(), n_rows, (int64_t)(cs->stride * esz), p->vecs.p, s));
    }
    if (pl.n_items > 0) {
        RC(upload(c, pl.items, items.data(), items.size() * sizeof(int64_t), s));
        RC(upload(c, pl.pending_init, pend.data(), pend.size() * sizeof(int32_t), s));
        RC(dev_alloc(c, pl.pending, pend.size() * sizeof(int32_t)));
        RC(dev_alloc(c, pl.cursor, sizeof(unsigned int)));
        pl.grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident_grid(c, v, pl.waves_per_cu), pl.n_items));
        RC(enqueue_body(c, p, cs, &pl, s, nullptr, false));
    } else {
        // every child is one reused chunk (a whole subtree of a parent): nothing runs but the fitness
        HIPC(c, launch_fitness(p->vtype, fit_params(p, cs), p->n_trees, s));
    }
    p->evaluated_with = cases_h;
    HIPC(c, hipStreamSynchronize(s));            // the plan and the row list are freed on return
    if (n_evaluated) *n_evaluated = n_eval;
    return GP_OK;
}

int enqueue_incremental(Ctx* c, const std::vector<IncJob>& jobs, gp_handle cases_h, const CaseSet* cs,
                        bool want_roots, hipStream_t s, IncOut* out, int64_t* launches)
{
    const int64_t n = (int64_t)jobs.size();
    if (n == 0) return GP_OK;
    const int vtype = cs->vtype;
    std::vector<WalkChild> wc(n);
    std::vector<int64_t> doffs(n + 1, 0);
    std::vector<uint8_t> dops;
    out->equiv_nodes = 0;
    out->child_nodes.assign(n, 0);
    const size_t esz = vtype == GP_BOOL ? 8 : 4;
    for (int64_t i = 0; i < n; ++i) {
        const IncJob& j = jobs[i];
        Pop* p = j.parent;
        if (p->vtype != vtype) return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": value type mismatch");
        if (j.tree < 0 || j.tree >= p->n_trees)
            return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": parent index out of range");
        if (j.point < 0 || j.point >= p->tree_nodes[j.tree])
            return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": crossover point out of range");
        if (p->evaluated_with != cases_h)
            return set_err(c, GP_ENOTFOUND, "child " + std::to_string(i) + ": the parent population has no parent "
                                            "caches for this case set; run gp_evaluate_full on it first");
        auto it = p->spine_of.find(((uint64_t)j.tree << 32) | (uint32_t)j.point);
        if (it == p->spine_of.end())
            return set_err(c, GP_ENOTFOUND, "child " + std::to_string(i) + ": point " + std::to_string(j.point) +
                                                " of tree " + std::to_string(j.tree) + " was not recorded");
        const SpineInfo& si = p->spines[it->second];
        if (j.donor_len < 1 || !j.donor) return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": empty donor");
        WalkChild& w = wc[i];
        w.levels = p->levels.as<SpineLvl>() + si.level_off;
        w.recs = (const uint8_t*)p->recs.p + (size_t)p->rec_base[j.tree] * cs->stride * esz;
        w.parent_vec = (const uint8_t*)p->vecs.p + (size_t)j.tree * cs->stride * esz;
        w.parent_fit = (const uint8_t*)p->fit.p + (size_t)j.tree * 8;
        w.n_levels = si.n_levels;
        w.at_point = si.at_point;
        w.donor_slot = (int32_t)i;
        w.pad = 0;
        w.donor_nodes = j.donor_len;
        out->child_nodes[i] = p->tree_nodes[j.tree] - si.removed_nodes + j.donor_len;
        out->equiv_nodes += out->child_nodes[i];
        dops.insert(dops.end(), j.donor, j.donor + j.donor_len);
        doffs[i + 1] = (int64_t)dops.size();
    }
    // Inserted subtrees: evaluated on every case like any population.
    RC(build_population(c, vtype, GP_PREFIX, jobs[0].parent->n_inputs, n, dops.data(), doffs.data(), nullptr,
                        nullptr, 0, &out->donors, s));
    const Launch L = choose_launch(c, vtype, cs, &out->donors);
    if (L.variant < 0) return set_err(c, GP_EINVAL, "no interpreter variant fits the donors");
    RC(upload(c, out->wc, wc.data(), wc.size() * sizeof(WalkChild), s));
    RC(dev_alloc(c, out->root, want_roots ? (size_t)n * cs->stride * esz : 256));
    RC(dev_alloc(c, out->fit, (size_t)n * 8));
    RC(dev_alloc(c, out->stop, (size_t)n * 4));
    RC(dev_alloc(c, out->interp, (size_t)n * 8));
    RC(enqueue_full(c, &out->donors, cases_h, cs, L, false, false, s, launches));
    WalkParams wp;
    wp.children = out->wc.as<WalkChild>();
    wp.inputs = cs->inputs.p;
    wp.donor_vecs = out->donors.vecs.p;
    wp.target = cs->target.p;
    wp.root_out = want_roots ? out->root.p : nullptr;
    wp.fit_out = out->fit.p;
    wp.stop_out = out->stop.as<int32_t>();
    wp.interp_out = out->interp.as<int64_t>();
    wp.stride = cs->stride;
    wp.n_valid = cs->T;
    wp.P = cs->P;
    HIPC(c, launch_walk(vtype, wp, n, s));
    if (launches) ++*launches;
    return GP_OK;
}

// Co-evaluation (Section 6.2): the mother is re-evaluated alongside her child
// from the crossover point up.  Round 0 evaluates every donor and every removed
// subtree; each round then evaluates, as one batched population, the sibling
// subtrees of the next levels of every child still walking (a budget of
// sibling nodes per child that grows eightfold per round, at least one level),
// and one co-evaluation launch walks those levels.  Siblings evaluated past a
// stop are the only wasted work, bounded by the budget growth.
int enqueue_coeval(Ctx* c, const std::vector<IncJob>& jobs, gp_handle cases_h, const CaseSet* cs,
                   bool want_roots, hipStream_t s, IncOut* out, int64_t* launches, int64_t* rounds)
{
    const int64_t n = (int64_t)jobs.size();
    if (n == 0) return GP_OK;
    Pop* p = jobs[0].parent;
    const int vtype = cs->vtype;
    const size_t esz = vtype == GP_BOOL ? 8 : 4;
    if (p->vtype != vtype) return set_err(c, GP_EINVAL, "value type mismatch");
    if (p->layout != GP_PREFIX) return set_err(c, GP_EINVAL, "co-evaluation needs a population loaded in prefix layout");
    if (p->host_ops.empty()) return set_err(c, GP_EINVAL, "the population keeps no copy of its trees");
    if (p->evaluated_with != cases_h)
        return set_err(c, GP_ENOTFOUND, "the mother population has not been evaluated on this case set; run "
                                        "gp_evaluate_full on it first");
    for (int64_t i = 0; i < n; ++i) {
        const IncJob& j = jobs[i];
        if (j.tree < 0 || j.tree >= p->n_trees)
            return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": parent index out of range");
        if (j.point < 0 || j.point >= p->tree_nodes[j.tree])
            return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": crossover point out of range");
        if (j.donor_len < 1 || !j.donor) return set_err(c, GP_EINVAL, "child " + std::to_string(i) + ": empty donor");
    }
    auto tree_of = [&](int64_t i) { return p->host_ops.data() + p->host_offsets[jobs[i].tree]; };
    const int nth_max = (int)std::min<int64_t>(16, std::max(1u, std::thread::hardware_concurrency()));
    auto parallel = [&](int64_t count, const std::function<void(int64_t)>& fn) {
        std::atomic<int64_t> next{0};
        auto work = [&]() {
            for (int64_t i; (i = next++) < count;) fn(i);
        };
        const int nth = (int)std::min<int64_t>(nth_max, count);
        std::vector<std::thread> th;
        for (int k = 1; k < nth; ++k) th.emplace_back(work);
        work();
        for (auto& t : th) t.join();
    };
    // the index of large subtrees, once per tree
    if (p->big_built.size() != (size_t)p->n_trees) {
        p->big_built.assign(p->n_trees, 0);
        p->big_ends.assign(p->n_trees, {});
    }
    std::vector<int64_t> need;
    for (int64_t i = 0; i < n; ++i)
        if (!p->big_built[jobs[i].tree]) {
            p->big_built[jobs[i].tree] = 1;
            need.push_back(jobs[i].tree);
        }
    parallel((int64_t)need.size(), [&](int64_t k) {
        const int64_t t = need[k];
        big_subtree_ends(p->host_ops.data() + p->host_offsets[t], p->tree_nodes[t], kBigSubtree, &p->big_ends[t]);
    });
    std::vector<std::vector<PathLevel>> path(n);
    std::vector<int64_t> rend(n);
    parallel(n, [&](int64_t i) {
        path_to_root(tree_of(i), p->tree_nodes[jobs[i].tree], jobs[i].point, p->big_ends[jobs[i].tree], &path[i],
                     &rend[i]);
    });
    out->equiv_nodes = 0;
    out->child_nodes.assign(n, 0);
    std::vector<int64_t> interp(n), walked(n, 0), done(n, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t removed = rend[i] - jobs[i].point;
        out->child_nodes[i] = p->tree_nodes[jobs[i].tree] - removed + jobs[i].donor_len;
        out->equiv_nodes += out->child_nodes[i];
        interp[i] = jobs[i].donor_len + removed;
    }
    RC(dev_alloc(c, out->root, want_roots ? (size_t)n * cs->stride * esz : 256));
    RC(dev_alloc(c, out->fit, (size_t)n * 8));
    RC(dev_alloc(c, out->stop, (size_t)n * 4));
    RC(dev_alloc(c, out->interp, (size_t)n * 8));
    DevBuf V, M;
    RC(dev_alloc(c, V, (size_t)n * cs->stride * esz));
    RC(dev_alloc(c, M, (size_t)n * cs->stride * esz));
    std::vector<int32_t> stop(n, -2);
    std::vector<int64_t> active(n);
    for (int64_t i = 0; i < n; ++i) active[i] = i;
    const size_t row = (size_t)cs->stride * esz;
    int64_t budget = 16384;
    int64_t r = 0;
    for (; !active.empty(); ++r, budget = std::min<int64_t>(budget * 8, int64_t(1) << 40)) {
        // A subtree's vector comes from the round's population (slot) or, when
        // the subtree is a chunk of the mother, from her last evaluation (row).
        struct Ref {
            int64_t slot, row;
            int64_t input = -1;                 // >= 0: a terminal, its case-set input row
        };
        struct Pick {
            int64_t child, first, count;
            Ref removed, donor;
            size_t refs_at;
        };
        std::vector<Pick> picks;
        std::vector<Ref> refs;                  // level siblings, pick after pick
        std::vector<uint8_t> ops;
        std::vector<int32_t> ext;               // per byte of ops: -1 or the input row it stands for
        std::vector<int64_t> ext_src;           // mother rows behind input rows n_inputs, n_inputs + 1, ...
        std::vector<int64_t> offs{0};
        const bool ckpt = vtype == GP_F32 && p->cuts.size() == (size_t)p->n_trees;
        const int64_t row_cap = ((int64_t(1) << 31) / (int64_t)row) - p->n_inputs - 1;   // row offsets stay < 2^31
        // Subtree [b, e) of child i's mother: chunks of the mother inside it are
        // read from her vectors (a placeholder terminal pushed from a gathered
        // input row); only the rest is compiled.  Returns the nodes executed.
        auto add_sub = [&](int64_t i, int64_t b, int64_t e, Ref* ref) -> int64_t {
            const uint8_t* t = tree_of(i);
            int64_t nodes = 0;
            if (e - b == 1 && !(t[b] & 0x80)) {  // a terminal: its input row, nothing to evaluate
                *ref = Ref{-1, -1, (int64_t)t[b]};
                return 0;
            }
            if (ckpt) {
                const auto& cl = p->cuts[jobs[i].tree];
                auto lb = [&](int64_t x) {
                    return std::lower_bound(cl.begin(), cl.end(), x,
                                            [](const Pop::CutSlot& a, int64_t v) { return a.node < v; });
                };
                auto it = lb(b);
                if (it != cl.end() && it->node == b && it->end == e) {
                    *ref = Ref{-1, it->slot};
                    return 0;
                }
                int64_t pos = b;
                it = lb(b + 1);
                for (;;) {
                    const int64_t u = (it != cl.end() && it->node < e) ? it->node : e;
                    ops.insert(ops.end(), t + pos, t + u);
                    ext.insert(ext.end(), (size_t)(u - pos), -1);
                    nodes += u - pos;
                    if (u == e) break;
                    if ((int64_t)ext_src.size() < row_cap) {
                        ops.push_back(0);
                        ext.push_back((int32_t)(p->n_inputs + (int64_t)ext_src.size()));
                        ext_src.push_back(it->slot);
                    } else {                    // no input row left: compile that chunk too
                        ops.insert(ops.end(), t + u, t + it->end);
                        ext.insert(ext.end(), (size_t)(it->end - u), -1);
                        nodes += it->end - u;
                    }
                    pos = it->end;
                    it = lb(pos);
                }
            } else {
                ops.insert(ops.end(), t + b, t + e);
                ext.insert(ext.end(), (size_t)(e - b), -1);
                nodes = e - b;
            }
            offs.push_back((int64_t)ops.size());
            *ref = Ref{(int64_t)offs.size() - 2, -1};
            return nodes;
        };
        for (int64_t i : active) {
            Pick pk{i, done[i], 0, Ref{-1, -1}, Ref{-1, -1}, refs.size()};
            if (r == 0) {
                interp[i] += add_sub(i, jobs[i].point, rend[i], &pk.removed) - (rend[i] - jobs[i].point);
                ops.insert(ops.end(), jobs[i].donor, jobs[i].donor + jobs[i].donor_len);
                ext.insert(ext.end(), (size_t)jobs[i].donor_len, -1);
                offs.push_back((int64_t)ops.size());
                pk.donor = Ref{(int64_t)offs.size() - 2, -1};
            }
            int64_t k = done[i], sum = 0;
            while (k < (int64_t)path[i].size()) {
                Ref rf;
                sum += add_sub(i, path[i][k].sib_begin, path[i][k].sib_end, &rf);
                refs.push_back(rf);
                ++k;
                if (sum > budget) break;
            }
            pk.count = k - pk.first;
            interp[i] += sum;
            done[i] = k;
            picks.push_back(pk);
        }
        Pop rp;
        CaseSet tcs;                            // the case set with the gathered mother rows appended
        DevBuf rows_d;
        const CaseSet* ecs = cs;
        if (offs.size() > 1) {
            if (!ext_src.empty()) {
                tcs.vtype = cs->vtype;
                tcs.n_inputs = cs->n_inputs + (int)ext_src.size();
                tcs.T = cs->T;
                tcs.n_elems = cs->n_elems;
                tcs.stride = cs->stride;
                tcs.P = cs->P;
                RC(dev_alloc(c, tcs.inputs, (size_t)tcs.n_inputs * row));
                HIPC(c, hipMemcpyAsync(tcs.inputs.p, cs->inputs.p, (size_t)cs->n_inputs * row, hipMemcpyDeviceToDevice, s));
                RC(upload(c, rows_d, ext_src.data(), ext_src.size() * sizeof(int64_t), s));
                HIPC(c, launch_gather_rows(p->vecs.p, rows_d.as<int64_t>(), (int64_t)ext_src.size(), (int64_t)row,
                                           tcs.inputs.as<uint8_t>() + (size_t)cs->n_inputs * row, s));
                RC(dev_alloc(c, tcs.target, row));
                HIPC(c, hipMemcpyAsync(tcs.target.p, cs->target.p, row, hipMemcpyDeviceToDevice, s));
                ecs = &tcs;
            }
            RC(build_population(c, vtype, GP_PREFIX, p->n_inputs, (int64_t)offs.size() - 1, ops.data(), offs.data(),
                                nullptr, nullptr, 0, &rp, s, false, ext.data()));
            const Launch L = choose_launch(c, vtype, ecs, &rp);
            if (L.variant < 0) return set_err(c, GP_EINVAL, "no interpreter variant fits the sibling subtrees");
            RC(enqueue_full(c, &rp, cases_h, ecs, L, false, false, s, launches));
        }
        const uint8_t* rv = (const uint8_t*)rp.vecs.p;
        const uint8_t* mv = (const uint8_t*)p->vecs.p;
        const uint8_t* iv = (const uint8_t*)cs->inputs.p;
        auto ptr = [&](const Ref& rf) -> const void* {
            if (rf.input >= 0) return (const void*)(iv + (size_t)rf.input * row);
            return rf.row >= 0 ? (const void*)(mv + (size_t)rf.row * row) : (const void*)(rv + (size_t)rf.slot * row);
        };
        std::vector<CoLevel> lv;
        std::vector<int64_t> lv_at(picks.size());
        for (size_t j = 0; j < picks.size(); ++j) {
            const Pick& pk = picks[j];
            lv_at[j] = (int64_t)lv.size();
            for (int64_t q = 0; q < pk.count; ++q) {
                const PathLevel& L = path[pk.child][pk.first + q];
                lv.push_back(CoLevel{ptr(refs[pk.refs_at + q]), L.f | (L.right ? 4 : 0), 0});
            }
        }
        DevBuf lvd, chd;
        if (lv.empty()) lv.push_back(CoLevel{nullptr, 0, 0});      // never read: every n_levels is 0
        RC(upload(c, lvd, lv.data(), lv.size() * sizeof(CoLevel), s));
        std::vector<CoChild> ch(picks.size());
        for (size_t j = 0; j < picks.size(); ++j) {
            const Pick& pk = picks[j];
            const int64_t i = pk.child, t = jobs[i].tree;
            CoChild& cc = ch[j];
            uint8_t* vi = V.as<uint8_t>() + (size_t)i * row;
            uint8_t* mi = M.as<uint8_t>() + (size_t)i * row;
            cc.v_in = r == 0 ? ptr(pk.donor) : vi;
            cc.m_in = r == 0 ? ptr(pk.removed) : mi;
            cc.v_out = vi;
            cc.m_out = mi;
            cc.levels = lvd.as<CoLevel>() + lv_at[j];
            cc.parent_vec = (const uint8_t*)p->vecs.p + (size_t)t * row;
            cc.parent_fit = (const uint8_t*)p->fit.p + (size_t)t * 8;
            cc.n_levels = (int32_t)pk.count;
            cc.level_base = (int32_t)pk.first;
            cc.check0 = r == 0 ? 1 : 0;
            cc.last = pk.first + pk.count == (int64_t)path[i].size() ? 1 : 0;
            cc.out_slot = (int32_t)i;
            cc.pad = 0;
        }
        if (lv.size() > 0x7fffffff || n > 0x7fffffff) return set_err(c, GP_EINVAL, "too many children or levels");
        RC(upload(c, chd, ch.data(), ch.size() * sizeof(CoChild), s));
        CoParams cp;
        cp.children = chd.as<CoChild>();
        cp.target = cs->target.p;
        cp.root_out = want_roots ? out->root.p : nullptr;
        cp.fit_out = out->fit.p;
        cp.stop_out = out->stop.as<int32_t>();
        cp.stride = cs->stride;
        cp.n_valid = cs->T;
        cp.P = cs->P;
        HIPC(c, launch_coeval(vtype, cp, (int64_t)picks.size(), s));
        if (launches) ++*launches;
        HIPC(c, hipMemcpyAsync(stop.data(), out->stop.p, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        std::vector<int64_t> still;
        for (const Pick& pk : picks) {
            const int64_t i = pk.child;
            const int32_t st = stop[i];
            walked[i] = st >= 0 ? st : pk.first + pk.count;
            if (st == -2) still.push_back(i);
        }
        active.swap(still);
    }
    for (int64_t i = 0; i < n; ++i) interp[i] += 2 * walked[i];
    RC(upload(c, out->interp, interp.data(), (size_t)n * 8, s));
    HIPC(c, hipStreamSynchronize(s));
    if (rounds) *rounds = r;
    return GP_OK;
}

}  // namespace gpe

using namespace gpe;

// =================================================================== C ABI
struct gp_ctx : public Ctx {};

static thread_local std::string g_static_err;

static double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

extern "C" {

int gp_create(int device, uint64_t hbm_budget_bytes, void* hip_stream, gp_ctx** out)
{
    if (!out) return GP_EINVAL;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        g_static_err = "no HIP device available";
        return GP_EDEVICE;
    }
    if (device < 0 || device >= n) {
        g_static_err = "device index out of range";
        return GP_EINVAL;
    }
    gp_ctx* c = new gp_ctx();
    c->device = device;
    auto fail = [&](hipError_t er, const char* what) {
        g_static_err = std::string(what) + ": " + hipGetErrorString(er);
        delete c;
        return GP_EDEVICE;
    };
    if ((e = hipSetDevice(device)) != hipSuccess) return fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_static_err = std::string("gpeval is built for gfx950, found ") + prop.gcnArchName;
        delete c;
        return GP_EDEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    c->device_name = std::string(prop.gcnArchName) + ":" + std::to_string(c->n_cu);
    size_t free_b = 0, total_b = 0;
    if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return fail(e, "hipMemGetInfo");
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
            return fail(e, "hipStreamCreate");
        c->own_stream = true;
    }
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess) return fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->ev1)) != hipSuccess) return fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->kev0)) != hipSuccess) return fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->kev1)) != hipSuccess) return fail(e, "hipEventCreate");
    // device address of the allocation-free index's scratch array on this device
    if ((e = ix_static_scratch(device, &c->ix_scratch)) != hipSuccess) return fail(e, "hipGetSymbolAddress");
    Variant* vt = variant_table();
    for (int v = 0; v < variant_count(); ++v) {
        int nb = 0;
        const size_t shm = variant_lds(vt[v], 8);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, vt[v].kernel, kWave, shm) != hipSuccess) {
            (void)hipGetLastError();
            nb = 4;
        }
        vt[v].max_blocks_per_cu = std::max(1, nb);
    }
    *out = c;
    return GP_OK;
}

int gp_server_stop(gp_ctx* ctx);

void gp_destroy(gp_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    gp_server_stop(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pops.clear();
    ctx->cases.clear();
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->kev0) (void)hipEventDestroy(ctx->kev0);
    if (ctx->kev1) (void)hipEventDestroy(ctx->kev1);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* gp_last_error(const gp_ctx* ctx)
{
    if (!ctx) return g_static_err.c_str();
    return ctx->err.c_str();
}

uint64_t gp_memory_used(const gp_ctx* ctx) { return ctx ? ctx->used.load() : 0; }

int gp_set_cases(gp_ctx* ctx, int vtype, int n_inputs, int64_t n_cases, const void* inputs,
                 const void* target, uint32_t flags, gp_handle* cases_out)
{
    if (!ctx || !cases_out) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    if (vtype != GP_F32 && vtype != GP_BOOL) return set_err(ctx, GP_EINVAL, "unknown value type");
    if (n_inputs < 1 || n_inputs > kMaxInputs) return set_err(ctx, GP_EINVAL, "n_inputs must be 1..64");
    if (n_cases < 1) return set_err(ctx, GP_EINVAL, "need at least one test case");
    if (vtype == GP_F32 && n_cases > 16384) return set_err(ctx, GP_EINVAL, "float32 case sets hold at most 16384 cases");
    if (vtype == GP_BOOL && n_cases > (int64_t(1) << 18)) return set_err(ctx, GP_EINVAL, "Boolean case sets hold at most 2^18 cases");
    if (!inputs || !target) return set_err(ctx, GP_EINVAL, "inputs and target are required");
    auto cs = std::make_shared<CaseSet>();
    cs->vtype = vtype;
    cs->n_inputs = n_inputs;
    cs->T = n_cases;
    cs->n_elems = elems_of(vtype, n_cases);
    cs->stride = pad_to(cs->n_elems, kPadCases);
    int64_t P = 64;
    while (P < n_cases) P *= 2;
    cs->P = P;
    const size_t esz = vtype == GP_BOOL ? 8 : 4;
    RC(dev_alloc(ctx, cs->inputs, (size_t)n_inputs * cs->stride * esz));
    RC(dev_alloc(ctx, cs->target, (size_t)cs->stride * esz));
    // zero padding keeps the unused lanes' arithmetic well defined
    std::vector<uint8_t> zeros((size_t)cs->stride * esz, 0);
    for (int j = 0; j < n_inputs; ++j)
        HIPC(ctx, hipMemcpyAsync(cs->inputs.as<uint8_t>() + (size_t)j * cs->stride * esz, zeros.data(),
                                 zeros.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPC(ctx, hipMemcpyAsync(cs->target.p, zeros.data(), zeros.size(), hipMemcpyHostToDevice, ctx->stream));
    const hipMemcpyKind kind = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPC(ctx, hipMemcpy2DAsync(cs->inputs.p, cs->stride * esz, inputs, cs->n_elems * esz, cs->n_elems * esz,
                               n_inputs, kind, ctx->stream));
    HIPC(ctx, hipMemcpyAsync(cs->target.p, target, cs->n_elems * esz, kind, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    gp_handle h = ctx->next_handle++;
    ctx->cases[h] = cs;
    *cases_out = h;
    return GP_OK;
}

// dst = src[0 .. n), in slices on up to 16 threads when large.
static void copy_host_bytes(std::vector<uint8_t, NoInitAlloc<uint8_t>>& dst, const uint8_t* src, size_t n)
{
    dst.resize(n);
    const size_t slice = size_t(64) << 20;
    const int nth = (int)std::min<size_t>({16, std::max(1u, std::thread::hardware_concurrency()), n / slice + 1});
    if (nth <= 1) {
        std::memcpy(dst.data(), src, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
            const size_t a = n * t / nth, b = n * (t + 1) / nth;
            std::memcpy(dst.data() + a, src + a, b - a);
        });
    for (auto& x : th) x.join();
}

int gp_load_population(gp_ctx* ctx, int vtype, int layout, int n_inputs, int64_t n_trees, const uint8_t* ops,
                       const int64_t* offsets, const int64_t* record_points, const int64_t* record_offsets,
                       int64_t chunk_nodes, uint32_t flags, gp_handle* pop_out)
{
    if (!ctx || !pop_out) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    auto p = std::make_shared<Pop>();
    if (flags & (GP_DEVICE_PTR | GP_DEVICE_COMPILE)) {
        if (layout != GP_PREFIX) return set_err(ctx, GP_EINVAL, "device compilation takes prefix trees");
        if (!ops || !offsets || n_trees < 1) return set_err(ctx, GP_EINVAL, "empty population");
        if (n_trees > INT32_MAX / 2) return set_err(ctx, GP_EINVAL, "too many trees");
        const bool on_dev = (flags & GP_DEVICE_PTR) != 0;
        std::vector<int64_t> hoff;
        const int64_t* offs = offsets;
        if (on_dev) {
            hoff.resize(n_trees + 1);
            HIPC(ctx, hipMemcpy(hoff.data(), offsets, (size_t)(n_trees + 1) * 8, hipMemcpyDeviceToHost));
            offs = hoff.data();
        }
        DevBuf keep;
        int rc = GP_OK;
        try {
            rc = build_population_device(ctx, vtype, n_inputs, n_trees, on_dev ? nullptr : ops,
                                         on_dev ? ops : nullptr, offs, record_points, record_offsets, chunk_nodes,
                                         p.get(), (flags & GP_KEEP_TREES) ? &keep : nullptr);
        } catch (const std::bad_alloc&) {
            rc = set_err(ctx, GP_ENOMEM, "out of host memory while compiling on the device");
        }
        RC(rc);
        p->auto_chunk = chunk_nodes <= 0;
        const size_t nb = (size_t)offs[n_trees];
        if (on_dev) {
            p->host_ops.resize(nb);
            HIPC(ctx, hipMemcpy(p->host_ops.data(), ops, nb, hipMemcpyDeviceToHost));
        } else {
            copy_host_bytes(p->host_ops, ops, nb);
        }
        p->host_offsets.assign(offs, offs + n_trees + 1);
        if (flags & GP_KEEP_TREES) {
            p->tree_ops.swap(keep);
            p->tree_off = p->host_offsets;
        }
        if (p->auto_chunk && record_points) {
            p->host_rec_offsets.assign(record_offsets, record_offsets + n_trees + 1);
            p->host_rec_points.assign(record_points, record_points + record_offsets[n_trees]);
        }
        gp_handle h = ctx->next_handle++;
        ctx->pops[h] = p;
        *pop_out = h;
        return GP_OK;
    }
    RC(build_population(ctx, vtype, layout, n_inputs, n_trees, ops, offsets, record_points, record_offsets,
                        chunk_nodes, p.get(), ctx->stream, true));
    p->auto_chunk = chunk_nodes <= 0;
    // host copy of the trees: re-chunking by the autotuner, sibling subtrees
    // for co-evaluation
    copy_host_bytes(p->host_ops, ops, (size_t)offsets[n_trees]);
    p->host_offsets.assign(offsets, offsets + n_trees + 1);
    if (flags & GP_KEEP_TREES) {
        const size_t nb = (size_t)offsets[n_trees];
        RC(dev_alloc(ctx, p->tree_ops, nb + 32));
        HIPC(ctx, hipMemcpyAsync(p->tree_ops.p, ops, nb, hipMemcpyHostToDevice, ctx->stream));
        p->tree_off.assign(offsets, offsets + n_trees + 1);
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (p->auto_chunk) {
        if (record_points) {
            p->host_rec_offsets.assign(record_offsets, record_offsets + n_trees + 1);
            p->host_rec_points.assign(record_points, record_points + record_offsets[n_trees]);
        }
    }
    gp_handle h = ctx->next_handle++;
    ctx->pops[h] = p;
    *pop_out = h;
    return GP_OK;
}

int gp_population_info(gp_ctx* ctx, gp_handle pop, gp_pop_info* out)
{
    if (!ctx || !out) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->pops.find(pop);
    if (it == ctx->pops.end()) return set_err(ctx, GP_EINVAL, "unknown population handle");
    Pop* p = it->second.get();
    out->n_trees = p->n_trees;
    out->total_nodes = p->total_nodes;
    out->n_chunks = p->n_chunks;
    out->n_instructions = p->n_code;
    out->n_records = p->n_records;
    out->n_spines = (int64_t)p->spines.size();
    uint64_t b = p->code.bytes + p->chunks.bytes + p->chunk_in.bytes + p->levels.bytes + p->vecs.bytes +
                 p->recs.bytes + p->fit.bytes;
    for (auto& kv : p->plans)
        b += kv.second->items.bytes + kv.second->pending.bytes + kv.second->pending_init.bytes + kv.second->cursor.bytes;
    out->device_bytes = (int64_t)b;
    out->max_stack = p->max_stack;
    out->chunk_nodes = (int32_t)p->chunk_nodes;
    out->max_code_len = p->max_code_len;
    return GP_OK;
}

// The compiled form of a population as one byte string: sections, each an
// int64 byte count and its bytes, in the order documented in gpeval.h.
static int dump_population(Ctx* c, const Pop* p, std::vector<uint8_t>* out)
{
    out->clear();
    auto sec = [&](const void* src, size_t bytes) {
        const int64_t b = (int64_t)bytes;
        const uint8_t* q = (const uint8_t*)&b;
        out->insert(out->end(), q, q + 8);
        out->insert(out->end(), (const uint8_t*)src, (const uint8_t*)src + bytes);
    };
    auto dev_sec = [&](const DevBuf& b, size_t bytes) -> int {
        std::vector<uint8_t> h(bytes);
        if (bytes) HIPC(c, hipMemcpy(h.data(), b.p, bytes, hipMemcpyDeviceToHost));
        sec(h.data(), bytes);
        return GP_OK;
    };
    const int64_t head[8] = {p->n_trees, p->n_chunks, p->n_code, p->n_records, p->max_stack, p->chunk_nodes,
                             p->total_nodes, p->layout};
    sec(head, sizeof(head));
    RC(dev_sec(p->code, (size_t)(p->n_code + 1) * 4));
    RC(dev_sec(p->chunks, (size_t)p->n_chunks * sizeof(DevChunk)));
    int64_t n_in = 0, n_lv = 0;
    for (int32_t v : p->chunk_n_in) n_in += v;
    for (const auto& si : p->spines) n_lv += si.n_levels;
    RC(dev_sec(p->chunk_in, (size_t)n_in * 4));
    sec(p->chunk_n_in.data(), p->chunk_n_in.size() * 4);
    sec(p->chunk_tree.data(), p->chunk_tree.size() * 4);
    sec(p->rec_base.data(), p->rec_base.size() * 8);
    std::vector<int64_t> v;
    for (const auto& lf : p->leaves) {
        v.push_back(lf.first);
        v.push_back(lf.second);
    }
    sec(v.data(), v.size() * 8);
    v.clear();
    for (const auto& si : p->spines) {
        for (int64_t x : {(int64_t)si.tree, (int64_t)si.at_point, si.level_off, (int64_t)si.n_levels, si.removed_nodes})
            v.push_back(x);
    }
    sec(v.data(), v.size() * 8);
    std::vector<std::pair<uint64_t, int32_t>> keys(p->spine_of.begin(), p->spine_of.end());
    std::sort(keys.begin(), keys.end());
    v.clear();
    for (const auto& kv : keys) {
        v.push_back((int64_t)kv.first);
        v.push_back(kv.second);
    }
    sec(v.data(), v.size() * 8);
    RC(dev_sec(p->levels, (size_t)n_lv * sizeof(SpineLvl)));
    v.clear();
    for (const auto& be : p->big_ends) {
        v.push_back((int64_t)be.size());
        for (const auto& x : be) {
            v.push_back(x.first);
            v.push_back(x.second);
        }
    }
    sec(v.data(), v.size() * 8);
    v.clear();
    for (const auto& cl : p->cuts) {
        v.push_back((int64_t)cl.size());
        for (const auto& x : cl)
            for (int64_t y : {(int64_t)x.node, (int64_t)x.end, (int64_t)x.slot}) v.push_back(y);
    }
    sec(v.data(), v.size() * 8);
    v.clear();
    for (const auto& kc : p->kept_chunks) {
        v.push_back((int64_t)kc.size());
        for (const Chunk& ch : kc) {
            for (int64_t y : {ch.code_off, ch.code_len, (int64_t)ch.parent, ch.root_node, ch.nodes, ch.path_nodes,
                              ch.end_node, ch.dev_src, (int64_t)ch.stores, ch.vec_slot, ch.src_vec,
                              (int64_t)ch.inputs.size()})
                v.push_back(y);
            for (int32_t y : ch.inputs) v.push_back(y);
        }
    }
    sec(v.data(), v.size() * 8);
    sec(p->kept_max_stack.data(), p->kept_max_stack.size() * 4);
    sec(p->tree_nodes.data(), p->tree_nodes.size() * 8);
    return GP_OK;
}

int gp_population_dump(gp_ctx* ctx, gp_handle pop, uint8_t* out, int64_t cap, int64_t* size)
{
    if (!ctx || !size) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    auto it = ctx->pops.find(pop);
    if (it == ctx->pops.end()) return set_err(ctx, GP_EINVAL, "unknown population handle");
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<uint8_t> d;
    RC(dump_population(ctx, it->second.get(), &d));
    *size = (int64_t)d.size();
    if (!out) return GP_OK;
    if (cap < (int64_t)d.size()) return set_err(ctx, GP_EINVAL, "dump buffer too small");
    std::memcpy(out, d.data(), d.size());
    return GP_OK;
}

int gp_free(gp_ctx* ctx, gp_handle h)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->pops.erase(h)) return GP_OK;
    if (ctx->cases.erase(h)) {
        for (auto& kv : ctx->pops) {
            if (kv.second->evaluated_with == h) kv.second->evaluated_with = 0;
            for (auto& pk : kv.second->plans)
                if (pk.second->graph_cases == h && pk.second->graph) {
                    (void)hipGraphExecDestroy(pk.second->graph);
                    pk.second->graph = nullptr;
                    pk.second->graph_cases = 0;
                }
        }
        return GP_OK;
    }
    return set_err(ctx, GP_EINVAL, "unknown handle");
}

static int lookup(gp_ctx* ctx, gp_handle pop, gp_handle cases, Pop** p, CaseSet** cs)
{
    auto ip = ctx->pops.find(pop);
    if (ip == ctx->pops.end()) return set_err(ctx, GP_EINVAL, "unknown population handle");
    auto ic = ctx->cases.find(cases);
    if (ic == ctx->cases.end()) return set_err(ctx, GP_EINVAL, "unknown case-set handle");
    *p = ip->second.get();
    *cs = ic->second.get();
    if ((*p)->vtype != (*cs)->vtype) return set_err(ctx, GP_EINVAL, "population and case set differ in value type");
    if ((*p)->n_inputs > (*cs)->n_inputs)
        return set_err(ctx, GP_EINVAL, "population uses more inputs than the case set provides");
    return GP_OK;
}

static int copy_out(gp_ctx* ctx, void* dst, const void* src, int64_t rows, int64_t elems, int64_t stride,
                    size_t esz, uint32_t flags)
{
    if (!dst || rows <= 0) return GP_OK;
    const hipMemcpyKind kind = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPC(ctx, hipMemcpy2DAsync(dst, elems * esz, src, stride * esz, elems * esz, rows, kind, ctx->stream));
    return GP_OK;
}

int gp_evaluate_full(gp_ctx* ctx, gp_handle pop, gp_handle cases, uint32_t flags, void* root_out,
                     void* fitness_out, gp_stats* st)
{
    if (!ctx) return GP_EINVAL;
    const double t0 = now_ms();
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    Pop* p;
    CaseSet* cs;
    RC(lookup(ctx, pop, cases, &p, &cs));
    if ((flags & GP_ASYNC) && !(flags & GP_DEVICE_PTR))
        return set_err(ctx, GP_EINVAL, "GP_ASYNC needs GP_DEVICE_PTR outputs");
    const Launch L = choose_launch(ctx, p->vtype, cs, p);
    if (L.variant < 0) return set_err(ctx, GP_EINVAL, "no interpreter variant fits this population");
    const bool per_tree = (flags & GP_PER_TREE) != 0;
    const bool graph = !(flags & GP_NO_GRAPH);
    int64_t launches = 0;
    HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    RC(enqueue_full(ctx, p, cases, cs, L, per_tree, graph, ctx->stream, &launches, !graph));
    HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    const size_t esz = p->vtype == GP_BOOL ? 8 : 4;
    RC(copy_out(ctx, root_out, p->vecs.p, p->n_trees, cs->n_elems, cs->stride, esz, flags));
    if (fitness_out) {
        const hipMemcpyKind kind = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIPC(ctx, hipMemcpyAsync(fitness_out, p->fit.p, (size_t)p->n_trees * 8, kind, ctx->stream));
    }
    float ms = 0.f, kms = 0.f;
    if (!(flags & GP_ASYNC)) {
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
        HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        if (!graph) HIPC(ctx, hipEventElapsedTime(&kms, ctx->kev0, ctx->kev1));
    }
    if (st) {
        st->device_ms = ms;
        st->kernel_ms = kms;
        st->equivalent_ops = p->total_nodes * cs->T;
        st->interpreted_ops = p->total_nodes * cs->T;
        st->launches = launches;
        st->variant = L.variant;
        st->waves_per_cu = std::max(0, L.waves_per_cu);
        st->wall_ms = now_ms() - t0;
    }
    return GP_OK;
}

int gp_fitness(gp_ctx* ctx, gp_handle cases, const void* outputs, int64_t n, uint32_t flags, void* fitness_out)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    auto ic = ctx->cases.find(cases);
    if (ic == ctx->cases.end()) return set_err(ctx, GP_EINVAL, "unknown case-set handle");
    CaseSet* cs = ic->second.get();
    if (n < 0 || (n > 0 && (!outputs || !fitness_out))) return set_err(ctx, GP_EINVAL, "bad outputs");
    if (n == 0) return GP_OK;
    const size_t esz = cs->vtype == GP_BOOL ? 8 : 4;
    DevBuf vecs, fit;
    RC(dev_alloc(ctx, vecs, (size_t)n * cs->stride * esz));
    RC(dev_alloc(ctx, fit, (size_t)n * 8));
    const hipMemcpyKind kin = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPC(ctx, hipMemcpy2DAsync(vecs.p, cs->stride * esz, outputs, cs->n_elems * esz, cs->n_elems * esz, n, kin,
                               ctx->stream));
    FitParams f;
    f.vecs = vecs.p;
    f.first_slot = 0;
    f.target = cs->target.p;
    f.fit_out = fit.p;
    f.stride = cs->stride;
    f.n_valid = cs->T;
    f.P = cs->P;
    HIPC(ctx, launch_fitness(cs->vtype, f, n, ctx->stream));
    const hipMemcpyKind kout = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPC(ctx, hipMemcpyAsync(fitness_out, fit.p, (size_t)n * 8, kout, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    return GP_OK;
}

int gp_evaluate_incremental_batch(gp_ctx* ctx, gp_handle pop, gp_handle cases, int64_t n_children,
                                  const int64_t* parent, const int64_t* point, const uint8_t* donor_ops,
                                  const int64_t* donor_offsets, uint32_t flags, void* root_out,
                                  void* fitness_out, gp_inc_result* res, gp_stats* st)
{
    if (!ctx) return GP_EINVAL;
    const double t0 = now_ms();
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    Pop* p;
    CaseSet* cs;
    RC(lookup(ctx, pop, cases, &p, &cs));
    if (n_children < 0) return set_err(ctx, GP_EINVAL, "negative child count");
    if (n_children == 0) return GP_OK;
    if (!parent || !point || !donor_ops || !donor_offsets) return set_err(ctx, GP_EINVAL, "missing child arrays");
    if ((flags & GP_ASYNC) && !(flags & GP_DEVICE_PTR))
        return set_err(ctx, GP_EINVAL, "GP_ASYNC needs GP_DEVICE_PTR outputs");
    if (donor_offsets[0] != 0) return set_err(ctx, GP_EINVAL, "donor_offsets[0] must be 0");
    std::vector<IncJob> jobs(n_children);
    std::vector<std::vector<uint8_t>> converted;   // donors given in postfix order
    if (p->layout == GP_POSTFIX) converted.resize(n_children);
    for (int64_t i = 0; i < n_children; ++i) {
        if (donor_offsets[i + 1] < donor_offsets[i]) return set_err(ctx, GP_EINVAL, "donor_offsets not increasing");
        const uint8_t* d = donor_ops + donor_offsets[i];
        const int64_t nd = donor_offsets[i + 1] - donor_offsets[i];
        if (p->layout == GP_POSTFIX) {
            std::vector<int64_t> map;
            std::string why;
            if (!postfix_to_prefix(d, nd, p->n_inputs, &converted[i], &map, &why))
                return set_err(ctx, GP_EINVAL, "donor " + std::to_string(i) + ": " + why);
            d = converted[i].data();
        }
        jobs[i] = IncJob{p, parent[i], point[i], d, nd};
    }
    IncOut io;
    int64_t launches = 0;
    if ((flags & GP_COEVAL) && (flags & GP_ASYNC))
        return set_err(ctx, GP_EINVAL, "GP_COEVAL runs synchronously; GP_ASYNC is not accepted with it");
    HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (flags & GP_COEVAL)
        RC(enqueue_coeval(ctx, jobs, cases, cs, root_out != nullptr, ctx->stream, &io, &launches, nullptr));
    else
        RC(enqueue_incremental(ctx, jobs, cases, cs, root_out != nullptr, ctx->stream, &io, &launches));
    HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    const size_t esz = p->vtype == GP_BOOL ? 8 : 4;
    RC(copy_out(ctx, root_out, io.root.p, n_children, cs->n_elems, cs->stride, esz, flags));
    if (fitness_out) {
        const hipMemcpyKind kind = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIPC(ctx, hipMemcpyAsync(fitness_out, io.fit.p, (size_t)n_children * 8, kind, ctx->stream));
    }
    std::vector<int32_t> stop(n_children);
    std::vector<int64_t> interp(n_children);
    HIPC(ctx, hipMemcpyAsync(stop.data(), io.stop.p, (size_t)n_children * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(ctx, hipMemcpyAsync(interp.data(), io.interp.p, (size_t)n_children * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    int64_t interp_total = 0;
    for (int64_t i = 0; i < n_children; ++i) {
        if (res) {
            res[i].stop_level = stop[i];
            res[i].reserved = 0;
            res[i].child_nodes = io.child_nodes[i];
            res[i].interpreted_nodes = interp[i];
        }
        interp_total += interp[i];
    }
    if (st) {
        st->device_ms = ms;
        st->kernel_ms = 0;
        st->equivalent_ops = io.equiv_nodes * cs->T;
        st->interpreted_ops = interp_total * cs->T;
        st->launches = launches;
        st->variant = -1;
        st->wall_ms = now_ms() - t0;
    }
    return GP_OK;
}

int gp_splice_children(gp_ctx* ctx, gp_handle pop, int64_t n_children, const int64_t* parent,
                       const int64_t* point, const uint8_t* donor_ops, const int64_t* donor_offsets,
                       uint32_t flags, uint8_t* child_ops, int64_t child_cap, int64_t* child_offsets,
                       gp_stats* st)
{
    if (!ctx) return GP_EINVAL;
    const double t0 = now_ms();
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    auto ip = ctx->pops.find(pop);
    if (ip == ctx->pops.end()) return set_err(ctx, GP_EINVAL, "unknown population handle");
    Pop* p = ip->second.get();
    if (n_children < 0) return set_err(ctx, GP_EINVAL, "negative child count");
    if (!child_offsets) return set_err(ctx, GP_EINVAL, "child_offsets is required");
    if (n_children > 0 && (!parent || !point || !donor_ops || !donor_offsets))
        return set_err(ctx, GP_EINVAL, "missing child arrays");
    if (!p->tree_ops.p) return set_err(ctx, GP_EINVAL, "the population was loaded without GP_KEEP_TREES");
    if (n_children > 0 && donor_offsets[0] != 0) return set_err(ctx, GP_EINVAL, "donor_offsets[0] must be 0");
    // Extents: child i = mother[0, a) + donor + mother[a + removed, n).
    std::vector<int64_t> offs(n_children + 1, 0), cut(n_children), removed(n_children);
    std::vector<uint8_t> pre;
    std::vector<int64_t> map;
    for (int64_t i = 0; i < n_children; ++i) {
        const std::string who = "child " + std::to_string(i) + ": ";
        const int64_t t = parent[i];
        if (t < 0 || t >= p->n_trees) return set_err(ctx, GP_EINVAL, who + "parent index out of range");
        if (point[i] < 0 || point[i] >= p->tree_nodes[t])
            return set_err(ctx, GP_EINVAL, who + "crossover point out of range");
        auto it = p->spine_of.find(((uint64_t)t << 32) | (uint32_t)point[i]);
        if (it == p->spine_of.end())
            return set_err(ctx, GP_ENOTFOUND, who + "point " + std::to_string(point[i]) + " of tree " +
                                                  std::to_string(t) + " was not recorded");
        const int64_t nd = donor_offsets[i + 1] - donor_offsets[i];
        if (nd < 1) return set_err(ctx, GP_EINVAL, who + "empty donor");
        const uint8_t* d = donor_ops + donor_offsets[i];
        std::string why;
        const bool ok = p->layout == GP_POSTFIX ? postfix_to_prefix(d, nd, p->n_inputs, &pre, &map, &why)
                                                : validate_prefix(d, nd, p->n_inputs, &why);
        if (!ok) return set_err(ctx, GP_EINVAL, who + "donor: " + why);
        removed[i] = p->spines[it->second].removed_nodes;
        cut[i] = p->layout == GP_POSTFIX ? point[i] - removed[i] + 1 : point[i];
        offs[i + 1] = offs[i] + p->tree_nodes[t] - removed[i] + nd;
    }
    const int64_t total = offs[n_children];
    float ms = 0.f;
    if (child_ops && total > 0) {
        if (child_cap < total)
            return set_err(ctx, GP_EINVAL, "child_ops holds " + std::to_string(child_cap) + " bytes; the children need " +
                                               std::to_string(total));
        DevBuf dd, items_d, stage;
        const int64_t nb = donor_offsets[n_children];
        RC(dev_alloc(ctx, dd, (size_t)nb + 32));
        HIPC(ctx, hipMemcpyAsync(dd.p, donor_ops, (size_t)nb, hipMemcpyHostToDevice, ctx->stream));
        uint8_t* out = child_ops;
        if (!(flags & GP_DEVICE_PTR)) {
            RC(dev_alloc(ctx, stage, (size_t)total));
            out = stage.as<uint8_t>();
        }
        // Pieces of at most 64 KiB that meet at 16-byte aligned output offsets.
        std::vector<SpliceItem> items;
        items.reserve((size_t)(total >> 16) + 3 * (size_t)n_children + 8);
        auto add = [&](const uint8_t* src, int64_t dst, int64_t len) {
            while (len > 0) {
                int64_t take = std::min<int64_t>(len, ((dst + 65536) & ~int64_t(15)) - dst);
                items.push_back(SpliceItem{src, dst, take});
                src += take;
                dst += take;
                len -= take;
            }
        };
        const uint8_t* base = p->tree_ops.as<uint8_t>();
        for (int64_t i = 0; i < n_children; ++i) {
            const int64_t t = parent[i], n = p->tree_nodes[t], nd = donor_offsets[i + 1] - donor_offsets[i];
            const uint8_t* m = base + p->tree_off[t];
            add(m, offs[i], cut[i]);
            add(dd.as<uint8_t>() + donor_offsets[i], offs[i] + cut[i], nd);
            add(m + cut[i] + removed[i], offs[i] + cut[i] + nd, n - cut[i] - removed[i]);
        }
        if ((int64_t)items.size() > (int64_t(1) << 24))
            return set_err(ctx, GP_EINVAL, "too many bytes for one splice launch");
        RC(upload(ctx, items_d, items.data(), items.size() * sizeof(SpliceItem), ctx->stream));
        HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        HIPC(ctx, launch_splice(items_d.as<SpliceItem>(), (int64_t)items.size(), out, ctx->stream));
        HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
        if (!(flags & GP_DEVICE_PTR))
            HIPC(ctx, hipMemcpyAsync(child_ops, out, (size_t)total, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
        HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    }
    std::copy(offs.begin(), offs.end(), child_offsets);
    if (st) {
        st->device_ms = ms;
        st->kernel_ms = ms;
        st->equivalent_ops = child_ops ? total : 0;
        st->interpreted_ops = 0;
        st->launches = child_ops && total > 0 ? 1 : 0;
        st->variant = -1;
        st->wall_ms = now_ms() - t0;
    }
    return GP_OK;
}

int gp_population_ops(gp_ctx* ctx, gp_handle pop, uint8_t* ops_out, int64_t ops_cap, int64_t* offsets_out)
{
    if (!ctx || !offsets_out) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->pops.find(pop);
    if (it == ctx->pops.end()) return set_err(ctx, GP_EINVAL, "unknown population handle");
    const Pop* p = it->second.get();
    if (p->host_offsets.size() != (size_t)p->n_trees + 1)
        return set_err(ctx, GP_EINVAL, "the population keeps no copy of its trees");
    const int64_t total = p->host_offsets[p->n_trees];
    if (ops_out) {
        if (ops_cap < total) return set_err(ctx, GP_EINVAL, "ops_out holds fewer bytes than the trees");
        std::memcpy(ops_out, p->host_ops.data(), (size_t)total);
    }
    std::copy(p->host_offsets.begin(), p->host_offsets.end(), offsets_out);
    return GP_OK;
}

int gp_population_results(gp_ctx* ctx, gp_handle pop, gp_handle cases, uint32_t flags, void* root_out,
                          void* fitness_out)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    Pop* p;
    CaseSet* cs;
    RC(lookup(ctx, pop, cases, &p, &cs));
    if (p->evaluated_with != cases || !p->vecs.p)
        return set_err(ctx, GP_ENOTFOUND, "the population's last full evaluation was not on this case set");
    const size_t esz = p->vtype == GP_BOOL ? 8 : 4;
    RC(copy_out(ctx, root_out, p->vecs.p, p->n_trees, cs->n_elems, cs->stride, esz, flags));
    if (fitness_out) {
        const hipMemcpyKind kind = (flags & GP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIPC(ctx, hipMemcpyAsync(fitness_out, p->fit.p, (size_t)p->n_trees * 8, kind, ctx->stream));
    }
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    return GP_OK;
}

int gp_evolve(gp_ctx* ctx, gp_handle pop, gp_handle cases, const gp_evolve_cfg* cfg, gp_gen_stats* stats,
              gp_gen_child* children, gp_handle* out_pop)
{
    if (!ctx || !cfg || !out_pop) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    Pop* p0;
    CaseSet* cs;
    RC(lookup(ctx, pop, cases, &p0, &cs));
    const int64_t G = cfg->generations, N = p0->n_trees;
    if (G < 1 || cfg->tournament < 1) return set_err(ctx, GP_EINVAL, "need generations >= 1 and tournament >= 1");
    if (cfg->first_generation < 0 || cfg->first_generation + G >= (int64_t(1) << 32))
        return set_err(ctx, GP_EINVAL, "generation counters must stay below 2^32");
    if (N < 1 || N >= (int64_t(1) << 31)) return set_err(ctx, GP_EINVAL, "population size out of range");
    if (p0->layout != GP_PREFIX) return set_err(ctx, GP_EINVAL, "evolution needs a population loaded in prefix layout");
    if (p0->evaluated_with != cases)
        return set_err(ctx, GP_ENOTFOUND, "the population has not been evaluated on this case set; run "
                                          "gp_evaluate_full on it first");
    const int vtype = p0->vtype;
    const bool boolean = vtype == GP_BOOL;
    hipStream_t s = ctx->stream;
    std::shared_ptr<Pop> holder;                 // the current generation once it is not the caller's
    Pop* cur = p0;
    std::vector<int64_t> slot_tree(N), slot_size(N);
    for (int64_t i = 0; i < N; ++i) {
        slot_tree[i] = i;
        slot_size[i] = p0->tree_nodes[i];
    }
    DevBuf fitv, fitn, sizes_d, sel, drawn_d;
    RC(dev_alloc(ctx, fitv, (size_t)N * 8));
    RC(dev_alloc(ctx, fitn, (size_t)N * 8));
    RC(dev_alloc(ctx, sel, (size_t)N * 4 * 8));
    RC(dev_alloc(ctx, drawn_d, (size_t)N * 4));
    HIPC(ctx, hipMemcpyAsync(fitv.p, p0->fit.p, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
    std::vector<int64_t> pick((size_t)N * 4);
    std::vector<int32_t> stop(N), drawn(N);
    std::vector<int64_t> interp(N), removed(N), dend(N);
    std::vector<uint8_t> fit_h((size_t)N * 8);
    DevBuf spare_vecs;
    for (int64_t gi = 0; gi < G; ++gi) {
        const double t0 = now_ms();
        const int64_t g = cfg->first_generation + gi;
        const int64_t* mother = pick.data();
        const int64_t* father = mother + N;
        const int64_t* point = father + N;
        const int64_t* dnode = point + N;
        // parents, points and donor nodes, drawn on the device
        RC(upload(ctx, sizes_d, slot_size.data(), (size_t)N * 8, s));
        SelectParams sp;
        sp.fit = fitv.p;
        sp.sizes = sizes_d.as<int64_t>();
        sp.n = N;
        sp.k = cfg->tournament;
        sp.boolean = boolean ? 1 : 0;
        sp.seed = cfg->seed;
        sp.generation = g;
        sp.mother = sel.as<int64_t>();
        sp.father = sp.mother + N;
        sp.point = sp.father + N;
        sp.donor_node = sp.point + N;
        HIPC(ctx, launch_select(sp, s));
        HIPC(ctx, hipMemcpyAsync(pick.data(), sel.p, (size_t)N * 4 * 8, hipMemcpyDeviceToHost, s));
        HIPC(ctx, hipStreamSynchronize(s));
        // score every child by co-evaluation with its mother
        std::vector<IncJob> jobs(N);
        for (int64_t i = 0; i < N; ++i) {
            const int64_t mt = slot_tree[mother[i]], ft = slot_tree[father[i]];
            if (mt < 0 || ft < 0) return set_err(ctx, GP_EINVAL, "internal error: a tournament winner was not built");
            const uint8_t* fb = cur->host_ops.data() + cur->host_offsets[ft];
            static const std::vector<SubtreeEnd> none;
            const auto& fbig = cur->big_ends.size() == (size_t)cur->n_trees ? cur->big_ends[ft] : none;
            const auto& mbig = cur->big_ends.size() == (size_t)cur->n_trees ? cur->big_ends[mt] : none;
            dend[i] = subtree_end_indexed(fb, cur->tree_nodes[ft], dnode[i], fbig);
            removed[i] = subtree_end_indexed(cur->host_ops.data() + cur->host_offsets[mt], cur->tree_nodes[mt], point[i],
                                             mbig) - point[i];
            jobs[i] = IncJob{cur, mt, point[i], fb + dnode[i], dend[i] - dnode[i]};
        }
        IncOut io;
        RC(enqueue_coeval(ctx, jobs, cases, cs, false, s, &io, nullptr, nullptr));
        HIPC(ctx, hipMemcpyAsync(fitn.p, io.fit.p, (size_t)N * 8, hipMemcpyDeviceToDevice, s));
        HIPC(ctx, hipMemcpyAsync(stop.data(), io.stop.p, (size_t)N * 4, hipMemcpyDeviceToHost, s));
        HIPC(ctx, hipMemcpyAsync(interp.data(), io.interp.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
        HIPC(ctx, hipMemcpyAsync(fit_h.data(), io.fit.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
        // fitness first: only children the next generation's tournaments draw are built
        const bool last = gi == G - 1;
        if (!last) {
            HIPC(ctx, launch_fill_i32(drawn_d.as<int32_t>(), N, 0, s));
            MarkParams mp;
            mp.fit = fitn.p;
            mp.n = N;
            mp.k = cfg->tournament;
            mp.boolean = sp.boolean;
            mp.seed = cfg->seed;
            mp.generation = g + 1;
            mp.drawn = drawn_d.as<int32_t>();
            HIPC(ctx, launch_mark(mp, s));
            HIPC(ctx, hipMemcpyAsync(drawn.data(), drawn_d.p, (size_t)N * 4, hipMemcpyDeviceToHost, s));
        }
        HIPC(ctx, hipStreamSynchronize(s));
        const double t1 = now_ms();
        if (last) std::fill(drawn.begin(), drawn.end(), 1);
        // build them on the device: mother's prefix, father's subtree, mother's suffix
        if (!cur->tree_ops.p) {
            const size_t nb = (size_t)cur->host_offsets[cur->n_trees];
            RC(dev_alloc(ctx, cur->tree_ops, nb + 32));
            HIPC(ctx, hipMemcpyAsync(cur->tree_ops.p, cur->host_ops.data(), nb, hipMemcpyHostToDevice, s));
            cur->tree_off = cur->host_offsets;
        }
        std::vector<int64_t> noffs{0}, child_nodes(N), new_slot(N, -1);
        for (int64_t i = 0; i < N; ++i) {
            child_nodes[i] = cur->tree_nodes[slot_tree[mother[i]]] - removed[i] + (dend[i] - dnode[i]);
            if (drawn[i] > 0) {
                new_slot[i] = (int64_t)noffs.size() - 1;
                noffs.push_back(noffs.back() + child_nodes[i]);
            }
        }
        const int64_t nb = (int64_t)noffs.size() - 1, total = noffs.back();
        auto np = std::make_shared<Pop>();
        {
            DevBuf out;
            RC(dev_alloc(ctx, out, (size_t)total + 32));
            std::vector<SpliceItem> items;
            const uint8_t* base = cur->tree_ops.as<uint8_t>();
            for (int64_t i = 0; i < N; ++i) {
                if (new_slot[i] < 0) continue;
                const int64_t mt = slot_tree[mother[i]], ft = slot_tree[father[i]], o = noffs[new_slot[i]];
                const uint8_t* m = base + cur->tree_off[mt];
                const int64_t nd = dend[i] - dnode[i];
                add_splice_item(items, m, o, point[i]);
                add_splice_item(items, base + cur->tree_off[ft] + dnode[i], o + point[i], nd);
                add_splice_item(items, m + point[i] + removed[i], o + point[i] + nd,
                                cur->tree_nodes[mt] - point[i] - removed[i]);
            }
            if ((int64_t)items.size() > (int64_t(1) << 24))
                return set_err(ctx, GP_EINVAL, "too many bytes to build in one generation");
            DevBuf items_d;
            RC(upload(ctx, items_d, items.data(), std::max<size_t>(1, items.size()) * sizeof(SpliceItem), s));
            HIPC(ctx, launch_splice(items_d.as<SpliceItem>(), (int64_t)items.size(), out.as<uint8_t>(), s));
            // the host copy of the same bytes, and the children's programs:
            // built from the parents' chunks when both parents' are kept,
            // else compiled whole
            bool compose = cur->kept_chunks.size() == (size_t)cur->n_trees &&
                           cur->big_ends.size() == (size_t)cur->n_trees;
            std::vector<int64_t> built(nb);
            for (int64_t i = 0; i < N; ++i)
                if (new_slot[i] >= 0) {
                    built[new_slot[i]] = i;
                    const int64_t mt = slot_tree[mother[i]], ft = slot_tree[father[i]];
                    compose = compose && !cur->kept_chunks[mt].empty() && !cur->kept_chunks[ft].empty();
                }
            np->host_ops.resize((size_t)total);
            std::vector<TreeProg> progs(nb);
            std::vector<std::string> errs(nb);
            std::vector<char> bad(nb, 0);
            CompileOptions opt;
            opt.vtype = vtype;
            opt.n_inputs = cur->n_inputs;
            opt.chunk_nodes = cur->chunk_nodes;
            opt.stack_slots = compile_stack_slots();
            opt.index_min_size = kBigSubtree;
            std::atomic<int64_t> next{0};
            auto work = [&]() {
                for (int64_t k; (k = next++) < nb;) {
                    const int64_t i = built[k];
                    const int64_t mt = slot_tree[mother[i]], ft = slot_tree[father[i]], nd = dend[i] - dnode[i];
                    const uint8_t* m = cur->host_ops.data() + cur->host_offsets[mt];
                    const uint8_t* f = cur->host_ops.data() + cur->host_offsets[ft];
                    uint8_t* o = np->host_ops.data() + noffs[k];
                    std::memcpy(o, m, (size_t)point[i]);
                    std::memcpy(o + point[i], f + dnode[i], (size_t)nd);
                    std::memcpy(o + point[i] + nd, m + point[i] + removed[i],
                                (size_t)(cur->tree_nodes[mt] - point[i] - removed[i]));
                    if (!compose) continue;
                    const auto& mc = cur->kept_chunks[mt];
                    const auto& fc = cur->kept_chunks[ft];
                    SrcTree ms{m, cur->tree_nodes[mt], mc.data(), (int64_t)mc.size(), &cur->big_ends[mt],
                               cur->kept_max_stack[mt]};
                    SrcTree fs{f, cur->tree_nodes[ft], fc.data(), (int64_t)fc.size(), &cur->big_ends[ft],
                               cur->kept_max_stack[ft]};
                    if (!compose_child(ms, point[i], point[i] + removed[i], fs, dnode[i], dend[i], o,
                                       noffs[k + 1] - noffs[k], opt, &progs[k], &errs[k]))
                        bad[k] = 1;
                }
            };
            const int nth = (int)std::min<int64_t>(std::min<int64_t>(16, std::max(1u, std::thread::hardware_concurrency())),
                                                   nb);
            std::vector<std::thread> th;
            for (int t = 1; t < nth; ++t) th.emplace_back(work);
            work();
            for (auto& t : th) t.join();
            for (int64_t k = 0; k < nb; ++k) {
                if (bad[k]) return set_err(ctx, GP_EINVAL, "child " + std::to_string(built[k]) + ": " + errs[k]);
                for (const Chunk& ch : progs[k].chunks)
                    if (ch.dev_src >= 0 && (ch.code_len < 1 || ch.dev_src + ch.code_len > cur->n_code))
                        return set_err(ctx, GP_EINVAL, "internal error: reused code out of range");
            }
            if (compose) {
                std::vector<int64_t> tn(nb);
                np->big_ends.resize(nb);
                for (int64_t k = 0; k < nb; ++k) {
                    tn[k] = noffs[k + 1] - noffs[k];
                    np->big_ends[k].swap(progs[k].big_ends);
                }
                np->big_built.assign(nb, 1);
                np->layout = GP_PREFIX;
                RC(assemble_population(ctx, vtype, cur->n_inputs, progs, tn, cur->chunk_nodes, np.get(), s,
                                       cur->code.as<uint32_t>()));
            } else {
                RC(build_population(ctx, vtype, GP_PREFIX, cur->n_inputs, nb, np->host_ops.data(), noffs.data(),
                                    nullptr, nullptr, 0, np.get(), s, true));
            }
            HIPC(ctx, hipStreamSynchronize(s));
            np->tree_ops.swap(out);                 // the built bytes stay on the device for the next generation
        }
        np->auto_chunk = true;
        np->host_offsets = noffs;
        np->tree_off = noffs;
        const double t2 = now_ms();
        const Launch L = choose_launch(ctx, vtype, cs, np.get());
        if (L.variant < 0) return set_err(ctx, GP_EINVAL, "no interpreter variant fits the children");
        int64_t n_eval = np->n_chunks;
        // the chunk vectors of the generation before last hold nothing needed any more: reused when large enough
        const size_t vec_bytes = (size_t)np->n_chunks * cs->stride * (boolean ? 8 : 4);
        if (spare_vecs.p && spare_vecs.bytes >= vec_bytes) {
            np->vecs.swap(spare_vecs);
            np->stride = cs->stride;
            RC(dev_alloc(ctx, np->fit, (size_t)np->n_trees * 8));
        }
        if (!np->promo_src.empty()) {
            // reused chunks take their parents' values; only the chunks compiled anew run
            RC(enqueue_promoted(ctx, np.get(), cur, cases, cs, L, s, &n_eval));
        } else {
            RC(enqueue_full(ctx, np.get(), cases, cs, L, false, false, s, nullptr));
            HIPC(ctx, hipStreamSynchronize(s));
        }
        const double t3 = now_ms();
        // statistics and records
        const double* ff = (const double*)fit_h.data();
        const int64_t* fi = (const int64_t*)fit_h.data();
        if (stats) {
            gp_gen_stats& st = stats[gi];
            st.best_f64 = std::numeric_limits<double>::quiet_NaN();
            st.best_i64 = std::numeric_limits<int64_t>::min();
            st.children = N;
            st.built = nb;
            st.child_nodes = 0;
            st.built_nodes = total;
            st.interpreted_nodes = 0;
            for (int64_t i = 0; i < N; ++i) {
                if (boolean) st.best_i64 = std::max(st.best_i64, fi[i]);
                else if (!std::isnan(ff[i]) && (std::isnan(st.best_f64) || ff[i] < st.best_f64)) st.best_f64 = ff[i];
                st.child_nodes += child_nodes[i];
                st.interpreted_nodes += interp[i];
            }
            st.ms = now_ms() - t0;
            st.ms_score = t1 - t0;
            st.ms_build = t2 - t1;
            st.ms_eval = t3 - t2;
            st.chunks = np->n_chunks;
            st.chunks_evaluated = n_eval;
        }
        if (children)
            for (int64_t i = 0; i < N; ++i) {
                gp_gen_child& r = children[gi * N + i];
                r.mother = mother[i];
                r.father = father[i];
                r.point = point[i];
                r.donor_node = dnode[i];
                r.nodes = child_nodes[i];
                r.fitness_f64 = boolean ? 0.0 : ff[i];
                r.fitness_i64 = boolean ? fi[i] : 0;
                r.stop_level = stop[i];
                r.drawn = last ? 0 : drawn[i];
            }
        // the children become the slots of the next generation
        for (int64_t i = 0; i < N; ++i) {
            slot_tree[i] = new_slot[i];
            slot_size[i] = new_slot[i] >= 0 ? child_nodes[i] : 0;
        }
        fitv.swap(fitn);
        spare_vecs.release();
        if (holder) spare_vecs.swap(holder->vecs);   // the generation before this one is dropped now
        holder = np;
        cur = np.get();
    }
    gp_handle h = ctx->next_handle++;
    ctx->pops[h] = holder;
    *out_pop = h;
    return GP_OK;
}

int gp_evaluate_incremental(gp_ctx* ctx, gp_handle pop, gp_handle cases, int64_t parent, int64_t point,
                            const uint8_t* donor_ops, int64_t donor_len, uint32_t flags, void* root_out,
                            void* fitness_out, gp_inc_result* res)
{
    int64_t offs[2] = {0, donor_len};
    return gp_evaluate_incremental_batch(ctx, pop, cases, 1, &parent, &point, donor_ops, offs, flags, root_out,
                                         fitness_out, res, nullptr);
}

const char* gp_variant_name(int variant)
{
    if (variant < 0 || variant >= variant_count()) return nullptr;
    return variant_table()[variant].name;
}

int gp_variant_count(void) { return variant_count(); }

int gp_set_variant(gp_ctx* ctx, int variant)
{
    if (!ctx) return GP_EINVAL;
    if (variant >= variant_count()) return set_err(ctx, GP_EINVAL, "unknown variant");
    ctx->forced_variant = variant < 0 ? -1 : variant;
    return GP_OK;
}

// One flat JSON object per line: string values ("...", no escapes) and
// integers.  False on anything else.
static bool parse_flat_json(const std::string& line, std::map<std::string, std::string>* kv)
{
    size_t i = 0;
    auto ws = [&] { while (i < line.size() && std::isspace((unsigned char)line[i])) ++i; };
    auto str = [&](std::string* out) {
        if (i >= line.size() || line[i] != '"') return false;
        const size_t e = line.find('"', i + 1);
        if (e == std::string::npos) return false;
        *out = line.substr(i + 1, e - i - 1);
        i = e + 1;
        return out->find('\\') == std::string::npos;
    };
    ws();
    if (i >= line.size() || line[i++] != '{') return false;
    for (;;) {
        ws();
        std::string k, v;
        if (!str(&k)) return false;
        ws();
        if (i >= line.size() || line[i++] != ':') return false;
        ws();
        if (i < line.size() && line[i] == '"') {
            if (!str(&v)) return false;
        } else {
            const size_t b = i;
            if (i < line.size() && line[i] == '-') ++i;
            while (i < line.size() && std::isdigit((unsigned char)line[i])) ++i;
            if (i == b || (i == b + 1 && line[b] == '-')) return false;
            v = line.substr(b, i - b);
        }
        (*kv)[k] = v;
        ws();
        if (i < line.size() && line[i] == ',') {
            ++i;
            continue;
        }
        if (i < line.size() && line[i] == '}') {
            ++i;
            ws();
            return i == line.size();
        }
        return false;
    }
}

int gp_tuning_save(gp_ctx* ctxp, const char* path)
{
    Ctx* ctx = ctxp;
    if (!ctx) return GP_EINVAL;
    if (!path) return set_err(ctx, GP_EINVAL, "no path");
    std::string out;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (const auto& kv : ctx->tuned) {
            const TuneKey& k = kv.first;
            const auto ch = ctx->tuned_chunk.find(k);
            out += "{\"device\": \"" + ctx->device_name + "\", \"vtype\": " + std::to_string(k.vtype) +
                   ", \"t_bucket\": " + std::to_string(k.tbucket) + ", \"s_bucket\": " + std::to_string(k.sbucket) +
                   ", \"variant\": \"" + variant_table()[kv.second.variant].name + "\", \"waves_per_cu\": " +
                   std::to_string(kv.second.waves_per_cu) + ", \"chunk_nodes\": " +
                   std::to_string(ch != ctx->tuned_chunk.end() ? ch->second : 0) + "}\n";
        }
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return set_err(ctx, GP_EINVAL, std::string("cannot write ") + path);
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok) return set_err(ctx, GP_EINVAL, std::string("cannot write ") + path);
    return GP_OK;
}

int gp_tuning_load(gp_ctx* ctxp, const char* path)
{
    Ctx* ctx = ctxp;
    if (!ctx) return GP_EINVAL;
    if (!path) return set_err(ctx, GP_EINVAL, "no path");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_err(ctx, GP_ENOTFOUND, std::string("cannot read ") + path);
    std::vector<std::pair<TuneKey, std::pair<Launch, int64_t>>> got;
    std::string line;
    int c = 0, lineno = 0;
    bool bad = false;
    std::string why;
    while (!bad) {
        line.clear();
        while ((c = std::fgetc(f)) != EOF && c != '\n') line.push_back((char)c);
        if (line.empty() && c == EOF) break;
        ++lineno;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::map<std::string, std::string> kv;
        if (!parse_flat_json(line, &kv)) {
            bad = true;
            why = "malformed line " + std::to_string(lineno);
            break;
        }
        for (const char* k : {"device", "vtype", "t_bucket", "s_bucket", "variant", "waves_per_cu", "chunk_nodes"})
            if (!kv.count(k)) {
                bad = true;
                why = "line " + std::to_string(lineno) + " lacks \"" + k + "\"";
            }
        if (bad) break;
        if (kv["device"] != ctx->device_name) continue;     // tuned on another device
        int v = -1;
        for (int i = 0; i < variant_count(); ++i)
            if (kv["variant"] == variant_table()[i].name) v = i;
        if (v < 0) continue;                                 // a variant this library does not have
        const TuneKey key{std::atoi(kv["vtype"].c_str()), std::atoi(kv["t_bucket"].c_str()),
                          std::atoi(kv["s_bucket"].c_str())};
        const int w = std::atoi(kv["waves_per_cu"].c_str());
        const int64_t cn = std::atoll(kv["chunk_nodes"].c_str());
        if ((key.vtype != GP_F32 && key.vtype != GP_BOOL) || variant_table()[v].vtype != key.vtype || w < 0 || cn < 0) {
            bad = true;
            why = "line " + std::to_string(lineno) + " has values out of range";
            break;
        }
        got.push_back({key, {Launch{v, w}, cn}});
    }
    std::fclose(f);
    if (bad) return set_err(ctx, GP_EINVAL, std::string(path) + ": " + why);
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto& e : got) {
        ctx->tuned[e.first] = e.second.first;
        ctx->tuned_chunk[e.first] = e.second.second;
        ctx->tuned_loaded[e.first] = true;
    }
    return GP_OK;
}

int gp_set_launch_width(gp_ctx* ctx, int waves_per_cu)
{
    if (!ctx) return GP_EINVAL;
    if (waves_per_cu < -1) return set_err(ctx, GP_EINVAL, "waves_per_cu must be -1, 0 or positive");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->forced_waves = waves_per_cu;
    return GP_OK;
}

// Time every interpreter variant, and for automatically chunked populations
// every candidate chunk size, on this population and case set; keep the
// fastest (chunk size: recompiled in place; variant: remembered per value
// type, case-count bucket and tree-size bucket).
// The population p recompiled at chunk size cn into a new Pop (from the kept
// device copy of the trees, else from the host copy).
static int rechunk(Ctx* ctx, Pop* p, int64_t cn, std::shared_ptr<Pop>* out)
{
    auto q = std::make_shared<Pop>();
    const bool rec = !p->host_rec_points.empty() || !p->host_rec_offsets.empty();
    if (p->device_compiled) {
        const bool kept = p->tree_ops.p && p->tree_off == p->host_offsets;
        RC(build_population_device(ctx, p->vtype, p->n_inputs, p->n_trees, kept ? nullptr : p->host_ops.data(),
                                   kept ? p->tree_ops.as<uint8_t>() : nullptr, p->host_offsets.data(),
                                   rec ? p->host_rec_points.data() : nullptr,
                                   rec ? p->host_rec_offsets.data() : nullptr, cn, q.get(), nullptr));
    } else {
        RC(build_population(ctx, p->vtype, p->layout, p->n_inputs, p->n_trees, p->host_ops.data(),
                            p->host_offsets.data(), rec ? p->host_rec_points.data() : nullptr,
                            rec ? p->host_rec_offsets.data() : nullptr, cn, q.get(), ctx->stream, true));
    }
    *out = std::move(q);
    return GP_OK;
}

// The re-chunked copy q replaces population p under the same handle; it takes
// over the host and device copies of the trees.
static Pop* replace_population(Ctx* ctx, gp_handle pop, Pop* p, const std::shared_ptr<Pop>& q)
{
    q->auto_chunk = true;
    q->host_ops.swap(p->host_ops);
    q->host_offsets.swap(p->host_offsets);
    q->host_rec_points.swap(p->host_rec_points);
    q->host_rec_offsets.swap(p->host_rec_offsets);
    q->tree_ops.swap(p->tree_ops);
    q->tree_off.swap(p->tree_off);
    ctx->pops[pop] = q;
    return q.get();
}

int gp_autotune(gp_ctx* ctx, gp_handle pop, gp_handle cases, int* best_variant, double* best_ms)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    Pop* p;
    CaseSet* cs;
    RC(lookup(ctx, pop, cases, &p, &cs));
    {
        // a choice read by gp_tuning_load: applied without timing the others
        const TuneKey key = tune_key(p->vtype, cs, p);
        auto it = ctx->tuned.find(key);
        if (ctx->tuned_loaded.count(key) && it != ctx->tuned.end() &&
            default_variant(p->vtype, cs, p, it->second.variant) == it->second.variant) {
            const Launch L = it->second;
            const int64_t cn = ctx->tuned_chunk.count(key) ? ctx->tuned_chunk[key] : p->chunk_nodes;
            if (p->auto_chunk && !p->host_ops.empty() && cn > 0 && cn != p->chunk_nodes) {
                std::shared_ptr<Pop> q;
                RC(rechunk(ctx, p, cn, &q));
                p = replace_population(ctx, pop, p, q);
            }
            RC(enqueue_full(ctx, p, cases, cs, L, false, true, ctx->stream, nullptr));   // warm-up + capture
            HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
            RC(enqueue_full(ctx, p, cases, cs, L, false, true, ctx->stream, nullptr));
            HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
            HIPC(ctx, hipStreamSynchronize(ctx->stream));
            float ms = 0.f;
            HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            if (best_variant) *best_variant = L.variant;
            if (best_ms) *best_ms = ms;
            return GP_OK;
        }
    }
    std::vector<int64_t> chunk_sizes{p->chunk_nodes};
    if (p->auto_chunk && !p->host_ops.empty()) {
        const int64_t mean = p->total_nodes / std::max<int64_t>(1, p->n_trees);
        // large populations of large trees keep large chunks; mid-size ones (10^8..10^9 nodes) are bound by
        // chains of chunk hand-offs and do best at 512..1024-node chunks; small ones, down to 128
        std::vector<int64_t> cand = p->total_nodes > 1000000000  ? std::vector<int64_t>{1024, 2048, 4096, 8192}
                                    : p->total_nodes > 200000000 ? std::vector<int64_t>{512, 768, 1024, 2048}
                                                                 : std::vector<int64_t>{128, 192, 256, 512, 1024, 2048, 4096};
        chunk_sizes.clear();
        for (int64_t c : cand)
            if (c <= std::max<int64_t>(256, 4 * mean)) chunk_sizes.push_back(c);
    }
    auto time_variant = [&](Pop* q, Launch L, float* out) -> int {
        RC(enqueue_full(ctx, q, cases, cs, L, false, true, ctx->stream, nullptr));   // warm-up + capture
        float tmin = 1e30f;
        for (int r = 0; r < 3; ++r) {
            HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
            RC(enqueue_full(ctx, q, cases, cs, L, false, true, ctx->stream, nullptr));
            HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
            HIPC(ctx, hipStreamSynchronize(ctx->stream));
            float ms = 0.f;
            HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            tmin = std::min(tmin, ms);
        }
        *out = tmin;
        return GP_OK;
    };
    int best = -1, best_w = 0;
    float best_t = 1e30f;
    std::shared_ptr<Pop> best_pop;
    for (int64_t cn : chunk_sizes) {
        std::shared_ptr<Pop> q;
        Pop* qp = p;
        if (cn != p->chunk_nodes) {
            RC(rechunk(ctx, p, cn, &q));
            qp = q.get();
        }
        bool improved = false;
        auto consider = [&](Launch L, float t) {
            if (t < best_t) {
                best_t = t;
                best = L.variant;
                best_w = L.waves_per_cu;
                improved = true;
            }
        };
        // every variant with all the waves that fit
        std::vector<std::pair<float, int>> full;
        for (int v = 0; v < variant_count(); ++v) {
            const Variant& vt = variant_table()[v];
            if (!variant_fits(vt, qp->vtype, qp->max_stack, qp->n_inputs, cs->n_elems, cs->stride,
                              qp->vtype == GP_BOOL ? 8 : 4))
                continue;
            float t = 0.f;
            RC(time_variant(qp, Launch{v, 0}, &t));
            full.emplace_back(t, v);
            consider(Launch{v, 0}, t);
        }
        // the two fastest of them with fewer resident waves per CU, from the
        // most that fit downwards, until two caps in a row are no faster than
        // that variant's best so far
        std::sort(full.begin(), full.end());
        for (size_t i = 0; i < std::min<size_t>(2, full.size()); ++i) {
            const int v = full[i].second;
            float vbest = full[i].first;
            int slower = 0;
            for (int w : {24, 16, 12, 8, 6, 4, 3, 2}) {
                if (w >= variant_table()[v].max_blocks_per_cu) continue;
                float t = 0.f;
                RC(time_variant(qp, Launch{v, w}, &t));
                consider(Launch{v, w}, t);
                if (t < vbest) {
                    vbest = t;
                    slower = 0;
                } else if (++slower == 2) {
                    break;
                }
            }
        }
        // keep only the compiled copy of the best chunk size so far
        if (improved) best_pop = q;
    }
    if (best < 0) return set_err(ctx, GP_EINVAL, "no interpreter variant fits this population");
    if (best_pop) p = replace_population(ctx, pop, p, best_pop);
    // keep only the chosen launch's plans
    for (auto it = p->plans.begin(); it != p->plans.end();) {
        if (std::get<0>(it->first) != best || std::get<1>(it->first) != best_w) it = p->plans.erase(it);
        else ++it;
    }
    RC(enqueue_full(ctx, p, cases, cs, Launch{best, best_w}, false, true, ctx->stream, nullptr));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const TuneKey key = tune_key(p->vtype, cs, p);
    ctx->tuned[key] = Launch{best, best_w};
    ctx->tuned_chunk[key] = p->chunk_nodes;
    ctx->tuned_loaded.erase(key);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return GP_OK;
}

// Arguments shared by both index entry points.
static int ix_check_args(Ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                         int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent)
{
    if (n_inputs < 1 || n_inputs > kMaxInputs) return set_err(ctx, GP_EINVAL, "n_inputs must be 1..64");
    if (n_trees < 1 || n_nodes < 1) return set_err(ctx, GP_EINVAL, "empty population");
    if (n_nodes > (int64_t)INT32_MAX - 1) return set_err(ctx, GP_EINVAL, "at most 2^31 - 2 nodes per call");
    if (n_trees > n_nodes) return set_err(ctx, GP_EINVAL, "more trees than nodes");
    if (!ops || !offsets || !valid || !end || !parent) return set_err(ctx, GP_EINVAL, "missing device array");
    if (((uintptr_t)ops & 15) != 0) return set_err(ctx, GP_EINVAL, "ops must be 16-byte aligned");
    return GP_OK;
}

// Min-tree levels of n positions: level 0 is E itself (n + 1 positions), each
// next one kIxFan times shorter, up to one group; every level after 0 starts
// on a whole group of seg and is padded to one.  Fills q.lvl, q.top and
// len[0 .. top]; returns the words of seg used (without the final padding).
static int64_t ix_levels(int64_t n, IxParams& q, int64_t (&len)[kIxMaxLevels])
{
    for (int l = 0; l < kIxMaxLevels; ++l) {
        len[l] = 0;
        q.lvl[2 * l] = q.lvl[2 * l + 1] = 0;
    }
    len[0] = n + 1;
    q.lvl[1] = len[0];
    int top = 0;
    int64_t seg_total = 0;
    while (len[top] > kIxFan) {
        ++top;
        len[top] = (len[top - 1] + kIxFan - 1) / kIxFan;
        q.lvl[2 * top] = seg_total;
        q.lvl[2 * top + 1] = len[top];
        seg_total += (len[top] + kIxFan - 1) / kIxFan * kIxFan;
    }
    q.top = top;
    return seg_total;
}

// The index kernels on ctx's stream with the given scratch (el, boff, bsum,
// seg sized for q.n; flag 2 words; bempty n_blocks + 1 bytes), then the host
// waits for the offsets flag (and, per Strahler level, for the level's count).
// Flags are cleared by a fill kernel.  Allocates nothing.
static int ix_run(Ctx* ctx, IxParams& q, int32_t* bsum, int32_t* flag, int64_t nb, const int64_t* len,
                  double* device_ms, hipStream_t st)
{
    q.bad_offsets = flag;
    // timed with the context's events (entry points that hold the context lock only)
    if (device_ms) HIPC(ctx, hipEventRecord(ctx->ev0, st));
    HIPC(ctx, launch_fill_i32(flag, 2, 0, st));
    if (q.sn) HIPC(ctx, launch_fill_u8(q.bempty, nb + 1, 1, st));      // block nb holds only E(n)
    HIPC(ctx, launch_index(q, bsum, nb, len, st));
    if (q.sn) {
        // one pass per level, while some function has two children at the
        // current level (the pass leaves their number in boff[nb])
        HIPC(ctx, launch_strahler_init(q, st));
        for (int level = 2; level < 64; ++level) {          // the initial numbers settle level 1
            HIPC(ctx, launch_strahler_level(q, level, bsum, nb, st));
            int32_t more = 0;
            HIPC(ctx, hipMemcpyAsync(&more, q.boff + nb, 4, hipMemcpyDeviceToHost, st));
            HIPC(ctx, hipStreamSynchronize(st));
            if (!more) break;
        }
    }
    int32_t bad = 0;
    if (device_ms) HIPC(ctx, hipEventRecord(ctx->ev1, st));
    HIPC(ctx, hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    if (device_ms) {
        float ms = 0.f;
        HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        *device_ms = ms;
    }
    if (bad) return set_err(ctx, GP_EINVAL, "offsets must run from 0 to n_nodes without decreasing");
    return GP_OK;
}

static IxParams ix_params(int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets, int64_t n_nodes,
                          int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler)
{
    IxParams q{};
    q.ops = ops;
    q.offsets = offsets;
    q.n_trees = n_trees;
    q.n = n_nodes;
    q.n_inputs = n_inputs;
    q.valid = valid;
    q.end = end;
    q.parent = parent;
    q.sn = strahler;
    return q;
}

}  // extern "C"

int gpe::index_trees(Ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                     int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler,
                     double* device_ms, hipStream_t st, DevArena* arena)
{
    RC(ix_check_args(ctx, n_inputs, n_trees, ops, offsets, n_nodes, valid, end, parent));
    IxParams q = ix_params(n_inputs, n_trees, ops, offsets, n_nodes, valid, end, parent, strahler);
    int64_t len[kIxMaxLevels];
    const int64_t seg_total = ix_levels(n_nodes, q, len);
    const int64_t nb = (n_nodes + kIxBlock - 1) / kIxBlock;
    DevBuf el, boff, bsum, seg, flag, bempty;
    RC(scratch_alloc(ctx, arena, el, (size_t)(nb * kIxBlock + kIxFan) * 4));
    RC(scratch_alloc(ctx, arena, boff, (size_t)(nb + 1) * 4));
    RC(scratch_alloc(ctx, arena, bsum, (size_t)nb * 4));
    RC(scratch_alloc(ctx, arena, seg, (size_t)(seg_total + kIxFan) * 4));
    RC(scratch_alloc(ctx, arena, flag, 8));
    if (strahler) RC(scratch_alloc(ctx, arena, bempty, (size_t)nb + 1));
    q.el = el.as<int16_t>();
    q.boff = boff.as<int32_t>();
    q.seg = seg.as<int32_t>();
    q.bempty = strahler ? bempty.as<uint8_t>() : nullptr;
    return ix_run(ctx, q, bsum.as<int32_t>(), flag.as<int32_t>(), nb, len, device_ms, st);
}

extern "C" {

int gp_index_trees(gp_ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                   int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler,
                   double* device_ms)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    return index_trees(ctx, n_inputs, n_trees, ops, offsets, n_nodes, valid, end, parent, strahler, device_ms,
                       ctx->stream);
}

static_assert(GP_INDEX_NOALLOC_MAX_NODES == kIxStaticMaxNodes, "header and scratch array disagree");

int gp_index_trees_noalloc(gp_ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                           int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler,
                           double* device_ms)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    RC(ix_check_args(ctx, n_inputs, n_trees, ops, offsets, n_nodes, valid, end, parent));
    if (n_nodes > kIxStaticMaxNodes)
        return set_err(ctx, GP_EINVAL, "gp_index_trees_noalloc takes at most 4194304 nodes per call "
                                       "(gp_index_trees takes more)");
    if (!ctx->ix_scratch) return set_err(ctx, GP_EDEVICE, "the index scratch array has no device address");
    IxParams q = ix_params(n_inputs, n_trees, ops, offsets, n_nodes, valid, end, parent, strahler);
    int64_t len[kIxMaxLevels];
    (void)ix_levels(n_nodes, q, len);
    const int64_t nb = (n_nodes + kIxBlock - 1) / kIxBlock;
    int32_t* base = ctx->ix_scratch;
    q.el = (int16_t*)(base + kIxStaticEl);
    q.boff = base + kIxStaticBoff;
    q.seg = base + kIxStaticSeg;
    q.bempty = strahler ? (uint8_t*)(base + kIxStaticBempty) : nullptr;
    return ix_run(ctx, q, base + kIxStaticBsum, base + kIxStaticFlag, nb, len, device_ms, ctx->stream);
}

int gp_valu_calibration(gp_ctx* ctx, int cls, int64_t n_waves, int64_t iters, double* device_ms)
{
    if (!ctx) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    HIPC(ctx, hipSetDevice(ctx->device));
    if (cls < 0 || cls > 9) return set_err(ctx, GP_EINVAL, "instruction class must be 0..9");
    if (n_waves < 1 || n_waves > (int64_t(1) << 24) || iters < 0) return set_err(ctx, GP_EINVAL, "bad size");
    DevBuf out;
    RC(dev_alloc(ctx, out, (size_t)n_waves * 64 * 4));
    HIPC(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    HIPC(ctx, launch_valu_cal(cls, n_waves, iters, out.as<float>(), ctx->stream));
    HIPC(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (device_ms) *device_ms = ms;
    return GP_OK;
}

int gp_validate_tree(int vtype, int n_inputs, const uint8_t* ops, int64_t n)
{
    if ((vtype != GP_F32 && vtype != GP_BOOL) || n_inputs < 1 || n_inputs > kMaxInputs || !ops) return GP_EINVAL;
    return validate_prefix(ops, n, n_inputs, nullptr) ? GP_OK : GP_EINVAL;
}

int64_t gp_inspect_path(const uint8_t* ops, int64_t n, int64_t c, int64_t index_min_size, int64_t* levels_out,
                        int64_t level_cap, int64_t* removed_end)
{
    if (!ops || !levels_out || !removed_end || c < 0 || c >= n) return GP_EINVAL;
    if (!validate_prefix(ops, n, kMaxInputs, nullptr)) return GP_EINVAL;
    std::vector<SubtreeEnd> big;
    if (index_min_size > 0) big_subtree_ends(ops, n, index_min_size, &big);
    std::vector<PathLevel> lv;
    int64_t e = -1;
    path_to_root(ops, n, c, big, &lv, &e);
    if ((int64_t)lv.size() > level_cap) return GP_ENOMEM;
    for (size_t k = 0; k < lv.size(); ++k) {
        levels_out[4 * k + 0] = lv[k].node;
        levels_out[4 * k + 1] = lv[k].sib_begin;
        levels_out[4 * k + 2] = lv[k].sib_end;
        levels_out[4 * k + 3] = lv[k].f | (lv[k].right ? 4 : 0);
    }
    *removed_end = e;
    return (int64_t)lv.size();
}

int64_t gp_inspect_child_program(int vtype, int n_inputs, const uint8_t* mother, int64_t n_mother, int64_t point,
                                 const int64_t* mother_records, int64_t n_mother_records,
                                 const uint8_t* father, int64_t n_father, int64_t donor_node, int64_t chunk_nodes,
                                 int stack_slots, int64_t index_min_size, uint32_t* code_out, int64_t code_cap,
                                 int64_t* chunk_out, int64_t chunk_cap, int32_t* inputs_out, int64_t inputs_cap,
                                 int64_t* big_out, int64_t big_cap, int64_t* n_code, int32_t* max_stack,
                                 int64_t* n_big, int64_t* n_reused)
{
    if ((vtype != GP_F32 && vtype != GP_BOOL) || n_inputs < 1 || n_inputs > kMaxInputs || !mother || !father ||
        index_min_size < 1)
        return GP_EINVAL;
    if (!validate_prefix(mother, n_mother, n_inputs, nullptr) || !validate_prefix(father, n_father, n_inputs, nullptr))
        return GP_EINVAL;
    if (point < 0 || point >= n_mother || donor_node < 0 || donor_node >= n_father) return GP_EINVAL;
    CompileOptions opt;
    opt.vtype = vtype;
    opt.n_inputs = n_inputs;
    opt.chunk_nodes = chunk_nodes > 0 ? chunk_nodes : 4096;
    opt.stack_slots = stack_slots > 0 ? stack_slots : compile_stack_slots();
    opt.index_min_size = index_min_size;
    TreeProg pm, pf, pc;
    std::string why;
    if (n_mother_records < 0 || (n_mother_records > 0 && !mother_records)) return GP_EINVAL;
    if (!compile_tree(mother, n_mother, opt, mother_records, n_mother_records, &pm, &why) ||
        !compile_tree(father, n_father, opt, nullptr, 0, &pf, &why))
        return GP_EINVAL;
    // the parents' programs as one uploaded program: the mother's code, then the father's
    std::vector<uint32_t> src(pm.code);
    src.insert(src.end(), pf.code.begin(), pf.code.end());
    for (Chunk& ch : pf.chunks) ch.code_off += (int64_t)pm.code.size();
    const int64_t c_end = subtree_end_indexed(mother, n_mother, point, pm.big_ends);
    const int64_t d_end = subtree_end_indexed(father, n_father, donor_node, pf.big_ends);
    std::vector<uint8_t> child(mother, mother + point);
    child.insert(child.end(), father + donor_node, father + d_end);
    child.insert(child.end(), mother + c_end, mother + n_mother);
    SrcTree m{mother, n_mother, pm.chunks.data(), (int64_t)pm.chunks.size(), &pm.big_ends, pm.max_stack};
    SrcTree f{father, n_father, pf.chunks.data(), (int64_t)pf.chunks.size(), &pf.big_ends, pf.max_stack};
    if (!compose_child(m, point, c_end, f, donor_node, d_end, child.data(), (int64_t)child.size(), opt, &pc, &why))
        return GP_EINVAL;
    int64_t total = 0, n_in = 0, reused = 0;
    for (const Chunk& ch : pc.chunks) {
        total += ch.code_len;
        n_in += (int64_t)ch.inputs.size();
        reused += ch.dev_src >= 0;
    }
    if (n_code) *n_code = total;
    if (max_stack) *max_stack = pc.max_stack;
    if (n_big) *n_big = (int64_t)pc.big_ends.size();
    if (n_reused) *n_reused = reused;
    if (total > code_cap || (int64_t)pc.chunks.size() > chunk_cap || n_in > inputs_cap ||
        (int64_t)pc.big_ends.size() > big_cap)
        return GP_ENOMEM;
    int64_t at = 0, k_in = 0;
    for (int64_t k = 0; k < (int64_t)pc.chunks.size(); ++k) {
        const Chunk& ch = pc.chunks[k];
        const uint32_t* from = ch.dev_src >= 0 ? src.data() + ch.dev_src : pc.code.data() + ch.code_off;
        if (code_out) std::memcpy(code_out + at, from, (size_t)ch.code_len * sizeof(uint32_t));
        if (chunk_out) {
            int64_t* o = chunk_out + 6 * k;
            o[0] = at;
            o[1] = ch.code_len;
            o[2] = ch.parent;
            o[3] = (int64_t)ch.inputs.size();
            o[4] = ch.root_node;
            o[5] = ch.end_node;
        }
        at += ch.code_len;
        for (int32_t in : ch.inputs)
            if (inputs_out) inputs_out[k_in++] = in;
    }
    for (size_t i = 0; i < pc.big_ends.size(); ++i)
        if (big_out) {
            big_out[2 * i] = pc.big_ends[i].first;
            big_out[2 * i + 1] = pc.big_ends[i].second;
        }
    return (int64_t)pc.chunks.size();
}

int64_t gp_inspect_program(int vtype, int n_inputs, const uint8_t* ops, int64_t n, int64_t chunk_nodes,
                           int stack_slots, int threads, uint32_t* code_out, int64_t code_cap, int64_t* chunk_out,
                           int64_t chunk_cap, int32_t* inputs_out, int64_t inputs_cap, int64_t* n_code,
                           int32_t* max_stack)
{
    if ((vtype != GP_F32 && vtype != GP_BOOL) || n_inputs < 1 || n_inputs > kMaxInputs || !ops) return GP_EINVAL;
    if (!validate_prefix(ops, n, n_inputs, nullptr)) return GP_EINVAL;
    CompileOptions opt;
    opt.vtype = vtype;
    opt.n_inputs = n_inputs;
    opt.chunk_nodes = chunk_nodes > 0 ? chunk_nodes : 4096;
    opt.stack_slots = stack_slots > 0 ? stack_slots : compile_stack_slots();
    opt.threads = std::max(1, std::min(threads, 64));
    TreeProg pg;
    std::string why;
    if (!compile_tree(ops, n, opt, nullptr, 0, &pg, &why)) return GP_EINVAL;
    if (n_code) *n_code = (int64_t)pg.code.size();
    if (max_stack) *max_stack = pg.max_stack;
    int64_t n_in = 0;
    for (auto& ch : pg.chunks) n_in += (int64_t)ch.inputs.size();
    if ((int64_t)pg.code.size() > code_cap || (int64_t)pg.chunks.size() > chunk_cap || n_in > inputs_cap)
        return GP_ENOMEM;
    if (code_out) std::memcpy(code_out, pg.code.data(), pg.code.size() * sizeof(uint32_t));
    int64_t k_in = 0;
    for (int64_t k = 0; k < (int64_t)pg.chunks.size(); ++k) {
        const Chunk& ch = pg.chunks[k];
        if (chunk_out) {
            chunk_out[4 * k + 0] = ch.code_off;
            chunk_out[4 * k + 1] = ch.code_len;
            chunk_out[4 * k + 2] = ch.parent;
            chunk_out[4 * k + 3] = (int64_t)ch.inputs.size();
        }
        for (int32_t in : ch.inputs)
            if (inputs_out) inputs_out[k_in++] = in;
    }
    return (int64_t)pg.chunks.size();
}

}  // extern "C"
