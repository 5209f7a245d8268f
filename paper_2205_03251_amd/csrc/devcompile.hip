// Device-side compilation of a population of prefix trees (Section 3.1):
// the programs, chunk tables and parent-cache spines that compile_tree and
// assemble_population build on the host, byte for byte, built from the trees'
// bytes in device memory.  The per-thread steps are in devcompile_core.h.
//
// Passes: the device tree index (validity, subtree ends, parents); one thread
// per terminal finishes nodes bottom-up (stack need, cuts, instruction form,
// code length); the crossover points' paths are read up the parent index and
// their records assigned on the host; chunk roots are compacted, numbered and
// given code offsets (host prefix sums over per-chunk lengths); one thread per
// chunk counts its LOADs, then writes its code straight into the population's
// program.  The host keeps only per-chunk and per-record tables.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <unordered_map>

#include "devcompile_core.h"
#include "runtime.h"

namespace gpe {

namespace {

// Values handed from one thread to another: agent-coherent (sc1) stores and
// loads, and a relaxed agent-scope counter.  The writer waits for its stores
// to complete before it counts; the reader loads only after the count
// returned (a compiler barrier keeps the loads after it; they depend on its
// value).  The same hand-off as the interpreter's chunk pending counters.
struct DevMem {
    __device__ static int32_t ld(const int32_t* p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void st(int32_t* p, int32_t v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static int32_t fetch_add(int32_t* p, int32_t v)
    {
        return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static uint64_t fetch_or64(uint64_t* p, uint64_t v)
    {
        return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void publish() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
    __device__ static void after_count() { asm volatile("" ::: "memory"); }
    __device__ static void err(int32_t* p, int32_t v) { atomicOr(p, v); }
};

__global__ __launch_bounds__(256) void k_dc_up(DcNodes q)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= q.n || (q.ops[g] & kFuncBit)) return;
    const int64_t t = dc_tree_of(q, g);
    const int64_t s = q.offsets[t], e = q.offsets[t + 1];
    dc_leaf<DevMem>(q, g);
    for (int64_t v = g; v >= 0;) v = dc_step<DevMem>(q, s, e, v);
}

// The same with the packed hand-off (chunk targets up to kDcPackMaxC): the
// values of a finished node reach its parent in the arrival atomic itself;
// the per-node stores are read only by later launches.
struct DevMemPacked : DevMem {
    __device__ static void st(int32_t* p, int32_t v) { *p = v; }
};

// Persistent waves: a wave takes kDcBatch positions at a time from a shared
// cursor, and each lane whose walk has ended takes the next terminal of the
// wave's batch, so no lane idles while the longest walk of its wave goes on.
constexpr int kDcBatch = 1024;

__device__ __forceinline__ int64_t dc_uniform(int64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The next batch [*pb, *pe) of [0, n) for this wave; false once none is left.
__device__ __forceinline__ bool dc_take_batch(unsigned long long* cursor, int64_t n, int64_t batch, int64_t* pb,
                                              int64_t* pe)
{
    int64_t b = 0;
    if ((threadIdx.x & 63) == 0) b = (int64_t)atomicAdd(cursor, (unsigned long long)batch);
    b = dc_uniform(b);
    *pb = b;
    *pe = b + batch < n ? b + batch : n;
    return b < n;
}

__global__ __launch_bounds__(256) void k_dc_up_packed(DcNodes q, unsigned long long* cursor)
{
    const uint64_t below = (1ull << (threadIdx.x & 63)) - 1;
    int64_t v = -1, s = 0, e = 0, ts = 0, te = 0, pb = 0, pe = 0;
    uint32_t w = 0;
    bool more = true;
    for (;;) {
        if (pb >= pe && more) more = dc_take_batch(cursor, q.n, kDcBatch, &pb, &pe);
        const uint64_t idle = __ballot(v < 0);
        if (v < 0 && pb < pe) {
            const int64_t g = pb + __popcll(idle & below);
            if (g < pe && !(q.ops[g] & kFuncBit)) {
                if (g < ts || g >= te) {
                    const int64_t t = dc_tree_of(q, g);
                    ts = q.offsets[t];
                    te = q.offsets[t + 1];
                }
                s = ts;
                e = te;
                w = dc_leaf_packed<DevMemPacked>(q, g);
                v = g;
            }
        }
        if (pb < pe) pb += __popcll(idle);
        if (v >= 0) v = dc_step_packed<DevMemPacked>(q, s, e, v, &w);
        if (!more && pb >= pe && __ballot(v >= 0) == 0) break;
    }
}

// After the bottom-up pass: cuts into the info words, chunk-root flags.
__global__ __launch_bounds__(256) void k_dc_finish(DcNodes q, uint8_t* flags)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < q.n) flags[g] = dc_finish(q, g) ? 1 : 0;
}

// Chunk roots: their chunk ids into cnt, their code lengths and subtree ends out.
__global__ __launch_bounds__(256) void k_dc_root_info(DcNodes q, const int64_t* roots, const int32_t* ids, int64_t n,
                                                      int32_t* rlen, int32_t* rend)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t g = roots[k];
    q.cnt[g] = ids[k];
    rlen[k] = q.len[g];
    rend[k] = q.endl[g];
}

// Subtree ends of listed nodes.
__global__ __launch_bounds__(256) void k_dc_ends(DcNodes q, const int64_t* nodes, int64_t n, int32_t* out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) out[k] = q.endl[nodes[k]];
}

// Paths of crossover points (global node pts[i]) up to the root.  Count pass
// (lv null): depth[i].  Write pass: per ancestor, nearest first, from
// lv[lv_off[i]]; the point's opcode and subtree end.
__global__ __launch_bounds__(256) void k_dc_paths(DcNodes q, const int64_t* pts, int64_t n_pts, const int64_t* lv_off,
                                                  int32_t* depth, DcPathLevel* lv, uint8_t* pop, int32_t* pend)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_pts) return;
    const int64_t c = pts[i];
    const int64_t s = q.offsets[dc_tree_of(q, c)];
    if (!lv) {
        int32_t d = 0;
        for (int32_t a = q.parl[c]; a >= 0; a = q.parl[s + a]) ++d;
        depth[i] = d;
        return;
    }
    pop[i] = q.ops[c];
    pend[i] = q.endl[c];
    DcPathLevel* out = lv + lv_off[i];
    int32_t below = (int32_t)(c - s);
    for (int32_t a = q.parl[c]; a >= 0; a = q.parl[s + a]) {
        const int32_t l = a + 1, r = q.endl[s + l];
        const bool right = below != l;
        const int32_t sib = right ? l : r;
        DcPathLevel x;
        x.a = a;
        x.sib = sib;
        x.fside = (q.ops[s + a] & 3) | (right ? 4 : 0);
        x.sib_op = q.ops[s + sib];
        *out++ = x;
        below = a;
    }
}

__global__ __launch_bounds__(256) void k_dc_cut_of(DcNodes q, const int64_t* nodes, int64_t n, uint8_t* out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) out[k] = dc_cut(q, nodes[k]) ? 1 : 0;
}

// Recorded nodes: their STOREs lengthen their own subtrees' code.
__global__ __launch_bounds__(256) void k_dc_store(DcNodes q, const int64_t* nodes, const int32_t* inc,
                                                  const int32_t* rec_id, int64_t n, int32_t* rec)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t g = nodes[k];
    q.len[g] += inc[k];
    rec[g] = rec_id[k];
}

// Compaction of a flag array, in order: a block takes kDcSpan positions, 16
// per thread.  Count pass: the block's set flags.  Write pass: each set
// position to out[boff[block] + its rank in the block].
constexpr int kDcSpan = 4096;

__device__ __forceinline__ uint32_t dc_flags16(const uint8_t* flags, int64_t base, int64_t n)
{
    uint32_t m = 0;
    if (base + 16 <= n) {                       // flags hold 0 or 1; base is a multiple of 16
        const uint4 x = *(const uint4*)(flags + base);
        const uint32_t wd[4] = {x.x, x.y, x.z, x.w};
        for (int j = 0; j < 16; ++j) m |= ((wd[j >> 2] >> (8 * (j & 3))) & 1u) << j;
        return m;
    }
    for (int j = 0; j < 16; ++j)
        if (base + j < n && flags[base + j]) m |= 1u << j;
    return m;
}

__global__ __launch_bounds__(256) void k_dc_compact_count(const uint8_t* flags, int64_t n, int64_t* bcount)
{
    __shared__ int32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * kDcSpan + (int64_t)threadIdx.x * 16;
    int32_t c = __popc(dc_flags16(flags, base, n));
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(256) void k_dc_compact_write(const uint8_t* flags, int64_t n, const int64_t* boff,
                                                          int64_t* out)
{
    __shared__ int32_t pre[256];
    const int64_t base = (int64_t)blockIdx.x * kDcSpan + (int64_t)threadIdx.x * 16;
    const uint32_t m = dc_flags16(flags, base, n);
    pre[threadIdx.x] = __popc(m);
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {              // inclusive scan over the block's threads
        const int32_t v = threadIdx.x >= (unsigned)o ? pre[threadIdx.x - o] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t at = boff[blockIdx.x] + pre[threadIdx.x] - __popc(m);
    for (int j = 0; j < 16; ++j)
        if (m & (1u << j)) out[at++] = base + j;
}

// Emission on persistent waves: a lane whose chunk is done takes the next
// chunk of its wave's batch.
constexpr int kDcEmitBatch = 64;

__global__ __launch_bounds__(256) void k_dc_emit(DcNodes q, DcChunks c, unsigned long long* cursor)
{
    const uint64_t below = (1ull << (threadIdx.x & 63)) - 1;
    int64_t pb = 0, pe = 0;
    bool more = true;
    int32_t busy = 0;                           // an integer, not a lane-mask boolean, across the branches
    DcEmit st{};
    for (;;) {
        if (pb >= pe && more) more = dc_take_batch(cursor, c.n, kDcEmitBatch, &pb, &pe);
        const uint64_t idle = __ballot(busy == 0);
        if (busy == 0 && pb < pe) {
            const int64_t k = pb + __popcll(idle & below);
            if (k < pe) {
                dc_emit_begin(q, c, k, st);
                busy = 1;
            }
        }
        if (pb < pe) pb += __popcll(idle);
        if (busy) busy = dc_emit_step(q, c, st) ? 1 : 0;
        if (!more && pb >= pe && __ballot(busy != 0) == 0) break;
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

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

int up(Ctx* c, DevArena* arena, DevBuf& b, const void* src, size_t bytes, hipStream_t s)
{
    RC(scratch_alloc(c, arena, b, bytes));
    if (bytes) HIPC(c, hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return GP_OK;
}

int down(Ctx* c, void* dst, const DevBuf& b, size_t bytes, hipStream_t s)
{
    if (bytes) HIPC(c, hipMemcpyAsync(dst, b.p, bytes, hipMemcpyDeviceToHost, s));
    return GP_OK;
}

// The flagged positions of flags[0 .. n), ascending, into out; their number
// into *count.
int dc_select(Ctx* c, DevArena* arena, const uint8_t* flags, int64_t n, DevBuf& out, int64_t* count, hipStream_t s)
{
    const int64_t nb = (n + kDcSpan - 1) / kDcSpan;
    DevBuf bc;
    RC(scratch_alloc(c, arena, bc, (size_t)nb * 8));
    hipLaunchKernelGGL(k_dc_compact_count, dim3((unsigned)nb), dim3(256), 0, s, flags, n, bc.as<int64_t>());
    HIPC(c, hipGetLastError());
    std::vector<int64_t> h(nb);
    RC(down(c, h.data(), bc, (size_t)nb * 8, s));
    HIPC(c, hipStreamSynchronize(s));
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t v = h[b];
        h[b] = run;
        run += v;
    }
    *count = run;
    RC(scratch_alloc(c, arena, out, (size_t)std::max<int64_t>(1, run) * 8));
    if (run == 0) return GP_OK;
    HIPC(c, hipMemcpyAsync(bc.p, h.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_dc_compact_write, dim3((unsigned)nb), dim3(256), 0, s, flags, n, bc.as<int64_t>(),
                       out.as<int64_t>());
    HIPC(c, hipGetLastError());
    HIPC(c, hipStreamSynchronize(s));
    return GP_OK;
}

// Blocks of persistent waves for a launch over `items` units of work.
unsigned dc_persistent_blocks(Ctx* c, int64_t items, int64_t batch, int max_blocks)
{
    const int64_t want = (items + batch * 4 - 1) / (batch * 4);
    int64_t cap = (int64_t)std::max(1, c->n_cu) * 8;
    if (max_blocks > 0) cap = std::min<int64_t>(cap, max_blocks);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, cap));
}

// f(i) for every i in [0, n), on up to 16 host threads taking blocks of
// consecutive indices.
template <class F> void dc_parallel(int64_t n, F f)
{
    const int64_t hw = std::min<int64_t>(16, std::max(1u, std::thread::hardware_concurrency()));
    const int nth = (int)std::min<int64_t>(hw, n);
    if (nth <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    const int64_t blk = std::max<int64_t>(1, n / (nth * 32));
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            const int64_t a = next.fetch_add(blk);
            if (a >= n) return;
            for (int64_t i = a; i < std::min(n, a + blk); ++i) f(i);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
}

// Phase times of a compilation on stderr when GPEVAL_TRACE_LOAD is set.
struct DcTrace {
    bool on = std::getenv("GPEVAL_TRACE_LOAD") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char* what)
    {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[devcompile] %-28s %9.2f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

}  // namespace

int device_compile_population(Ctx* c, int vtype, int n_inputs, int64_t n_trees, const uint8_t* dops,
                              const int64_t* doffs, const int64_t* offsets, const uint8_t* host_ops,
                              const int64_t* rec_points, const int64_t* rec_offsets, const int64_t* key_points,
                              int64_t chunk_nodes, int64_t index_min_size, Pop* out,
                              std::vector<TreeProg>* progs_out, DevArena* arena, hipStream_t s, int max_blocks)
{
    const int64_t n = offsets[n_trees];
    if (n < 1 || n > (int64_t)INT32_MAX - 1) return set_err(c, GP_EINVAL, "at most 2^31 - 2 nodes per load");
    if (n_trees > INT32_MAX / 2) return set_err(c, GP_EINVAL, "too many trees");
    // crossover points: checked before any device work
    int64_t n_pts = 0;
    if (rec_points) {
        for (int64_t t = 0; t < n_trees; ++t) {
            if (rec_offsets[t + 1] < rec_offsets[t])
                return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + ": record_offsets not increasing");
            for (int64_t i = rec_offsets[t]; i < rec_offsets[t + 1]; ++i)
                if (rec_points[i] < 0 || rec_points[i] >= offsets[t + 1] - offsets[t])
                    return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + ": record point " +
                                                     std::to_string(rec_points[i]) + " out of range");
        }
        n_pts = rec_offsets[n_trees];
    }
    DcTrace tr;
    // validity, subtree ends and parents
    DevBuf valid, endl, parl;
    RC(scratch_alloc(c, arena, valid, (size_t)n_trees * 4));
    RC(scratch_alloc(c, arena, endl, (size_t)n * 4));
    RC(scratch_alloc(c, arena, parl, (size_t)n * 4));
    RC(index_trees(c, n_inputs, n_trees, dops, doffs, n, valid.as<int32_t>(), endl.as<int32_t>(),
                   parl.as<int32_t>(), nullptr, nullptr, s, arena));
    {
        std::vector<int32_t> v(n_trees);
        RC(down(c, v.data(), valid, (size_t)n_trees * 4, s));
        HIPC(c, hipStreamSynchronize(s));
        for (int64_t t = 0; t < n_trees; ++t) {
            if (v[t]) continue;
            // the host check of that tree says what is wrong with it
            std::vector<uint8_t> tree((size_t)(offsets[t + 1] - offsets[t]));
            if (host_ops) std::copy(host_ops + offsets[t], host_ops + offsets[t + 1], tree.begin());
            else HIPC(c, hipMemcpy(tree.data(), dops + offsets[t], tree.size(), hipMemcpyDeviceToHost));
            std::string why = "not a valid prefix tree";
            validate_prefix(tree.data(), (int64_t)tree.size(), n_inputs, &why);
            return set_err(c, GP_EINVAL, "tree " + std::to_string(t) + ": " + why);
        }
    }
    valid.release();
    tr.mark("index");

    // the packed hand-off when every value it carries fits (see devcompile_core.h)
    const int64_t C = std::max<int64_t>(2, chunk_nodes);
    const bool packed = C <= kDcPackMaxC && compile_stack_slots() <= 32;
    DevBuf info, len, open, cnt, ncut, slot64, err, flags, big, counter;
    if (index_min_size > 0) RC(scratch_alloc(c, arena, big, (size_t)n));
    RC(scratch_alloc(c, arena, info, (size_t)n * 4));
    RC(scratch_alloc(c, arena, len, (size_t)n * 4));
    RC(scratch_alloc(c, arena, open, (size_t)n * 4));
    RC(scratch_alloc(c, arena, cnt, (size_t)n * 4));
    RC(scratch_alloc(c, arena, ncut, (size_t)n));
    RC(scratch_alloc(c, arena, err, 4));
    RC(scratch_alloc(c, arena, counter, 16));
    if (packed) {
        RC(scratch_alloc(c, arena, slot64, (size_t)n * 8));
        HIPC(c, launch_fill_i32(slot64.as<int32_t>(), 2 * n, 0, s));
    } else {
        HIPC(c, launch_fill_i32(cnt.as<int32_t>(), n, 0, s));
    }
    HIPC(c, launch_fill_u8(ncut.as<uint8_t>(), n, 0, s));
    HIPC(c, launch_fill_i32(err.as<int32_t>(), 1, 0, s));
    DcNodes q{};
    q.ops = dops;
    q.offsets = doffs;
    q.n_trees = n_trees;
    q.n = n;
    q.endl = endl.as<int32_t>();
    q.parl = parl.as<int32_t>();
    q.info = info.as<int32_t>();
    q.len = len.as<int32_t>();
    q.open = open.as<int32_t>();
    q.cnt = cnt.as<int32_t>();
    q.slot64 = slot64.as<uint64_t>();
    q.ncut = ncut.as<uint8_t>();
    q.big = index_min_size > 0 ? big.as<uint8_t>() : nullptr;
    q.big_min = index_min_size;
    q.err = err.as<int32_t>();
    q.boolean = vtype == GP_BOOL ? 1 : 0;
    q.S = compile_stack_slots();
    q.C = C;
    if (packed) {
        HIPC(c, launch_fill_i32(counter.as<int32_t>(), 4, 0, s));
        hipLaunchKernelGGL(k_dc_up_packed, dim3(dc_persistent_blocks(c, n, kDcBatch, max_blocks)), dim3(256), 0, s, q,
                           counter.as<unsigned long long>());
    } else {
        hipLaunchKernelGGL(k_dc_up, dim3(blocks_for(n)), dim3(256), 0, s, q);
    }
    HIPC(c, hipGetLastError());
    int32_t errv = 0;
    HIPC(c, hipMemcpyAsync(&errv, err.p, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    if (errv) return set_err(c, GP_EINVAL, "internal error: inconsistent tree index (" + std::to_string(errv) + ")");
    slot64.release();
    tr.mark(packed ? "bottom-up pass (packed)" : "bottom-up pass");

    // parent-cache records (Section 6.2): the points' paths, read on the device
    std::vector<int64_t> rec_base(n_trees, 0), n_rec(n_trees, 0);
    std::vector<std::vector<Spine>> spines(n_trees);
    DevBuf rec;
    if (n_pts > 0) {
        std::vector<int64_t> pts(n_pts);
        for (int64_t t = 0; t < n_trees; ++t)
            for (int64_t i = rec_offsets[t]; i < rec_offsets[t + 1]; ++i) pts[i] = offsets[t] + rec_points[i];
        DevBuf pts_d, depth_d, lvoff_d, lv_d, pop_d, pend_d;
        RC(up(c, arena, pts_d, pts.data(), (size_t)n_pts * 8, s));
        RC(scratch_alloc(c, arena, depth_d, (size_t)n_pts * 4));
        hipLaunchKernelGGL(k_dc_paths, dim3(blocks_for(n_pts)), dim3(256), 0, s, q, pts_d.as<int64_t>(), n_pts,
                           (const int64_t*)nullptr, depth_d.as<int32_t>(), (DcPathLevel*)nullptr, (uint8_t*)nullptr,
                           (int32_t*)nullptr);
        HIPC(c, hipGetLastError());
        std::vector<int32_t> depth(n_pts);
        RC(down(c, depth.data(), depth_d, (size_t)n_pts * 4, s));
        HIPC(c, hipStreamSynchronize(s));
        std::vector<int64_t> lv_off(n_pts + 1, 0);
        for (int64_t i = 0; i < n_pts; ++i) lv_off[i + 1] = lv_off[i] + depth[i];
        RC(up(c, arena, lvoff_d, lv_off.data(), (size_t)(n_pts + 1) * 8, s));
        RC(scratch_alloc(c, arena, lv_d, (size_t)std::max<int64_t>(1, lv_off[n_pts]) * sizeof(DcPathLevel)));
        RC(scratch_alloc(c, arena, pop_d, (size_t)n_pts));
        RC(scratch_alloc(c, arena, pend_d, (size_t)n_pts * 4));
        hipLaunchKernelGGL(k_dc_paths, dim3(blocks_for(n_pts)), dim3(256), 0, s, q, pts_d.as<int64_t>(), n_pts,
                           lvoff_d.as<int64_t>(), (int32_t*)nullptr, lv_d.as<DcPathLevel>(), pop_d.as<uint8_t>(),
                           pend_d.as<int32_t>());
        HIPC(c, hipGetLastError());
        std::vector<DcPathLevel> lv((size_t)lv_off[n_pts]);
        std::vector<uint8_t> pop(n_pts);
        std::vector<int32_t> pend(n_pts);
        RC(down(c, lv.data(), lv_d, lv.size() * sizeof(DcPathLevel), s));
        RC(down(c, pop.data(), pop_d, (size_t)n_pts, s));
        RC(down(c, pend.data(), pend_d, (size_t)n_pts * 4, s));
        HIPC(c, hipStreamSynchronize(s));
        // per tree, in parallel: its records and spines, then (once the cut
        // flags are known) the words its recorded nodes add
        std::vector<std::vector<DcStored>> st_t(n_trees);
        dc_parallel(n_trees, [&](int64_t t) {
            const int64_t p0 = rec_offsets[t], np = rec_offsets[t + 1] - p0;
            std::vector<int64_t> loff(np + 1);
            for (int64_t i = 0; i <= np; ++i) loff[i] = lv_off[p0 + i] - lv_off[p0];
            n_rec[t] = dc_tree_records(offsets[t], np, rec_points + p0, pop.data() + p0, pend.data() + p0,
                                       loff.data(), lv.data() + lv_off[p0], &spines[t], &st_t[t]);
            if (key_points)
                for (int64_t i = 0; i < np; ++i) spines[t][i].point = key_points[p0 + i];
        });
        std::vector<int64_t> st_off(n_trees + 1, 0);
        int64_t rb = 0;
        for (int64_t t = 0; t < n_trees; ++t) {
            if (n_rec[t] > (int64_t)kMaxPayload)
                return set_err(c, GP_EINVAL,
                               "tree " + std::to_string(t) + ": too many parent-cache records in one tree");
            rec_base[t] = rb;
            rb += n_rec[t];
            st_off[t + 1] = st_off[t] + (int64_t)st_t[t].size();
        }
        if (rb > INT32_MAX / 2) return set_err(c, GP_EINVAL, "population too large for one load");
        const int64_t ns = st_off[n_trees];
        if (ns > 0) {
            std::vector<int64_t> nodes(ns);
            std::vector<int32_t> ids(ns), inc(ns);
            dc_parallel(n_trees, [&](int64_t t) {
                for (size_t i = 0; i < st_t[t].size(); ++i) {
                    nodes[st_off[t] + i] = st_t[t][i].node;
                    ids[st_off[t] + i] = st_t[t][i].rec;
                }
            });
            DevBuf nodes_d, cut_d, inc_d, ids_d;
            RC(up(c, arena, nodes_d, nodes.data(), (size_t)ns * 8, s));
            RC(scratch_alloc(c, arena, cut_d, (size_t)ns));
            hipLaunchKernelGGL(k_dc_cut_of, dim3(blocks_for(ns)), dim3(256), 0, s, q, nodes_d.as<int64_t>(), ns,
                               cut_d.as<uint8_t>());
            HIPC(c, hipGetLastError());
            std::vector<uint8_t> cut(ns);
            RC(down(c, cut.data(), cut_d, (size_t)ns, s));
            HIPC(c, hipStreamSynchronize(s));
            dc_parallel(n_trees, [&](int64_t t) {
                dc_store_words(st_t[t].data(), cut.data() + st_off[t], st_t[t].size(), inc.data() + st_off[t]);
            });
            RC(up(c, arena, inc_d, inc.data(), (size_t)ns * 4, s));
            RC(up(c, arena, ids_d, ids.data(), (size_t)ns * 4, s));
            RC(scratch_alloc(c, arena, rec, (size_t)n * 4));
            HIPC(c, launch_fill_i32(rec.as<int32_t>(), n, -1, s));
            hipLaunchKernelGGL(k_dc_store, dim3(blocks_for(ns)), dim3(256), 0, s, q, nodes_d.as<int64_t>(),
                               inc_d.as<int32_t>(), ids_d.as<int32_t>(), ns, rec.as<int32_t>());
            HIPC(c, hipGetLastError());
            HIPC(c, hipStreamSynchronize(s));
            q.rec = rec.as<int32_t>();
        }
    }
    tr.mark("records");
    // chunk roots, ascending, and their numbering
    RC(scratch_alloc(c, arena, flags, (size_t)n));
    hipLaunchKernelGGL(k_dc_finish, dim3(blocks_for(n)), dim3(256), 0, s, q, flags.as<uint8_t>());
    HIPC(c, hipGetLastError());
    DevBuf roots_d;
    int64_t nch = 0;
    RC(dc_select(c, arena, flags.as<uint8_t>(), n, roots_d, &nch, s));   // waits for the stream
    flags.release();
    ncut.release();
    q.ncut = nullptr;                                               // the cuts are in the info words now
    if (nch < n_trees || nch > INT32_MAX / 2) return set_err(c, GP_EINVAL, "population too large for one load");
    std::vector<int64_t> roots_asc(nch);
    RC(down(c, roots_asc.data(), roots_d, (size_t)nch * 8, s));
    HIPC(c, hipStreamSynchronize(s));
    std::vector<int64_t> root, tstart, cbase;
    std::vector<int32_t> ctree, ids;
    if (!dc_number_chunks(roots_asc, offsets, n_trees, &root, &tstart, &ctree, &ids, &cbase))
        return set_err(c, GP_EINVAL, "internal error: a tree without its root chunk");
    std::vector<int32_t> rlen(nch), rend(nch);
    {
        DevBuf ids_d, rlen_d, rend_d;
        RC(up(c, arena, ids_d, ids.data(), (size_t)nch * 4, s));
        RC(scratch_alloc(c, arena, rlen_d, (size_t)nch * 4));
        RC(scratch_alloc(c, arena, rend_d, (size_t)nch * 4));
        hipLaunchKernelGGL(k_dc_root_info, dim3(blocks_for(nch)), dim3(256), 0, s, q, roots_d.as<int64_t>(),
                           ids_d.as<int32_t>(), nch, rlen_d.as<int32_t>(), rend_d.as<int32_t>());
        HIPC(c, hipGetLastError());
        // in ascending root order
        std::vector<int32_t> a(nch), b(nch);
        RC(down(c, a.data(), rlen_d, (size_t)nch * 4, s));
        RC(down(c, b.data(), rend_d, (size_t)nch * 4, s));
        HIPC(c, hipStreamSynchronize(s));
        for (int64_t j = 0; j < nch; ++j) {
            rlen[ids[j]] = a[j];
            rend[ids[j]] = b[j];
        }
    }
    roots_d.release();
    tr.mark("chunk roots");
    std::vector<int64_t> code_len(nch), code_off(nch + 1, 0);
    for (int64_t k = 0; k < nch; ++k) {
        code_len[k] = (int64_t)rlen[k] + 1;
        code_off[k + 1] = code_off[k] + code_len[k];
    }
    const int64_t n_code = code_off[nch];
    if (out) out->max_code_len = nch ? *std::max_element(code_len.begin(), code_len.end()) : 0;

    // code emission, one pass: each child chunk learns its parent and which of
    // the parent's LOADs reads it; the LOAD lists are then put together here
    DevBuf root_d, ts_d, off_d, nin_d, par_d, lix_d, nodes_d, ms_d, st_d, slot;
    RC(up(c, arena, root_d, root.data(), (size_t)nch * 8, s));
    RC(up(c, arena, ts_d, tstart.data(), (size_t)nch * 8, s));
    RC(up(c, arena, off_d, code_off.data(), (size_t)nch * 8, s));
    RC(scratch_alloc(c, arena, nin_d, (size_t)nch * 4));
    RC(scratch_alloc(c, arena, par_d, (size_t)nch * 4));
    RC(scratch_alloc(c, arena, lix_d, (size_t)nch * 4));
    RC(scratch_alloc(c, arena, nodes_d, (size_t)nch * 8));
    RC(scratch_alloc(c, arena, ms_d, (size_t)nch * 4));
    RC(scratch_alloc(c, arena, st_d, (size_t)nch));
    RC(scratch_alloc(c, arena, slot, (size_t)n));
    q.slot = slot.as<uint8_t>();
    HIPC(c, launch_fill_i32(par_d.as<int32_t>(), nch, -1, s));
    HIPC(c, launch_fill_i32(lix_d.as<int32_t>(), nch, -1, s));
    // the program: the population's own buffer, or a temporary one copied to the host
    DevBuf code_tmp;
    DevBuf& code = out ? out->code : code_tmp;
    if (out) RC(dev_alloc(c, code, (size_t)(n_code + 1) * 4));
    else RC(scratch_alloc(c, arena, code, (size_t)(n_code + 1) * 4));
    HIPC(c, launch_fill_i32((int32_t*)code.p + n_code, 1, 0, s));   // one word past the end for the fetch-ahead
    DcChunks ck{};
    ck.n = nch;
    ck.root = root_d.as<int64_t>();
    ck.tree_start = ts_d.as<int64_t>();
    ck.code_off = off_d.as<int64_t>();
    ck.code = code.as<uint32_t>();
    ck.n_in = nin_d.as<int32_t>();
    ck.parent = par_d.as<int32_t>();
    ck.load_idx = lix_d.as<int32_t>();
    ck.nodes = nodes_d.as<int64_t>();
    ck.max_slot = ms_d.as<int32_t>();
    ck.stores = st_d.as<uint8_t>();
    HIPC(c, launch_fill_i32(counter.as<int32_t>(), 4, 0, s));
    hipLaunchKernelGGL(k_dc_emit, dim3(dc_persistent_blocks(c, nch, kDcEmitBatch, max_blocks)), dim3(256), 0, s, q, ck,
                       counter.as<unsigned long long>());
    HIPC(c, hipGetLastError());
    if (tr.on) {
        HIPC(c, hipStreamSynchronize(s));
        tr.mark("emission kernel");
    }
    std::vector<int32_t> n_in(nch), parent(nch), load_idx(nch), max_slot(nch);
    std::vector<int64_t> nodes(nch);
    std::vector<uint8_t> stores(nch);
    RC(down(c, n_in.data(), nin_d, (size_t)nch * 4, s));
    RC(down(c, parent.data(), par_d, (size_t)nch * 4, s));
    RC(down(c, load_idx.data(), lix_d, (size_t)nch * 4, s));
    RC(down(c, nodes.data(), nodes_d, (size_t)nch * 8, s));
    RC(down(c, max_slot.data(), ms_d, (size_t)nch * 4, s));
    RC(down(c, stores.data(), st_d, (size_t)nch, s));
    HIPC(c, hipStreamSynchronize(s));
    slot.release();
    for (int64_t k = 0; k < nch; ++k)
        if ((uint32_t)n_in[k] > kMaxPayload) return set_err(c, GP_EINVAL, "chunk reads too many child chunks");
    std::vector<int64_t> in_off;
    std::vector<int32_t> ins;
    if (!dc_scatter_inputs(nch, n_in.data(), parent.data(), load_idx.data(), &in_off, &ins) ||
        in_off[nch] != nch - n_trees) {
        int64_t loads = 0, orphans = 0, first = -1;
        for (int64_t k = 0; k < nch; ++k) {
            loads += n_in[k];
            const bool top = k == cbase[ctree[k] + 1] - 1;
            if (!top && parent[k] < 0 && orphans++ == 0) first = k;
        }
        return set_err(c, GP_EINVAL, "internal error: chunk inputs do not add up (" + std::to_string(loads) +
                                         " LOADs, " + std::to_string(nch - n_trees) + " child chunks, " +
                                         std::to_string(orphans) + " without a parent, first " +
                                         std::to_string(first) + ")");
    }
    tr.mark("emission");

    // subtrees of at least index_min_size nodes (co-evaluation's path search),
    // flagged by the bottom-up pass
    std::vector<int64_t> big_nodes;
    std::vector<int32_t> big_end;
    if (index_min_size > 0) {
        DevBuf big_d;
        int64_t nb = 0;
        RC(dc_select(c, arena, big.as<uint8_t>(), n, big_d, &nb, s));
        if (nb > 0) {
            DevBuf bend_d;
            RC(scratch_alloc(c, arena, bend_d, (size_t)nb * 4));
            hipLaunchKernelGGL(k_dc_ends, dim3(blocks_for(nb)), dim3(256), 0, s, q, big_d.as<int64_t>(), nb,
                               bend_d.as<int32_t>());
            HIPC(c, hipGetLastError());
            big_nodes.resize(nb);
            big_end.resize(nb);
            RC(down(c, big_nodes.data(), big_d, (size_t)nb * 8, s));
            RC(down(c, big_end.data(), bend_d, (size_t)nb * 4, s));
            HIPC(c, hipStreamSynchronize(s));
        }
    }
    tr.mark("large subtrees");
    if (progs_out) {
        // each tree's program in host memory, as compile_tree leaves it
        std::vector<uint32_t> words((size_t)n_code);
        HIPC(c, hipMemcpyAsync(words.data(), code.p, (size_t)n_code * 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        progs_out->assign(n_trees, TreeProg());
        int bad = 0;
        dc_parallel(n_trees, [&](int64_t t) {
            TreeProg& pg = (*progs_out)[t];
            const int64_t b = cbase[t], m = cbase[t + 1] - b, s0 = offsets[t], w0 = code_off[b];
            pg.code.assign(words.begin() + w0, words.begin() + code_off[cbase[t + 1]]);
            pg.chunks.resize(m);
            int32_t tms = 0;
            for (int64_t i = m - 1; i >= 0; --i) {
                const int64_t k = b + i;
                Chunk& ch = pg.chunks[i];
                const bool top = i == m - 1;
                if (top != (parent[k] < 0) || (!top && (parent[k] <= k || parent[k] >= b + m))) {
                    bad = 1;
                    return;
                }
                ch.code_off = code_off[k] - w0;
                ch.code_len = code_len[k];
                ch.parent = top ? -1 : parent[k] - (int32_t)b;
                ch.root_node = root[k] - s0;
                ch.nodes = nodes[k];
                ch.path_nodes = nodes[k] + (top ? 0 : pg.chunks[ch.parent].path_nodes);
                ch.end_node = index_min_size > 0 ? rend[k] : -1;
                ch.stores = stores[k] != 0;
                ch.inputs.resize(n_in[k]);
                for (int64_t j = in_off[k]; j < in_off[k + 1]; ++j) ch.inputs[j - in_off[k]] = ins[j] - (int32_t)b;
                tms = std::max(tms, max_slot[k] + 1);
            }
            pg.max_stack = tms;
            pg.n_records = n_rec[t];
            pg.spines.swap(spines[t]);
        });
        if (bad) return set_err(c, GP_EINVAL, "internal error: inconsistent chunk graph");
        for (int64_t t = 0; t < n_trees; ++t)
            if ((*progs_out)[t].max_stack > compile_stack_slots())
                return set_err(c, GP_EINVAL, "internal error: stack bound exceeded");
        if (index_min_size > 0) {
            int64_t t = 0;
            for (size_t i = 0; i < big_nodes.size(); ++i) {
                while (big_nodes[i] >= offsets[t + 1]) ++t;
                (*progs_out)[t].big_ends.push_back({(int32_t)(big_nodes[i] - offsets[t]), big_end[i]});
            }
        }
        tr.mark("programs to the host");
        return GP_OK;
    }

    // the population's tables, as assemble_population builds them
    out->vtype = vtype;
    out->n_inputs = n_inputs;
    out->n_trees = n_trees;
    out->chunk_nodes = chunk_nodes;
    out->tree_nodes.resize(n_trees);
    for (int64_t t = 0; t < n_trees; ++t) out->tree_nodes[t] = offsets[t + 1] - offsets[t];
    out->total_nodes = n;
    out->n_chunks = nch;
    out->n_code = n_code;
    out->rec_base = rec_base;
    out->chunk_n_in = n_in;
    out->chunk_tree = ctree;
    out->promo_src.clear();
    out->promo_in.clear();
    out->promo_rows.clear();
    out->chunk_path.clear();
    out->leaves.clear();
    out->spines.clear();
    out->spine_of.clear();
    std::vector<int64_t> out_slot(nch), path(nch, 0);
    {
        int64_t next_slot = n_trees;
        for (int64_t t = 0; t < n_trees; ++t)
            for (int64_t k = cbase[t]; k < cbase[t + 1]; ++k) out_slot[k] = (k == cbase[t + 1] - 1) ? t : next_slot++;
    }
    for (int64_t k = nch - 1; k >= 0; --k) {
        const int64_t last = cbase[ctree[k] + 1] - 1;
        const bool top = k == last;
        if (top != (parent[k] < 0) || (!top && (parent[k] <= k || parent[k] > last)))
            return set_err(c, GP_EINVAL, "internal error: inconsistent chunk graph");
        path[k] = nodes[k] + (top ? 0 : path[parent[k]]);
    }
    // with the subtree index, each tree's chunk list and chunk roots are kept
    // for building children (as assemble_population does)
    const bool keep = index_min_size > 0;
    std::vector<DevChunk> dch(nch);
    std::vector<int32_t> chunk_in((size_t)in_off[nch]), tree_ms(n_trees, 0);
    out->kept_chunks.clear();
    out->kept_max_stack.clear();
    out->cuts.clear();
    if (keep) {
        out->kept_chunks.resize(n_trees);
        out->cuts.resize(n_trees);
    }
    dc_parallel(n_trees, [&](int64_t t) {
        const int64_t b = cbase[t], m = cbase[t + 1] - b, s0 = offsets[t];
        int32_t tms = 0;
        for (int64_t i = 0; i < m; ++i) {
            const int64_t k = b + i;
            DevChunk& d = dch[k];
            d.code_off = code_off[k];
            d.code_len = (int32_t)code_len[k];
            d.parent = parent[k];
            d.out_slot = (int32_t)out_slot[k];
            d.in_off = (int32_t)in_off[k];
            d.rec_base = (int32_t)rec_base[t];
            d.n_in = n_in[k];
            for (int64_t j = in_off[k]; j < in_off[k + 1]; ++j) chunk_in[j] = (int32_t)out_slot[ins[j]];
            tms = std::max(tms, max_slot[k] + 1);
        }
        tree_ms[t] = tms;
        if (!keep) return;
        auto& kc = out->kept_chunks[t];
        kc.resize(m);
        auto& cl = out->cuts[t];
        cl.reserve(m);
        for (int64_t i = 0; i < m; ++i) {
            const int64_t k = b + i;
            Chunk& ch = kc[i];
            ch.code_off = code_off[k];
            ch.code_len = code_len[k];
            ch.parent = parent[k] >= 0 ? parent[k] - (int32_t)b : -1;
            ch.root_node = root[k] - s0;
            ch.nodes = nodes[k];
            ch.path_nodes = path[k];
            ch.end_node = rend[k];
            ch.dev_src = -1;
            ch.stores = stores[k] != 0;
            ch.vec_slot = out_slot[k];
            ch.src_vec = -1;
            ch.inputs.resize(n_in[k]);
            for (int64_t j = in_off[k]; j < in_off[k + 1]; ++j) ch.inputs[j - in_off[k]] = ins[j] - (int32_t)b;
            cl.push_back(Pop::CutSlot{(int32_t)ch.root_node, rend[k], (int32_t)out_slot[k]});
        }
        std::sort(cl.begin(), cl.end(), [](const Pop::CutSlot& x, const Pop::CutSlot& y) { return x.node < y.node; });
    });
    if (keep) out->kept_max_stack = tree_ms;
    for (int64_t k = 0; k < nch; ++k)
        if (n_in[k] == 0) out->leaves.emplace_back(path[k], (int32_t)k);
    std::vector<SpineLvl> levels;
    out->max_stack = 0;
    int64_t n_records = 0;
    for (int64_t t = 0; t < n_trees; ++t) {
        const int32_t tms = tree_ms[t];
        if (tms > compile_stack_slots()) return set_err(c, GP_EINVAL, "internal error: stack bound exceeded");
        out->max_stack = std::max(out->max_stack, tms);
        for (auto& sp : spines[t]) {
            const uint64_t key = ((uint64_t)t << 32) | (uint32_t)sp.point;
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
        n_records += n_rec[t];
    }
    out->n_records = n_records;
    tr.mark("chunk tables and spines");
    if (index_min_size > 0) {
        // the list is sorted by node, so each tree's entries are one range
        out->big_ends.assign(n_trees, {});
        out->big_built.assign(n_trees, 1);
        dc_parallel(n_trees, [&](int64_t t) {
            const auto a = std::lower_bound(big_nodes.begin(), big_nodes.end(), offsets[t]);
            const auto b = std::lower_bound(a, big_nodes.end(), offsets[t + 1]);
            auto& be = out->big_ends[t];
            be.resize(b - a);
            for (auto it = a; it != b; ++it) {
                const size_t i = (size_t)(it - big_nodes.begin());
                be[it - a] = {(int32_t)(big_nodes[i] - offsets[t]), big_end[i]};
            }
        });
    }
    tr.mark("large-subtree lists");
    std::stable_sort(out->leaves.begin(), out->leaves.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                         return x.first > y.first;
                     });
    tr.mark("leaf order");
    RC(up(c, nullptr, out->chunks, dch.data(), dch.size() * sizeof(DevChunk), s));
    RC(up(c, nullptr, out->chunk_in, chunk_in.data(), chunk_in.size() * 4, s));
    RC(up(c, nullptr, out->levels, levels.data(), levels.size() * sizeof(SpineLvl), s));
    HIPC(c, hipStreamSynchronize(s));
    tr.mark("tables to the device");
    return GP_OK;
}

}  // namespace gpe
