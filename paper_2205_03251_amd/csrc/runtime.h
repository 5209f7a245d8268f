// Internal runtime objects of the gpeval library (context, populations,
// case sets, launch plans).  Shared by runtime.hip and server.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <sys/mman.h>

#include <atomic>
#include <cstdlib>
#include <new>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/gpeval.h"
#include "dev.h"
#include "prep.h"

namespace gpe {

struct Ctx;

// Device allocation charged against the context's HBM budget.
struct DevBuf {
    Ctx* ctx = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;       // memory of a DevArena: not freed by release()
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void release();
    void swap(DevBuf& o)
    {
        std::swap(ctx, o.ctx);
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(borrowed, o.borrowed);
    }
    template <class T> T* as() const { return (T*)p; }
};

// Device memory a caller reuses across calls (a server's prep thread
// compiling tree after tree): temporaries are carved from one buffer instead
// of being allocated and freed one by one, since a free waits for the whole
// device and would stall every batch in flight.
struct DevArena {
    DevBuf buf;
    size_t used = 0;             // bytes handed out since the last reset
    size_t high = 0;             // most ever asked for between two resets
};

struct CaseSet {
    int vtype = 0;
    int n_inputs = 0;
    int64_t T = 0;               // test cases
    int64_t n_elems = 0;         // float: T; Boolean: words = ceil(T/64)
    int64_t stride = 0;          // n_elems padded to kPadCases
    int64_t P = 64;              // fitness halving width
    DevBuf inputs;               // [n_inputs][stride]
    DevBuf target;               // [stride]
};

// How a full evaluation is launched: the interpreter variant, and how many of
// its one-wave workgroups may be resident per compute unit (0: as many as
// fit).  Fewer resident waves give the waves on the longest chunk chains more
// of their SIMD's issue slots, which shortens launches bound by those chains.
struct Launch {
    int variant = -1;
    int waves_per_cu = 0;
};

// Launch plan of one population for one launch choice and slicing.
struct Plan {
    int variant = -1;
    int waves_per_cu = 0;
    bool per_tree = false;
    int32_t n_slices = 0;
    int64_t n_items = 0;
    int grid = 0;
    DevBuf items;                // int64 work items
    DevBuf pending_init;         // int32 [n_chunks * n_slices]
    DevBuf pending;
    DevBuf cursor;               // one per tree in per-tree mode
    std::vector<int64_t> tree_item_begin, tree_item_count;
    hipGraphExec_t graph = nullptr;
    gp_handle graph_cases = 0;
    ~Plan();
};

struct SpineInfo {
    int32_t tree;
    int32_t at_point;
    int64_t level_off;
    int32_t n_levels;
    int64_t removed_nodes;
};

// Allocator whose resize leaves new elements uninitialised: large byte
// buffers that are written at once need no zeroing pass first.  Blocks of
// 64 MiB or more are 2 MiB aligned and marked for transparent huge pages, so
// filling gigabytes takes thousands of page faults rather than millions.
template <class T> struct NoInitAlloc : std::allocator<T> {
    template <class U> struct rebind {
        using other = NoInitAlloc<U>;
    };
    static constexpr size_t kHuge = size_t(1) << 21, kLarge = size_t(1) << 26;
    NoInitAlloc() = default;
    template <class U> NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <class U> void construct(U* p) noexcept { ::new ((void*)p) U; }
    template <class U, class... A> void construct(U* p, A&&... a) { ::new ((void*)p) U(std::forward<A>(a)...); }
    T* allocate(size_t n)
    {
        const size_t bytes = n * sizeof(T);
        if (bytes < kLarge) return std::allocator<T>::allocate(n);
        void* p = std::aligned_alloc(kHuge, (bytes + kHuge - 1) & ~(kHuge - 1));
        if (!p) throw std::bad_alloc();
        (void)madvise(p, bytes, MADV_HUGEPAGE);
        return (T*)p;
    }
    void deallocate(T* p, size_t n)
    {
        if (n * sizeof(T) < kLarge) std::allocator<T>::deallocate(p, n);
        else std::free(p);
    }
};

struct Pop {
    int vtype = 0;
    int n_inputs = 0;
    int layout = 0;
    bool auto_chunk = false;                // chunk size may be re-tuned
    bool device_compiled = false;           // compiled on the device (re-chunked there too)
    // host copy of the trees, for re-chunking by the autotuner
    std::vector<uint8_t, NoInitAlloc<uint8_t>> host_ops;
    std::vector<int64_t> host_offsets, host_rec_points, host_rec_offsets;
    int64_t n_trees = 0;
    int64_t total_nodes = 0;
    int64_t chunk_nodes = 0;
    int32_t max_stack = 0;
    int64_t max_code_len = 0;               // longest chunk program, in words
    std::vector<int64_t> tree_nodes;
    // compiled program
    int64_t n_chunks = 0;
    int64_t n_code = 0;
    int64_t n_records = 0;
    std::vector<int64_t> rec_base;          // per tree
    std::vector<int32_t> chunk_n_in;        // per chunk
    std::vector<int32_t> chunk_tree;        // per chunk
    std::vector<std::pair<int64_t, int32_t>> leaves;  // (priority, chunk), sorted
    DevBuf code, chunks, chunk_in;
    // parent caches
    std::unordered_map<uint64_t, int32_t> spine_of;   // (tree, point) -> spine
    std::vector<SpineInfo> spines;
    DevBuf levels;                          // SpineLvl per spine level
    // the trees' bytes in device memory (GP_KEEP_TREES), for building children
    DevBuf tree_ops;                        // load layout, 32 bytes of padding
    std::vector<int64_t> tree_off;          // [n_trees + 1]
    // per tree, the ends of its large subtrees (built on first co-evaluation)
    std::vector<std::vector<SubtreeEnd>> big_ends;
    std::vector<uint8_t> big_built;
    // per tree, its chunk roots sorted by node: after a full evaluation their
    // vectors sit in vecs[slot] (kept with the subtree index)
    struct CutSlot {
        int32_t node, end, slot;
    };
    std::vector<std::vector<CutSlot>> cuts;
    // per tree, its chunks with their code offsets in `code` (populations
    // compiled with the subtree index), for building children from them
    std::vector<std::vector<Chunk>> kept_chunks;
    std::vector<int32_t> kept_max_stack;
    // composed children (assemble_population with reused chunks): per chunk,
    // the vector slot of the chunk it reuses in the population it comes from
    // (-1: compiled anew), and its longest chunk chain to the tree root
    std::vector<int64_t> promo_src;
    std::vector<int32_t> promo_in;          // per chunk: how many of its inputs are reused chunks
    std::vector<int64_t> promo_rows;        // (vector slot, source vector slot) of every reused chunk
    std::vector<int64_t> chunk_path;
    // evaluation state
    int64_t stride = 0;                     // case stride of vecs/recs
    DevBuf vecs;                            // [n_chunks][stride]: roots are slots 0..n_trees-1
    DevBuf recs;                            // [n_records][stride]
    DevBuf fit;                             // [n_trees] double or int64
    gp_handle evaluated_with = 0;           // case set of the last full evaluation
    std::map<std::tuple<int, int, int>, std::unique_ptr<Plan>> plans;  // (variant, waves_per_cu, per_tree)
};

struct TuneKey {
    int vtype, tbucket, sbucket;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(vtype, tbucket, sbucket) < std::tie(o.vtype, o.tbucket, o.sbucket);
    }
};

struct Server;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    int n_cu = 0;
    std::string err;
    std::mutex err_mu;                      // server threads may report errors too
    std::mutex mu;                          // guards handles (server threads share the ctx)
    gp_handle next_handle = 1;
    std::unordered_map<gp_handle, std::shared_ptr<CaseSet>> cases;
    std::unordered_map<gp_handle, std::shared_ptr<Pop>> pops;
    int forced_variant = -1;
    int forced_waves = -1;                  // -1: tuned or all that fit; 0: all that fit; n: at most n per CU
    std::map<TuneKey, Launch> tuned;
    std::map<TuneKey, int64_t> tuned_chunk; // chunk size of each tuned choice
    std::map<TuneKey, bool> tuned_loaded;   // read by gp_tuning_load, not timed in this process
    std::string device_name;                // architecture and compute units, keys saved tuning
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t kev0 = nullptr, kev1 = nullptr;   // around the interpreter launch
    Server* server = nullptr;
    int32_t* ix_scratch = nullptr;          // this device's copy of the index scratch array
};

// ------------------------------------------------------------ internals
int set_err(Ctx* c, int code, const std::string& msg);
int dev_alloc(Ctx* c, DevBuf& b, size_t bytes);
// b = bytes of temporary device memory: from arena a when it is given and has
// room (b then does not own it), else allocated.
int scratch_alloc(Ctx* c, DevArena* a, DevBuf& b, size_t bytes);
// All of the arena's memory is free again (nothing may still use it); it
// grows to the most that was asked for since the last reset.
int arena_reset(Ctx* c, DevArena* a);
int hip_check(Ctx* c, hipError_t e, const char* what);

// Compile and upload a population (prefix or postfix trees) on stream s
// (s synchronised before return).
// index_subtrees: keep each tree's index of large subtrees (prefix layout),
// for co-evaluation.
// ext_rows (prefix layout, may be null): per byte of ops, -1 or the input row
// a terminal stands for (see compile_tree).
int build_population(Ctx* c, int vtype, int layout, int n_inputs, int64_t n_trees,
                     const uint8_t* ops, const int64_t* offsets, const int64_t* rec_points,
                     const int64_t* rec_offsets, int64_t chunk_nodes, Pop* out, hipStream_t s,
                     bool index_subtrees = false, const int32_t* ext_rows = nullptr);
// Assemble already compiled trees into a population and upload it on s.
// Chunks with dev_src >= 0 take their code from dev_code_src (device words).
int assemble_population(Ctx* c, int vtype, int n_inputs, std::vector<TreeProg>& progs,
                        const std::vector<int64_t>& tree_nodes, int64_t chunk_nodes, Pop* out,
                        hipStream_t s, const uint32_t* dev_code_src = nullptr);
// Make sure vecs/recs/fit match the case set; allocate if needed.
int ensure_eval_buffers(Ctx* c, Pop* p, const CaseSet* cs);
// Full evaluation of composed children (p->promo_src filled) whose reused
// chunks take their values from src, the population their code comes from,
// as src's last full evaluation on the same case set left them: those rows
// of src->vecs are copied, and only the chunks compiled anew are evaluated.
// Synchronises s.  n_evaluated (may be null) receives their number.
int enqueue_promoted(Ctx* c, Pop* p, const Pop* src, gp_handle cases_h, const CaseSet* cs, Launch L,
                     hipStream_t s, int64_t* n_evaluated);
// Enqueue a full evaluation on stream s (no copies out, no synchronisation).
// time_kernel: record c->kev0/kev1 around the interpreter launch.
int enqueue_full(Ctx* c, Pop* p, gp_handle cases_h, const CaseSet* cs, Launch L, bool per_tree,
                 bool use_graph, hipStream_t s, int64_t* launches, bool time_kernel = false);
// Build the walk descriptors of an incremental batch and enqueue donor
// evaluation + walk on s.  Outputs are device buffers owned by the caller.
struct IncJob {
    Pop* parent;                 // population holding the mother
    int64_t tree;                // mother's tree index in it
    int64_t point;               // crossover point (caller's layout)
    const uint8_t* donor;        // donor bytes (prefix)
    int64_t donor_len;
};
struct IncOut {
    DevBuf wc, root, fit, stop, interp;
    Pop donors;
    int64_t equiv_nodes = 0;
    std::vector<int64_t> child_nodes;
};
int enqueue_incremental(Ctx* c, const std::vector<IncJob>& jobs, gp_handle cases_h, const CaseSet* cs,
                        bool want_roots, hipStream_t s, IncOut* out, int64_t* launches);
// The same outputs by co-evaluating each child with its mother instead of
// reading parent caches (any crossover point; prefix populations).  Runs its
// rounds synchronously on s; interp receives the nodes actually executed.
int enqueue_coeval(Ctx* c, const std::vector<IncJob>& jobs, gp_handle cases_h, const CaseSet* cs,
                   bool want_roots, hipStream_t s, IncOut* out, int64_t* launches, int64_t* rounds);
// Device tree index (gp_index_trees without the lock) on stream st; waits for
// the result.  device_ms (may be null) uses the context's events: only for
// callers holding the context lock.
int index_trees(Ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler, double* device_ms,
                hipStream_t st, DevArena* arena = nullptr);
// Compile a population of prefix trees on the device (devcompile.hip): the
// same programs and tables as build_population.  dops/doffs: the trees and
// offsets in device memory (dops 16-byte aligned); offsets: host copy;
// host_ops (may be null): host copy, for error messages; record points as
// build_population's, host arrays (prefix indices); key_points (may be null):
// the caller's indices of the same points, for the spine keys.
// index_min_size > 0: index large subtrees and keep each tree's chunk list
// for building children (as build_population with index_subtrees).  The
// result goes to exactly one of out (a population on the device) or
// progs_out (each tree's program in host memory, as compile_tree gives it,
// for assemble_population).  arena (may be null): where temporaries come
// from.  max_blocks > 0 caps the workgroups of its persistent kernels (a
// compilation that shares the device with running work).  Runs on stream s
// (any thread; it does not use the context stream or events) and waits for it.
int device_compile_population(Ctx* c, int vtype, int n_inputs, int64_t n_trees, const uint8_t* dops,
                              const int64_t* doffs, const int64_t* offsets, const uint8_t* host_ops,
                              const int64_t* rec_points, const int64_t* rec_offsets, const int64_t* key_points,
                              int64_t chunk_nodes, int64_t index_min_size, Pop* out,
                              std::vector<TreeProg>* progs_out, DevArena* arena, hipStream_t s, int max_blocks = 0);
// build_population on the device for prefix trees given in host memory
// (host_ops) or device memory (dev_ops); offsets in host memory.  When
// ops_keep is given, it receives a device copy of the trees (32 bytes of
// padding) for the population's tree_ops.
int build_population_device(Ctx* c, int vtype, int n_inputs, int64_t n_trees, const uint8_t* host_ops,
                            const uint8_t* dev_ops, const int64_t* offsets, const int64_t* rec_points,
                            const int64_t* rec_offsets, int64_t chunk_nodes, Pop* out, DevBuf* ops_keep);
// The launch for a full evaluation of p on cs: the forced variant, else the
// tuned one for this value type and size buckets, else a default (variant -1
// when none fits); the forced width, else the tuned one, else all that fit.
Launch choose_launch(Ctx* c, int vtype, const CaseSet* cs, const Pop* p);
// Workgroups of one launch of variant v: the resident ones, at most
// waves_per_cu per compute unit when that is positive.
int64_t resident_grid(const Ctx* c, const Variant& v, int waves_per_cu);
int64_t auto_chunk_nodes(int vtype, int64_t total_nodes, int64_t n_trees, int64_t T);
int compile_stack_slots();

}  // namespace gpe
