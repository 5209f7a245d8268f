// Device-visible structures and kernel launchers of the gpeval library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gpe {

// Test cases are processed in slices of 64 lanes x K cases; vectors are
// stored with a stride padded to a multiple of kPadCases.
constexpr int kWave = 64;
constexpr int kMaxK = 8;
constexpr int64_t kPadCases = kWave * kMaxK;

struct DevChunk {            // 32 bytes
    int64_t code_off;        // first instruction (global)
    int32_t code_len;
    int32_t parent;          // global chunk id, -1 for a tree's root chunk
    int32_t out_slot;        // vector slot receiving this chunk's value
    int32_t in_off;          // chunk_in[in_off + k] = vector slot read by LOAD k
    int32_t rec_base;        // global record slot of this tree's record 0
    int32_t n_in;            // LOAD inputs: chunk_in[in_off .. in_off + n_in)
};

// Work item = (chunk << 16) | slice.
struct EvalParams {
    const uint32_t* code;
    const DevChunk* chunks;
    const int32_t* chunk_in;
    const int64_t* items;        // leaf work items in priority order
    int64_t n_items;
    int32_t* pending;            // [n_chunks][n_slices] unfinished inputs
    unsigned int* cursor;        // next item to hand out
    const void* inputs;          // [n_inputs][stride]
    void* vecs;                  // [n_slots][stride] chunk and root values
    void* recs;                  // [n_records][stride] parent caches
    int64_t stride;              // padded cases (float) or words (Boolean)
    int32_t n_slices;
    int32_t n_inputs;
};

// One incremental child.  Pointers refer to the mother's population, so one
// launch may walk children of different populations.
struct SpineLvl {
    int32_t fside, sib, par, pad;   // see SpineLevel in prep.h
};

struct WalkChild {
    const SpineLvl* levels;      // the spine's ancestor levels, nearest first
    const void* recs;            // the mother's record slot 0
    const void* parent_vec;      // the mother's root vector
    const void* parent_fit;      // the mother's fitness (double or int64)
    int32_t n_levels;
    int32_t at_point;            // mother's vector at the point (source code)
    int32_t donor_slot;          // donor's root vector slot in the donor run
    int32_t pad;
    int64_t donor_nodes;
};

struct WalkParams {
    const WalkChild* children;
    const void* inputs;          // [n_inputs][stride]
    const void* donor_vecs;      // donor root vectors
    const void* target;          // [stride]
    void* root_out;              // [n_children][stride] or null
    void* fit_out;               // [n_children]
    int32_t* stop_out;           // [n_children]
    int64_t* interp_out;         // [n_children]
    int64_t stride;
    int64_t n_valid;             // T (float) or T bits (Boolean)
    int64_t P;                   // fitness halving width (float)
};

// Co-evaluation of child and mother without parent caches (Section 6.2):
// per level the ancestor's function, the side of the path operand and the
// sibling subtree's vector, evaluated on demand.
struct CoLevel {
    const void* sib;
    int32_t fside;               // f | 4 when the path operand is the right one
    int32_t pad;
};

struct CoChild {
    const void* v_in;            // child's running vector (first round: the donor's)
    const void* m_in;            // mother's running vector (first round: the removed subtree's)
    void* v_out;                 // running vectors kept for the next round
    void* m_out;
    const CoLevel* levels;       // this round's levels, nearest the point first
    const void* parent_vec;      // the mother's root vector
    const void* parent_fit;      // the mother's fitness (double or int64)
    int32_t n_levels;
    int32_t level_base;          // levels walked in earlier rounds
    int32_t check0;              // compare v_in with m_in first (level 0)
    int32_t last;                // this round's levels end at the root
    int32_t out_slot;            // the child's index in the outputs
    int32_t pad;
};

struct CoParams {
    const CoChild* children;
    const void* target;          // [stride]
    void* root_out;              // [n_children][stride] or null
    void* fit_out;               // [n_children]
    int32_t* stop_out;           // [n_children]: stop level, -1 root reached, -2 walk goes on
    int64_t stride;
    int64_t n_valid;             // T (float) or T bits (Boolean)
    int64_t P;                   // fitness halving width (float)
};

struct FitParams {
    const void* vecs;            // [n][stride]
    int64_t first_slot;
    const void* target;
    void* fit_out;
    int64_t stride;
    int64_t n_valid;             // T
    int64_t P;
};

// ----------------------------------------------------------- launchers
// One piece of a child under construction: len bytes from src to
// out + dst.  Pieces of one segment meet at 16-byte aligned output offsets.
struct SpliceItem {
    const uint8_t* src;
    int64_t dst;
    int64_t len;
};

struct Variant {
    const char* name;
    int vtype;                   // 0 float32, 1 Boolean
    int K;                       // cases (words) per lane
    int S;                       // register-stack slots
    const void* kernel;          // for occupancy queries
    int max_blocks_per_cu;       // filled at context creation
    int table;                   // runs the generated table-dispatch loop
    int max_inputs;              // input rows held in registers (0: any count, staged in LDS)
    int max_elems;               // > 0: at most this many case words (Boolean) or cases (float)
};

// Whether variant v can run a population of value type vtype whose programs
// need max_stack slots, on n_inputs input rows of stride elements of esz bytes
// (the table loops address a row with a 32-bit byte stride).
inline bool variant_fits(const Variant& v, int vtype, int max_stack, int n_inputs, int64_t n_elems,
                         int64_t stride, int esz)
{
    if (v.vtype != vtype || v.S < max_stack) return false;
    if (v.max_elems > 0 && n_elems > v.max_elems) return false;
    if (v.max_inputs > 0 && n_inputs > v.max_inputs) return false;
    if (v.table && stride * esz > (int64_t)0xffffffffLL) return false;
    return true;
}

// Bytes of dynamic LDS a launch of v takes for n_inputs input rows.
inline size_t variant_lds(const Variant& v, int n_inputs)
{
    return v.vtype == 1 && v.max_inputs == 0 ? (size_t)n_inputs * kWave * v.K * sizeof(uint64_t) : 0;
}

int variant_count();
Variant* variant_table();

hipError_t launch_init(int32_t* pending, const int32_t* init, int64_t n, unsigned int* cursor,
                       int n_cursors, hipStream_t s);
hipError_t launch_eval(int variant, const EvalParams& p, int grid, hipStream_t s);
hipError_t launch_fitness(int vtype, const FitParams& p, int64_t n, hipStream_t s);
hipError_t launch_walk(int vtype, const WalkParams& p, int64_t n_children, hipStream_t s);
hipError_t launch_splice(const SpliceItem* items, int64_t n_items, uint8_t* out, hipStream_t s);

// Device-side tree index (index.hip).  E(k), the sum of node steps before
// position k, is held as el[k] + boff[k / kIxBlock].
constexpr int kIxBlock = 4096;          // positions per scan block
constexpr int kIxFan = 16;              // min-tree fan-out
constexpr int kIxMaxLevels = 16;        // min-tree levels (16^15 positions)

struct IxParams {
    const uint8_t* ops;                 // 16-byte aligned
    const int64_t* offsets;             // [n_trees + 1]
    int64_t n_trees;
    int64_t n;                          // positions in all
    int n_inputs;
    int top;                            // highest min-tree level (at most kIxFan entries)
    int16_t* el;                        // [n_blocks * kIxBlock + kIxFan], within-block values (|x| <= kIxBlock)
    int32_t* boff;                      // [n_blocks + 1]
    int32_t* seg;                       // min-tree levels 1..top, each padded to whole groups
    int64_t lvl[2 * kIxMaxLevels];      // offset in seg and length of each level; level 0 = E, length n + 1
    int32_t* valid;                     // [n_trees]
    int32_t* end;                       // [n], tree-local
    int32_t* parent;                    // [n], tree-local, -1 at a root
    uint8_t* sn;                        // [n] Strahler numbers (0 in invalid trees), or null
    uint8_t* bempty;                    // [n_blocks + 1]: the Strahler pass marked nothing in the block
    int32_t* bad_offsets;               // set to 1 when offsets are not 0..n, non-decreasing
};

hipError_t launch_index(const IxParams& q, int32_t* bsum, int64_t n_blocks, const int64_t* host_len,
                        hipStream_t s);
// dst[0 .. n) = v, by a kernel (no memset node in a captured stream).
hipError_t launch_fill_u8(uint8_t* dst, int64_t n, uint8_t v, hipStream_t s);

// Scratch of the allocation-free tree index (gp_index_trees_noalloc): a
// file-scope device array of kIxStaticWords int32 words in index.hip, enough
// for populations of up to kIxStaticMaxNodes nodes.  Regions, each starting
// on a 256-byte boundary: el, boff, bsum, seg, flags (4 words), bempty.
constexpr int64_t kIxStaticMaxNodes = int64_t(1) << 22;
constexpr int64_t ix_round64(int64_t w) { return (w + 63) / 64 * 64; }
constexpr int64_t ix_seg_words(int64_t n)
{
    int64_t len = n + 1, total = 0;
    while (len > kIxFan) {
        len = (len + kIxFan - 1) / kIxFan;
        total += (len + kIxFan - 1) / kIxFan * kIxFan;
    }
    return total + kIxFan;
}
constexpr int64_t kIxStaticBlocks = (kIxStaticMaxNodes + kIxBlock - 1) / kIxBlock;
constexpr int64_t kIxStaticEl = 0;
constexpr int64_t kIxStaticBoff = kIxStaticEl + ix_round64(kIxStaticBlocks * kIxBlock + kIxFan);
constexpr int64_t kIxStaticBsum = kIxStaticBoff + ix_round64(kIxStaticBlocks + 1);
constexpr int64_t kIxStaticSeg = kIxStaticBsum + ix_round64(kIxStaticBlocks);
constexpr int64_t kIxStaticFlag = kIxStaticSeg + ix_round64(ix_seg_words(kIxStaticMaxNodes));
constexpr int64_t kIxStaticBempty = kIxStaticFlag + 64;
constexpr int64_t kIxStaticWords = kIxStaticBempty + ix_round64((kIxStaticBlocks + 1 + 3) / 4);
// The device address of that array on the current device (device, which
// must be current), looked up once per device; hipSuccess or the lookup's
// error.
hipError_t ix_static_scratch(int device, int32_t** out);
// 1 at a terminal and 2 at a function of a valid tree (every function has two children of at least 1), 0 else.
hipError_t launch_strahler_init(const IxParams& q, hipStream_t s);
// One level: raises to level + 1 every node with a function below it whose children are both at level or
// more; sets *any when there is such a function.  Reuses el and boff.
// Pass `level` of the Strahler numbers; afterwards boff[n_blocks] holds the
// number of functions it marked (none: the numbers are final).
hipError_t launch_strahler_level(const IxParams& q, int level, int32_t* bsum, int64_t n_blocks, hipStream_t s);
hipError_t launch_coeval(int vtype, const CoParams& p, int64_t n_children, hipStream_t s);
// One generation's random choices (Section 6.3): per slot i, the winners of
// tournaments (i, g, 0) and (i, g, 1) over fit, the crossover point in the
// mother and the donor node in the father.
struct SelectParams {
    const void* fit;             // [n] double (lower wins, NaN worst) or int64 (higher wins)
    const int64_t* sizes;        // [n] nodes of each slot's tree (0: not built)
    int64_t n;
    int32_t k;                   // tournament size
    int32_t boolean;
    uint64_t seed;
    int64_t generation;
    int64_t* mother;             // [n] outputs
    int64_t* father;
    int64_t* point;
    int64_t* donor_node;
};
// Fitness first: the tournaments of generation g over the children's fitness,
// counting how often each child is drawn as a parent.
struct MarkParams {
    const void* fit;
    int64_t n;
    int32_t k;
    int32_t boolean;
    uint64_t seed;
    int64_t generation;
    int32_t* drawn;              // [n], zeroed by the caller's fill kernel
};

hipError_t launch_select(const SelectParams& p, hipStream_t s);
hipError_t launch_mark(const MarkParams& p, hipStream_t s);
hipError_t launch_fill_i32(int32_t* dst, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_gather_rows(const void* src, const int64_t* src_rows, int64_t n_rows, int64_t row_bytes, void* dst,
                              hipStream_t s);
// Counter calibration: n_waves single-wave workgroups, each running iters x 32
// VALU instructions of class cls (see k_valu_cal); out: n_waves * 64 floats.
hipError_t launch_valu_cal(int cls, int64_t n_waves, int64_t iters, float* out, hipStream_t s);
// Row rows[2k] of dst = row rows[2k + 1] of src, k < n_rows (rows of row_bytes, a multiple of 16).
hipError_t launch_move_rows(const void* src, const int64_t* rows, int64_t n_rows, int64_t row_bytes, void* dst,
                            hipStream_t s);

}  // namespace gpe
