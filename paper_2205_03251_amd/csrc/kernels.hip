// HIP kernels of the gpeval library (gfx950).
//
// Interpreter (Section 4.2 of the paper: every opcode runs on every test
// case).  Test cases lie across the 64 lanes of a wavefront, K per lane, so
// one instruction word drives 64*K case evaluations.  The instruction stream
// is wave-uniform: it is fetched through the scalar cache and decoded on the
// scalar unit, and every handler works on a register-resident evaluation
// stack st[S][K] at a slot fixed by the instruction, so no register is ever
// indexed at run time.  The host compiler (prep.cpp) orders evaluation so
// that S slots suffice and folds terminal operands into their parent's
// instruction.
//
// Batching: one persistent launch evaluates a whole population.  Each
// wavefront repeatedly takes a work item (a leaf chunk of some tree, on one
// slice of test cases) from an atomic cursor over a list sorted by longest
// remaining chain first, evaluates it, publishes the chunk's value vector,
// and decrements its parent chunk's counter; the wavefront that brings the
// counter to zero goes on to evaluate the parent.  No wavefront ever waits
// on another, so the launch always drains.
//
// Incremental evaluation (Section 6.2, Figure 3): one workgroup per child
// walks from the crossover point to the root over the mother's recorded
// vectors, comparing with the mother at each level and stopping at the first
// level where all test cases agree.
#include <algorithm>

#include "dev.h"
#include "prep.h"

namespace gpe {

#define UNROLL _Pragma("unroll")

// Read-only tables (instruction words, chunk descriptors, work items, input
// lists, spine levels) are read through the constant address space: uniform
// reads then go through the scalar data cache into SGPRs.
#define GP_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const GP_CONST T* cst(const T* p)
{
    return (const GP_CONST T*)p;
}

// ---------------------------------------------------------------- ops
template <int F>
__device__ __forceinline__ float fop(float a, float b)
{
    if constexpr (F == 0) return a + b;
    else if constexpr (F == 1) return a - b;
    else if constexpr (F == 2) return a * b;
    else {
        const float q = a / b;                 // IEEE correctly rounded
        return (fabsf(b) < 1e-6f) ? 1.0f : q;  // protected divide
    }
}

__device__ __forceinline__ float fop_rt(int f, float a, float b)
{
    switch (f) {
    case 0: return fop<0>(a, b);
    case 1: return fop<1>(a, b);
    case 2: return fop<2>(a, b);
    default: return fop<3>(a, b);
    }
}

template <int F>
__device__ __forceinline__ uint64_t bop(uint64_t a, uint64_t b)
{
    if constexpr (F == 0) return a & b;
    else if constexpr (F == 1) return a | b;
    else if constexpr (F == 2) return ~(a & b);
    else return ~(a | b);
}

__device__ __forceinline__ uint64_t bop_rt(int f, uint64_t a, uint64_t b)
{
    switch (f) {
    case 0: return bop<0>(a, b);
    case 1: return bop<1>(a, b);
    case 2: return bop<2>(a, b);
    default: return bop<3>(a, b);
    }
}

// Bit-equal, or both NaN.
__device__ __forceinline__ bool same_f32(float a, float b)
{
    return (__float_as_uint(a) == __float_as_uint(b)) || (a != a && b != b);
}

__device__ __forceinline__ uint64_t valid_bits(int64_t w, int64_t T)
{
    const int64_t lo = w * 64;
    if (lo + 64 <= T) return ~0ull;
    if (lo >= T) return 0ull;
    return (1ull << (T - lo)) - 1ull;
}

struct ChunkHdr {
    int64_t code_off;
    int32_t code_len, parent, out_slot, in_off, rec_base, n_in;
};

__device__ __forceinline__ ChunkHdr load_chunk(const GP_CONST DevChunk* c)
{
    ChunkHdr h;
    h.code_off = c->code_off;
    h.code_len = c->code_len;
    h.parent = c->parent;
    h.out_slot = c->out_slot;
    h.in_off = c->in_off;
    h.rec_base = c->rec_base;
    h.n_in = c->n_in;
    return h;
}

// --------------------------------------------------- float interpreter
struct ItemF32 {
    const float* inputs;     // input 0 at this lane's first case
    const float* vecs;       // vector slot 0 at this lane's first case
    float* recs;             // record slot 0 at this lane's first case
    const GP_CONST int32_t* chunk_in;
    int64_t stride;
    int32_t rec_base;
};

template <int D, int K, int S>
__device__ __forceinline__ void step_f32(uint32_t fm, uint32_t pl, float (&st)[S][K],
                                         const float (&x)[K], const ItemF32& c)
{
    if constexpr (D < S) {
        switch (fm) {
#define GP_F32_CASES(F)                                                                       \
    case (F) | (M_XX << 2):                                                                   \
        UNROLL for (int k = 0; k < K; ++k) st[D][k] = fop<F>(x[k], x[k]);                     \
        break;                                                                                \
    case (F) | (M_XS << 2):                                                                   \
        UNROLL for (int k = 0; k < K; ++k) st[D][k] = fop<F>(x[k], st[D][k]);                 \
        break;                                                                                \
    case (F) | (M_SX << 2):                                                                   \
        UNROLL for (int k = 0; k < K; ++k) st[D][k] = fop<F>(st[D][k], x[k]);                 \
        break;                                                                                \
    case (F) | (M_SS << 2):                                                                   \
        if constexpr (D + 1 < S) {                                                            \
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = fop<F>(st[D][k], st[D + 1][k]);     \
        }                                                                                     \
        break;                                                                                \
    case (F) | (M_RS << 2):                                                                   \
        if constexpr (D + 1 < S) {                                                            \
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = fop<F>(st[D + 1][k], st[D][k]);     \
        }                                                                                     \
        break;
            GP_F32_CASES(0)
            GP_F32_CASES(1)
            GP_F32_CASES(2)
            GP_F32_CASES(3)
#undef GP_F32_CASES
        case (M_PUSH << 2):
            if (pl == 0) {
                UNROLL for (int k = 0; k < K; ++k) st[D][k] = x[k];
            } else {
                const float* src = c.inputs + (int64_t)pl * c.stride;
                UNROLL for (int k = 0; k < K; ++k) st[D][k] = src[kWave * k];
            }
            break;
        case (M_LOAD << 2): {
            const float* src = c.vecs + (int64_t)c.chunk_in[pl] * c.stride;
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = src[kWave * k];
            break;
        }
        case (M_STORE << 2): {
            float* dst = c.recs + (int64_t)(c.rec_base + (int32_t)pl) * c.stride;
            UNROLL for (int k = 0; k < K; ++k) dst[kWave * k] = st[D][k];
            break;
        }
        default:
            break;
        }
    }
}

#define GP_DEPTH_CASES(STEP)                                                                  \
    STEP(0) STEP(1) STEP(2) STEP(3) STEP(4) STEP(5) STEP(6) STEP(7) STEP(8) STEP(9) STEP(10)  \
    STEP(11) STEP(12) STEP(13) STEP(14) STEP(15) STEP(16) STEP(17) STEP(18) STEP(19)          \
    STEP(20) STEP(21) STEP(22) STEP(23) STEP(24) STEP(25) STEP(26) STEP(27) STEP(28)          \
    STEP(29) STEP(30) STEP(31)

template <int K, int S>
__device__ __forceinline__ void run_f32(const GP_CONST uint32_t* code, int32_t len,
                                        float (&st)[S][K], const float (&x)[K], const ItemF32& c)
{
    // The next word is fetched before the current one is executed; the code
    // array carries one padding word past its end.
    uint32_t nxt = code[0];
    // Settle the first fetch before the loop (0xffffffff is no valid word),
    // so that inside it only the loop latch waits, for the word fetched
    // while the current handler ran.
    if (nxt == 0xffffffffu) len = 0;
    for (int32_t i = 0; i < len; ++i) {
        const uint32_t ins = __builtin_amdgcn_readfirstlane(nxt);
        nxt = code[i + 1];
        const uint32_t fm = ins & 31u;
        const uint32_t pl = ins >> kPayloadShift;
        switch ((ins >> 5) & 31u) {
#define GP_STEP(D)                                     \
    case D:                                            \
        step_f32<D, K, S>(fm, pl, st, x, c);           \
        break;
            GP_DEPTH_CASES(GP_STEP)
#undef GP_STEP
        }
    }
}

template <int K, int S>
__global__ __launch_bounds__(64) void k_eval_f32(EvalParams p)
{
    const int lane = threadIdx.x;
    float st[S][K];
    float x[K];
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(p.cursor, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((int64_t)it >= p.n_items) break;
        const int64_t item = cst(p.items)[it];
        int32_t c = (int32_t)(item >> 16);
        const int32_t s = (int32_t)(item & 0xffff);
        const int64_t case0 = (int64_t)s * (kWave * K) + lane;
        const float* xin = (const float*)p.inputs + case0;
        UNROLL for (int k = 0; k < K; ++k) x[k] = xin[kWave * k];
        ItemF32 ic;
        ic.inputs = xin;
        ic.vecs = (const float*)p.vecs + case0;
        ic.recs = (float*)p.recs + case0;
        ic.stride = p.stride;
        for (;;) {
            const GP_CONST DevChunk* chp = cst(p.chunks) + c;
            const ChunkHdr ch = load_chunk(chp);
            ic.chunk_in = cst(p.chunk_in) + ch.in_off;
            ic.rec_base = ch.rec_base;
            run_f32<K, S>(cst(p.code) + ch.code_off, ch.code_len, st, x, ic);
            float* dst = (float*)p.vecs + (int64_t)ch.out_slot * p.stride + case0;
            UNROLL for (int k = 0; k < K; ++k) dst[kWave * k] = st[0][k];
            if (ch.parent < 0) break;
            // Publish this chunk's vector, then count it against the parent;
            // whoever finishes the parent's last input evaluates the parent.
            int old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(p.pending + (int64_t)ch.parent * p.n_slices + s, -1,
                                             __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old != 1) break;
            c = ch.parent;
        }
    }
}

// -------------------------------- float interpreter, table dispatch
// Same work items, chunk hand-off and memory layout as k_eval_f32; the
// chunk's program runs in the generated dispatch loop (gen_dispatch.py),
// which chooses each handler through a branch table.
#include "dispatch_f32.inc"

template <int K, int S, bool DIRECT>
__device__ __forceinline__ void run_f32_dispatch(const GP_CONST uint32_t* code, const float* inb, const float* vb,
                                                 float* rb, const GP_CONST int32_t* cin, uint32_t strideb,
                                                 float* outb, uint32_t voff, uint32_t code_len)
{
    // lane l touches the code lines at words 16 l + 1024 i, i < 4 (clamped to the chunk's last word)
    const uint32_t last = code_len > 0 ? code_len - 1 : 0, l16 = (voff / 4u) * 16u;
    const uint32_t vc0 = min(l16, last) * 4u, vc1 = min(l16 + 1024u, last) * 4u;
    const uint32_t vc2 = min(l16 + 2048u, last) * 4u, vc3 = min(l16 + 3072u, last) * 4u;
    if constexpr (K == 4 && S == 10 && !DIRECT)
        run_f32_dispatch_4_10(code, inb, vb, rb, cin, strideb, outb, voff, vc0, vc1, vc2, vc3);
    else if constexpr (K == 8 && S == 10 && !DIRECT)
        run_f32_dispatch_8_10(code, inb, vb, rb, cin, strideb, outb, voff, vc0, vc1, vc2, vc3);
    else if constexpr (K == 4 && S == 10 && DIRECT)
        run_f32d_dispatch_4_10(code, inb, vb, rb, cin, strideb, outb, voff, vc0, vc1, vc2, vc3);
    else if constexpr (K == 8 && S == 10 && DIRECT)
        run_f32d_dispatch_8_10(code, inb, vb, rb, cin, strideb, outb, voff, vc0, vc1, vc2, vc3);
    else static_assert(K == 4 && S == 10, "no generated dispatch loop for this K and S");
}

// DIRECT: the loop that dispatches into handler slots (see gen_dispatch.py).
template <int K, int S, bool DIRECT = false>
__global__ __launch_bounds__(64) void k_eval_f32_tbl(EvalParams p)
{
    const int lane = threadIdx.x;
    const uint32_t voff = (uint32_t)lane * 4u;
    const uint32_t strideb = (uint32_t)(p.stride * 4);
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(p.cursor, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((int64_t)it >= p.n_items) break;
        const int64_t item = cst(p.items)[it];
        int32_t c = (int32_t)(item >> 16);
        const int32_t s = (int32_t)(item & 0xffff);
        const int64_t case0 = (int64_t)s * (kWave * K);
        const float* inb = (const float*)p.inputs + case0;
        const float* vb = (const float*)p.vecs + case0;
        ChunkHdr ch = load_chunk(cst(p.chunks) + c);
        for (;;) {
            // the parent's header is fetched with this chunk's, so continuing
            // into the parent waits for no load
            ChunkHdr next = ch;
            if (ch.parent >= 0) next = load_chunk(cst(p.chunks) + ch.parent);
            float* rb = (float*)p.recs + (int64_t)ch.rec_base * p.stride + case0;
            float* outb = (float*)p.vecs + (int64_t)ch.out_slot * p.stride + case0;
            run_f32_dispatch<K, S, DIRECT>(cst(p.code) + ch.code_off, inb, vb, rb, cst(p.chunk_in) + ch.in_off,
                                           strideb, outb, voff, (uint32_t)ch.code_len);
            if (ch.parent < 0) break;
            // The loop wrote the chunk's vector with agent-coherent stores and
            // waited for them to complete, and LOAD reads vectors with
            // agent-coherent loads, so the hand-off needs no cache write-back
            // or invalidation: a relaxed decrement orders it.
            int old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(p.pending + (int64_t)ch.parent * p.n_slices + s, -1,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old != 1) break;
            c = ch.parent;
            ch = next;
        }
    }
}

// ------------------------------------------------- Boolean interpreter
struct ItemBool {
    const uint64_t* lin;     // staged input words in LDS, this lane's first word
    const uint64_t* vecs;
    uint64_t* recs;
    const GP_CONST int32_t* chunk_in;
    int64_t stride;
    int32_t rec_base;
    int32_t lds_row;         // words per staged input row (64*K)
};

template <int D, int K, int S>
__device__ __forceinline__ void step_bool(uint32_t fm, uint32_t pl, uint64_t (&st)[S][K],
                                          const ItemBool& c)
{
    if constexpr (D < S) {
        switch (fm) {
#define GP_BOOL_CASES(F)                                                                      \
    case (F) | (M_XX << 2): {                                                                 \
        const uint64_t* a = c.lin + (int32_t)(pl & 2047u) * c.lds_row;                        \
        const uint64_t* b = c.lin + (int32_t)(pl >> 11) * c.lds_row;                          \
        UNROLL for (int k = 0; k < K; ++k) st[D][k] = bop<F>(a[kWave * k], b[kWave * k]);     \
        break;                                                                                \
    }                                                                                         \
    case (F) | (M_XS << 2): {                                                                 \
        const uint64_t* a = c.lin + (int32_t)pl * c.lds_row;                                  \
        UNROLL for (int k = 0; k < K; ++k) st[D][k] = bop<F>(a[kWave * k], st[D][k]);         \
        break;                                                                                \
    }                                                                                         \
    case (F) | (M_SS << 2):                                                                   \
        if constexpr (D + 1 < S) {                                                            \
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = bop<F>(st[D][k], st[D + 1][k]);     \
        }                                                                                     \
        break;
            GP_BOOL_CASES(0)
            GP_BOOL_CASES(1)
            GP_BOOL_CASES(2)
            GP_BOOL_CASES(3)
#undef GP_BOOL_CASES
        case (M_PUSH << 2): {
            const uint64_t* a = c.lin + (int32_t)pl * c.lds_row;
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = a[kWave * k];
            break;
        }
        case (M_LOAD << 2): {
            const uint64_t* src = c.vecs + (int64_t)c.chunk_in[pl] * c.stride;
            UNROLL for (int k = 0; k < K; ++k) st[D][k] = src[kWave * k];
            break;
        }
        case (M_STORE << 2): {
            uint64_t* dst = c.recs + (int64_t)(c.rec_base + (int32_t)pl) * c.stride;
            UNROLL for (int k = 0; k < K; ++k) dst[kWave * k] = st[D][k];
            break;
        }
        default:
            break;
        }
    }
}

template <int K, int S>
__device__ __forceinline__ void run_bool(const GP_CONST uint32_t* code, int32_t len,
                                         uint64_t (&st)[S][K], const ItemBool& c)
{
    uint32_t nxt = code[0];
    if (nxt == 0xffffffffu) len = 0;      // settle the first fetch, as in run_f32
    for (int32_t i = 0; i < len; ++i) {
        const uint32_t ins = __builtin_amdgcn_readfirstlane(nxt);
        nxt = code[i + 1];
        const uint32_t fm = ins & 31u;
        const uint32_t pl = ins >> kPayloadShift;
        switch ((ins >> 5) & 31u) {
#define GP_STEP(D)                                 \
    case D:                                        \
        step_bool<D, K, S>(fm, pl, st, c);         \
        break;
            GP_DEPTH_CASES(GP_STEP)
#undef GP_STEP
        }
    }
}

template <int K, int S>
__global__ __launch_bounds__(64) void k_eval_bool(EvalParams p)
{
    extern __shared__ uint64_t lds_in[];       // [n_inputs][64*K] input words of the slice
    const int lane = threadIdx.x;
    uint64_t st[S][K];
    const int32_t row = kWave * K;
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(p.cursor, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((int64_t)it >= p.n_items) break;
        const int64_t item = cst(p.items)[it];
        int32_t c = (int32_t)(item >> 16);
        const int32_t s = (int32_t)(item & 0xffff);
        const int64_t case0 = (int64_t)s * row + lane;
        __syncthreads();                       // previous item's reads are done
        for (int j = 0; j < p.n_inputs; ++j) {
            const uint64_t* src = (const uint64_t*)p.inputs + (int64_t)j * p.stride + case0;
            UNROLL for (int k = 0; k < K; ++k) lds_in[j * row + kWave * k + lane] = src[kWave * k];
        }
        __syncthreads();
        ItemBool ic;
        ic.lin = lds_in + lane;
        ic.vecs = (const uint64_t*)p.vecs + case0;
        ic.recs = (uint64_t*)p.recs + case0;
        ic.stride = p.stride;
        ic.lds_row = row;
        for (;;) {
            const GP_CONST DevChunk* chp = cst(p.chunks) + c;
            const ChunkHdr ch = load_chunk(chp);
            ic.chunk_in = cst(p.chunk_in) + ch.in_off;
            ic.rec_base = ch.rec_base;
            run_bool<K, S>(cst(p.code) + ch.code_off, ch.code_len, st, ic);
            uint64_t* dst = (uint64_t*)p.vecs + (int64_t)ch.out_slot * p.stride + case0;
            UNROLL for (int k = 0; k < K; ++k) dst[kWave * k] = st[0][k];
            if (ch.parent < 0) break;
            int old = 0;
            if (lane == 0)
                old = __hip_atomic_fetch_add(p.pending + (int64_t)ch.parent * p.n_slices + s, -1,
                                             __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old != 1) break;
            c = ch.parent;
        }
    }
}

// ------------------------------ Boolean interpreter, table dispatch
// Same work items and chunk hand-off as k_eval_bool.  The generated loop
// (gen_dispatch.py) loads the slice's input words, at most kBoolRegInputs
// rows, and the vectors of the chunk's first LOAD inputs into registers when
// a chunk starts and reads them by index in GPR index mode, so no LDS is
// staged and no barrier is taken.
#include "dispatch_bool.inc"

constexpr int kBoolRegInputs = kBoolDispatchInputs;

template <int K, int S>
__device__ __forceinline__ void run_bool_dispatch(const GP_CONST uint32_t* code, const uint64_t* inb,
                                                  const uint64_t* vb, uint64_t* rb, const GP_CONST int32_t* cin,
                                                  uint32_t strideb, uint64_t* outb, uint32_t voff, uint32_t nin,
                                                  uint32_t nload, uint32_t vcoff)
{
    if constexpr (K == 1 && S == 10)
        run_bool_dispatch_1_10(code, inb, vb, rb, cin, strideb, outb, voff, nin, nload, vcoff);
    else if constexpr (K == 2 && S == 10)
        run_bool_dispatch_2_10(code, inb, vb, rb, cin, strideb, outb, voff, nin, nload, vcoff);
    else static_assert(K == 1 && S == 10, "no generated Boolean loop for this K and S");
}

// WORD: the one-word loop (T <= 64: the whole case set in lane 0's word, kept
// in SGPRs), with K = 1.
template <int K, int S, bool WORD = false>
__global__ __launch_bounds__(64) void k_eval_bool_tbl(EvalParams p)
{
    const int lane = threadIdx.x;
    const uint32_t voff = (uint32_t)lane * 8u;
    const uint32_t strideb = (uint32_t)(p.stride * 8);
    const uint32_t nin = (uint32_t)p.n_inputs;
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(p.cursor, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if ((int64_t)it >= p.n_items) break;
        const int64_t item = cst(p.items)[it];
        int32_t c = (int32_t)(item >> 16);
        const int32_t s = (int32_t)(item & 0xffff);
        const int64_t case0 = (int64_t)s * (kWave * K);
        const uint64_t* inb = (const uint64_t*)p.inputs + case0;
        const uint64_t* vb = (const uint64_t*)p.vecs + case0;
        ChunkHdr ch = load_chunk(cst(p.chunks) + c);
        for (;;) {
            ChunkHdr next = ch;          // the parent's header, fetched with this chunk's
            if (ch.parent >= 0) next = load_chunk(cst(p.chunks) + ch.parent);
            uint64_t* rb = (uint64_t*)p.recs + (int64_t)ch.rec_base * p.stride + case0;
            uint64_t* outb = (uint64_t*)p.vecs + (int64_t)ch.out_slot * p.stride + case0;
            // lane l touches the code line at word 16 l (clamped to the chunk's last word)
            const uint32_t vcoff = (uint32_t)min(lane * 16, max(ch.code_len - 1, 0)) * 4u;
            if constexpr (WORD) {
                static_assert(K == 1 && S == 10, "one generated one-word loop: K = 1, S = 10");
                run_boolw_dispatch_10(cst(p.code) + ch.code_off, inb, vb, rb, cst(p.chunk_in) + ch.in_off, strideb,
                                      outb, voff, nin, (uint32_t)ch.n_in, vcoff);
            } else {
                run_bool_dispatch<K, S>(cst(p.code) + ch.code_off, inb, vb, rb, cst(p.chunk_in) + ch.in_off,
                                        strideb, outb, voff, nin, (uint32_t)ch.n_in, vcoff);
            }
            if (ch.parent < 0) break;
            int old = 0;      // relaxed, as in k_eval_f32_tbl
            if (lane == 0)
                old = __hip_atomic_fetch_add(p.pending + (int64_t)ch.parent * p.n_slices + s, -1,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old != 1) break;
            c = ch.parent;
            ch = next;
        }
    }
}

// ------------------------------------------------------------- init
__global__ void k_init(int32_t* pending, const int32_t* init, int64_t n, unsigned int* cursor,
                       int n_cursors)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) pending[i] = init[i];
    if (i0 < n_cursors) cursor[i0] = 0u;
}

// ---------------------------------------------------------- fitness
// Sum of |out - y| in double over P = max(64, 2^ceil(log2 T)) zero-padded
// slots by the halving tree s[i] += s[i + h], h = P/2 ... 1.  Thread t holds
// slots t + 256 m (m < R = max(1, P/256)); the levels h >= 256 pair slots of
// the same thread, the rest go through LDS.
template <int R>
__device__ double halving_sum(double (&e)[R], int64_t P, double* red)
{
    const int tid = threadIdx.x;
    UNROLL for (int r = R / 2; r >= 1; r /= 2)
        UNROLL for (int m = 0; m < r; ++m) e[m] = e[m] + e[m + r];
    const int Pp = P < 256 ? (int)P : 256;
    red[tid] = e[0];
    __syncthreads();
    for (int h = Pp / 2; h >= 1; h >>= 1) {
        if (tid < h) red[tid] = red[tid] + red[tid + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <int R>
__global__ __launch_bounds__(256) void k_fit_f32(FitParams p)
{
    __shared__ double red[256];
    const int64_t row = blockIdx.x;
    const float* v = (const float*)p.vecs + (p.first_slot + row) * p.stride;
    const float* y = (const float*)p.target;
    double e[R];
    UNROLL for (int m = 0; m < R; ++m) {
        const int64_t i = threadIdx.x + 256 * m;
        double val = 0.0;
        if (i < p.n_valid) {
            const float d = v[i] - y[i];
            val = (double)fabsf(d);
        }
        e[m] = val;
    }
    const double f = halving_sum<R>(e, p.P, red);
    if (threadIdx.x == 0) ((double*)p.fit_out)[row] = f;
}

__device__ int64_t block_sum_i64(int64_t v, int64_t* red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    const int64_t r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_fit_bool(FitParams p)
{
    __shared__ int64_t red[256];
    const int64_t row = blockIdx.x;
    const uint64_t* v = (const uint64_t*)p.vecs + (p.first_slot + row) * p.stride;
    const uint64_t* t = (const uint64_t*)p.target;
    const int64_t W = (p.n_valid + 63) / 64;
    int64_t hits = 0;
    for (int64_t w = threadIdx.x; w < W; w += 256)
        hits += __popcll(~(v[w] ^ t[w]) & valid_bits(w, p.n_valid));
    const int64_t h = block_sum_i64(hits, red);
    if (threadIdx.x == 0) ((int64_t*)p.fit_out)[row] = h;
}

// ------------------------------------------------------ incremental walk
// One workgroup of 256 threads per child.  Level 0 compares the donor's
// vector with the mother's vector at the crossover point; level k applies
// the k-th ancestor's function with the path operand replaced by the
// child's running vector and the other operand taken from the mother's
// recorded sibling vector, then compares with the mother's vector at that
// ancestor.  A workgroup-wide AND over the test cases decides the stop.
template <int R>
__global__ __launch_bounds__(256) void k_walk_f32(WalkParams p)
{
    __shared__ double red[256];
    const int64_t ci = blockIdx.x;
    const GP_CONST WalkChild* wcp = cst(p.children) + ci;
    const SpineLvl* levels = wcp->levels;
    const void* w_recs = wcp->recs;
    const void* w_pvec = wcp->parent_vec;
    const void* w_pfit = wcp->parent_fit;
    const int32_t n_levels = wcp->n_levels;
    const int32_t at_point = wcp->at_point;
    const int32_t donor_slot = wcp->donor_slot;
    const int64_t donor_nodes = wcp->donor_nodes;
    const int tid = threadIdx.x;
    const int64_t T = p.n_valid;
    const float* in = (const float*)p.inputs;
    const float* recs = (const float*)w_recs;
    const float* dv = (const float*)p.donor_vecs + (int64_t)donor_slot * p.stride;
    float v[R];
    UNROLL for (int m = 0; m < R; ++m) {
        const int64_t i = tid + 256 * m;
        v[m] = (i < T) ? dv[i] : 0.0f;
    }
    const float* a0 = at_point >= 0 ? recs + (int64_t)at_point * p.stride
                                    : in + (int64_t)(-at_point - 1) * p.stride;
    bool eq = true;
    UNROLL for (int m = 0; m < R; ++m) {
        const int64_t i = tid + 256 * m;
        if (i < T) eq = eq && same_f32(v[m], a0[i]);
    }
    int stop = -1;
    if (__syncthreads_and(eq)) {
        stop = 0;
    } else {
        for (int k = 0; k < n_levels; ++k) {
            const GP_CONST SpineLvl* lp = cst(levels) + k;
            const SpineLvl lv{lp->fside, lp->sib, lp->par, 0};
            const float* sb = lv.sib >= 0 ? recs + (int64_t)lv.sib * p.stride
                                          : in + (int64_t)(-lv.sib - 1) * p.stride;
            const float* pr = recs + (int64_t)lv.par * p.stride;
            const int f = lv.fside & 3;
            const bool right = (lv.fside & 4) != 0;
            eq = true;
            UNROLL for (int m = 0; m < R; ++m) {
                const int64_t i = tid + 256 * m;
                if (i < T) {
                    const float s = sb[i];
                    const float r = right ? fop_rt(f, s, v[m]) : fop_rt(f, v[m], s);
                    v[m] = r;
                    eq = eq && same_f32(r, pr[i]);
                }
            }
            if (__syncthreads_and(eq)) {
                stop = k + 1;
                break;
            }
        }
    }
    if (tid == 0) {
        p.stop_out[ci] = stop;
        p.interp_out[ci] = donor_nodes + (stop >= 0 ? stop : n_levels);
    }
    float* ro = p.root_out ? (float*)p.root_out + ci * p.stride : nullptr;
    if (stop >= 0) {
        // The difference died out: the child's values above the stop are
        // the mother's, and so is its fitness.
        const float* pv = (const float*)w_pvec;
        if (ro)
            for (int64_t i = tid; i < T; i += 256) ro[i] = pv[i];
        if (tid == 0) ((double*)p.fit_out)[ci] = *(const double*)w_pfit;
    } else {
        const float* y = (const float*)p.target;
        double e[R];
        UNROLL for (int m = 0; m < R; ++m) {
            const int64_t i = tid + 256 * m;
            double val = 0.0;
            if (i < T) {
                if (ro) ro[i] = v[m];
                const float d = v[m] - y[i];
                val = (double)fabsf(d);
            }
            e[m] = val;
        }
        const double f = halving_sum<R>(e, p.P, red);
        if (tid == 0) ((double*)p.fit_out)[ci] = f;
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_walk_bool(WalkParams p)
{
    __shared__ int64_t red[256];
    const int64_t ci = blockIdx.x;
    const GP_CONST WalkChild* wcp = cst(p.children) + ci;
    const SpineLvl* levels = wcp->levels;
    const void* w_recs = wcp->recs;
    const void* w_pvec = wcp->parent_vec;
    const void* w_pfit = wcp->parent_fit;
    const int32_t n_levels = wcp->n_levels;
    const int32_t at_point = wcp->at_point;
    const int32_t donor_slot = wcp->donor_slot;
    const int64_t donor_nodes = wcp->donor_nodes;
    const int tid = threadIdx.x;
    const int64_t T = p.n_valid;
    const int64_t W = (T + 63) / 64;
    const uint64_t* in = (const uint64_t*)p.inputs;
    const uint64_t* recs = (const uint64_t*)w_recs;
    const uint64_t* dv = (const uint64_t*)p.donor_vecs + (int64_t)donor_slot * p.stride;
    uint64_t v[R];
    UNROLL for (int m = 0; m < R; ++m) {
        const int64_t i = tid + 256 * m;
        v[m] = (i < W) ? dv[i] : 0ull;
    }
    const uint64_t* a0 = at_point >= 0 ? recs + (int64_t)at_point * p.stride
                                       : in + (int64_t)(-at_point - 1) * p.stride;
    bool eq = true;
    UNROLL for (int m = 0; m < R; ++m) {
        const int64_t i = tid + 256 * m;
        if (i < W) eq = eq && (((v[m] ^ a0[i]) & valid_bits(i, T)) == 0);
    }
    int stop = -1;
    if (__syncthreads_and(eq)) {
        stop = 0;
    } else {
        for (int k = 0; k < n_levels; ++k) {
            const GP_CONST SpineLvl* lp = cst(levels) + k;
            const SpineLvl lv{lp->fside, lp->sib, lp->par, 0};
            const uint64_t* sb = lv.sib >= 0 ? recs + (int64_t)lv.sib * p.stride
                                             : in + (int64_t)(-lv.sib - 1) * p.stride;
            const uint64_t* pr = recs + (int64_t)lv.par * p.stride;
            const int f = lv.fside & 3;
            const bool right = (lv.fside & 4) != 0;
            eq = true;
            UNROLL for (int m = 0; m < R; ++m) {
                const int64_t i = tid + 256 * m;
                if (i < W) {
                    const uint64_t s = sb[i];
                    const uint64_t r = right ? bop_rt(f, s, v[m]) : bop_rt(f, v[m], s);
                    v[m] = r;
                    eq = eq && (((r ^ pr[i]) & valid_bits(i, T)) == 0);
                }
            }
            if (__syncthreads_and(eq)) {
                stop = k + 1;
                break;
            }
        }
    }
    if (tid == 0) {
        p.stop_out[ci] = stop;
        p.interp_out[ci] = donor_nodes + (stop >= 0 ? stop : n_levels);
    }
    uint64_t* ro = p.root_out ? (uint64_t*)p.root_out + ci * p.stride : nullptr;
    if (stop >= 0) {
        const uint64_t* pv = (const uint64_t*)w_pvec;
        if (ro)
            for (int64_t i = tid; i < W; i += 256) ro[i] = pv[i];
        if (tid == 0) ((int64_t*)p.fit_out)[ci] = *(const int64_t*)w_pfit;
    } else {
        const uint64_t* t = (const uint64_t*)p.target;
        int64_t hits = 0;
        UNROLL for (int m = 0; m < R; ++m) {
            const int64_t i = tid + 256 * m;
            if (i < W) {
                if (ro) ro[i] = v[m];
                hits += __popcll(~(v[m] ^ t[i]) & valid_bits(i, T));
            }
        }
        const int64_t h = block_sum_i64(hits, red);
        if (tid == 0) ((int64_t*)p.fit_out)[ci] = h;
    }
}

// ---------------------------------------------------------- variants
// Interpreter variants: K test cases (words) per lane and S stack slots.
// Fewer slots free registers for more resident waves; a population can use
// a variant when its programs need at most S slots.
static Variant g_variants[] = {
    {"f32_k1_s16", 0, 1, 16, (const void*)k_eval_f32<1, 16>, 0},
    {"f32_k2_s16", 0, 2, 16, (const void*)k_eval_f32<2, 16>, 0},
    {"f32_k4_s16", 0, 4, 16, (const void*)k_eval_f32<4, 16>, 0},
    {"f32_k8_s16", 0, 8, 16, (const void*)k_eval_f32<8, 16>, 0},
    {"f32_k4_s10", 0, 4, 10, (const void*)k_eval_f32<4, 10>, 0},
    {"f32_k8_s10", 0, 8, 10, (const void*)k_eval_f32<8, 10>, 0},
    {"f32t_k4_s10", 0, 4, 10, (const void*)k_eval_f32_tbl<4, 10>, 0, 1, 0},
    {"f32t_k8_s10", 0, 8, 10, (const void*)k_eval_f32_tbl<8, 10>, 0, 1, 0},
    {"f32d_k4_s10", 0, 4, 10, (const void*)k_eval_f32_tbl<4, 10, true>, 0, 1, 0},
    {"f32d_k8_s10", 0, 8, 10, (const void*)k_eval_f32_tbl<8, 10, true>, 0, 1, 0},
    {"bool_k1_s16", 1, 1, 16, (const void*)k_eval_bool<1, 16>, 0},
    {"bool_k2_s16", 1, 2, 16, (const void*)k_eval_bool<2, 16>, 0},
    {"bool_k1_s10", 1, 1, 10, (const void*)k_eval_bool<1, 10>, 0},
    {"boolw_s10", 1, 1, 10, (const void*)k_eval_bool_tbl<1, 10, true>, 0, 1, kBoolWordInputs, 1},
    {"boolt_k1_s10", 1, 1, 10, (const void*)k_eval_bool_tbl<1, 10>, 0, 1, kBoolRegInputs},
    {"boolt_k2_s10", 1, 2, 10, (const void*)k_eval_bool_tbl<2, 10>, 0, 1, kBoolRegInputs},
};

int variant_count() { return (int)(sizeof(g_variants) / sizeof(g_variants[0])); }
Variant* variant_table() { return g_variants; }

hipError_t launch_eval(int variant, const EvalParams& p, int grid, hipStream_t s)
{
    const Variant& v = g_variants[variant];
    const size_t shm = variant_lds(v, p.n_inputs);
    hipLaunchKernelGGL((void (*)(EvalParams))v.kernel, dim3(grid), dim3(kWave), shm, s, p);
    return hipGetLastError();
}

hipError_t launch_init(int32_t* pending, const int32_t* init, int64_t n, unsigned int* cursor,
                       int n_cursors, hipStream_t s)
{
    int64_t need = std::max<int64_t>(n, n_cursors);
    int grid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (need + 255) / 256));
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(256), 0, s, pending, init, n, cursor, n_cursors);
    return hipGetLastError();
}

static int halving_rows(int64_t P) { return P <= 256 ? 1 : (int)(P / 256); }

hipError_t launch_fitness(int vtype, const FitParams& p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (vtype == 1) {
        hipLaunchKernelGGL(k_fit_bool, dim3((unsigned)n), dim3(256), 0, s, p);
        return hipGetLastError();
    }
    switch (halving_rows(p.P)) {
    case 1: hipLaunchKernelGGL(k_fit_f32<1>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_fit_f32<2>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_fit_f32<4>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_fit_f32<8>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 16: hipLaunchKernelGGL(k_fit_f32<16>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 32: hipLaunchKernelGGL(k_fit_f32<32>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    case 64: hipLaunchKernelGGL(k_fit_f32<64>, dim3((unsigned)n), dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------- co-evaluation
// One workgroup of 256 threads per child, over the levels of one round: the
// child's running vector v and the mother's m both take the ancestor's
// function with the same sibling vector as the other operand (the mother is
// re-evaluated alongside her child), and the walk stops at the first level
// where they agree on every case.  Level 0 compares the donor's vector with
// the removed subtree's.  A walk that neither stops nor reaches the root in
// this round leaves v and m for the next one.
template <int R>
__global__ __launch_bounds__(256) void k_coeval_f32(CoParams p)
{
    __shared__ double red[256];
    const GP_CONST CoChild* cp = cst(p.children) + blockIdx.x;
    const float* vin = (const float*)cp->v_in;
    const float* min_ = (const float*)cp->m_in;
    float* vout = (float*)cp->v_out;
    float* mout = (float*)cp->m_out;
    const CoLevel* levels = cp->levels;
    const float* pvec = (const float*)cp->parent_vec;
    const double* pfit = (const double*)cp->parent_fit;
    const int32_t n_levels = cp->n_levels, level_base = cp->level_base, check0 = cp->check0, last = cp->last;
    const int64_t slot = cp->out_slot;
    const int tid = threadIdx.x;
    const int64_t T = p.n_valid;
    float v[R], m[R];
    UNROLL for (int k = 0; k < R; ++k) {
        const int64_t i = tid + 256 * k;
        v[k] = (i < T) ? vin[i] : 0.0f;
        m[k] = (i < T) ? min_[i] : 0.0f;
    }
    int stop = -2;
    if (check0) {
        bool eq = true;
        UNROLL for (int k = 0; k < R; ++k)
            if (tid + 256 * k < T) eq = eq && same_f32(v[k], m[k]);
        if (__syncthreads_and(eq)) stop = 0;
    }
    for (int l = 0; stop == -2 && l < n_levels; ++l) {
        const GP_CONST CoLevel* lp = cst(levels) + l;
        const float* sb = (const float*)lp->sib;
        const int fs = lp->fside;
        const int f = fs & 3;
        const bool right = (fs & 4) != 0;
        bool eq = true;
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < T) {
                const float s = sb[i];
                v[k] = right ? fop_rt(f, s, v[k]) : fop_rt(f, v[k], s);
                m[k] = right ? fop_rt(f, s, m[k]) : fop_rt(f, m[k], s);
                eq = eq && same_f32(v[k], m[k]);
            }
        }
        if (__syncthreads_and(eq)) stop = level_base + l + 1;
    }
    if (stop == -2 && last) stop = -1;
    if (tid == 0) p.stop_out[slot] = stop;
    float* ro = p.root_out ? (float*)p.root_out + slot * p.stride : nullptr;
    if (stop >= 0) {
        if (ro)
            for (int64_t i = tid; i < T; i += 256) ro[i] = pvec[i];
        if (tid == 0) ((double*)p.fit_out)[slot] = *pfit;
    } else if (stop == -1) {
        const float* y = (const float*)p.target;
        double e[R];
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            double val = 0.0;
            if (i < T) {
                if (ro) ro[i] = v[k];
                const float d = v[k] - y[i];
                val = (double)fabsf(d);
            }
            e[k] = val;
        }
        const double f = halving_sum<R>(e, p.P, red);
        if (tid == 0) ((double*)p.fit_out)[slot] = f;
    } else {
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < T) {
                vout[i] = v[k];
                mout[i] = m[k];
            }
        }
    }
}

template <int R>
__global__ __launch_bounds__(256) void k_coeval_bool(CoParams p)
{
    __shared__ int64_t red[256];
    const GP_CONST CoChild* cp = cst(p.children) + blockIdx.x;
    const uint64_t* vin = (const uint64_t*)cp->v_in;
    const uint64_t* min_ = (const uint64_t*)cp->m_in;
    uint64_t* vout = (uint64_t*)cp->v_out;
    uint64_t* mout = (uint64_t*)cp->m_out;
    const CoLevel* levels = cp->levels;
    const uint64_t* pvec = (const uint64_t*)cp->parent_vec;
    const int64_t* pfit = (const int64_t*)cp->parent_fit;
    const int32_t n_levels = cp->n_levels, level_base = cp->level_base, check0 = cp->check0, last = cp->last;
    const int64_t slot = cp->out_slot;
    const int tid = threadIdx.x;
    const int64_t T = p.n_valid;
    const int64_t W = (T + 63) / 64;
    uint64_t v[R], m[R];
    UNROLL for (int k = 0; k < R; ++k) {
        const int64_t i = tid + 256 * k;
        v[k] = (i < W) ? vin[i] : 0ull;
        m[k] = (i < W) ? min_[i] : 0ull;
    }
    int stop = -2;
    if (check0) {
        bool eq = true;
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < W) eq = eq && (((v[k] ^ m[k]) & valid_bits(i, T)) == 0);
        }
        if (__syncthreads_and(eq)) stop = 0;
    }
    for (int l = 0; stop == -2 && l < n_levels; ++l) {
        const GP_CONST CoLevel* lp = cst(levels) + l;
        const uint64_t* sb = (const uint64_t*)lp->sib;
        const int fs = lp->fside;
        const int f = fs & 3;
        const bool right = (fs & 4) != 0;
        bool eq = true;
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < W) {
                const uint64_t s = sb[i];
                v[k] = right ? bop_rt(f, s, v[k]) : bop_rt(f, v[k], s);
                m[k] = right ? bop_rt(f, s, m[k]) : bop_rt(f, m[k], s);
                eq = eq && (((v[k] ^ m[k]) & valid_bits(i, T)) == 0);
            }
        }
        if (__syncthreads_and(eq)) stop = level_base + l + 1;
    }
    if (stop == -2 && last) stop = -1;
    if (tid == 0) p.stop_out[slot] = stop;
    uint64_t* ro = p.root_out ? (uint64_t*)p.root_out + slot * p.stride : nullptr;
    if (stop >= 0) {
        if (ro)
            for (int64_t i = tid; i < W; i += 256) ro[i] = pvec[i];
        if (tid == 0) ((int64_t*)p.fit_out)[slot] = *pfit;
    } else if (stop == -1) {
        const uint64_t* t = (const uint64_t*)p.target;
        int64_t hits = 0;
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < W) {
                if (ro) ro[i] = v[k];
                hits += __popcll(~(v[k] ^ t[i]) & valid_bits(i, T));
            }
        }
        const int64_t h = block_sum_i64(hits, red);
        if (tid == 0) ((int64_t*)p.fit_out)[slot] = h;
    } else {
        UNROLL for (int k = 0; k < R; ++k) {
            const int64_t i = tid + 256 * k;
            if (i < W) {
                vout[i] = v[k];
                mout[i] = m[k];
            }
        }
    }
}

hipError_t launch_coeval(int vtype, const CoParams& p, int64_t n_children, hipStream_t s)
{
    if (n_children <= 0) return hipSuccess;
    if (n_children > 0x7fffffff) return hipErrorInvalidValue;
    if (vtype == 1) {
        const int64_t W = (p.n_valid + 63) / 64;
        const int rows = W <= 256 ? 1 : (int)((W + 255) / 256);
        if (rows == 1) hipLaunchKernelGGL(k_coeval_bool<1>, dim3((unsigned)n_children), dim3(256), 0, s, p);
        else if (rows == 2) hipLaunchKernelGGL(k_coeval_bool<2>, dim3((unsigned)n_children), dim3(256), 0, s, p);
        else if (rows <= 4) hipLaunchKernelGGL(k_coeval_bool<4>, dim3((unsigned)n_children), dim3(256), 0, s, p);
        else if (rows <= 16) hipLaunchKernelGGL(k_coeval_bool<16>, dim3((unsigned)n_children), dim3(256), 0, s, p);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    switch (halving_rows(p.P)) {
    case 1: hipLaunchKernelGGL(k_coeval_f32<1>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_coeval_f32<2>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_coeval_f32<4>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_coeval_f32<8>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 16: hipLaunchKernelGGL(k_coeval_f32<16>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 32: hipLaunchKernelGGL(k_coeval_f32<32>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 64: hipLaunchKernelGGL(k_coeval_f32<64>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------- selection
// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two
// 32x32 -> 64-bit products whose halves are mixed with the other counter words
// and the round key; the key advances by the two Weyl constants per round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
    UNROLL for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Word j of stream s for index i at generation g (counter (i, g, s, j / 4)).
__device__ __forceinline__ uint32_t gen_draw(uint64_t seed, int64_t i, int64_t g, int s, int j)
{
    const uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)g, (uint32_t)s, (uint32_t)(j / 4)),
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    const int q = j & 3;
    return q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
}

// floor(u * n / 2^32) for n < 2^32.
__device__ __forceinline__ int64_t gen_uniform(uint32_t u, int64_t n)
{
    return (int64_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

// k draws with replacement; a candidate replaces the winner only if strictly
// better, so ties keep the earlier draw.
__device__ int64_t tournament(const void* fit, bool boolean, int64_t n, int k, uint64_t seed, int64_t i,
                              int64_t g, int s)
{
    int64_t best = gen_uniform(gen_draw(seed, i, g, s, 0), n);
    for (int j = 1; j < k; ++j) {
        const int64_t c = gen_uniform(gen_draw(seed, i, g, s, j), n);
        if (boolean) {
            const int64_t* h = (const int64_t*)fit;
            if (h[c] > h[best]) best = c;
        } else {
            const double* e = (const double*)fit;
            const double a = e[c], b = e[best];
            if (!isnan(a) && (isnan(b) || a < b)) best = c;
        }
    }
    return best;
}

__global__ __launch_bounds__(256) void k_select(SelectParams p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= p.n) return;
    const bool b = p.boolean != 0;
    const int64_t m = tournament(p.fit, b, p.n, p.k, p.seed, i, p.generation, 0);
    const int64_t f = tournament(p.fit, b, p.n, p.k, p.seed, i, p.generation, 1);
    p.mother[i] = m;
    p.father[i] = f;
    p.point[i] = gen_uniform(gen_draw(p.seed, i, p.generation, 2, 0), p.sizes[m]);
    p.donor_node[i] = gen_uniform(gen_draw(p.seed, i, p.generation, 2, 1), p.sizes[f]);
}

__global__ __launch_bounds__(256) void k_mark(MarkParams p)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= p.n) return;
    const bool b = p.boolean != 0;
    atomicAdd(p.drawn + tournament(p.fit, b, p.n, p.k, p.seed, j, p.generation, 0), 1);
    atomicAdd(p.drawn + tournament(p.fit, b, p.n, p.k, p.seed, j, p.generation, 1), 1);
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* dst, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = v;
}

hipError_t launch_select(const SelectParams& p, hipStream_t s)
{
    if (p.n <= 0) return hipSuccess;
    if (p.n >= (int64_t(1) << 32) || p.k < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_mark(const MarkParams& p, hipStream_t s)
{
    if (p.n <= 0) return hipSuccess;
    if (p.n >= (int64_t(1) << 32) || p.k < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mark, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* dst, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, n, v);
    return hipGetLastError();
}

// Row k of dst = row src_rows[k] of src (rows of row_bytes, a multiple of 16):
// chunk values of a mother gathered into an input matrix for co-evaluation.
__global__ __launch_bounds__(256) void k_gather_rows(const uint4* src, const int64_t* src_rows, uint4* dst,
                                                     int64_t row_u4)
{
    const int64_t k = blockIdx.x;
    const int64_t r = src_rows[k];
    for (int64_t i = threadIdx.x; i < row_u4; i += 256) dst[k * row_u4 + i] = src[r * row_u4 + i];
}

hipError_t launch_gather_rows(const void* src, const int64_t* src_rows, int64_t n_rows, int64_t row_bytes, void* dst,
                              hipStream_t s)
{
    if (n_rows <= 0) return hipSuccess;
    if (n_rows > 0x7fffffff || row_bytes % 16 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)n_rows), dim3(256), 0, s, (const uint4*)src, src_rows,
                       (uint4*)dst, row_bytes / 16);
    return hipGetLastError();
}

// Row rows[2k] of dst = row rows[2k + 1] of src: the values of chunks a child
// reuses from its parents, moved from the parents' chunk vectors.  Each
// workgroup moves whole rows, one 16-byte word per thread per step.
__global__ __launch_bounds__(256) void k_move_rows(const uint4* src, const int64_t* rows, int64_t n_rows, uint4* dst,
                                                   int64_t row_u4)
{
    for (int64_t k = blockIdx.x; k < n_rows; k += gridDim.x) {
        const int64_t d = rows[2 * k], r = rows[2 * k + 1];
        for (int64_t i = threadIdx.x; i < row_u4; i += 256) dst[d * row_u4 + i] = src[r * row_u4 + i];
    }
}

hipError_t launch_move_rows(const void* src, const int64_t* rows, int64_t n_rows, int64_t row_bytes, void* dst,
                            hipStream_t s)
{
    if (n_rows <= 0) return hipSuccess;
    if (row_bytes % 16 != 0) return hipErrorInvalidValue;
    const int64_t grid = std::min<int64_t>(n_rows, 65536);
    hipLaunchKernelGGL(k_move_rows, dim3((unsigned)grid), dim3(256), 0, s, (const uint4*)src, rows, n_rows,
                       (uint4*)dst, row_bytes / 16);
    return hipGetLastError();
}

// ---------------------------------------------------------- measurement
// Counter calibration: every wave runs `iters` times a block of 32 VALU
// instructions of one class over eight independent registers (so no
// instruction waits for the one before it), the loop itself being scalar.
// A run with iters = 0 gives the fixed instructions around the loop, so the
// difference of two runs is exactly 32 x iters VALU instructions per wave.
#define GP_CAL8(op) op(0) op(1) op(2) op(3) op(4) op(5) op(6) op(7)
#define GP_CAL32(op) GP_CAL8(op) GP_CAL8(op) GP_CAL8(op) GP_CAL8(op)
#define GP_ADD(i) "v_add_f32_e32 %" #i ", %" #i ", %8\n"
#define GP_MUL(i) "v_mul_f32_e32 %" #i ", %" #i ", %8\n"
#define GP_FMA(i) "v_fma_f32 %" #i ", %" #i ", %8, %9\n"
#define GP_RCP(i) "v_rcp_f32_e32 %" #i ", %" #i "\n"
#define GP_CND(i) "v_cndmask_b32_e32 %" #i ", %" #i ", %8, vcc\n"
#define GP_CMP(i) "v_cmp_lt_f32_e32 vcc, %" #i ", %8\n"
#define GP_MAX3(i) "v_max3_f32 %" #i ", %" #i ", %8, %9\n"
#define GP_MOV(i) "v_mov_b32_e32 %" #i ", %8\n"
#define GP_ADDRCP(i) "v_add_f32_e32 %" #i ", %" #i ", %8\nv_rcp_f32_e32 %9, %8\n"
#define GP_ADDCMP(i) "v_add_f32_e32 %" #i ", %" #i ", %8\nv_cmp_lt_f32_e32 vcc, %" #i ", %8\n"

template <int CLS>
__global__ __launch_bounds__(64) void k_valu_cal(int64_t iters, float* out)
{
    float a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    float b = 1.0f + 1e-7f * threadIdx.x, c = 0.5f;
    asm volatile("s_mov_b64 vcc, -1" ::: "vcc");
    for (int64_t it = 0; it < iters; ++it) {
#define GP_CAL_ASM(body) \
        asm volatile(body : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) \
                     : "v"(b), "v"(c) : "vcc")
        if constexpr (CLS == 0) GP_CAL_ASM(GP_CAL32(GP_ADD));
        else if constexpr (CLS == 1) GP_CAL_ASM(GP_CAL32(GP_MUL));
        else if constexpr (CLS == 2) GP_CAL_ASM(GP_CAL32(GP_FMA));
        else if constexpr (CLS == 3) GP_CAL_ASM(GP_CAL32(GP_RCP));
        else if constexpr (CLS == 4) GP_CAL_ASM(GP_CAL32(GP_CND));
        else if constexpr (CLS == 5) GP_CAL_ASM(GP_CAL32(GP_CMP));
        else if constexpr (CLS == 6) GP_CAL_ASM(GP_CAL32(GP_MAX3));
        else if constexpr (CLS == 7) GP_CAL_ASM(GP_CAL32(GP_MOV));
        else if constexpr (CLS == 8) GP_CAL_ASM(GP_CAL8(GP_ADDRCP) GP_CAL8(GP_ADDRCP));
        else GP_CAL_ASM(GP_CAL8(GP_ADDCMP) GP_CAL8(GP_ADDCMP));
#undef GP_CAL_ASM
    }
    out[(int64_t)blockIdx.x * 64 + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

hipError_t launch_valu_cal(int cls, int64_t n_waves, int64_t iters, float* out, hipStream_t s)
{
    if (n_waves < 1 || n_waves > 0x7fffffff || iters < 0) return hipErrorInvalidValue;
    const dim3 g((unsigned)n_waves), b(64);
    switch (cls) {
    case 0: hipLaunchKernelGGL(k_valu_cal<0>, g, b, 0, s, iters, out); break;
    case 1: hipLaunchKernelGGL(k_valu_cal<1>, g, b, 0, s, iters, out); break;
    case 2: hipLaunchKernelGGL(k_valu_cal<2>, g, b, 0, s, iters, out); break;
    case 3: hipLaunchKernelGGL(k_valu_cal<3>, g, b, 0, s, iters, out); break;
    case 4: hipLaunchKernelGGL(k_valu_cal<4>, g, b, 0, s, iters, out); break;
    case 5: hipLaunchKernelGGL(k_valu_cal<5>, g, b, 0, s, iters, out); break;
    case 6: hipLaunchKernelGGL(k_valu_cal<6>, g, b, 0, s, iters, out); break;
    case 7: hipLaunchKernelGGL(k_valu_cal<7>, g, b, 0, s, iters, out); break;
    case 8: hipLaunchKernelGGL(k_valu_cal<8>, g, b, 0, s, iters, out); break;
    case 9: hipLaunchKernelGGL(k_valu_cal<9>, g, b, 0, s, iters, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- splice
// Children are built from three contiguous byte ranges each (the mother's
// nodes before the replaced subtree, the donor, the mother's nodes after it;
// Figure 1), copied here at memory speed.  One workgroup per piece: whole
// 16-byte aligned output words are assembled from 4-byte aligned source words
// with byte funnel shifts (the source offset within a word is the same for
// the whole piece), and the unaligned head and tail bytes of the piece are
// copied one by one.  Reads start at most 3 bytes before and end at most 4
// bytes after a piece's source range (both inside 4-byte words that overlap
// it); source buffers start 4-byte aligned and carry 32 bytes of padding.
__global__ __launch_bounds__(256) void k_splice(const SpliceItem* items, uint8_t* out)
{
    typedef __attribute__((address_space(1))) uint8_t gu8;
    typedef __attribute__((address_space(1))) uint32_t gu32;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) u32x4 gu128;
    const GP_CONST SpliceItem* ip = cst(items) + blockIdx.x;
    const gu8* src = (const gu8*)ip->src;
    const int64_t len = ip->len;
    gu8* dst = (gu8*)(out + ip->dst);
    const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + (uintptr_t)len;
    const uintptr_t a0 = (d0 + 15) & ~(uintptr_t)15, a1 = d1 & ~(uintptr_t)15;
    const int tid = threadIdx.x;
    if (a0 >= a1) {
        for (int64_t i = tid; i < len; i += 256) dst[i] = src[i];
        return;
    }
    const int64_t head = (int64_t)(a0 - d0), tail = (int64_t)(d1 - a1);
    if (tid < head) dst[tid] = src[tid];
    if (tid >= 64 && tid - 64 < tail) {
        const int64_t i = (int64_t)(a1 - d0) + (tid - 64);
        dst[i] = src[i];
    }
    const int64_t nw = (int64_t)((a1 - a0) >> 4);
    const uintptr_t sa = (uintptr_t)(src + head);
    const uint32_t sh = (uint32_t)(sa & 3);
    const gu32* s4 = (const gu32*)(sa & ~(uintptr_t)3);
    gu128* o = (gu128*)a0;
    if (sh == 0) {
        for (int64_t w = tid; w < nw; w += 256) {
            const gu32* q = s4 + 4 * w;
            o[w] = u32x4{q[0], q[1], q[2], q[3]};
        }
    } else {
        for (int64_t w = tid; w < nw; w += 256) {
            const gu32* q = s4 + 4 * w;
            const uint32_t v0 = q[0], v1 = q[1], v2 = q[2], v3 = q[3], v4 = q[4];
            o[w] = u32x4{__builtin_amdgcn_alignbyte(v1, v0, sh), __builtin_amdgcn_alignbyte(v2, v1, sh),
                         __builtin_amdgcn_alignbyte(v3, v2, sh), __builtin_amdgcn_alignbyte(v4, v3, sh)};
        }
    }
}

hipError_t launch_splice(const SpliceItem* items, int64_t n_items, uint8_t* out, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (n_items > (int64_t(1) << 24)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_splice, dim3((unsigned)n_items), dim3(256), 0, s, items, out);
    return hipGetLastError();
}

hipError_t launch_walk(int vtype, const WalkParams& p, int64_t n_children, hipStream_t s)
{
    if (n_children <= 0) return hipSuccess;
    if (vtype == 1) {
        const int64_t W = (p.n_valid + 63) / 64;
        const int rows = W <= 256 ? 1 : (int)((W + 255) / 256);
        switch (rows) {
        case 1: hipLaunchKernelGGL(k_walk_bool<1>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
        case 2: hipLaunchKernelGGL(k_walk_bool<2>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
        case 3:
        case 4: hipLaunchKernelGGL(k_walk_bool<4>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
        default:
            if (rows <= 16) {
                hipLaunchKernelGGL(k_walk_bool<16>, dim3((unsigned)n_children), dim3(256), 0, s, p);
                break;
            }
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (halving_rows(p.P)) {
    case 1: hipLaunchKernelGGL(k_walk_f32<1>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_walk_f32<2>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_walk_f32<4>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_walk_f32<8>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 16: hipLaunchKernelGGL(k_walk_f32<16>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 32: hipLaunchKernelGGL(k_walk_f32<32>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    case 64: hipLaunchKernelGGL(k_walk_f32<64>, dim3((unsigned)n_children), dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpe
