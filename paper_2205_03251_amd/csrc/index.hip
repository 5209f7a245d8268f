// Device-side index of a population of prefix trees: the first steps of
// loading (Section 3.1 flattens each tree into one byte per node in prefix
// order).  For every tree it decides validity, and for every node of a valid
// tree it finds the end of the node's subtree and the node's parent.
//
// A node's step is +1 for a function (binary: it opens two child positions
// and fills one) and -1 for anything else.  E(k) is the sum of the steps of
// the positions before k, over the whole population.  The tree on [s, e) is
// valid iff each byte is a known function or a terminal below n_inputs,
// E(k) >= E(s) for s < k < e, and E(e) = E(s) - 1 (the count of open child
// positions never runs out early and ends exhausted).  The subtree of node k
// ends (exclusively) at the first j > k with E(j) < E(k): k + 1 for a
// terminal.  Its parent is the last i < k with E(i) <= E(k).  Both searches
// run per 4096-position block, in registers and in the block's minima in
// LDS; the few that leave the block continue in a min-tree of E (level 0 is
// E, each entry of level l the minimum of a group of kIxFan entries of level
// l - 1, so a search step reads one 64-byte group).  On request the Strahler
// number of every node follows, one level per pass over the subtree ranges.
#include <algorithm>
#include <mutex>

#include "dev.h"

namespace gpe {

// Scratch of the allocation-free index entry point (layout in dev.h).  Host
// code never names it except to look up its device address: on each device
// the array has its own copy at its own address.
static __device__ __align__(256) int32_t scratch[kIxStaticWords];

hipError_t ix_static_scratch(int device, int32_t** out)
{
    static std::mutex mu;
    static int32_t* addr[256] = {};
    if (device < 0 || device >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (int32_t*)p;
    }
    *out = addr[device];
    return hipSuccess;
}

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* dst, int64_t n, uint8_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = v;
}

hipError_t launch_fill_u8(uint8_t* dst, int64_t n, uint8_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t grid = std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)grid), dim3(256), 0, s, dst, n, v);
    return hipGetLastError();
}

static_assert(kIxFan == 16, "a group is read as four 16-byte loads");

// Two int16 values (within +-32767) in one word, the first in the low half.
__device__ __forceinline__ int32_t ix_pack16(int32_t lo, int32_t hi)
{
    return (int32_t)(((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16));
}

__device__ __forceinline__ int32_t ix_e(const IxParams& q, int64_t k)
{
    return q.el[k] + q.boff[k / kIxBlock];
}

__device__ __forceinline__ bool ix_bad_byte(uint8_t b, int n_inputs)
{
    return (b & 0x80) ? (b & 0x7f) > 3 : (int)b >= n_inputs;
}

// Last tree t with offsets[t] <= k (offsets non-decreasing; any t in range
// otherwise).
__device__ __forceinline__ int64_t ix_tree_of(const IxParams& q, int64_t k)
{
    int64_t lo = 0, hi = q.n_trees;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (q.offsets[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The last tree t in [lo, hi] with offsets[t] <= k, or lo.
__device__ __forceinline__ int64_t ix_tree_in(const IxParams& q, int64_t lo, int64_t hi, int64_t k)
{
    ++hi;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (q.offsets[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Group g of min-tree level l (the kIxFan entries from g, g a multiple of
// kIxFan), read with four 16-byte loads (two for el); levels and el are
// padded to whole groups.  Entries past the level's length hold whatever the padding holds.
__device__ __forceinline__ void ix_load_group(const IxParams& q, int l, int64_t g, int32_t (&x)[kIxFan])
{
    if (l == 0) {
        // 16 int16 entries, two 16-byte loads
        const int4* src = (const int4*)(q.el + g);
        const int32_t add = q.boff[g / kIxBlock];   // a group never straddles a scan block
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int4 w = src[i];
            const int32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                x[8 * i + 2 * h] = (int32_t)(int16_t)(u[h] & 0xffff) + add;
                x[8 * i + 2 * h + 1] = (u[h] >> 16) + add;
            }
        }
        return;
    }
    const int4* src = (const int4*)(q.seg + q.lvl[2 * l] + g);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int4 w = src[i];
        x[4 * i] = w.x;
        x[4 * i + 1] = w.y;
        x[4 * i + 2] = w.z;
        x[4 * i + 3] = w.w;
    }
}

// The first index in [p, end of p's group) of level l whose value is below
// v, or -1.
__device__ __forceinline__ int64_t ix_scan_in(const int32_t (&x)[kIxFan], int64_t g, int64_t p, int64_t len,
                                             int32_t v)
{
    int64_t hit = -1;
#pragma unroll
    for (int i = kIxFan - 1; i >= 0; --i) {
        const int64_t idx = g + i;
        if (idx >= p && idx < len && x[i] < v) hit = idx;
    }
    return hit;
}

__device__ __forceinline__ int64_t ix_scan_group(const IxParams& q, int l, int64_t p, int32_t v)
{
    const int64_t g = p & ~(int64_t)(kIxFan - 1);
    int32_t x[kIxFan];
    ix_load_group(q, l, g, x);
    return ix_scan_in(x, g, p, q.lvl[2 * l + 1], v);
}

// First position at or after entry p of level l whose E is below v, or -1
// (p times kIxFan^l is the first position searched).  Going up, every
// position from there to the end of the current node's parent has been
// checked when a group scan fails, so the search continues at the parent's
// next sibling; going down, it takes the first child whose minimum is below v.
__device__ __forceinline__ int64_t ix_first_below_at(const IxParams& q, int l, int64_t p, int32_t v)
{
    int64_t hit = -1;
    for (;;) {
        if (p >= q.lvl[2 * l + 1]) return -1;
        hit = ix_scan_group(q, l, p, v);
        if (hit >= 0) break;
        if (l == q.top) return -1;
        p = p / kIxFan + 1;
        ++l;
    }
    while (l > 0 && hit >= 0) {
        --l;
        hit = ix_scan_group(q, l, hit * kIxFan, v);
    }
    return hit;
}

// Last position at or before the end of entry p of level l whose E is at
// most v, or -1: the mirror image of ix_first_below_at.
__device__ __forceinline__ int64_t ix_last_at_most_at(const IxParams& q, int l, int64_t p, int32_t v)
{
    int64_t hit = -1;
    int32_t x[kIxFan];
    for (;;) {
        if (p < 0) return -1;
        const int64_t g = p & ~(int64_t)(kIxFan - 1);
        ix_load_group(q, l, g, x);
#pragma unroll
        for (int i = 0; i < kIxFan; ++i)
            if (g + i <= p && x[i] <= v) hit = g + i;
        if (hit >= 0) break;
        if (l == q.top) return -1;
        p = g / kIxFan - 1;
        ++l;
    }
    while (l > 0) {
        --l;
        const int64_t g = hit * kIxFan, len = q.lvl[2 * l + 1];
        ix_load_group(q, l, g, x);
        hit = -1;
#pragma unroll
        for (int i = 0; i < kIxFan; ++i)
            if (g + i < len && x[i] <= v) hit = g + i;
        if (hit < 0) return -1;
    }
    return hit;
}

// Steps of one 4096-position block: el = exclusive prefix within the block,
// bsum = the block's total.  Positions past n step by 0.
__global__ __launch_bounds__(256) void k_ix_scan(IxParams q, int32_t* bsum)
{
    __shared__ int32_t wtot[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kIxBlock + (int64_t)tid * 16;
    uint32_t word[4] = {0, 0, 0, 0};
    if (base + 16 <= q.n) {
        const uint4 v = *(const uint4*)(q.ops + base);
        word[0] = v.x;
        word[1] = v.y;
        word[2] = v.z;
        word[3] = v.w;
    } else {
        for (int j = 0; j < 16; ++j)
            if (base + j < q.n) word[j >> 2] |= (uint32_t)q.ops[base + j] << (8 * (j & 3));
    }
    int32_t pre[16];
    int32_t run = 0;
    for (int j = 0; j < 16; ++j) {
        pre[j] = run;
        const uint32_t b = (word[j >> 2] >> (8 * (j & 3))) & 0xffu;
        run += base + j < q.n ? ((b & 0x80u) ? 1 : -1) : 0;
    }
    int32_t incl = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += wtot[i];
    const int32_t excl = wbase + incl - run;
    int4* dst = (int4*)(q.el + base);
    for (int j = 0; j < 2; ++j)
        dst[j] = make_int4(ix_pack16(excl + pre[8 * j], excl + pre[8 * j + 1]),
                           ix_pack16(excl + pre[8 * j + 2], excl + pre[8 * j + 3]),
                           ix_pack16(excl + pre[8 * j + 4], excl + pre[8 * j + 5]),
                           ix_pack16(excl + pre[8 * j + 6], excl + pre[8 * j + 7]));
    if (tid == 255) bsum[blockIdx.x] = excl + run;
}

// Exclusive prefix of the block totals bsum[0 .. nb) into boff, boff[nb] =
// their sum (E(n) after the position scan), and el[nb * kIxBlock] = 0 so that
// E(n) = el[n] + boff[n / kIxBlock] also when n is a multiple of the block.
// Three launches: the prefix within each group of kIxBlock totals (a
// workgroup per group, 16 a thread), whose sum then replaces the group's
// first total (read by then); the group sums scanned in place by one
// workgroup; each group's offset added.  bsum is left clobbered.
__global__ __launch_bounds__(256) void k_ix_top_local(IxParams q, int32_t* bsum, int64_t nb)
{
    __shared__ int32_t wtot[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kIxBlock, i0 = g0 + (int64_t)tid * 16;
    int32_t pre[16];
    int32_t run = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        pre[j] = run;
        run += i0 + j < nb ? bsum[i0 + j] : 0;
    }
    int32_t incl = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += wtot[i];
    const int32_t excl = wbase + incl - run;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (i0 + j < nb) q.boff[i0 + j] = excl + pre[j];
    __syncthreads();                          // every total of the group read
    if (tid == 255) bsum[g0] = excl + run;
}

constexpr int kIxTopGroups = 256;         // groups of kIxBlock totals one workgroup scans

__global__ __launch_bounds__(kIxTopGroups) void k_ix_top_groups(IxParams q, int32_t* bsum, int64_t nb)
{
    __shared__ int32_t wtot[kIxTopGroups / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ng = (nb + kIxBlock - 1) / kIxBlock;
    const int32_t v = tid < ng ? bsum[(int64_t)tid * kIxBlock] : 0;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += wtot[i];
    if (tid < ng) bsum[(int64_t)tid * kIxBlock] = wbase + incl - v;
    if (tid == kIxTopGroups - 1) {
        q.boff[nb] = wbase + incl;
        q.el[nb * kIxBlock] = 0;
    }
}

__global__ __launch_bounds__(256) void k_ix_top_add(IxParams q, const int32_t* bsum, int64_t nb)
{
    for (int64_t i = kIxBlock + (int64_t)blockIdx.x * 256 + threadIdx.x; i < nb; i += (int64_t)gridDim.x * 256)
        q.boff[i] += bsum[i / kIxBlock * kIxBlock];
}

static hipError_t launch_top(const IxParams& q, int32_t* bsum, int64_t nb, hipStream_t s)
{
    const int64_t ng = (nb + kIxBlock - 1) / kIxBlock;
    if (ng > kIxTopGroups) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ix_top_local, dim3((unsigned)ng), dim3(256), 0, s, q, bsum, nb);
    hipLaunchKernelGGL(k_ix_top_groups, dim3(1), dim3(kIxTopGroups), 0, s, q, bsum, nb);
    if (ng > 1) {
        const int64_t grid = std::min<int64_t>(65536, (nb - kIxBlock + 255) / 256);
        hipLaunchKernelGGL(k_ix_top_add, dim3((unsigned)grid), dim3(256), 0, s, q, (const int32_t*)bsum, nb);
    }
    return hipGetLastError();
}

// Level l >= 1 of the min-tree: the minimum of each group of level l - 1.
__global__ __launch_bounds__(256) void k_ix_level(IxParams q, int l)
{
    const int64_t len = q.lvl[2 * l + 1], src_len = q.lvl[2 * (l - 1) + 1];
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < len; p += (int64_t)gridDim.x * 256) {
        const int64_t g = p * kIxFan;
        int32_t x[kIxFan];
        ix_load_group(q, l - 1, g, x);
        int32_t m = INT32_MAX;
        for (int i = 0; i < kIxFan; ++i)
            if (g + i < src_len) m = min(m, x[i]);
        q.seg[q.lvl[2 * l] + p] = m;
    }
}

// valid[t] = 1 for a tree whose offsets are in order and inside [0, n];
// flags offsets that do not run from 0 to n without decreasing.
__global__ __launch_bounds__(256) void k_ix_init(IxParams q)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < q.n_trees; t += (int64_t)gridDim.x * 256) {
        const int64_t s = q.offsets[t], e = q.offsets[t + 1];
        const bool inside = 0 <= s && s < e && e <= q.n;
        q.valid[t] = inside ? 1 : 0;
        if (e < s || (t == 0 && s != 0) || (t == q.n_trees - 1 && e != q.n)) *q.bad_offsets = 1;
    }
}

// The 16 bytes at p + k0 (zero past n), four to a word.
__device__ __forceinline__ void ix_bytes16(const uint8_t* p, int64_t k0, int64_t n, uint32_t (&w)[4])
{
    if (k0 + 16 <= n && (((uintptr_t)(p + k0)) & 15) == 0) {
        const uint4 v = *(const uint4*)(p + k0);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    } else {
        w[0] = w[1] = w[2] = w[3] = 0;
        for (int j = 0; j < 16; ++j)
            if (k0 + j < n) w[j >> 2] |= (uint32_t)p[k0 + j] << (8 * (j & 3));
    }
}

// The positions of one thread: 16 consecutive ones, walking the trees they
// fall in.  body(k, t, s, e, op, ek) runs for each position k inside a
// well-formed tree t = [s, e), with k's opcode byte op and E(k); other(k) for
// the rest.  The opcodes come in one 16-byte load and E is carried along from
// E(k0) by the steps, so the walk itself reads nothing per position.
template <class Body, class Other>
__device__ __forceinline__ void ix_positions(const IxParams& q, Body body, Other other)
{
    const int64_t k0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (k0 >= q.n) return;
    uint32_t w[4];
    ix_bytes16(q.ops, k0, q.n, w);
    int32_t ek = ix_e(q, k0);
    int64_t t = ix_tree_of(q, k0);
    int64_t s = q.offsets[t], e = q.offsets[t + 1];
    for (int j = 0; j < 16; ++j) {
        const int64_t k = k0 + j;
        if (k >= q.n) break;
        const uint32_t wj = j < 8 ? (j < 4 ? w[0] : w[1]) : (j < 12 ? w[2] : w[3]);
        const uint8_t op = (uint8_t)(wj >> (8 * (j & 3)));
        while (k >= e && t + 1 < q.n_trees) {
            ++t;
            s = q.offsets[t];
            e = q.offsets[t + 1];
        }
        if (0 <= s && s <= k && k < e && e <= q.n) body(k, t, s, e, op, ek);
        else other(k);
        ek += (op & 0x80) ? 1 : -1;
    }
}

// Validity, in two parts.  Every byte a known opcode: one pass over the
// bytes, which looks a tree up only for a bad byte.  The count of open child
// positions never running out before the end and running out there: with
// steps of +-1, the first j > s with E(j) < E(s) is e, one search per tree.
__global__ __launch_bounds__(256) void k_ix_bytes(IxParams q, const int32_t* tfirst)
{
    const int64_t k0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (k0 >= q.n) return;
    uint32_t w[4];
    ix_bytes16(q.ops, k0, q.n, w);
    uint32_t bad = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (k0 + j < q.n && ix_bad_byte((uint8_t)(w[j >> 2] >> (8 * (j & 3))), q.n_inputs)) bad |= 1u << j;
    if (!bad) return;
    const int64_t b = k0 / kIxBlock, nb = (q.n + kIxBlock - 1) / kIxBlock;
    int64_t t = ix_tree_in(q, tfirst[b], b + 1 < nb ? tfirst[b + 1] : q.n_trees - 1, k0);
    int64_t s = q.offsets[t], e = q.offsets[t + 1];
    while (bad) {
        const int64_t k = k0 + (__ffs(bad) - 1);
        bad &= bad - 1;
        while (k >= e && t + 1 < q.n_trees) {
            ++t;
            s = q.offsets[t];
            e = q.offsets[t + 1];
        }
        if (0 <= s && s <= k && k < e) q.valid[t] = 0;
    }
}

__global__ __launch_bounds__(256) void k_ix_trees(IxParams q)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < q.n_trees; t += (int64_t)gridDim.x * 256) {
        const int64_t s = q.offsets[t], e = q.offsets[t + 1];
        if (!(0 <= s && s < e && e <= q.n)) continue;           // refused by k_ix_init
        if (ix_first_below_at(q, 0, s + 1, ix_e(q, s)) != e) q.valid[t] = 0;
    }
}

// Within one block: E of its positions less the block's offset (the scan's
// el, which stays within +-kIxBlock), the minimum of each group of kIxFan
// (one thread's positions) and of each kIxFan of those.
struct alignas(16) IxBlockMins {
    int16_t e0[kIxBlock];
    int16_t m1[kIxBlock / kIxFan];
    int16_t m2[kIxBlock / kIxFan / kIxFan];
};
static_assert(kIxBlock == kIxFan * kIxFan * kIxFan, "a block is three min-tree levels");

// The kIxFan entries of a block level from g (a multiple of kIxFan), with
// two 16-byte LDS reads.
__device__ __forceinline__ void ix_lds_group(const int16_t* a, int g, int32_t (&x)[kIxFan])
{
    const int4* p = (const int4*)(a + g);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int4 w = p[i];
        const int32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            x[8 * i + 2 * h] = (int32_t)(int16_t)(u[h] & 0xffff);
            x[8 * i + 2 * h + 1] = u[h] >> 16;
        }
    }
}

// First index in [g + from, g + kIxFan) whose entry is below v, or -1.
__device__ __forceinline__ int ix_first_lt(const int32_t (&x)[kIxFan], int g, int from, int32_t v)
{
    int hit = kIxFan;
#pragma unroll
    for (int i = kIxFan - 1; i >= 0; --i)
        if (i >= from && x[i] < v) hit = i;
    return hit < kIxFan ? g + hit : -1;
}

// Last index in [g, g + upto] whose entry is at most v, or -1.
__device__ __forceinline__ int ix_last_le(const int32_t (&x)[kIxFan], int g, int upto, int32_t v)
{
    int hit = -1;
#pragma unroll
    for (int i = 0; i < kIxFan; ++i)
        if (i <= upto && x[i] <= v) hit = i;
    return hit >= 0 ? g + hit : -1;
}

// First block position whose E is below v after the group of position i
// (that group already searched), or -1.
__device__ __forceinline__ int ix_lds_first_below(const IxBlockMins& b, int i, int32_t v)
{
    int32_t x[kIxFan];
    const int g1 = i / kIxFan;
    ix_lds_group(b.m1, g1 & ~(kIxFan - 1), x);
    int h1 = ix_first_lt(x, g1 & ~(kIxFan - 1), (g1 & (kIxFan - 1)) + 1, v);
    if (h1 < 0) {
        ix_lds_group(b.m2, 0, x);
        const int h2 = ix_first_lt(x, 0, g1 / kIxFan + 1, v);
        if (h2 < 0) return -1;
        ix_lds_group(b.m1, kIxFan * h2, x);
        h1 = ix_first_lt(x, kIxFan * h2, 0, v);
        if (h1 < 0) return -1;
    }
    ix_lds_group(b.e0, kIxFan * h1, x);
    return ix_first_lt(x, kIxFan * h1, 0, v);
}

// Last block position whose E is at most v before the group of position i
// (that group already searched), or -1.
__device__ __forceinline__ int ix_lds_last_at_most(const IxBlockMins& b, int i, int32_t v)
{
    int32_t x[kIxFan];
    const int g1 = i / kIxFan;
    ix_lds_group(b.m1, g1 & ~(kIxFan - 1), x);
    int h1 = ix_last_le(x, g1 & ~(kIxFan - 1), (g1 & (kIxFan - 1)) - 1, v);
    if (h1 < 0) {
        ix_lds_group(b.m2, 0, x);
        const int h2 = ix_last_le(x, 0, g1 / kIxFan - 1, v);
        if (h2 < 0) return -1;
        ix_lds_group(b.m1, kIxFan * h2, x);
        h1 = ix_last_le(x, kIxFan * h2, kIxFan - 1, v);
        if (h1 < 0) return -1;
    }
    ix_lds_group(b.e0, kIxFan * h1, x);
    return ix_last_le(x, kIxFan * h1, kIxFan - 1, v);
}

// tfirst[b] = the tree holding the first position of scan block b (bsum,
// free once the block offsets are summed, holds them).
__global__ __launch_bounds__(256) void k_ix_tfirst(IxParams q, int32_t* tfirst, int64_t nb)
{
    for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < nb; b += (int64_t)gridDim.x * 256)
        tfirst[b] = (int32_t)ix_tree_of(q, b * kIxBlock);
}

constexpr int kIxQueue = 1024;            // block-leaving searches shared out per workgroup

// A search that left the block, continued in the global min-tree from the
// level whose entries are whole blocks (or the top): the end (parent = false)
// or the parent of position k of tree [s, e), whose E is v.
__device__ __forceinline__ int32_t ix_global_link(const IxParams& q, int64_t B, int64_t k, int64_t s, int64_t e,
                                                  int32_t v, bool parent)
{
    const int L = q.top < 3 ? q.top : 3;
    if (!parent) {
        const int64_t J = ix_first_below_at(q, L, (B + kIxBlock) >> (4 * L), v);
        return J > k && J <= e ? (int32_t)(J - s) : -1;
    }
    const int64_t P = B > 0 ? ix_last_at_most_at(q, L, (B >> (4 * L)) - 1, v) : -1;
    return P >= s && P < k ? (int32_t)(P - s) : -1;
}

// Subtree end and parent of every position, one scan block per workgroup.
// The end of function k is the first j > k with E(j) < E(k); its parent (any
// non-root k) is the last i < k with E(i) <= E(k): the previous position when
// that is a function (k is its first child), else the function whose first
// child's subtree ends at k, since every position strictly between that
// function and k has a larger E.  Ends, then parents: each thread settles
// what its own positions answer (in registers); the searches that go past
// them are listed and shared out over the workgroup, which runs them in the
// block's minima in LDS with every lane busy (run where they arise, a wave
// would step through every search any of its lanes needs); those that leave
// the block (for a random walk about the square root of the block's length)
// are queued and continued in the global min-tree, and a search that finds
// the queue full continues at once.  Results are gathered in LDS and written
// out in whole lines: written per position, a wave's stores spread over 64
// lines and reach memory one partial line at a time.
__global__ __launch_bounds__(256) void k_ix_links(IxParams q, const int32_t* tfirst)
{
    __shared__ IxBlockMins bm;
    __shared__ uint16_t work[kIxBlock];       // block positions searched in the block minima
    __shared__ uint16_t queue[kIxQueue];      // block positions searched in the global min-tree
    __shared__ int32_t res[kIxBlock];         // this pass's results, tree-local
    __shared__ int32_t n_work, queued;
    const int tid = threadIdx.x;
    const int64_t B = (int64_t)blockIdx.x * kIxBlock, k0 = B + (int64_t)tid * kIxFan;
    const int64_t nb = (q.n + kIxBlock - 1) / kIxBlock;
    const int64_t t_lo = tfirst[blockIdx.x], t_hi = blockIdx.x + 1 < nb ? tfirst[blockIdx.x + 1] : q.n_trees - 1;
    const int here = (int)min<int64_t>(kIxBlock, q.n - B);
    uint32_t w[4];
    ix_bytes16(q.ops, k0, q.n, w);
    int32_t ev[kIxFan];
    int32_t run = q.el[k0];                   // as the scan: positions past n step by 0
#pragma unroll
    for (int j = 0; j < kIxFan; ++j) {
        ev[j] = run;
        const uint32_t b = (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
        run += k0 + j < q.n ? ((b & 0x80u) ? 1 : -1) : 0;
    }
    int32_t mn = ev[0];
#pragma unroll
    for (int j = 1; j < kIxFan; ++j) mn = min(mn, ev[j]);
#pragma unroll
    for (int j = 0; j < kIxFan; j += 8)
        *(int4*)&bm.e0[tid * kIxFan + j] =
            make_int4((ev[j] & 0xffff) | (ev[j + 1] << 16), (ev[j + 2] & 0xffff) | (ev[j + 3] << 16),
                      (ev[j + 4] & 0xffff) | (ev[j + 5] << 16), (ev[j + 6] & 0xffff) | (ev[j + 7] << 16));
    bm.m1[tid] = (int16_t)mn;
    // both searches within the thread's own positions, four bits per
    // position: the distance less one, 15 when the answer lies outside
    uint64_t nxt = 0, prv = 0;
#pragma unroll
    for (int j = 0; j < kIxFan; ++j) {
        uint32_t f = 15, b = 15;
#pragma unroll
        for (int m = kIxFan - 1; m > j; --m)
            if (ev[m] < ev[j]) f = (uint32_t)(m - j - 1);
#pragma unroll
        for (int m = 0; m < j; ++m)
            if (ev[m] <= ev[j]) b = (uint32_t)(j - m - 1);
        nxt |= (uint64_t)f << (4 * j);
        prv |= (uint64_t)b << (4 * j);
    }
    __syncthreads();
    if (tid < kIxFan) {
        int32_t x = bm.m1[tid * kIxFan];
        for (int i = 1; i < kIxFan; ++i) x = min(x, (int32_t)bm.m1[tid * kIxFan + i]);
        bm.m2[tid] = (int16_t)x;
    }
    const int32_t boff = q.boff[blockIdx.x];
    for (int pass = 0; pass < 2; ++pass) {
        const bool parent = pass == 1;
        if (tid == 0) n_work = queued = 0;
        __syncthreads();
        if (k0 < q.n) {
            const uint64_t near = parent ? prv : nxt;
            int64_t t = ix_tree_in(q, t_lo, t_hi, k0);
            int64_t s = q.offsets[t], e = q.offsets[t + 1];
            bool ok = q.valid[t] != 0;
            const bool one_tree = ok && 0 <= s && s <= k0 && k0 + kIxFan <= e && e <= q.n;
            if (one_tree) {
                // the common case: all 16 positions in one valid tree
                const int32_t base = (int32_t)(k0 - s);
#pragma unroll
                for (int j = 0; j < kIxFan; ++j) {
                    const uint32_t d = (uint32_t)(near >> (4 * j)) & 15u;
                    const bool fn = ((w[j >> 2] >> (8 * (j & 3))) & 0x80u) != 0;
                    int32_t r = -1;
                    if (!parent) {
                        if (!fn) r = base + j + 1;
                        else if (d < 15) r = base + j + 1 + (int32_t)d;
                        else work[atomicAdd(&n_work, 1)] = (uint16_t)(tid * kIxFan + j);
                    } else if (base + j > 0) {
                        if (d < 15) r = base + j - 1 - (int32_t)d;
                        else work[atomicAdd(&n_work, 1)] = (uint16_t)(tid * kIxFan + j);
                    }
                    res[tid * kIxFan + j] = r;
                }
            }
            for (int j = 0; j < kIxFan && !one_tree; ++j) {
                const int64_t k = k0 + j;
                if (k >= q.n) break;
                while (k >= e && t + 1 < q.n_trees) {
                    ++t;
                    s = q.offsets[t];
                    e = q.offsets[t + 1];
                    ok = q.valid[t] != 0;
                }
                int32_t r = -1;
                if (ok && 0 <= s && s <= k && k < e && e <= q.n) {
                    const uint32_t d = (uint32_t)(near >> (4 * j)) & 15u;
                    const uint32_t wj = j < 8 ? (j < 4 ? w[0] : w[1]) : (j < 12 ? w[2] : w[3]);
                    const bool fn = ((wj >> (8 * (j & 3))) & 0x80u) != 0;
                    if (!parent) {
                        if (!fn) r = (int32_t)(k + 1 - s);
                        else if (d < 15) r = (int32_t)(k + 1 + d - s);
                        else work[atomicAdd(&n_work, 1)] = (uint16_t)(tid * kIxFan + j);
                    } else if (k > s) {
                        if (d < 15) r = (int32_t)(k - 1 - d - s);
                        else work[atomicAdd(&n_work, 1)] = (uint16_t)(tid * kIxFan + j);
                    }
                }
                res[tid * kIxFan + j] = r;          // a listed search overwrites it
            }
        }
        __syncthreads();
        const int nw = n_work;
        for (int x = tid; x < nw; x += 256) {
            const int i = work[x];
            const int64_t k = B + i;
            const int32_t v = bm.e0[i];
            const int m = parent ? ix_lds_last_at_most(bm, i, v) : ix_lds_first_below(bm, i, v);
            const int64_t t = ix_tree_in(q, t_lo, t_hi, k);
            const int64_t s = q.offsets[t], e = q.offsets[t + 1];
            if (m >= 0) {
                const int64_t J = B + m;
                res[i] = (parent ? J >= s : J <= e) ? (int32_t)(J - s) : -1;
            } else {
                const int slot = atomicAdd(&queued, 1);
                if (slot < kIxQueue) queue[slot] = (uint16_t)i;
                else res[i] = ix_global_link(q, B, k, s, e, v + boff, parent);
            }
        }
        __syncthreads();
        const int nq = min(queued, kIxQueue);
        for (int x = tid; x < nq; x += 256) {
            const int i = queue[x];
            const int64_t t = ix_tree_in(q, t_lo, t_hi, B + i);
            res[i] = ix_global_link(q, B, B + i, q.offsets[t], q.offsets[t + 1], bm.e0[i] + boff, parent);
        }
        __syncthreads();
        int32_t* out = parent ? q.parent : q.end;
        for (int x = tid; x < here; x += 256) out[B + x] = res[x];
    }
}

// Trees [lo, hi] that scan block b may hold, for the Strahler passes: the
// per-block first trees are copied into the global min-tree's storage, free
// once ends and parents are written (with no min-tree levels the population
// has at most kIxFan positions, one block).
__device__ __forceinline__ void ix_block_trees(const IxParams& q, int64_t b, int64_t& lo, int64_t& hi)
{
    const int64_t nb = (q.n + kIxBlock - 1) / kIxBlock;
    if (q.top == 0) {
        lo = 0;
        hi = q.n_trees - 1;
        return;
    }
    lo = q.seg[b];
    hi = b + 1 < nb ? q.seg[b + 1] : q.n_trees - 1;
}

// Strahler numbers, one level per pass.  A node's number is at least k + 1
// iff its subtree holds a function whose two children both have at least k
// (numbers never decrease towards the root, and a node whose children differ
// takes the larger).  Pass k marks those functions, counts them with a prefix
// sum over positions (kept in el/boff, whose E values the ends and parents no
// longer need), and raises every function whose subtree range holds one.
__global__ __launch_bounds__(256) void k_ix_sinit(IxParams q)
{
    const int64_t k0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (k0 + 16 <= q.n && (((uintptr_t)(q.sn + k0)) & 15) == 0) {
        // 16 positions in one tree: the numbers from the opcode bytes at once
        int64_t lo, hi;
        ix_block_trees(q, k0 / kIxBlock, lo, hi);
        const int64_t t = ix_tree_in(q, lo, hi, k0);
        const int64_t s = q.offsets[t], e = q.offsets[t + 1];
        if (0 <= s && s <= k0 && k0 + 16 <= e && e <= q.n) {
            uint32_t w[4];
            ix_bytes16(q.ops, k0, q.n, w);
            const bool ok = q.valid[t] != 0;
            uint32_t v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = ok ? ((w[i] & 0x80808080u) >> 7) + 0x01010101u : 0u;
            *(uint4*)(q.sn + k0) = make_uint4(v[0], v[1], v[2], v[3]);
            return;
        }
    }
    ix_positions(
        q,
        [&](int64_t k, int64_t t, int64_t, int64_t, uint8_t op, int32_t) {
            q.sn[k] = q.valid[t] ? ((op & 0x80) ? 2 : 1) : 0;               // a function is at least 2
        },
        [&](int64_t k) { q.sn[k] = 0; });
}

// Positions of this thread's 16 that hold a function still at level: only
// they can be marked or raised, and a thread with none skips the tree lookup.
__device__ __forceinline__ uint32_t ix_at_level(const IxParams& q, int64_t k0, int level, uint32_t (&sn)[4])
{
    uint32_t ops[4];
    ix_bytes16(q.ops, k0, q.n, ops);
    ix_bytes16(q.sn, k0, q.n, sn);
    uint32_t m = 0;
    for (int j = 0; j < 16; ++j) {
        const uint32_t o = (ops[j >> 2] >> (8 * (j & 3))) & 0xffu, v = (sn[j >> 2] >> (8 * (j & 3))) & 0xffu;
        if (k0 + j < q.n && (o & 0x80u) && v == (uint32_t)level) m |= 1u << j;
    }
    return m;
}

__device__ __forceinline__ uint32_t ix_at_level(const IxParams& q, int64_t k0, int level)
{
    uint32_t sn[4];
    return ix_at_level(q, k0, level, sn);
}

// end[k0 .. k0 + 16), with four 16-byte loads where aligned (k0 + 16 <= n).
__device__ __forceinline__ void ix_ends16(const IxParams& q, int64_t k0, int32_t (&en)[kIxFan])
{
    if ((((uintptr_t)(q.end + k0)) & 15) == 0) {
        const int4* p = (const int4*)(q.end + k0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int4 v = p[i];
            en[4 * i] = v.x;
            en[4 * i + 1] = v.y;
            en[4 * i + 2] = v.z;
            en[4 * i + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kIxFan; ++i) en[i] = q.end[k0 + i];
    }
}

// For each set bit j of m, body(k0 + j, tree start, tree end), walking the
// trees from tree t = [s, e), the one holding k0.
template <class Body>
__device__ __forceinline__ void ix_each_from(const IxParams& q, int64_t k0, uint32_t m, int64_t t, int64_t s, int64_t e,
                                             Body body)
{
    while (m) {
        const int j = __ffs(m) - 1;
        m &= m - 1;
        const int64_t k = k0 + j;
        while (k >= e && t + 1 < q.n_trees) {
            ++t;
            s = q.offsets[t];
            e = q.offsets[t + 1];
        }
        if (0 <= s && s <= k && k < e && e <= q.n) body(k, s, e);
    }
}

__global__ __launch_bounds__(256) void k_ix_sflag(IxParams q, int level, int32_t* bsum)
{
    __shared__ int32_t wtot[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t base = ((int64_t)blockIdx.x * 256 + tid) * 16;
    uint32_t bits = 0;
    // a function with both children at level or more is itself at level already
    uint32_t snw[4];
    const uint32_t m = base < q.n ? ix_at_level(q, base, level, snw) : 0u;
    int64_t t = 0, s = 0, e = 0;
    if (m) {
        int64_t lo, hi;
        ix_block_trees(q, blockIdx.x, lo, hi);
        t = ix_tree_in(q, lo, hi, base);
        s = q.offsets[t];
        e = q.offsets[t + 1];
    }
    if (m && 0 <= s && s <= base && base + kIxFan < e && e <= q.n) {
        // every position and its first child in one tree: the ends and the
        // right children's numbers are loaded all at once
        int32_t en[kIxFan];
        ix_ends16(q, base, en);                                          // end[base .. base + 15]
        const int32_t en16 = q.end[base + kIxFan];
        const uint32_t sn16 = q.sn[base + kIxFan];
        uint32_t snr[kIxFan];
#pragma unroll
        for (int j = 0; j < kIxFan; ++j) {
            const int64_t r = s + (j + 1 < kIxFan ? en[j + 1] : en16);  // the right child of base + j
            snr[j] = ((m >> j) & 1u) && r > base + j + 1 && r < e ? q.sn[r] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kIxFan; ++j) {
            const uint32_t sl = j + 1 < kIxFan ? (snw[(j + 1) >> 2] >> (8 * ((j + 1) & 3))) & 0xffu : sn16;
            if (((m >> j) & 1u) && sl >= (uint32_t)level && snr[j] >= (uint32_t)level) bits |= 1u << j;
        }
    } else {
        ix_each_from(q, base, m, t, s, e, [&](int64_t k, int64_t s, int64_t e) {
            if (k + 1 < e) {
                const int64_t r = s + q.end[k + 1];                  // the right child
                if (r > k + 1 && r < e && q.sn[k + 1] >= level && q.sn[r] >= level) bits |= 1u << (int)(k - base);
            }
        });
    }
    // past the first levels most blocks mark nothing: their prefix is left
    // unwritten and read as zero
    if (!__syncthreads_or(bits != 0)) {
        if (tid == 0) {
            bsum[blockIdx.x] = 0;
            q.bempty[blockIdx.x] = 1;
        }
        return;
    }
    if (tid == 0) q.bempty[blockIdx.x] = 0;
    const int32_t run = __popc(bits);
    int32_t incl = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += wtot[i];
    const int32_t excl = wbase + incl - run;
    int32_t pre[16];
    for (int j = 0; j < 16; ++j) pre[j] = excl + __popc(bits & ((1u << j) - 1u));
    int4* dst = (int4*)(q.el + base);
    for (int j = 0; j < 2; ++j)
        dst[j] = make_int4(ix_pack16(pre[8 * j], pre[8 * j + 1]), ix_pack16(pre[8 * j + 2], pre[8 * j + 3]),
                           ix_pack16(pre[8 * j + 4], pre[8 * j + 5]), ix_pack16(pre[8 * j + 6], pre[8 * j + 7]));
    if (tid == 255) bsum[blockIdx.x] = excl + run;
}

// Marked functions before position x (x <= n): a block that marked none
// holds no prefix of its own.
__device__ __forceinline__ int32_t ix_count_before(const IxParams& q, int64_t x)
{
    const int64_t b = x / kIxBlock;
    return q.bempty[b] ? q.boff[b] : ix_e(q, x);
}

// DENSE: the first pass, where every function starts at the level, so each
// thread has several nodes to test; later passes test few nodes per thread
// and run the plain walk (the batched loads' registers would cost them
// resident waves).
template <bool DENSE>
__global__ __launch_bounds__(256) void k_ix_supd(IxParams q, int level)
{
    const int64_t k0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (k0 >= q.n) return;
    // only a node at level can rise
    uint32_t snw[4];
    const uint32_t m = ix_at_level(q, k0, level, snw);
    if (!m) return;
    int64_t lo, hi;
    ix_block_trees(q, k0 / kIxBlock, lo, hi);
    const int64_t t = ix_tree_in(q, lo, hi, k0);
    const int64_t s = q.offsets[t], e = q.offsets[t + 1];
    if (DENSE && 0 <= s && s <= k0 && k0 + kIxFan <= e && e <= q.n) {
        // all 16 positions in one tree: their ends, then the counts at the
        // subtree ends, loaded all at once; the numbers written back together
        int32_t en[kIxFan];
        ix_ends16(q, k0, en);
        int32_t cx[kIxFan];
#pragma unroll
        for (int j = 0; j < kIxFan; ++j) {
            const int64_t x = s + en[j];                                 // the subtree is [k0 + j, x)
            cx[j] = ((m >> j) & 1u) && x > k0 + j && x <= e ? ix_count_before(q, x) : INT32_MIN;
        }
        uint32_t raised = 0;
#pragma unroll
        for (int j = 0; j < kIxFan; ++j)
            if (cx[j] != INT32_MIN && cx[j] > ix_count_before(q, k0 + j)) raised |= 1u << j;
        if (!raised) return;
#pragma unroll
        for (int j = 0; j < kIxFan; ++j)
            if ((raised >> j) & 1u)
                snw[j >> 2] = (snw[j >> 2] & ~(0xffu << (8 * (j & 3)))) | ((uint32_t)(level + 1) << (8 * (j & 3)));
        if ((((uintptr_t)(q.sn + k0)) & 15) == 0) {
            *(uint4*)(q.sn + k0) = make_uint4(snw[0], snw[1], snw[2], snw[3]);
        } else {
#pragma unroll
            for (int j = 0; j < kIxFan; ++j)
                if ((raised >> j) & 1u) q.sn[k0 + j] = (uint8_t)(level + 1);
        }
        return;
    }
    ix_each_from(q, k0, m, t, s, e, [&](int64_t k, int64_t s, int64_t e) {
        const int64_t x = s + q.end[k];                              // the subtree is [k, x)
        if (x > k && x <= e && ix_count_before(q, x) > ix_count_before(q, k)) q.sn[k] = (uint8_t)(level + 1);
    });
}

hipError_t launch_strahler_init(const IxParams& q, hipStream_t s)
{
    if (q.top > 0) {
        const int64_t nb = (q.n + kIxBlock - 1) / kIxBlock;
        const int64_t bg = std::min<int64_t>(65536, std::max<int64_t>(1, (nb + 255) / 256));
        hipLaunchKernelGGL(k_ix_tfirst, dim3((unsigned)bg), dim3(256), 0, s, q, q.seg, nb);
    }
    const int64_t pg = (q.n + 16 * 256 - 1) / (16 * 256);
    hipLaunchKernelGGL(k_ix_sinit, dim3((unsigned)pg), dim3(256), 0, s, q);
    return hipGetLastError();
}

hipError_t launch_strahler_level(const IxParams& q, int level, int32_t* bsum, int64_t nb,
                                 hipStream_t s)
{
    const int64_t pg = (q.n + 16 * 256 - 1) / (16 * 256);
    hipLaunchKernelGGL(k_ix_sflag, dim3((unsigned)nb), dim3(256), 0, s, q, level, bsum);
    const hipError_t et = launch_top(q, bsum, nb, s);
    if (et != hipSuccess) return et;
    if (level == 2) hipLaunchKernelGGL(k_ix_supd<true>, dim3((unsigned)pg), dim3(256), 0, s, q, level);
    else hipLaunchKernelGGL(k_ix_supd<false>, dim3((unsigned)pg), dim3(256), 0, s, q, level);
    return hipGetLastError();
}

hipError_t launch_index(const IxParams& q, int32_t* bsum, int64_t nb, const int64_t* host_len, hipStream_t s)
{
    hipLaunchKernelGGL(k_ix_scan, dim3((unsigned)nb), dim3(256), 0, s, q, bsum);
    const hipError_t et = launch_top(q, bsum, nb, s);
    if (et != hipSuccess) return et;
    for (int l = 1; l <= q.top; ++l) {
        const int64_t len = host_len[l];
        const int64_t grid = std::min<int64_t>(65536, std::max<int64_t>(1, (len + 255) / 256));
        hipLaunchKernelGGL(k_ix_level, dim3((unsigned)grid), dim3(256), 0, s, q, l);
    }
    const int64_t tg = std::min<int64_t>(65536, std::max<int64_t>(1, (q.n_trees + 255) / 256));
    hipLaunchKernelGGL(k_ix_init, dim3((unsigned)tg), dim3(256), 0, s, q);
    const int64_t bg = std::min<int64_t>(65536, std::max<int64_t>(1, (nb + 255) / 256));
    hipLaunchKernelGGL(k_ix_tfirst, dim3((unsigned)bg), dim3(256), 0, s, q, bsum, nb);
    const int64_t pg = (q.n + 16 * 256 - 1) / (16 * 256);
    hipLaunchKernelGGL(k_ix_bytes, dim3((unsigned)pg), dim3(256), 0, s, q, (const int32_t*)bsum);
    hipLaunchKernelGGL(k_ix_trees, dim3((unsigned)tg), dim3(256), 0, s, q);
    hipLaunchKernelGGL(k_ix_links, dim3((unsigned)pg), dim3(256), 0, s, q, (const int32_t*)bsum);
    return hipGetLastError();
}

}  // namespace gpe
