/*
 * CPU oracle for tree-GP fitness evaluation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library: it is a
 * plain, slow, single-threaded restatement of what the paper's method
 * computes, used to prove the GPU results.
 *
 * Sources (W. B. Langdon, "A Trillion Genetic Programming Instructions per
 * Second", arXiv 2205.03251):
 *   - Section 3.1: trees are flattened to one opcode per node in depth-first
 *     (prefix) order; evaluation uses an explicit stack whose depth is the
 *     tree height.
 *   - Section 4.2: the whole-test-set interpreter executes every opcode on
 *     every test case; Boolean problems pack 64 test cases in one 64-bit word
 *     and evaluate them with bitwise operations.
 *   - Section 6.2 and Figure 3: bottom-up incremental evaluation.  The donor
 *     subtree is evaluated on all test cases, its values replace those of the
 *     removed subtree, and differences are propagated up the mother towards
 *     the root, re-evaluating the mother alongside, until either the child and
 *     mother agree on every test case (failed disruption propagation: the
 *     child's fitness is then the mother's) or the root is reached.
 *   - Figure 1: a child is the mother's prefix before the crossover point,
 *     the donor subtree, then the mother's suffix after the removed subtree.
 *
 * Readings where the paper is silent (each is a stated choice):
 *   - float functions ADD, SUB, MUL, PDIV; PDIV(a,b) = 1.0f when
 *     fabsf(b) < 1e-6f (compared in float32), else the IEEE quotient a/b.
 *     All arithmetic is binary32, round-to-nearest-even, no contraction, no
 *     flush of denormals.
 *   - "identical on all test cases" means every case is bit-equal or both
 *     values are NaN (Boolean: equal on every valid bit).
 *   - float fitness = sum over cases of (double)fabsf(out - y), the
 *     subtraction in float32, summed in double by a halving tree over
 *     P = max(64, next power of two >= T) slots (zero padded):
 *     s[i] += s[i+h] for h = P/2, P/4, ..., 1.
 *   - Boolean fitness = number of valid bits where out equals the target.
 *   - bit i of word w holds test case 64*w + i.
 *   - interpreted node count of an incremental evaluation = donor nodes +
 *     one per ancestor level computed for the child.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------ tree format */

static int is_func(uint8_t b) { return (b & 0x80) != 0; }

/* Section 3.1 flattened prefix tree.  Valid iff every byte is a known
 * function (0x80..0x83, arity 2) or a terminal below n_inputs (arity 0), the
 * running sum of (arity - 1) stays >= 0 before the last node and ends at -1. */
int orc_validate(const uint8_t* ops, int64_t n, int n_inputs)
{
    if (n < 1) return ORC_EINVAL;
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint8_t b = ops[i];
        if (is_func(b)) {
            if ((b & 0x7f) > 3) return ORC_EINVAL;
            s += 1;
        } else {
            if ((int)b >= n_inputs) return ORC_EINVAL;
            s -= 1;
        }
        if (i < n - 1 && s < 0) return ORC_EINVAL;
    }
    return s == -1 ? ORC_OK : ORC_EINVAL;
}

/* End (exclusive) of the subtree rooted at i: scan forward until the number
 * of open child slots drops to zero. */
int64_t orc_subtree_end(const uint8_t* ops, int64_t n, int64_t i)
{
    int64_t open = 1, j = i;
    while (open > 0) {
        if (j >= n) return ORC_EINVAL;
        open += is_func(ops[j]) ? 1 : -1;
        ++j;
    }
    return j;
}

/* end[] of every node in one right-to-left pass with a stack of node ids. */
static int all_ends(const uint8_t* ops, int64_t n, int64_t* end)
{
    int64_t* st = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!st) return ORC_ENOMEM;
    int64_t sp = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        if (is_func(ops[i])) {
            sp -= 2;                 /* st[sp+1] = left child (i+1), st[sp] = right child */
            end[i] = end[st[sp]];
        } else {
            end[i] = i + 1;
        }
        st[sp++] = i;
    }
    free(st);
    return ORC_OK;
}

/* Section 3.1: the subtree end of every node (the same right-to-left pass). */
int orc_all_ends(const uint8_t* ops, int64_t n, int64_t* end)
{
    if (n < 1) return ORC_EINVAL;
    return all_ends(ops, n, end);
}

/* Section 3.1: the parent of every node, -1 at the root.  Reading the prefix
 * form left to right, a function opens two child positions; each node takes
 * the next open position of the most recently read function that still has
 * one, so a stack of functions with positions left is enough. */
int orc_parents(const uint8_t* ops, int64_t n, int64_t* parent)
{
    if (n < 1) return ORC_EINVAL;
    int64_t* st = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int* left = (int*)malloc(sizeof(int) * (size_t)n);
    if (!st || !left) {
        free(st);
        free(left);
        return ORC_ENOMEM;
    }
    int64_t sp = 0;
    for (int64_t j = 0; j < n; ++j) {
        parent[j] = sp > 0 ? st[sp - 1] : -1;
        if (sp > 0 && --left[sp - 1] == 0) --sp;
        if (is_func(ops[j])) {
            st[sp] = j;
            left[sp] = 2;
            ++sp;
        }
    }
    free(st);
    free(left);
    return ORC_OK;
}

/* Strahler number of every node: 1 at a terminal; at a function the larger
 * of its children's numbers, plus one when they are equal.  Section 6.2 notes
 * that the operands may be evaluated in any order; evaluating the child with
 * the larger number first, a stack evaluation of the subtree needs as many
 * slots as this number.  Right-to-left pass with a stack of values. */
int orc_strahler(const uint8_t* ops, int64_t n, int32_t* out)
{
    if (n < 1) return ORC_EINVAL;
    int32_t* st = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!st) return ORC_ENOMEM;
    int64_t sp = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        int32_t v = 1;
        if (is_func(ops[i])) {
            int32_t l = st[--sp];          /* left child's number (pushed last) */
            int32_t r = st[--sp];
            v = l == r ? l + 1 : (l > r ? l : r);
        }
        out[i] = v;
        st[sp++] = v;
    }
    free(st);
    return ORC_OK;
}

/* ------------------------------------------------------- float32 semantics */

static float op_f32(int f, float a, float b)
{
    switch (f) {
    case 0: return a + b;
    case 1: return a - b;
    case 2: return a * b;
    default: return (fabsf(b) < 1e-6f) ? 1.0f : a / b;
    }
}

static int same_f32(float a, float b)
{
    if (isnan(a) && isnan(b)) return 1;
    uint32_t ua, ub;
    memcpy(&ua, &a, 4);
    memcpy(&ub, &b, 4);
    return ua == ub;
}

/* Value of the subtree ops[0..n) on one test case t, by scanning the prefix
 * array right to left with an explicit stack: a terminal pushes its input, a
 * function pops its left operand (top) then its right operand and pushes the
 * result.  This is the RPN evaluation of Section 3.1 read backwards. */
static float eval_case_f32(const uint8_t* ops, int64_t n, const float* inputs, int64_t T,
                           int64_t t, float* stack)
{
    int64_t sp = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        uint8_t b = ops[i];
        if (is_func(b)) {
            float l = stack[--sp];
            float r = stack[--sp];
            stack[sp++] = op_f32(b & 3, l, r);
        } else {
            stack[sp++] = inputs[(int64_t)b * T + t];
        }
    }
    return stack[0];
}

/* Section 4.2: run the tree on every test case.  inputs is [n_inputs][T]. */
int orc_eval_f32(const uint8_t* ops, int64_t n, int n_inputs, const float* inputs, int64_t T,
                 float* out)
{
    if (orc_validate(ops, n, n_inputs) != ORC_OK || T < 0) return ORC_EINVAL;
    float* stack = (float*)malloc(sizeof(float) * (size_t)(n + 1));
    if (!stack) return ORC_ENOMEM;
    for (int64_t t = 0; t < T; ++t) out[t] = eval_case_f32(ops, n, inputs, T, t, stack);
    free(stack);
    return ORC_OK;
}

/* Every node's output vector: node_out is [n][T]; node i's row is the value
 * of the subtree rooted at i, evaluated as a tree of its own. */
int orc_eval_f32_nodes(const uint8_t* ops, int64_t n, int n_inputs, const float* inputs,
                       int64_t T, float* node_out)
{
    if (orc_validate(ops, n, n_inputs) != ORC_OK) return ORC_EINVAL;
    int64_t* end = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    float* stack = (float*)malloc(sizeof(float) * (size_t)(n + 1));
    if (!end || !stack) { free(end); free(stack); return ORC_ENOMEM; }
    all_ends(ops, n, end);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = 0; t < T; ++t)
            node_out[i * T + t] = eval_case_f32(ops + i, end[i] - i, inputs, T, t, stack);
    free(end);
    free(stack);
    return ORC_OK;
}

/* Fitness: sum of |out - y| over the T cases, by the fixed halving tree. */
double orc_fitness_f32(const float* out, const float* y, int64_t T)
{
    int64_t P = 64;
    while (P < T) P *= 2;
    double* s = (double*)calloc((size_t)P, sizeof(double));
    if (!s) return NAN;
    for (int64_t t = 0; t < T; ++t) {
        float e = out[t] - y[t];
        s[t] = (double)fabsf(e);
    }
    for (int64_t h = P / 2; h >= 1; h /= 2)
        for (int64_t i = 0; i < h; ++i) s[i] = s[i] + s[i + h];
    double r = s[0];
    free(s);
    return r;
}

/* ------------------------------------------------------- Boolean semantics */

static uint64_t op_bool(int f, uint64_t a, uint64_t b)
{
    switch (f) {
    case 0: return a & b;
    case 1: return a | b;
    case 2: return ~(a & b);
    default: return ~(a | b);
    }
}

static uint64_t valid_mask(int64_t w, int64_t T)
{
    int64_t lo = w * 64;
    if (lo + 64 <= T) return ~(uint64_t)0;
    if (lo >= T) return 0;
    return ((uint64_t)1 << (T - lo)) - 1;
}

/* Section 4.2 bitwise evaluation: 64 test cases per word.  inputs is
 * [n_inputs][W]; out is [W]. */
int orc_eval_bool(const uint8_t* ops, int64_t n, int n_inputs, const uint64_t* inputs, int64_t W,
                  uint64_t* out)
{
    if (orc_validate(ops, n, n_inputs) != ORC_OK || W < 0) return ORC_EINVAL;
    uint64_t* stack = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    if (!stack) return ORC_ENOMEM;
    for (int64_t w = 0; w < W; ++w) {
        int64_t sp = 0;
        for (int64_t i = n - 1; i >= 0; --i) {
            uint8_t b = ops[i];
            if (is_func(b)) {
                uint64_t l = stack[--sp];
                uint64_t r = stack[--sp];
                stack[sp++] = op_bool(b & 3, l, r);
            } else {
                stack[sp++] = inputs[(int64_t)b * W + w];
            }
        }
        out[w] = stack[0];
    }
    free(stack);
    return ORC_OK;
}

/* One test case, one bit: the textbook scalar Boolean evaluation, used to
 * pin the packed evaluator by brute force over all input combinations. */
int orc_eval_bool_bit(const uint8_t* ops, int64_t n, int n_inputs, const int* bits)
{
    if (orc_validate(ops, n, n_inputs) != ORC_OK) return ORC_EINVAL;
    int* stack = (int*)malloc(sizeof(int) * (size_t)(n + 1));
    int64_t sp = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        uint8_t b = ops[i];
        if (is_func(b)) {
            int l = stack[--sp], r = stack[--sp], v;
            switch (b & 3) {
            case 0: v = l && r; break;
            case 1: v = l || r; break;
            case 2: v = !(l && r); break;
            default: v = !(l || r); break;
            }
            stack[sp++] = v;
        } else {
            stack[sp++] = bits[b] ? 1 : 0;
        }
    }
    int r = stack[0];
    free(stack);
    return r;
}

int64_t orc_fitness_bool(const uint64_t* out, const uint64_t* target, int64_t W, int64_t T)
{
    int64_t hits = 0;
    for (int64_t w = 0; w < W; ++w) {
        uint64_t m = ~(out[w] ^ target[w]) & valid_mask(w, T);
        while (m) { hits += (int64_t)(m & 1u); m >>= 1; }
    }
    return hits;
}

/* ------------------------------------------------------------- population */

/* Full evaluation and fitness (Section 4.2) of the listed trees of a
 * population, tree which[k] being ops[offsets[which[k]] .. offsets[which[k] + 1]),
 * one after another: the loop a caller would otherwise write around
 * orc_eval_f32 and orc_fitness_f32 (orc_eval_bool and orc_fitness_bool).
 * fit[k] receives tree which[k]'s fitness. */
int orc_population_f32(const uint8_t* ops, const int64_t* offsets, const int64_t* which, int64_t n_which,
                       int n_inputs, const float* inputs, const float* y, int64_t T, double* fit)
{
    float* out = (float*)malloc(sizeof(float) * (size_t)T);
    if (!out) return ORC_ENOMEM;
    for (int64_t k = 0; k < n_which; ++k) {
        const int64_t s = offsets[which[k]], e = offsets[which[k] + 1];
        int rc = orc_eval_f32(ops + s, e - s, n_inputs, inputs, T, out);
        if (rc != ORC_OK) {
            free(out);
            return rc;
        }
        fit[k] = orc_fitness_f32(out, y, T);
    }
    free(out);
    return ORC_OK;
}

int orc_population_bool(const uint8_t* ops, const int64_t* offsets, const int64_t* which, int64_t n_which,
                        int n_inputs, const uint64_t* inputs, const uint64_t* target, int64_t W, int64_t T,
                        int64_t* fit)
{
    uint64_t* out = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)W);
    if (!out) return ORC_ENOMEM;
    for (int64_t k = 0; k < n_which; ++k) {
        const int64_t s = offsets[which[k]], e = offsets[which[k] + 1];
        int rc = orc_eval_bool(ops + s, e - s, n_inputs, inputs, W, out);
        if (rc != ORC_OK) {
            free(out);
            return rc;
        }
        fit[k] = orc_fitness_bool(out, target, W, T);
    }
    free(out);
    return ORC_OK;
}

/* -------------------------------------------------------------- crossover */

/* Figure 1: child = P[0:c] ++ D ++ P[end(c):].  Returns the child's length,
 * or ORC_EINVAL when c is out of range or cap is too small. */
int64_t orc_splice(const uint8_t* P, int64_t n, int64_t c, const uint8_t* D, int64_t nd,
                   uint8_t* child, int64_t cap)
{
    if (c < 0 || c >= n) return ORC_EINVAL;
    int64_t e = orc_subtree_end(P, n, c);
    if (e < 0) return ORC_EINVAL;
    int64_t len = c + nd + (n - e);
    if (len > cap) return ORC_EINVAL;
    memcpy(child, P, (size_t)c);
    memcpy(child + c, D, (size_t)nd);
    memcpy(child + c + nd, P + e, (size_t)(n - e));
    return len;
}

/* ------------------------------------------------- incremental evaluation */

/* Path from the root down to node c: path[0] = root, path[len-1] = c. */
static int64_t root_path(const uint8_t* ops, const int64_t* end, int64_t c, int64_t* path)
{
    int64_t len = 0, v = 0;
    for (;;) {
        path[len++] = v;
        if (v == c) return len;
        int64_t l = v + 1, r = end[l];
        v = (c < r) ? l : r;
    }
}

/* Section 6.2 / Figure 3, float32.  The donor D is evaluated on every test
 * case and compared with the mother's value at the crossover point c.  While
 * they differ, each ancestor a_k of c is re-evaluated for the child with the
 * path operand replaced and, alongside, for the mother; the sibling subtree
 * at each level is evaluated once and serves both.  The first level where
 * child and mother agree on every case is the stop level (0 = at c itself);
 * -1 means the difference reached the root.  After a stop the child's values
 * are the mother's, so its root vector is the mother's root vector.
 *
 * Outputs: root_out[T], *stop_level, *interpreted (donor nodes + ancestor
 * levels computed for the child before the stop), *fitness. */
int orc_incremental_f32(const uint8_t* P, int64_t n, int64_t c, const uint8_t* D, int64_t nd,
                        int n_inputs, const float* inputs, const float* y, int64_t T,
                        float* root_out, int32_t* stop_level, int64_t* interpreted, double* fitness)
{
    if (orc_validate(P, n, n_inputs) != ORC_OK || orc_validate(D, nd, n_inputs) != ORC_OK)
        return ORC_EINVAL;
    if (c < 0 || c >= n || T < 1) return ORC_EINVAL;
    int64_t* end = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* path = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    float* child = (float*)malloc(sizeof(float) * (size_t)T);
    float* mother = (float*)malloc(sizeof(float) * (size_t)T);
    float* sib = (float*)malloc(sizeof(float) * (size_t)T);
    if (!end || !path || !child || !mother || !sib) {
        free(end); free(path); free(child); free(mother); free(sib);
        return ORC_ENOMEM;
    }
    all_ends(P, n, end);
    int64_t len = root_path(P, end, c, path);

    orc_eval_f32(D, nd, n_inputs, inputs, T, child);
    orc_eval_f32(P + c, end[c] - c, n_inputs, inputs, T, mother);
    int64_t interp = nd;

    int agreed = 1;
    for (int64_t t = 0; t < T; ++t) agreed &= same_f32(child[t], mother[t]);
    int32_t level = agreed ? 0 : -1;

    for (int64_t k = 1; k < len; ++k) {
        int64_t a = path[len - 1 - k];           /* ancestor k levels above c */
        int64_t below = path[len - k];           /* its child on the path */
        int64_t l = a + 1, r = end[l];
        int64_t s = (below == l) ? r : l;        /* sibling subtree */
        orc_eval_f32(P + s, end[s] - s, n_inputs, inputs, T, sib);
        int f = P[a] & 3;
        for (int64_t t = 0; t < T; ++t) {
            float m = (below == l) ? op_f32(f, mother[t], sib[t]) : op_f32(f, sib[t], mother[t]);
            if (level < 0) {
                float v = (below == l) ? op_f32(f, child[t], sib[t]) : op_f32(f, sib[t], child[t]);
                child[t] = v;
            }
            mother[t] = m;
        }
        if (level < 0) {
            interp += 1;
            agreed = 1;
            for (int64_t t = 0; t < T; ++t) agreed &= same_f32(child[t], mother[t]);
            if (agreed) level = (int32_t)k;
        }
    }
    for (int64_t t = 0; t < T; ++t) root_out[t] = (level >= 0) ? mother[t] : child[t];
    *stop_level = level;
    *interpreted = interp;
    *fitness = orc_fitness_f32(root_out, y, T);
    free(end); free(path); free(child); free(mother); free(sib);
    return ORC_OK;
}

/* Section 6.2 / Figure 3, Boolean (W words of packed cases, T valid bits). */
int orc_incremental_bool(const uint8_t* P, int64_t n, int64_t c, const uint8_t* D, int64_t nd,
                         int n_inputs, const uint64_t* inputs, const uint64_t* target, int64_t W,
                         int64_t T, uint64_t* root_out, int32_t* stop_level, int64_t* interpreted,
                         int64_t* fitness)
{
    if (orc_validate(P, n, n_inputs) != ORC_OK || orc_validate(D, nd, n_inputs) != ORC_OK)
        return ORC_EINVAL;
    if (c < 0 || c >= n || W < 1) return ORC_EINVAL;
    int64_t* end = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* path = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    uint64_t* child = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)W);
    uint64_t* mother = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)W);
    uint64_t* sib = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)W);
    if (!end || !path || !child || !mother || !sib) {
        free(end); free(path); free(child); free(mother); free(sib);
        return ORC_ENOMEM;
    }
    all_ends(P, n, end);
    int64_t len = root_path(P, end, c, path);

    orc_eval_bool(D, nd, n_inputs, inputs, W, child);
    orc_eval_bool(P + c, end[c] - c, n_inputs, inputs, W, mother);
    int64_t interp = nd;
    int agreed = 1;
    for (int64_t w = 0; w < W; ++w) agreed &= ((child[w] ^ mother[w]) & valid_mask(w, T)) == 0;
    int32_t level = agreed ? 0 : -1;

    for (int64_t k = 1; k < len; ++k) {
        int64_t a = path[len - 1 - k];
        int64_t below = path[len - k];
        int64_t l = a + 1, r = end[l];
        int64_t s = (below == l) ? r : l;
        orc_eval_bool(P + s, end[s] - s, n_inputs, inputs, W, sib);
        int f = P[a] & 3;
        for (int64_t w = 0; w < W; ++w) {
            uint64_t m = (below == l) ? op_bool(f, mother[w], sib[w]) : op_bool(f, sib[w], mother[w]);
            if (level < 0)
                child[w] = (below == l) ? op_bool(f, child[w], sib[w]) : op_bool(f, sib[w], child[w]);
            mother[w] = m;
        }
        if (level < 0) {
            interp += 1;
            agreed = 1;
            for (int64_t w = 0; w < W; ++w)
                agreed &= ((child[w] ^ mother[w]) & valid_mask(w, T)) == 0;
            if (agreed) level = (int32_t)k;
        }
    }
    for (int64_t w = 0; w < W; ++w) root_out[w] = (level >= 0) ? mother[w] : child[w];
    *stop_level = level;
    *interpreted = interp;
    *fitness = orc_fitness_bool(root_out, target, W, T);
    free(end); free(path); free(child); free(mother); free(sib);
    return ORC_OK;
}

/* ------------------------------------------------------------ selection */

/* Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC 2011), from its definition: ten rounds; each
 * multiplies counter words 0 and 2 by the two round multipliers, mixes the
 * high halves with words 1 and 3 and the round key, and the key is bumped by
 * the two Weyl constants after each round.  The random draws of a generation
 * are not part of the paper's method; this generator is one both sides
 * implement from its published definition. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform integer in [0, n) from one 32-bit word: floor(u * n / 2^32), for
 * n < 2^32. */
uint64_t orc_uniform(uint32_t u, uint64_t n) { return ((uint64_t)u * n) >> 32; }

/* Word j of stream s for index i at generation g: word j mod 4 of Philox with
 * counter (i, g, s, j / 4) and key (seed low, seed high). */
uint32_t orc_draw(uint64_t seed, int64_t i, int64_t g, int s, int64_t j)
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)g, (uint32_t)s, (uint32_t)(j / 4)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox(ctr, key, out);
    return out[j % 4];
}

/* Tournament of size k over n fitness values (Section 6.3): k draws uniform
 * with replacement; a candidate replaces the current winner only if strictly
 * better (so ties keep the earlier draw).  Float fitness is an error (lower is
 * better, NaN worst); Boolean fitness counts hits (higher is better). */
int64_t orc_tournament_f64(const double* fit, int64_t n, int k, uint64_t seed, int64_t i, int64_t g, int s)
{
    int64_t best = (int64_t)orc_uniform(orc_draw(seed, i, g, s, 0), (uint64_t)n);
    for (int j = 1; j < k; ++j) {
        int64_t c = (int64_t)orc_uniform(orc_draw(seed, i, g, s, j), (uint64_t)n);
        double a = fit[c], b = fit[best];
        if (!isnan(a) && (isnan(b) || a < b)) best = c;
    }
    return best;
}

int64_t orc_tournament_i64(const int64_t* fit, int64_t n, int k, uint64_t seed, int64_t i, int64_t g, int s)
{
    int64_t best = (int64_t)orc_uniform(orc_draw(seed, i, g, s, 0), (uint64_t)n);
    for (int j = 1; j < k; ++j) {
        int64_t c = (int64_t)orc_uniform(orc_draw(seed, i, g, s, j), (uint64_t)n);
        if (fit[c] > fit[best]) best = c;
    }
    return best;
}
