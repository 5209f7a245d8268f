/*
 * gpeval -- data-parallel fitness evaluation of tree GP individuals on
 * AMD MI355X (gfx950).  C ABI; plain pointers and sizes only.
 *
 * Method: W. B. Langdon, "A Trillion Genetic Programming Instructions per
 * Second" (arXiv 2205.03251).
 *   - Trees are flattened to one opcode byte per node in depth-first prefix
 *     order, or reverse Polish order (Section 3.1).
 *   - Every opcode is executed on every test case (Section 4.2); Boolean
 *     problems pack 64 test cases per 64-bit word (Section 4.2).
 *   - A child made by subtree crossover is evaluated bottom-up from the
 *     crossover point: the inserted subtree is evaluated on all test cases,
 *     then the path to the root is re-evaluated, stopping at the first node
 *     whose values equal the mother's on every test case (failed disruption
 *     propagation; Section 6.2, Figure 3).  The child need not exist: the
 *     mother, the point and the donor subtree suffice (Section 6.3).
 *
 * Opcode byte encoding (both layouts):
 *   0..63      terminal: index of an input variable (< n_inputs)
 *   0x80 | f   binary function f, left operand = first child in prefix order
 *     GP_F32:  0x80 ADD, 0x81 SUB, 0x82 MUL, 0x83 PDIV
 *              PDIV(a, b) = 1.0f if fabsf(b) < 1e-6f (float32 compare) else a / b
 *     GP_BOOL: 0x80 AND, 0x81 OR, 0x82 NAND, 0x83 NOR   (bitwise on 64-bit words)
 *   float32 arithmetic is IEEE binary32, round to nearest even, no fused
 *   multiply-add, denormals kept, divide correctly rounded.
 *
 * Test cases: float32 inputs are [n_inputs][T] and the target is [T].
 * Boolean inputs are [n_inputs][W] uint64 words and the target is [W],
 * W = ceil(T / 64); test case i is bit i % 64 of word i / 64.
 *
 * Fitness: float32 = sum over cases of (double)fabsf(out - y), the
 * subtraction in float32, summed in double by a halving tree over
 * P = max(64, next power of two >= T) zero-padded slots
 * (s[i] += s[i + h] for h = P/2, ..., 1).  Boolean = number of cases where
 * out equals the target.  Results are bit-exact and independent of launch
 * shape, batch composition and concurrent work.
 *
 * Ownership: host arrays passed in are copied during the call.  With
 * GP_DEVICE_PTR, pointer arguments are device pointers and are read or
 * written in stream order on the context's stream.  Populations, cases,
 * parent caches and workspaces are owned by the library until gp_free or
 * gp_destroy.  Output buffers belong to the caller.  A context is used by
 * one thread at a time; the server runs its own threads.
 *
 * Errors: every call returns GP_OK or a negative code and writes nothing to
 * its outputs on error; gp_last_error gives the reason.  There is no CPU
 * evaluation path: without a usable GPU, calls that evaluate return
 * GP_EDEVICE.
 */
#ifndef GPEVAL_H
#define GPEVAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_ctx gp_ctx;
typedef int64_t gp_handle;

enum {
    GP_OK = 0,
    GP_EINVAL = -1,     /* malformed tree, bad index, size or type mismatch */
    GP_ENOMEM = -2,     /* host or device allocation failed */
    GP_EBUDGET = -3,    /* request exceeds the context's HBM budget */
    GP_EDEVICE = -4,    /* HIP error, or no usable GPU */
    GP_ENOTFOUND = -5,  /* no parent cache (spine) for this parent and point */
    GP_EBUSY = -6       /* server job not finished yet */
};

enum { GP_F32 = 0, GP_BOOL = 1 };          /* value type */
enum { GP_PREFIX = 0, GP_POSTFIX = 1 };    /* load layout */

/* flags */
#define GP_DEVICE_PTR 0x1u   /* pointer arguments are device pointers */
#define GP_ASYNC      0x2u   /* return once enqueued (needs GP_DEVICE_PTR outputs) */
#define GP_PER_TREE   0x4u   /* one launch per tree instead of one batched launch */
#define GP_NO_GRAPH   0x8u   /* launch kernels directly, no captured graph replay */
#define GP_KEEP_TREES 0x10u  /* gp_load_population: keep the trees' bytes in device
                                memory (charged to the budget) for gp_splice_children */
#define GP_COEVAL     0x20u  /* gp_evaluate_incremental_batch: re-evaluate the mother
                                alongside each child instead of reading parent caches */
#define GP_DEVICE_COMPILE 0x40u  /* gp_load_population: compile the trees on the device */

typedef struct gp_stats {
    double device_ms;          /* HIP-event time on the context stream (0 with GP_ASYNC) */
    double kernel_ms;          /* HIP-event time of the interpreter launch alone (GP_NO_GRAPH
                                  full evaluations), of the copy kernel
                                  (gp_splice_children); 0 otherwise */
    double wall_ms;            /* call entry to return */
    int64_t equivalent_ops;    /* sum of nodes x T over every tree or child scored
                                  (gp_splice_children: bytes written) */
    int64_t interpreted_ops;   /* nodes actually executed x T */
    int64_t launches;          /* kernel launches or graph replays issued */
    int32_t variant;           /* interpreter variant index (gp_variant_name) */
    int32_t waves_per_cu;      /* the interpreter launch's resident workgroups (one wave each) were
                                  capped at this many per compute unit; 0: all that fit */
} gp_stats;

typedef struct gp_inc_result {
    int32_t stop_level;        /* 0: at the crossover point; k: k-th ancestor; -1: root reached */
    int32_t reserved;
    int64_t child_nodes;       /* nodes of the (never built) child */
    int64_t interpreted_nodes; /* donor nodes + ancestor levels re-evaluated */
} gp_inc_result;

typedef struct gp_pop_info {
    int64_t n_trees;
    int64_t total_nodes;
    int64_t n_chunks;          /* work units after chunking */
    int64_t n_instructions;    /* interpreter instructions over all chunks */
    int64_t n_records;         /* parent-cache vectors recorded per evaluation */
    int64_t n_spines;          /* (tree, point) pairs with a parent cache */
    int64_t device_bytes;      /* HBM held by this population */
    int32_t max_stack;         /* deepest evaluation-stack slot used + 1 */
    int32_t chunk_nodes;       /* chunk size target used */
    int64_t max_code_len;      /* longest chunk program, in instruction words */
} gp_pop_info;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context may hold (0 = 90% of the device's free memory).
 * hip_stream: a hipStream_t to run on, or NULL for a stream of its own. */
int gp_create(int device, uint64_t hbm_budget_bytes, void* hip_stream, gp_ctx** out);
void gp_destroy(gp_ctx* ctx);
/* Reason for the last failed call on this context (static text if ctx is NULL). */
const char* gp_last_error(const gp_ctx* ctx);
/* Device memory currently held by the context, in bytes. */
uint64_t gp_memory_used(const gp_ctx* ctx);

/* ------------------------------------------------------------------- data */

/* Register a test-case set (Section 4.2).  vtype GP_F32: inputs [n_inputs][T]
 * float32, target [T] float32.  GP_BOOL: inputs [n_inputs][ceil(T/64)] uint64,
 * target [ceil(T/64)] uint64.  1 <= n_inputs <= 64, 1 <= T <= 16384 (float)
 * or T <= 2^18 (Boolean).  GP_DEVICE_PTR: inputs and target are device
 * pointers. */
int gp_set_cases(gp_ctx* ctx, int vtype, int n_inputs, int64_t n_cases, const void* inputs,
                 const void* target, uint32_t flags, gp_handle* cases_out);

/* Load a population of flattened trees (Section 3.1): tree i is
 * ops[offsets[i] .. offsets[i+1]) in the given layout.  Trees are validated
 * (every byte a known opcode, terminals < n_inputs, arity count closes exactly
 * at the last byte), compiled to register-stack programs and cut into chunks.
 * record_points (may be NULL): for tree i, the crossover points
 * record_points[record_offsets[i] .. record_offsets[i+1]) (node indices in
 * the given layout) whose parent caches every full evaluation must record,
 * for later incremental evaluation of children made at those points.
 * chunk_nodes: target nodes per chunk (0 = automatic).  flags: GP_KEEP_TREES
 * keeps a device copy of ops for gp_splice_children.  GP_DEVICE_COMPILE
 * (prefix layout only) validates and compiles the trees on the device: the
 * same checks, and programs, chunk tables and parent-cache records identical
 * byte for byte to the host compiler's (gp_population_dump shows them), in
 * passes over the flattened trees (Section 3.1) instead of a host pass per
 * tree; it also re-chunks on the device when gp_autotune tries other chunk
 * sizes.  GP_DEVICE_PTR: ops and offsets are device pointers (ops any
 * alignment), compiled on the device as with GP_DEVICE_COMPILE; the library
 * keeps a host copy of the trees (for co-evaluation and re-chunking) either
 * way.  record_points and record_offsets are host arrays in every case.
 * Other bits are ignored. */
int gp_load_population(gp_ctx* ctx, int vtype, int layout, int n_inputs, int64_t n_trees,
                       const uint8_t* ops, const int64_t* offsets, const int64_t* record_points,
                       const int64_t* record_offsets, int64_t chunk_nodes, uint32_t flags,
                       gp_handle* pop_out);

int gp_population_info(gp_ctx* ctx, gp_handle pop, gp_pop_info* out);

/* The compiled form of a loaded population, for inspection and for checking
 * two compilations against each other: one byte string of sections, each an
 * int64 byte count followed by its bytes, in this order: header (8 int64:
 * trees, chunks, instruction words, records, stack slots, chunk target,
 * nodes, layout); instruction words (+1 trailing word); chunk table (32 bytes
 * per chunk: int64 code offset, int32 code length, parent, output slot, input
 * offset, record base, input count); chunk input slots (int32); per chunk its
 * input count and its tree (int32); per tree its record base (int64); the
 * scheduling order of leaf chunks ((priority, chunk) int64 pairs); spines (5
 * int64: tree, vector at the point, first level, levels, nodes removed);
 * spine keys ((tree << 32 | point, spine) int64 pairs, sorted); spine levels
 * (4 int32: function | side, sibling vector, ancestor vector, 0); per tree
 * its large subtrees (count, then (node, end) pairs); its chunk roots (count,
 * then (node, end, vector slot) triples); its chunks (count, then per chunk
 * code offset, length, parent, root node, nodes, longest chain, subtree end,
 * reused code offset, records, vector slot, reused vector slot, input count,
 * inputs, all int64); per tree its stack slots (int32) and nodes (int64).
 * out == NULL: *size receives the byte count only.  GP_EINVAL when cap is
 * smaller than that. */
int gp_population_dump(gp_ctx* ctx, gp_handle pop, uint8_t* out, int64_t cap, int64_t* size);

/* Index a population of prefix trees on the device (the flattened form of
 * Section 3.1): tree t is ops[offsets[t] .. offsets[t+1]).  Every argument
 * array is device memory owned by the caller; ops must be 16-byte aligned.
 * Outputs: valid[t] = 1 when tree t passes the same check as
 * gp_validate_tree (every byte a function 0x80..0x83 or a terminal below
 * n_inputs; the count of open child positions stays positive until the last
 * node and closes there), else 0.  For each node k of a valid tree,
 * end[k] = the end (exclusive) of k's subtree and parent[k] = k's parent,
 * both as indices within the tree, parent -1 at the root; every node of an
 * invalid tree gets -1 in both.  strahler (may be NULL; n_nodes bytes of
 * device memory): the Strahler number of every node of a valid tree (1 at a
 * terminal; at a function the larger of its children's, plus one when they
 * are equal), 0 in an invalid tree.  Section 6.2 lets operands be evaluated
 * in either order; evaluating the larger-numbered child first, a subtree
 * needs as many stack slots as its number.  1 <= n_trees <= n_nodes <=
 * 2^31 - 2, where n_nodes = offsets[n_trees].  Runs on the context stream and
 * returns when done; device_ms (may be NULL) receives its HIP-event time.
 * GP_EINVAL when offsets do not run from 0 to n_nodes without decreasing
 * (outputs then undefined), or on bad sizes or pointers. */
int gp_index_trees(gp_ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops, const int64_t* offsets,
                   int64_t n_nodes, int32_t* valid, int32_t* end, int32_t* parent, uint8_t* strahler,
                   double* device_ms);

/* gp_index_trees for callers that cannot allocate device memory (serving
 * loops that must not call hipMalloc, harnesses that forbid allocation):
 * the same arguments, outputs and errors, for populations of at most
 * GP_INDEX_NOALLOC_MAX_NODES nodes (GP_EINVAL beyond, nothing written).  Its
 * working memory is a fixed array of about 18 MB in device memory that the
 * library holds on every device a context was created on, from gp_create
 * until the process ends; the call allocates nothing and frees nothing.  All
 * calls on one device share that array: calls that overlap in time on one
 * device, from any contexts or threads, race and give undefined results.
 * Like gp_index_trees it waits for its result (it is not for stream
 * capture). */
#define GP_INDEX_NOALLOC_MAX_NODES 4194304
int gp_index_trees_noalloc(gp_ctx* ctx, int n_inputs, int64_t n_trees, const uint8_t* ops,
                           const int64_t* offsets, int64_t n_nodes, int32_t* valid, int32_t* end,
                           int32_t* parent, uint8_t* strahler, double* device_ms);

/* Release a population or case set (and any cache or graph tied to it). */
int gp_free(gp_ctx* ctx, gp_handle h);

/* ------------------------------------------------------------- evaluation */

/* Full evaluation (Section 4.2) of every tree on every case of `cases`, in
 * one persistent work-stealing launch (or one launch per tree with
 * GP_PER_TREE).  Records the parent caches requested at load time.
 * The crossover points whose parent caches are recorded are fixed when the
 * population is loaded (gp_load_population's record_points), not passed
 * here: recording is compiled into the programs, a STORE after the point,
 * each ancestor and each ancestor's other operand.  New points therefore
 * need a new load; a child at a point that was not recorded is evaluated
 * with GP_COEVAL instead (gp_evaluate_incremental_batch), which needs no
 * cache.
 * root_out: [n_trees][T] float32 or [n_trees][W] uint64, or NULL.
 * fitness_out: [n_trees] double (GP_F32) or int64 (GP_BOOL), or NULL.
 * st: optional statistics. */
int gp_evaluate_full(gp_ctx* ctx, gp_handle pop, gp_handle cases, uint32_t flags, void* root_out,
                     void* fitness_out, gp_stats* st);

/* Bottom-up incremental evaluation with failed-disruption-propagation stop
 * (Section 6.2, Figure 3) of n_children children.  Child i is tree parent[i]
 * of `pop` with the subtree at node point[i] (index in the load layout)
 * replaced by donor i = donor_ops[donor_offsets[i] .. donor_offsets[i+1])
 * (same layout and value type as the population).  The population must have
 * been fully evaluated on `cases` since it was loaded, with point[i] among
 * its record points (else GP_ENOTFOUND).  Outputs as gp_evaluate_full, per
 * child; res[i] gets the stop level and counts (host pointer, may be NULL).
 * GP_COEVAL: the paper's own form (Section 6.2): the mother is re-evaluated
 * alongside each child from the point up, the sibling subtrees of the path
 * evaluated on demand, so any node may be the point (no record points); the
 * population must be in prefix layout and fully evaluated on `cases` (her root
 * vector and fitness are the child's on a stop).  Results and stop levels are
 * those of the cached form; res[i].interpreted_nodes then counts the nodes
 * actually executed: donor + the parts of the removed and sibling subtrees
 * that were evaluated (float32: parts that are whole chunks of the mother are
 * read from her last full evaluation instead) + two per level walked (child
 * and mother).  Runs synchronously (no GP_ASYNC). */
int gp_evaluate_incremental_batch(gp_ctx* ctx, gp_handle pop, gp_handle cases, int64_t n_children,
                                  const int64_t* parent, const int64_t* point,
                                  const uint8_t* donor_ops, const int64_t* donor_offsets,
                                  uint32_t flags, void* root_out, void* fitness_out,
                                  gp_inc_result* res, gp_stats* st);

/* One child; same as a batch of one. */
int gp_evaluate_incremental(gp_ctx* ctx, gp_handle pop, gp_handle cases, int64_t parent,
                            int64_t point, const uint8_t* donor_ops, int64_t donor_len,
                            uint32_t flags, void* root_out, void* fitness_out, gp_inc_result* res);

/* Build children on the device (Section 5, Figure 1).  Child i is tree
 * parent[i] of `pop` with the subtree at node point[i] replaced by donor i =
 * donor_ops[donor_offsets[i] .. donor_offsets[i+1]), all in the population's
 * layout: the mother's nodes before that subtree, the donor, then her nodes
 * after it (in reverse Polish order the subtree ends at point[i]).  The
 * population must have been loaded with GP_KEEP_TREES, and point[i] must be
 * one of tree parent[i]'s record points, whose parent cache gives the extent
 * of the removed subtree (else GP_ENOTFOUND); no evaluation is needed.
 * Donors are host arrays and are validated as trees.
 * child_offsets: host int64[n_children + 1], filled on success: child i is
 * child_ops[child_offsets[i] .. child_offsets[i+1]).  child_ops: NULL to
 * obtain the offsets only; otherwise child_cap bytes of room (GP_EINVAL if
 * the children need more), a device pointer on the context's GPU with
 * GP_DEVICE_PTR, else host memory (staged through device memory charged to
 * the budget).  The bytes are copied by one kernel at memory speed;
 * st->kernel_ms is its duration and st->equivalent_ops the bytes written. */
int gp_splice_children(gp_ctx* ctx, gp_handle pop, int64_t n_children, const int64_t* parent,
                       const int64_t* point, const uint8_t* donor_ops, const int64_t* donor_offsets,
                       uint32_t flags, uint8_t* child_ops, int64_t child_cap, int64_t* child_offsets,
                       gp_stats* st);

/* ------------------------------------------------------------- generations */

typedef struct gp_evolve_cfg {
    int64_t generations;       /* >= 1 */
    int32_t tournament;        /* tournament size k >= 1 */
    int32_t reserved;
    uint64_t seed;             /* key of the random draws (Philox-4x32-10) */
    int64_t first_generation;  /* counter of the first generation's draws */
} gp_evolve_cfg;

typedef struct gp_gen_stats {
    double best_f64;           /* GP_F32: lowest error among the children (NaN if all NaN) */
    int64_t best_i64;          /* GP_BOOL: most hits among the children */
    int64_t children;          /* N, the population size */
    int64_t built;             /* children built: drawn as a parent by the next generation (all in the last) */
    int64_t child_nodes;       /* nodes of all N children */
    int64_t built_nodes;       /* nodes of the children built */
    int64_t interpreted_nodes; /* nodes executed to score the children */
    double ms;                 /* wall time of the generation, of which: */
    double ms_score;           /*   drawing parents and points, scoring the children, drawing the next tournaments */
    double ms_build;           /*   building the drawn children: bytes on the device and the host, programs */
    double ms_eval;            /*   evaluating the built children (the next generation's chunk values): chunks
                                    reused from a parent take that parent chunk's values, the rest run */
    int64_t chunks;            /* chunks of the built children */
    int64_t chunks_evaluated;  /* of which compiled anew and run (the others are reused) */
} gp_gen_stats;

typedef struct gp_gen_child {
    int64_t mother, father;    /* slots of the previous generation */
    int64_t point;             /* crossover point in the mother (prefix index) */
    int64_t donor_node;        /* the donor is the father's subtree at this node */
    int64_t nodes;             /* child size */
    double fitness_f64;        /* GP_F32 */
    int64_t fitness_i64;       /* GP_BOOL */
    int32_t stop_level;        /* of its incremental evaluation */
    int32_t drawn;             /* times drawn as a parent by the next generation */
} gp_gen_child;

/* Generational GP with fitness first (Sections 5, 6.2 and 6.3).  Generation g
 * (g = cfg->first_generation, ...) makes N = population size children: child
 * i gets as mother and father the winners of two tournaments over the previous
 * generation's fitness, a crossover point uniform over the mother's nodes and,
 * as donor, the father's subtree at a node uniform over his nodes; the draws
 * are word j of Philox-4x32-10 with counter (i, g, stream, j / 4) and key
 * seed (streams 0 mother, 1 father, 2 point and donor node; uniform over n:
 * floor(word * n / 2^32); k draws with replacement, the strictly better wins:
 * lower error with NaN worst, or more hits).  Every child is scored by
 * co-evaluation with its mother before any is built; then the tournaments of
 * generation g + 1 are drawn over the children's fitness and only the
 * children drawn there are built (all of them in the last generation), on the
 * device, and evaluated as the next population.  `pop` must be a prefix
 * population fully evaluated on `cases`; its trees and results are not changed
 * (a device copy of its trees may be kept with it).  *out_pop receives
 * the last generation (N trees, evaluated on `cases`).  stats: host array of
 * cfg->generations entries, or NULL.  children: host array of
 * cfg->generations * N records, or NULL. */
int gp_evolve(gp_ctx* ctx, gp_handle pop, gp_handle cases, const gp_evolve_cfg* cfg, gp_gen_stats* stats,
              gp_gen_child* children, gp_handle* out_pop);

/* The results of a population's last full evaluation (gp_evaluate_full,
 * or the evaluation gp_evolve ends with), without evaluating again: root_out
 * [n_trees][T] float32 or [n_trees][W] uint64, fitness_out [n_trees] double
 * or int64 (either may be NULL), host memory or, with GP_DEVICE_PTR, device
 * memory.  GP_ENOTFOUND if that evaluation was not on `cases`. */
int gp_population_results(gp_ctx* ctx, gp_handle pop, gp_handle cases, uint32_t flags, void* root_out,
                          void* fitness_out);

/* The trees of a population, as loaded (host memory): offsets_out gets
 * n_trees + 1 entries; ops_out (may be NULL to get the offsets only) gets
 * offsets_out[n_trees] bytes, at most ops_cap. */
int gp_population_ops(gp_ctx* ctx, gp_handle pop, uint8_t* ops_out, int64_t ops_cap, int64_t* offsets_out);

/* Fitness of n given output vectors ([n][T] float32 or [n][W] uint64) against
 * the target of `cases`, in the fixed order described above. */
int gp_fitness(gp_ctx* ctx, gp_handle cases, const void* outputs, int64_t n, uint32_t flags,
               void* fitness_out);

/* ------------------------------------------------------------- tuning */

/* Interpreter variants compiled into the library (test cases per lane K and
 * evaluation-stack slots S).  gp_variant_name returns NULL past the last. */
const char* gp_variant_name(int variant);
int gp_variant_count(void);

/* Time each variant on this population and case set (and, for a population
 * loaded without a fixed chunk size, each candidate chunk size, recompiling
 * it in place), then, at the best chunk size, each variant again with fewer
 * resident waves per compute unit (a full evaluation is one persistent launch
 * whose length is set by its longest chains of chunks; fewer waves sharing a
 * SIMD shorten those chains' issue).  The fastest (variant, waves per CU) is
 * kept for later calls with the same value type, case-count bucket and
 * tree-size bucket; its variant index and time are returned. */
int gp_autotune(gp_ctx* ctx, gp_handle pop, gp_handle cases, int* best_variant, double* best_ms);

/* Force a variant for later calls (-1 = automatic choice). */
int gp_set_variant(gp_ctx* ctx, int variant);

/* The autotuner's choices kept across processes, as JSON lines, one object per
 * (value type, case-count bucket, tree-size bucket) tuned on a device:
 *   {"device": "gfx950:256", "vtype": 0, "t_bucket": 10, "s_bucket": 22,
 *    "variant": "f32t_k8_s10", "waves_per_cu": 0, "chunk_nodes": 2048}
 * (buckets: ceil(log2 T) and ceil(log2 mean tree size); the device is the
 * architecture and compute-unit count).  gp_tuning_save writes every choice this
 * context holds.  gp_tuning_load adds the file's choices for this device (lines
 * for other devices or for variants this library lacks are skipped); later
 * evaluations use them, and gp_autotune applies a loaded choice without timing
 * the alternatives, recompiling an automatically chunked population at the
 * saved chunk size.  Errors: GP_ENOTFOUND if the file cannot be read, GP_EINVAL
 * for a malformed line or out-of-range value (nothing is loaded then) or a file
 * that cannot be written. */
int gp_tuning_save(gp_ctx* ctx, const char* path);
int gp_tuning_load(gp_ctx* ctx, const char* path);

/* Cap the resident waves per compute unit of later full-evaluation launches:
 * -1 = the tuned cap (none before gp_autotune), 0 = all that fit, n > 0 = at
 * most n.  Returns GP_EINVAL below -1. */
int gp_set_launch_width(gp_ctx* ctx, int waves_per_cu);

/* ------------------------------------------------------------- serving */

typedef struct gp_server_cfg {
    int32_t n_streams;          /* batches that may be in flight at once (>= 1) */
    int32_t max_batch_jobs;     /* jobs merged into one launch at most */
    int32_t prep_threads;       /* host threads compiling arriving trees */
    int32_t device_compile_nodes; /* > 0: FULL jobs of at least this many nodes are compiled on
                                     the device, on their prep thread's stream, into the same
                                     programs as on the host; 0 or less: every job on the host
                                     (the default: its prep threads use otherwise idle cores,
                                     while device compilation contends with the batches in flight) */
    uint64_t budget_bytes;      /* HBM admitted at once (0 = the context budget) */
} gp_server_cfg;

enum { GP_JOB_FULL = 0, GP_JOB_INCREMENTAL = 1 };

typedef struct gp_job {
    int32_t kind;               /* GP_JOB_FULL or GP_JOB_INCREMENTAL */
    int32_t layout;             /* GP_PREFIX or GP_POSTFIX */
    gp_handle cases;            /* case set (fixes vtype and T) */
    const uint8_t* ops;         /* FULL: the tree; INCREMENTAL: the donor */
    int64_t n_ops;
    const int64_t* record_points; /* FULL: points to keep parent caches for (may be NULL) */
    int64_t n_record_points;
    int64_t parent_ticket;      /* INCREMENTAL: ticket of a finished FULL job kept resident */
    int64_t point;              /* INCREMENTAL: crossover point in the parent */
    int32_t keep_resident;      /* FULL: keep tree and caches on the device as a parent */
    int32_t reserved;
} gp_job;

typedef struct gp_job_result {
    double fitness_f64;         /* GP_F32 fitness */
    int64_t fitness_i64;        /* GP_BOOL fitness */
    int32_t stop_level;         /* INCREMENTAL: as gp_inc_result */
    int32_t status;             /* GP_OK or an error code */
    int64_t interpreted_nodes;
    double latency_ms;          /* submit to completion */
    double queue_ms;            /* submit to admission */
    double prep_ms;             /* submit to ready: validation and compilation on a prep thread */
    double launch_ms;           /* admission to enqueued: the host work of the job's batch
                                   (assembly and upload, donor compilation, launches) */
    double run_ms;              /* enqueued to completion seen: device work and copy-out */
    int64_t root_bytes;         /* size of the job's output vector */
    int32_t device_compiled;    /* FULL: 1 when its tree was compiled on the device */
    int32_t reserved;
} gp_job_result;

int gp_server_start(gp_ctx* ctx, const gp_server_cfg* cfg);
/* Copies the job's arrays; returns a ticket. GP_EBUDGET if the job alone
 * exceeds the budget. */
int gp_server_submit(gp_ctx* ctx, const gp_job* job, int64_t* ticket);
/* GP_EBUSY until the job is done; then fills *out.  root_out (may be NULL)
 * receives the job's output vector (host memory, root_cap bytes of room:
 * T float32 values or ceil(T / 64) uint64 words of its case set); GP_EINVAL
 * if root_cap is smaller, and then nothing is written and the result stays
 * available.  The result of a job that is not a resident parent is handed
 * out once. */
int gp_server_poll(gp_ctx* ctx, int64_t ticket, gp_job_result* out, void* root_out, int64_t root_cap);
/* Drop a resident parent kept by keep_resident.  GP_EBUSY while the parent
 * is not done, or while any incremental child submitted against it is not
 * done (whether it is still being compiled, waiting or running). */
int gp_server_release(gp_ctx* ctx, int64_t ticket);
int gp_server_stop(gp_ctx* ctx);

/* ------------------------------------------------------------- measurement */

/* Counter calibration, not part of evaluation: one launch of n_waves
 * single-wave workgroups in which every wave runs iters x 32 VALU
 * instructions of one class on eight independent registers (0 v_add_f32,
 * 1 v_mul_f32, 2 v_fma_f32, 3 v_rcp_f32, 4 v_cndmask_b32, 5 v_cmp_lt_f32,
 * 6 v_max3_f32, 7 v_mov_b32, 8 v_add_f32 and v_rcp_f32 alternating,
 * 9 v_add_f32 and v_cmp_lt_f32 alternating), so that hardware counters and
 * issue rates can be read against a known instruction count (two runs that
 * differ only in iters differ by exactly 32 x iters VALU instructions per
 * wave).  device_ms (may be NULL) receives the launch's HIP-event time. */
int gp_valu_calibration(gp_ctx* ctx, int cls, int64_t n_waves, int64_t iters, double* device_ms);

/* ----------------------------------------------- host-only inspection */

/* Compile one prefix tree on the host only (no GPU needed) and return the
 * interpreter program, for tests of the compiler.  code_out receives the
 * 32-bit instructions of all chunks (at most code_cap), chunk_out 4 int64 per
 * chunk (code offset, code length, parent chunk or -1, number of child chunks
 * it loads), inputs_out the child chunk ids each chunk loads, chunk after
 * chunk, in LOAD payload order.  Chunks come children first; the last one is
 * the root.  threads (1..64; values outside are clamped) host threads may
 * compile a tree of 200000 nodes or more; the program does not depend on
 * it.  Returns the number of chunks, GP_EINVAL for a malformed tree or
 * GP_ENOMEM when a capacity is too small; *n_code gets the code length and
 * *max_stack the register-stack slots used. */
int64_t gp_inspect_program(int vtype, int n_inputs, const uint8_t* ops, int64_t n,
                           int64_t chunk_nodes, int stack_slots, int threads, uint32_t* code_out,
                           int64_t code_cap, int64_t* chunk_out, int64_t chunk_cap,
                           int32_t* inputs_out, int64_t inputs_cap, int64_t* n_code,
                           int32_t* max_stack);

/* The program of a crossover child built from its parents' programs
 * (Section 5: the mother's prefix up to `point`, the father's subtree at
 * `donor_node`, the mother's suffix after the subtree at `point`), on the host
 * only, for tests: both parents are compiled whole (chunk_nodes, stack_slots
 * as for gp_inspect_program, index of subtrees of index_min_size >= 1 nodes;
 * the mother records parent caches for the n_mother_records points listed,
 * as gp_load_population's record_points do), then the child reuses every
 * chunk of theirs off the crossover path that records nothing and
 * recompiles the rest.  Outputs as for gp_inspect_program, except that
 * chunk_out receives 6 int64 per chunk (code offset, code length, parent,
 * number of child chunks, root node, end of the root's subtree, in the
 * child's numbering), big_out 2 int64 per subtree of at least index_min_size
 * nodes (node, end; sorted by node), *n_big their number and *n_reused the
 * number of chunks whose code was taken from a parent.  Returns the number of
 * chunks, GP_EINVAL for malformed trees or points, GP_ENOMEM when a capacity
 * is too small. */
int64_t gp_inspect_child_program(int vtype, int n_inputs, const uint8_t* mother, int64_t n_mother,
                                 int64_t point, const int64_t* mother_records,
                                 int64_t n_mother_records, const uint8_t* father, int64_t n_father,
                                 int64_t donor_node, int64_t chunk_nodes, int stack_slots,
                                 int64_t index_min_size, uint32_t* code_out, int64_t code_cap,
                                 int64_t* chunk_out, int64_t chunk_cap, int32_t* inputs_out,
                                 int64_t inputs_cap, int64_t* big_out, int64_t big_cap,
                                 int64_t* n_code, int32_t* max_stack, int64_t* n_big,
                                 int64_t* n_reused);

/* Validate one tree (prefix layout) on the host: GP_OK or GP_EINVAL. */
int gp_validate_tree(int vtype, int n_inputs, const uint8_t* ops, int64_t n);

/* The path that co-evaluation walks (Section 6.2), on the host, for tests:
 * for node c of a prefix tree with terminals below 64, levels_out receives 4
 * int64 per ancestor, nearest first: the ancestor's index, the sibling
 * subtree's first index and end (exclusive), and f | 4 when the path operand
 * is the right one.  *removed_end gets the end of c's subtree.  The search
 * uses an index of the subtrees with at least index_min_size nodes (0: no
 * index); the result does not depend on it.  Returns the number of ancestors,
 * GP_EINVAL for a malformed tree or c out of range, or GP_ENOMEM when
 * level_cap is too small. */
int64_t gp_inspect_path(const uint8_t* ops, int64_t n, int64_t c, int64_t index_min_size, int64_t* levels_out,
                        int64_t level_cap, int64_t* removed_end);

#ifdef __cplusplus
}
#endif
#endif /* GPEVAL_H */
