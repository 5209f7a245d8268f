// Host-side tree compiler of the gpeval library: validation, layout
// conversion, evaluation-order choice, chunking and parent-cache (spine)
// planning.  Pure C++ (no HIP); the runtime uploads what it produces.
//
// A tree is flattened in prefix order, one opcode byte per node (Section 3.1
// of the paper).  Trees are side-effect free, so any evaluation order gives
// the same values (Section 6.2).  The compiler uses that freedom: it
// evaluates the child needing more stack first (Ershov / Sethi-Ullman order),
// so the register stack needs at most about log2(n) slots instead of the
// tree height, and it folds terminal operands into their parent's
// instruction.  Non-commutative operations whose right operand is evaluated
// first get a "reversed" instruction that still computes op(left, right).
#pragma once
#include <cstdint>
#include <utility>
#include <string>
#include <vector>

namespace gpe {

// ---------------------------------------------------------------- opcodes
constexpr uint8_t kFuncBit = 0x80;
constexpr int kMaxInputs = 64;

// ------------------------------------------------------ instruction words
// One 32-bit word per instruction:
//   bits 0..1   f      function (ADD/SUB/MUL/PDIV or AND/OR/NAND/NOR)
//   bits 2..4   mode   operand sources (below)
//   bits 5..9   d      evaluation-stack slot the result goes to
//   bits 10..31 payload
// Modes ("x" = a terminal operand folded into the instruction):
//   XX    st[d] = f(x_a, x_b)            float: x = input 0; Boolean: payload = a | b << 11
//   XS    st[d] = f(x, st[d])            Boolean: payload = input index (f symmetric)
//   SX    st[d] = f(st[d], x)            float only
//   SS    st[d] = f(st[d], st[d+1])      left operand evaluated first
//   RS    st[d] = f(st[d+1], st[d])      right operand evaluated first
//   PUSH  st[d] = input[payload]
//   LOAD  st[d] = output of child chunk number `payload` of this chunk
//   STORE record st[d] into parent-cache slot rec_base + payload
// Every chunk's code ends with the word kEndWord (mode STORE, f = 1, d = 0),
// which no other instruction uses: the register-indexed dispatch loop stops
// there; the counted loop treats it as a no-op.
enum Mode : uint32_t { M_XX = 0, M_XS = 1, M_SX = 2, M_SS = 3, M_RS = 4, M_PUSH = 5, M_LOAD = 6, M_STORE = 7 };
constexpr int kPayloadShift = 10;
constexpr uint32_t kKeyMask = 0x3ffu;
constexpr uint32_t kMaxPayload = (1u << 22) - 1;
constexpr int kMaxStackSlots = 32;
// A child built from its parents' chunks: a subtree of at least this many
// nodes hanging off the path from the crossover point to the root is
// compiled as a chunk of its own (see compose_child).
constexpr int64_t kPathSiblingChunk = 64;

inline uint32_t ins_word(uint32_t f, uint32_t mode, uint32_t d, uint32_t payload)
{
    return f | (mode << 2) | (d << 5) | (payload << kPayloadShift);
}
constexpr uint32_t kEndWord = 1u | (7u << 2);

struct Chunk {
    int64_t code_off = 0;        // offset in TreeProg::code
    int64_t code_len = 0;
    int32_t parent = -1;         // local chunk id, -1 for the tree root chunk
    int64_t root_node = 0;       // prefix index of the chunk's root
    int64_t nodes = 0;           // tree nodes evaluated by this chunk
    int64_t path_nodes = 0;      // nodes on the longest chunk chain from here to the tree root
    int64_t end_node = -1;       // end of the root's subtree (with CompileOptions::index_min_size)
    int64_t dev_src = -1;        // >= 0: the code is not in TreeProg::code but at this word
                                 // offset of an already uploaded program (see compose_child)
    bool stores = false;         // records parent caches (STORE words)
    int64_t vec_slot = -1;       // its vector slot in its population (chunks kept for children)
    int64_t src_vec = -1;        // reused (dev_src >= 0): the vector slot of the chunk it copies in the
                                 // population it comes from; its last values are this chunk's values
    std::vector<int32_t> inputs; // local chunk ids read by LOAD payload 0, 1, ...
};

// Source of a cached vector: >= 0 a record slot (local to the tree),
// < 0 the input vector -(src + 1).
struct SpineLevel {
    int32_t fside;    // f | (path operand is the right one) << 2
    int32_t sib;      // sibling subtree's vector
    int32_t par;      // the mother's vector at this ancestor
};

struct Spine {
    int64_t point = 0;           // prefix index of the crossover point
    int32_t at_point = 0;        // the mother's vector at the point
    int64_t child_nodes_removed = 0;  // nodes of the subtree at the point
    std::vector<SpineLevel> levels;   // ancestors, nearest first
};

// (node, end of its subtree) within one tree; trees hold fewer than 2^31 nodes.
using SubtreeEnd = std::pair<int32_t, int32_t>;

struct TreeProg {
    std::vector<uint32_t> code;
    std::vector<Chunk> chunks;   // children before parents; the last is the root chunk
    int32_t max_stack = 0;       // highest slot used + 1
    int64_t n_records = 0;       // parent-cache vectors this tree records
    std::vector<Spine> spines;
    std::vector<SubtreeEnd> big_ends;   // see CompileOptions::index_min_size
};

struct CompileOptions {
    int vtype = 0;               // 0 float32, 1 Boolean
    int n_inputs = 1;
    int64_t chunk_nodes = 4096;  // target nodes per chunk
    int stack_slots = 16;        // register-stack slots available
    int64_t index_min_size = 0;  // > 0: list (node, end) of subtrees this large, sorted by node
    int threads = 1;             // threads for compiling a large tree (same program for any count)
};

// Section 3.1 format check of one prefix array.
bool validate_prefix(const uint8_t* ops, int64_t n, int n_inputs, std::string* why);

// Reverse Polish to prefix.  post_to_pre[i] = prefix index of postfix node i.
bool postfix_to_prefix(const uint8_t* post, int64_t n, int n_inputs, std::vector<uint8_t>* pre,
                       std::vector<int64_t>* post_to_pre, std::string* why);

// The path from node c of a validated prefix tree up to the root, for
// co-evaluating a child with its mother (Section 6.2): the removed subtree is
// [c, removed_end); level k (k = 1 for c's parent, the last level for the
// root) applies function f of ancestor `node`, with the path operand on the
// right when `right`, and the other operand is the sibling subtree
// [sib_begin, sib_end), a contiguous slice of the tree.
struct PathLevel {
    int64_t node;
    int64_t sib_begin, sib_end;
    int32_t f;
    int32_t right;
};
// Subtree ends of every node whose subtree has at least min_size nodes, as
// (node, end) pairs sorted by node: an index that lets path_to_root skip
// large subtrees.  One pass over the tree.
void big_subtree_ends(const uint8_t* ops, int64_t n, int64_t min_size,
                      std::vector<SubtreeEnd>* out);
// `big` is that index for the same tree (any min_size; smaller subtrees are
// scanned).  Cost: the first-operand subtrees along the path that the index
// does not cover, instead of the whole tree.
// End of node x's subtree, from the index when listed, else by scanning.
int64_t subtree_end_indexed(const uint8_t* ops, int64_t n, int64_t x, const std::vector<SubtreeEnd>& big);
void path_to_root(const uint8_t* ops, int64_t n, int64_t c, const std::vector<SubtreeEnd>& big,
                  std::vector<PathLevel>* levels, int64_t* removed_end);

// A tree in which some subtrees are chunks compiled already: each of them is
// collapsed to one leaf that LOADs that chunk.  Chunk ids in the output
// (inputs, parent) are then final ids: id_base + k for the k-th chunk compiled
// here, opaque[v] for the collapsed leaf v.  Nodes are reported in the full
// tree's numbering: node v of the collapsed tree is node_map[v] of the full
// tree (node_map has n + 1 entries, the last the full tree's size), and the
// index of large subtrees uses full sizes.  path_nodes is left to the caller.
struct Collapsed {
    const int32_t* opaque;       // per node: -1, or the chunk id of a collapsed leaf
    const int64_t* node_map;
    int32_t id_base;
    const uint8_t* cut_at = nullptr;  // per node (may be null): 1 = a function node that roots a chunk
                                      // of its own whatever its size
};

// Compile one validated prefix tree.  points: crossover points (prefix
// indices) whose parent caches must be recorded.  ext (may be null): per
// node, -1 or the row of the input matrix that a terminal node stands for; such
// a node is pushed from that row instead of being read as its input.
// col (may be null; then no points): collapsed subtrees, as above.
bool compile_tree(const uint8_t* ops, int64_t n, const CompileOptions& opt, const int64_t* points,
                  int64_t n_points, TreeProg* out, std::string* why, const int32_t* ext = nullptr,
                  const Collapsed* col = nullptr);

// A compiled tree kept with its population, for building children from it:
// its bytes, its chunks (children first, the root chunk last, each with its
// subtree end; code_off is the word offset of the chunk's code in the
// population's uploaded program), its index of large subtrees and stack use.
struct SrcTree {
    const uint8_t* ops;
    int64_t n;
    const Chunk* chunks;
    int64_t n_chunks;
    const std::vector<SubtreeEnd>* big;
    int32_t max_stack;
};

// The program of a crossover child (Section 5: the mother's prefix, the
// subtree [d, d_end) of the father, the mother's suffix after the removed
// subtree [c, c_end)) built from its parents' programs instead of compiling
// it whole.  A chunk whose subtree neither holds nor lies in the removed
// subtree is the mother's chunk unchanged; a chunk inside the donor subtree is
// the father's; both keep their code where it is (Chunk::dev_src = its word
// offset there).  Only the chunks on the path from c to the root, the
// father's chunk holding d and chunks that record parent caches are compiled
// again, as a tree in which the reused chunks are collapsed leaves.  child: the child's bytes (n_child).
// The index of large subtrees (opt.index_min_size > 0, required) comes from
// the parents' indexes and the recompiled part.  Each chunk's code computes
// the same values as a whole compilation would; the chunking differs only
// on the path.
bool compose_child(const SrcTree& m, int64_t c, int64_t c_end, const SrcTree& f, int64_t d, int64_t d_end,
                   const uint8_t* child, int64_t n_child, const CompileOptions& opt, TreeProg* out,
                   std::string* why);

}  // namespace gpe
