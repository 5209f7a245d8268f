"""Seeded synthetic inputs for tree-GP fitness evaluation (tests and benchmarks).

This module is shared by the CPU oracle's tests and by the GPU library's tests
and benchmark.  It holds no evaluation arithmetic: it draws tree shapes, opcode
labels, crossover points, donor subtrees and test-case data from numpy's seeded
PCG64 generator, and writes down the two problem targets (the sextic
polynomial and even parity) that define what a tree is scored against.

Opcode byte encoding (one byte per node, prefix order, left child first):
  0..63        terminal: index of an input variable
  0x80 | f     binary function f
    float32:   0x80 ADD, 0x81 SUB, 0x82 MUL, 0x83 PDIV (protected divide)
    Boolean:   0x80 AND, 0x81 OR,  0x82 NAND, 0x83 NOR
The flattened prefix layout is the paper's linear tree representation
(Section 3.1); the byte values are this project's choice.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F_ADD, F_SUB, F_MUL, F_PDIV = 0x80, 0x81, 0x82, 0x83
B_AND, B_OR, B_NAND, B_NOR = 0x80, 0x81, 0x82, 0x83
FUNCS = np.array([0x80, 0x81, 0x82, 0x83], dtype=np.uint8)

VT_F32, VT_BOOL = 0, 1


def rng_for(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- populations
@dataclass
class Population:
    """Concatenated prefix arrays: tree i is ops[offsets[i]:offsets[i+1]]."""
    ops: np.ndarray                      # uint8
    offsets: np.ndarray                  # int64, len = n_trees + 1
    vtype: int = VT_F32
    n_inputs: int = 1

    @property
    def n_trees(self) -> int:
        return len(self.offsets) - 1

    def tree(self, i: int) -> np.ndarray:
        return self.ops[self.offsets[i]:self.offsets[i + 1]]

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)


def pack(trees, vtype=VT_F32, n_inputs=1) -> Population:
    sizes = np.array([len(t) for t in trees], dtype=np.int64)
    offsets = np.zeros(len(trees) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    ops = np.concatenate([np.asarray(t, dtype=np.uint8) for t in trees]) if trees else np.zeros(0, np.uint8)
    return Population(ops, offsets, vtype, n_inputs)


def subtree_end(tree: np.ndarray, i: int, max_len: int | None = None) -> int:
    """First index past the subtree rooted at i (arity scan of a prefix array).
    With max_len, returns -1 when the subtree is longer than max_len."""
    n = len(tree)
    j, open_ = i, 1
    stop = n if max_len is None else min(n, i + max_len)
    step = 4096
    while j < stop:
        blk = tree[j:min(stop, j + step)]
        run = open_ + np.cumsum(np.where(blk & 0x80, 1, -1), dtype=np.int64)
        hit = np.flatnonzero(run == 0)
        if len(hit):
            return j + int(hit[0]) + 1
        open_ = int(run[-1])
        j += len(blk)
        step = min(step * 4, 1 << 24)
    if max_len is not None and j < n:
        return -1
    raise ValueError("truncated prefix array")


def subtree_ends(tree: np.ndarray) -> np.ndarray:
    """end[i] for every node, by one right-to-left pass (structural only)."""
    n = len(tree)
    end = np.empty(n, dtype=np.int64)
    stack = []
    for i in range(n - 1, -1, -1):
        if tree[i] & 0x80:
            stack.pop()                 # left child
            r = stack.pop()             # right child
            end[i] = end[r]
        else:
            end[i] = i + 1
        stack.append(i)
    return end


# ------------------------------------------------- ramped half-and-half (cfg0)
def _grow(rng, depth, max_depth, full, funcs, n_terms, out):
    # root (depth 0) is always a function; below max depth "grow" draws
    # uniformly from functions and terminals together, "full" draws functions.
    if depth == max_depth:
        out.append(int(rng.integers(n_terms)))
        return
    if depth == 0 or full:
        out.append(int(funcs[rng.integers(len(funcs))]))
    else:
        k = int(rng.integers(len(funcs) + n_terms))
        if k >= len(funcs):
            out.append(k - len(funcs))
            return
        out.append(int(funcs[k]))
    _grow(rng, depth + 1, max_depth, full, funcs, n_terms, out)
    _grow(rng, depth + 1, max_depth, full, funcs, n_terms, out)


def ramped_half_and_half(seed: int, n_trees: int = 100, min_depth: int = 2, max_depth: int = 6,
                         n_terms: int = 1, max_nodes: int = 200, vtype: int = VT_F32) -> Population:
    """Koza's ramped half-and-half: equal numbers of trees per depth in
    [min_depth, max_depth], half "full" and half "grow" (root = depth 0)."""
    rng = rng_for(seed)
    depths = list(range(min_depth, max_depth + 1))
    trees = []
    for i in range(n_trees):
        d = depths[(i // 2) % len(depths)] if n_trees < 2 * len(depths) else depths[i * len(depths) // n_trees]
        full = (i % 2 == 0)
        out: list[int] = []
        _grow(rng, 0, d, full, FUNCS, n_terms, out)
        assert len(out) <= max_nodes
        trees.append(np.array(out, dtype=np.uint8))
    return pack(trees, vtype, n_terms)


# --------------------------------------------------- uniformly shaped trees
def sized_tree(rng: np.random.Generator, n: int, n_terms: int = 1, funcs=FUNCS) -> np.ndarray:
    """A binary tree with n nodes (n odd), shape uniform over all such trees.

    Cycle lemma: a random arrangement of (n-1)/2 "+1" steps (functions) and
    (n+1)/2 "-1" steps (terminals) has exactly one rotation whose proper
    prefix sums stay >= 0; it starts just after the first position where the
    prefix sum is minimal.  Labels are uniform over functions / terminals.
    """
    if n < 1 or n % 2 == 0:
        raise ValueError("binary trees have an odd node count")
    steps = np.full(n, -1, dtype=np.int8)
    steps[: (n - 1) // 2] = 1
    steps = rng.permutation(steps)
    m = int(np.argmin(np.cumsum(steps, dtype=np.int64)))
    steps = np.roll(steps, -(m + 1))
    is_f = steps > 0
    ops = np.empty(n, dtype=np.uint8)
    nf = int(is_f.sum())
    ops[is_f] = np.asarray(funcs, dtype=np.uint8)[rng.integers(len(funcs), size=nf)]
    ops[~is_f] = rng.integers(n_terms, size=n - nf).astype(np.uint8)
    return ops


def log_uniform_odd(rng: np.random.Generator, lo: int, hi: int, size=None):
    """Odd integers, log-uniform over [lo, hi]."""
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))
    v = np.floor(v).astype(np.int64)
    v = np.clip(v, lo, hi)
    v = v | 1
    v = np.where(v > hi, v - 2, v)
    return v


def sized_population(seed: int, n_trees: int, lo: int, hi: int, n_terms: int = 1,
                     vtype: int = VT_F32, threads: int = 1) -> Population:
    """n_trees uniformly shaped trees with log-uniform odd sizes in [lo, hi].
    Tree i draws from its own seed stream, so the result does not depend on
    how many threads build it."""
    rng = rng_for(seed)
    sizes = log_uniform_odd(rng, lo, hi, n_trees)
    seqs = np.random.SeedSequence(seed).spawn(n_trees)

    def one(i):
        return sized_tree(np.random.default_rng(seqs[i]), int(sizes[i]), n_terms)

    if threads > 1 and n_trees > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            trees = list(ex.map(one, range(n_trees)))
    else:
        trees = [one(i) for i in range(n_trees)]
    return pack(trees, vtype, n_terms)


# ------------------------------------------------------------ test cases
def sextic(x: np.ndarray) -> np.ndarray:
    """Target y = x^6 - 2x^4 + x^2 in float32, evaluated as the fixed tree
    ((s*(s*s)) - ((s*s) + (s*s))) + s with s = x*x."""
    x = np.asarray(x, dtype=np.float32)
    s = x * x
    return ((s * (s * s)) - ((s * s) + (s * s))) + s


def sextic_tree() -> np.ndarray:
    """The same target as a GP tree over x (prefix bytes), so that a correct
    interpreter scores it exactly 0."""
    s = [F_MUL, 0, 0]
    ss = [F_MUL] + s + s
    t = [F_ADD, F_SUB, F_MUL] + s + ss + [F_ADD] + ss + ss + s
    return np.array(t, dtype=np.uint8)


@dataclass
class FloatCases:
    x: np.ndarray          # [n_inputs][T] float32
    y: np.ndarray          # [T] float32

    @property
    def T(self) -> int:
        return self.y.shape[0]


def float_cases(seed: int, T: int) -> FloatCases:
    rng = rng_for(seed)
    x = rng.uniform(-1.0, 1.0, T).astype(np.float32)
    return FloatCases(x[None, :].copy(), sextic(x))


@dataclass
class BoolCases:
    inputs: np.ndarray     # [k][W] uint64
    target: np.ndarray     # [W] uint64
    T: int


def bool_cases(k: int) -> BoolCases:
    """All 2^k input combinations, combination i at bit i%64 of word i//64;
    input j is bit j of i; target is even parity (true iff an even number of
    inputs are 1)."""
    T = 1 << k
    W = (T + 63) // 64
    i = np.arange(W * 64, dtype=np.uint64)
    bits = np.zeros((k, W * 64), dtype=np.uint64)
    for j in range(k):
        bits[j] = (i >> np.uint64(j)) & np.uint64(1)
    par = np.zeros(W * 64, dtype=np.uint64)
    for j in range(k):
        par ^= bits[j]
    even = (par == 0).astype(np.uint64)
    even[T:] = 0
    shifts = np.arange(64, dtype=np.uint64)

    def packw(b):
        return (b.reshape(W, 64) << shifts).sum(axis=1, dtype=np.uint64)

    inputs = np.stack([packw(bits[j]) for j in range(k)]) if k else np.zeros((0, W), np.uint64)
    return BoolCases(inputs.astype(np.uint64), packw(even).astype(np.uint64), T)


# ------------------------------------------------- crossover children
def plus_minus_tree(rng: np.random.Generator, n: int) -> np.ndarray:
    """A tree over {ADD, SUB} and terminal 0 only: its value is a sum of at
    most n inputs in [-1, 1], so it is always finite."""
    return sized_tree(rng, n, 1, funcs=np.array([F_ADD, F_SUB], np.uint8))


def neutral_donor(rng: np.random.Generator, removed: np.ndarray, size: int) -> np.ndarray:
    """(SUB S (SUB R R)): S is a copy of the removed subtree, R a finite
    {+,-} tree, so the donor's value equals S's on every case."""
    r = max(1, (size - 2 - len(removed)) // 2) | 1
    R = plus_minus_tree(rng, r)
    return np.concatenate([[F_SUB], removed, [F_SUB], R, R]).astype(np.uint8)


@dataclass
class Children:
    parent: np.ndarray         # int64 [C]  tree index in the parent population
    point: np.ndarray          # int64 [C]  prefix index in the parent
    donors: Population         # donor subtrees
    neutral: np.ndarray        # bool  [C]


def crossover_children(seed: int, parents: Population, n_children: int, donor_lo: int = 1,
                       donor_hi: int = 10_000, neutral_frac: float = 0.5, n_terms: int = 1,
                       one_per_parent: bool = True) -> Children:
    """Children = parent with the subtree at a uniform node replaced by a donor.

    Donor sizes are log-uniform in [donor_lo, donor_hi].  The first
    round(neutral_frac * n) children get a neutral donor wrapping a copy of
    the removed subtree; for those the point is redrawn until the copy fits
    the drawn donor size.  The rest get a random tree of the drawn size.
    """
    rng = rng_for(seed)
    n_neutral = int(round(neutral_frac * n_children))
    par = np.arange(n_children, dtype=np.int64) % parents.n_trees if one_per_parent else \
        rng.integers(parents.n_trees, size=n_children).astype(np.int64)
    pts = np.zeros(n_children, dtype=np.int64)
    donors = []
    neutral = np.zeros(n_children, dtype=bool)
    for ci in range(n_children):
        tree = parents.tree(int(par[ci]))
        n = len(tree)
        m = int(log_uniform_odd(rng, donor_lo, donor_hi))
        if ci < n_neutral:
            m = max(m, 5)
            while True:
                c = int(rng.integers(n))
                e = subtree_end(tree, c, max_len=m - 4)
                if e > 0:
                    break
            donors.append(neutral_donor(rng, tree[c:e].copy(), m))
            neutral[ci] = True
        else:
            c = int(rng.integers(n))
            donors.append(sized_tree(rng, m, n_terms))
        pts[ci] = c
    return Children(par, pts, pack(donors, parents.vtype, parents.n_inputs), neutral)


def splice(parent: np.ndarray, c: int, donor: np.ndarray) -> np.ndarray:
    """child = parent[0:c] ++ donor ++ parent[end(c):]  (structural copy)."""
    e = subtree_end(parent, c)
    return np.concatenate([parent[:c], donor, parent[e:]]).astype(np.uint8)


# ----------------------------------------------------------- served stream
def bool_neutral_donor(rng: np.random.Generator, removed: np.ndarray, size: int, n_terms: int) -> np.ndarray:
    """AND(S, OR(R, NAND(R, R))) = AND(S, true) = S for every input."""
    r = max(1, (size - 4 - len(removed)) // 3) | 1
    R = sized_tree(rng, r, n_terms)
    return np.concatenate([[B_AND], removed, [B_OR], R, [B_NAND], R, R]).astype(np.uint8)


@dataclass
class ServedJob:
    kind: int                 # 0 full, 1 incremental
    vtype: int
    T: int
    ops: np.ndarray
    arrival: float            # seconds at unit arrival rate
    points: np.ndarray | None = None   # full: crossover points to keep caches for
    parent: int = -1          # incremental: index of the parent job in the stream
    point: int = 0
    neutral: bool = False


def served_stream(seed: int, n_jobs: int, full_frac: float = 0.3, node_lo: int = 10, node_hi: int = 10**7,
                  t_choices=(256, 512, 1024, 2048, 4096), bool_frac: float = 0.5, donor_hi: int = 10**4,
                  points_per_parent: int = 3, threads: int = 1) -> list:
    """Jobs with exponential inter-arrival gaps (mean 1); a share full_frac of
    full jobs (kept resident as parents, each with crossover points drawn
    ahead), the rest incremental children of earlier parents with the same
    value type and case count; half of the children's donors neutral.
    Boolean jobs with T cases use k = log2(T) inputs.

    The job list (kinds, sizes, points, parents) is drawn first from one
    stream; then every tree is built from a seed stream of its own (parents,
    then donors, which may copy a subtree of their parent), so the result does
    not depend on the number of threads."""
    rng = rng_for(seed)
    jobs: list = []
    parents: dict = {}
    t = 0.0
    for i in range(n_jobs):
        t += float(rng.exponential(1.0))
        vtype = VT_BOOL if rng.random() < bool_frac else VT_F32
        T = int(t_choices[int(rng.integers(len(t_choices)))])
        key = (vtype, T)
        if key not in parents or rng.random() < full_frac:
            n = int(log_uniform_odd(rng, node_lo, node_hi))
            pts = np.unique(rng.integers(n, size=points_per_parent)).astype(np.int64)
            jobs.append(ServedJob(0, vtype, T, np.empty(n, np.uint8), t, points=pts))
            parents.setdefault(key, []).append(len(jobs) - 1)
        else:
            pj = parents[key][int(rng.integers(len(parents[key])))]
            c = int(jobs[pj].points[int(rng.integers(len(jobs[pj].points)))])
            m = int(log_uniform_odd(rng, 1, donor_hi))
            neutral = rng.random() < 0.5
            jobs.append(ServedJob(1, vtype, T, np.empty(m, np.uint8), t, parent=pj, point=c, neutral=neutral))
    seqs = np.random.SeedSequence([seed, n_jobs]).spawn(n_jobs)

    def n_terms(j):
        return j.T.bit_length() - 1 if j.vtype == VT_BOOL else 1

    def build_parent(i):
        j = jobs[i]
        j.ops = sized_tree(np.random.default_rng(seqs[i]), len(j.ops), n_terms(j))

    def build_donor(i):
        j = jobs[i]
        r = np.random.default_rng(seqs[i])
        m = len(j.ops)
        donor = None
        if j.neutral:
            ptree = jobs[j.parent].ops
            e = subtree_end(ptree, j.point, max_len=max(1, m - 4))
            if e > 0:
                S = ptree[j.point:e].copy()
                donor = neutral_donor(r, S, m) if j.vtype == VT_F32 else bool_neutral_donor(r, S, m, n_terms(j))
            else:
                j.neutral = False
        j.ops = donor if donor is not None else sized_tree(r, m, n_terms(j))

    full = sorted((i for i, j in enumerate(jobs) if j.kind == 0), key=lambda i: -len(jobs[i].ops))
    inc = [i for i, j in enumerate(jobs) if j.kind == 1]
    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(build_parent, full))
            list(ex.map(build_donor, inc))
    else:
        for i in full:
            build_parent(i)
        for i in inc:
            build_donor(i)
    return jobs
