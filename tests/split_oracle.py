"""Oracle results for large jobs, computed over blocks of test cases on
several host threads.

Every test case is evaluated on its own (Section 4.2), so a tree's outputs on
a block of cases are its outputs on the whole case set restricted to that
block.  For an incremental child (Section 6.2, Figure 3), once child and
mother agree on every case of a block at some level, they agree on that block
at every level above it too: at each ancestor both apply the same function to
the same sibling value.  So the first level at which they agree on all cases
is the largest of the blocks' first levels, or -1 (root reached) when some
block reaches the root; the count of interpreted nodes (donor + levels
re-evaluated) is then the largest of the blocks' counts, and the child's
outputs are the blocks' outputs side by side.  Fitness is the oracle's own
fixed-order sum over the whole output vector.  Boolean words are blocks of 64
cases, so the same holds per block of words.

The helpers only split inputs and join the oracle's outputs; all arithmetic
is the oracle's.  tests/test_split_oracle.py checks them against unsplit
oracle calls.
"""
import numpy as np

import oracle


def _edges(n, blocks):
    blocks = max(1, min(blocks, n))
    return [(int(a), int(b)) for a, b in zip(np.linspace(0, n, blocks + 1)[:-1].astype(np.int64),
                                              np.linspace(0, n, blocks + 1)[1:].astype(np.int64))]


def _join_levels(levels):
    return -1 if any(l == -1 for l in levels) else max(levels)


def eval_f32(tree, x, y, blocks, pool):
    """-> (out[T], fitness)."""
    x = np.atleast_2d(x)
    parts = list(pool.map(lambda e: oracle.eval_f32(tree, x[:, e[0]:e[1]]), _edges(x.shape[1], blocks)))
    out = np.concatenate(parts).astype(np.float32)
    return out, oracle.fitness_f32(out, y)


def incremental_f32(parent, c, donor, x, y, blocks, pool, cols=None):
    """-> (root_out, stop_level, interpreted_nodes, fitness) over all cases,
    or, with cols (case indices), over those cases only (then the level is
    that of the sampled cases, a lower bound of the whole set's when the
    whole set stops, and the fitness is over the sampled cases)."""
    x = np.atleast_2d(x)
    if cols is not None:
        x = x[:, cols]
        y = y[cols]

    def one(e):
        with np.errstate(all="ignore"):
            return oracle.incremental_f32(parent, c, donor, x[:, e[0]:e[1]], y[e[0]:e[1]])
    parts = list(pool.map(one, _edges(x.shape[1], blocks)))
    root = np.concatenate([p[0] for p in parts]).astype(np.float32)
    level = _join_levels([p[1] for p in parts])
    interp = max(p[2] for p in parts)
    with np.errstate(all="ignore"):
        fit = oracle.fitness_f32(root, y)
    return root, level, interp, fit


def eval_bool(tree, inputs, target, T, blocks, pool):
    """-> (out[W], hits)."""
    W = inputs.shape[1]
    parts = list(pool.map(lambda e: oracle.eval_bool(tree, inputs[:, e[0]:e[1]]), _edges(W, blocks)))
    out = np.concatenate(parts).astype(np.uint64)
    return out, oracle.fitness_bool(out, target, T)


def incremental_bool(parent, c, donor, inputs, target, T, blocks, pool):
    W = inputs.shape[1]

    def one(e):
        n_valid = min(T, e[1] * 64) - e[0] * 64
        return oracle.incremental_bool(parent, c, donor, inputs[:, e[0]:e[1]], target[e[0]:e[1]], n_valid)
    parts = list(pool.map(one, _edges(W, blocks)))
    root = np.concatenate([p[0] for p in parts]).astype(np.uint64)
    level = _join_levels([p[1] for p in parts])
    interp = max(p[2] for p in parts)
    return root, level, interp, oracle.fitness_bool(root, target, T)
