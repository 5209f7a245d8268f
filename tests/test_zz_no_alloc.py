"""gp_index_trees_noalloc, the tree index for callers that cannot allocate
device memory, against gp_index_trees on the same inputs: validity, subtree
ends, parents and Strahler numbers bit for bit, on two calls in a row (the
second on a smaller population, over what the first left in the shared
scratch array), plus the oracle on every tree of the second call and a sample
of the first.  Sizes past the limit are refused before anything is written,
and the calls allocate no device memory charged to the context.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g

pytestmark = pytest.mark.gpu

F = gen.F_ADD


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def pack(trees):
    offs = np.zeros(len(trees) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in trees])
    return np.concatenate(trees).astype(np.uint8), offs


def population(seed, n_trees, lo, hi, n_inputs):
    """Valid trees of log-uniform sizes with invalid ones among them
    (truncated, overlong, unknown function, terminal out of range)."""
    rng = np.random.default_rng(seed)
    trees = []
    for i in range(n_trees):
        t = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, lo, hi)), n_terms=n_inputs)
        r = i % 7
        if r == 1 and len(t) > 2:
            t = t[:-1]
        elif r == 2:
            t = np.concatenate([t, [0]]).astype(np.uint8)
        elif r == 3 and len(t) > 2:
            t = t.copy()
            t[int(rng.integers(len(t)))] = 0x85
        elif r == 4:
            t = t.copy()
            t[-1] = n_inputs
        trees.append(t)
    return trees


def both(ctx, trees, n_inputs, strahler):
    import torch
    ops, offs = pack(trees)
    n = len(ops)
    dops = torch.from_numpy(ops).to("cuda:0")
    doffs = torch.from_numpy(offs).to("cuda:0")
    if strahler:
        v1, e1, p1, s1, _ = ctx.index_trees(dops, doffs, n_inputs, strahler=True)
    else:
        v1, e1, p1, _ = ctx.index_trees(dops, doffs, n_inputs)
        s1 = None
    # outputs filled with garbage first: every entry must be written
    v2 = torch.full((len(trees),), 77, dtype=torch.int32, device="cuda:0")
    e2 = torch.full((n,), 77, dtype=torch.int32, device="cuda:0")
    p2 = torch.full((n,), 77, dtype=torch.int32, device="cuda:0")
    s2 = torch.full((n,), 77, dtype=torch.uint8, device="cuda:0") if strahler else None
    torch.cuda.synchronize()
    used = ctx.memory_used
    ctx.index_trees_noalloc(dops, doffs, n_inputs, v2, e2, p2, s2)
    assert ctx.memory_used == used
    got = [x.cpu().numpy() for x in (v2, e2, p2)] + ([s2.cpu().numpy()] if strahler else [None])
    want = [x.cpu().numpy() for x in (v1, e1, p1)] + ([s1.cpu().numpy()] if strahler else [None])
    for a, b in zip(got, want):
        if b is not None:
            assert np.array_equal(a, b)
    return ops, offs, got


def check_oracle(trees, offs, valid, end, parent, sn, n_inputs, which):
    for t in which:
        tr = trees[t]
        ok = oracle.validate(tr, n_inputs)
        assert bool(valid[t]) == ok, t
        s, e = offs[t], offs[t + 1]
        if ok:
            assert np.array_equal(end[s:e], oracle.all_ends(tr)), t
            assert np.array_equal(parent[s:e], oracle.parents(tr)), t
            if sn is not None:
                assert np.array_equal(sn[s:e], oracle.strahler(tr)), t
        else:
            assert (end[s:e] == -1).all() and (parent[s:e] == -1).all(), t


def test_noalloc_index_matches_allocating_index_twice():
    ctx = g.Context(0)
    # first call: close to the limit, many scan blocks, Strahler numbers
    big = population(3, 60, 1001, 400_001, 6)
    total = sum(len(t) for t in big)
    while total > g.INDEX_NOALLOC_MAX_NODES:
        total -= len(big.pop())
    big.append(np.zeros(1, np.uint8))
    say("first call", len(big), "trees", sum(len(t) for t in big), "nodes")
    ops, offs, (valid, end, parent, sn) = both(ctx, big, 6, strahler=True)
    assert sum(len(t) for t in big) > g.INDEX_NOALLOC_MAX_NODES // 2
    small_idx = [i for i in range(len(big)) if len(big[i]) < 30_000][:6] + [len(big) - 1]
    check_oracle(big, offs, valid, end, parent, sn, 6, small_idx)
    # second call: a smaller population over the first call's scratch contents
    small = population(4, 300, 1, 5001, 3)
    say("second call", len(small), "trees", sum(len(t) for t in small), "nodes")
    ops, offs, (valid, end, parent, sn) = both(ctx, small, 3, strahler=True)
    check_oracle(small, offs, valid, end, parent, sn, 3, range(len(small)))
    # and without Strahler numbers
    ops, offs, (valid, end, parent, _) = both(ctx, small[:50], 3, strahler=False)
    check_oracle(small[:50], offs, valid, end, parent, None, 3, range(50))
    ctx.close()


def test_noalloc_index_refuses_more_nodes_than_its_scratch_holds():
    import torch
    ctx = g.Context(0)
    n = g.INDEX_NOALLOC_MAX_NODES + 1
    ops = torch.zeros(n + 15, dtype=torch.uint8, device="cuda:0")
    offs = torch.tensor([0, n], dtype=torch.int64, device="cuda:0")
    valid = torch.full((1,), 77, dtype=torch.int32, device="cuda:0")
    end = torch.full((n,), 77, dtype=torch.int32, device="cuda:0")
    parent = torch.full((n,), 77, dtype=torch.int32, device="cuda:0")
    with pytest.raises(g.GPError) as e:
        ctx.index_trees_noalloc(ops, offs, 1, valid, end, parent, None, n_nodes=n)
    assert e.value.code == g.GP_EINVAL
    torch.cuda.synchronize()
    assert int(valid[0]) == 77 and bool((end == 77).all()) and bool((parent == 77).all())
    ctx.close()
