"""Device-side tree index (gp_index_trees) against the oracle.

Validity of each tree must equal the oracle's check, and for a valid tree
every node's subtree end and parent must equal the oracle's; invalid trees
(truncated, overlong, unknown function, terminal out of range, a corrupted
byte) get -1 throughout.  Sizes span several 4096-position scan blocks,
ragged tails and trees that start and end at block edges.
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


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def bad_trees():
    return [np.array(t, np.uint8) for t in
            ([F, 0], [0, 0], [F, 0, 0, 0], [0, F, 0], [0x84, 0, 0], [F, 0, 7], [F, F, 0], [9])]


def pack(trees):
    offs = np.zeros(len(trees) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in trees])
    return np.concatenate(trees).astype(np.uint8), offs


def run_index(ctx, trees, n_inputs, strahler=False):
    import torch
    ops, offs = pack(trees)
    dev = torch.from_numpy(ops).to("cuda:0")
    doffs = torch.from_numpy(offs).to("cuda:0")
    if strahler:
        valid, end, parent, sn, ms = ctx.index_trees(dev, doffs, n_inputs, strahler=True)
        return (ops, offs, valid.cpu().numpy(), end.cpu().numpy(), parent.cpu().numpy(), ms,
                sn.cpu().numpy())
    valid, end, parent, ms = ctx.index_trees(dev, doffs, n_inputs)
    return ops, offs, valid.cpu().numpy(), end.cpu().numpy(), parent.cpu().numpy(), ms


def check(trees, offs, valid, end, parent, n_inputs, sn=None):
    for t, tr in enumerate(trees):
        ok = oracle.validate(tr, n_inputs)
        assert bool(valid[t]) == ok, (t, valid[t], ok)
        s, e = offs[t], offs[t + 1]
        if ok:
            assert np.array_equal(end[s:e], oracle.all_ends(tr)), t
            assert np.array_equal(parent[s:e], oracle.parents(tr)), t
            if sn is not None:
                assert np.array_equal(sn[s:e], oracle.strahler(tr)), t
        else:
            assert (end[s:e] == -1).all() and (parent[s:e] == -1).all(), t
            if sn is not None:
                assert (sn[s:e] == 0).all(), t


@pytest.mark.parametrize("seed", range(4))
def test_index_mixed_population(ctx, seed):
    rng = np.random.default_rng(70 + seed)
    n_inputs = [1, 3, 6, 64][seed]
    trees = []
    for _ in range(int(rng.integers(20, 300))):
        r = rng.random()
        if r < 0.15:
            trees.append(bad_trees()[int(rng.integers(0, 8))])
            continue
        n = int(gen.log_uniform_odd(rng, 1, 20001))
        tr = gen.sized_tree(rng, n, n_terms=min(n_inputs, 6))
        if r < 0.25 and n > 3:
            tr = tr.copy()
            tr[int(rng.integers(0, n))] = int(rng.choice([0x84, 0x80, 0, 63, 200]))
        trees.append(tr)
    ops, offs, valid, end, parent, ms = run_index(ctx, trees, n_inputs)
    say("index mixed", seed, len(trees), "trees", len(ops), "nodes", round(ms, 3), "ms")
    check(trees, offs, valid, end, parent, n_inputs)
    ops, offs, valid, end, parent, ms, sn = run_index(ctx, trees, n_inputs, strahler=True)
    say("index mixed with Strahler numbers", round(ms, 3), "ms")
    check(trees, offs, valid, end, parent, n_inputs, sn)


@pytest.mark.parametrize("sizes", [[1], [4095], [4095, 1], [4097], [8191, 4095, 1, 4097], [1] * 5000])
def test_index_block_edges(ctx, sizes):
    rng = np.random.default_rng(len(sizes) + sum(sizes))
    trees = [gen.sized_tree(rng, n, n_terms=2) for n in sizes]
    ops, offs, valid, end, parent, _, sn = run_index(ctx, trees, 2, strahler=True)
    assert valid.all()
    check(trees, offs, valid, end, parent, 2, sn)


def _complete(depth):
    out = []

    def rec(d):
        if d == 0:
            out.append(0)
        else:
            out.append(F)
            rec(d - 1)
            rec(d - 1)
    rec(depth)
    return out


def test_index_deep_and_large_trees(ctx):
    """A left comb and a right comb (height n/2), a random 2e6-node tree and a
    complete tree of depth 17 (Strahler number 18 at its root)."""
    d = 30000
    left = np.array([F] * d + [0] * (d + 1), np.uint8)
    right = np.array([F, 0] * d + [0], np.uint8)
    big = gen.sized_tree(np.random.default_rng(3), 2_000_001, n_terms=1)
    full = np.array(_complete(17), np.uint8)
    trees = [left, right, big, full]
    ops, offs, valid, end, parent, ms, sn = run_index(ctx, trees, 1, strahler=True)
    say("index deep/large:", len(ops), "nodes", round(ms, 3), "ms")
    check(trees, offs, valid, end, parent, 1, sn)
    assert sn[offs[3]] == 18


def test_index_errors(ctx):
    import torch
    ops, offs = pack([np.array([F, 0, 0], np.uint8), np.array([0], np.uint8)])
    dev = torch.from_numpy(np.concatenate([np.zeros(16, np.uint8), ops])).to("cuda:0")
    doffs = torch.from_numpy(offs).to("cuda:0")
    with pytest.raises(g.GPError):                       # ops not 16-byte aligned
        ctx.index_trees(dev[1:], doffs, 1, n_nodes=len(ops))
    bad = torch.from_numpy(np.array([0, 3, 2], np.int64)).to("cuda:0")
    with pytest.raises(g.GPError):                       # decreasing offsets
        ctx.index_trees(dev[16:], bad, 1, n_nodes=len(ops))
    short = torch.from_numpy(np.array([0, 3, 3], np.int64)).to("cuda:0")
    with pytest.raises(g.GPError):                       # offsets end before n_nodes
        ctx.index_trees(dev[16:], short, 1, n_nodes=len(ops))
    with pytest.raises(g.GPError):                       # n_inputs out of range
        ctx.index_trees(dev[16:], doffs, 0, n_nodes=len(ops))
    with pytest.raises(g.GPError):                       # beyond 2^31 - 2 nodes
        ctx.index_trees(dev[16:], doffs, 1, n_nodes=2**31)
    valid, end, parent, _ = ctx.index_trees(dev[16:], doffs, 1, n_nodes=len(ops))   # still works after errors
    assert valid.cpu().tolist() == [1, 1]
    assert end.cpu().tolist() == [3, 2, 3, 1] and parent.cpu().tolist() == [-1, 0, 0, -1]


def test_index_outputs_at_odd_addresses(ctx):
    """Ends, parents and Strahler numbers written to caller buffers that start
    4 and 1 bytes past a 16-byte boundary (where the kernels' 16-byte loads
    and stores of a thread's positions fall back to single elements) equal
    those of the aligned buffers the allocating call returns."""
    import torch
    rng = np.random.default_rng(91)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 200001)), n_terms=2) for _ in range(30)]
    ops, offs = pack(trees)
    n = len(ops)
    assert n <= g.INDEX_NOALLOC_MAX_NODES
    dev = torch.from_numpy(ops).to("cuda:0")
    doffs = torch.from_numpy(offs).to("cuda:0")
    v1, e1, p1, s1, _ = ctx.index_trees(dev, doffs, 2, strahler=True)
    v2 = torch.full((len(trees),), 77, dtype=torch.int32, device="cuda:0")
    eb = torch.full((n + 1,), 77, dtype=torch.int32, device="cuda:0")
    pb = torch.full((n + 1,), 77, dtype=torch.int32, device="cuda:0")
    sb = torch.full((n + 1,), 77, dtype=torch.uint8, device="cuda:0")
    say("index at odd addresses:", len(trees), "trees", n, "nodes")
    ctx.index_trees_noalloc(dev, doffs, 2, v2, eb[1:], pb[1:], sb[1:])
    assert eb[1:].data_ptr() % 16 == 4 and sb[1:].data_ptr() % 16 == 1
    assert np.array_equal(v2.cpu().numpy(), v1.cpu().numpy())
    assert np.array_equal(eb[1:].cpu().numpy(), e1.cpu().numpy())
    assert np.array_equal(pb[1:].cpu().numpy(), p1.cpu().numpy())
    assert np.array_equal(sb[1:].cpu().numpy(), s1.cpu().numpy())
    assert int(eb[0]) == 77 and int(pb[0]) == 77 and int(sb[0]) == 77
    check(trees, offs, v1.cpu().numpy(), e1.cpu().numpy(), p1.cpu().numpy(), 2, s1.cpu().numpy())
