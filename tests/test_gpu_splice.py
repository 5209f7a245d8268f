"""Children built on the device (gp_splice_children) against the oracle's
splice (Section 5, Figure 1): byte for byte, in device and host memory, for
prefix and reverse-Polish populations, at every alignment of the three copied
ranges, plus the error paths and agreement with incremental evaluation."""
import sys

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g
from tests.scalar_ref import same_f32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def record_lists(n_trees, parent, point):
    pts = [[] for _ in range(n_trees)]
    for p, c in zip(parent, point):
        if int(c) not in pts[int(p)]:
            pts[int(p)].append(int(c))
    offs = np.cumsum([0] + [len(p) for p in pts]).astype(np.int64)
    return np.array([c for p in pts for c in p], np.int64), offs


def expected_children(pop, parent, point, donors):
    kids = [oracle.splice(pop.tree(int(p)), int(c), donors.tree(i)) for i, (p, c) in enumerate(zip(parent, point))]
    offs = np.cumsum([0] + [len(k) for k in kids]).astype(np.int64)
    return kids, offs


def check_children(ops, offs, kids, want_offs):
    ops = np.asarray(ops)
    assert np.array_equal(offs, want_offs)
    for i, k in enumerate(kids):
        assert np.array_equal(ops[offs[i]:offs[i + 1]], k), i


def splice_both_ways(ctx, ph, parent, point, donors):
    host_ops, offs, st = ctx.splice_children(ph, parent, point, donors.ops, donors.offsets)
    dev_ops, offs2, st2 = ctx.splice_children(ph, parent, point, donors.ops, donors.offsets, device=True)
    assert np.array_equal(offs, offs2)
    assert st["equivalent_ops"] == offs[-1] and st["launches"] == 1
    return host_ops, dev_ops.cpu().numpy(), offs


def test_splice_prefix_matches_oracle(ctx):
    pop = gen.sized_population(51, 40, 1, 3001)
    kids = gen.crossover_children(52, pop, 300, donor_hi=300, one_per_parent=False)
    parent, point = list(kids.parent), list(kids.point)
    donors = [kids.donors.tree(i) for i in range(300)]
    # edge cases: the whole tree replaced, the last node replaced, one-node donors and parents
    one = int(np.argmin(pop.sizes()))
    for p, c, d in [(0, 0, np.array([0], np.uint8)), (1, pop.sizes()[1] - 1, np.array([0], np.uint8)),
                    (2, 0, gen.sized_tree(np.random.default_rng(1), 999)), (one, 0, np.array([0], np.uint8)),
                    (3, pop.sizes()[3] - 1, gen.sized_tree(np.random.default_rng(2), 5001))]:
        parent.append(p)
        point.append(c)
        donors.append(d)
    donors = gen.pack(donors)
    rp, ro = record_lists(pop.n_trees, parent, point)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro, keep_trees=True)
    want, want_offs = expected_children(pop, parent, point, donors)
    host_ops, dev_ops, offs = splice_both_ways(ctx, ph, parent, point, donors)
    check_children(host_ops, offs, want, want_offs)
    check_children(dev_ops, offs, want, want_offs)
    assert all(oracle.validate(k) for k in want)
    # sizes only
    n = len(parent)
    o = np.zeros(n + 1, np.int64)
    par, pts = np.asarray(parent, np.int64), np.asarray(point, np.int64)     # kept alive across the call
    rc = g.lib().gp_splice_children(ctx._h, ph, n, g._ptr(par), g._ptr(pts), g._ptr(donors.ops),
                                    g._ptr(donors.offsets), 0, None, 0, g._ptr(o), None)
    assert rc == 0 and np.array_equal(o, want_offs)
    ctx.free(ph)


def test_splice_every_alignment(ctx):
    """One 200001-node parent: cut points with every residue mod 16, donors of
    1..40 bytes, removed subtrees small and large, so every head/tail length
    and source offset within a 4-byte word occurs, and the long ranges span
    several 64 KiB pieces."""
    rng = np.random.default_rng(8)
    big = gen.sized_tree(rng, 200001)
    small = gen.sized_tree(rng, 777)
    pop = gen.pack([big, small])
    ends = gen.subtree_ends(big)
    parent, point, donors = [], [], []
    for r in range(16):
        for nd in (1, 3, 5, 17, 39):
            c = 16 * int(rng.integers(1, 12000)) + r
            parent.append(0)
            point.append(c)
            donors.append(gen.sized_tree(rng, nd))
    for c in (0, 1, 2, 100001, 199999, 200000):           # root, big and tiny removed subtrees
        parent.append(0)
        point.append(c)
        donors.append(gen.sized_tree(rng, 21))
    for c in range(0, 777, 37):
        parent.append(1)
        point.append(c)
        donors.append(gen.sized_tree(rng, 1 + 2 * (c % 20)))
    donors = gen.pack(donors)
    removed = [int(ends[c]) - c for p, c in zip(parent, point) if p == 0]
    assert max(removed) > 100000 and min(removed) == 1
    rp, ro = record_lists(2, parent, point)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro, keep_trees=True)
    want, want_offs = expected_children(pop, parent, point, donors)
    host_ops, dev_ops, offs = splice_both_ways(ctx, ph, parent, point, donors)
    check_children(host_ops, offs, want, want_offs)
    check_children(dev_ops, offs, want, want_offs)
    # into a device buffer at an odd offset: the output alignment changes too
    import torch
    buf = torch.zeros(int(offs[-1]) + 64, dtype=torch.uint8, device="cuda:0")
    view = buf[7:7 + int(offs[-1])]
    ops3, offs3, _ = ctx.splice_children(ph, parent, point, donors.ops, donors.offsets, out=view)
    check_children(view.cpu().numpy(), offs3, want, want_offs)
    assert int(buf[:7].sum()) == 0 and int(buf[7 + int(offs[-1]):].sum()) == 0
    ctx.free(ph)


def to_postfix(t):
    """Reverse-Polish copy of a prefix tree, and the postfix index of each
    prefix node."""
    ends = gen.subtree_ends(t)
    out, where = [], np.zeros(len(t), np.int64)
    stack = [(0, False)]
    while stack:
        i, done = stack.pop()
        if t[i] & 0x80 and not done:
            stack.append((i, True))
            stack.append((int(ends[i + 1]), False))
            stack.append((i + 1, False))
        else:
            where[i] = len(out)
            out.append(int(t[i]))
    return np.array(out, np.uint8), where


def test_splice_postfix_population(ctx):
    pop = gen.sized_population(61, 12, 1, 2001)
    kids = gen.crossover_children(62, pop, 60, donor_hi=200, one_per_parent=False)
    post, maps = zip(*[to_postfix(pop.tree(i)) for i in range(pop.n_trees)])
    ppop = gen.pack(list(post))
    ppoint = [int(maps[int(p)][int(c)]) for p, c in zip(kids.parent, kids.point)]
    pdonors = gen.pack([to_postfix(kids.donors.tree(i))[0] for i in range(60)])
    rp, ro = record_lists(pop.n_trees, kids.parent, ppoint)
    ph = ctx.load_population(g.GP_F32, ppop.ops, ppop.offsets, layout=g.GP_POSTFIX, record_points=rp,
                             record_offsets=ro, keep_trees=True)
    want_pre, _ = expected_children(pop, kids.parent, kids.point, kids.donors)
    want = [to_postfix(k)[0] for k in want_pre]
    want_offs = np.cumsum([0] + [len(k) for k in want]).astype(np.int64)
    host_ops, dev_ops, offs = splice_both_ways(ctx, ph, kids.parent, ppoint, pdonors)
    check_children(host_ops, offs, want, want_offs)
    check_children(dev_ops, offs, want, want_offs)
    ctx.free(ph)


def test_splice_errors(ctx):
    pop = gen.sized_population(71, 4, 11, 101)
    d = gen.pack([np.array([0], np.uint8)])
    rp, ro = record_lists(4, [0, 1], [1, 2])
    plain = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro)
    with pytest.raises(g.GPError) as e:                       # loaded without GP_KEEP_TREES
        ctx.splice_children(plain, [0], [1], d.ops, d.offsets)
    assert e.value.code == g.GP_EINVAL
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro, keep_trees=True)
    with pytest.raises(g.GPError) as e:                       # point not recorded
        ctx.splice_children(ph, [0], [2], d.ops, d.offsets)
    assert e.value.code == g.GP_ENOTFOUND
    bad = gen.pack([np.array([gen.F_ADD, 0], np.uint8)])
    with pytest.raises(g.GPError) as e:                       # malformed donor
        ctx.splice_children(ph, [0], [1], bad.ops, bad.offsets)
    assert e.value.code == g.GP_EINVAL
    with pytest.raises(g.GPError) as e:                       # parent out of range
        ctx.splice_children(ph, [4], [1], d.ops, d.offsets)
    assert e.value.code == g.GP_EINVAL
    import torch
    small = torch.zeros(1, dtype=torch.uint8, device="cuda:0")     # every child here has >= 3 nodes
    with pytest.raises(g.GPError) as e:                       # output too small
        ctx.splice_children(ph, [0], [1], d.ops, d.offsets, out=small)
    assert e.value.code == g.GP_EINVAL and int(small.sum()) == 0
    ops, offs, st = ctx.splice_children(ph, [], [], np.zeros(0, np.uint8), np.zeros(1, np.int64))
    assert len(ops) == 0 and list(offs) == [0]
    ctx.free(plain)
    ctx.free(ph)


def test_spliced_children_evaluate_like_incremental(ctx):
    """Children built on the device, loaded and fully evaluated, give the
    incremental evaluation's outputs and fitness."""
    pop = gen.sized_population(81, 16, 101, 20001)
    kids = gen.crossover_children(82, pop, 64, donor_hi=500, one_per_parent=False)
    cases = gen.float_cases(83, 300)
    rp, ro = record_lists(pop.n_trees, kids.parent, kids.point)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro, keep_trees=True)
    ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, cases.T)
    iroots, ifit, _ = ctx.evaluate_incremental(ph, ch, g.GP_F32, cases.T, kids.parent, kids.point,
                                               kids.donors.ops, kids.donors.offsets)
    ops, offs, _ = ctx.splice_children(ph, kids.parent, kids.point, kids.donors.ops, kids.donors.offsets)
    kh = ctx.load_population(g.GP_F32, ops, offs)
    froots, ffit, _ = ctx.evaluate_full(kh, ch, g.GP_F32, len(offs) - 1, cases.T)
    assert same_f32(froots, iroots).all()
    assert np.array_equal(ffit, ifit) or all(a == b or (np.isnan(a) and np.isnan(b)) for a, b in zip(ffit, ifit))
    ctx.free(kh)
    ctx.free(ph)
    ctx.free(ch)


def test_splice_after_autotune(ctx):
    """The autotuner re-chunks a population under the same handle; the kept
    device copy of its trees must move with it."""
    pop = gen.sized_population(91, 8, 1001, 30001)
    kids = gen.crossover_children(92, pop, 16, donor_hi=300, one_per_parent=False)
    cases = gen.float_cases(93, 256)
    rp, ro = record_lists(pop.n_trees, kids.parent, kids.point)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, record_points=rp, record_offsets=ro, keep_trees=True)
    ctx.autotune(ph, ch)
    want, want_offs = expected_children(pop, kids.parent, kids.point, kids.donors)
    host_ops, dev_ops, offs = splice_both_ways(ctx, ph, kids.parent, kids.point, kids.donors)
    check_children(host_ops, offs, want, want_offs)
    check_children(dev_ops, offs, want, want_offs)
    ctx.free(ph)
    ctx.free(ch)
