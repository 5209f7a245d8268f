"""Full-size parity on the GPU, in the launch configuration bench.py uses.

Where the oracle is fast enough (Boolean, 64 cases) every tree is compared;
for the large float populations a sample of trees / children is compared with
the oracle one by one (several independent oracle instances in threads; for
the children of the largest parents, one oracle walk per block of cases) and
properties that hold at any size are checked for all of them.
"""
import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g
from tests import split_oracle
from tests.scalar_ref import same_f32

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def test_boolean_parity6_full_size_all_trees(ctx):
    pop = gen.sized_population(2, 1000, 10**3, 10**5, n_terms=6, vtype=gen.VT_BOOL, threads=16)
    cases = gen.bool_cases(6)
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, 64)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=6)
    roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, 64)
    want_r, want_f = oracle.eval_population_bool(pop, cases.inputs, cases.target, 64, threads=16)
    assert np.array_equal(roots, want_r)
    assert np.array_equal(fit, want_f)
    r2, f2, _ = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, 64, per_tree=True)
    assert np.array_equal(r2, roots) and np.array_equal(f2, fit)
    say("boolean full size:", st)
    # chunk vectors pass between waves without cache maintenance: every replay of
    # the captured launch, with other device work between some of them, and with
    # smaller chunks (more hand-offs), must give the same words
    for rep in range(30):
        r3, f3, _ = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, 64)
        assert np.array_equal(r3, roots) and np.array_equal(f3, fit), rep
        if rep % 10 == 9:
            ctx.fitness(ch, g.GP_BOOL, r3)
    ph2 = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=6, chunk_nodes=32)
    for rep in range(5):
        r4, f4, _ = ctx.evaluate_full(ph2, ch, g.GP_BOOL, pop.n_trees, 64)
        assert np.array_equal(r4, roots) and np.array_equal(f4, fit), rep
    ctx.free(ph2)
    ctx.free(ph)
    ctx.free(ch)


def test_large_float_full_size_sampled(ctx):
    pop = gen.sized_population(3, 1000, 10**4, 10**6, threads=16)
    cases = gen.float_cases(3, 1024)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets)
    v, ms = ctx.autotune(ph, ch)
    roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, 1024)
    say("large float:", g.variant_names()[v], ctx.population_info(ph)["chunk_nodes"], st)
    sizes = pop.sizes()
    order = np.argsort(sizes)
    rng = np.random.default_rng(0)
    # the 10 smallest, 54 at random and the 16 largest (about 1e6 nodes) of the 1000
    sample = list(order[:10]) + list(rng.choice(pop.n_trees, 54, replace=False)) + list(order[-16:])

    def check(i):
        with np.errstate(all="ignore"):
            want = oracle.eval_f32(pop.tree(int(i)), cases.x)
        return bool(same_f32(roots[i], want).all()), (oracle.fitness_f32(want, cases.y), fit[i])

    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(check, sample))
    for i, (ok, (wf, gf)) in zip(sample, res):
        assert ok, f"tree {i} differs"
        assert wf == gf or (math.isnan(wf) and math.isnan(gf)), (i, wf, gf)
    # properties for every tree: fitness from the returned outputs, same order
    f_again = ctx.fitness(ch, g.GP_F32, roots)
    assert all(a == b or (math.isnan(a) and math.isnan(b)) for a, b in zip(f_again, fit))
    # replays of the captured launch give the same bits (chunk vectors pass between
    # waves without cache maintenance)
    for rep in range(10):
        r3, _, _ = ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, 1024)
        assert np.array_equal(r3.view(np.uint32), roots.view(np.uint32)), rep
    ctx.free(ph)
    ctx.free(ch)


def test_incremental_full_size_sampled(ctx):
    parents = gen.sized_population(4, 500, 10**6, 10**7, threads=16)
    cases = gen.float_cases(4, 1024)
    kids = gen.crossover_children(40, parents, 500, donor_lo=1, donor_hi=10**4, neutral_frac=0.5)
    pts = [[] for _ in range(parents.n_trees)]
    for p, c in zip(kids.parent, kids.point):
        pts[int(p)].append(int(c))
    ro = np.cumsum([0] + [len(p) for p in pts]).astype(np.int64)
    rp = np.array([c for p in pts for c in p], np.int64)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, parents.ops, parents.offsets, record_points=rp, record_offsets=ro,
                             chunk_nodes=8192, keep_trees=True)
    proots, pfit, _ = ctx.evaluate_full(ph, ch, g.GP_F32, parents.n_trees, 1024)
    roots, fit, info = ctx.evaluate_incremental(ph, ch, g.GP_F32, 1024, kids.parent, kids.point,
                                                kids.donors.ops, kids.donors.offsets)
    stop = info["stop_level"]
    say("incremental full size: stops at point", int((stop == 0).sum()), "reached root", int((stop < 0).sum()))
    # properties for all 500 children
    for i in range(500):
        p = int(kids.parent[i])
        nd = len(kids.donors.tree(i))
        if kids.neutral[i]:
            assert stop[i] == 0
        if stop[i] >= 0:
            assert info["interpreted_nodes"][i] == nd + stop[i]
            assert fit[i] == pfit[p] or (math.isnan(fit[i]) and math.isnan(pfit[p]))
            assert same_f32(roots[i], proots[p]).all()
        else:
            assert info["interpreted_nodes"][i] > nd
    # the oracle, one by one, on the children of the smallest parents (both kinds)
    sizes = parents.sizes()
    by_size = sorted(range(500), key=lambda i: sizes[int(kids.parent[i])])
    sample = [i for i in by_size if kids.neutral[i]][:3] + [i for i in by_size if not kids.neutral[i]][:5]

    def check(i):
        P = parents.tree(int(kids.parent[i]))
        with np.errstate(all="ignore"):
            return oracle.incremental_f32(P, int(kids.point[i]), kids.donors.tree(i), cases.x, cases.y)

    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(check, sample))
    for i, (w_root, w_lvl, w_int, w_fit) in zip(sample, res):
        assert stop[i] == w_lvl, (i, stop[i], w_lvl)
        assert info["interpreted_nodes"][i] == w_int
        assert same_f32(roots[i], w_root).all()
        assert fit[i] == w_fit or (math.isnan(fit[i]) and math.isnan(w_fit))
    # children of the largest parents (about 1e7 nodes; one neutral, two random) on all 1024 cases, the
    # oracle's incremental walk computed over blocks of cases on host threads (tests/split_oracle.py)
    big = ([i for i in reversed(by_size) if kids.neutral[i]][:1] +
           [i for i in reversed(by_size) if not kids.neutral[i]][:2])
    with ThreadPoolExecutor(16) as pool:
        for i in big:
            say("oracle on the child of a", int(sizes[int(kids.parent[i])]), "node parent")
            w_root, w_lvl, w_int, w_fit = split_oracle.incremental_f32(
                parents.tree(int(kids.parent[i])), int(kids.point[i]), kids.donors.tree(i), cases.x, cases.y,
                32, pool)
            assert stop[i] == w_lvl, (i, stop[i], w_lvl)
            assert info["interpreted_nodes"][i] == w_int
            assert same_f32(roots[i], w_root).all()
            assert fit[i] == w_fit or (math.isnan(fit[i]) and math.isnan(w_fit))
    # the paper's form: the mother co-evaluated alongside, no parent caches
    r2, f2, i2 = ctx.evaluate_incremental(ph, ch, g.GP_F32, 1024, kids.parent, kids.point, kids.donors.ops,
                                          kids.donors.offsets, coeval=True)
    say("co-evaluation full size:", round(i2["wall_ms"], 1), "ms,", int(i2["interpreted_nodes"].sum()),
        "nodes executed,", i2["launches"], "launches")
    assert np.array_equal(i2["stop_level"], stop)
    assert same_f32(r2, roots).all()
    assert all(a == b or (math.isnan(a) and math.isnan(b)) for a, b in zip(f2, fit))
    # all 500 children built on the device, byte for byte against the oracle's splice
    ops, offs, sst = ctx.splice_children(ph, kids.parent, kids.point, kids.donors.ops, kids.donors.offsets,
                                         device=True)
    say("splice full size:", int(offs[-1]), "bytes in", round(sst["kernel_ms"], 3), "ms")
    assert np.array_equal(np.diff(offs), info["child_nodes"])
    host = ops.cpu().numpy()
    del ops

    def same_child(i):
        want = oracle.splice(parents.tree(int(kids.parent[i])), int(kids.point[i]), kids.donors.tree(i))
        return np.array_equal(host[offs[i]:offs[i + 1]], want)

    with ThreadPoolExecutor(8) as ex:
        assert all(ex.map(same_child, range(500)))
    # two generations with fitness first from these parents: the children's
    # programs are built from their parents' chunks; the final trees compiled
    # whole, and the oracle on the smallest of them, score the same
    nh, gst, rec = ctx.evolve(ph, ch, 2, 7, 2022)
    say("evolve full size:", [(round(x["ms"], 1), x["built"]) for x in gst])
    _, fit_c, _ = ctx.evaluate_full(nh, ch, g.GP_F32, 500, 1024)
    last = rec["fitness_f64"][-1]
    assert np.all((last == fit_c) | (np.isnan(last) & np.isnan(fit_c)))
    ops2, offs2 = ctx.population_ops(nh)
    wh = ctx.load_population(g.GP_F32, ops2, offs2, chunk_nodes=8192)
    _, fit_w, _ = ctx.evaluate_full(wh, ch, g.GP_F32, 500, 1024)
    assert np.all((fit_w == fit_c) | (np.isnan(fit_w) & np.isnan(fit_c)))
    ctx.free(wh)
    small = np.argsort(np.diff(offs2))[:4]

    def final_fit(t):
        with np.errstate(all="ignore"):
            return oracle.fitness_f32(oracle.eval_f32(ops2[offs2[t]:offs2[t + 1]], cases.x), cases.y)

    with ThreadPoolExecutor(4) as ex:
        for t, w in zip(small, ex.map(final_fit, small)):
            assert fit_c[t] == w or (math.isnan(fit_c[t]) and math.isnan(w)), t
    ctx.free(nh)
    ctx.free(ph)
    ctx.free(ch)


def test_index_full_size(ctx):
    """The device index of the default 500-tree population (2.1e9 nodes):
    every tree valid, the four smallest compared with the oracle node by
    node (ends, parents, Strahler numbers), 64 sampled nodes of every tree
    compared with the oracle's subtree end, for every sampled node its
    parent's children include it, and every 25th tree's root number."""
    import torch
    pop = gen.sized_population(4, 500, 10**6, 10**7, threads=16)
    dev = torch.from_numpy(pop.ops).to("cuda:0")
    doffs = torch.from_numpy(pop.offsets).to("cuda:0")
    valid, end, parent, sn, ms = ctx.index_trees(dev, doffs, 1, strahler=True)
    say("index full size (with Strahler numbers):", int(pop.offsets[-1]), "nodes in", round(ms, 2), "ms")
    del dev
    assert bool((valid == 1).all())
    sizes = pop.sizes()
    rng = np.random.default_rng(11)
    for t in range(pop.n_trees):
        s, e = int(pop.offsets[t]), int(pop.offsets[t + 1])
        tr = pop.tree(t)
        ks = rng.integers(0, e - s, 64)
        idx = torch.from_numpy((s + ks).astype(np.int64)).to(end.device)
        te = end[idx].cpu().numpy()
        tp = parent[idx].cpu().numpy()
        for k, ek, pk in zip(ks.tolist(), te.tolist(), tp.tolist()):
            assert ek == oracle.subtree_end(tr, k), (t, k)
            if k == 0:
                assert pk == -1
            else:
                assert tr[pk] & 0x80 and (k == pk + 1 or k == int(end[s + pk + 1]))
    for t in np.argsort(sizes)[:4].tolist():
        s, e = int(pop.offsets[t]), int(pop.offsets[t + 1])
        tr = pop.tree(t)
        assert np.array_equal(end[s:e].cpu().numpy(), oracle.all_ends(tr))
        assert np.array_equal(parent[s:e].cpu().numpy(), oracle.parents(tr))
        assert np.array_equal(sn[s:e].cpu().numpy(), oracle.strahler(tr))
    # every tree's root number equals the oracle's
    roots = sn[torch.from_numpy(pop.offsets[:-1].astype(np.int64)).to(sn.device)].cpu().numpy()
    for t in range(0, pop.n_trees, 25):
        assert roots[t] == oracle.strahler(pop.tree(t))[0], t


def test_device_compilation_full_size(ctx):
    """The default 500-tree population (2.1e9 nodes) with one recorded point
    per child, loaded as bench.py loads it: compiled on the device, its
    program, chunk tables, records, spines, subtree index and per-tree chunk
    lists equal the host compiler's byte for byte (gp_population_dump,
    section by section)."""
    parents = gen.sized_population(4, 500, 10**6, 10**7, threads=16)
    kids = gen.crossover_children(40, parents, 500, donor_lo=1, donor_hi=10**4, neutral_frac=0.5)
    pts = [[] for _ in range(parents.n_trees)]
    for p, c in zip(kids.parent, kids.point):
        pts[int(p)].append(int(c))
    ro = np.cumsum([0] + [len(p) for p in pts]).astype(np.int64)
    rp = np.array([c for p in pts for c in p], np.int64)

    def sections(d):
        out, i = [], 0
        while i < len(d):
            n = int(np.frombuffer(d[i:i + 8], np.int64)[0])
            out.append(np.frombuffer(d, np.uint8, count=n, offset=i + 8))
            i += 8 + n
        assert i == len(d)
        return out

    dumps = []
    for dc in (False, True):
        h = ctx.load_population(g.GP_F32, parents.ops, parents.offsets, record_points=rp, record_offsets=ro,
                                keep_trees=True, device_compile=dc)
        dumps.append(ctx.population_dump(h))
        say("dump", "device" if dc else "host", len(dumps[-1]), "bytes")
        ctx.free(h)
    a, b = (sections(d) for d in dumps)
    assert len(a) == len(b) == 16
    for k, (x, y) in enumerate(zip(a, b)):
        assert x.size == y.size and np.array_equal(x, y), k
