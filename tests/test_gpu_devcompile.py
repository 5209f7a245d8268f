"""Device-side compilation (gp_load_population with GP_DEVICE_COMPILE or
device-resident trees) against the host compiler and the oracle.

The compiled population (instruction words, chunk table, chunk inputs,
scheduling order, records, spines, the large-subtree index, the per-tree
chunk lists kept for building children) must equal the host compiler's byte
for byte, section by section of gp_population_dump.  Populations cover float
and Boolean trees, one and several inputs, chunk targets from 16 to 4096
nodes, stack-need cuts (complete trees), combs, one-node trees and crossover
points at the root, at terminals, repeated and on shared paths.  A device
compiled population then evaluates to the oracle's outputs and fitness, full
and incremental, and the error paths say what the host compiler says.
"""
import sys

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g

pytestmark = pytest.mark.gpu

SECTIONS = ["header", "code", "chunks", "chunk_in", "chunk_n_in", "chunk_tree", "rec_base", "leaves", "spines",
            "spine_keys", "levels", "big_ends", "cuts", "kept_chunks", "kept_max_stack", "tree_nodes"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def sections(d: bytes):
    out, i = [], 0
    while i < len(d):
        n = int(np.frombuffer(d[i:i + 8], np.int64)[0])
        out.append(d[i + 8:i + 8 + n])
        i += 8 + n
    assert i == len(d) and len(out) == len(SECTIONS)
    return out


def same_dump(a: bytes, b: bytes):
    for name, x, y in zip(SECTIONS, sections(a), sections(b)):
        if x != y:
            xa, ya = np.frombuffer(x, np.uint8), np.frombuffer(y, np.uint8)
            k = int(np.argmax(xa[:min(len(xa), len(ya))] != ya[:min(len(xa), len(ya))])) if len(xa) == len(ya) else -1
            raise AssertionError(f"section {name} differs: {len(x)} vs {len(y)} bytes, first byte {k}")


def record_lists(pts):
    ro = np.cumsum([0] + [len(p) for p in pts]).astype(np.int64)
    rp = np.array([c for p in pts for c in p], np.int64)
    return rp, ro


def random_points(seed, pop, per_tree):
    rng = np.random.default_rng(seed)
    pts = []
    for t in range(pop.n_trees):
        n = int(pop.sizes()[t])
        p = [int(v) for v in rng.integers(0, n, size=per_tree)]
        if per_tree:
            p += [0, p[0]]
        pts.append(p)
    return pts


def compare(ctx, pop, chunk_nodes, pts=None, label=""):
    rp, ro = record_lists(pts) if pts is not None else (None, None)
    say(f"[devcompile] {label}: {pop.n_trees} trees, {int(pop.offsets[-1])} nodes, chunk {chunk_nodes}, "
        f"points {0 if rp is None else len(rp)}")
    hh = ctx.load_population(pop.vtype, pop.ops, pop.offsets, n_inputs=pop.n_inputs, record_points=rp,
                             record_offsets=ro, chunk_nodes=chunk_nodes)
    dh = ctx.load_population(pop.vtype, pop.ops, pop.offsets, n_inputs=pop.n_inputs, record_points=rp,
                             record_offsets=ro, chunk_nodes=chunk_nodes, device_compile=True)
    try:
        same_dump(ctx.population_dump(hh), ctx.population_dump(dh))
        assert ctx.population_info(hh) == ctx.population_info(dh)
    finally:
        ctx.free(hh)
    return dh


def complete(depth, n_terms=1, seed=0):
    rng = np.random.default_rng(seed)
    out = []

    def rec(d):
        if d == depth:
            out.append(int(rng.integers(n_terms)))
            return
        out.append(0x80 + int(rng.integers(4)))
        rec(d + 1)
        rec(d + 1)
    rec(0)
    return np.array(out, np.uint8)


def comb(depth, left, seed=0):
    rng = np.random.default_rng(seed)
    if left:
        return np.array([0x80 + int(v) for v in rng.integers(4, size=depth)] + [0] * (depth + 1), np.uint8)
    ops = []
    for f in rng.integers(4, size=depth):
        ops += [0x80 + int(f), 0]
    return np.array(ops + [0], np.uint8)


@pytest.mark.parametrize("chunk_nodes", [16, 64, 256])
def test_ramped_float_and_boolean(ctx, chunk_nodes):
    pop = gen.ramped_half_and_half(3, 100)
    ctx.free(compare(ctx, pop, chunk_nodes, random_points(5, pop, 2), "ramped float"))
    bpop = gen.ramped_half_and_half(4, 100, n_terms=6, vtype=gen.VT_BOOL)
    ctx.free(compare(ctx, bpop, chunk_nodes, random_points(6, bpop, 3), "ramped Boolean"))
    ctx.free(compare(ctx, pop, chunk_nodes, None, "ramped float, no points"))


@pytest.mark.parametrize("vtype,n_terms", [(gen.VT_F32, 1), (gen.VT_F32, 3), (gen.VT_BOOL, 6)])
@pytest.mark.parametrize("chunk_nodes", [17, 1024, 4096])
def test_sized_populations(ctx, vtype, n_terms, chunk_nodes):
    pop = gen.sized_population(20 + chunk_nodes, 40, 1, 100001, n_terms=n_terms, vtype=vtype)
    ctx.free(compare(ctx, pop, chunk_nodes, random_points(21, pop, 2), f"sized vtype {vtype} inputs {n_terms}"))


def test_stack_cuts_combs_and_single_nodes(ctx):
    trees = [complete(d, seed=d) for d in (11, 12, 13, 14)] + [comb(3000, True, 1), np.array([0], np.uint8),
                                                               comb(2999, False, 2), np.array([0x81, 0, 0], np.uint8)]
    pop = gen.pack(trees, gen.VT_F32, 1)
    pts = random_points(9, pop, 3)
    for c in (16, 128, 10 ** 6):
        ctx.free(compare(ctx, pop, c, pts, "complete trees and combs"))


def test_automatic_chunk_size_and_one_large_tree(ctx):
    pop = gen.sized_population(31, 1, 2000001, 2000001)
    ctx.free(compare(ctx, pop, 0, [[0, 1, 12345, 1999999]], "one 2e6-node tree"))
    big = gen.sized_population(32, 12, 10001, 400001)
    ctx.free(compare(ctx, big, 0, random_points(33, big, 1), "12 trees up to 4e5 nodes"))


def test_many_batches_per_wave(ctx):
    # the persistent kernels run at most 8 blocks of 4 waves per compute unit;
    # beyond 8192 waves' single batches (8.4e6 nodes in the bottom-up pass,
    # 524288 chunks in emission) waves take several batches each
    pop = gen.sized_population(35, 30, 300001, 500001, threads=8)
    assert pop.offsets[-1] > 9_000_000
    ph = compare(ctx, pop, 16, random_points(36, pop, 1), "30 trees, 16-node chunks")
    assert ctx.population_info(ph)["n_chunks"] > 600_000
    ctx.free(ph)


def test_device_resident_trees(ctx):
    import torch
    pop = gen.sized_population(41, 30, 1, 20001)
    hh = ctx.load_population(pop.vtype, pop.ops, pop.offsets, chunk_nodes=64)
    # an odd start address: the library copies the trees to an aligned buffer
    raw = torch.zeros(len(pop.ops) + 1, dtype=torch.uint8, device="cuda:0")
    raw[1:] = torch.from_numpy(pop.ops).to("cuda:0")
    dh = ctx.load_population(pop.vtype, raw[1:], torch.from_numpy(pop.offsets).to("cuda:0"), chunk_nodes=64)
    same_dump(ctx.population_dump(hh), ctx.population_dump(dh))
    ops, offs = ctx.population_ops(dh)
    assert np.array_equal(ops, pop.ops) and np.array_equal(offs, pop.offsets)
    ctx.free(hh)
    ctx.free(dh)


def test_evaluation_matches_the_oracle(ctx):
    pop = gen.ramped_half_and_half(51, 100)
    cases = gen.float_cases(52, 300)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, device_compile=True)
    roots, fit, _ = ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, cases.T)
    with np.errstate(all="ignore"):
        want_r, want_f = oracle.eval_population_f32(pop, cases.x, cases.y)
    assert ((roots.view(np.uint32) == want_r.view(np.uint32)) | (np.isnan(roots) & np.isnan(want_r))).all()
    assert all(a == b or (np.isnan(a) and np.isnan(b)) for a, b in zip(fit, want_f))

    bpop = gen.sized_population(53, 20, 101, 20001, n_terms=6, vtype=gen.VT_BOOL)
    bc = gen.bool_cases(6)
    bh = ctx.set_cases(g.GP_BOOL, bc.inputs, bc.target, bc.T)
    bp = ctx.load_population(g.GP_BOOL, bpop.ops, bpop.offsets, n_inputs=6, device_compile=True, chunk_nodes=256)
    broots, bfit, _ = ctx.evaluate_full(bp, bh, g.GP_BOOL, bpop.n_trees, bc.T)
    want_r, want_f = oracle.eval_population_bool(bpop, bc.inputs, bc.target, bc.T)
    assert np.array_equal(broots.view(np.uint64), want_r) and np.array_equal(bfit, want_f)

    # incremental children through parent caches recorded by device-compiled programs
    parents = gen.sized_population(54, 6, 101, 30001)
    kids = gen.crossover_children(55, parents, 12, donor_hi=60)
    pts = [[int(c) for p, c in zip(kids.parent, kids.point) if p == t] for t in range(parents.n_trees)]
    rp, ro = record_lists(pts)
    c2 = gen.float_cases(56, 256)
    ch2 = ctx.set_cases(g.GP_F32, c2.x, c2.y)
    pp = ctx.load_population(g.GP_F32, parents.ops, parents.offsets, record_points=rp, record_offsets=ro,
                             chunk_nodes=512, device_compile=True)
    ctx.evaluate_full(pp, ch2, g.GP_F32, parents.n_trees, c2.T)
    r2, f2, info = ctx.evaluate_incremental(pp, ch2, g.GP_F32, c2.T, kids.parent, kids.point, kids.donors.ops,
                                            kids.donors.offsets)
    for i in range(len(kids.parent)):
        with np.errstate(all="ignore"):
            w_r, w_l, w_i, w_f = oracle.incremental_f32(parents.tree(int(kids.parent[i])), int(kids.point[i]),
                                                        kids.donors.tree(i), c2.x, c2.y)
        assert info["stop_level"][i] == w_l and info["interpreted_nodes"][i] == w_i
        assert ((r2[i].view(np.uint32) == w_r.view(np.uint32)) | (np.isnan(r2[i]) & np.isnan(w_r))).all()
        assert f2[i] == w_f or (np.isnan(f2[i]) and np.isnan(w_f))
    for h in (ph, bp, pp):
        ctx.free(h)


def test_autotune_rechunks_on_the_device(ctx):
    pop = gen.sized_population(61, 16, 1001, 60001)
    cases = gen.float_cases(62, 512)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    dh = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, device_compile=True, keep_trees=True)
    ctx.autotune(dh, ch)
    cn = ctx.population_info(dh)["chunk_nodes"]
    hh = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, chunk_nodes=cn)
    same_dump(ctx.population_dump(hh), ctx.population_dump(dh))
    r1, f1, _ = ctx.evaluate_full(dh, ch, g.GP_F32, pop.n_trees, cases.T)
    r2, f2, _ = ctx.evaluate_full(hh, ch, g.GP_F32, pop.n_trees, cases.T)
    assert np.array_equal(r1.view(np.uint32), r2.view(np.uint32)) and np.array_equal(f1.view(np.uint64),
                                                                                     f2.view(np.uint64))
    ctx.free(hh)
    ctx.free(dh)


def test_errors_match_the_host_compiler(ctx):
    good = np.array([0x80, 0, 0], np.uint8)
    for bad in ([0x80, 0], [0x84, 0, 0], [0x80, 0, 3], [0, 0]):
        trees = [good, np.array(bad, np.uint8)]
        ops = np.concatenate(trees)
        offs = np.array([0, 3, len(ops)], np.int64)
        msgs = []
        for dc in (False, True):
            with pytest.raises(g.GPError) as e:
                ctx.load_population(g.GP_F32, ops, offs, n_inputs=2, device_compile=dc)
            msgs.append(str(e.value))
        assert msgs[0] == msgs[1], msgs
    with pytest.raises(g.GPError, match="prefix"):
        ctx.load_population(g.GP_F32, good[[1, 2, 0]], [0, 3], layout=g.GP_POSTFIX, device_compile=True)
    with pytest.raises(g.GPError, match="out of range"):
        ctx.load_population(g.GP_F32, good, [0, 3], record_points=[3], record_offsets=[0, 1], device_compile=True)
