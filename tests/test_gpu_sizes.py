"""GPU parity at every case count the kernels specialise on.

The walk, co-evaluation and fitness kernels hold R = max(1, P / 256) values per
thread (P = max(64, next power of two >= T)), so float case counts up to
16384 select R = 1 .. 64; Boolean walks hold R = 1, 2, 4 or 16 words per
thread (up to 4096 words, 2^18 cases).  Every R is run here against the
oracle element by element, with ragged case counts between the powers of
two, for full evaluation, the cached walk (Section 6.2, Figure 3) and
co-evaluation with the mother, in prefix and in reverse Polish layout
(Section 3.1).  Outputs must be bit-equal (float: or both NaN), fitness
bit-equal, stop levels and interpreted counts identical.
"""
import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g
from tests.scalar_ref import same_f32

pytestmark = pytest.mark.gpu

POOL = 8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def fit_equal(a, b):
    return (a == b) or (math.isnan(a) and math.isnan(b))


def rows_per_thread(T):
    P = max(64, 1 << (T - 1).bit_length())
    return max(1, P // 256)


def record_lists(parents, parent_idx, points):
    pts = [[] for _ in range(parents.n_trees)]
    for p, c in zip(parent_idx, points):
        if int(c) not in pts[int(p)]:
            pts[int(p)].append(int(c))
    offs = np.zeros(parents.n_trees + 1, np.int64)
    offs[1:] = np.cumsum([len(p) for p in pts])
    flat = np.array([c for p in pts for c in p], np.int64)
    return flat, offs


def oracle_children_f32(parents, kids, cases):
    def one(i):
        with np.errstate(all="ignore"):
            return oracle.incremental_f32(parents.tree(int(kids.parent[i])), int(kids.point[i]),
                                          kids.donors.tree(i), cases.x, cases.y)
    with ThreadPoolExecutor(POOL) as ex:
        return list(ex.map(one, range(len(kids.parent))))


def oracle_children_bool(parents, kids, cases):
    def one(i):
        return oracle.incremental_bool(parents.tree(int(kids.parent[i])), int(kids.point[i]),
                                       kids.donors.tree(i), cases.inputs, cases.target, cases.T)
    with ThreadPoolExecutor(POOL) as ex:
        return list(ex.map(one, range(len(kids.parent))))


def check_f32_children(roots, fit, info, want, parents, kids, cached=True):
    for i, (w_root, w_lvl, w_interp, w_fit) in enumerate(want):
        assert same_f32(roots[i], w_root).all(), (i, int((~same_f32(roots[i], w_root)).sum()))
        assert fit_equal(fit[i], w_fit), (i, fit[i], w_fit)
        assert info["stop_level"][i] == w_lvl, (i, info["stop_level"][i], w_lvl)
        if cached:
            assert info["interpreted_nodes"][i] == w_interp, i
        P = parents.tree(int(kids.parent[i]))
        c = int(kids.point[i])
        assert info["child_nodes"][i] == len(P) - (oracle.subtree_end(P, c) - c) + len(kids.donors.tree(i))


# (T, chunk nodes): R = 8, 8, 16, 16, 32, 32, 64, 64; every other one with
# small chunks, so that co-evaluation reads siblings from the mother's chunks
F32_SIZES = [(1500, 0), (2048, 64), (3001, 0), (4096, 64), (5000, 64), (8192, 0), (12289, 64), (16384, 0)]


@pytest.mark.parametrize("T,chunk_nodes", F32_SIZES)
def test_float_full_walk_and_coeval_every_R(ctx, T, chunk_nodes):
    say("float T", T, "R", rows_per_thread(T), "chunk", chunk_nodes)
    parents = gen.sized_population(700 + T % 97, 6, 101, 2001)
    kids = gen.crossover_children(701 + T % 89, parents, 16, donor_hi=200, neutral_frac=0.5,
                                  one_per_parent=False)
    cases = gen.float_cases(702 + T % 83, T)
    # signed zeros in the inputs; for the odd case counts an infinity and a
    # NaN too (most fitness values are then NaN)
    cases.x[0, 5] = -0.0
    cases.x[0, T - 1] = 0.0
    if T % 2:
        cases.x[0, T // 2] = np.inf
        cases.x[0, T // 3] = np.nan
    with np.errstate(all="ignore"):
        cases.y[:] = gen.sextic(cases.x[0])
    rp, ro = record_lists(parents, kids.parent, kids.point)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, parents.ops, parents.offsets, record_points=rp, record_offsets=ro,
                             chunk_nodes=chunk_nodes)
    proots, pfit, _ = ctx.evaluate_full(ph, ch, g.GP_F32, parents.n_trees, T)
    with np.errstate(all="ignore"):
        w_roots, w_fit = oracle.eval_population_f32(parents, cases.x, cases.y, threads=POOL)
    assert same_f32(proots, w_roots).all()
    for i in range(parents.n_trees):
        assert fit_equal(pfit[i], w_fit[i]), (i, pfit[i], w_fit[i])
    want = oracle_children_f32(parents, kids, cases)
    r1, f1, i1 = ctx.evaluate_incremental(ph, ch, g.GP_F32, T, kids.parent, kids.point, kids.donors.ops,
                                          kids.donors.offsets)
    check_f32_children(r1, f1, i1, want, parents, kids)
    r2, f2, i2 = ctx.evaluate_incremental(ph, ch, g.GP_F32, T, kids.parent, kids.point, kids.donors.ops,
                                          kids.donors.offsets, coeval=True)
    check_f32_children(r2, f2, i2, want, parents, kids, cached=False)
    stops = [w[1] for w in want]
    assert any(s == 0 for s in stops) and any(s != 0 for s in stops)
    # fitness of given vectors (k_fit_f32 at this R) through gp_fitness
    got = ctx.fitness(ch, g.GP_F32, w_roots)
    for i in range(parents.n_trees):
        assert fit_equal(got[i], w_fit[i])
    ctx.free(ph)
    ctx.free(ch)


# k inputs -> 2^k cases in W = 2^(k-6) words: R = 1 (W <= 256), 2, 4, 16
BOOL_K = [9, 10, 12, 14, 15, 16, 17, 18]


@pytest.mark.parametrize("k", BOOL_K)
def test_boolean_full_walk_and_coeval_many_words(ctx, k):
    cases = gen.bool_cases(k)
    W = cases.inputs.shape[1]
    say("bool k", k, "words", W)
    parents = gen.sized_population(800 + k, 6, 101, 2001, n_terms=k, vtype=gen.VT_BOOL)
    kids = gen.crossover_children(801 + k, parents, 16, donor_hi=150, neutral_frac=0.0, n_terms=k,
                                  one_per_parent=False)
    # half the donors neutral: AND(S, OR(R, NAND(R, R))) = S
    rng = np.random.default_rng(802 + k)
    donors = []
    for i in range(len(kids.parent)):
        if i % 2 == 0:
            P = parents.tree(int(kids.parent[i]))
            c = int(kids.point[i])
            S = P[c:oracle.subtree_end(P, c)].copy()
            donors.append(gen.bool_neutral_donor(rng, S, len(S) + 10, k))
        else:
            donors.append(kids.donors.tree(i))
    kids.donors = gen.pack(donors, gen.VT_BOOL, k)
    rp, ro = record_lists(parents, kids.parent, kids.point)
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, parents.ops, parents.offsets, n_inputs=k, record_points=rp,
                             record_offsets=ro, chunk_nodes=64 if k % 2 else 0)
    proots, pfit, _ = ctx.evaluate_full(ph, ch, g.GP_BOOL, parents.n_trees, cases.T)
    w_roots, w_fit = oracle.eval_population_bool(parents, cases.inputs, cases.target, cases.T, threads=POOL)
    assert np.array_equal(proots, w_roots)
    assert np.array_equal(pfit, w_fit)
    want = oracle_children_bool(parents, kids, cases)
    for coeval in (False, True):
        r, f, info = ctx.evaluate_incremental(ph, ch, g.GP_BOOL, cases.T, kids.parent, kids.point,
                                              kids.donors.ops, kids.donors.offsets, coeval=coeval)
        for i, (w_root, w_lvl, w_interp, w_f) in enumerate(want):
            assert np.array_equal(r[i], w_root), (coeval, i)
            assert f[i] == w_f, (coeval, i, f[i], w_f)
            assert info["stop_level"][i] == w_lvl, (coeval, i, info["stop_level"][i], w_lvl)
            if not coeval:
                assert info["interpreted_nodes"][i] == w_interp
    stops = [w[1] for w in want]
    assert any(s == 0 for s in stops) and any(s != 0 for s in stops)
    ctx.free(ph)
    ctx.free(ch)


def to_postfix(t):
    """Reverse Polish form of a prefix tree, and the RPN index of every
    prefix node (operands left then right, then the function)."""
    ends = gen.subtree_ends(t)
    out = []
    where = np.empty(len(t), np.int64)
    stack = [(0, False)]
    while stack:
        i, done = stack.pop()
        if done or not (int(t[i]) & 0x80):
            where[i] = len(out)
            out.append(int(t[i]))
            continue
        stack.append((i, True))
        stack.append((int(ends[i + 1]), False))
        stack.append((i + 1, False))
    return np.array(out, np.uint8), where


@pytest.mark.parametrize("vtype,T,chunk_nodes", [("f32", 300, 0), ("f32", 4096, 64), ("bool", 1024, 32)])
def test_incremental_postfix_population_matches_oracle(ctx, vtype, T, chunk_nodes):
    """A population loaded in reverse Polish order, with points and donors in
    that order, gives the oracle's results for the same children."""
    boolean = vtype == "bool"
    k = T.bit_length() - 1 if boolean else 1
    parents = gen.sized_population(900 + T, 8, 101, 3001, n_terms=k, vtype=gen.VT_BOOL if boolean else gen.VT_F32)
    kids = gen.crossover_children(901 + T, parents, 24, donor_hi=150, neutral_frac=0.0 if boolean else 0.5,
                                  n_terms=k, one_per_parent=False)
    post_trees, where = zip(*[to_postfix(parents.tree(i)) for i in range(parents.n_trees)])
    post = gen.pack(list(post_trees), parents.vtype, k)
    rpn_points = np.array([where[int(p)][int(c)] for p, c in zip(kids.parent, kids.point)], np.int64)
    post_donors = gen.pack([to_postfix(kids.donors.tree(i))[0] for i in range(len(kids.parent))],
                           parents.vtype, k)
    rp, ro = record_lists(parents, kids.parent, rpn_points)
    gt = g.GP_BOOL if boolean else g.GP_F32
    if boolean:
        cases = gen.bool_cases(k)
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    else:
        cases = gen.float_cases(902 + T, T)
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(gt, post.ops, post.offsets, n_inputs=k, layout=g.GP_POSTFIX, record_points=rp,
                             record_offsets=ro, chunk_nodes=chunk_nodes)
    ctx.evaluate_full(ph, ch, gt, parents.n_trees, T)
    r, f, info = ctx.evaluate_incremental(ph, ch, gt, T, kids.parent, rpn_points, post_donors.ops,
                                          post_donors.offsets)
    if boolean:
        want = oracle_children_bool(parents, kids, cases)
        for i, (w_root, w_lvl, w_interp, w_f) in enumerate(want):
            assert np.array_equal(r[i], w_root), i
            assert f[i] == w_f and info["stop_level"][i] == w_lvl and info["interpreted_nodes"][i] == w_interp, i
    else:
        want = oracle_children_f32(parents, kids, cases)
        check_f32_children(r, f, info, want, parents, kids)
    stops = [w[1] for w in want]
    assert any(s != 0 for s in stops)
    # the RPN point of a node that was not recorded is refused, not guessed
    p0 = int(kids.parent[0])
    recorded = set(int(q) for q in rp[ro[p0]:ro[p0 + 1]])
    other = next(q for q in range(len(post.tree(p0))) if q not in recorded)
    d0 = gen.pack([post_donors.tree(0)], parents.vtype, k)
    with pytest.raises(g.GPError) as e:
        ctx.evaluate_incremental(ph, ch, gt, T, [p0], [other], d0.ops, d0.offsets)
    assert e.value.code == g.GP_ENOTFOUND
    ctx.free(ph)
    ctx.free(ch)


def test_case_counts_beyond_the_kernels_are_refused(ctx):
    """Float case sets above 16384 and Boolean above 2^18 cases have no walk
    or fitness kernel; gp_set_cases refuses them."""
    x = np.zeros((1, 16385), np.float32)
    with pytest.raises(g.GPError) as e:
        ctx.set_cases(g.GP_F32, x, x[0])
    assert e.value.code == g.GP_EINVAL
    W = (1 << 18) // 64 + 1
    words = np.zeros((1, W), np.uint64)
    with pytest.raises(g.GPError) as e:
        ctx.set_cases(g.GP_BOOL, words, words[0], W * 64)
    assert e.value.code == g.GP_EINVAL
