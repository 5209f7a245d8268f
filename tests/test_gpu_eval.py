"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Outputs must be bit-exact per test case (both NaN counts as equal), fitness
bit-exact, incremental stop levels and interpreted counts identical.
"""
import math
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


def f32_variants():
    return [i for i, n in enumerate(g.variant_names()) if n.startswith("f32")]


def bool_variants():
    return [i for i, n in enumerate(g.variant_names()) if n.startswith("bool")]


def fit_equal(a, b):
    return (a == b) or (math.isnan(a) and math.isnan(b))


def check_float_pop(ctx, pop_np, cases, chunk_nodes=0, per_tree=False, graph=True, variant=-1, threads=8):
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop_np.ops, pop_np.offsets, n_inputs=cases.x.shape[0],
                             chunk_nodes=chunk_nodes)
    ctx.set_variant(variant)
    roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_F32, pop_np.n_trees, cases.T, per_tree=per_tree, graph=graph)
    ctx.set_variant(-1)
    with np.errstate(all="ignore"):
        want_roots, want_fit = oracle.eval_population_f32(pop_np, cases.x, cases.y, threads=threads)
    ok = same_f32(roots, want_roots)
    assert ok.all(), f"{(~ok).sum()} cases differ; first tree {np.argwhere(~ok)[0]}"
    for i in range(pop_np.n_trees):
        assert fit_equal(fit[i], want_fit[i]), (i, fit[i], want_fit[i])
    assert st["equivalent_ops"] == pop_np.sizes().sum() * cases.T
    ctx.free(ph)
    ctx.free(ch)
    return st


def test_cfg0_ramped_half_and_half_all_variants(ctx):
    pop = gen.ramped_half_and_half(1)
    cases = gen.float_cases(1, 48)
    for v in f32_variants():
        say("cfg0 variant", g.variant_names()[v])
        check_float_pop(ctx, pop, cases, variant=v)
        check_float_pop(ctx, pop, cases, variant=v, per_tree=True, graph=False)


def test_sextic_target_scores_zero_on_gpu(ctx):
    cases = gen.float_cases(2, 333)
    pop = gen.pack([gen.sextic_tree(), np.array([0], np.uint8)])
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets)
    roots, fit, _ = ctx.evaluate_full(ph, ch, g.GP_F32, 2, cases.T)
    assert np.all(roots[0].view(np.uint32) == cases.y.view(np.uint32))
    assert fit[0] == 0.0
    assert np.all(roots[1] == cases.x[0])
    ctx.free(ph)
    ctx.free(ch)


def test_special_values_and_two_inputs(ctx):
    rng = np.random.default_rng(3)
    x0 = np.array([0, -0.0, 1e-7, -1e-7, 1e-6, 1e-20, 1e30, -3e38, np.inf, -np.inf, np.nan, 1.0, 2.5, -7.0,
                   1e-45, 3.0], np.float32)
    x = np.stack([x0, x0[::-1].copy()])
    y = np.zeros(len(x0), np.float32)
    cases = gen.FloatCases(x, y)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 401)), n_terms=2) for _ in range(60)]
    pop = gen.pack(trees, n_inputs=2)
    for v in f32_variants():
        check_float_pop(ctx, pop, cases, chunk_nodes=32, variant=v)


def _signed_pow2(rng, lo, hi, n):
    return (np.exp2(rng.uniform(lo, hi, n)) * rng.choice([-1.0, 1.0], n)).astype(np.float32)


def _short_divide_cases():
    """16384 cases over three inputs in blocks of 512 (one wave slice for
    K = 8, two for K = 4): blocks that keep every value inside the
    short-divide ranges (exact bounds included), blocks with one value just
    outside, blocks of extremes and blocks like the benchmark's inputs."""
    rng = np.random.default_rng(77)
    B = 512
    up = lambda v: np.nextafter(np.float32(v), np.float32(np.inf))
    down = lambda v: np.nextafter(np.float32(v), np.float32(0))
    cols = [[], [], []]
    for blk in range(32):
        kind = blk % 10
        if kind in (0, 1):      # stack / x short path: |x0| <= 2^20, |x1| in [2^-90, 2^70]
            x0 = _signed_pow2(rng, -19.9, 20, B)
            x1 = _signed_pow2(rng, -90, 70, B)
            x2 = _signed_pow2(rng, -25, 36, B)
            x0[:6] = [1e-6, -1e-6, 2.0 ** 20, -(2.0 ** 20), 0.0, 1e-7]          # protected lanes allowed
            x1[:4] = [2.0 ** -90, -(2.0 ** -90), 2.0 ** 70, -(2.0 ** 70)]
            x2[:6] = [2.0 ** 36, -(2.0 ** 36), 1e-6, 0.0, -0.0, 1e-45]
        elif kind in (2, 3):    # x / stack short path: x0 in [2^-60, 2^60], |x1| <= 2^64
            x0 = _signed_pow2(rng, -60, 60, B)
            x1 = _signed_pow2(rng, -25, 64, B)
            x2 = _signed_pow2(rng, -25, 36, B)
            x0[:4] = [2.0 ** -60, -(2.0 ** -60), 2.0 ** 60, -(2.0 ** 60)]
            x1[:8] = [2.0 ** 64, -(2.0 ** 64), 1e-6, 9.99e-7, 0.0, -0.0, 1e-45, -1e-7]
        elif kind == 4:         # one value just outside each range
            x0 = _signed_pow2(rng, -19.9, 20, B)
            x1 = _signed_pow2(rng, -60, 60, B)
            x2 = _signed_pow2(rng, -20, 20, B)
            x0[rng.integers(B)] = up(2.0 ** 20)
            x1[rng.integers(B)] = up(2.0 ** 70)
            x1[rng.integers(B)] = down(2.0 ** -90)
            x1[rng.integers(B)] = up(2.0 ** 64)
            x2[rng.integers(B)] = up(2.0 ** 36)
        elif kind == 5:         # x just outside [2^-60, 2^60]
            x0 = _signed_pow2(rng, -60, 60, B)
            x1 = _signed_pow2(rng, -20, 20, B)
            x2 = _signed_pow2(rng, -20, 20, B)
            x0[rng.integers(B)] = down(2.0 ** -60)
            x0[rng.integers(B)] = up(2.0 ** 60)
        elif kind == 6:         # extremes
            pool = np.array([0.0, -0.0, 1e-45, -1e-40, 1.17549435e-38, 1e-30, 3.4e38, -3.4e38, np.inf, -np.inf,
                             np.nan, 1e-6, 2.0 ** 100, 2.0 ** -100, 1.0, -2.5], np.float32)
            x0, x1, x2 = (rng.choice(pool, B) for _ in range(3))
        elif kind == 8:         # stack / stack short path: |x1| in [2^-60, 2^60], |x2| <= 2^64
            x0 = _signed_pow2(rng, -20, 20, B)
            x1 = _signed_pow2(rng, -60, 60, B)
            x2 = _signed_pow2(rng, -25, 64, B)
            x1[:4] = [2.0 ** -60, -(2.0 ** -60), 2.0 ** 60, -(2.0 ** 60)]
            x2[:8] = [2.0 ** 64, -(2.0 ** 64), 1e-6, 9.99e-7, 0.0, -0.0, 1e-45, -1e-7]
            if (blk // 10) % 2:     # a NaN operand, passed over by the range check
                x1[rng.integers(8, B)] = np.nan
                x2[rng.integers(8, B)] = np.nan
        elif kind == 9:         # stack / stack: one value just outside
            x0 = _signed_pow2(rng, -20, 20, B)
            x1 = _signed_pow2(rng, -60, 60, B)
            x2 = _signed_pow2(rng, -25, 64, B)
            which = (blk // 10) % 3
            j = rng.integers(B)
            if which == 0:
                x1[j] = down(2.0 ** -60)
            elif which == 1:
                x1[j] = -up(2.0 ** 60)
            else:
                x2[j] = up(2.0 ** 64)
                x2[(j + 1) % B] = -np.inf
        else:                   # like the benchmark: uniform in [-1, 1]
            x0, x1, x2 = (rng.uniform(-1, 1, B).astype(np.float32) for _ in range(3))
        for c, v in zip(cols, (x0, x1, x2)):
            c.append(v)
    x = np.stack([np.concatenate(c) for c in cols]).astype(np.float32)
    return gen.FloatCases(x, np.zeros(x.shape[1], np.float32))


def _near_midpoint_pairs(rng, n, a_exp, b_exp):
    """(a, b) float32 pairs whose quotient lies within 63 * 2^-48 (relative)
    of a midpoint between floats: for an odd 24-bit significand B and small
    odd k, M = k / B mod 2^25 (odd, 25 bits) and X = (B*M - k) / 2^25 give
    X / B = M / 2^25 - k / (2^25 B).  Exponents are drawn from a_exp, b_exp."""
    out_a, out_b = [], []
    while sum(len(v) for v in out_a) < n:
        B = (rng.integers(0, 1 << 23, 4096, dtype=np.uint64) | np.uint64(0x800001))
        inv = B.copy()
        for _ in range(5):                              # Newton's iteration for 1/B mod 2^32
            inv = (inv * (np.uint64(2) - B * inv)) & np.uint64(0xffffffff)
        k = (rng.integers(0, 32, B.size) * 2 - 63).astype(np.int64)
        M = ((inv * (k.astype(np.uint64) & np.uint64(0xffffffff))) & np.uint64(0x1ffffff)).astype(np.int64)
        num = B.astype(np.int64) * M - k
        assert not np.any(num & 0x1ffffff)
        X = num >> 25
        ok = (M >= 1 << 24) & (X >= 1 << 23) & (X < 1 << 24)
        X, Bk = X[ok], B[ok].astype(np.int64)
        ea = rng.integers(a_exp[0], a_exp[1], X.size)
        eb = rng.integers(b_exp[0], b_exp[1], X.size)
        sa = rng.choice([-1.0, 1.0], X.size)
        sb = rng.choice([-1.0, 1.0], X.size)
        out_a.append((sa * np.ldexp(X.astype(np.float64), ea - 23)).astype(np.float32))
        out_b.append((sb * np.ldexp(Bk.astype(np.float64), eb - 23)).astype(np.float32))
    return np.concatenate(out_a)[:n], np.concatenate(out_b)[:n]


def test_short_divides_near_midpoints(ctx):
    """Quotients next to rounding midpoints, the hardest inputs for a
    division by reciprocal, through every form of the short divide (x /
    stack, stack / stack, stack / x), unprotected and, in one slice, with a
    protected divisor; against the oracle's IEEE division."""
    from tests.golden_cases import parse_tree
    rng = np.random.default_rng(91)
    s0, s1 = "(+ x0 (- x1 x1))", "(+ x1 (- x0 x0))"
    xs_ss = gen.pack([parse_tree(t) for t in [f"(% x0 {s1})", f"(% {s0} {s1})", f"(% {s0} (% {s1} (* x0 x0)))"]],
                     n_inputs=3)
    sx = gen.pack([parse_tree(t) for t in [f"(% {s1} x0)", f"(- (% {s1} x0) x0)"]], n_inputs=3)
    T = 16384
    for rep in range(3):
        a, b = _near_midpoint_pairs(rng, T, (-59, 59), (-20, 63))    # x0 = a, x1 = b
        b[7] = np.float32(1e-7)                                      # one protected divisor
        cases = gen.FloatCases(np.stack([a, b, b]), np.zeros(T, np.float32))
        for v in f32_variants():
            check_float_pop(ctx, xs_ss, cases, variant=v)
        a, b = _near_midpoint_pairs(rng, T, (-89, 69), (-20, 19))    # x0 = b (the divisor), x1 = a
        cases = gen.FloatCases(np.stack([b, a, a]), np.zeros(T, np.float32))
        for v in f32_variants():
            check_float_pop(ctx, sx, cases, variant=v)
    say("near-midpoint divides: ok")


def test_reciprocal_every_float_of_a_binade(ctx):
    """1 / b for every float b in [1, 2) (all 2^23 significands, both signs
    alternating), through the x / stack short divide of each table-dispatch
    variant, against the oracle's IEEE division."""
    from tests.golden_cases import parse_tree
    tree = parse_tree("(% x0 (+ x1 (- x0 x0)))")
    pop = gen.pack([tree], n_inputs=2)
    T = 16384
    sig = np.arange(1 << 23, dtype=np.uint32)
    b_all = (np.uint32(127 << 23) | sig).view(np.float32) * np.where(sig & 1, -1, 1).astype(np.float32)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, n_inputs=2)
    names = g.variant_names()
    tbl = [v for v in f32_variants() if names[v].startswith(("f32t_", "f32d_"))]
    assert tbl
    for blk in range(0, b_all.size, T):
        b = b_all[blk:blk + T]
        x = np.stack([np.ones(T, np.float32), b])
        ch = ctx.set_cases(g.GP_F32, x, np.zeros(T, np.float32))
        want = oracle.eval_f32(tree, x)
        for v in tbl:
            ctx.set_variant(v)
            roots, _, _ = ctx.evaluate_full(ph, ch, g.GP_F32, 1, T)
            assert np.array_equal(roots[0].view(np.uint32), want.view(np.uint32)), (names[v], blk)
        ctx.set_variant(-1)
        ctx.free(ch)
    ctx.free(ph)


def test_short_divides_bit_exact(ctx):
    """Divisions by x, of x and of one stack value by another, with operands
    at, inside and just outside the ranges where the table-dispatch loop
    takes its short divide (NaN operands included), against the oracle's
    IEEE division."""
    from tests.golden_cases import parse_tree
    cases = _short_divide_cases()
    a1 = "(+ x1 (- x0 x0))"                  # x1 on the stack (x0 - x0 = +0 for finite x0)
    a2 = "(+ x2 (- x0 x0))"
    trees = [f"(% {a1} x0)", f"(% x0 {a1})", f"(% (% {a1} x0) x0)", f"(% x0 (% x0 {a1}))",
             f"(% (* {a1} x0) x0)", f"(% (% x0 {a1}) (% {a1} x0))", f"(- (% {a1} x0) (% x0 {a1}))",
             f"(% {a1} {a2})", f"(% (+ (- x0 x0) {a1}) {a2})", f"(% {a1} (+ (- x0 x0) {a2}))",
             f"(% {a2} (% {a1} {a2}))", f"(% (% {a1} {a2}) (* {a2} {a2}))", f"(% {a1} (+ {a2} (- {a2} {a1})))"]
    pop = gen.pack([parse_tree(t) for t in trees], n_inputs=3)
    for v in f32_variants():
        say("short divides", g.variant_names()[v])
        check_float_pop(ctx, pop, cases, variant=v)


@pytest.mark.parametrize("chunk_nodes", [16, 300, 4096])
def test_multi_chunk_ragged_cases(ctx, chunk_nodes):
    pop = gen.sized_population(11, 24, 101, 30001)
    cases = gen.float_cases(5, 300)            # not a multiple of 64
    for v in f32_variants():
        say("multi-chunk", chunk_nodes, g.variant_names()[v])
        check_float_pop(ctx, pop, cases, chunk_nodes=chunk_nodes, variant=v)
    check_float_pop(ctx, pop, cases, chunk_nodes=chunk_nodes, per_tree=True)


def test_results_independent_of_batch(ctx):
    pop = gen.sized_population(12, 30, 11, 5001)
    cases = gen.float_cases(6, 1024)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets, chunk_nodes=128)
    r_all, f_all, _ = ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, cases.T)
    for rep in range(3):
        r2, f2, _ = ctx.evaluate_full(ph, ch, g.GP_F32, pop.n_trees, cases.T)
        assert np.array_equal(r_all.view(np.uint32), r2.view(np.uint32))
    for i in [0, 7, 29]:
        one = gen.pack([pop.tree(i)])
        p1 = ctx.load_population(g.GP_F32, one.ops, one.offsets, chunk_nodes=4096)
        r1, f1, _ = ctx.evaluate_full(p1, ch, g.GP_F32, 1, cases.T)
        assert np.array_equal(r1[0].view(np.uint32), r_all[i].view(np.uint32))
        assert f1[0] == f_all[i] or (np.isnan(f1[0]) and np.isnan(f_all[i]))
        ctx.free(p1)
    ctx.free(ph)
    ctx.free(ch)


def test_postfix_layout(ctx):
    rng = np.random.default_rng(21)
    cases = gen.float_cases(7, 64)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 999))) for _ in range(10)]

    def to_postfix(t):
        ends = gen.subtree_ends(t)
        out = []

        def rec(i):
            if t[i] & 0x80:
                rec(i + 1)
                rec(int(ends[i + 1]))
            out.append(int(t[i]))
        sys.setrecursionlimit(10000)
        rec(0)
        return np.array(out, np.uint8)

    pre = gen.pack(trees)
    post = gen.pack([to_postfix(t) for t in trees])
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    a = ctx.load_population(g.GP_F32, pre.ops, pre.offsets)
    b = ctx.load_population(g.GP_F32, post.ops, post.offsets, layout=g.GP_POSTFIX)
    ra, fa, _ = ctx.evaluate_full(a, ch, g.GP_F32, 10, 64)
    rb, fb, _ = ctx.evaluate_full(b, ch, g.GP_F32, 10, 64)
    assert same_f32(ra, rb).all()
    ctx.free(a)
    ctx.free(b)
    ctx.free(ch)


def test_gp_fitness_entry_point(ctx):
    rng = np.random.default_rng(9)
    for T in [1, 48, 65, 1024, 4096]:
        cases = gen.float_cases(T, T)
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
        outs = rng.normal(size=(5, T)).astype(np.float32)
        outs[0, 0] = np.nan
        got = ctx.fitness(ch, g.GP_F32, outs)
        for i in range(5):
            assert fit_equal(got[i], oracle.fitness_f32(outs[i], cases.y))
        ctx.free(ch)


# ------------------------------------------------------------------ Boolean
def check_bool_pop(ctx, pop, cases, chunk_nodes=0, variant=-1, per_tree=False):
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=cases.inputs.shape[0],
                             chunk_nodes=chunk_nodes)
    ctx.set_variant(variant)
    roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T, per_tree=per_tree)
    ctx.set_variant(-1)
    want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
    W = (cases.T + 63) // 64
    assert roots.shape == (pop.n_trees, W)
    assert np.array_equal(roots, want_roots)
    assert np.array_equal(fit, want_fit)
    ctx.free(ph)
    ctx.free(ch)


def test_boolean_parity6_small(ctx):
    cases = gen.bool_cases(6)
    pop = gen.sized_population(2, 60, 11, 20001, n_terms=6, vtype=gen.VT_BOOL)
    x = [0]
    for j in range(1, 6):
        x = [gen.B_NOR, gen.B_AND] + x + [j] + [gen.B_NOR] + x + [j]
    even6 = np.array([gen.B_NOR] + x + x, np.uint8)
    trees = [pop.tree(i) for i in range(pop.n_trees)] + [even6, np.array([3], np.uint8)]
    pop = gen.pack(trees, gen.VT_BOOL, 6)
    for v in bool_variants():
        for C in [32, 0]:
            say("bool6 variant", g.variant_names()[v], C)
            check_bool_pop(ctx, pop, cases, chunk_nodes=C, variant=v)
    check_bool_pop(ctx, pop, cases, per_tree=True)


@pytest.mark.parametrize("k", [8, 10, 12])
def test_boolean_multiword(ctx, k):
    cases = gen.bool_cases(k)
    pop = gen.sized_population(3 + k, 20, 11, 5001, n_terms=k, vtype=gen.VT_BOOL)
    for v in bool_variants():
        check_bool_pop(ctx, pop, cases, chunk_nodes=64, variant=v)


@pytest.mark.parametrize("k,C", [(6, 32), (6, 300), (8, 64), (12, 128), (16, 64)])
def test_boolean_table_variants(ctx, k, C):
    """The table-dispatch Boolean loops, which hold up to 16 input rows in
    registers, against the oracle; the forced variant must be the one that ran."""
    cases = gen.bool_cases(k)
    pop = gen.sized_population(40 + k, 24, 11, 5001, n_terms=k, vtype=gen.VT_BOOL)
    trees = [pop.tree(i) for i in range(pop.n_trees)] + [np.array([k - 1], np.uint8)]
    pop = gen.pack(trees, gen.VT_BOOL, k)
    names = g.variant_names()
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=k, chunk_nodes=C)
    assert ctx.population_info(ph)["max_stack"] <= 10
    want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
    table = [v for v, n in enumerate(names) if n.startswith("boolt")]
    assert table
    for v in table:
        say("bool table", names[v], k, C)
        ctx.set_variant(v)
        roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T)
        ctx.set_variant(-1)
        assert st["variant"] == v
        assert np.array_equal(roots, want_roots)
        assert np.array_equal(fit, want_fit)
    ctx.free(ph)
    ctx.free(ch)


@pytest.mark.parametrize("k,C", [(1, 7), (3, 13), (5, 32), (6, 7), (6, 64), (6, 300), (6, 900), (6, 2000),
                                 (8, 48)])
def test_boolean_one_word_variant(ctx, k, C):
    """The one-word loop (all cases in one 64-bit word, evaluated on the scalar
    unit) against the oracle: every operand mode, chunks with more LOADs than
    are fetched ahead (complete trees cut into small chunks), programs longer
    than the lines touched at chunk start, one-node trees, and a case set of
    64 random cases over 8 inputs.  It is the default choice for such case
    sets."""
    rng = np.random.default_rng(90 + k + C)
    if k == 8:
        inputs = rng.integers(0, 2 ** 63, size=(8, 1), dtype=np.uint64)
        target = rng.integers(0, 2 ** 63, size=1, dtype=np.uint64)
        cases = gen.BoolCases(inputs, target, 64)
    else:
        cases = gen.bool_cases(k)
    pop = gen.sized_population(80 + k, 30, 11, 20001, n_terms=k, vtype=gen.VT_BOOL)
    trees = [pop.tree(i) for i in range(pop.n_trees)] + [np.array([k - 1], np.uint8)]
    full = gen.ramped_half_and_half(81 + k, 20, min_depth=6, max_depth=9, n_terms=k, max_nodes=1100,
                                     vtype=gen.VT_BOOL)
    trees += [full.tree(i) for i in range(full.n_trees)]
    pop = gen.pack(trees, gen.VT_BOOL, k)
    names = g.variant_names()
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=k, chunk_nodes=C)
    want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
    assert ctx.population_info(ph)["max_code_len"] > 1024 or C < 2000
    try:
        roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T)
        assert names[st["variant"]] == "boolw_s10"
        assert np.array_equal(roots, want_roots)
        assert np.array_equal(fit, want_fit)
        for w in (1, 3):
            ctx.set_launch_width(w)
            roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T, graph=False)
            assert names[st["variant"]] == "boolw_s10"
            assert np.array_equal(roots, want_roots)
            assert np.array_equal(fit, want_fit)
    finally:
        ctx.set_launch_width(-1)
        ctx.free(ph)
        ctx.free(ch)


def test_boolean_one_word_variant_limits(ctx):
    """More than one word of cases, or more inputs than the loop holds in
    SGPRs: the one-word loop is passed over even when forced."""
    names = g.variant_names()
    w = names.index("boolw_s10")
    for k, T in ((7, 128), (9, 64)):
        if T == 128:
            cases = gen.bool_cases(k)
        else:
            rng = np.random.default_rng(k)
            cases = gen.BoolCases(rng.integers(0, 2 ** 63, size=(k, 1), dtype=np.uint64),
                                  rng.integers(0, 2 ** 63, size=1, dtype=np.uint64), T)
        pop = gen.sized_population(95 + k, 8, 11, 3001, n_terms=k, vtype=gen.VT_BOOL)
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
        ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=k, chunk_nodes=32)
        ctx.set_variant(w)
        try:
            roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T)
        finally:
            ctx.set_variant(-1)
        assert st["variant"] != w
        want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
        assert np.array_equal(roots, want_roots)
        assert np.array_equal(fit, want_fit)
        ctx.free(ph)
        ctx.free(ch)


@pytest.mark.parametrize("vtype,C", [(gen.VT_BOOL, 32), (gen.VT_BOOL, 2000), (gen.VT_F32, 64)])
def test_launch_width(ctx, vtype, C):
    """Capping the resident waves per CU (down to one) leaves every result
    unchanged; the cap that ran is reported; the autotuner's choice is the one
    later calls use."""
    if vtype == gen.VT_BOOL:
        cases = gen.bool_cases(6)
        pop = gen.sized_population(71, 40, 11, 20001, n_terms=6, vtype=gen.VT_BOOL)
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
        want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
        vt = g.GP_BOOL
    else:
        cases = gen.float_cases(72, 300)
        pop = gen.sized_population(72, 40, 11, 8001)
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
        with np.errstate(all="ignore"):
            want_roots, want_fit = oracle.eval_population_f32(pop, cases.x, cases.y, threads=8)
        vt = g.GP_F32
    ph = ctx.load_population(vt, pop.ops, pop.offsets, n_inputs=pop.n_inputs, chunk_nodes=C)

    def check(st, roots, fit):
        if vt == g.GP_BOOL:
            assert np.array_equal(roots, want_roots)
            assert np.array_equal(fit, want_fit)
        else:
            assert same_f32(roots, want_roots).all()
            assert all(fit_equal(a, b) for a, b in zip(fit, want_fit))

    try:
        for w in (1, 2, 5, 0):
            ctx.set_launch_width(w)
            for graph in (True, False):
                roots, fit, st = ctx.evaluate_full(ph, ch, vt, pop.n_trees, cases.T, graph=graph)
                say("width", w, "variant", g.variant_names()[st["variant"]], "graph", graph)
                assert st["waves_per_cu"] == w
                check(st, roots, fit)
        with pytest.raises(g.GPError):
            ctx.set_launch_width(-2)
        ctx.set_launch_width(-1)
        v, _ = ctx.autotune(ph, ch)
        roots, fit, st = ctx.evaluate_full(ph, ch, vt, pop.n_trees, cases.T)
        say("tuned", g.variant_names()[v], st["waves_per_cu"])
        assert st["variant"] == v and st["waves_per_cu"] >= 0
        check(st, roots, fit)
    finally:
        ctx.set_launch_width(-1)
        ctx.free(ph)
        ctx.free(ch)


def test_tuning_saved_and_loaded(ctx, tmp_path):
    """gp_tuning_save writes the autotuner's choice (variant, launch width,
    chunk size) keyed by device and buckets; another context that loads it
    applies the same choice without timing the others (recompiling an
    automatically chunked population at the saved chunk size) and gets the
    oracle's results.  Malformed and missing files are refused; lines for
    another device are skipped."""
    import json
    cases = gen.bool_cases(6)
    pop = gen.sized_population(73, 60, 101, 20001, n_terms=6, vtype=gen.VT_BOOL)
    want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
    names = g.variant_names()
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=6)
    v, _ = ctx.autotune(ph, ch)
    info = ctx.population_info(ph)
    _, _, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T)
    path = str(tmp_path / "tuning.jsonl")
    ctx.tuning_save(path)
    lines = [json.loads(line) for line in open(path)]
    mine = [e for e in lines if e["vtype"] == g.GP_BOOL and e["variant"] == names[v]]
    assert mine and mine[0]["chunk_nodes"] == info["chunk_nodes"] and mine[0]["waves_per_cu"] == st["waves_per_cu"]
    ctx.free(ph)
    ctx.free(ch)

    c2 = g.Context(0)
    try:
        c2.tuning_load(path)
        ch2 = c2.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
        ph2 = c2.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=6, chunk_nodes=1024)
        roots, fit, st2 = c2.evaluate_full(ph2, ch2, g.GP_BOOL, pop.n_trees, cases.T)
        assert st2["variant"] == v and st2["waves_per_cu"] == st["waves_per_cu"]      # loaded choice, no tuning
        assert np.array_equal(roots, want_roots) and np.array_equal(fit, want_fit)
        ph3 = c2.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=6)
        v3, _ = c2.autotune(ph3, ch2)
        assert v3 == v and c2.population_info(ph3)["chunk_nodes"] == info["chunk_nodes"]
        roots, fit, _ = c2.evaluate_full(ph3, ch2, g.GP_BOOL, pop.n_trees, cases.T)
        assert np.array_equal(roots, want_roots) and np.array_equal(fit, want_fit)

        bad = str(tmp_path / "bad.jsonl")
        open(bad, "w").write('{"device": "x", "vtype": 1\n')
        with pytest.raises(g.GPError) as e:
            c2.tuning_load(bad)
        assert e.value.code == g.GP_EINVAL
        open(bad, "w").write('{"device": "x", "vtype": 1, "t_bucket": 6}\n')
        with pytest.raises(g.GPError) as e:
            c2.tuning_load(bad)
        assert e.value.code == g.GP_EINVAL
        with pytest.raises(g.GPError) as e:
            c2.tuning_load(str(tmp_path / "missing.jsonl"))
        assert e.value.code == g.GP_ENOTFOUND
        other = str(tmp_path / "other.jsonl")
        open(other, "w").write(open(path).read().replace(lines[0]["device"], "gfx000:1"))
        c3 = g.Context(0)
        try:
            c3.tuning_load(other)
            c3.tuning_save(str(tmp_path / "none.jsonl"))
            assert open(str(tmp_path / "none.jsonl")).read() == ""
        finally:
            c3.close()
    finally:
        c2.close()


def test_boolean_table_variants_refuse_many_inputs(ctx):
    """With more input rows than the registers hold, a forced table variant is
    passed over for one that stages the inputs in LDS."""
    k = 17
    cases = gen.bool_cases(k)
    pop = gen.sized_population(57, 6, 11, 2001, n_terms=k, vtype=gen.VT_BOOL)
    names = g.variant_names()
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    ph = ctx.load_population(g.GP_BOOL, pop.ops, pop.offsets, n_inputs=k, chunk_nodes=64)
    ctx.set_variant(names.index("boolt_k2_s10"))
    roots, fit, st = ctx.evaluate_full(ph, ch, g.GP_BOOL, pop.n_trees, cases.T)
    ctx.set_variant(-1)
    assert not names[st["variant"]].startswith("boolt")
    want_roots, want_fit = oracle.eval_population_bool(pop, cases.inputs, cases.target, cases.T, threads=8)
    assert np.array_equal(roots, want_roots)
    assert np.array_equal(fit, want_fit)
    ctx.free(ph)
    ctx.free(ch)


# -------------------------------------------------------------- incremental
def make_children(parents, seed, n, donor_hi=200, neutral_frac=0.5, n_terms=1):
    return gen.crossover_children(seed, parents, n, donor_hi=donor_hi, neutral_frac=neutral_frac,
                                  n_terms=n_terms, one_per_parent=False)


def record_lists(parents, children):
    pts = [[] for _ in range(parents.n_trees)]
    for p, c in zip(children.parent, children.point):
        pts[int(p)].append(int(c))
    offs = np.zeros(parents.n_trees + 1, np.int64)
    offs[1:] = np.cumsum([len(p) for p in pts])
    flat = np.array([c for p in pts for c in p], np.int64)
    return flat, offs


@pytest.mark.parametrize("chunk_nodes,T,variant", [(64, 100, ""), (4096, 1024, ""), (0, 48, ""),
                                                   (64, 300, "f32t_k4_s10"), (2048, 1024, "f32t_k8_s10")])
def test_incremental_float_matches_oracle(ctx, chunk_nodes, T, variant):
    parents = gen.sized_population(31, 12, 101, 20001)
    children = make_children(parents, 32, 60)
    cases = gen.float_cases(33, T)
    rp, ro = record_lists(parents, children)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, parents.ops, parents.offsets, record_points=rp, record_offsets=ro,
                             chunk_nodes=chunk_nodes)
    if variant:
        assert ctx.population_info(ph)["max_stack"] <= 10
        ctx.set_variant(g.variant_names().index(variant))
    proots, pfit, st = ctx.evaluate_full(ph, ch, g.GP_F32, parents.n_trees, T)
    if variant:
        assert g.variant_names()[st["variant"]] == variant
    roots, fit, info = ctx.evaluate_incremental(ph, ch, g.GP_F32, T, children.parent, children.point,
                                                children.donors.ops, children.donors.offsets)
    ctx.set_variant(-1)
    stops = []
    for i in range(len(children.parent)):
        P = parents.tree(int(children.parent[i]))
        c = int(children.point[i])
        D = children.donors.tree(i)
        with np.errstate(all="ignore"):
            w_root, w_lvl, w_interp, w_fit = oracle.incremental_f32(P, c, D, cases.x, cases.y)
        assert same_f32(roots[i], w_root).all(), i
        assert fit_equal(fit[i], w_fit), (i, fit[i], w_fit)
        assert info["stop_level"][i] == w_lvl, (i, info["stop_level"][i], w_lvl)
        assert info["interpreted_nodes"][i] == w_interp
        assert info["child_nodes"][i] == len(P) - (oracle.subtree_end(P, c) - c) + len(D)
        if children.neutral[i]:
            assert w_lvl == 0
        stops.append(w_lvl)
    assert any(s > 0 for s in stops) and any(s == 0 for s in stops)
    ctx.free(ph)
    ctx.free(ch)


def test_incremental_boolean_matches_oracle(ctx):
    cases = gen.bool_cases(6)
    parents = gen.sized_population(41, 10, 101, 5001, n_terms=6, vtype=gen.VT_BOOL)
    children = make_children(parents, 42, 50, donor_hi=100, n_terms=6)
    rp, ro = record_lists(parents, children)
    ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, 64)
    ph = ctx.load_population(g.GP_BOOL, parents.ops, parents.offsets, n_inputs=6, record_points=rp,
                             record_offsets=ro, chunk_nodes=64)
    ctx.evaluate_full(ph, ch, g.GP_BOOL, parents.n_trees, 64)
    roots, fit, info = ctx.evaluate_incremental(ph, ch, g.GP_BOOL, 64, children.parent, children.point,
                                                children.donors.ops, children.donors.offsets)
    for i in range(len(children.parent)):
        P = parents.tree(int(children.parent[i]))
        w_root, w_lvl, w_interp, w_fit = oracle.incremental_bool(P, int(children.point[i]),
                                                                 children.donors.tree(i), cases.inputs,
                                                                 cases.target, 64)
        assert np.array_equal(roots[i], w_root)
        assert fit[i] == w_fit
        assert info["stop_level"][i] == w_lvl
        assert info["interpreted_nodes"][i] == w_interp
    ctx.free(ph)
    ctx.free(ch)


def _coeval_bounds(P, c, D, walked):
    """Bounds of the co-evaluation's executed-node count: the donor and two
    nodes per walked level at least (subtrees may be read whole from the
    mother's chunk values), the removed subtree and every sibling at most."""
    from paper_2205_03251_amd.gpeval import inspect_path
    levels, e = inspect_path(P, c)
    sib = [int(r[2] - r[1]) for r in levels]
    return len(D) + 2 * walked, len(D) + (e - c) + sum(sib) + 2 * walked


@pytest.mark.parametrize("T,vtype,chunk_nodes", [(300, "f32", 0), (300, "f32", 16), (1024, "f32", 0),
                                                 (64, "bool", 0)])
def test_coeval_matches_cached_walk_and_oracle(ctx, T, vtype, chunk_nodes):
    """Co-evaluating the mother (no parent caches) gives the cached walk's
    outputs, fitness and stop levels, and the oracle's, also for points that
    were never recorded.  With 16-node chunks most float siblings and removed
    subtrees are read from the mother's chunk values rather than evaluated."""
    boolean = vtype == "bool"
    nt = 6 if boolean else 1
    parents = gen.sized_population(35, 10, 101, 20001, n_terms=nt, vtype=gen.VT_BOOL if boolean else gen.VT_F32)
    kids = gen.crossover_children(36, parents, 60, donor_hi=200, neutral_frac=0.5, n_terms=nt, one_per_parent=False)
    extra = gen.crossover_children(37, parents, 20, donor_hi=50, neutral_frac=0.3, n_terms=nt, one_per_parent=False)
    extra.point[:4] = 0                                   # the whole tree replaced
    gt = g.GP_BOOL if boolean else g.GP_F32
    if boolean:
        cases = gen.bool_cases(6)
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, 64)
    else:
        cases = gen.float_cases(39, T)
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    rp, ro = record_lists(parents, kids)
    ph = ctx.load_population(gt, parents.ops, parents.offsets, n_inputs=nt, record_points=rp, record_offsets=ro,
                             chunk_nodes=chunk_nodes)
    ctx.evaluate_full(ph, ch, gt, parents.n_trees, T)
    r1, f1, i1 = ctx.evaluate_incremental(ph, ch, gt, T, kids.parent, kids.point, kids.donors.ops, kids.donors.offsets)
    r2, f2, i2 = ctx.evaluate_incremental(ph, ch, gt, T, kids.parent, kids.point, kids.donors.ops, kids.donors.offsets,
                                          coeval=True)
    assert np.array_equal(i1["stop_level"], i2["stop_level"])
    if boolean:
        assert np.array_equal(r1, r2) and np.array_equal(f1, f2)
    else:
        assert same_f32(r1, r2).all()
        assert all(fit_equal(a, b) for a, b in zip(f1, f2))
    assert np.array_equal(i1["child_nodes"], i2["child_nodes"])
    # points never recorded: only co-evaluation can take them
    recorded = set(zip(kids.parent.tolist(), kids.point.tolist()))
    j = next(i for i in range(len(extra.parent)) if (int(extra.parent[i]), int(extra.point[i])) not in recorded)
    dj = gen.pack([extra.donors.tree(j)])
    with pytest.raises(g.GPError) as e:
        ctx.evaluate_incremental(ph, ch, gt, T, extra.parent[j:j + 1], extra.point[j:j + 1], dj.ops, dj.offsets)
    assert e.value.code == g.GP_ENOTFOUND
    r3, f3, i3 = ctx.evaluate_incremental(ph, ch, gt, T, extra.parent, extra.point, extra.donors.ops,
                                          extra.donors.offsets, coeval=True)
    for i in range(len(extra.parent)):
        P = parents.tree(int(extra.parent[i]))
        c = int(extra.point[i])
        D = extra.donors.tree(i)
        if boolean:
            w_root, w_lvl, _, w_fit = oracle.incremental_bool(P, c, D, cases.inputs, cases.target, 64)
            assert np.array_equal(r3[i], w_root) and f3[i] == w_fit
        else:
            with np.errstate(all="ignore"):
                w_root, w_lvl, _, w_fit = oracle.incremental_f32(P, c, D, cases.x, cases.y)
            assert same_f32(r3[i], w_root).all() and fit_equal(f3[i], w_fit)
        assert i3["stop_level"][i] == w_lvl, (i, i3["stop_level"][i], w_lvl)
        walked = w_lvl if w_lvl >= 0 else len(g.inspect_path(P, c)[0])
        lo, hi = _coeval_bounds(P, c, D, walked)
        assert lo <= i3["interpreted_nodes"][i] <= hi, (i, lo, i3["interpreted_nodes"][i], hi)
    ctx.free(ph)
    ctx.free(ch)


def test_coeval_errors(ctx):
    cases = gen.float_cases(41, 64)
    pop = gen.sized_population(42, 3, 11, 101)
    d = gen.pack([np.array([0], np.uint8)])
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets)
    with pytest.raises(g.GPError) as e:                       # mother not evaluated yet
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [1], d.ops, d.offsets, coeval=True)
    assert e.value.code == g.GP_ENOTFOUND
    ctx.evaluate_full(ph, ch, g.GP_F32, 3, 64)
    with pytest.raises(g.GPError) as e:                       # point out of range
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [10 ** 6], d.ops, d.offsets, coeval=True)
    assert e.value.code == g.GP_EINVAL
    bad = gen.pack([np.array([gen.F_ADD, 0], np.uint8)])
    with pytest.raises(g.GPError) as e:                       # malformed donor
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [1], bad.ops, bad.offsets, coeval=True)
    assert e.value.code == g.GP_EINVAL
    post = ctx.load_population(g.GP_F32, np.array([0, 0, gen.F_ADD], np.uint8), np.array([0, 3], np.int64),
                               layout=g.GP_POSTFIX)
    ctx.evaluate_full(post, ch, g.GP_F32, 1, 64)
    with pytest.raises(g.GPError) as e:                       # reverse Polish population
        ctx.evaluate_incremental(post, ch, g.GP_F32, 64, [0], [0], d.ops, d.offsets, coeval=True)
    assert e.value.code == g.GP_EINVAL
    ctx.free(post)
    ctx.free(ph)
    ctx.free(ch)


def test_incremental_errors(ctx):
    parents = gen.sized_population(51, 3, 11, 101)
    cases = gen.float_cases(52, 64)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, parents.ops, parents.offsets,
                             record_points=np.array([0, 1], np.int64),
                             record_offsets=np.array([0, 2, 2, 2], np.int64))
    d = np.array([0], np.uint8)
    with pytest.raises(g.GPError) as e:        # not evaluated yet
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [1], d, [0, 1])
    assert e.value.code == g.GP_ENOTFOUND
    ctx.evaluate_full(ph, ch, g.GP_F32, 3, 64)
    with pytest.raises(g.GPError) as e:        # point not recorded
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [1], [0], d, [0, 1])
    assert e.value.code == g.GP_ENOTFOUND
    with pytest.raises(g.GPError) as e:        # malformed donor
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [1], np.array([0x80, 0], np.uint8), [0, 2])
    assert e.value.code == g.GP_EINVAL
    with pytest.raises(g.GPError) as e:        # point out of range
        ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [10**6], d, [0, 1])
    assert e.value.code == g.GP_EINVAL
    r, f, info = ctx.evaluate_incremental(ph, ch, g.GP_F32, 64, [0], [0], d, [0, 1])   # replace the root
    assert np.all(r[0] == cases.x[0])
    ctx.free(ph)
    ctx.free(ch)


def test_malformed_population_rejected(ctx):
    with pytest.raises(g.GPError) as e:
        ctx.load_population(g.GP_F32, np.array([0x80, 0, 0x80, 0], np.uint8), np.array([0, 3, 4], np.int64))
    assert e.value.code == g.GP_EINVAL
    with pytest.raises(g.GPError) as e:
        ctx.load_population(g.GP_F32, np.array([0x80, 0, 1], np.uint8), np.array([0, 3], np.int64))
    assert e.value.code == g.GP_EINVAL


def test_budget_enforced():
    c = g.Context(0, budget_bytes=256 << 10)
    pop = gen.sized_population(3, 8, 10001, 20001)
    cases = gen.float_cases(1, 1024)
    ch = c.set_cases(g.GP_F32, cases.x, cases.y)
    with pytest.raises(g.GPError) as e:
        ph = c.load_population(g.GP_F32, pop.ops, pop.offsets)
        c.evaluate_full(ph, ch, g.GP_F32, 4, 1024)
    assert e.value.code == g.GP_EBUDGET
    c.close()
