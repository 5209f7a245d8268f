"""Generations with fitness first (gp_evolve) against the oracle's generational
loop (Sections 5 and 6.3): every parent, point, donor, child fitness, stop
level and build decision, and the final trees, bit for bit."""
import math
import sys

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def run_both(ctx, trees, boolean, cases, G, k, seed, n_inputs=1, chunk_nodes=0):
    pop = gen.pack(trees, vtype=gen.VT_BOOL if boolean else gen.VT_F32, n_inputs=n_inputs)
    gt = g.GP_BOOL if boolean else g.GP_F32
    if boolean:
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, cases.T)
    else:
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(gt, pop.ops, pop.offsets, n_inputs=n_inputs, chunk_nodes=chunk_nodes)
    ctx.evaluate_full(ph, ch, gt, pop.n_trees, cases.T)
    nh, stats, rec = ctx.evolve(ph, ch, G, k, seed)
    want, final = oracle.evolve(trees, boolean, cases, G, k, seed)
    return ph, ch, nh, stats, rec, want, final, gt


def check(rec, want, final, ctx, nh, boolean):
    G = len(want)
    for gi in range(G):
        w = want[gi]
        for key in ("mother", "father", "point", "donor_node", "nodes"):
            assert np.array_equal(rec[key][gi], w[key]), (gi, key)
        assert np.array_equal(rec["stop_level"][gi], w["stop_level"]), gi
        if boolean:
            assert np.array_equal(rec["fitness_i64"][gi], w["fitness"]), gi
        else:
            a, b = rec["fitness_f64"][gi], w["fitness"]
            assert np.all((a == b) | (np.isnan(a) & np.isnan(b))), gi
        if gi < G - 1:
            assert np.array_equal(rec["drawn"][gi] > 0, w["built"]), gi
    ops, offs = ctx.population_ops(nh)
    assert len(offs) - 1 == len(final)
    for i, t in enumerate(final):
        assert np.array_equal(ops[offs[i]:offs[i + 1]], t), i


@pytest.mark.parametrize("G,k,T,chunk_nodes", [(3, 3, 48, 0), (2, 7, 300, 16)])
def test_evolve_float_matches_oracle(ctx, G, k, T, chunk_nodes):
    rng = np.random.default_rng(101 + G)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 5, 2001))) for _ in range(40)]
    cases = gen.float_cases(102, T)
    ph, ch, nh, stats, rec, want, final, gt = run_both(ctx, trees, False, cases, G, k, 7, chunk_nodes=chunk_nodes)
    check(rec, want, final, ctx, nh, False)
    for gi in range(G - 1):
        assert stats[gi]["built"] == int(want[gi]["built"].sum()) < 40
    assert stats[-1]["built"] == 40
    # the last generation, fully evaluated by the library, scores as its co-evaluation did
    _, fit, _ = ctx.evaluate_full(nh, ch, gt, 40, T)
    a, b = fit, want[-1]["fitness"]
    assert np.all((a == b) | (np.isnan(a) & np.isnan(b)))
    say("evolve float: built", [s["built"] for s in stats], "of 40")
    for h in (nh, ph, ch):
        ctx.free(h)


def test_evolve_boolean_matches_oracle(ctx):
    rng = np.random.default_rng(103)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 5, 1001)), n_terms=6) for _ in range(30)]
    cases = gen.bool_cases(6)
    ph, ch, nh, stats, rec, want, final, gt = run_both(ctx, trees, True, cases, 3, 4, 11, n_inputs=6)
    check(rec, want, final, ctx, nh, True)
    for h in (nh, ph, ch):
        ctx.free(h)


def test_fitness_first_saving_converged(ctx):
    """Section 6.3: in a converged population every tournament returns its
    first draw, so a child is drawn by none of the next generation's 2N
    tournaments with probability (1 - 1/N)^(2N), close to e^-2 (13.5 %)."""
    N = 2000
    cases = gen.float_cases(104, 64)
    pop = gen.pack([np.array([0], np.uint8)] * N)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets)
    ctx.evaluate_full(ph, ch, g.GP_F32, N, 64)
    nh, stats, rec = ctx.evolve(ph, ch, 2, 7, 5)
    unbuilt = 1 - stats[0]["built"] / N
    say("converged: unbuilt fraction", unbuilt)
    assert abs(unbuilt - math.exp(-2)) < 0.03
    for h in (nh, ph, ch):
        ctx.free(h)


def test_evolve_errors(ctx):
    cases = gen.float_cases(105, 64)
    pop = gen.sized_population(106, 4, 11, 101)
    ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph = ctx.load_population(g.GP_F32, pop.ops, pop.offsets)
    with pytest.raises(g.GPError) as e:                        # not evaluated yet
        ctx.evolve(ph, ch, 1, 3, 1)
    assert e.value.code == g.GP_ENOTFOUND
    ctx.evaluate_full(ph, ch, g.GP_F32, 4, 64)
    with pytest.raises(g.GPError) as e:
        ctx.evolve(ph, ch, 0, 3, 1)
    assert e.value.code == g.GP_EINVAL
    with pytest.raises(g.GPError) as e:
        ctx.evolve(ph, ch, 1, 0, 1)
    assert e.value.code == g.GP_EINVAL
    post = ctx.load_population(g.GP_F32, np.array([0, 0, gen.F_ADD], np.uint8), np.array([0, 3], np.int64),
                               layout=g.GP_POSTFIX)
    ctx.evaluate_full(post, ch, g.GP_F32, 1, 64)
    with pytest.raises(g.GPError) as e:
        ctx.evolve(post, ch, 1, 3, 1)
    assert e.value.code == g.GP_EINVAL
    for h in (post, ph, ch):
        ctx.free(h)


@pytest.mark.parametrize("boolean,T,chunk_nodes", [(False, 1000, 16), (False, 48, 64), (True, 256, 16)])
def test_promoted_children_equal_full_evaluation(ctx, boolean, T, chunk_nodes):
    """Built children take the values of the chunks they reuse from their
    parents' last evaluation and run only the chunks compiled anew (Section 5,
    Figure 1): their outputs and fitness equal a full evaluation of the same
    population and the oracle's, and the next generation, whose co-evaluation
    reads those chunk values, still matches the oracle draw by draw."""
    rng = np.random.default_rng(107 + T)
    k = T.bit_length() - 1 if boolean else 1
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 101, 3001)), n_terms=k) for _ in range(36)]
    cases = gen.bool_cases(k) if boolean else gen.float_cases(108, T)
    ph, ch, nh, stats, rec, want, final, gt = run_both(ctx, trees, boolean, cases, 3, 3, 13, n_inputs=k,
                                                      chunk_nodes=chunk_nodes)
    check(rec, want, final, ctx, nh, boolean)
    for st in stats:
        assert 0 < st["chunks_evaluated"] < st["chunks"], st
    r1, f1 = ctx.population_results(nh, ch, gt, cases.T)
    r2, f2, _ = ctx.evaluate_full(nh, ch, gt, len(final), cases.T)
    if boolean:
        assert np.array_equal(r1, r2) and np.array_equal(f1, f2)
        wr, wf = oracle.eval_population_bool(gen.pack(final, gen.VT_BOOL, k), cases.inputs, cases.target, cases.T)
        assert np.array_equal(r1, wr) and np.array_equal(f1, wf)
    else:
        same = (r1.view(np.uint32) == r2.view(np.uint32)) | (np.isnan(r1) & np.isnan(r2))
        assert same.all() and np.all((f1 == f2) | (np.isnan(f1) & np.isnan(f2)))
        with np.errstate(all="ignore"):
            wr, wf = oracle.eval_population_f32(gen.pack(final), cases.x, cases.y)
        same = (r1.view(np.uint32) == wr.view(np.uint32)) | (np.isnan(r1) & np.isnan(wr))
        assert same.all() and np.all((f1 == wf) | (np.isnan(f1) & np.isnan(wf)))
    say("promoted: chunks evaluated", [(s["chunks_evaluated"], s["chunks"]) for s in stats])
    for h in (nh, ph, ch):
        ctx.free(h)
