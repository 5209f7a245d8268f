"""The HIP path (through the C ABI) against the hand-worked fixtures in
tests/golden/: outputs bit-exact (both NaN counts as equal), fitness equal,
incremental stop levels and interpreted counts identical."""
import sys

import numpy as np
import pytest

from paper_2205_03251_amd import gpeval as g
from tests.golden_cases import f32, load, num, parse_tree, same_fitness, valid_mask, words
from tests.scalar_ref import same_f32

pytestmark = pytest.mark.gpu
G = load()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(0)
    yield c
    c.close()


def packed(trees):
    offs = np.zeros(len(trees) + 1, np.int64)
    offs[1:] = np.cumsum([len(t) for t in trees])
    return np.concatenate(trees).astype(np.uint8), offs


@pytest.mark.parametrize("case", G["float"], ids=lambda c: c["name"])
def test_float_golden_gpu(ctx, case):
    say("golden float:", case["name"])
    x = np.stack([f32(r) for r in case["x"]])
    y, want = f32(case["y"]), f32(case["out"])
    ops, offs = packed([parse_tree(case["tree"])])
    ch = ctx.set_cases(g.GP_F32, x, y)
    ph = ctx.load_population(g.GP_F32, ops, offs, n_inputs=x.shape[0])
    for per_tree in (False, True):
        roots, fit, _ = ctx.evaluate_full(ph, ch, g.GP_F32, 1, len(y), per_tree=per_tree, graph=not per_tree)
        assert same_f32(roots[0], want).all(), (roots[0], want)
        assert same_fitness(fit[0], num(case["fitness"])), (fit[0], case["fitness"])
    ctx.free(ph)
    ctx.free(ch)


@pytest.mark.parametrize("group", G["bool"], ids=lambda g_: g_["name"])
def test_bool_golden_gpu(ctx, group):
    say("golden bool:", group["name"])
    T = 1 << group["k"]
    x = np.stack([words(r) for r in group["x"]])
    target = words(group["target"])
    mask = valid_mask(x.shape[1], T)
    trees = [parse_tree(c["tree"], boolean=True) for c in group["cases"]]
    ops, offs = packed(trees)
    ch = ctx.set_cases(g.GP_BOOL, x, target, T)
    ph = ctx.load_population(g.GP_BOOL, ops, offs, n_inputs=x.shape[0])
    roots, fit, _ = ctx.evaluate_full(ph, ch, g.GP_BOOL, len(trees), T)
    for i, c in enumerate(group["cases"]):
        assert np.array_equal(np.asarray(roots[i]).view(np.uint64) & mask, words(c["out"])), c["tree"]
        assert fit[i] == c["hits"], (c["tree"], fit[i])
    ctx.free(ph)
    ctx.free(ch)


@pytest.mark.parametrize("case", G["incremental_float"], ids=lambda c: c["name"])
def test_incremental_float_golden_gpu(ctx, case):
    say("golden incremental float:", case["name"])
    x = np.stack([f32(r) for r in case["x"]])
    y, want = f32(case["y"]), f32(case["out"])
    ops, offs = packed([parse_tree(case["parent"])])
    dops, doffs = packed([parse_tree(case["donor"])])
    ch = ctx.set_cases(g.GP_F32, x, y)
    ph = ctx.load_population(g.GP_F32, ops, offs, n_inputs=x.shape[0],
                             record_points=np.array([case["point"]], np.int64),
                             record_offsets=np.array([0, 1], np.int64))
    ctx.evaluate_full(ph, ch, g.GP_F32, 1, len(y))
    roots, fit, info = ctx.evaluate_incremental(ph, ch, g.GP_F32, len(y), [0], [case["point"]], dops, doffs)
    assert same_f32(roots[0], want).all(), (roots[0], want)
    assert same_fitness(fit[0], num(case["fitness"])), (fit[0], case["fitness"])
    assert info["stop_level"][0] == case["stop_level"]
    assert info["interpreted_nodes"][0] == case["interpreted"]
    ctx.free(ph)
    ctx.free(ch)


@pytest.mark.parametrize("group", G["incremental_bool"], ids=lambda g_: g_["name"])
def test_incremental_bool_golden_gpu(ctx, group):
    T = 1 << group["k"]
    x = np.stack([words(r) for r in group["x"]])
    target = words(group["target"])
    mask = valid_mask(x.shape[1], T)
    ch = ctx.set_cases(g.GP_BOOL, x, target, T)
    for c in group["cases"]:
        say("golden incremental bool:", c["why"][:60])
        ops, offs = packed([parse_tree(c["parent"], True)])
        dops, doffs = packed([parse_tree(c["donor"], True)])
        ph = ctx.load_population(g.GP_BOOL, ops, offs, n_inputs=x.shape[0],
                                 record_points=np.array([c["point"]], np.int64),
                                 record_offsets=np.array([0, 1], np.int64))
        ctx.evaluate_full(ph, ch, g.GP_BOOL, 1, T)
        roots, fit, info = ctx.evaluate_incremental(ph, ch, g.GP_BOOL, T, [0], [c["point"]], dops, doffs)
        assert np.array_equal(np.asarray(roots[0]).view(np.uint64) & mask, words(c["out"])), c["why"]
        assert fit[0] == c["hits"], c["why"]
        assert info["stop_level"][0] == c["stop_level"], c["why"]
        assert info["interpreted_nodes"][0] == c["interpreted"], c["why"]
        ctx.free(ph)
    ctx.free(ch)
