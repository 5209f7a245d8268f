"""The oracle against the hand-worked fixtures in tests/golden/ (no GPU).

Every expected value in the fixture was worked out by hand from the cited
definitions; none was produced by the oracle or by the GPU library.
"""
import numpy as np
import pytest

import gen
import oracle
from tests.golden_cases import f32, load, num, parse_tree, same_fitness, valid_mask, words
from tests.scalar_ref import eval_bool_case, eval_f32_case, same_f32

G = load()


@pytest.mark.parametrize("case", G["float"], ids=lambda c: c["name"])
def test_float_golden(case):
    tree = parse_tree(case["tree"])
    x = np.stack([f32(r) for r in case["x"]])
    y, want = f32(case["y"]), f32(case["out"])
    with np.errstate(all="ignore"):
        got = oracle.eval_f32(tree, x)
        rec = np.array([eval_f32_case(tree, x[:, t]) for t in range(x.shape[1])], np.float32)
    assert same_f32(got, want).all(), (got, want)
    assert same_f32(rec, want).all(), (rec, want)           # the independent scalar recursion too
    assert same_fitness(oracle.fitness_f32(want, y), num(case["fitness"]))


def test_sextic_fixture_is_the_generator_tree():
    case = next(c for c in G["float"] if c["name"].startswith("sextic target"))
    assert np.array_equal(parse_tree(case["tree"]), gen.sextic_tree())
    x = f32(case["x"][0])
    assert np.all(gen.sextic(x).view(np.uint32) == f32(case["y"]).view(np.uint32))


@pytest.mark.parametrize("group", G["bool"], ids=lambda g: g["name"])
def test_bool_golden(group):
    k, T = group["k"], 1 << group["k"]
    x = np.stack([words(r) for r in group["x"]])
    target = words(group["target"])
    c = gen.bool_cases(k)
    mask = valid_mask(x.shape[1], T)
    assert np.array_equal(c.inputs & mask, x) and np.array_equal(c.target, target)
    for case in group["cases"]:
        tree = parse_tree(case["tree"], boolean=True)
        got = oracle.eval_bool(tree, x) & mask
        assert np.array_equal(got, words(case["out"])), case["tree"]
        assert oracle.fitness_bool(got, target, T) == case["hits"], case["tree"]
        for i in range(T):                                     # bit by bit through the scalar recursion
            bits = [(i >> j) & 1 for j in range(k)]
            assert eval_bool_case(tree, bits) == (int(got[i // 64]) >> (i % 64)) & 1


@pytest.mark.parametrize("case", G["incremental_float"], ids=lambda c: c["name"])
def test_incremental_float_golden(case):
    P, D = parse_tree(case["parent"]), parse_tree(case["donor"])
    x = np.stack([f32(r) for r in case["x"]])
    y, want = f32(case["y"]), f32(case["out"])
    with np.errstate(all="ignore"):
        out, lvl, interp, fit = oracle.incremental_f32(P, case["point"], D, x, y)
        full = oracle.eval_f32(oracle.splice(P, case["point"], D), x)
    assert same_f32(out, want).all(), (out, want)
    assert same_f32(full, want).all()
    assert lvl == case["stop_level"]
    assert interp == case["interpreted"]
    assert same_fitness(fit, num(case["fitness"]))


@pytest.mark.parametrize("group", G["incremental_bool"], ids=lambda g: g["name"])
def test_incremental_bool_golden(group):
    T = 1 << group["k"]
    x = np.stack([words(r) for r in group["x"]])
    target = words(group["target"])
    mask = valid_mask(x.shape[1], T)
    for case in group["cases"]:
        P, D = parse_tree(case["parent"], True), parse_tree(case["donor"], True)
        out, lvl, interp, hits = oracle.incremental_bool(P, case["point"], D, x, target, T)
        assert np.array_equal(out & mask, words(case["out"])), case["why"]
        assert (lvl, interp, hits) == (case["stop_level"], case["interpreted"], case["hits"]), case["why"]
