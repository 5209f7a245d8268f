"""The block-split oracle helpers (tests/split_oracle.py) give exactly what
one unsplit oracle call gives: outputs, fitness, stop level and interpreted
count, for full evaluation and incremental children (float and Boolean),
including children that stop at the point, on the way up, and at the root."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import gen
import oracle
from tests import split_oracle as so
from tests.scalar_ref import same_f32


def test_split_float_matches_unsplit():
    parents = gen.sized_population(61, 6, 51, 801)
    kids = gen.crossover_children(62, parents, 24, donor_hi=60, neutral_frac=0.5, one_per_parent=False)
    cases = gen.float_cases(63, 1000)
    levels = set()
    with ThreadPoolExecutor(4) as pool:
        for b in (1, 3, 7, 64):
            for t in range(parents.n_trees):
                with np.errstate(all="ignore"):
                    out, fit = so.eval_f32(parents.tree(t), cases.x, cases.y, b, pool)
                    w = oracle.eval_f32(parents.tree(t), cases.x)
                assert same_f32(out, w).all()
                assert fit == oracle.fitness_f32(w, cases.y) or (np.isnan(fit))
            for i in range(len(kids.parent)):
                P, c, D = parents.tree(int(kids.parent[i])), int(kids.point[i]), kids.donors.tree(i)
                with np.errstate(all="ignore"):
                    got = so.incremental_f32(P, c, D, cases.x, cases.y, b, pool)
                    want = oracle.incremental_f32(P, c, D, cases.x, cases.y)
                assert same_f32(got[0], want[0]).all(), (b, i)
                assert got[1:3] == want[1:3], (b, i, got[1:3], want[1:3])
                assert got[3] == want[3] or (np.isnan(got[3]) and np.isnan(want[3]))
                levels.add(want[1])
    assert 0 in levels and any(l > 0 for l in levels)


def test_split_float_root_reached():
    # a child whose difference reaches the root: x -> (* x x) under a chain of ADDs
    P = np.array([gen.F_ADD, gen.F_ADD, 0, 0, 0], np.uint8)
    D = np.array([gen.F_MUL, 0, 0], np.uint8)
    cases = gen.float_cases(64, 500)
    with ThreadPoolExecutor(4) as pool:
        got = so.incremental_f32(P, 2, D, cases.x, cases.y, 5, pool)
    want = oracle.incremental_f32(P, 2, D, cases.x, cases.y)
    assert want[1] == -1 and got[1] == -1 and got[2] == want[2]
    assert same_f32(got[0], want[0]).all() and got[3] == want[3]


def test_split_boolean_matches_unsplit():
    k = 9
    cases = gen.bool_cases(k)
    parents = gen.sized_population(65, 5, 51, 801, n_terms=k, vtype=gen.VT_BOOL)
    kids = gen.crossover_children(66, parents, 20, donor_hi=60, neutral_frac=0.0, n_terms=k, one_per_parent=False)
    levels = set()
    with ThreadPoolExecutor(4) as pool:
        for b in (1, 3, 8):
            for t in range(parents.n_trees):
                out, hits = so.eval_bool(parents.tree(t), cases.inputs, cases.target, cases.T, b, pool)
                w = oracle.eval_bool(parents.tree(t), cases.inputs)
                assert np.array_equal(out, w) and hits == oracle.fitness_bool(w, cases.target, cases.T)
            for i in range(len(kids.parent)):
                P, c, D = parents.tree(int(kids.parent[i])), int(kids.point[i]), kids.donors.tree(i)
                got = so.incremental_bool(P, c, D, cases.inputs, cases.target, cases.T, b, pool)
                want = oracle.incremental_bool(P, c, D, cases.inputs, cases.target, cases.T)
                assert np.array_equal(got[0], want[0]) and got[1:] == want[1:], (b, i)
                levels.add(want[1])
    assert len(levels) > 1
