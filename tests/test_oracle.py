"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: hand-worked
values, numpy float32 arithmetic, brute force over all Boolean input
combinations, a scalar recursive evaluator written separately, closed forms and
the invariants Section 6.2 states (incremental = full evaluation of the child;
the stop level is the first ancestor where child and mother agree).
"""
import math

import numpy as np
import pytest

import gen
import oracle
from tests.scalar_ref import eval_bool_case, eval_f32_case, same_f32

A, S, M, D = gen.F_ADD, gen.F_SUB, gen.F_MUL, gen.F_PDIV
X = 0


def t(*ops):
    return np.array(ops, dtype=np.uint8)


SPECIAL = np.array([0.0, -0.0, 1.0, -1.0, 0.5, 1e-7, -1e-7, 1e-6, 2.5e-6, 3.0, 1e-20, -1e-30,
                    1e30, 3.4e38, np.inf, -np.inf, np.nan, 1.17549435e-38, 1e-45], dtype=np.float32)


# --------------------------------------------------------------- format (C1)
def test_validate_corpus():
    assert oracle.validate(t(X))
    assert oracle.validate(t(A, X, X))
    assert oracle.validate(t(A, S, X, X, X))
    assert not oracle.validate(t())
    assert not oracle.validate(t(A, X))             # truncated
    assert not oracle.validate(t(X, X))             # trailing node
    assert not oracle.validate(t(A, X, X, X))       # trailing node after a full tree
    assert not oracle.validate(t(X, A, X))          # final count is right, but the tree ends at node 0
    assert not oracle.validate(t(0x84, X, X))       # unknown function
    assert not oracle.validate(t(A, X, 1))          # terminal index >= n_inputs
    assert oracle.validate(t(A, X, 1), n_inputs=2)


def test_subtree_end():
    tree = t(A, S, X, X, M, X, X)
    assert oracle.subtree_end(tree, 0) == 7
    assert oracle.subtree_end(tree, 1) == 4
    assert oracle.subtree_end(tree, 4) == 7
    assert oracle.subtree_end(tree, 6) == 7


def test_all_ends_and_parents_hand_worked():
    tree = t(A, S, X, X, M, X, X)
    assert oracle.all_ends(tree).tolist() == [7, 4, 3, 4, 7, 6, 7]
    assert oracle.parents(tree).tolist() == [-1, 0, 1, 1, 0, 4, 4]
    assert oracle.all_ends(t(X)).tolist() == [1]
    assert oracle.parents(t(X)).tolist() == [-1]


def test_all_ends_and_parents_combs():
    """Closed forms: a left comb F..F x..x of d functions has node k (< d) as the
    left child of k - 1 and the right child of function k - 1 at 2d - k; a right
    comb (F x)^d x has node 2k + 1 and 2k + 2 as the children of function 2k."""
    for d in [1, 2, 5, 40]:
        left = t(*([A] * d + [X] * (d + 1)))
        ends, par = oracle.all_ends(left), oracle.parents(left)
        for k in range(d):
            assert ends[k] == 2 * d + 1 - k
            assert par[k] == k - 1
            assert par[2 * d - k] == k
        assert par[d] == d - 1
        right = t(*([A, X] * d + [X]))
        ends, par = oracle.all_ends(right), oracle.parents(right)
        for k in range(d):
            assert ends[2 * k] == 2 * d + 1
            assert par[2 * k + 1] == 2 * k and par[2 * k + 2] == 2 * k


@pytest.mark.parametrize("seed", range(6))
def test_all_ends_and_parents_brute_force(seed):
    """Against the forward-scanning subtree end, node by node, and the parent as
    the nearest earlier node whose subtree holds the node."""
    rng = np.random.default_rng(900 + seed)
    for n in [1, 3, 9, 31, 101, 255]:
        tree = gen.sized_tree(rng, n, n_terms=3)
        ends, par = oracle.all_ends(tree), oracle.parents(tree)
        for i in range(n):
            assert ends[i] == oracle.subtree_end(tree, i)
        for j in range(n):
            enclosing = [p for p in range(j) if oracle.subtree_end(tree, p) > j]
            assert par[j] == (max(enclosing) if enclosing else -1)


def _full_tree(depth):
    """Complete binary tree of the given depth (prefix form)."""
    return [A] + _full_tree(depth - 1) + _full_tree(depth - 1) if depth else [X]


def test_strahler_closed_forms():
    for d in range(0, 9):
        s = oracle.strahler(t(*_full_tree(d)))
        assert s[0] == d + 1                    # a complete tree of depth d
        assert s.max() == d + 1 and s.min() == 1
    for d in [1, 3, 50]:
        left = t(*([A] * d + [X] * (d + 1)))    # each function has a terminal child
        assert oracle.strahler(left).tolist() == [2] * d + [1] * (d + 1)
        right = t(*([A, X] * d + [X]))
        assert oracle.strahler(right).tolist() == [2, 1] * d + [1]
    # a function whose children have different numbers takes the larger
    assert oracle.strahler(t(A, *_full_tree(2), X)).tolist()[0] == 3
    assert oracle.strahler(t(A, *_full_tree(2), *_full_tree(2)))[0] == 4


@pytest.mark.parametrize("seed", range(4))
def test_strahler_brute_force(seed):
    """Against the characterisation: a node's number is at least k + 1 iff its
    subtree holds a function whose two children both have at least k, checked
    level by level from the subtree ranges."""
    rng = np.random.default_rng(950 + seed)
    for n in [1, 3, 7, 31, 127, 511]:
        tree = gen.sized_tree(rng, n, n_terms=2)
        got = oracle.strahler(tree)
        end = [oracle.subtree_end(tree, i) for i in range(n)]
        s = np.ones(n, np.int64)
        k = 1
        while True:
            flag = [bool(tree[u] & 0x80) and s[u + 1] >= k and s[end[u + 1]] >= k for u in range(n)]
            up = [any(flag[v:end[v]]) for v in range(n)]
            if not any(up):
                break
            for v in range(n):
                if up[v]:
                    s[v] = k + 1
            k += 1
        assert np.array_equal(got, s)


# -------------------------------------------------------- float semantics (C2)
def test_hand_worked_float():
    x = SPECIAL[None, :]
    finite = np.isfinite(SPECIAL)
    with np.errstate(all="ignore"):
        sub = oracle.eval_f32(t(S, X, X), x)
        assert np.all(sub[finite].view(np.uint32) == 0)                  # x - x = +0.0
        assert np.all(np.isnan(sub[~finite]))
        prot = oracle.eval_f32(t(D, X, S, X, X), x)                          # x / (x - x)
        assert np.all(prot[finite] == 1.0)                                  # protected: divisor +0
        same = oracle.eval_f32(t(D, X, X), x)
        assert np.all(same[finite] == 1.0)                                  # x/x = 1 or protected
        dbl = oracle.eval_f32(t(A, X, X), x)
        assert np.all(same_f32(dbl, SPECIAL * np.float32(2)))


def test_operand_order():
    x = np.array([[3.0, 8.0], [1.0, 2.0]], np.float32)      # x0, x1 on two cases
    assert list(oracle.eval_f32(t(S, 0, 1), x)) == [2.0, 6.0]
    assert list(oracle.eval_f32(t(D, 0, 1), x)) == [3.0, 4.0]
    assert list(oracle.eval_f32(t(S, 1, 0), x)) == [-2.0, -6.0]


def test_protected_threshold_is_float32():
    tiny = np.float32(1e-6)
    below = np.nextafter(tiny, np.float32(0))
    x = np.array([[2.0, 2.0, 2.0, 2.0], [tiny, below, -below, -tiny]], np.float32)
    out = oracle.eval_f32(t(D, 0, 1), x)
    assert out[0] == np.float32(2.0) / tiny           # 1e-6f itself is not protected
    assert out[1] == 1.0 and out[2] == 1.0
    assert out[3] == np.float32(2.0) / -tiny


def test_nan_and_inf_divisors():
    x = np.array([[5.0, 5.0, np.nan, np.nan], [np.nan, np.inf, 0.0, 1.0]], np.float32)
    with np.errstate(all="ignore"):
        out = oracle.eval_f32(t(D, 0, 1), x)
    assert np.isnan(out[0])                 # |NaN| < 1e-6 is false -> 5/NaN
    assert out[1] == 0.0
    assert out[2] == 1.0                    # protected even for a NaN dividend
    assert np.isnan(out[3])


def test_cube_closed_form():
    rng = np.random.default_rng(7)
    xs = rng.uniform(-1, 1, 4096).astype(np.float32)
    got = oracle.eval_f32(t(M, M, X, X, X), xs[None, :])
    want = (xs * xs) * xs                                           # numpy float32
    assert np.all(got.view(np.uint32) == want.view(np.uint32))
    exact = xs.astype(np.float64) ** 3
    ulp = np.spacing(np.abs(got)).astype(np.float64)
    ok = np.abs(got.astype(np.float64) - exact) <= 2 * ulp
    assert ok[np.abs(exact) > 1e-30].all()


def test_denormals_kept():
    x = np.array([[1e-20, -3e-22, 1e-23]], np.float32)
    got = oracle.eval_f32(t(M, X, X), x)
    want = x[0] * x[0]
    assert np.all(got.view(np.uint32) == want.view(np.uint32))
    assert got[0] != 0.0 and got[0] < np.finfo(np.float32).tiny     # a denormal survives


def test_random_trees_vs_scalar_recursion():
    rng = np.random.default_rng(11)
    x = np.concatenate([SPECIAL, rng.uniform(-2, 2, 13).astype(np.float32)])
    xin = np.stack([x, x[::-1].copy()])
    for i in range(60):
        n = int(gen.log_uniform_odd(rng, 1, 151))
        tree = gen.sized_tree(rng, n, n_terms=2)
        with np.errstate(all="ignore"):
            got = oracle.eval_f32(tree, xin)
            want = np.array([eval_f32_case(tree, xin[:, k]) for k in range(xin.shape[1])], np.float32)
        assert same_f32(got, want).all(), i


def test_sextic_target_tree_scores_zero():
    cases = gen.float_cases(1, 48)
    out = oracle.eval_f32(gen.sextic_tree(), cases.x)
    assert np.all(out.view(np.uint32) == cases.y.view(np.uint32))
    assert oracle.fitness_f32(out, cases.y) == 0.0


# ------------------------------------------------------------- fitness (C5)
def test_fitness_halving_order_hand_worked():
    # three cases, P = 64: the halving tree adds slot 2 into slot 0 first
    # (h = 2), then slot 1 (h = 1): (2^-23 + 2^-23) + 2^30 = 2^30 + 2^-22
    # exactly, whereas a left-to-right sum would round 2^30 + 2^-23 to 2^30.
    y = np.zeros(3, np.float32)
    out = np.array([2.0 ** -23, 2.0 ** 30, 2.0 ** -23], np.float32)
    assert oracle.fitness_f32(out, y) == 2.0 ** 30 + 2.0 ** -22
    assert (2.0 ** -23 + 2.0 ** 30) + 2.0 ** -23 == 2.0 ** 30


def test_fitness_against_fsum():
    rng = np.random.default_rng(3)
    for T in [1, 5, 48, 63, 64, 65, 1000, 1024, 4096]:
        out = rng.normal(size=T).astype(np.float32) * np.float32(1e3)
        y = rng.normal(size=T).astype(np.float32)
        e = [float(abs(np.float32(out[i] - y[i]))) for i in range(T)]
        exact = math.fsum(e)
        got = oracle.fitness_f32(out, y)
        # a depth-log2(P) tree of non-negative terms: relative error <= log2(P) * 2^-53
        bound = max(6, math.ceil(math.log2(max(T, 64)))) * 2.0 ** -53 * exact
        assert abs(got - exact) <= bound + 1e-300
    ones = np.ones(100, np.float32)
    assert oracle.fitness_f32(ones, np.zeros(100, np.float32)) == 100.0
    assert math.isnan(oracle.fitness_f32(np.array([np.nan, 1], np.float32), np.zeros(2, np.float32)))


# ------------------------------------------------------------ Boolean (C3)
def test_parity_target_constant():
    c = gen.bool_cases(6)
    assert c.inputs.shape == (6, 1)
    assert int(c.target[0]) == 0x9669699669969669
    assert [int(v) for v in c.inputs[:, 0]] == [0xAAAAAAAAAAAAAAAA, 0xCCCCCCCCCCCCCCCC,
                                                0xF0F0F0F0F0F0F0F0, 0xFF00FF00FF00FF00,
                                                0xFFFF0000FFFF0000, 0xFFFFFFFF00000000]


def _xor(a, b):
    # XOR(a, b) = NOR(AND(a, b), NOR(a, b))
    return [gen.B_NOR, gen.B_AND] + a + b + [gen.B_NOR] + a + b


def test_boolean_closed_forms():
    c = gen.bool_cases(6)
    assert oracle.fitness_bool(oracle.eval_bool(t(0), c.inputs), c.target, 64) == 32
    const_true = t(gen.B_OR, 0, gen.B_NAND, 0, 0)
    out = oracle.eval_bool(const_true, c.inputs)
    assert int(out[0]) == 0xFFFFFFFFFFFFFFFF
    assert oracle.fitness_bool(out, c.target, 64) == 32
    x = [0]
    for j in range(1, 6):
        x = _xor(x, [j])
    xor6 = np.array(x, np.uint8)
    out = oracle.eval_bool(xor6, c.inputs)
    assert int(out[0]) == (~int(c.target[0])) & 0xFFFFFFFFFFFFFFFF      # odd parity
    even6 = np.array([gen.B_NOR] + x + x, np.uint8)                     # NOT(x) = NOR(x, x)
    assert oracle.fitness_bool(oracle.eval_bool(even6, c.inputs), c.target, 64) == 64


def test_boolean_brute_force_all_combinations():
    rng = np.random.default_rng(5)
    for k in [3, 6, 8]:
        c = gen.bool_cases(k)
        for i in range(15):
            n = int(gen.log_uniform_odd(rng, 1, 99))
            tree = gen.sized_tree(rng, n, n_terms=k)
            out = oracle.eval_bool(tree, c.inputs)
            for comb in range(c.T):
                bits = [(comb >> j) & 1 for j in range(k)]
                want = eval_bool_case(tree, bits)
                got = (int(out[comb // 64]) >> (comb % 64)) & 1
                assert got == int(want)
                if comb < 8:
                    assert oracle.eval_bool_bit(tree, bits, k) == int(want)


def test_boolean_fitness_masks_tail():
    c = gen.bool_cases(3)                    # T = 8, one word, 56 padding bits
    ones = np.array([0xFFFFFFFFFFFFFFFF], np.uint64)
    zeros = np.array([0], np.uint64)
    assert oracle.fitness_bool(ones, c.target, 8) + oracle.fitness_bool(zeros, c.target, 8) == 8


# -------------------------------------------------------------- splice (C6)
def test_splice_identities():
    rng = np.random.default_rng(2)
    for i in range(40):
        p = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 301)))
        d = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 51)))
        c = int(rng.integers(len(p)))
        e = oracle.subtree_end(p, c)
        child = oracle.splice(p, c, d)
        assert len(child) == len(p) - (e - c) + len(d)
        assert oracle.validate(child)
        assert np.array_equal(child, gen.splice(p, c, d))
        assert np.array_equal(oracle.splice(p, c, p[c:e]), p)
        assert np.array_equal(oracle.splice(p, 0, d), d)


# --------------------------------------------------------- incremental (C7)
def _path_to(tree, c):
    ends = gen.subtree_ends(tree)
    path, v = [0], 0
    while v != c:
        l = v + 1
        v = l if c < ends[l] else ends[l]
        path.append(v)
    return path


def _brute_force_stop(parent, child, c, x):
    pv = oracle.eval_f32_nodes(parent, x)
    cv = oracle.eval_f32_nodes(child, x)
    path = _path_to(parent, c)[::-1]         # c, a_1, ..., root (same indices in both trees)
    for k, a in enumerate(path):
        if same_f32(pv[a], cv[a]).all():
            return k
    return -1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_incremental_equals_full_and_brute_force_stop(seed):
    rng = np.random.default_rng(100 + seed)
    cases = gen.float_cases(seed, 37)
    levels = []
    for i in range(40):
        p = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 3, 201)))
        c = int(rng.integers(len(p)))
        if i % 3 == 0:
            e = oracle.subtree_end(p, c)
            d = gen.neutral_donor(rng, p[c:e].copy(), int(rng.integers(5, 40)))
        else:
            d = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 41)))
        with np.errstate(all="ignore"):
            root, lvl, interp, fit = oracle.incremental_f32(p, c, d, cases.x, cases.y)
            child = oracle.splice(p, c, d)
            full = oracle.eval_f32(child, cases.x)
            assert same_f32(root, full).all()
            ffit = oracle.fitness_f32(full, cases.y)
            assert (fit == ffit) or (math.isnan(fit) and math.isnan(ffit))
            assert lvl == _brute_force_stop(p, child, c, cases.x)
        depth = len(_path_to(p, c)) - 1
        assert interp == len(d) + (depth if lvl < 0 else lvl)
        if i % 3 == 0:
            assert lvl == 0
        levels.append(lvl)
    assert any(l < 0 for l in levels) and any(l > 0 for l in levels)


def test_incremental_stops_at_protected_root():
    # root = (/ S (- x x)): the divisor is +0, so the root is 1.0 whatever S is
    rng = np.random.default_rng(9)
    cases = gen.float_cases(4, 64)
    for i in range(20):
        s = gen.sized_tree(rng, 31)
        p = np.concatenate([[D], s, [S, X, X]]).astype(np.uint8)
        c = 1 + int(rng.integers(len(s)))
        d = gen.sized_tree(rng, 7)
        root, lvl, interp, fit = oracle.incremental_f32(p, c, d, cases.x, cases.y)
        assert lvl >= 0
        assert np.all(root == 1.0)


def test_incremental_boolean():
    rng = np.random.default_rng(12)
    c6 = gen.bool_cases(6)
    seen_stop = False
    for i in range(60):
        p = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 3, 201)), n_terms=6)
        c = int(rng.integers(len(p)))
        d = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 21)), n_terms=6)
        root, lvl, interp, fit = oracle.incremental_bool(p, c, d, c6.inputs, c6.target, 64)
        child = oracle.splice(p, c, d)
        full = oracle.eval_bool(child, c6.inputs)
        assert np.array_equal(root, full)
        assert fit == oracle.fitness_bool(full, c6.target, 64)
        seen_stop |= lvl >= 0
        # brute force over bits: first ancestor whose scalar truth tables agree
        path = _path_to(p, c)[::-1]
        ends_p, ends_c = gen.subtree_ends(p), gen.subtree_ends(child)
        want = -1
        for k, a in enumerate(path):
            pv = oracle.eval_bool(p[a:ends_p[a]], c6.inputs)
            cv = oracle.eval_bool(child[a:ends_c[a]], c6.inputs)
            if np.array_equal(pv, cv):
                want = k
                break
        assert lvl == want
    assert seen_stop


# ----------------------------------------------------------- generators (C8)
def test_generators_deterministic_and_valid():
    a = gen.ramped_half_and_half(1)
    b = gen.ramped_half_and_half(1)
    assert np.array_equal(a.ops, b.ops) and np.array_equal(a.offsets, b.offsets)
    assert a.n_trees == 100 and a.sizes().max() <= 200
    for i in range(a.n_trees):
        assert oracle.validate(a.tree(i))
        assert a.tree(i)[0] & 0x80                       # root is a function
    p = gen.sized_population(3, 20, 11, 2001)
    assert np.all(p.sizes() % 2 == 1)
    for i in range(p.n_trees):
        assert oracle.validate(p.tree(i))
    q = gen.sized_population(3, 20, 11, 2001)
    assert np.array_equal(p.ops, q.ops)


def test_children_generator():
    parents = gen.sized_population(4, 6, 101, 2001)
    ch = gen.crossover_children(5, parents, 12, donor_hi=300)
    x = gen.float_cases(4, 32)
    assert ch.neutral.sum() == 6
    for i in range(12):
        p = parents.tree(int(ch.parent[i]))
        assert oracle.validate(ch.donors.tree(i))
        if ch.neutral[i]:
            _, lvl, _, _ = oracle.incremental_f32(p, int(ch.point[i]), ch.donors.tree(i), x.x, x.y)
            assert lvl == 0


# --------------------------------------------------- selection (Section 6.3)
def test_philox_known_answers():
    # Known-answer vectors of Philox-4x32-10 published with the generator
    # (Random123): counter, key -> output.
    assert oracle.philox((0, 0, 0, 0), (0, 0)) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert oracle.philox((0xffffffff,) * 4, (0xffffffff,) * 2) == [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert oracle.philox((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0)) == \
        [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_uniform_mapping_closed_forms():
    for n in [1, 2, 3, 7, 1000, 2 ** 31 - 1, 2 ** 32 - 1]:
        assert oracle.uniform(0, n) == 0
        assert oracle.uniform(2 ** 32 - 1, n) == n - 1          # (2^32 - 1) n / 2^32 = n - n / 2^32
        assert oracle.uniform(2 ** 31, n) == n // 2
    # every residue of n = 3 gets floor or ceil of 2^32 / 3 words
    edges = [0] + [-(-(2 ** 32) * r // 3) for r in (1, 2)]          # first u mapping to 1, to 2
    assert [oracle.uniform(e, 3) for e in edges] == [0, 1, 2]
    assert [oracle.uniform(e - 1, 3) for e in edges[1:]] == [0, 1]


def test_draws_follow_the_counter_layout():
    seed = 0x0123456789ABCDEF
    words = oracle.philox((5, 9, 2, 1), (seed & 0xffffffff, seed >> 32))
    assert [oracle.draw(seed, 5, 9, 2, j) for j in range(4, 8)] == words


def test_tournament_properties():
    rng = np.random.default_rng(4)
    fit = rng.normal(size=50)
    fit[[3, 7]] = np.nan
    seed = 77
    for i in range(200):
        w1 = oracle.tournament(fit, 1, seed, i, 0, 0)
        assert w1 == oracle.uniform(oracle.draw(seed, i, 0, 0, 0), 50)
        for k in (2, 5):
            w = oracle.tournament(fit, k, seed, i, 0, 0)
            drawn = [oracle.uniform(oracle.draw(seed, i, 0, 0, j), 50) for j in range(k)]
            assert w in drawn
            ok = [c for c in drawn if not np.isnan(fit[c])]
            if ok:
                assert not np.isnan(fit[w]) and fit[w] == min(fit[c] for c in ok)
                assert w == next(c for c in drawn if fit[c] == fit[w])       # ties keep the earlier draw
            else:
                assert w == drawn[0]
    same = np.full(50, 0.25)
    for i in range(50):                                           # all tied: the first draw wins
        assert oracle.tournament(same, 5, seed, i, 2, 0) == oracle.uniform(oracle.draw(seed, i, 2, 0, 0), 50)
        assert oracle.tournament(np.full(50, 7, np.int64), 5, seed, i, 2, 1) == \
            oracle.uniform(oracle.draw(seed, i, 2, 1, 0), 50)
    hits = rng.integers(0, 64, 50).astype(np.int64)
    for i in range(100):
        w = oracle.tournament(hits, 4, seed, i, 1, 1)
        drawn = [oracle.uniform(oracle.draw(seed, i, 1, 1, j), 50) for j in range(4)]
        assert hits[w] == max(hits[c] for c in drawn)


def test_fitness_first_savings_closed_forms():
    """Section 6.3: children drawn as nobody's parent need not be built.
    Converged population, two parents per child: the chance a child is never
    drawn in 2N tournaments is (1 - 1/N)^(2N) -> e^-2 = 13.5 % (the paper's
    14 %).  Diverse fitness, one tournament of size k per child: a child whose
    fitness beats a fraction 1 - x of the others wins k (1 - x)^(k - 1)
    tournaments on average, so the share never drawn is the integral of
    exp(-k (1 - x)^(k - 1)) over [0, 1]: 0.671 for k = 7."""
    N = 4000
    same = np.zeros(N, np.float64)
    drawn = np.zeros(N, bool)
    for j in range(N):
        drawn[oracle.tournament(same, 7, 11, j, 1, 0)] = True
        drawn[oracle.tournament(same, 7, 11, j, 1, 1)] = True
    assert abs((~drawn).mean() - math.exp(-2)) < 0.03
    distinct = np.random.default_rng(5).permutation(N).astype(np.float64)
    drawn[:] = False
    for j in range(N):
        drawn[oracle.tournament(distinct, 7, 12, j, 1, 0)] = True
    y = np.linspace(0, 1, 200001)
    want = float(np.mean(np.exp(-7 * y ** 6)))
    assert abs(want - 0.6707) < 1e-3
    assert abs((~drawn).mean() - want) < 0.03


def test_evolve_invariants_small():
    rng = np.random.default_rng(6)
    trees = [gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 5, 301))) for _ in range(24)]
    cases = gen.float_cases(7, 48)
    recs, final = oracle.evolve(trees, False, cases, 3, 3, 99)
    assert len(recs) == 3 and all(t is not None for t in final)
    for g, r in enumerate(recs):
        if g < 2:
            nxt = recs[g + 1]
            assert r["built"][nxt["mother"]].all() and r["built"][nxt["father"]].all()
            assert 0 < r["built"].sum() < 24
    with np.errstate(all="ignore"):
        for t, f in zip(final, recs[-1]["fitness"]):
            assert oracle.validate(t)
            out = oracle.eval_f32(t, cases.x)
            got = oracle.fitness_f32(out, cases.y)
            assert got == f or (math.isnan(got) and math.isnan(f))        # incremental = full evaluation


def test_population_loop_equals_per_tree_calls():
    """orc_population_* is the plain loop over trees: each listed tree's
    fitness equals eval + fitness of that tree alone (in any order, repeats
    allowed)."""
    pop = gen.sized_population(91, 12, 1, 2001)
    cases = gen.float_cases(92, 100)
    which = np.array([3, 0, 11, 3, 7], np.int64)
    got = oracle.population_fitness(pop, which, cases)
    for k, t in enumerate(which):
        with np.errstate(all="ignore"):
            w = oracle.fitness_f32(oracle.eval_f32(pop.tree(int(t)), cases.x), cases.y)
        assert got[k] == w or (np.isnan(got[k]) and np.isnan(w))
    bc = gen.bool_cases(7)
    bpop = gen.sized_population(93, 9, 1, 901, n_terms=7, vtype=gen.VT_BOOL)
    which = np.arange(9)[::-1].copy()
    got = oracle.population_fitness(bpop, which, bc)
    for k, t in enumerate(which):
        assert got[k] == oracle.fitness_bool(oracle.eval_bool(bpop.tree(int(t)), bc.inputs), bc.target, bc.T)
