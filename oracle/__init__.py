"""CPU oracle for tree-GP fitness evaluation -- test infrastructure only.

Loads the plain C oracle (oracle.c) through ctypes.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use this package; the GPU library
never imports it, and it imports nothing from the GPU library.  See oracle.c
for the paper passages each routine follows and the readings it takes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (scalar SSE float, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
L = C.c_int64


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GPE_ORACLE_LIB")     # a planted-mistake build, in tests only
        if not path:
            build(force=False)
            path = _LIB
        h = C.CDLL(path)
        h.orc_validate.argtypes = [u8p, L, C.c_int]
        h.orc_subtree_end.argtypes = [u8p, L, L]
        h.orc_subtree_end.restype = L
        h.orc_all_ends.argtypes = [u8p, L, i64p]
        h.orc_parents.argtypes = [u8p, L, i64p]
        h.orc_strahler.argtypes = [u8p, L, i32p]
        h.orc_eval_f32.argtypes = [u8p, L, C.c_int, f32p, L, f32p]
        h.orc_eval_f32_nodes.argtypes = [u8p, L, C.c_int, f32p, L, f32p]
        h.orc_fitness_f32.argtypes = [f32p, f32p, L]
        h.orc_fitness_f32.restype = C.c_double
        h.orc_eval_bool.argtypes = [u8p, L, C.c_int, u64p, L, u64p]
        h.orc_eval_bool_bit.argtypes = [u8p, L, C.c_int, np.ctypeslib.ndpointer(np.int32)]
        h.orc_fitness_bool.argtypes = [u64p, u64p, L, L]
        h.orc_fitness_bool.restype = L
        h.orc_splice.argtypes = [u8p, L, L, u8p, L, u8p, L]
        h.orc_splice.restype = L
        h.orc_incremental_f32.argtypes = [u8p, L, L, u8p, L, C.c_int, f32p, f32p, L, f32p,
                                          i32p, i64p, f64p]
        h.orc_incremental_bool.argtypes = [u8p, L, L, u8p, L, C.c_int, u64p, u64p, L, L, u64p,
                                           i32p, i64p, i64p]
        h.orc_population_f32.argtypes = [u8p, i64p, i64p, L, C.c_int, f32p, f32p, L, f64p]
        h.orc_population_bool.argtypes = [u8p, i64p, i64p, L, C.c_int, u64p, u64p, L, L, i64p]
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        h.orc_philox.argtypes = [u32p, u32p, u32p]
        h.orc_uniform.argtypes = [C.c_uint32, C.c_uint64]
        h.orc_uniform.restype = C.c_uint64
        h.orc_draw.argtypes = [C.c_uint64, L, L, C.c_int, L]
        h.orc_draw.restype = C.c_uint32
        h.orc_tournament_f64.argtypes = [f64p, L, C.c_int, C.c_uint64, L, L, C.c_int]
        h.orc_tournament_f64.restype = L
        h.orc_tournament_i64.argtypes = [i64p, L, C.c_int, C.c_uint64, L, L, C.c_int]
        h.orc_tournament_i64.restype = L
        _lib = h
    return _lib


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def validate(tree, n_inputs: int = 1) -> bool:
    t = _u8(tree)
    return lib().orc_validate(t, len(t), n_inputs) == 0


def subtree_end(tree, i: int) -> int:
    t = _u8(tree)
    return int(lib().orc_subtree_end(t, len(t), i))


def all_ends(tree) -> np.ndarray:
    """Subtree end (exclusive) of every node of a valid prefix tree."""
    t = _u8(tree)
    out = np.zeros(len(t), np.int64)
    if lib().orc_all_ends(t, len(t), out) != 0:
        raise ValueError("empty tree")
    return out


def parents(tree) -> np.ndarray:
    """Parent of every node of a valid prefix tree, -1 at the root."""
    t = _u8(tree)
    out = np.zeros(len(t), np.int64)
    if lib().orc_parents(t, len(t), out) != 0:
        raise ValueError("empty tree")
    return out


def strahler(tree) -> np.ndarray:
    """Strahler number of every node of a valid prefix tree (1 at a terminal)."""
    t = _u8(tree)
    out = np.zeros(len(t), np.int32)
    if lib().orc_strahler(t, len(t), out) != 0:
        raise ValueError("empty tree")
    return out


def eval_f32(tree, x) -> np.ndarray:
    """x: [n_inputs][T] float32 -> out[T]."""
    t = _u8(tree)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float32)
    out = np.empty(x.shape[1], np.float32)
    rc = lib().orc_eval_f32(t, len(t), x.shape[0], x, x.shape[1], out)
    if rc != 0:
        raise ValueError(f"oracle eval_f32 failed ({rc})")
    return out


def eval_f32_nodes(tree, x) -> np.ndarray:
    t = _u8(tree)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float32)
    out = np.empty((len(t), x.shape[1]), np.float32)
    rc = lib().orc_eval_f32_nodes(t, len(t), x.shape[0], x, x.shape[1], out)
    if rc != 0:
        raise ValueError(f"oracle eval_f32_nodes failed ({rc})")
    return out


def fitness_f32(out, y) -> float:
    out = np.ascontiguousarray(out, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    return float(lib().orc_fitness_f32(out, y, len(y)))


def eval_bool(tree, inputs) -> np.ndarray:
    """inputs: [n_inputs][W] uint64 -> out[W]."""
    t = _u8(tree)
    inp = np.ascontiguousarray(inputs, dtype=np.uint64)
    out = np.empty(inp.shape[1], np.uint64)
    rc = lib().orc_eval_bool(t, len(t), inp.shape[0], inp, inp.shape[1], out)
    if rc != 0:
        raise ValueError(f"oracle eval_bool failed ({rc})")
    return out


def eval_bool_bit(tree, bits, n_inputs: int) -> int:
    t = _u8(tree)
    b = np.ascontiguousarray(bits, dtype=np.int32)
    return int(lib().orc_eval_bool_bit(t, len(t), n_inputs, b))


def fitness_bool(out, target, T: int) -> int:
    out = np.ascontiguousarray(out, np.uint64)
    target = np.ascontiguousarray(target, np.uint64)
    return int(lib().orc_fitness_bool(out, target, len(target), T))


def splice(parent, c: int, donor) -> np.ndarray:
    p, d = _u8(parent), _u8(donor)
    cap = len(p) + len(d)
    child = np.empty(cap, np.uint8)
    n = lib().orc_splice(p, len(p), c, d, len(d), child, cap)
    if n < 0:
        raise ValueError("oracle splice failed")
    return child[:n].copy()


def incremental_f32(parent, c: int, donor, x, y):
    """-> (root_out[T], stop_level, interpreted_nodes, fitness)."""
    p, d = _u8(parent), _u8(donor)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float32)
    y = np.ascontiguousarray(y, np.float32)
    T = x.shape[1]
    out = np.empty(T, np.float32)
    lvl = np.zeros(1, np.int32)
    interp = np.zeros(1, np.int64)
    fit = np.zeros(1, np.float64)
    rc = lib().orc_incremental_f32(p, len(p), c, d, len(d), x.shape[0], x, y, T, out, lvl, interp, fit)
    if rc != 0:
        raise ValueError(f"oracle incremental_f32 failed ({rc})")
    return out, int(lvl[0]), int(interp[0]), float(fit[0])


def incremental_bool(parent, c: int, donor, inputs, target, T: int):
    p, d = _u8(parent), _u8(donor)
    inp = np.ascontiguousarray(inputs, dtype=np.uint64)
    tg = np.ascontiguousarray(target, dtype=np.uint64)
    W = inp.shape[1]
    out = np.empty(W, np.uint64)
    lvl = np.zeros(1, np.int32)
    interp = np.zeros(1, np.int64)
    fit = np.zeros(1, np.int64)
    rc = lib().orc_incremental_bool(p, len(p), c, d, len(d), inp.shape[0], inp, tg, W, T, out, lvl,
                                    interp, fit)
    if rc != 0:
        raise ValueError(f"oracle incremental_bool failed ({rc})")
    return out, int(lvl[0]), int(interp[0]), int(fit[0])


# ----------------------------------------------------------- population helpers
def population_fitness(pop, which, cases, T=None):
    """Fitness of trees `which` of a population (float32 cases: .x/.y;
    Boolean: .inputs/.target/.T), evaluated one after another in C."""
    which = np.ascontiguousarray(which, np.int64)
    ops = _u8(pop.ops)
    offs = np.ascontiguousarray(pop.offsets, np.int64)
    if hasattr(cases, "x"):
        x = np.ascontiguousarray(np.atleast_2d(cases.x), np.float32)
        y = np.ascontiguousarray(cases.y, np.float32)
        fit = np.empty(len(which), np.float64)
        rc = lib().orc_population_f32(ops, offs, which, len(which), x.shape[0], x, y, x.shape[1], fit)
    else:
        inp = np.ascontiguousarray(cases.inputs, np.uint64)
        tg = np.ascontiguousarray(cases.target, np.uint64)
        fit = np.empty(len(which), np.int64)
        rc = lib().orc_population_bool(ops, offs, which, len(which), inp.shape[0], inp, tg, inp.shape[1],
                                       cases.T if T is None else T, fit)
    if rc != 0:
        raise ValueError(f"oracle population evaluation failed ({rc})")
    return fit


def eval_population_f32(pop, x, y, threads: int = 1):
    """Evaluate every tree; several independent single-threaded oracle
    instances when threads > 1 (ctypes releases the GIL during each call)."""
    T = np.atleast_2d(x).shape[1]
    outs = np.empty((pop.n_trees, T), np.float32)
    fits = np.empty(pop.n_trees, np.float64)

    def one(i):
        outs[i] = eval_f32(pop.tree(i), x)
        fits[i] = fitness_f32(outs[i], y)

    if threads <= 1:
        for i in range(pop.n_trees):
            one(i)
    else:
        order = np.argsort(-pop.sizes(), kind="stable")
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, order))
    return outs, fits


def eval_population_bool(pop, inputs, target, T: int, threads: int = 1):
    W = np.asarray(inputs).shape[1]
    outs = np.empty((pop.n_trees, W), np.uint64)
    fits = np.empty(pop.n_trees, np.int64)

    def one(i):
        outs[i] = eval_bool(pop.tree(i), inputs)
        fits[i] = fitness_bool(outs[i], target, T)

    if threads <= 1:
        for i in range(pop.n_trees):
            one(i)
    else:
        order = np.argsort(-pop.sizes(), kind="stable")
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, order))
    return outs, fits


# ------------------------------------------------------------------ selection
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return [int(v) for v in out]


def uniform(u: int, n: int) -> int:
    return int(lib().orc_uniform(u, n))


def draw(seed: int, i: int, g: int, s: int, j: int) -> int:
    return int(lib().orc_draw(seed, i, g, s, j))


def tournament(fit, k: int, seed: int, i: int, g: int, s: int) -> int:
    """Winner of tournament i (stream s, generation g) over `fit`: float64
    errors (lower wins, NaN worst) or int64 hits (higher wins)."""
    fit = np.ascontiguousarray(fit)
    if fit.dtype == np.float64:
        return int(lib().orc_tournament_f64(fit, len(fit), k, seed, i, g, s))
    return int(lib().orc_tournament_i64(np.ascontiguousarray(fit, np.int64), len(fit), k, seed, i, g, s))


def evolve(trees, boolean: bool, cases, generations: int, k: int, seed: int):
    """Generational GP with fitness first (Sections 5 and 6.3), as plainly as
    possible.  Generation g creates N = len(trees) children; child i has the
    winners of tournaments (i, g, stream 0) and (i, g, stream 1) over the
    current fitness as mother and father, a crossover point uniform over the
    mother's nodes (draw (i, g, 2, word 0)) and, as donor, the father's subtree
    at a node uniform over his nodes (word 1).  Every child is scored by
    incremental evaluation before any is built; unless g is the last
    generation, the tournaments of generation g + 1 are drawn over the
    children's fitness and only their winners are built.  Returns one record
    per generation and the final trees (all built)."""
    if boolean:
        inputs, target, T = cases.inputs, cases.target, cases.T
        fit = np.array([fitness_bool(eval_bool(t, inputs), target, T) for t in trees], np.int64)
    else:
        with np.errstate(all="ignore"):
            fit = np.array([fitness_f32(eval_f32(t, cases.x), cases.y) for t in trees], np.float64)
    trees = [np.asarray(t, np.uint8) for t in trees]
    N = len(trees)
    records = []
    for g in range(generations):
        mother = np.array([tournament(fit, k, seed, i, g, 0) for i in range(N)], np.int64)
        father = np.array([tournament(fit, k, seed, i, g, 1) for i in range(N)], np.int64)
        point = np.array([uniform(draw(seed, i, g, 2, 0), len(trees[mother[i]])) for i in range(N)], np.int64)
        dnode = np.array([uniform(draw(seed, i, g, 2, 1), len(trees[father[i]])) for i in range(N)], np.int64)
        cfit = np.zeros(N, np.int64 if boolean else np.float64)
        stop = np.zeros(N, np.int32)
        donors = []
        for i in range(N):
            P, F = trees[mother[i]], trees[father[i]]
            assert P is not None and F is not None, "a tournament winner was not built"
            D = F[dnode[i]:subtree_end(F, int(dnode[i]))].copy()
            donors.append(D)
            if boolean:
                _, lvl, _, fv = incremental_bool(P, int(point[i]), D, inputs, target, T)
            else:
                with np.errstate(all="ignore"):
                    _, lvl, _, fv = incremental_f32(P, int(point[i]), D, cases.x, cases.y)
            cfit[i], stop[i] = fv, lvl
        if g == generations - 1:
            built = np.ones(N, bool)
        else:
            built = np.zeros(N, bool)
            for j in range(N):
                built[tournament(cfit, k, seed, j, g + 1, 0)] = True
                built[tournament(cfit, k, seed, j, g + 1, 1)] = True
        new = [splice(trees[mother[i]], int(point[i]), donors[i]) if built[i] else None for i in range(N)]
        records.append({"mother": mother, "father": father, "point": point, "donor_node": dnode,
                        "fitness": cfit, "stop_level": stop, "built": built,
                        "nodes": np.array([len(trees[mother[i]]) - (subtree_end(trees[mother[i]], int(point[i])) -
                                           int(point[i])) + len(donors[i]) for i in range(N)], np.int64)})
        trees, fit = new, cfit
    return records, trees
