"""The device tree compiler's steps, run on the CPU, give the host compiler's
programs byte for byte.

tests/csrc/devcompile_emu.cpp runs the per-thread steps of
paper_2205_03251_amd/csrc/devcompile_core.h (the same source the HIP kernels
instantiate) with its terminal threads in random interleavings, then compares
every tree with compile_tree: code words, chunk tables, stack bound, records,
spines and the index of large subtrees.  The shapes cover the cut rules: chunk
size cuts at several targets, stack-need cuts (complete trees need more slots
than the 10 the programs are compiled for), combs leaning either way, one-node
trees, float and Boolean folding, and crossover points at the root, at
terminals, repeated, and on shared paths."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("emu") / "devcompile_emu")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "csrc", "devcompile_emu.cpp"),
                    os.path.join(ROOT, "paper_2205_03251_amd", "csrc", "prep.cpp")], check=True)
    return exe


def run(exe, pop, chunk_nodes, index_min=0, points=None, seed=1, mode=1, handoffs=None, host_threads=1):
    """Runs both hand-offs (the packed one where the chunk target allows it)
    and checks each against compile_tree (on host_threads threads)."""
    if handoffs is None:
        handoffs = [0, 1] if chunk_nodes <= 8192 else [0]
    got = None
    for h in handoffs:
        got = run_one(exe, pop, chunk_nodes, index_min, points, seed, mode, h, host_threads)
    return got


def run_one(exe, pop, chunk_nodes, index_min, points, seed, mode, handoff, host_threads):
    pts = points if points is not None else [[] for _ in range(pop.n_trees)]
    ro = np.cumsum([0] + [len(p) for p in pts])
    words = [pop.vtype, pop.n_inputs, chunk_nodes, index_min, pop.n_trees, seed, mode, handoff, host_threads]
    text = " ".join(map(str, words)) + "\n" + " ".join(map(str, pop.offsets.tolist())) + "\n" + \
        " ".join(map(str, pop.ops.tolist())) + "\n" + " ".join(map(str, ro.tolist())) + "\n" + \
        " ".join(str(c) for p in pts for c in p) + "\n"
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    f = r.stdout.split()
    assert f[0] == "ok"
    return dict(zip(f[1::2], map(int, f[2::2])))


def random_points(seed, pop, per_tree):
    rng = np.random.default_rng(seed)
    pts = []
    for t in range(pop.n_trees):
        n = int(pop.sizes()[t])
        p = [int(v) for v in rng.integers(0, n, size=per_tree)]
        if per_tree:
            p += [0, p[0]]                       # the root, and a repeated point
        pts.append(p)
    return pts


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


def comb(depth, left, n_terms=1, seed=0):
    rng = np.random.default_rng(seed)
    # left comb: F (F (F x x) x) x; right comb: F x (F x (F x x))
    if left:
        ops = [0x80 + int(v) for v in rng.integers(4, size=depth)] + \
              [int(v) for v in rng.integers(n_terms, size=depth + 1)]
    else:
        ops = []
        for f in rng.integers(4, size=depth):
            ops += [0x80 + int(f), int(rng.integers(n_terms))]
        ops.append(int(rng.integers(n_terms)))
    return np.array(ops, np.uint8)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("chunk_nodes", [16, 33, 256])
def test_ramped_float(emu, chunk_nodes, mode):
    pop = gen.ramped_half_and_half(3, 100)
    got = run(emu, pop, chunk_nodes, 0, random_points(5, pop, 2), seed=chunk_nodes, mode=mode)
    assert got["records"] > 0


@pytest.mark.parametrize("chunk_nodes", [16, 64])
def test_ramped_boolean(emu, chunk_nodes):
    pop = gen.ramped_half_and_half(4, 100, n_terms=6, vtype=gen.VT_BOOL)
    run(emu, pop, chunk_nodes, 0, random_points(6, pop, 3))


@pytest.mark.parametrize("vtype,n_terms", [(gen.VT_F32, 1), (gen.VT_BOOL, 6)])
@pytest.mark.parametrize("chunk_nodes", [17, 256, 1024])
def test_sized_trees(emu, vtype, n_terms, chunk_nodes):
    pop = gen.sized_population(7 + chunk_nodes, 24, 1, 30001, n_terms=n_terms, vtype=vtype)
    got = run(emu, pop, chunk_nodes, 512, random_points(8, pop, 2), seed=chunk_nodes)
    assert got["chunks"] > pop.n_trees


def test_stack_need_cuts(emu):
    # complete trees of depth 11 to 14 need 12 to 15 slots: the need rule cuts
    # them even when the chunk target is never reached
    trees = [complete(d, seed=d) for d in (11, 12, 13, 14)] + [complete(12, n_terms=6, seed=9)]
    pop = gen.pack(trees[:4], gen.VT_F32, 1)
    got = run(emu, pop, 10 ** 6, 64, random_points(9, pop, 4))
    assert got["chunks"] > pop.n_trees
    run(emu, pop, 100, 64, random_points(10, pop, 4), mode=0)
    run(emu, gen.pack(trees[4:], gen.VT_BOOL, 6), 1000, 0, [[0, 1, 4000, 8190]])


def test_combs_and_single_nodes(emu):
    trees = [comb(3000, True, seed=1), np.array([0], np.uint8), comb(2999, False, seed=2),
             np.array([0x81, 0, 0], np.uint8), np.array([0], np.uint8)]
    pop = gen.pack(trees, gen.VT_F32, 1)
    pts = [[0, 5, 2999, 6000], [0], [1, 5997, 3000], [0, 1, 2], []]
    for c in (2, 16, 128, 5000, 8192, 8193):
        run(emu, pop, c, 64, pts, seed=c)


def test_one_large_tree_interleaved(emu):
    pop = gen.sized_population(11, 1, 200001, 200001)
    got = run(emu, pop, 1024, 4096, [[0, 7, 1000, 150000]])
    assert got["chunks"] > 100
    run(emu, pop, 8192, 4096, [[0, 7, 1000, 150000]], mode=0)


@pytest.mark.parametrize("host_threads", [2, 4, 7])
def test_host_compiler_on_several_threads_with_records(emu, host_threads):
    # compile_tree's parallel pass (trees of 2e5 nodes and more): segments of
    # the array, then the nodes whose subtrees cross a segment's end; with
    # crossover points recorded it must give the same programs as one thread
    # (and as the device steps)
    pop = gen.sized_population(60 + host_threads, 4, 200001, 600001)
    pts = random_points(61, pop, 3)
    run(emu, pop, 256, 4096, pts, host_threads=host_threads, handoffs=[1])
    run(emu, pop, 16, 0, pts, host_threads=host_threads, handoffs=[1], mode=0)
