"""The serving loop at the served-stream configuration's shape: float32 jobs
with 4096 cases and Boolean jobs with k = 12 inputs (4096 cases, 64 words),
resident parents of 10^6 to 10^7 nodes with three recorded points each,
incremental children at those points (donors of 1 to 10^4 nodes, one in
three neutral) and small full jobs in between.

Every job's result is the same alone (submitted and waited for one at a
time) and in the mix (everything submitted at once), bit for bit: outputs,
fitness, stop level and interpreted count (Section 4.1: independent jobs
share the device).  Against the oracle: every Boolean job, the small jobs,
and the 1.2e6-node float parent with its children on all 4096 cases (split
over blocks of cases, tests/split_oracle.py); the 9e6-node float parent and
its children on a sample of 256 cases (outputs bit-equal there, the
sample's stop level at most the job's, fitness equal to the oracle's fixed-
order sum over the job's output vector).
"""
import math
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g
from tests import split_oracle as so
from tests.scalar_ref import same_f32

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

POOL = 16
T = 4096
K = 12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def wait(ctx, ticket, vtype, timeout=120.0):
    t0 = time.time()
    while True:
        r = ctx.server_poll(ticket, vtype, T)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, f"job {ticket} did not finish"
        time.sleep(0.0005)


def build(seed=11):
    rng = np.random.default_rng(seed)
    parents = []    # (name, vtype, tree, points, children [(point, donor, neutral)])
    for name, vt, n in [("F1", g.GP_F32, 1_200_001), ("F2", g.GP_F32, 9_000_001),
                        ("B1", g.GP_BOOL, 2_000_001), ("B2", g.GP_BOOL, 10_000_001)]:
        nt = K if vt == g.GP_BOOL else 1
        tree = gen.sized_tree(rng, n, n_terms=nt)
        pts = [int(p) for p in np.unique(rng.integers(n, size=3))]
        kids = []
        for ci, p in enumerate(pts):
            m = int(gen.log_uniform_odd(rng, 1, 10_001))
            e = gen.subtree_end(tree, p, max_len=max(1, m - 4))
            if ci == 0 and e > 0:
                S = tree[p:e].copy()
                d = gen.neutral_donor(rng, S, m) if vt == g.GP_F32 else gen.bool_neutral_donor(rng, S, m, nt)
                kids.append((p, d, True))
            else:
                kids.append((p, gen.sized_tree(rng, m, n_terms=nt), False))
        parents.append((name, vt, tree, pts, kids))
    small = []
    for i in range(8):
        vt = g.GP_BOOL if i % 2 else g.GP_F32
        small.append((vt, gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 11, 100_001)),
                                         n_terms=K if vt == g.GP_BOOL else 1)))
    return parents, small


def run(ctx, handles, parents, small, mix):
    out = {}
    pt = {}
    order = []
    for pi, (name, vt, tree, pts, kids) in enumerate(parents):
        t = ctx.server_submit(g.GP_JOB_FULL, handles[vt], tree, record_points=np.array(pts, np.int64),
                              keep_resident=True)
        pt[pi] = t
        order.append((("p", pi), t, vt))
        if not mix:
            out[("p", pi)] = wait(ctx, t, vt)
        if pi < len(small):
            vs, ts = small[pi]
            st = ctx.server_submit(g.GP_JOB_FULL, handles[vs], ts)
            order.append((("s", pi), st, vs))
            if not mix:
                out[("s", pi)] = wait(ctx, st, vs)
        for ki, (p, d, _) in enumerate(kids):
            kt = ctx.server_submit(g.GP_JOB_INCREMENTAL, handles[vt], d, parent_ticket=t, point=p)
            order.append((("c", pi, ki), kt, vt))
            if not mix:
                out[("c", pi, ki)] = wait(ctx, kt, vt)
    for si in range(len(parents), len(small)):
        vs, ts = small[si]
        st = ctx.server_submit(g.GP_JOB_FULL, handles[vs], ts)
        order.append((("s", si), st, vs))
        if not mix:
            out[("s", si)] = wait(ctx, st, vs)
    if mix:
        for key, t, vt in order:
            out[key] = wait(ctx, t, vt)
    for t in pt.values():
        ctx.server_release(t)
    return out


def same_result(a, b):
    if a["status"] != 0 or b["status"] != 0:
        return False
    if a["root"].dtype == np.float32:
        fa, fb = a["fitness_f64"], b["fitness_f64"]
        ok = same_f32(a["root"], b["root"]).all() and (fa == fb or (math.isnan(fa) and math.isnan(fb)))
    else:
        ok = np.array_equal(a["root"], b["root"]) and a["fitness_i64"] == b["fitness_i64"]
    return ok and a["stop_level"] == b["stop_level"] and a["interpreted_nodes"] == b["interpreted_nodes"]


def fit_equal(a, b):
    return a == b or (math.isnan(a) and math.isnan(b))


def test_served_stream_shape_alone_mix_and_oracle():
    fc = gen.float_cases(12, T)
    bc = gen.bool_cases(K)
    say("generating trees")
    parents, small = build()
    ctx = g.Context(0)
    handles = {g.GP_F32: ctx.set_cases(g.GP_F32, fc.x, fc.y),
               g.GP_BOOL: ctx.set_cases(g.GP_BOOL, bc.inputs, bc.target, T)}
    ctx.server_start(n_streams=4, max_batch_jobs=16, prep_threads=8, device_compile_nodes=262144)
    say("alone")
    alone = run(ctx, handles, parents, small, mix=False)
    say("mix")
    mixed = run(ctx, handles, parents, small, mix=True)
    ctx.server_stop()
    ctx.close()
    assert alone.keys() == mixed.keys()
    for k in alone:
        assert same_result(alone[k], mixed[k]), k
    for pi in range(len(parents)):                  # trees of 1.2e6..1e7 nodes: compiled on the device
        assert alone[("p", pi)]["device_compiled"] == 1 and mixed[("p", pi)]["device_compiled"] == 1
    say("oracle")
    with ThreadPoolExecutor(POOL) as pool:
        sample = np.concatenate([np.arange(0, 128), np.arange(T - 128, T)])
        for pi, (name, vt, tree, pts, kids) in enumerate(parents):
            say("oracle", name)
            got = alone[("p", pi)]
            if vt == g.GP_BOOL:
                w_out, w_hits = so.eval_bool(tree, bc.inputs, bc.target, T, POOL, pool)
                assert np.array_equal(got["root"], w_out) and got["fitness_i64"] == w_hits, name
            elif name == "F1":
                with np.errstate(all="ignore"):
                    w_out, w_fit = so.eval_f32(tree, fc.x, fc.y, POOL * 2, pool)
                assert same_f32(got["root"], w_out).all() and fit_equal(got["fitness_f64"], w_fit), name
            else:
                with np.errstate(all="ignore"):
                    w_out, _ = so.eval_f32(tree, fc.x[:, sample], fc.y[sample], POOL, pool)
                    assert fit_equal(got["fitness_f64"], oracle.fitness_f32(got["root"], fc.y))
                assert same_f32(got["root"][sample], w_out).all(), name
            for ki, (p, d, neutral) in enumerate(kids):
                c = alone[("c", pi, ki)]
                if vt == g.GP_BOOL:
                    w = so.incremental_bool(tree, p, d, bc.inputs, bc.target, T, POOL, pool)
                    assert np.array_equal(c["root"], w[0]) and c["fitness_i64"] == w[3], (name, ki)
                    assert c["stop_level"] == w[1] and c["interpreted_nodes"] == w[2], (name, ki)
                elif name == "F1":
                    w = so.incremental_f32(tree, p, d, fc.x, fc.y, POOL * 2, pool)
                    assert same_f32(c["root"], w[0]).all() and fit_equal(c["fitness_f64"], w[3]), (name, ki)
                    assert c["stop_level"] == w[1] and c["interpreted_nodes"] == w[2], (name, ki)
                else:
                    w = so.incremental_f32(tree, p, d, fc.x, fc.y, POOL, pool, cols=sample)
                    assert same_f32(c["root"][sample], w[0]).all(), (name, ki)
                    level = c["stop_level"]
                    assert w[1] != -1 or level == -1, (name, ki, w[1], level)
                    assert level == -1 or w[1] <= level, (name, ki, w[1], level)
                    with np.errstate(all="ignore"):
                        assert fit_equal(c["fitness_f64"], oracle.fitness_f32(c["root"], fc.y)), (name, ki)
                if neutral:
                    assert c["stop_level"] == 0, (name, ki)
        for si, (vs, ts) in enumerate(small):
            got = alone[("s", si)]
            if vs == g.GP_BOOL:
                w_out, w_hits = so.eval_bool(ts, bc.inputs, bc.target, T, 4, pool)
                assert np.array_equal(got["root"], w_out) and got["fitness_i64"] == w_hits, si
            else:
                with np.errstate(all="ignore"):
                    w_out, w_fit = so.eval_f32(ts, fc.x, fc.y, 8, pool)
                assert same_f32(got["root"], w_out).all() and fit_equal(got["fitness_f64"], w_fit), si
