"""Serving loop (continuous batching) on the GPU: every job's result is the
same alone and in the mix, and matches the oracle.  Results are compared
bit-exactly (float outputs: bit-equal or both NaN)."""
import math
import sys
import time

import numpy as np
import pytest

import gen
import oracle
from paper_2205_03251_amd import gpeval as g
from tests.scalar_ref import same_f32

pytestmark = pytest.mark.gpu


def wait(ctx, ticket, vtype, T, timeout=60.0):
    t0 = time.time()
    while True:
        r = ctx.server_poll(ticket, vtype, T)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, f"job {ticket} did not finish"
        time.sleep(0.0005)


def build_jobs(seed=1):
    rng = np.random.default_rng(seed)
    fc = {T: gen.float_cases(T, T) for T in (256, 1024)}
    # Boolean: 8 inputs (256 cases, four words) and 6 inputs (64 cases, the one-word loop)
    bc = {256: gen.bool_cases(8), 64: gen.bool_cases(6)}
    jobs = []   # (vtype, T, parent tree, points, children [(point, donor)])
    for i in range(8):
        vt = g.GP_BOOL if i % 4 == 3 or i == 5 else g.GP_F32
        T = (64 if i == 5 else 256) if vt == g.GP_BOOL else (256 if i % 2 else 1024)
        n_terms = (6 if T == 64 else 8) if vt == g.GP_BOOL else 1
        tree = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 11, 60001)), n_terms=n_terms)
        pts = sorted(set(int(p) for p in rng.integers(len(tree), size=3)))
        kids = []
        for p in pts:
            e = gen.subtree_end(tree, p)
            if rng.random() < 0.5:
                d = gen.neutral_donor(rng, tree[p:e].copy(), 40) if vt == g.GP_F32 else tree[p:e].copy()
            else:
                d = gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 301)), n_terms=n_terms)
            kids.append((p, d))
        jobs.append((vt, T, tree, pts, kids))
    return jobs, fc, bc


def run(ctx, jobs, handles, mix):
    out = {}
    tickets = []
    for ji, (vt, T, tree, pts, kids) in enumerate(jobs):
        h = handles[(vt, T)]
        t = ctx.server_submit(g.GP_JOB_FULL, h, tree, record_points=np.array(pts, np.int64), keep_resident=True)
        if not mix:
            out[("p", ji)] = wait(ctx, t, vt, T)
        tickets.append((ji, t))
    kid_tickets = []
    for ji, t in tickets:
        vt, T, tree, pts, kids = jobs[ji]
        for ki, (p, d) in enumerate(kids):
            kt = ctx.server_submit(g.GP_JOB_INCREMENTAL, handles[(vt, T)], d, parent_ticket=t, point=p)
            if not mix:
                out[("c", ji, ki)] = wait(ctx, kt, vt, T)
            kid_tickets.append((ji, ki, kt))
    if mix:
        for ji, t in tickets:
            vt, T = jobs[ji][0], jobs[ji][1]
            out[("p", ji)] = wait(ctx, t, vt, T)
        for ji, ki, kt in kid_tickets:
            vt, T = jobs[ji][0], jobs[ji][1]
            out[("c", ji, ki)] = wait(ctx, kt, vt, T)
    for ji, t in tickets:
        ctx.server_release(t)
    return out


def test_served_results_same_alone_and_in_mix_and_match_oracle():
    ctx = g.Context(0)
    jobs, fc, bc = build_jobs()
    handles = {(g.GP_F32, T): ctx.set_cases(g.GP_F32, c.x, c.y) for T, c in fc.items()}
    for T, c in bc.items():
        handles[(g.GP_BOOL, T)] = ctx.set_cases(g.GP_BOOL, c.inputs, c.target, T)
    ctx.server_start(n_streams=4, max_batch_jobs=16, prep_threads=4)
    alone = run(ctx, jobs, handles, mix=False)
    print("alone done", file=sys.stderr, flush=True)
    mixed = run(ctx, jobs, handles, mix=True)
    ctx.server_stop()
    assert alone.keys() == mixed.keys()
    for k in alone:
        a, b = alone[k], mixed[k]
        assert a["status"] == 0 and b["status"] == 0, k
        if a["root"].dtype == np.float32:
            assert same_f32(a["root"], b["root"]).all(), k
            assert a["fitness_f64"] == b["fitness_f64"] or (math.isnan(a["fitness_f64"]) and math.isnan(b["fitness_f64"]))
        else:
            assert np.array_equal(a["root"], b["root"]) and a["fitness_i64"] == b["fitness_i64"], k
        assert a["stop_level"] == b["stop_level"], k
    # against the oracle
    for ji, (vt, T, tree, pts, kids) in enumerate(jobs):
        p = alone[("p", ji)]
        if vt == g.GP_F32:
            with np.errstate(all="ignore"):
                want = oracle.eval_f32(tree, fc[T].x)
                w_fit = oracle.fitness_f32(want, fc[T].y)
            assert same_f32(p["root"], want).all()
            assert p["fitness_f64"] == w_fit or (math.isnan(p["fitness_f64"]) and math.isnan(w_fit))
        else:
            want = oracle.eval_bool(tree, bc[T].inputs)
            assert np.array_equal(p["root"], want)
            assert p["fitness_i64"] == oracle.fitness_bool(want, bc[T].target, T)
        for ki, (pt, d) in enumerate(kids):
            c = alone[("c", ji, ki)]
            if vt == g.GP_F32:
                with np.errstate(all="ignore"):
                    w_root, w_lvl, w_int, w_fit = oracle.incremental_f32(tree, pt, d, fc[T].x, fc[T].y)
                assert same_f32(c["root"], w_root).all()
                assert c["fitness_f64"] == w_fit or (math.isnan(c["fitness_f64"]) and math.isnan(w_fit))
            else:
                w_root, w_lvl, w_int, w_fit = oracle.incremental_bool(tree, pt, d, bc[T].inputs, bc[T].target, T)
                assert np.array_equal(c["root"], w_root)
                assert c["fitness_i64"] == w_fit
            assert c["stop_level"] == w_lvl
            assert c["interpreted_nodes"] == w_int
    ctx.close()


def test_server_rejects_bad_jobs():
    ctx = g.Context(0)
    c = gen.float_cases(1, 64)
    h = ctx.set_cases(g.GP_F32, c.x, c.y)
    ctx.server_start(n_streams=2, max_batch_jobs=4, prep_threads=2)
    t = ctx.server_submit(g.GP_JOB_FULL, h, np.array([0x80, 0], np.uint8))      # malformed
    r = wait(ctx, t, g.GP_F32, 64)
    assert r["status"] == g.GP_EINVAL
    with pytest.raises(g.GPError):                                               # unknown parent
        ctx.server_submit(g.GP_JOB_INCREMENTAL, h, np.array([0], np.uint8), parent_ticket=999, point=0)
    p = ctx.server_submit(g.GP_JOB_FULL, h, np.array([0x80, 0, 0], np.uint8), record_points=np.array([1]),
                          keep_resident=True)
    with pytest.raises(g.GPError) as e:                                          # point not recorded
        ctx.server_submit(g.GP_JOB_INCREMENTAL, h, np.array([0], np.uint8), parent_ticket=p, point=2)
    assert e.value.code == g.GP_ENOTFOUND
    k = ctx.server_submit(g.GP_JOB_INCREMENTAL, h, np.array([0], np.uint8), parent_ticket=p, point=1)
    r = wait(ctx, k, g.GP_F32, 64)
    assert r["status"] == 0 and r["stop_level"] == 0
    ctx.server_release(p)
    ctx.server_stop()
    ctx.close()


def test_server_budget_admission():
    # a budget that fits only a few jobs at once still completes all of them
    ctx = g.Context(0)
    c = gen.float_cases(2, 1024)
    h = ctx.set_cases(g.GP_F32, c.x, c.y)
    ctx.server_start(n_streams=4, max_batch_jobs=8, prep_threads=4, budget_bytes=2 << 20)
    rng = np.random.default_rng(3)
    trees = [gen.sized_tree(rng, 20001) for _ in range(12)]
    ts = [ctx.server_submit(g.GP_JOB_FULL, h, t) for t in trees]
    for t, tree in zip(ts, trees):
        r = wait(ctx, t, g.GP_F32, 1024)
        assert r["status"] == 0
        with np.errstate(all="ignore"):
            assert same_f32(r["root"], oracle.eval_f32(tree, c.x)).all()
    with pytest.raises(g.GPError) as e:
        ctx.server_submit(g.GP_JOB_FULL, h, gen.sized_tree(rng, 30_000_001))
    assert e.value.code == g.GP_EBUDGET
    ctx.server_stop()
    ctx.close()


def test_release_waits_for_children_still_compiling():
    """A resident parent cannot be released while a child submitted against
    it is not done, including a child whose donor a prep thread is still
    compiling; every child completes with the oracle's result."""
    ctx = g.Context(0)
    c = gen.float_cases(4, 512)
    h = ctx.set_cases(g.GP_F32, c.x, c.y)
    ctx.server_start(n_streams=2, max_batch_jobs=4, prep_threads=2)
    rng = np.random.default_rng(5)
    tree = gen.sized_tree(rng, 40001)
    pts = [1, 17, 333]
    p = ctx.server_submit(g.GP_JOB_FULL, h, tree, record_points=np.array(pts, np.int64), keep_resident=True)
    assert wait(ctx, p, g.GP_F32, 512)["status"] == 0
    donors = [gen.sized_tree(rng, 200001) for _ in pts]
    kids = [ctx.server_submit(g.GP_JOB_INCREMENTAL, h, d, parent_ticket=p, point=q) for d, q in zip(donors, pts)]
    released = False
    try:
        ctx.server_release(p)
        released = True
    except g.GPError as e:
        assert e.code == g.GP_EBUSY
    for k, d, q in zip(kids, donors, pts):
        r = wait(ctx, k, g.GP_F32, 512)
        assert r["status"] == 0
        with np.errstate(all="ignore"):
            w_root, w_lvl, w_int, w_fit = oracle.incremental_f32(tree, q, d, c.x, c.y)
        assert same_f32(r["root"], w_root).all() and r["stop_level"] == w_lvl
        assert r["fitness_f64"] == w_fit or (math.isnan(r["fitness_f64"]) and math.isnan(w_fit))
        assert r["root_bytes"] == 512 * 4
    if not released:
        ctx.server_release(p)
    with pytest.raises(g.GPError):                    # gone now
        ctx.server_release(p)
    ctx.server_stop()
    ctx.close()


def test_poll_refuses_a_small_output_buffer():
    """gp_server_poll writes the output vector only into a buffer that holds
    it; the result stays available for a second poll."""
    import ctypes as C
    ctx = g.Context(0)
    c = gen.float_cases(6, 300)
    h = ctx.set_cases(g.GP_F32, c.x, c.y)
    ctx.server_start(n_streams=1, max_batch_jobs=2, prep_threads=1)
    t = ctx.server_submit(g.GP_JOB_FULL, h, np.array([gen.F_MUL, 0, 0], np.uint8))
    small = np.zeros(299, np.float32)
    r = g.JobResult()
    deadline = time.time() + 60
    while True:
        rc = g.lib().gp_server_poll(ctx._h, t, C.byref(r), small.ctypes.data, small.nbytes)
        if rc != g.GP_EBUSY:
            break
        assert time.time() < deadline
        time.sleep(0.001)
    assert rc == g.GP_EINVAL
    assert not small.any()
    out = wait(ctx, t, g.GP_F32, 300)
    assert out["status"] == 0 and out["root_bytes"] == 1200
    assert same_f32(out["root"], c.x[0] * c.x[0]).all()
    ctx.server_stop()
    ctx.close()


def to_postfix(t):
    """Reverse Polish form of a prefix tree and the RPN index of every prefix
    node (operands left then right, then the function)."""
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


def test_device_compiled_jobs_match_host_compiled():
    """Full jobs compiled on the device (every one of them, down to one-node
    trees, with device_compile_nodes=1) give the same results, and their
    children the same incremental results, as with host compilation; a job
    given in reverse Polish order keeps its caller's point indices."""
    rng = np.random.default_rng(5)
    fc = gen.float_cases(7, 512)
    bc = gen.bool_cases(8)
    ctx = g.Context(0)
    hf = ctx.set_cases(g.GP_F32, fc.x, fc.y)
    hb = ctx.set_cases(g.GP_BOOL, bc.inputs, bc.target, 256)
    jobs = []    # (vtype, handle, layout, ops, points (job layout), children [(point (job layout), donor (job layout))])
    for n, vt in [(1, g.GP_F32), (3, g.GP_BOOL), (2001, g.GP_F32), (40001, g.GP_BOOL), (300001, g.GP_F32),
                  (120001, g.GP_F32)]:
        nt = 8 if vt == g.GP_BOOL else 1
        tree = gen.sized_tree(rng, n, n_terms=nt)
        pts = sorted(set(int(p) for p in rng.integers(n, size=3)))
        kids = [(p, gen.sized_tree(rng, int(gen.log_uniform_odd(rng, 1, 201)), n_terms=nt)) for p in pts]
        jobs.append((vt, hb if vt == g.GP_BOOL else hf, g.GP_PREFIX, tree, pts, kids))
    # the last one in reverse Polish order, points and donors too
    vt, h, _, tree, pts, kids = jobs[-1]
    post, where = to_postfix(tree)
    jobs[-1] = (vt, h, g.GP_POSTFIX, post, [int(where[p]) for p in pts],
                [(int(where[p]), to_postfix(d)[0]) for p, d in kids])
    results = {}
    for dcn in (-1, 1):
        ctx.server_start(n_streams=4, max_batch_jobs=8, prep_threads=4, device_compile_nodes=dcn)
        out, tickets = {}, []
        for ji, (vt, h, lay, ops, pts, kids) in enumerate(jobs):
            tickets.append(ctx.server_submit(g.GP_JOB_FULL, h, ops, layout=lay, record_points=np.array(pts, np.int64),
                                             keep_resident=True))
        kid_t = []
        for ji, (vt, h, lay, ops, pts, kids) in enumerate(jobs):
            for ki, (p, d) in enumerate(kids):
                kid_t.append((ji, ki, ctx.server_submit(g.GP_JOB_INCREMENTAL, h, d, layout=lay,
                                                        parent_ticket=tickets[ji], point=p)))
        Ts = {hf: fc.T, hb: 256}
        for ji, t in enumerate(tickets):
            out[("p", ji)] = wait(ctx, t, jobs[ji][0], Ts[jobs[ji][1]])
        for ji, ki, t in kid_t:
            out[("c", ji, ki)] = wait(ctx, t, jobs[ji][0], Ts[jobs[ji][1]])
        for t in tickets:
            ctx.server_release(t)
        ctx.server_stop()
        results[dcn] = out
    host, dev = results[-1], results[1]
    for k in host:
        a, b = host[k], dev[k]
        assert a["status"] == 0 and b["status"] == 0, k
        if a["root"].dtype == np.float32:
            assert same_f32(a["root"], b["root"]).all(), k
            assert a["fitness_f64"] == b["fitness_f64"] or (math.isnan(a["fitness_f64"]) and math.isnan(b["fitness_f64"]))
        else:
            assert np.array_equal(a["root"], b["root"]) and a["fitness_i64"] == b["fitness_i64"], k
        assert a["stop_level"] == b["stop_level"] and a["interpreted_nodes"] == b["interpreted_nodes"], k
        if k[0] == "p":
            assert a["device_compiled"] == 0 and b["device_compiled"] == 1, k
    ctx.close()
    # the device-compiled parents against the oracle (their children were compared above)
    for ji, (vt, h, lay, ops, pts, kids) in enumerate(jobs[:-1]):
        got = dev[("p", ji)]
        if vt == g.GP_F32:
            with np.errstate(all="ignore"):
                want = oracle.eval_f32(ops, fc.x)
            assert same_f32(got["root"], want).all(), ji
        else:
            assert np.array_equal(got["root"], oracle.eval_bool(ops, bc.inputs)), ji
