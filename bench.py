#!/usr/bin/env python3
"""Benchmark: equivalent and interpreted GP operations per second on one MI355X.

Default workload (incremental evaluation in a converged population): 500
parent trees of 1e6..1e7 nodes (log-uniform, uniform random shapes, float32
functions + - * /protected over terminal x), 1024 test cases x ~ U[-1, 1),
sextic target; one crossover child per parent (point uniform over nodes,
donor 1..1e4 nodes, half of the donors semantically neutral).

One step = one pass over the whole evaluation path on device-resident data:
  full batched evaluation of the parent population in one persistent launch
  (recording the parent caches along each child's path), then bottom-up
  incremental evaluation of the 500 children with the failed-disruption stop.
Host-side loading (validation, compilation, chunking, upload) happens once
before the timed region and is reported separately.

Prints ONE JSON line.  `value` = equivalent GPop/s of the step (tree nodes x
test cases per second, every tree and child counted in full).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import gen  # noqa: E402

# FP32 VALU peak: 256 CUs x 4 SIMDs x 32 lane-operations per cycle x 2.4 GHz = 78.64e12 lane-ops/s, the published
# 157.3 TFLOP/s with an FMA counted as two flops (a wave64 add, mul or fma issues every two cycles per SIMD; the
# VALU calibration measures 2.34)
PEAK_FP32_LANE_OPS = 256 * 4 * 32 * 2.4e9
PEAK_HBM_GBPS = 8000.0                        # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_inputs(name: str, scale: float, threads: int):
    if name == "incremental":
        n = max(2, int(round(500 * scale)))
        parents = gen.sized_population(4, n, 10**6, 10**7, threads=threads)
        cases = gen.float_cases(4, 1024)
        kids = gen.crossover_children(40, parents, n, donor_lo=1, donor_hi=10**4, neutral_frac=0.5)
        desc = {"workload": "incremental_converged", "parents": n, "parent_nodes": "log-uniform 1e6..1e7",
                "children": n, "donor_nodes": "log-uniform 1..1e4", "neutral_frac": 0.5, "test_cases": 1024,
                "value_type": "float32"}
        return parents, cases, kids, desc
    if name == "full_large":
        n = max(2, int(round(1000 * scale)))
        pop = gen.sized_population(3, n, 10**4, 10**6, threads=threads)
        return pop, gen.float_cases(3, 1024), None, {
            "workload": "full_large", "trees": n, "tree_nodes": "log-uniform 1e4..1e6", "test_cases": 1024,
            "value_type": "float32"}
    if name == "boolean":
        n = max(2, int(round(1000 * scale)))
        pop = gen.sized_population(2, n, 10**3, 10**5, n_terms=6, vtype=gen.VT_BOOL, threads=threads)
        return pop, gen.bool_cases(6), None, {
            "workload": "boolean_parity6", "trees": n, "tree_nodes": "log-uniform 1e3..1e5", "test_cases": 64,
            "value_type": "bool"}
    if name == "small":
        return gen.ramped_half_and_half(1), gen.float_cases(1, 48), None, {
            "workload": "small_ramped", "trees": 100, "test_cases": 48, "value_type": "float32"}
    raise SystemExit(f"unknown workload {name}")


def load_timed(ctx, vtype, pop, host=True, **kw):
    """Load pop compiled on the device (returned, with its wall time) and,
    when host is set, the same trees compiled on the host (timed, freed)."""
    host_s = None
    if host:
        t = time.perf_counter()
        h = ctx.load_population(vtype, pop.ops, pop.offsets, n_inputs=pop.n_inputs, **kw)
        host_s = time.perf_counter() - t
        ctx.free(h)
    t = time.perf_counter()
    ph = ctx.load_population(vtype, pop.ops, pop.offsets, n_inputs=pop.n_inputs, device_compile=True, **kw)
    return ph, time.perf_counter() - t, host_s


def record_lists(n_trees, kids):
    pts = [[] for _ in range(n_trees)]
    for p, c in zip(kids.parent, kids.point):
        pts[int(p)].append(int(c))
    offs = np.zeros(n_trees + 1, np.int64)
    offs[1:] = np.cumsum([len(p) for p in pts])
    return np.array([c for p in pts for c in p], np.int64), offs


def host_cpu():
    """The GPU host's CPU: nproc (CPUs this process may run on), os.cpu_count()
    and the model name from lscpu (else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count(), "model": model}


def oracle_full(pop, cases, vtype, threads, budget_s, cpu, gpu_fit=None):
    """The oracle as it stands (single-threaded C stack interpreter, its
    plain loop over trees), as `threads` independent instances, each taking a
    share of a bounded sample balanced by size (longest tree to the least
    loaded instance): the smallest trees, at least one per instance, until
    about budget_s of work per instance at the rate the oracle measures on
    the smallest tree.  A sample that is the whole population is run again
    until it takes a measurable time.  With gpu_fit, the sample's fitness
    values are compared with the GPU's."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    T = cases.T
    sizes = pop.sizes()
    order = np.argsort(sizes, kind="stable")
    # the oracle's rate on this population, from its smallest trees (a few ms)
    probe, tot = [], 0
    for i in order:
        probe.append(int(i))
        tot += int(sizes[i])
        if tot * T >= 2e6:
            break
    tp = time.perf_counter()
    oracle.population_fitness(pop, np.array(probe, np.int64), cases)
    rate = max(1e6, tot * T / max(1e-6, time.perf_counter() - tp))
    target = budget_s * rate * threads
    chosen, tot = [], 0
    for i in order:
        if tot >= target and len(chosen) >= threads:
            break
        chosen.append(int(i))
        tot += int(sizes[i]) * T
    shares = [[] for _ in range(min(threads, len(chosen)))]
    load = np.zeros(len(shares))
    for i in sorted(chosen, key=lambda i: -sizes[i]):
        k = int(np.argmin(load))
        shares[k].append(i)
        load[k] += sizes[i]
    shares = [np.array(sh, np.int64) for sh in shares]
    fits = {}
    # a whole small population: each instance repeats its share for about 50 ms per call
    whole = len(chosen) == pop.n_trees
    reps = max(1, int(0.05 * rate / max(1, tot / len(shares)))) if whole else 1

    def one(sh):
        for _ in range(reps):
            f = oracle.population_fitness(pop, sh, cases)
        for i, v in zip(sh.tolist(), f.tolist()):
            fits[i] = v
        return int(sizes[sh].sum()) * T * reps

    t0 = time.perf_counter()
    ops_done, passes = 0, 0
    with ThreadPoolExecutor(len(shares)) as ex:
        while passes == 0 or (whole and time.perf_counter() - t0 < min(1.0, budget_s)):
            ops_done += sum(ex.map(one, shares))
            passes += reps
    dt = time.perf_counter() - t0
    out = {"value": round(ops_done / dt / 1e9, 4), "unit": "GPop/s", "cores": len(shares),
           "kind": "oracle", "nproc": cpu["nproc"], "cpu_model": cpu["model"],
           "sample": f"full evaluation of the {len(chosen)} smallest of the {pop.n_trees} trees "
                     f"({int(sizes[chosen].sum())} nodes) on all {T} cases"
                     + (f", {passes} passes" if passes > 1 else "") + f", {dt:.2f} s"}
    if gpu_fit is not None:
        same = all(fits[i] == gpu_fit[i] or (np.isnan(fits[i]) and np.isnan(gpu_fit[i])) for i in chosen)
        out["sample_fitness_equals_gpu"] = bool(same)
    return out


def oracle_incremental(pop, cases, kids, threads, cpu, gpu_fit=None, gpu_stop=None):
    """The oracle's incremental evaluation (the paper's co-evaluation of the
    mother alongside the child, Section 6.2) of the children of the `threads`
    smallest parents, one child per thread."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    T = cases.T
    psz = pop.sizes()
    order = [int(i) for i in np.argsort(psz[kids.parent], kind="stable")[:threads]]
    res = {}

    def one(i):
        P = pop.tree(int(kids.parent[i]))
        with np.errstate(all="ignore"):
            r = oracle.incremental_f32(P, int(kids.point[i]), kids.donors.tree(i), cases.x, cases.y)
        res[i] = r
        c = int(kids.point[i])
        child = len(P) - (gen.subtree_end(P, c) - c) + len(kids.donors.tree(i))
        return child * T, (len(P) + len(kids.donors.tree(i))) * T

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        done = list(ex.map(one, order))
    dt = time.perf_counter() - t0
    out = {"value": round(sum(d[0] for d in done) / dt / 1e9, 4), "unit": "equivalent GPop/s",
           "executed_gpops": round(sum(d[1] for d in done) / dt / 1e9, 4),
           "cores": int(min(threads, len(order))), "kind": "oracle", "nproc": cpu["nproc"],
           "cpu_model": cpu["model"],
           "sample": f"incremental evaluation (mother co-evaluated) of the {len(order)} children of the smallest "
                     f"parents ({int(psz[kids.parent[order]].sum())} mother nodes) on all {T} cases, {dt:.1f} s"}
    if gpu_fit is not None:
        out["sample_equals_gpu"] = bool(all(
            (res[i][3] == gpu_fit[i] or (np.isnan(res[i][3]) and np.isnan(gpu_fit[i]))) and
            res[i][1] == gpu_stop[i] for i in order))
    return out


def add_counted(roofline, workload, chunk_nodes, variant, waves_per_cu, kernel_ms):
    """Fill roofline's traffic and counter VALU rate from profiles/counters.json:
    a record of the same workload, chunk size, variant and launch width, taken
    with the current kernel sources.  Returns the file's contents, or None."""
    try:
        import hashlib
        rec = json.load(open(os.path.join(ROOT, "profiles", "counters.json")))
        h = hashlib.sha256()
        for f in rec["kernel_source_files"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["kernel_source_sha256"]:
            return None
        for r in rec["records"]:
            if (r.get("workload", rec["workload"]) == workload and r["chunk_nodes"] == chunk_nodes
                    and r["variant"] == variant and r.get("waves_per_cu", 0) == waves_per_cu):
                # read bytes by request size (FETCH_SIZE counts a 128-byte request as 64 bytes on this chip)
                roofline["traffic"] = int(r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"])
                roofline["traffic_GBps"] = round(roofline["traffic"] / (kernel_ms * 1e-3) / 1e9, 1)
                roofline["valu_lane_op_frac_counters"] = round(
                    r["valu_instructions_per_launch"] * 64 / (kernel_ms * 1e-3) / PEAK_FP32_LANE_OPS, 4)
                roofline["counters_source"] = r.get("source")
                return rec
    except (OSError, KeyError, ValueError):
        pass
    return None


def measure_config(ctx, g, name, threads, cpu, cpu_budget_s, no_cpu=False):
    """One full-evaluation configuration on its own: autotuned batched launch
    (graph replay) against one launch per tree, the interpreter kernel's
    roofline, and the oracle on 1 core and on `threads` cores."""
    t0 = time.perf_counter()
    pop, cases, _, desc = workload_inputs(name, 1.0, threads)
    vtype = g.GP_BOOL if desc["value_type"] == "bool" else g.GP_F32
    T = cases.T
    n = pop.n_trees
    total = int(pop.sizes().sum())
    if vtype == g.GP_BOOL:
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, T)
    else:
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    ph, load_s, host_load_s = load_timed(ctx, vtype, pop)
    v, _ = ctx.autotune(ph, ch)
    info = ctx.population_info(ph)
    _, fit, st = ctx.evaluate_full(ph, ch, vtype, n, T, roots=False)
    reps = 50 if total * T < 10**9 else 10
    bms, wms = [], []
    for _ in range(reps):
        _, _, st = ctx.evaluate_full(ph, ch, vtype, n, T, roots=False, device=True)
        bms.append(st["device_ms"])
        wms.append(st["wall_ms"])
    batched_ms = float(np.median(bms))
    kms = [ctx.evaluate_full(ph, ch, vtype, n, T, roots=False, graph=False)[2]["kernel_ms"] for _ in range(5)]
    kernel_ms = float(np.median(kms))
    pts = [ctx.evaluate_full(ph, ch, vtype, n, T, roots=False, per_tree=True, graph=False)[2]["device_ms"]
           for _ in range(2 if total * T < 10**10 else 1)]
    per_tree_ms = float(min(pts))
    func_nodes = (total - n) // 2
    achieved = func_nodes * T / (kernel_ms * 1e-3)
    out = {**desc, "total_nodes": total, "chunk_nodes": info["chunk_nodes"], "variant": g.variant_names()[v],
           "waves_per_cu": st["waves_per_cu"],
           "device_load_s": round(load_s, 3), "host_load_s": round(host_load_s, 3),
           "batched_ms": round(batched_ms, 4), "batched_wall_ms": round(float(np.median(wms)), 4),
           "per_tree_ms": round(per_tree_ms, 3), "batched_speedup": round(per_tree_ms / batched_ms, 1),
           "equivalent_gpops": round(total * T / (batched_ms * 1e-3) / 1e9, 2),
           "roofline": {"bound": "alu", "kernel": "k_eval_" + ("bool" if vtype == g.GP_BOOL else "f32") + "_tbl",
                        "kernel_ms": round(kernel_ms, 4), "achieved": round(achieved / 1e12, 4),
                        "peak": round(PEAK_FP32_LANE_OPS / 1e12, 2), "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_FP32_LANE_OPS, 4), "traffic": None}}
    add_counted(out["roofline"], desc["workload"], info["chunk_nodes"], g.variant_names()[v], st["waves_per_cu"],
                kernel_ms)
    if vtype == g.GP_BOOL:
        out["roofline"]["unit"] = "Tbit-op/s"
        out["roofline"]["note"] = ("one 64-bit word operation per function node evaluates 64 cases; achieved counts "
                                   "function nodes x cases against the 32-bit lane-op issue rate")
    if not no_cpu:
        out["cpu_1core"] = oracle_full(pop, cases, pop.vtype, 1, cpu_budget_s, cpu, gpu_fit=fit)
        out["cpu_baseline"] = oracle_full(pop, cases, pop.vtype, threads, cpu_budget_s, cpu, gpu_fit=fit)
    ctx.free(ph)
    ctx.free(ch)
    out["bench_s"] = round(time.perf_counter() - t0, 1)
    log(f"[config] {desc['workload']}: {out}")
    return out


def oracle_stream(jobs, cases_of, threads, budget_s, cpu):
    """The oracle on the first jobs of the served stream (arrival order), as
    `threads` independent single-threaded instances taking jobs from a shared
    queue: a full job is the tree's evaluation and fitness, an incremental
    child the oracle's bottom-up evaluation with its mother co-evaluated."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    # about budget_s of work per thread at ~1e8 node-cases/s (the oracle's float rate on this host class);
    # a job that alone would take more than half of that on one thread is left out of the sample
    rate = 1.0e8
    target = budget_s * rate * threads
    chosen, skipped, tot = [], 0, 0
    for i, j in enumerate(jobs):
        if tot >= target:
            break
        n = len(j.ops) if j.kind == 0 else len(jobs[j.parent].ops) + len(j.ops)
        cost = n * (j.T if j.vtype == gen.VT_F32 else (j.T + 63) // 64)
        if cost > 0.5 * budget_s * rate:
            skipped += 1
            continue
        chosen.append(i)
        tot += cost

    def one(i):
        j = jobs[i]
        c = cases_of[(j.vtype, j.T)]
        if j.kind == 0:
            if j.vtype == gen.VT_BOOL:
                oracle.fitness_bool(oracle.eval_bool(j.ops, c.inputs), c.target, j.T)
            else:
                with np.errstate(all="ignore"):
                    oracle.fitness_f32(oracle.eval_f32(j.ops, c.x), c.y)
            return len(j.ops) * j.T
        P = jobs[j.parent].ops
        if j.vtype == gen.VT_BOOL:
            oracle.incremental_bool(P, j.point, j.ops, c.inputs, c.target, j.T)
        else:
            with np.errstate(all="ignore"):
                oracle.incremental_f32(P, j.point, j.ops, c.x, c.y)
        return (len(P) - (gen.subtree_end(P, j.point) - j.point) + len(j.ops)) * j.T

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        eq = sum(ex.map(one, sorted(chosen, key=lambda i: -len(jobs[i].ops))))
    dt = time.perf_counter() - t0
    return {"jobs_per_s": round(len(chosen) / dt, 2), "equivalent_gpops": round(eq / dt / 1e9, 3),
            "cores": threads, "kind": "oracle", "nproc": cpu["nproc"], "cpu_model": cpu["model"],
            "sample": f"{len(chosen)} of the first {len(chosen) + skipped} jobs of the stream in arrival order "
                      f"(left out: {skipped} jobs above {0.5 * budget_s * rate:.0e} node-cases), {dt:.1f} s"}


def serve_bench(ctx, g, n_jobs, threads, budget_gb=200.0, loads=(0.5, 0.8, 0.95), cpu=None, oracle_s=8.0,
                device_compile_nodes=0):
    """Served mixed stream: full jobs (kept resident as parents) and
    incremental children arriving over time; continuous batching in the
    library's server.  All jobs at once (saturation), then Poisson arrivals at
    the given fractions of the saturation rate.  Returns throughput, latency
    percentiles and where the latency goes."""
    t0 = time.perf_counter()
    jobs = gen.served_stream(5, n_jobs, threads=threads)
    log(f"[serve] generated {n_jobs} jobs in {time.perf_counter() - t0:.1f} s")
    handles, cases_of = {}, {}
    for j in jobs:
        key = (j.vtype, j.T)
        if key not in handles:
            if j.vtype == gen.VT_BOOL:
                bc = gen.bool_cases(j.T.bit_length() - 1)
                handles[key] = ctx.set_cases(g.GP_BOOL, bc.inputs, bc.target, j.T)
                cases_of[key] = bc
            else:
                fc = gen.float_cases(j.T, j.T)
                handles[key] = ctx.set_cases(g.GP_F32, fc.x, fc.y)
                cases_of[key] = fc
    equiv = np.zeros(len(jobs), np.int64)
    for i, j in enumerate(jobs):
        if j.kind == 0:
            equiv[i] = len(j.ops) * j.T
        else:
            p = jobs[j.parent].ops
            equiv[i] = (len(p) - (gen.subtree_end(p, j.point) - j.point) + len(j.ops)) * j.T
    base_mem = ctx.memory_used

    def run(rate):
        ctx.server_start(n_streams=4, max_batch_jobs=64, prep_threads=threads, budget_bytes=int(budget_gb * 2**30),
                         device_compile_nodes=device_compile_nodes)
        tickets = [0] * len(jobs)
        done = {}
        pending = []
        peak = [0]
        t_start = time.perf_counter()

        def sweep():
            peak[0] = max(peak[0], ctx.memory_used - base_mem)
            return [k for k in pending if not collect(k, done, tickets)]

        for i, j in enumerate(jobs):
            if rate:
                wait_s = j.arrival / rate - (time.perf_counter() - t_start)
                while wait_s > 0:
                    # collect finished jobs while waiting for the next arrival
                    pending = sweep()
                    wait_s = j.arrival / rate - (time.perf_counter() - t_start)
                    if wait_s > 0.0005:
                        time.sleep(min(wait_s, 0.0005))
            if j.kind == 0:
                tickets[i] = ctx.server_submit(g.GP_JOB_FULL, handles[(j.vtype, j.T)], j.ops,
                                               record_points=j.points, keep_resident=True)
            else:
                tickets[i] = ctx.server_submit(g.GP_JOB_INCREMENTAL, handles[(j.vtype, j.T)], j.ops,
                                               parent_ticket=tickets[j.parent], point=j.point)
            pending.append(i)
        while pending:
            pending = sweep()
            time.sleep(0.0002)
        wall = time.perf_counter() - t_start
        for i, j in enumerate(jobs):
            if j.kind == 0:
                ctx.server_release(tickets[i])
        ctx.server_stop()
        return done, wall, peak[0]

    def collect(i, done, tickets):
        j = jobs[i]
        r = ctx.server_poll(tickets[i], g.GP_BOOL if j.vtype == gen.VT_BOOL else g.GP_F32, j.T, want_root=False)
        if r is None:
            return False
        done[i] = r
        return True

    def summary(done, wall, peak):
        def pct(key, sel):
            v = np.array([done[i][key] for i, j in enumerate(jobs) if sel(j)])
            return {"mean": round(float(v.mean()), 3), "p50": round(float(np.percentile(v, 50)), 3),
                    "p99": round(float(np.percentile(v, 99)), 3)}
        lat = np.array([done[i]["latency_ms"] for i in range(len(jobs))])
        bad = sum(1 for r in done.values() if r["status"] != 0)
        full = [j.kind == 0 for j in jobs]
        return {"jobs": len(jobs), "failed": bad, "wall_s": round(wall, 3),
                "jobs_per_s": round(len(jobs) / wall, 1),
                "equivalent_gpops": round(float(equiv.sum()) / wall / 1e9, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "full_p50_ms": round(float(np.percentile(lat[full], 50)), 3),
                "full_p99_ms": round(float(np.percentile(lat[full], 99)), 3),
                "incremental_p50_ms": round(float(np.percentile(lat[~np.array(full)], 50)), 3),
                "incremental_p99_ms": round(float(np.percentile(lat[~np.array(full)], 99)), 3),
                # where a job's latency goes: prep threads (validate, compile), waiting for admission,
                # its batch's host work (assembly, upload, launches), device work and copy-out
                "split_ms": {k: pct(k, lambda j: True) for k in ("prep_ms", "queue_ms", "launch_ms", "run_ms")},
                "peak_device_gb": round(peak / 2**30, 2)}

    out = {"stream": f"{n_jobs} jobs, 30% full (resident parents, 3 recorded points) / 70% incremental; "
                     "10..1e7 nodes log-uniform; float32 or Boolean 50/50; 256..4096 cases; donors 1..1e4 nodes, "
                     "half neutral; budget 200 GB",
           "parent_nodes": int(sum(len(j.ops) for j in jobs if j.kind == 0))}
    done, wall, peak = run(None)
    out["saturation"] = summary(done, wall, peak)
    log(f"[serve] saturation: {out['saturation']}")
    for load in loads:
        rate = load * len(jobs) / wall / max(1e-9, jobs[-1].arrival / len(jobs))
        d2, w2, p2 = run(rate)
        out[f"poisson_{load:.2f}x"] = summary(d2, w2, p2)
        log(f"[serve] at {load:.2f} x saturation: {out[f'poisson_{load:.2f}x']}")
    for h in handles.values():
        ctx.free(h)
    if cpu is not None:
        out["cpu_baseline"] = oracle_stream(jobs, cases_of, threads, oracle_s, cpu)
        log(f"[serve] oracle on the stream: {out['cpu_baseline']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="incremental",
                    choices=["incremental", "full_large", "boolean", "small"])
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the population size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning-file", default="",
                    help="JSON lines of autotuner choices: loaded first when the file exists (the autotuner then "
                         "applies its choices without timing), written after the run")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip per-tree launches and the full re-evaluation of the built children")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the small, Boolean and large full-evaluation configurations")
    ap.add_argument("--cpu-budget", type=float, default=1.5,
                    help="seconds of oracle work per thread for each configuration's CPU baselines")
    # the host's CPU share for one GPU is 16 threads, whatever nproc shows
    ap.add_argument("--threads", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--serve-jobs", type=int, default=20000, help="served-stream jobs (0 = skip serving)")
    ap.add_argument("--serve-only", action="store_true", help="run the served stream alone")
    ap.add_argument("--serve-device-compile", type=int, default=0,
                    help="served full jobs of at least this many nodes compile on the device (0: none, the "
                         "library's default)")
    ap.add_argument("--generations", type=int, default=2, help="generations of the evolution leg (0 = skip)")
    ap.add_argument("--chunk-nodes", type=int, default=0, help="fix the chunk size (0 = automatic / tuned)")
    ap.add_argument("--variant", default="", help="fix the interpreter variant, e.g. f32_k4_s16")
    ap.add_argument("--waves-per-cu", type=int, default=-1,
                    help="cap the interpreter launch's resident waves per CU (0: all that fit; -1: tuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only run launches of known VALU instruction counts per class (reference for VALU counters)")
    args = ap.parse_args()
    if args.calibrate_valu:
        import torch
        from paper_2205_03251_amd import gpeval as g
        torch.cuda.init()
        ctx = g.Context(0)
        names = ["v_add_f32", "v_mul_f32", "v_fma_f32", "v_rcp_f32", "v_cndmask_b32", "v_cmp_lt_f32",
                 "v_max3_f32", "v_mov_b32", "v_add_f32+v_rcp_f32", "v_add_f32+v_cmp_lt_f32"]
        waves, iters = 256 * 4 * 8, 4000        # eight waves per SIMD; 128000 VALU instructions per wave
        res = []
        for cls, name in enumerate(names):
            ctx.valu_calibration(cls, waves, 0)
            t0 = min(ctx.valu_calibration(cls, waves, 0) for _ in range(3))
            t1 = min(ctx.valu_calibration(cls, waves, iters) for _ in range(3))
            n = waves * 32 * iters
            rate = n * 64 / ((t1 - t0) * 1e-3)
            res.append({"class": cls, "instructions": name, "waves": waves, "valu_per_wave_loop": 32 * iters,
                        "ms": round(t1, 4), "ms_iters0": round(t0, 4), "lane_ops_per_s": rate,
                        "frac_of_peak": round(rate / PEAK_FP32_LANE_OPS, 4),
                        "instr_per_simd_cycle": round(n / 1024 / ((t1 - t0) * 1e-3 * 2.4e9), 4)})
            log(f"[calibrate] {res[-1]}")
        print(json.dumps({"valu_calibration": res}))
        ctx.close()
        return
    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 3}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the evaluation path is not "
                                   "sharded across GPUs",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2205_03251_amd import gpeval as g

    if args.serve_only:
        torch.cuda.init()
        ctx = g.Context(0)
        hc = host_cpu()
        res = serve_bench(ctx, g, args.serve_jobs, args.threads, cpu=None if args.no_cpu_baseline else hc,
                          device_compile_nodes=args.serve_device_compile)
        print(json.dumps({"serving": res, "host_cpu": hc}), flush=True)
        ctx.close()
        return

    t0 = time.perf_counter()
    pop, cases, kids, desc = workload_inputs(args.workload, args.scale, args.threads)
    vtype = g.GP_BOOL if desc["value_type"] == "bool" else g.GP_F32
    T = cases.T
    gen_s = time.perf_counter() - t0
    log(f"[bench] generated {desc['workload']}: {pop.n_trees} trees, {int(pop.sizes().sum())} nodes "
        f"in {gen_s:.1f} s")

    torch.cuda.init()
    ctx = g.Context(0)
    if args.tuning_file and os.path.exists(args.tuning_file):
        ctx.tuning_load(args.tuning_file)
    if vtype == g.GP_BOOL:
        ch = ctx.set_cases(g.GP_BOOL, cases.inputs, cases.target, T)
    else:
        ch = ctx.set_cases(g.GP_F32, cases.x, cases.y)
    if kids is not None:
        rp, ro = record_lists(pop.n_trees, kids)
        ph, load_s, host_load_s = load_timed(ctx, vtype, pop, host=not args.no_compare, record_points=rp,
                                             record_offsets=ro, chunk_nodes=args.chunk_nodes, keep_trees=True)
    else:
        ph, load_s, host_load_s = load_timed(ctx, vtype, pop, host=not args.no_compare,
                                             chunk_nodes=args.chunk_nodes)
    info = ctx.population_info(ph)
    log(f"[bench] loaded in {load_s:.2f} s compiled on the device ({host_load_s} s on the host): {info}")

    tuned = None
    if args.waves_per_cu >= 0:
        ctx.set_launch_width(args.waves_per_cu)
    if args.variant:
        ctx.set_variant(g.variant_names().index(args.variant))
        tuned = args.variant
    elif not args.no_autotune:
        v, ms = ctx.autotune(ph, ch)
        tuned = g.variant_names()[v]
        log(f"[bench] autotune picked {tuned} ({ms:.2f} ms per full evaluation)")

    final_info = ctx.population_info(ph)
    n_trees = pop.n_trees
    fdt = torch.float64 if vtype == g.GP_F32 else torch.int64
    fit_buf = torch.empty(n_trees, dtype=fdt, device="cuda:0")
    total_nodes = int(pop.sizes().sum())

    used = {}

    def step():
        _, _, st_full = ctx.evaluate_full(ph, ch, vtype, n_trees, T, roots=False, device=True, async_=True,
                                          fit_buf=fit_buf)
        used["variant"] = g.variant_names()[st_full["variant"]]
        used["waves_per_cu"] = st_full["waves_per_cu"]
        if kids is None:
            return st_full, None
        _, _, st_inc = ctx.evaluate_incremental(ph, ch, vtype, T, kids.parent, kids.point, kids.donors.ops,
                                                kids.donors.offsets, roots=False, device=True)
        return st_full, st_inc

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    inc_stats = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        _, inc_stats = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed / args.steps * 1e3

    # host copies of the results, for comparison with the oracle's samples
    _, gfit, _ = ctx.evaluate_full(ph, ch, vtype, n_trees, T, roots=False)
    inc_fit = None
    if kids is not None:
        _, inc_fit, _ = ctx.evaluate_incremental(ph, ch, vtype, T, kids.parent, kids.point, kids.donors.ops,
                                                 kids.donors.offsets, roots=False)

    equiv_nodes = total_nodes
    interp_nodes = total_nodes
    extra = {}
    if kids is not None:
        child_nodes = int(inc_stats["child_nodes"].sum())
        equiv_nodes += child_nodes
        interp_nodes += int(inc_stats["interpreted_nodes"].sum())
        stops = inc_stats["stop_level"]
        extra["incremental"] = {
            "children": int(len(stops)), "child_nodes": child_nodes,
            "interpreted_nodes": int(inc_stats["interpreted_nodes"].sum()),
            "stop_at_point": int((stops == 0).sum()), "reached_root": int((stops < 0).sum()),
            "median_stop_level": float(np.median(stops[stops >= 0])) if (stops >= 0).any() else None,
            "device_ms": inc_stats["device_ms"],
            "equivalent_gpops": child_nodes * T / (inc_stats["device_ms"] * 1e-3) / 1e9,
            "interpreted_gpops": int(inc_stats["interpreted_nodes"].sum()) * T / (inc_stats["device_ms"] * 1e-3) / 1e9,
        }

    # dominant kernel: the interpreter launch, timed with HIP events on the library stream
    kms = []
    for _ in range(3):
        _, _, st = ctx.evaluate_full(ph, ch, vtype, n_trees, T, roots=False, graph=False)
        kms.append(st["kernel_ms"])
    kernel_ms = float(np.median(kms))
    func_nodes = (total_nodes - n_trees) // 2
    achieved = func_nodes * T / (kernel_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_FP32_LANE_OPS / 1e12, 2),
                "unit": "TFLOP/s", "frac": round(achieved * 1e12 / PEAK_FP32_LANE_OPS, 4), "traffic": None,
                "kernel": "k_eval_" + ("bool" if vtype == g.GP_BOOL else "f32") + "_tbl", "kernel_ms": round(kernel_ms, 3),
                "gp_ops_per_s": round(total_nodes * T / (kernel_ms * 1e-3) / 1e12, 4),
                "peak_note": "256 CU x 4 SIMD x 32 lane-ops/cycle x 2.4 GHz: the published 157.3 TFLOP/s counts an FMA as "
                             "two flops; + - x / are one op per lane at the same issue rate. achieved = function nodes "
                             "x cases / interpreter launch time (terminals excluded)"}
    if vtype == g.GP_BOOL:
        roofline["note"] = "Boolean: one 64-bit word op per function node per 64 cases"
    # HBM bytes from the committed counter runs, valid only for the kernel source they were taken with
    counted = add_counted(roofline, desc["workload"], final_info["chunk_nodes"], used.get("variant", tuned),
                          used.get("waves_per_cu", 0), kernel_ms)

    # the paper's own incremental form: the mother co-evaluated alongside each child (no parent caches)
    if kids is not None:
        co = []
        for _ in range(2):
            _, _, st_co = ctx.evaluate_incremental(ph, ch, vtype, T, kids.parent, kids.point, kids.donors.ops,
                                                   kids.donors.offsets, roots=False, device=True, coeval=True)
            co.append(st_co)
        st_co = co[-1]
        cn = int(st_co["child_nodes"].sum())
        ci = int(st_co["interpreted_nodes"].sum())
        extra["incremental_coeval"] = {
            "children": int(len(kids.parent)), "wall_ms": round(st_co["wall_ms"], 3),
            "device_ms": round(st_co["device_ms"], 3), "launches": int(st_co["launches"]),
            "interpreted_nodes": ci, "equivalent_gpops": round(cn * T / (st_co["wall_ms"] * 1e-3) / 1e9, 1),
            "interpreted_gpops": round(ci * T / (st_co["wall_ms"] * 1e-3) / 1e9, 1),
            "same_stop_levels_as_cached": bool(np.array_equal(st_co["stop_level"], inc_stats["stop_level"]))}

    # children built on the device (memory-bound copy kernel): 2 x bytes of HBM traffic
    child_ops = None
    if kids is not None:
        sms = []
        for _ in range(5):
            child_ops, child_offs, sst = ctx.splice_children(ph, kids.parent, kids.point, kids.donors.ops,
                                                             kids.donors.offsets, device=True, out=child_ops)
            sms.append(sst["kernel_ms"])
        sbytes = int(child_offs[-1])
        skms = float(np.median(sms[1:]))
        gbps = 2 * sbytes / (skms * 1e-3) / 1e9
        # reference: torch's own device-to-device copy of the same byte count
        src = torch.empty(sbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cms = []
        for _ in range(5):
            ev0.record()
            dst.copy_(src)
            ev1.record()
            torch.cuda.synchronize()
            cms.append(ev0.elapsed_time(ev1))
        del src, dst
        copy_gbps = 2 * sbytes / (float(np.median(cms[1:])) * 1e-3) / 1e9
        extra["splice"] = {"children": int(len(kids.parent)), "bytes": sbytes, "kernel": "k_splice",
                           "kernel_ms": round(skms, 4), "bound": "hbm", "achieved": round(gbps, 1),
                           "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": round(gbps / PEAK_HBM_GBPS, 4),
                           "algorithmic_bytes": 2 * sbytes, "device_copy_same_bytes_GBps": round(copy_gbps, 1),
                           "traffic": None}
        if counted is not None and "splice" in counted:
            extra["splice"]["traffic"] = int(counted["splice"]["fetch_bytes_per_launch"] +
                                             counted["splice"]["write_bytes_per_launch"])

    # the first steps of loading, on the device: validity, subtree ends and parents of every node
    if total_nodes <= 2**31 - 2:
        dops = torch.from_numpy(pop.ops).to("cuda:0")
        doffs = torch.from_numpy(pop.offsets).to("cuda:0")
        ims = []
        for _ in range(3):
            valid, iend, ipar, ims_one = ctx.index_trees(dops, doffs, pop.n_inputs)
            ims.append(ims_one)
        all_valid = bool((valid == 1).all())
        del valid, iend, ipar
        _, _, _, isn, ims_sn = ctx.index_trees(dops, doffs, pop.n_inputs, strahler=True)
        max_sn = int(isn.max())
        del dops, doffs, isn
        ix_ms = float(np.median(ims[1:]))
        ix_bytes = 9 * total_nodes          # each node's byte read, its end and parent (int32) written
        ix_gbps = ix_bytes / (ix_ms * 1e-3) / 1e9
        extra["tree_index"] = {"trees": n_trees, "nodes": total_nodes, "device_ms": round(ix_ms, 3),
                               "nodes_per_s": round(total_nodes / (ix_ms * 1e-3), 1), "bound": "hbm",
                               "achieved": round(ix_gbps, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                               "frac": round(ix_gbps / PEAK_HBM_GBPS, 4), "algorithmic_bytes": ix_bytes,
                               "all_valid": all_valid, "with_strahler_ms": round(ims_sn, 3),
                               "max_strahler": max_sn}

    # the two legs of the step, each timed on its own (HIP events on the library stream)
    bms = [ctx.evaluate_full(ph, ch, vtype, n_trees, T, roots=False, device=True, fit_buf=fit_buf)[2]["device_ms"]
           for _ in range(5)]
    batched_ms = float(np.median(bms))
    legs = {"parents_full_evaluation": {"trees": n_trees, "nodes": total_nodes, "device_ms": round(batched_ms, 3),
                                        "equivalent_gpops": round(total_nodes * T / (batched_ms * 1e-3) / 1e9, 1)}}
    if kids is not None:
        legs["children_incremental"] = {
            "children": int(len(kids.parent)), "nodes": int(inc_stats["child_nodes"].sum()),
            "device_ms": round(inc_stats["device_ms"], 3),
            "equivalent_gpops": round(extra["incremental"]["equivalent_gpops"], 1),
            "interpreted_gpops": round(extra["incremental"]["interpreted_gpops"], 1)}
    extra["legs"] = legs
    if not args.no_compare:
        log("[bench] one launch per tree ...")
        _, _, st_pt = ctx.evaluate_full(ph, ch, vtype, n_trees, T, roots=False, per_tree=True, graph=False)
        extra["compare"] = {"batched_launch_ms": round(batched_ms, 3), "per_tree_launch_ms": round(st_pt["device_ms"], 3),
                            "batched_speedup": round(st_pt["device_ms"] / batched_ms, 1)}
        if kids is not None:
            log("[bench] full re-evaluation of the built children ...")
            n_kids = len(child_offs) - 1
            t_c = time.perf_counter()
            c_host = child_ops.cpu().numpy()
            hph = ctx.load_population(vtype, c_host, child_offs, n_inputs=pop.n_inputs)
            c_host_load_s = time.perf_counter() - t_c
            ctx.free(hph)
            del c_host
            # the children as the splice left them, in device memory, compiled there
            torch.cuda.synchronize()
            t_c = time.perf_counter()
            cph = ctx.load_population(vtype, child_ops, torch.from_numpy(child_offs).to("cuda:0"),
                                      n_inputs=pop.n_inputs)
            c_load_s = time.perf_counter() - t_c
            ctx.autotune(cph, ch)
            rms = [ctx.evaluate_full(cph, ch, vtype, n_kids, T, roots=False)[2]["device_ms"] for _ in range(3)]
            reeval_ms = float(np.median(rms))
            inc_ms = inc_stats["device_ms"]
            extra["compare"].update({
                "children_full_reeval_ms": round(reeval_ms, 3), "children_incremental_ms": round(inc_ms, 3),
                "incremental_speedup": round(reeval_ms / inc_ms, 1), "children_device_load_s": round(c_load_s, 2),
                "children_host_load_s": round(c_host_load_s, 2),
                "children_full_reeval_gpops": round(int(child_offs[-1]) * T / (reeval_ms * 1e-3) / 1e9, 1)})
            ctx.free(cph)
    del child_ops

    # generations with fitness first (tournaments of 7, the paper's size): children scored by
    # co-evaluation, only those drawn by the next generation's tournaments built and compiled
    if kids is not None and args.generations > 0:
        nh, gstats, _ = ctx.evolve(ph, ch, args.generations, 7, 2022)
        extra["evolve"] = {
            "generations": args.generations, "tournament": 7, "population": n_trees,
            "ms_per_generation": [round(x["ms"], 1) for x in gstats],
            "ms_score_build_eval": [[round(x["ms_score"], 1), round(x["ms_build"], 1), round(x["ms_eval"], 1)]
                                    for x in gstats],
            "built_fraction": [round(x["built"] / x["children"], 4) for x in gstats],
            "chunks_evaluated_of_built": [[int(x["chunks_evaluated"]), int(x["chunks"])] for x in gstats],
            "child_nodes": [int(x["child_nodes"]) for x in gstats],
            "interpreted_nodes": [int(x["interpreted_nodes"]) for x in gstats],
            "best_error": [x["best_f64"] if vtype == g.GP_F32 else int(x["best_i64"]) for x in gstats],
            "note": "the last generation builds all children; building includes the children's programs, made "
                    "from their parents' chunks; evaluating them runs only the chunks compiled anew, the reused ones "
                    "take their parents' values"}
        ctx.free(nh)

    serving = None
    if args.serve_jobs > 0:
        ctx.free(ph)
        serving = serve_bench(ctx, g, args.serve_jobs, args.threads,
                              cpu=None if args.no_cpu_baseline else host_cpu(),
                              device_compile_nodes=args.serve_device_compile)

    hostcpu = host_cpu()
    configs = None
    if not args.no_configs and args.workload == "incremental":
        configs = {}
        for name, key in (("small", "small_ramped"), ("boolean", "boolean_parity6"), ("full_large", "full_large")):
            log(f"[bench] configuration {key} ...")
            configs[key] = measure_config(ctx, g, name, args.threads, hostcpu, args.cpu_budget, args.no_cpu_baseline)
    if args.tuning_file:
        ctx.tuning_save(args.tuning_file)

    cpu = cpu1 = cpu_inc = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on bounded samples ...")
        cpu = oracle_full(pop, cases, pop.vtype, args.threads, 10.0, hostcpu, gpu_fit=gfit)
        cpu1 = oracle_full(pop, cases, pop.vtype, 1, 8.0, hostcpu, gpu_fit=gfit)
        if kids is not None:
            cpu_inc = oracle_incremental(pop, cases, kids, args.threads, hostcpu, gpu_fit=inc_fit,
                                         gpu_stop=inc_stats["stop_level"])

    value = equiv_nodes * T / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "equivalent GPop/s (tree nodes x test cases per second)",
        "value": round(value, 3),
        "unit": "GPop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bool" if vtype == g.GP_BOOL else "f32",
        "data": "synthetic",
        "config": {**desc, "chunk_nodes": final_info["chunk_nodes"], "variant": used.get("variant", tuned),
                   "waves_per_cu": used.get("waves_per_cu", 0), "parallelism": "single_gpu"},
        "interpreted_gpops": round(interp_nodes * T / (ms_per_step * 1e-3) / 1e9, 3),
        "load": {"device_compile_s": round(load_s, 2),
                 "host_compile_s": None if host_load_s is None else round(host_load_s, 2),
                 "note": "loading the parents: validation, compilation into chunked programs and upload, on the "
                         "device (the population benchmarked) and on the host (the same programs, timed and "
                         "freed)"},
        "value_note": "equivalent GPop/s of the whole step: (parent nodes + child nodes) x cases / step time; the "
                      "two legs' own rates are under legs",
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_1core": cpu1,
        "cpu_incremental": cpu_inc,
        "host_cpu": hostcpu,
        **extra,
        "configs": configs,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
