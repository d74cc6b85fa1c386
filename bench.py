"""Benchmark: mixed-monotonicity embedding RK4 on MI355X.

Workload (one timed "step" = one whole reach_embed_rk4 call): the 1-D
reaction-diffusion chain, n = 2^26 cells, FP64, interval input u in
[-0.1, 0.1], seeded box of width U(0, 0.02) around the first Dirichlet sine
mode, dt = 0.1, 1000 RK4 steps.  Inputs are generated on the host, copied to
HBM, and are resident before the timed region.

Prints ONE JSON line with the throughput (state-steps/s, a state being one of
the 2n lower/upper components), the roofline of the dominant kernel measured
live with HIP events, the K = 1 streaming HBM fraction, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12          # FLOP/s, MI355X FP64 vector (FMA = 2 flops)
FP32_PEAK = 157.3e12         # FLOP/s, MI355X FP32 vector (published, packed)
# VALU lane-instruction issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (a wave64 vector instruction occupies a SIMD for four cycles)
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic FP64 operations of one RK4 state-step of the RD chain (an FMA
# counts 2): four right-hand sides of 8 (two adds, a scaling by 1/h^2, 2*y,
# y^3 as two products, the input and the reaction term), three stage inputs
# z + c K of 2, the weighted sum K1 + 2K2 + 2K3 + K4 of 5 and z + dt/6 * sum of 2.
RD_FLOPS_PER_STATE_STEP = 45
# The same count for the CTM chain: per right-hand side one flux (v*y, c - y,
# w*(c - y), two minimum operations) and its difference with the neighbour's,
# 6; plus 13 for the stage inputs and the update.
CTM_OPS_PER_STATE_STEP = 37
# 3-D heat: per stencil application 5 adds, one FMA and one multiply (8),
# plus the update FMA (2), four applications per RK4 step (the step's
# stability polynomial in nested form).  One pass = one step: 8 B read + 8 B
# written.
HEAT_OPS_PER_CELL_STEP = 40
HEAT_BYTES_PER_CELL_STEP = 16


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the kernel sources a PMC summary is tied to (the pass structs in kernels.hpp
# change with the kernels that read them)
EMBED_SOURCES = ("dev.hpp", "embed.hip")
HEAT_SOURCES = ("dev.hpp", "heat3d.hip")
# the packed batch's kernel sources (its instruction count also follows the
# planner's packing, whose changes call for a new summary)
BATCH_SOURCES = ("dev.hpp", "batch.hip")
MC_SOURCES = ("dev.hpp", "mc.hip")
# FP64 VALU instructions of one state-step's arithmetic in the batch kernels
# (per cell and stage: RD 4, CTM 5 for the right-hand side; the RK4 updates
# 1 + 2 + 2 + 2 over the four stages)
USEFUL_VALU_PER_STATE_STEP = {2: 23, 1: 27}


def source_hash(files=EMBED_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2001_10635_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_value(name, key, files=EMBED_SOURCES):
    """A figure of a committed PMC summary, if the summary was taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash(files):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def traffic_from_profile(name="embed_tile_kernel_rd2p26_f64_pmc.txt", files=EMBED_SOURCES):
    """HBM bytes per launch from a committed PMC summary (None if stale)."""
    return profile_value(name, "hbm_bytes_per_launch", files)


def hbm_probe(R, torch, n, stream, reps=3):
    """The HBM ceiling for one embedding pass's traffic: the project's stream
    kernel (libreach_probe.so) copying two arrays of n doubles into two, over
    its launch shapes (16-byte vectors in flight per thread, non-temporal or
    not, grid size); the fastest shape, timed as the fastest of `reps` calls."""
    P = R.probe_lib()
    a = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    nbytes = 8 * n
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sp = stream.cuda_stream
    best, table = None, []
    for unroll in (1, 2, 4, 8):
        for nt in (0, 1):
            for blocks in (cus * 4, cus * 8, cus * 16, cus * 32, -(-nbytes // (16 * 256 * unroll))):
                args = (a.data_ptr(), a.data_ptr() + nbytes, b.data_ptr(), b.data_ptr() + nbytes,
                        nbytes, unroll, nt, int(blocks), sp)
                assert P.reach_probe_stream2(*args) == 0
                t = None
                for _ in range(reps):
                    ev0.record(stream)
                    P.reach_probe_stream2(*args)
                    ev1.record(stream)
                    ev1.synchronize()
                    dt = ev0.elapsed_time(ev1) / 1e3
                    t = dt if t is None else min(t, dt)
                table.append((unroll, nt, int(blocks), t))
                if best is None or t < best[3]:
                    best = (unroll, nt, int(blocks), t)
    ok = bool(torch.equal(a, b))
    del a, b
    gbps = 4.0 * nbytes / best[3] / 1e9
    return {"kernel": "stream2_kernel (libreach_probe.so)", "unroll": best[0],
            "nontemporal": bool(best[1]), "blocks": best[2], "us": round(best[3] * 1e6, 1),
            "GBps": round(gbps, 1), "frac": round(gbps * 1e9 / HBM_PEAK, 4),
            "copy_correct": ok, "shapes_timed": len(table)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, steps: int):
    """The oracle on the host: all threads on the full chain for `steps` of
    the workload's steps, and one thread on its first 2^20 cells."""
    import oracle
    lo, hi = p.box()
    pl, ph = p.inputs()
    threads = oracle.get_threads()
    t = time.perf_counter()
    oracle.embed_rk4(p.kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=steps)
    el = time.perf_counter() - t
    n1, s1 = min(p.n, 1 << 20), 10
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        oracle.embed_rk4(p.kind, p.prm, lo[:n1], hi[:n1], pl, ph, dt=p.dt, nsteps=s1)
        el1 = time.perf_counter() - t
    finally:
        oracle.set_threads(threads)
    return {"value": 2.0 * p.n * steps / el, "unit": "state-steps/s", "cores": threads,
            "kind": "oracle", "seconds": round(el, 2), "cpu_model": cpu_model(),
            "sample": f"FP64 oracle on the full {p.n}-cell chain for {steps} of the "
                      f"{p.nsteps} RK4 steps (same box, inputs and dt)",
            "one_thread": {"value": 2.0 * n1 * s1 / el1, "unit": "state-steps/s",
                           "sample": f"first {n1} cells, {s1} steps"}}


def latency_ctm64(rc, R, torch, workloads, reps=1000, cpu=True):
    """The 64-cell CTM chain (FP64, 100 steps) and its 1000-sample Monte Carlo:
    microseconds per call, HIP events around `reps` back-to-back calls."""
    p = workloads.ctm64_f64()
    lo, hi = p.box()
    x_lo, x_hi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    r_lo, r_hi = torch.empty_like(x_lo), torch.empty_like(x_hi)
    sysd = R.make_system(p.kind, p.n, p.prm, 0)
    run = lambda: R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, None, None, 0.0,
                                    p.dt, p.nsteps, r_lo, r_hi, None, 0, None)
    for _ in range(10):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    emb_us = e0.elapsed_time(e1) * 1e3 / reps
    rc.montecarlo(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, p.m, p.seed)
    torch.cuda.synchronize()
    mc_reps = reps
    e0.record()
    for _ in range(mc_reps):
        rc.montecarlo(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, p.m, p.seed)
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    mc_us = e0.elapsed_time(e1) * 1e3 / mc_reps
    out = {"workload": "CTM chain n=64 FP64, dt=0.01, 100 RK4 steps; Monte Carlo m=1000",
           "embed_us_per_call": round(emb_us, 2), "mc_us_per_call": round(mc_us, 2),
           "reps": reps, "mc_reps": mc_reps}
    if cpu:
        import oracle
        threads = oracle.get_threads()
        oracle.set_threads(1)
        try:
            k = 200
            t = time.perf_counter()
            for _ in range(k):
                oracle.embed_rk4(p.kind, p.prm, lo, hi, dt=p.dt, nsteps=p.nsteps)
            out["cpu_oracle_us_per_call_1_thread"] = round((time.perf_counter() - t) * 1e6 / k, 1)
        finally:
            oracle.set_threads(threads)
    return out


def query_mix(rc, R, torch, workloads, nq, cpu=True):
    """A Poisson stream of nq CTM / RD queries at 5e4/s, n log-uniform
    in [4, 512], 10-1000 RK4 steps, FP64.  Offline: one persistent-kernel batch
    vs one launch per query.  Online: served with the persistent kernel vs
    one launch per query, p50 / p99 from arrival to result on the host."""
    p4 = workloads.serve_mix_f64()
    qs = workloads.query_stream(nq, p4.extra["rate"], seed=p4.seed)
    ns = np.array([q.problem.n for q in qs])
    offs = np.concatenate([[0], np.cumsum(ns)])
    tot = int(offs[-1])
    h_lo = np.empty(tot)
    h_hi = np.empty(tot)
    u_lo = np.zeros(nq)
    u_hi = np.zeros(nq)
    for i, q in enumerate(qs):
        pr = q.problem
        pr.box(out=(h_lo[offs[i]:offs[i + 1]], h_hi[offs[i]:offs[i + 1]]))
        if pr.n_in:
            u_lo[i], u_hi[i] = pr.p_lo[0], pr.p_hi[0]
    state_steps = float(np.sum(2.0 * ns * np.array([q.problem.nsteps for q in qs])))
    log(f"query mix: {nq} queries, {tot} cells, {state_steps:.3e} state-steps")
    dev = torch.device("cuda", 0)
    d_lo = torch.from_numpy(h_lo).to(dev)
    d_hi = torch.from_numpy(h_hi).to(dev)
    d_u = torch.from_numpy(np.stack([u_lo, u_hi], 1).reshape(-1)).to(dev)
    r_lo = torch.empty_like(d_lo)
    r_hi = torch.empty_like(d_hi)

    def qstruct(i, base_lo, base_hi, out_lo, out_hi, ulo, uhi, el=8):
        pr = qs[i].problem
        return R.make_query(pr.kind, pr.n, pr.prm, R.REACH_F64, base_lo + el * offs[i],
                            base_hi + el * offs[i], out_lo + el * offs[i], out_hi + el * offs[i],
                            pr.dt, pr.nsteps, (ulo(i) if pr.n_in else None),
                            (uhi(i) if pr.n_in else None), n_in=pr.n_in)

    dq = R.query_array([qstruct(i, d_lo.data_ptr(), d_hi.data_ptr(), r_lo.data_ptr(),
                                r_hi.data_ptr(), lambda i: d_u.data_ptr() + 16 * i,
                                lambda i: d_u.data_ptr() + 16 * i + 8) for i in range(nq)])
    nbw = R.reach_batch_workspace_bytes(nq)
    wsb = torch.empty(nbw, dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream()
    out = {"workload": f"{nq} queries, Poisson 5e4/s, CTM/RD, n log-uniform [4,512], "
                       f"10-1000 RK4 steps, FP64", "state_steps": state_steps}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        t = time.perf_counter()
        tune = R.reach_autotune_batch(rc.ctx, dq, wsb, nbw, s)  # pack widths, waves
        t_tune = time.perf_counter() - t
        R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, s)        # capture + first replay
        s.synchronize()
        # five whole batches, each timed on its own (host planning, upload and
        # kernel); the median is reported
        runs = []
        for _ in range(5):
            t = time.perf_counter()
            ev0.record(s)
            R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, s)
            ev1.record(s)
            s.synchronize()
            runs.append((time.perf_counter() - t, ev0.elapsed_time(ev1) / 1e3))
        runs.sort()
        tb, gpu_s = runs[len(runs) // 2]
        ref_one = r_lo.cpu().numpy()
        # the same batch issued back to back (a client with a stream of
        # batches): each call plans and uploads while the previous batch's
        # kernel runs; 3 untimed, then 10 timed from the first call to the
        # last kernel's end
        for _ in range(3):
            R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, s)
        s.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, s)
        s.synchronize()
        t_b2b = (time.perf_counter() - t) / 10
    assert rc.sync(s) == R.REACH_OK
    assert np.array_equal(r_lo.cpu().numpy(), ref_one)
    plan = R.reach_plan_batch(rc.ctx, dq, with_E=True)
    kinds = np.array([q.problem.kind for q in qs])
    steps = np.array([q.problem.nsteps for q in qs])
    slots = sum((64 * E if E else 64 * -(-ns[it[0]] // 64)) *
                int(max(steps[i] for i in it)) for E, it in plan)
    lanes = [sum(-(-int(ns[i]) // E) for i in it) for E, it in plan if E]
    useful = float(sum(2.0 * ns[kinds == k] @ steps[kinds == k] * c
                       for k, c in USEFUL_VALU_PER_STATE_STEP.items()))
    valu = profile_value("pack_kernel_mix1e5_f64_pmc.txt", "valu_wave_instructions_per_batch",
                         BATCH_SOURCES)
    out["batch_plan"] = {"items": len(plan), "packs": len(lanes),
                         "items_by_E": {str(e): int(sum(1 for E, _ in plan if E == e))
                                        for e in sorted({E for E, _ in plan})},
                         "mean_lanes_per_pack": round(float(np.mean(lanes)), 2) if lanes else None,
                         "cell_step_slots_used": round(float(ns @ steps) / slots, 4),
                         "autotune": tune, "autotune_s": round(t_tune, 3),
                         # useful FP64 lane-instructions over the issued ones
                         # (rocprof SQ_INSTS_VALU of the committed summary, taken
                         # on the current batch sources)
                         "useful_valu_lane_frac": (round(useful / (valu * 64), 4)
                                                   if valu else None)}
    ref_lo = r_lo.cpu().numpy()
    t = time.perf_counter()
    R.reach_embed_rk4_each(rc.ctx, dq, 8)
    te = time.perf_counter() - t
    assert rc.sync() == R.REACH_OK
    same = bool(np.array_equal(r_lo.cpu().numpy(), ref_lo))
    # the kernel's own duration is the committed trace summary's (the events
    # around the call also hold the host's planning, during which the device
    # waits)
    k_us = profile_value("pack_kernel_mix1e5_f64_trace.txt", "last_launch_us", BATCH_SOURCES)
    out["batch"] = {"queries_per_s": nq / tb, "seconds": round(tb, 4),
                    "seconds_min_max_of_5": [round(runs[0][0], 5), round(runs[-1][0], 5)],
                    "state_steps_per_s": state_steps / tb,
                    "call_gpu_seconds": round(gpu_s, 5),
                    "profiled_kernel_us": k_us,
                    "valu_issue_frac_of_profiled_kernel": (
                        round(valu * 64 / (k_us * 1e-6) / VALU_LANE_PEAK, 4)
                        if valu and k_us else None),
                    # the same launch in GPU cycles (GRBM_COUNT of the PMC
                    # summary): wave-instructions per CU-cycle, the launch at
                    # the 2.4 GHz peak clock, and the clock the GPU ran at
                    "valu_issue_per_cu_cycle": profile_value(
                        "pack_kernel_mix1e5_f64_pmc.txt", "valu_issue_per_cu_cycle", BATCH_SOURCES),
                    "profiled_kernel_us_at_2p4_ghz": profile_value(
                        "pack_kernel_mix1e5_f64_pmc.txt", "launch_us_at_2.4_ghz", BATCH_SOURCES),
                    "profiled_gpu_clock_ghz": profile_value(
                        "pack_kernel_mix1e5_f64_pmc.txt", "gpu_clock_ghz_in_this_run",
                        BATCH_SOURCES),
                    "back_to_back": {
                        "batches": 10, "seconds_per_batch": round(t_b2b, 5),
                        "queries_per_s": nq / t_b2b,
                        # the kernel when batches follow each other (committed
                        # summary on the current batch sources)
                        "profiled_kernel_us": profile_value(
                            "pack_kernel_mix1e5_f64_back_to_back.txt",
                            "back_to_back_launch_us_mean", BATCH_SOURCES),
                        "profiled_gpu_clock_ghz": profile_value(
                            "pack_kernel_mix1e5_f64_back_to_back.txt", "pmc_gpu_clock_ghz_mean",
                            BATCH_SOURCES)}}
    out["one_launch_per_query"] = {"queries_per_s": nq / te, "seconds": round(te, 4)}
    out["batch_speedup"] = round(te / tb, 2)
    out["batch_equals_per_query"] = same
    log(f"batch {out['batch']}, per-query launches {out['one_launch_per_query']}")
    del d_lo, d_hi, r_lo, r_hi, wsb

    # online: host arrays, Poisson arrivals; each query is submitted at its
    # scheduled arrival (or as soon after it as the client gets to it) and its
    # latency counts from the scheduled arrival to its box in host memory
    o_lo = np.empty(tot)
    o_hi = np.empty(tot)
    hq = [qstruct(i, h_lo.ctypes.data, h_hi.ctypes.data, o_lo.ctypes.data, o_hi.ctypes.data,
                  lambda i: u_lo.ctypes.data + 8 * i, lambda i: u_hi.ctypes.data + 8 * i)
          for i in range(nq)]
    arrivals = np.array([q.arrival for q in qs])
    pool = torch.empty(256 << 20, dtype=torch.uint8, device=dev)

    def serve(mode, count, rate_scale):
        rc.set_option("serve.mode", mode)
        o_lo.fill(np.nan)
        sched = arrivals[:count] * rate_scale
        R.reach_server_start(rc.ctx, pool, pool.numel(), 1024)
        tickets = []
        lag = longest = 0.0
        t_lib = R.reach_clock_us()
        t0 = time.perf_counter()
        i = 0
        while i < count:
            now = time.perf_counter() - t0
            while i < count and sched[i] <= now:
                ts = time.perf_counter()
                tickets.append(R.reach_submit_at(rc.ctx, hq[i], t_lib + sched[i] * 1e6))
                te = time.perf_counter()
                lag = max(lag, ts - t0 - sched[i])
                longest = max(longest, te - ts)
                i += 1
        pending = tickets
        while pending:
            nxt = []
            for tk in pending:
                st, res = R.reach_poll(rc.ctx, tk)
                if st == R.REACH_PENDING:
                    nxt.append(tk)
                else:
                    assert res == R.REACH_OK
            pending = nxt
        wall = time.perf_counter() - t0
        stats = R.reach_server_stats(rc.ctx)
        R.reach_server_stop(rc.ctx)
        offered = count / sched[count - 1] if count > 1 else float("nan")
        same = bool(np.array_equal(o_lo[:offs[count]], ref_lo[:offs[count]]))
        # every box was in host memory by the last arrival plus the largest
        # latency (the server's stamps); the client's own wall time also holds
        # its final poll over every ticket
        done_by = sched[count - 1] + stats["max_us"] * 1e-6
        return {"queries": count, "offered_per_s": round(offered, 1),
                "queries_per_s": count / done_by, "client_wall_s": round(wall, 4),
                "p50_us": round(stats["p50_us"], 1),
                "p99_us": round(stats["p99_us"], 1), "max_us": round(stats["max_us"], 1),
                "latency_from": "scheduled arrival to box in host memory",
                "client_max_lag_us": round(lag * 1e6, 1),
                "client_longest_submit_us": round(longest * 1e6, 1),
                "equals_batch": same}

    for mode, name in ((0, "served_persistent"), (1, "served_launch_per_query")):
        out[name] = serve(mode, nq, 1.0)
        log(f"{name}: {out[name]}")
    # the same stream offered twice as fast (1e5/s): the persistent server's
    # headroom over the workload's rate (faster than that, the client loop in
    # Python falls behind its own schedule)
    out["served_persistent_at_2x_rate"] = serve(0, nq, 0.5)
    log(f"served at 2x: {out['served_persistent_at_2x_rate']}")
    # what a query costs with the server otherwise idle: the query at the 99th
    # percentile of the wave time ceil(n / 64) x steps, and the longest one,
    # each submitted alone and polled to its result (median of 20 after one
    # that may start the grid), beside the served p99, which adds queueing
    # behind other queries to such times
    cost = np.array([-(-int(q.problem.n) // 64) * int(q.problem.nsteps) for q in qs])
    order = np.argsort(cost, kind="stable")
    rc.set_option("serve.mode", 0)
    R.reach_server_start(rc.ctx, pool, pool.numel(), 1024)
    alone = {}
    for name, i in (("p99_cost_query", int(order[int(0.99 * (nq - 1))])),
                    ("max_cost_query", int(order[-1]))):
        reps = []
        for _ in range(21):
            t = time.perf_counter()
            tk = R.reach_submit(rc.ctx, hq[i])
            while R.reach_poll(rc.ctx, tk)[0] == R.REACH_PENDING:
                pass
            reps.append(time.perf_counter() - t)
        alone[name] = {"n": int(qs[i].problem.n), "nsteps": int(qs[i].problem.nsteps),
                       "submit_to_result_us": round(float(np.median(reps[1:])) * 1e6, 1)}
    R.reach_server_stop(rc.ctx)
    out["served_persistent"]["alone_on_idle_server"] = alone
    log(f"alone: {alone}")
    # launch per query cannot keep up with 5e4/s: its latency then grows with
    # the backlog.  Its rate under that overload is the most it sustains; the
    # same stream slowed to 80% of that rate (the first 2 s of it) gives its
    # latency at a load it can carry.
    lpq = out["served_launch_per_query"]
    if lpq["queries_per_s"] < 0.95 * lpq["offered_per_s"]:
        scale = lpq["offered_per_s"] / (0.8 * lpq["queries_per_s"])
        count = int(min(nq, np.searchsorted(arrivals * scale, 2.0)))
        out["served_launch_per_query_at_80pct_of_its_max"] = serve(1, count, scale)
        log(f"launch per query slowed: {out['served_launch_per_query_at_80pct_of_its_max']}")
    rc.set_option("serve.mode", 0)
    if cpu:
        out["cpu_oracle"] = oracle_queries(qs, h_lo, h_hi, offs, u_lo, u_hi, min(nq, 2000))
        log(f"oracle queries: {out['cpu_oracle']}")
    return out


def batch_only(rc, R, torch, workloads, nq, tune_first=False, back_to_back=0):
    """One offline batch of the query mix (the batch kernel alone, profiling;
    the last batch launch is the timed one), after the batch autotuner if
    tune_first; then, if back_to_back, 3 untimed and that many timed batches
    issued without waiting in between (those launches come last)."""
    p4 = workloads.serve_mix_f64()
    qs = workloads.query_stream(nq, p4.extra["rate"], seed=p4.seed)
    ns = np.array([q.problem.n for q in qs])
    offs = np.concatenate([[0], np.cumsum(ns)])
    h_lo = np.empty(int(offs[-1]))
    h_hi = np.empty(int(offs[-1]))
    u = np.zeros(2 * nq)
    for i, q in enumerate(qs):
        q.problem.box(out=(h_lo[offs[i]:offs[i + 1]], h_hi[offs[i]:offs[i + 1]]))
        if q.problem.n_in:
            u[2 * i], u[2 * i + 1] = q.problem.p_lo[0], q.problem.p_hi[0]
    d_lo, d_hi, d_u = (torch.from_numpy(a).cuda() for a in (h_lo, h_hi, u))
    r_lo, r_hi = torch.empty_like(d_lo), torch.empty_like(d_hi)
    dq = R.query_array([R.make_query(q.problem.kind, q.problem.n, q.problem.prm, R.REACH_F64,
                                     d_lo.data_ptr() + 8 * offs[i], d_hi.data_ptr() + 8 * offs[i],
                                     r_lo.data_ptr() + 8 * offs[i], r_hi.data_ptr() + 8 * offs[i],
                                     q.problem.dt, q.problem.nsteps,
                                     d_u.data_ptr() + 16 * i if q.problem.n_in else None,
                                     d_u.data_ptr() + 16 * i + 8 if q.problem.n_in else None,
                                     n_in=q.problem.n_in) for i, q in enumerate(qs)])
    nbw = R.reach_batch_workspace_bytes(nq)
    wsb = torch.empty(nbw, dtype=torch.uint8, device="cuda")
    tune = None
    if tune_first:
        tune = R.reach_autotune_batch(rc.ctx, dq, wsb, nbw, None)
    R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, None)
    torch.cuda.synchronize()
    t = time.perf_counter()
    R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, None)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    assert rc.sync() == R.REACH_OK
    out = {"workload": f"{nq} queries of the mix, one batch", "seconds": round(tb, 4),
           "queries_per_s": nq / tb, "autotune": tune}
    if back_to_back:
        ref = r_lo.cpu().numpy()
        for _ in range(3):
            R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, None)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(back_to_back):
            R.reach_embed_rk4_batch(rc.ctx, dq, wsb, nbw, None)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / back_to_back
        assert rc.sync() == R.REACH_OK
        assert np.array_equal(r_lo.cpu().numpy(), ref)
        out["back_to_back"] = {"batches": back_to_back, "seconds_per_batch": round(el, 5),
                               "queries_per_s": nq / el}
    return out


def oracle_queries(qs, h_lo, h_hi, offs, u_lo, u_hi, k):
    """The oracle on the first k queries of the mix, one query per host thread
    (each single-threaded); queries/s."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def one(i):
        pr = qs[i].problem
        a, b = offs[i], offs[i + 1]
        pl = np.array([u_lo[i]]) if pr.n_in else None
        ph = np.array([u_hi[i]]) if pr.n_in else None
        oracle.embed_rk4(pr.kind, pr.prm, h_lo[a:b], h_hi[a:b], pl, ph, dt=pr.dt,
                         nsteps=pr.nsteps)

    with ThreadPoolExecutor(workers, initializer=oracle.set_threads, initargs=(1,)) as ex:
        list(ex.map(lambda i: None, range(workers)))      # start the workers
        t = time.perf_counter()
        list(ex.map(one, range(k)))
        el = time.perf_counter() - t
    return {"queries_per_s": k / el, "threads": workers, "sample": f"first {k} queries",
            "kind": "oracle"}


def extra_ctm_2p31_f32(rc, R, torch, workloads, steps=2, cpu_oracle=True):
    """CTM chain n = 2^31 FP32, 200 RK4 steps: the largest single-GPU embedding."""
    p = workloads.ctm_2p31_f32()
    lo = np.empty(p.n, dtype=np.float32)
    hi = np.empty(p.n, dtype=np.float32)
    t = time.perf_counter()
    p.box(out=(lo, hi))
    log(f"ctm 2^31 inputs in {time.perf_counter() - t:.1f} s")
    x_lo = torch.from_numpy(lo).cuda()
    x_hi = torch.from_numpy(hi).cuda()
    del lo, hi
    r_lo, r_hi = torch.empty_like(x_lo), torch.empty_like(x_hi)
    sysd = R.make_system(p.kind, p.n, p.prm, 0)
    nb = R.reach_workspace_bytes(rc.ctx, sysd, R.REACH_F32, 0)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F32, p.nsteps)
    run = lambda: R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F32, x_lo, x_hi, None, None, 0.0, p.dt,
                                    p.nsteps, r_lo, r_hi, ws, nb, None)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3 / steps
    launch = sec / plan["passes"]
    ops = 2.0 * p.n * (p.nsteps / plan["passes"]) * CTM_OPS_PER_STATE_STEP   # per launch, on average
    byts = 4.0 * p.n * 4
    out = {"workload": "CTM chain n=2^31 FP32, dt=0.01, 200 RK4 steps",
           "state_steps_per_s": 2.0 * p.n * p.nsteps / sec, "seconds": round(sec, 4),
           "plan": plan, "launch_us": round(launch * 1e6, 1),
           "alu_frac_fp32_published": round(ops / launch / FP32_PEAK, 4),
           "alu_frac_fp32_nonpacked": round(ops / launch / (FP32_PEAK / 2), 4),
           "hbm_frac": round(byts / launch / HBM_PEAK, 4)}
    del x_lo, x_hi, r_lo, r_hi, ws
    torch.cuda.empty_cache()
    if cpu_oracle:
        import oracle
        q = workloads.small_problem(workloads.KIND_CTM, 1 << 24, p.seed, 4)
        qlo, qhi = q.box()
        t = time.perf_counter()
        oracle.embed_rk4(q.kind, q.prm, qlo, qhi, dt=q.dt, nsteps=q.nsteps)
        csec = time.perf_counter() - t
        out["cpu_oracle"] = {"state_steps_per_s": 2.0 * q.n * q.nsteps / csec,
                             "sample": "FP64 oracle, CTM n = 2^24, 4 steps; extrapolated per "
                                       "state-step to the 2^31 chain",
                             "threads": oracle.get_threads()}
    return out


def extra_heat3d_1000(rc, R, torch, workloads, cpu_oracle=True, steps=0):
    """The heat diffusion case study at its stated size: 1000^3 grid (n = 10^9),
    FP64, 1000 RK4 steps of dt = 0.02, embedding of the heated-corner box
    (`steps` overrides the step count)."""
    p = workloads.heat3d_1000_f64()
    if steps:
        p.nsteps = steps
    lo = np.empty(p.n, dtype=np.float64)
    hi = np.empty(p.n, dtype=np.float64)
    t = time.perf_counter()
    p.box(out=(lo, hi))
    log(f"heat 1000^3 inputs in {time.perf_counter() - t:.1f} s")
    x_lo = torch.from_numpy(lo).cuda()
    x_hi = torch.from_numpy(hi).cuda()
    del lo, hi
    r_lo, r_hi = torch.empty_like(x_lo), torch.empty_like(x_hi)
    sysd = R.make_system(p.kind, p.n, list(p.prm), 0)
    nb = R.reach_workspace_bytes(rc.ctx, sysd, R.REACH_F64, 0)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, p.nsteps)
    run = lambda k: R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, None, None, 0.0,
                                      p.dt, k, r_lo, r_hi, ws, nb, None)
    run(4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run(p.nsteps)
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3
    launch = sec / p.nsteps
    cells = 2.0 * p.n
    out = {"workload": f"3-D heat diffusion 1000^3 (n=1e9) FP64, dt=0.02, {p.nsteps} RK4 steps "
                       "(embedding, 2n states)",
           "cell_steps_per_s": cells * p.nsteps / sec, "seconds": round(sec, 3),
           "plan": plan, "launch_ms": round(launch * 1e3, 3),
           "roofline": {"bound": "hbm",
                        "achieved": round(cells * HEAT_BYTES_PER_CELL_STEP / launch / 1e9, 1),
                        "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(cells * HEAT_BYTES_PER_CELL_STEP / launch / HBM_PEAK, 4),
                        "traffic": traffic_from_profile("heat3d_kernel_1000cube_f64_pmc.txt",
                                                        HEAT_SOURCES)},
           "alu_frac_fp64": round(cells * HEAT_OPS_PER_CELL_STEP / launch / FP64_PEAK, 4),
           "paper_cpu_minutes": {"m4.10xlarge": 472, "c5.24xlarge": 350.2}}
    del x_lo, x_hi, r_lo, r_hi, ws
    torch.cuda.empty_cache()
    if cpu_oracle:
        import oracle
        q = workloads.heat3d_problem(200, 200, 200, workloads.BASE_SEED + 6, 5)
        qlo, qhi = q.box()
        t = time.perf_counter()
        oracle.embed_rk4(q.kind, list(q.prm), qlo, qhi, dt=q.dt, nsteps=q.nsteps)
        csec = time.perf_counter() - t
        out["cpu_oracle"] = {"cell_steps_per_s": 2.0 * q.n * q.nsteps / csec,
                             "sample": "200^3 grid, 5 steps",
                             "cores": oracle.get_threads()}
    return out


LIN3_OPS_PER_STATE_STEP = 41    # growth-bound half-width: 4 right-hand sides of 7 + 13


def next_rows_rd(rc, R, torch, p, x_lo, x_hi, p_lo, p_hi, ref_s, stream):
    """The growth bound and the reach tube on the benchmark's own RD 2^26
    workload (inputs resident), against the plain embedding's time ref_s."""
    out = {}
    sysd = R.make_system(p.kind, p.n, p.prm, p.n_in)
    nb = R.reach_growth_bound_workspace_bytes(rc.ctx, sysd, R.REACH_F64)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    g_lo, g_hi = torch.empty_like(x_lo), torch.empty_like(x_hi)
    run = lambda: R.reach_growth_bound(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0,
                                       p.dt, p.nsteps, g_lo, g_hi, ws, nb, stream)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(2):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    assert rc.sync(stream) == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3 / 2
    ss = 2.0 * p.n * p.nsteps
    ops = p.n * p.nsteps * (RD_FLOPS_PER_STATE_STEP + LIN3_OPS_PER_STATE_STEP)
    out["growth_bound_rd2p26_f64"] = {
        "workload": "growth bound (Algorithm 2), RD chain n=2^26 FP64, 1000 RK4 steps "
                    "(center and half-width runs)",
        "state_steps_per_s": ss / sec, "seconds": round(sec, 4),
        "vs_embedding_time": round(sec / ref_s, 3) if ref_s else None,
        "roofline": {"bound": "alu", "achieved": round(ops / sec / 1e12, 3),
                     "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": round(ops / sec / FP64_PEAK, 4)}}
    del ws, g_lo, g_hi
    every = 100
    slots = p.nsteps // every
    t_lo = torch.empty(slots * p.n, dtype=torch.float64, device="cuda")
    t_hi = torch.empty_like(t_lo)
    nbe = R.reach_workspace_bytes(rc.ctx, sysd, R.REACH_F64, 0)
    wse = torch.empty(max(nbe, 1), dtype=torch.uint8, device="cuda")
    tube = lambda: R.reach_embed_rk4_tube(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0,
                                          p.dt, p.nsteps, every, t_lo, t_hi, wse, nbe, stream)
    tube()
    torch.cuda.synchronize()
    e0.record(stream)
    tube()
    e1.record(stream)
    torch.cuda.synchronize()
    assert rc.sync(stream) == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3
    out["tube_rd2p26_f64"] = {
        "workload": "reach tube, RD chain n=2^26 FP64, 1000 RK4 steps, a box every 100 steps "
                    "(10 boxes, 10 GiB)",
        "state_steps_per_s": ss / sec, "seconds": round(sec, 4),
        "vs_embedding_time": round(sec / ref_s, 3) if ref_s else None}
    del t_lo, t_hi, wse
    torch.cuda.empty_cache()
    return out


def extra_user_sine(rc, R, torch):
    """A user system compiled at run time: the nonlinear sine chain
    (f_i = -a x_i + b sin(x_{i-1}) + c u with its tight decomposition), n = 2^22
    FP64, 200 RK4 steps, and its Monte Carlo at n = 512, 2^16 samples."""
    from tests import user_sources as us     # the same text the tests use
    t = time.perf_counter()
    user = rc.user(us.SINE)
    compile_s = time.perf_counter() - t
    n, N = 1 << 22, 200
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x_lo = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) * 6.0 - 3.0
    x_hi = x_lo + 0.5
    pl = torch.tensor([-0.2], dtype=torch.float64, device="cuda")
    ph = torch.tensor([0.3], dtype=torch.float64, device="cuda")
    rc.embed_user(user, us.SINE_PRM, x_lo, x_hi, 0.05, 4, p_lo=pl, p_hi=ph)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rc.embed_user(user, us.SINE_PRM, x_lo, x_hi, 0.05, N, p_lo=pl, p_hi=ph)
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3
    m = 1 << 16
    ml, mh = x_lo[:512].contiguous(), x_hi[:512].contiguous()
    rc.montecarlo_user(user, us.SINE_PRM, ml, mh, 0.05, N, 1024, 3, p_lo=pl, p_hi=ph)
    torch.cuda.synchronize()
    e0.record()
    rc.montecarlo_user(user, us.SINE_PRM, ml, mh, 0.05, N, m, 3, p_lo=pl, p_hi=ph)
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    msec = e0.elapsed_time(e1) / 1e3
    R.reach_user_destroy(user)
    out = {"workload": "user sine chain (hipRTC) n=2^22 FP64, dt=0.05, 200 RK4 steps; Monte "
                       "Carlo n=512, 2^16 samples",
           "compile_seconds": round(compile_s, 2),
           "embed_state_steps_per_s": 2.0 * n * N / sec, "embed_seconds": round(sec, 4),
           "mc_cell_steps_per_s": 512.0 * m * N / msec, "mc_seconds": round(msec, 4)}
    # cost of the run-time path itself: the reaction-diffusion chain as user
    # text in the built-in kernel's operation order against the built-in
    # kernel, same inputs (n = 2^24, 200 steps)
    user = rc.user(us.RD_FUSED)
    n2 = 1 << 24
    c_lo = torch.rand(n2, dtype=torch.float64, device="cuda", generator=g) * 0.5
    c_hi = c_lo + 0.02
    pl2 = torch.tensor([-0.1], dtype=torch.float64, device="cuda")
    ph2 = torch.tensor([0.1], dtype=torch.float64, device="cuda")
    runs = {"user": lambda: rc.embed_user(user, (1.0, 2.0), c_lo, c_hi, 0.1, N, p_lo=pl2,
                                          p_hi=ph2),
            "builtin": lambda: rc.embed(R.REACH_RD, (1.0,), c_lo, c_hi, 0.1, N, p_lo=pl2,
                                        p_hi=ph2)}
    secs = {}
    for name, f in runs.items():
        f()
        torch.cuda.synchronize()
        e0.record()
        f()
        e1.record()
        torch.cuda.synchronize()
        assert rc.sync() == R.REACH_OK
        secs[name] = e0.elapsed_time(e1) / 1e3
    R.reach_user_destroy(user)
    out["user_rd_vs_builtin"] = {
        "workload": "reaction-diffusion chain n=2^24 FP64, dt=0.1, 200 RK4 steps",
        "user_state_steps_per_s": 2.0 * n2 * N / secs["user"],
        "builtin_state_steps_per_s": 2.0 * n2 * N / secs["builtin"],
        "user_over_builtin_time": round(secs["user"] / secs["builtin"], 3)}
    return out


def extra_mc_ctm4096(rc, R, torch, workloads, cpu_samples):
    """Monte Carlo, CTM n = 4096 FP32, 2^20 samples, 500 RK4 steps."""
    import oracle
    p = workloads.mc_ctm4096_f32()
    lo, hi = p.box()
    x_lo, x_hi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    rc.montecarlo(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, 4096, p.seed)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    mn, mx = rc.montecarlo(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, p.m, p.seed)
    e1.record()
    torch.cuda.synchronize()
    assert rc.sync() == R.REACH_OK
    sec = e0.elapsed_time(e1) / 1e3
    cell_steps = float(p.n) * p.m * p.nsteps
    ops = cell_steps * CTM_OPS_PER_STATE_STEP
    out = {"workload": "Monte Carlo, CTM n=4096 FP32, 2^20 samples, dt=0.01, 500 RK4 steps",
           "cell_steps_per_s": cell_steps / sec, "seconds": round(sec, 4),
           "roofline": {"bound": "alu", "achieved": round(ops / sec / 1e12, 3),
                        "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
                        "frac": round(ops / sec / FP32_PEAK, 4),
                        "frac_of_nonpacked_peak": round(ops / sec / (FP32_PEAK / 2), 4)}}
    # VALU issue of this launch from the committed PMC summary (taken on the
    # current Monte Carlo sources), and per CU-cycle at the clock of that run
    valu = profile_value("mc_kernel_ctm4096_f32_pmc.txt", "valu_wave_instructions_per_launch",
                         MC_SOURCES)
    if valu:
        out["roofline"]["valu_lane_instructions_per_cell_step"] = round(valu * 64 / cell_steps, 2)
        out["roofline"]["valu_issue_frac"] = round(valu * 64 / sec / VALU_LANE_PEAK, 4)
        out["roofline"]["valu_issue_per_cu_cycle"] = profile_value(
            "mc_kernel_ctm4096_f32_pmc.txt", "valu_issue_per_cu_cycle", MC_SOURCES)
    # containment in the FP64 embedding box of the same problem (the FP32 box
    # values are exact in FP64), with the FP32-vs-FP64 slack of the tests
    e_lo, e_hi = rc.embed(p.kind, p.prm, x_lo.double(), x_hi.double(), p.dt, p.nsteps)
    assert rc.sync() == R.REACH_OK
    e_lo, e_hi = e_lo.cpu().numpy(), e_hi.cpu().numpy()
    g_mn, g_mx = mn.double().cpu().numpy(), mx.double().cpu().numpy()
    slack_lo = 1e-5 * np.maximum(np.abs(e_lo), 1.0)
    slack_hi = 1e-5 * np.maximum(np.abs(e_hi), 1.0)
    ratio = (g_mx - g_mn) / np.maximum(e_hi - e_lo, np.finfo(np.float64).tiny)
    out["containment"] = {
        "violations": int(np.sum(g_mn < e_lo - slack_lo) + np.sum(g_mx > e_hi + slack_hi)),
        "violations_without_slack": int(np.sum(g_mn < e_lo) + np.sum(g_mx > e_hi)),
        "cells": int(p.n), "slack": "1e-5 max(|x|, 1)",
        "width_ratio_mc_over_embedding": {"mean": round(float(ratio.mean()), 4),
                                          "min": round(float(ratio.min()), 4),
                                          "max": round(float(ratio.max()), 4)}}
    if cpu_samples:
        # the GPU on the same sample prefix, compared with the oracle's result
        s_mn, s_mx = rc.montecarlo(p.kind, p.prm, x_lo, x_hi, p.dt, p.nsteps, cpu_samples,
                                   p.seed)
        assert rc.sync() == R.REACH_OK
        t = time.perf_counter()
        o_mn, o_mx = oracle.montecarlo(p.kind, p.prm, lo.astype(np.float64),
                                       hi.astype(np.float64), dt=p.dt, nsteps=p.nsteps,
                                       m=cpu_samples, seed=p.seed, ubits=24)
        el = time.perf_counter() - t
        err = max(float(np.max(np.abs(g.double().cpu().numpy() - o) / np.maximum(np.abs(o), 1.0)))
                  for g, o in ((s_mn, o_mn), (s_mx, o_mx)))
        out["cpu_baseline"] = {"value": float(p.n) * cpu_samples * p.nsteps / el,
                               "unit": "cell-steps/s", "kind": "oracle", "seconds": round(el, 2),
                               "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                           os.cpu_count() or 1)),
                               "sample": f"first {cpu_samples} of the 2^20 samples",
                               "gpu_same_samples_max_rel_err": err,
                               "gpu_same_samples_within_1e-5": bool(err <= 1e-5)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--E", type=int, default=0, help="cells per lane (0 = tuned)")
    ap.add_argument("--K", type=int, default=0, help="RK4 steps per HBM pass (0 = tuned)")
    ap.add_argument("--S", type=int, default=0, help="sides per wavefront, 1 or 2 (0 = tuned)")
    ap.add_argument("--cpu-steps", type=int, default=120)
    ap.add_argument("--cpu-mc-samples", type=int, default=4096)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-queries", action="store_true")
    ap.add_argument("--queries", type=int, default=100000)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP32 2^31-cell embedding and the Monte Carlo run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--heat-only", type=int, default=0, metavar="STEPS",
                    help="only run the 1000^3 heat grid for STEPS RK4 steps (profiling)")
    ap.add_argument("--heat-P", type=int, default=0, help="rows per wave of the heat kernel")
    ap.add_argument("--only", choices=("mc", "ctm31", "batch", "latency", "user", "next"),
                    default=None,
                    help="only run one extra row (profiling): the Monte Carlo run, the 2^31 "
                         "FP32 chain (one call), one batch of the query mix, the 64-cell "
                         "latency calls, the run-time compiled systems, or the growth bound "
                         "and reach tube on the RD 2^26 workload")
    ap.add_argument("--batch-pack", type=int, default=0,
                    help="option batch.pack for --only batch (0 auto, 1 always, 2 never)")
    ap.add_argument("--batch-E", type=int, default=0,
                    help="option batch.E for --only batch (largest cells per lane of a pack)")
    ap.add_argument("--batch-waves", type=int, default=0,
                    help="option batch.waves for --only batch (resident waves)")
    ap.add_argument("--batch-back-to-back", type=int, default=0, metavar="K",
                    help="--only batch: then 3 untimed and K timed batches issued back to back")
    ap.add_argument("--stream-probe", action="store_true",
                    help="time the HBM stream probe over its shapes and print it (only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of one embedding pass's bytes "
                         "(the reference kernel for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU library: runs with --gpus 1 only (the "
                                   "multi-GPU decomposition is a design, not launched)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads
    import paper_2001_10635_amd as R

    if args.only:
        rc = R.Reach(0)
        if args.only == "mc":
            out = extra_mc_ctm4096(rc, R, torch, workloads, 0)
        elif args.only == "user":
            out = extra_user_sine(rc, R, torch)
        elif args.only == "latency":
            out = latency_ctm64(rc, R, torch, workloads, reps=200, cpu=False)
        elif args.only == "ctm31":
            out = extra_ctm_2p31_f32(rc, R, torch, workloads, steps=1, cpu_oracle=False)
        elif args.only == "next":
            p = workloads.rd_2p26_f64()
            lo, hi = p.box()
            pl, ph = p.inputs()
            out = next_rows_rd(rc, R, torch, p, torch.from_numpy(lo).cuda(),
                               torch.from_numpy(hi).cuda(), torch.from_numpy(pl).cuda(),
                               torch.from_numpy(ph).cuda(), None,
                               torch.cuda.current_stream())
        else:
            rc.set_option("batch.pack", args.batch_pack)
            rc.set_option("batch.E", args.batch_E)
            rc.set_option("batch.waves", args.batch_waves)
            out = batch_only(rc, R, torch, workloads, args.queries,
                             tune_first=not (args.batch_pack or args.batch_E or args.batch_waves
                                             or args.no_tune),
                             back_to_back=args.batch_back_to_back)
        print(json.dumps(out), flush=True)
        rc.close()
        return

    if args.heat_only:
        rc = R.Reach(0)
        if args.heat_P:
            rc.set_option("heat.P", args.heat_P)
        out = extra_heat3d_1000(rc, R, torch, workloads, cpu_oracle=False, steps=args.heat_only)
        print(json.dumps(out), flush=True)
        rc.close()
        return

    p = workloads.rd_2p26_f64()
    if args.stream_probe:
        print(json.dumps(hbm_probe(R, torch, p.n, torch.cuda.current_stream())), flush=True)
        return
    if args.copy_probe:
        # one embedding pass reads 2n doubles and writes 2n doubles; a copy of
        # 2n doubles moves exactly the same bytes
        src = torch.ones(2 * p.n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 8,
                          "copy_probe_bytes_written": dst.numel() * 8}))
        return
    log(f"workload {p.name}: n={p.n} N={p.nsteps} dt={p.dt}")
    lo, hi = p.box()
    pl, ph = p.inputs()
    dev = torch.device("cuda", 0)
    x_lo = torch.from_numpy(lo).to(dev)
    x_hi = torch.from_numpy(hi).to(dev)
    p_lo = torch.from_numpy(pl).to(dev)
    p_hi = torch.from_numpy(ph).to(dev)
    r_lo = torch.empty_like(x_lo)
    r_hi = torch.empty_like(x_hi)
    del lo, hi

    rc = R.Reach(0)
    if args.E:
        rc.set_option("embed.E", args.E)
    if args.K:
        rc.set_option("embed.K", args.K)
    if args.S:
        rc.set_option("embed.S", args.S)
    sysd = R.make_system(p.kind, p.n, p.prm, p.n_in)
    nbytes = 2 * p.n * 8
    ws = rc.workspace(nbytes)
    stream = torch.cuda.current_stream()
    tuned = None
    if not (args.E or args.K or args.S or args.no_tune):
        tuned = R.reach_autotune_embed(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, p.dt,
                                       48, r_lo, r_hi, ws, nbytes, stream)
        log(f"autotuned {tuned}")
    plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, p.nsteps)
    log(f"plan {plan}")
    assert R.reach_workspace_bytes(rc.ctx, sysd, R.REACH_F64, 0) <= nbytes

    def one():
        R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0, p.dt,
                          p.nsteps, r_lo, r_hi, ws, nbytes, stream)

    for i in range(args.warmup):
        one()
        log(f"warmup {i + 1}/{args.warmup}")
    assert rc.sync(stream) == R.REACH_OK
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        one()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    st = rc.sync(stream)
    assert st == R.REACH_OK, f"device status {st}"
    ms_per_step = wall * 1e3 / args.steps
    state_steps = 2.0 * p.n * p.nsteps
    value = state_steps / (ms_per_step / 1e3)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.3e} state-steps/s")

    # roofline of the dominant kernel (the embedding pass), live
    launches = args.steps * plan["passes"]
    launch_s = gpu_ms / 1e3 / launches
    bytes_per_launch = 4.0 * p.n * 8            # read lo, hi; write lo, hi
    # average steps per launch (the last pass of a run may be shorter than K)
    flops_per_launch = 2.0 * p.n * (p.nsteps / plan["passes"]) * RD_FLOPS_PER_STATE_STEP
    hbm_ach = bytes_per_launch / launch_s
    alu_ach = flops_per_launch / launch_s
    hbm_frac, alu_frac = hbm_ach / HBM_PEAK, alu_ach / FP64_PEAK
    traffic = traffic_from_profile()
    # VALU issue: rocprof lane instructions per state-step (PMC summary of the
    # same kernel source) times this run's state-steps per second of launch
    lanes_per_ss = profile_value("embed_tile_kernel_rd2p26_f64_pmc.txt",
                                 "valu_lane_instructions_per_state_step")
    ss_per_launch_s = 2.0 * p.n * (p.nsteps / plan["passes"]) / launch_s
    extra_roof = {"kernel": "embed_tile_kernel<RD,double>", "launch_us": round(launch_s * 1e6, 1),
                  "algorithmic_GBps": round(hbm_ach / 1e9, 1),
                  "valu_lane_instructions_per_state_step": lanes_per_ss,
                  "valu_issue_frac": (round(lanes_per_ss * ss_per_launch_s / VALU_LANE_PEAK, 4)
                                      if lanes_per_ss else None),
                  # the same issue in GPU cycles (GRBM_COUNT of the PMC summary's
                  # run): wave-instructions per CU-cycle at the clock the GPU ran
                  "valu_issue_per_cu_cycle": profile_value(
                      "embed_tile_kernel_rd2p26_f64_pmc.txt", "valu_issue_per_cu_cycle"),
                  "profiled_gpu_clock_ghz": profile_value(
                      "embed_tile_kernel_rd2p26_f64_pmc.txt", "gpu_clock_ghz_in_this_run"),
                  # rocprof DRAM bytes (read + write) per launch over this launch time
                  "hbm_frac_measured": (round(traffic / launch_s / HBM_PEAK, 4)
                                        if traffic else None)}
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(alu_ach / 1e12, 3), "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": traffic,
                "hbm_frac_same_launch": round(hbm_frac, 4), **extra_roof}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_ach / 1e9, 1), "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic,
                "alu_frac_same_launch": round(alu_frac, 4), **extra_roof}

    # K = 1 streaming pass: the same kernel as a pure HBM stream
    stream_k1 = None
    if not args.no_stream:
        # one step per pass: the tile width that streams best (the chosen one,
        # else E = 24: at K = 1 the halo is 4 cells and more waves per pass pay)
        rc.set_option("embed.K", 1)
        nk = 20
        best = None
        for e1 in dict.fromkeys((plan["E"], 24)):
            rc.set_option("embed.E", e1)
            plan1 = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, nk)
            R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0, p.dt, nk,
                              r_lo, r_hi, ws, nbytes, stream)
            torch.cuda.synchronize()
            for _ in range(3):      # the fastest of three calls, as for the copy below
                ev0.record(stream)
                R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0, p.dt,
                                  nk, r_lo, r_hi, ws, nbytes, stream)
                ev1.record(stream)
                torch.cuda.synchronize()
                t = ev0.elapsed_time(ev1) / 1e3 / plan1["passes"]
                if best is None or t < best[0]:
                    best = (t, plan1)
        t1, plan1 = best
        rc.set_option("embed.E", args.E)
        # the device's plain-copy rate for the same bytes (two arrays of n
        # doubles in, two out), the practical ceiling of any HBM stream
        c_in = torch.empty(2 * p.n, dtype=torch.float64, device="cuda")
        c_out = torch.empty_like(c_in)
        tc = None
        with torch.cuda.stream(stream):
            for _ in range(3):
                c_out.copy_(c_in)
            for _ in range(3):      # the fastest of three rounds of 5
                ev0.record(stream)
                for _ in range(5):
                    c_out[:p.n].copy_(c_in[:p.n])
                    c_out[p.n:].copy_(c_in[p.n:])
                ev1.record(stream)
                ev1.synchronize()
                t = ev0.elapsed_time(ev1) / 1e3 / 5
                tc = t if tc is None else min(tc, t)
        torch.cuda.synchronize()
        del c_in, c_out
        probe = hbm_probe(R, torch, p.n, stream)
        log(f"HBM stream probe: {probe}")
        stream_k1 = {"E": plan1["E"], "launch_us": round(t1 * 1e6, 1),
                     "achieved_GBps": round(bytes_per_launch / t1 / 1e9, 1),
                     "frac": round(bytes_per_launch / t1 / HBM_PEAK, 4),
                     "state_steps_per_s": 2.0 * p.n / t1,
                     "device_copy_us": round(tc * 1e6, 1),
                     "device_copy_GBps": round(bytes_per_launch / tc / 1e9, 1),
                     "frac_of_device_copy": round(tc / t1, 4),
                     "stream_probe": probe,
                     "frac_of_stream_probe": round(probe["us"] / 1e6 / t1, 4)}
        rc.set_option("embed.K", args.K)
        assert rc.sync(stream) == R.REACH_OK
        log(f"K=1 stream: {stream_k1}")
    next_rows = {}
    if not args.no_extra:
        next_rows = next_rows_rd(rc, R, torch, p, x_lo, x_hi, p_lo, p_hi, ms_per_step / 1e3,
                                 stream)
        log(f"growth bound / tube: {next_rows}")
    del x_lo, x_hi, p_lo, p_hi, r_lo, r_hi
    rc._ws = None
    torch.cuda.empty_cache()

    queries = None
    if not args.no_queries:
        queries = query_mix(rc, R, torch, workloads, args.queries, cpu=not args.no_cpu)
    extra = {}
    if not args.no_extra:
        extra["latency_ctm64_f64"] = latency_ctm64(rc, R, torch, workloads, cpu=not args.no_cpu)
        log(f"ctm64 latency: {extra['latency_ctm64_f64']}")
        extra["embed_ctm_2p31_f32"] = extra_ctm_2p31_f32(rc, R, torch, workloads,
                                                         cpu_oracle=not args.no_cpu)
        log(f"ctm 2^31 f32: {extra['embed_ctm_2p31_f32']}")
        extra["mc_ctm4096_f32"] = extra_mc_ctm4096(rc, R, torch, workloads,
                                                   0 if args.no_cpu else args.cpu_mc_samples)
        log(f"mc: {extra['mc_ctm4096_f32']}")
        extra.update(next_rows)
        extra["user_sine_f64"] = extra_user_sine(rc, R, torch)
        log(f"user sine: {extra['user_sine_f64']}")
        extra["embed_heat3d_1000_f64"] = extra_heat3d_1000(rc, R, torch, workloads,
                                                           not args.no_cpu)
        if stream_k1:
            hr = extra["embed_heat3d_1000_f64"]["roofline"]
            hr["frac_of_device_copy"] = round(hr["achieved"] / stream_k1["device_copy_GBps"], 4)
        log(f"heat 1000^3: {extra['embed_heat3d_1000_f64']}")

    cpu = None
    if not args.no_cpu:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps on the full chain")
        cpu = cpu_baseline(p, args.cpu_steps)
        log(f"cpu baseline {cpu}")

    out = {
        "metric": "embedding RK4 state-steps/s & %HBM peak; batched queries/s + p99 latency",
        "value": value,
        "unit": "state-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "reaction-diffusion chain n=2^26 FP64, interval input "
                               "u in [-0.1,0.1], dt=0.1, 1000 RK4 steps (mixed-monotone "
                               "embedding, 2n states)",
                   "n": p.n, "rk4_steps": p.nsteps, "E": plan["E"], "K": plan["K"],
                   "sides_per_wave": plan["S"],
                   "passes": plan["passes"], "parallelism": "single GPU"},
        "roofline": roof,
        "hbm_stream_k1": stream_k1,
        "autotune": tuned,
        "queries": queries,
        "other_rows": extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    rc.close()


if __name__ == "__main__":
    main()
