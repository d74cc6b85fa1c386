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
RD_FLOPS_PER_STATE_STEP = 45  # see the design doc: 4 x 8 (RHS) + 3 x 2 (stage inputs) + 5 + 2


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dev.hpp", "embed.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2001_10635_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(per_launch_units: float):
    """HBM bytes per launch from the committed PMC summary, if it matches the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "embed_tile_rd2p26_f64_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(p, steps: int):
    import oracle
    lo, hi = p.box()
    pl, ph = p.inputs()
    t = time.perf_counter()
    oracle.embed_rk4(p.kind, p.prm, lo, hi, pl, ph, dt=p.dt, nsteps=steps)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 2.0 * p.n * steps / el, "unit": "state-steps/s", "cores": cores,
            "kind": "oracle", "seconds": round(el, 2),
            "sample": f"FP64 oracle on the full {p.n}-cell chain for {steps} of the "
                      f"{p.nsteps} RK4 steps (same box, inputs and dt)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--E", type=int, default=0, help="cells per lane (0 = tuned)")
    ap.add_argument("--K", type=int, default=0, help="RK4 steps per HBM pass (0 = tuned)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the sharded design is described "
                                   "in DESIGN.md and not launched", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads
    import paper_2001_10635_amd as R

    p = workloads.config(1)
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
    sysd = R.make_system(p.kind, p.n, p.prm, p.n_in)
    plan = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, p.nsteps)
    log(f"plan {plan}")
    nbytes = R.reach_workspace_bytes(rc.ctx, sysd, R.REACH_F64, 0)
    ws = rc.workspace(nbytes)
    stream = torch.cuda.current_stream()

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
    flops_per_launch = 2.0 * p.n * plan["K"] * RD_FLOPS_PER_STATE_STEP
    hbm_ach = bytes_per_launch / launch_s
    alu_ach = flops_per_launch / launch_s
    hbm_frac, alu_frac = hbm_ach / HBM_PEAK, alu_ach / FP64_PEAK
    traffic = traffic_from_profile(bytes_per_launch)
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(alu_ach / 1e12, 3), "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": traffic,
                "kernel": "embed_tile_kernel<RD,double>", "launch_us": round(launch_s * 1e6, 1),
                "hbm_frac_same_launch": round(hbm_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_ach / 1e9, 1), "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic,
                "kernel": "embed_tile_kernel<RD,double>", "launch_us": round(launch_s * 1e6, 1),
                "alu_frac_same_launch": round(alu_frac, 4)}

    # K = 1 streaming pass: the same kernel as a pure HBM stream
    stream_k1 = None
    if not args.no_stream:
        rc.set_option("embed.K", 1)
        nk = 20
        plan1 = R.reach_plan_embed(rc.ctx, sysd, R.REACH_F64, nk)
        R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0, p.dt, nk,
                          r_lo, r_hi, ws, nbytes, stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        R.reach_embed_rk4(rc.ctx, sysd, R.REACH_F64, x_lo, x_hi, p_lo, p_hi, 0.0, p.dt, nk,
                          r_lo, r_hi, ws, nbytes, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        t1 = ev0.elapsed_time(ev1) / 1e3 / plan1["passes"]
        stream_k1 = {"E": plan1["E"], "launch_us": round(t1 * 1e6, 1),
                     "achieved_GBps": round(bytes_per_launch / t1 / 1e9, 1),
                     "frac": round(bytes_per_launch / t1 / HBM_PEAK, 4),
                     "state_steps_per_s": 2.0 * p.n / t1}
        rc.set_option("embed.K", args.K)
        assert rc.sync(stream) == R.REACH_OK
        log(f"K=1 stream: {stream_k1}")

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
                   "passes": plan["passes"], "parallelism": "single GPU"},
        "roofline": roof,
        "hbm_stream_k1": stream_k1,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    rc.close()


if __name__ == "__main__":
    main()
