#!/usr/bin/env python3
"""Benchmark of the Langevin-XY hot path on one MI355X.

Headline: site-updates/s of the FP32 fused BBK step on one 4096 x 4096
periodic lattice (J_x = 1, J_y = -0.1, h = 0.5, gamma = 1, dt = 0.01,
T = 0.3, seed 1) with the FP64 observables (energy, staggered order
parameter, structure-factor modes for the Binder cumulant and the
correlation length) fused into every 500th step.  One "step" is one BBK
step of the whole lattice.  The state is resident in HBM before timing.

Also reported on the same line:
  * roofline of the dominant kernel (the plain FP32 step): algorithmic bytes
    (16 B per site: read angle and velocity, write both) / average kernel
    duration from HIP events around back-to-back launches, against 8 TB/s;
  * HBM traffic per launch from rocprofv3 counters when the committed
    counter summary matches the current kernel source, else null;
  * batched-ensemble vs one-launch-per-replica throughput on the 288-replica
    finite-size-scaling ensemble (L = 32..512);
  * adjoint / forward time on the 512 x 512 differentiation workload;
  * frozen-domain labelling time on one 2048 x 2048 quench replica;
  * the FP64 CPU oracle timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
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

HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE_F32 = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_f32_4096_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("xyl_step.hip", "xyl_device.hpp", "xyl_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2409_06412_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(L):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash() or t.get("L") != L:
        return None
    return t.get("bytes_per_launch")


def time_step_kernel(torch, lat, nlaunch):
    """Average duration of the plain step kernel: HIP events on the lattice's
    stream around nlaunch back-to-back launches (no graph, no measurement)."""
    lat.set_graph_steps(0)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.step(5)
    e0.record(s)
    lat.step(nlaunch)
    e1.record(s)
    e1.synchronize()
    lat.set_graph_steps(32)
    return e0.elapsed_time(e1) / nlaunch


def bench_ensemble(torch, xyl, workloads, nsteps):
    specs = workloads.fss_ensemble(nsteps=10 ** 9)
    out = {}
    for mode, name in ((0, "batched"), (1, "per_replica")):
        ens = xyl.Ensemble(specs, dtype="f32", stream=torch.cuda.current_stream().cuda_stream)
        ens.set_mode(mode)
        ens.step(3)
        ens.sync()
        t0 = time.perf_counter()
        ens.step(nsteps)
        ens.sync()
        out[name] = time.perf_counter() - t0
        ens.close()
    sites = sum(s.Lx * s.Ly for s in specs)
    return {"replicas": len(specs), "sites": sites, "steps": nsteps,
            "batched_site_updates_per_s": sites * nsteps / out["batched"],
            "per_replica_site_updates_per_s": sites * nsteps / out["per_replica"],
            "speedup": out["per_replica"] / out["batched"]}


def bench_adjoint(torch, xyl, workloads):
    spec = workloads.adjoint_512()
    lat = xyl.Lattice(spec.Lx, spec.Ly, dtype="f32", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    try:
        lat.init_random()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.adjoint_forward(spec.nsteps, 100, 1000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.adjoint_backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    except xyl.XylError as e:
        lat.close()
        return {"error": str(e)}
    # plain forward of the same run for reference
    lat.init_random()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lat.step_measured(spec.nsteps, 1) if False else lat.step(spec.nsteps)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    lat.close()
    return {"L": spec.Lx, "steps": spec.nsteps, "forward_with_loss_s": t1 - t0, "backward_s": t2 - t1,
            "plain_forward_s": t4 - t3, "adjoint_over_forward": (t2 - t1) / (t1 - t0)}


def bench_domains(torch, xyl):
    lat = xyl.Lattice(2048, 2048, dtype="f32", schedule=[(0, 1.5), (1000, 0.0)], seed=0,
                      stream=torch.cuda.current_stream().cuda_stream)
    lat.init_random()
    lat.step(1200)
    lat.domains(want_labels=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sizes, counts, nd, mx = lat.domains(want_labels=False)
    t1 = time.perf_counter()
    lat.close()
    return {"L": 2048, "seconds": t1 - t0, "n_domains": int(nd), "max_size": int(mx)}


def cpu_baseline(L, nsteps):
    import oracle
    from paper_2409_06412_amd import workloads
    spec = workloads.large_fp32(0, L)
    o = oracle.Oracle(**spec.oracle_kwargs())
    th, om = o.init_random()
    t0 = time.perf_counter()
    o.run(th, om, 0, nsteps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": L * L * nsteps / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, %dx%d lattice, %d BBK steps (%.1f s)" % (L, L, nsteps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--L", type=int, default=4096)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=12)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2409_06412_amd as xyl
    from paper_2409_06412_amd import workloads

    assert torch.cuda.is_available(), "no GPU visible"
    L = args.L
    spec = workloads.large_fp32(0, L)
    stream = torch.cuda.current_stream().cuda_stream
    lat = xyl.Lattice(L, L, dtype="f32", schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                      stream=stream, **spec.params())
    lat.init_random()
    launch = lat.autotune()
    log("launch shape (rows per strip, waves per workgroup):", launch)
    lat.step(args.warmup)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    samples = lat.step_measured(args.steps, args.every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = L * L * args.steps / wall
    log("timed %d steps in %.4f s: %.4g site-updates/s (%d samples)" % (args.steps, wall, value, len(samples)))

    kern_ms = time_step_kernel(torch, lat, 500)
    achieved = BYTES_PER_SITE_F32 * L * L / (kern_ms * 1e-3) / 1e9
    traffic = load_traffic(L)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_step<float, store>", "avg_kernel_us": kern_ms * 1e3,
                "algorithmic_bytes_per_launch": BYTES_PER_SITE_F32 * L * L}
    log("step kernel %.2f us -> %.1f GB/s algorithmic (%.1f%% of 8 TB/s)" % (kern_ms * 1e3, achieved,
                                                                              100 * achieved / HBM_PEAK_GBS))
    lat.close()

    extras = {}
    if not args.no_extras:
        extras["ensemble_fss"] = bench_ensemble(torch, xyl, workloads, 200)
        log("ensemble:", extras["ensemble_fss"])
        extras["adjoint_512"] = bench_adjoint(torch, xyl, workloads)
        log("adjoint:", extras["adjoint_512"])
        extras["domains_2048"] = bench_domains(torch, xyl)
        log("domains:", extras["domains_2048"])

    cpu = None if args.no_cpu else cpu_baseline(L, args.cpu_steps)
    if cpu:
        log("cpu baseline:", cpu)
    line = {
        "metric": "site-updates/s at 4096^2 fp32 (% HBM roofline); adjoint/forward time ratio",
        "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single %dx%d periodic lattice, fp32 state, fp64 observables every %d steps"
                               % (L, L, args.every),
                   "L": L, "T": spec.schedule[0][1], "seed": spec.seed, "launch": list(launch)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "adjoint_512" in extras and "adjoint_over_forward" in extras["adjoint_512"]:
        line["adjoint_over_forward"] = extras["adjoint_512"]["adjoint_over_forward"]
    if "ensemble_fss" in extras:
        line["batched_over_per_replica"] = extras["ensemble_fss"]["speedup"]
    line["extras"] = extras
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
