#!/usr/bin/env python3
"""Benchmark of the Langevin-XY hot path on one MI355X.

Headline: site-updates/s of the FP32 fused BBK step on one 4096 x 4096
periodic lattice (J_x = 1, J_y = -0.1, h = 0.5, gamma = 1, dt = 0.01,
T = 0.3, seed 1) with the FP64 observables (energy, staggered order
parameter, structure-factor modes for the Binder cumulant and the
correlation length) fused into every 500th step.  One "step" is one BBK
step of the whole lattice.  The state is resident in HBM before timing.

Also reported on the same line:
  * roofline of the dominant kernel, the two-steps-per-pass FP32 kernel
    (k_step2: one launch advances every site two steps, reading angle and
    velocity once and writing both once, 16 B per site per launch): its
    average launch duration from HIP events on the lattice's stream around
    back-to-back launches; the VALU instructions per launch from rocprofv3
    counters (bound "alu": against the VALU issue rate of 256 CUs x 4 SIMDs
    at 2.4 GHz, one wave64 instruction per SIMD every 4 cycles) and the
    algorithmic HBM rate (16 B per site / duration, against 8 TB/s and the
    measured streaming ceiling of the same access shape); the single-step
    kernel measured the same way beside it;
  * HBM traffic per launch from rocprofv3 counters when the committed
    counter summary matches the current kernel source, else null;
  * batched-ensemble vs one-launch-per-replica throughput on the 288-replica
    finite-size-scaling ensemble (L = 32..512);
  * adjoint / forward time on the 512 x 512 differentiation workload;
  * frozen-domain labelling time on one 2048 x 2048 quench replica;
  * the directional structure factor (both axes) and Lorentzian correlation
    lengths of a 4096 x 4096 lattice;
  * the step kernel of the paper's Si(001) model variant on 4096 x 4096 and
    its 128-replica finite-size-scaling ensemble;
  * the FP64 CPU oracle timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs, each SIMD 16 lanes wide, so one
# wave64 VALU issue slot (4 cycles) per SIMD at a time, at 2.4 GHz
# (= 157.3 TFLOP/s FP32 / 2 flops per FMA / 2 for packed FP32 / 64 lanes), in
# G slots/s.  A full-rate instruction takes one slot, an FP32 transcendental
# two (measured: SQ_ACTIVE_INST_VALU = SQ_INSTS_VALU + SQ_INSTS_VALU_TRANS_F32).
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
BYTES_PER_SITE_F32 = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2_f32_4096_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "step2_f32_4096_valu.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the step kernels' code: the sources with comments and
    whitespace removed, so that only a change to the code itself marks the
    committed counter summaries as taken of another kernel."""
    import re
    h = hashlib.sha256()
    for f in ("xyl_step.hip", "xyl_device.hpp", "xyl_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2409_06412_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_profile(path, L, key):
    """A figure from a committed counter summary, if it was taken of the
    current kernel source at this lattice size, else None."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash() or t.get("L") != L:
        return None
    return t.get(key)


def time_steps(torch, lat, nsteps):
    """Average time per step of plain stepping, no graph, no measurement: HIP
    events on the lattice's stream (torch's current stream) around nsteps
    steps (a multiple of 4, so that with two steps per pass every launch is a
    two-step pass).  In ms."""
    assert nsteps % 4 == 0
    lat.set_graph_steps(0)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.step(8)
    e0.record(s)
    lat.step(nsteps)
    e1.record(s)
    e1.synchronize()
    lat.set_graph_steps(32)
    return e0.elapsed_time(e1) / nsteps


def step_kernels(torch, lat, L, nsteps):
    """Launch durations of the two stepping kernels on this lattice: the
    two-step pass where it applies (16 B per site per launch for two
    site-updates) and the single step (16 B per site per launch for one)."""
    sp, rows = lat.fusion()
    out = {}
    if rows:
        ms = time_steps(torch, lat, nsteps)
        us = 2e3 * ms
        gbs = BYTES_PER_SITE_F32 * L * L / (us * 1e-6) / 1e9
        _, tile_waves, tiles = lat.step2_shape()
        out["two_step"] = {"kernel": "k_step2_tiled" if tiles > 1 else "k_step2", "rows_per_strip": rows,
                           "tiles": tiles, "tile_waves": tile_waves,
                           "avg_kernel_us": us,
                           "us_per_step": 1e3 * ms, "site_updates_per_s": L * L / (ms * 1e-3),
                           "algorithmic_GBs": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS}
    lat.set_fusion(1)
    ms = time_steps(torch, lat, nsteps)
    lat.set_fusion(sp)
    gbs = BYTES_PER_SITE_F32 * L * L / (ms * 1e-3) / 1e9
    out["single_step"] = {"kernel": "k_step", "launch": list(lat.launch()), "avg_kernel_us": 1e3 * ms,
                          "site_updates_per_s": L * L / (ms * 1e-3), "algorithmic_GBs": gbs,
                          "frac_of_8TBs": gbs / HBM_PEAK_GBS}
    return out


def bench_ensemble(torch, xyl, workloads, nsteps, every=100):
    """The 288-replica FSS ensemble sampled every 100 steps, batched launches vs
    one launch per replica per step."""
    specs = workloads.fss_ensemble(nsteps=10 ** 9)
    out = {}
    for mode, name in ((0, "batched"), (1, "per_replica")):
        ens = xyl.Ensemble(specs, dtype="f32", stream=torch.cuda.current_stream().cuda_stream)
        ens.set_mode(mode)
        if mode == 0:
            ens.autotune()
        # the timed path once, from step 0 as the configuration runs (its
        # first chunks set up what they use); the timed call then starts on a
        # sample step, as every later stretch of the run does
        ens.step(every, every=every)
        ens.sync()
        t0 = time.perf_counter()
        ens.step(nsteps, every=every)
        ens.sync()
        out[name] = time.perf_counter() - t0
        if mode == 0:
            # a longer sampled run: its chunks repeat, so from the second one
            # on they replay as captured graphs
            t0 = time.perf_counter()
            ens.step(10 * every, every=every)
            ens.sync()
            out["batched_long"] = time.perf_counter() - t0
            out["batched_fusion"] = ens.fusion()
        ens.close()
    out.update(bench_solo_lattices(torch, xyl, specs, nsteps, every))
    sites = sum(s.Lx * s.Ly for s in specs)
    return {"replicas": len(specs), "sites": sites, "steps": nsteps, "sample_every": every,
            "batched_site_updates_per_s": sites * nsteps / out["batched"],
            "batched_%d_steps_site_updates_per_s" % (10 * every): sites * 10 * every / out["batched_long"],
            "batched_steps_per_pass": out["batched_fusion"],
            "per_replica_site_updates_per_s": sites * nsteps / out["per_replica"],
            "speedup": out["per_replica"] / out["batched"],
            # the replicas as separate lattices through the single-lattice path
            # (graph-captured steps): one after the other with their samples,
            # and all at once on a stream each (plain stepping, no samples)
            "solo_sequential_site_updates_per_s": sites * nsteps / out["solo_sequential"],
            "solo_concurrent_streams_site_updates_per_s": sites * nsteps / out["solo_concurrent"],
            "speedup_over_solo_sequential": out["solo_sequential"] / out["batched"],
            "speedup_over_solo_concurrent_streams": out["solo_concurrent"] / out["batched"]}


def bench_solo_lattices(torch, xyl, specs, nsteps, every):
    """The ensemble's replicas as separate single lattices: seconds for nsteps
    steps of every replica run one after the other, sampled every `every`
    steps, and for nsteps plain steps of all of them issued together, each
    lattice on a stream of its own (default priority)."""
    streams = [torch.cuda.Stream() for _ in specs]
    lats = []
    try:
        for sp, st in zip(specs, streams):
            lat = xyl.Lattice(sp.Lx, sp.Ly, dtype="f32", schedule=sp.schedule, seed=sp.seed, replica=sp.replica,
                              stream=st.cuda_stream, **sp.params())
            lat.init_random()
            lat.step(2 * every)          # captures the lattice's step graphs
            lats.append(lat)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lat in lats:
            lat.step_measured(nsteps, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for lat in lats:
            lat.step(nsteps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    finally:
        for lat in lats:
            lat.close()
    return {"solo_sequential": t1 - t0, "solo_concurrent": t2 - t1}


def bench_quench(torch, xyl, workloads, nsteps):
    """The 60-replica 2048^2 quench batch for a bounded number of steps, then
    the union-find labelling of one end state."""
    specs = workloads.kz_quench()
    ens = xyl.Ensemble(specs, dtype="f32", stream=torch.cuda.current_stream().cuda_stream)
    launch = ens.autotune()
    ens.step(2)
    ens.sync()
    t0 = time.perf_counter()
    ens.step(nsteps)
    ens.sync()
    t1 = time.perf_counter()
    sites = sum(s.Lx * s.Ly for s in specs)
    ens.close()
    return {"replicas": len(specs), "sites": sites, "steps": nsteps, "launch": list(launch),
            "site_updates_per_s": sites * nsteps / (t1 - t0),
            "full_run_site_updates": sum(s.Lx * s.Ly * s.nsteps for s in specs),
            # the whole batch (each replica's ramp and hold) at this rate
            "full_run_projected_s": sum(s.Lx * s.Ly * s.nsteps for s in specs) / (sites * nsteps / (t1 - t0))}


def bench_adjoint(torch, xyl, workloads):
    spec = workloads.adjoint_512()
    lat = xyl.Lattice(spec.Lx, spec.Ly, dtype="f32", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    try:
        lat.init_random()
        launch = lat.autotune()
        # one untimed gradient evaluation: captures the step and backward graphs,
        # which later evaluations of the same configuration reuse
        lat.adjoint_forward(spec.nsteps, 100, 1000)
        lat.adjoint_backward()
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
    lat.step(spec.nsteps)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    lat.close()
    return {"L": spec.Lx, "steps": spec.nsteps, "checkpoint_every": 100, "window": 1000, "launch": list(launch),
            "forward_with_loss_s": t1 - t0, "backward_s": t2 - t1, "plain_forward_s": t4 - t3,
            "adjoint_over_forward": (t2 - t1) / (t1 - t0),
            "adjoint_over_plain_forward": (t2 - t1) / (t4 - t3)}


def bench_copy(torch, nbytes=1 << 30, reps=20):
    """Plain device-to-device copy bandwidth (read + write bytes per second):
    the practical streaming ceiling beside the 8 TB/s peak."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_copied": nbytes, "ms": ms, "GBs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}


def bench_control_8192(torch, xyl, workloads, nlaunch=200):
    """An 8192^2 lattice (805 MB of state, larger than the 256 MB Infinity
    Cache): the HBM-resident rates of the single-step kernel and of the
    two-step pass, which runs there as column tiles of up to 16 waves with
    one-quad halos."""
    spec = workloads.large_fp32(0, 8192)
    lat = xyl.Lattice(8192, 8192, dtype="f32", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    lat.init_random()
    lat.autotune()
    out = step_kernels(torch, lat, 8192, nlaunch)
    lat.close()
    ceiling = xyl.stream_ceiling(8192 * 8192, 30)
    for k in out.values():
        k["stream_ceiling_GBs"] = ceiling
        k["frac_of_stream_ceiling"] = k["algorithmic_GBs"] / ceiling
    return {"L": 8192, **out}


def bench_si_4096(torch, xyl, workloads, nlaunch=500, launch=None):
    """Stepping kernels of the Si(001) model variant (q = 2, p = 2.5,
    half-circle angles) on 4096^2 at T_c: same bytes per site as the XY model,
    one more transcendental per site.  launch = (rows, waves) fixes the shape
    of the single-step kernel instead of autotuning."""
    spec = workloads.si_lattice(4096, 4096)
    lat = xyl.Lattice(4096, 4096, dtype="f32", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    lat.init_random()
    if launch:
        lat.set_launch(*launch)
        launch = lat.launch()
    else:
        launch = lat.autotune()
    lat.step(200)
    out = step_kernels(torch, lat, 4096, nlaunch)
    lat.close()
    return {"L": 4096, "model": "si", "p": spec.p, "T": spec.schedule[0][1], **out}


def bench_c1_temperatures(torch, xyl, workloads, nsteps=20000, every=500):
    """The single-lattice configuration at all eight of its temperatures
    (T = 0.3 .. 1.2), batched: eight 4096^2 FP32 replicas advanced together,
    energy and staggered order parameter every 500 steps, and the Binder
    cumulant of each temperature from its samples after the first 20%.  A
    bounded number of steps (the configuration runs 100,000); the rate is what
    the full run would proceed at."""
    specs = [workloads.large_fp32(j) for j in range(8)]
    ens = xyl.Ensemble(specs, dtype="f32", stream=torch.cuda.current_stream().cuda_stream)
    try:
        ens.autotune()
        # warm-up on the timed path from step 0 (the timed call starts on a
        # sample step, as the configuration's run does)
        ens.step(every, every=every)
        ens.sync()
        t0 = time.perf_counter()
        samples = ens.step(nsteps, every=every)
        ens.sync()
        dt = time.perf_counter() - t0
    finally:
        ens.close()
    sites = sum(sp.Lx * sp.Ly for sp in specs)
    rate = sites * nsteps / dt
    per_T = []
    for sp, smp in zip(specs, samples):
        m = smp[:, 2]
        try:
            U, se = xyl.binder(m, discard=len(m) // 5)
        except xyl.XylError:
            U, se = None, None
        per_T.append({"T": sp.schedule[0][1], "U": U, "U_se": se, "e_pot": float(smp[-1, 0]),
                      "m_s": float(m[-1]), "samples": int(len(m))})
    return {"replicas": len(specs), "L": 4096, "steps": nsteps, "sample_every": every, "site_updates_per_s": rate,
            "full_run_projected_s": sites * 100_000 / rate, "per_temperature": per_T}


def bench_fp64_4096(torch, xyl, workloads, nsteps=200):
    """The FP64 single-step kernel on the headline's lattice: 32 B per
    site-update (read theta, u; write theta', u' in binary64), against 8 TB/s.
    Its per-site arithmetic (FP64 sine, cosine, logarithm and square root in
    software) is the other bound."""
    spec = workloads.large_fp32(0, 4096)
    lat = xyl.Lattice(4096, 4096, dtype="f64", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    lat.init_random()
    launch = lat.autotune()
    lat.step(20)
    ms = time_steps(torch, lat, nsteps)
    lat.close()
    gbs = 32.0 * 4096 * 4096 / (ms * 1e-3) / 1e9
    return {"L": 4096, "dtype": "f64", "kernel": "k_step<double>", "launch": list(launch), "us_per_step": 1e3 * ms,
            "site_updates_per_s": 4096 * 4096 / (ms * 1e-3), "algorithmic_GBs": gbs,
            "frac_of_8TBs": gbs / HBM_PEAK_GBS}


def bench_si_fss(torch, xyl, workloads, nsteps=200, every=100):
    """The Si-model finite-size-scaling ensemble (128 replicas, L = 32..144),
    batched, sampled every 100 steps."""
    specs = workloads.si_fss_ensemble(nsteps=10 ** 9)
    ens = xyl.Ensemble(specs, dtype="f32", stream=torch.cuda.current_stream().cuda_stream)
    launch = ens.autotune()
    # warm-up on the timed path from step 0, so the timed call starts on a
    # sample step as the configuration's run does
    ens.step(every, every=every)
    ens.sync()
    t0 = time.perf_counter()
    ens.step(nsteps, every=every)
    ens.sync()
    t1 = time.perf_counter()
    ens.close()
    sites = sum(s.Lx * s.Ly for s in specs)
    return {"replicas": len(specs), "sites": sites, "steps": nsteps, "sample_every": every, "launch": list(launch),
            "site_updates_per_s": sites * nsteps / (t1 - t0)}


def bench_structure_factor(torch, xyl, workloads, reps=5):
    """S_delta(k) for k = 0..L/2 along both axes of a 4096^2 lattice (the
    paper's correlation-length observable, App. C), the Lorentzian xi of each
    axis, and the correlation function C_delta(r) for r = 0..L/2, on a lattice
    quenched for 1000 steps."""
    spec = workloads.large_fp32(0, 4096)
    lat = xyl.Lattice(4096, 4096, dtype="f32", schedule=spec.schedule, seed=spec.seed,
                      stream=torch.cuda.current_stream().cuda_stream, **spec.params())
    lat.init_random()
    lat.step(1000)
    out = {"L": 4096, "kmax": 2048}
    for axis, name in ((0, "x"), (1, "y")):
        lat.structure_factor(axis, 2048)
        t0 = time.perf_counter()
        for _ in range(reps):
            S = lat.structure_factor(axis, 2048)
        out["ms_" + name] = 1e3 * (time.perf_counter() - t0) / reps
        lat.correlation(axis, 2048)
        t0 = time.perf_counter()
        for _ in range(reps):
            C = lat.correlation(axis, 2048)
        out["corr_ms_" + name] = 1e3 * (time.perf_counter() - t0) / reps
        # nearest-neighbour correlation of the staggered field along this axis
        out["C1_over_C0_" + name] = float(C[1] / C[0])
        try:
            out["xi_" + name] = xyl.lorentzian_xi(S, 4096, 1, 64)[0]
        except xyl.XylError as e:
            # along y the rows couple through |Jy| = 0.1 only: xi is below one
            # spacing and S(k) over k = 1..64 is flat to within its sample noise
            out["xi_" + name] = None
            out["fit_" + name] = "no Lorentzian over k = 1..64 (%s)" % e
    lat.close()
    return out


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


def device_info(torch):
    """What the device reports about itself: torch's properties and `amd-smi
    static` (ASIC, memory and clock levels), beside the published peaks the
    roofline uses.  Fields amd-smi does not give are left out."""
    p = torch.cuda.get_device_properties(0)
    out = {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
           "memory_bytes": p.total_memory}
    try:
        r = subprocess.run(["amd-smi", "static", "--asic", "--vram", "--clock", "--json"], capture_output=True,
                           text=True, timeout=60)
        g = json.loads(r.stdout)["gpu_data"][0]
        asic, vram, clk = g.get("asic", {}), g.get("vram", {}), g.get("clock", {})
        smi = {"market_name": asic.get("market_name"), "compute_units": asic.get("num_compute_units"),
               "target": asic.get("target_graphics_version"), "vram_type": vram.get("type"),
               "vram_bit_width": vram.get("bit_width"),
               "vram_max_bandwidth_GBs": (vram.get("max_bandwidth") or {}).get("value")}
        levels = (clk.get("sys") or {}).get("frequency_levels") or {}
        mhz = [float(v.split()[0]) for v in levels.values() if v.split()[0].replace(".", "").isdigit()]
        if mhz:
            smi["sclk_max_MHz"] = max(mhz)
            if smi["compute_units"]:
                # one wave64 VALU instruction per SIMD every 4 cycles, 4 SIMDs per CU
                smi["valu_issue_peak_G_per_s"] = smi["compute_units"] * 4 * max(mhz) * 1e-3 / 4
        out["amd_smi"] = smi
    except Exception as e:          # amd-smi missing or its output not as expected
        out["amd_smi"] = {"error": repr(e)[:200]}
    return out


def cpu_baseline(L, nsteps):
    """The FP64 oracle on the host: the headline's lattice for a bounded number
    of steps on all the threads OpenMP uses, plus (informational) one thread on
    a smaller sample and the 64^2 FP64 acceptance run in full."""
    import oracle
    from paper_2409_06412_amd import workloads
    cores = oracle.max_threads()
    spec = workloads.large_fp32(0, L)
    o = oracle.Oracle(**spec.oracle_kwargs())
    th, om = o.init_random()
    t0 = time.perf_counter()
    o.run(th, om, 0, nsteps)
    dt = time.perf_counter() - t0
    out = {"value": L * L * nsteps / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
           "sample": "FP64 oracle, %dx%d lattice, %d BBK steps (%.1f s)" % (L, L, nsteps, dt)}
    # one thread, 1024^2 x 20 steps
    oracle.set_threads(1)
    try:
        o1 = oracle.Oracle(**workloads.large_fp32(0, 1024).oracle_kwargs())
        th1, om1 = o1.init_random()
        t0 = time.perf_counter()
        o1.run(th1, om1, 0, 20)
        out["single_thread"] = {"value": 1024 * 1024 * 20 / (time.perf_counter() - t0),
                                "sample": "1024x1024, 20 steps"}
    finally:
        oracle.set_threads(cores)
    # the small FP64 configuration in full: 64^2, 10,000 steps, observables every 100
    s0 = workloads.small_fp64()
    o0 = oracle.Oracle(**s0.oracle_kwargs())
    th0, om0 = o0.init_random()
    t0 = time.perf_counter()
    o0.run(th0, om0, 0, s0.nsteps, every=100)
    t = time.perf_counter() - t0
    out["small_fp64_full"] = {"seconds": t, "value": 64 * 64 * s0.nsteps / t,
                              "sample": "64x64, 10,000 steps, observables every 100"}
    out["host"] = host_info()
    return out


def host_info():
    """The host the oracle ran on: CPU model, logical CPUs, and those this
    process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


# ----------------------------------------------------------- profile summaries
STEP_KERNEL = "xyl::k_step<float, 1, 0>"   # single plain store step of the XY model
STEP2_KERNEL = "xyl::k_step2<0, false, false>"    # two steps per pass of the XY model (full waves)
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def summarize_trace(d, out_md, command):
    """Kernel statistics of a `rocprofv3 --kernel-trace --stats` run as markdown."""
    import csv
    files = _csvs(d, "kernel_stats.csv")
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % d)
    rows = list(csv.DictReader(open(files[0])))
    lines = ["# Kernel statistics: %s" % os.path.basename(out_md).replace(".md", ""), "",
             "Command (from the repository root):", "", "    " + command, "",
             "| kernel | calls | total (ms) | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:12]:
        name = r["Name"].replace("|", "/")
        lines.append("| %s | %s | %.3f | %.2f | %.2f | %.2f | %.1f%% |" % (
            name[:80], r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    open(out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_means(d, counter, L, kernel):
    """Mean counter value of the kernel at its most frequent grid and the
    largest value for plain device copies (the copy of one L*L*4-byte array)."""
    import csv
    from collections import defaultdict
    files = _csvs(d, "counter_collection.csv")
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    step = defaultdict(list)
    copy = []
    for r in csv.DictReader(open(files[0])):
        if r.get("Counter_Name") != counter:
            continue
        v = float(r["Counter_Value"])
        name = r["Kernel_Name"]
        if kernel in name:
            step[(r["Grid_Size"], r["Workgroup_Size"])].append(v)
        elif COPY_KERNEL in name and int(r["Grid_Size"]) > 4096:
            copy.append(v)
    key = max(step, key=lambda k: len(step[k]))
    return sum(step[key]) / len(step[key]), max(copy) if copy else None, key


def summarize_traffic(fetch_dir, write_dir, out_json, out_md, L, commands, kernel):
    """HBM traffic of one launch of the kernel from FETCH_SIZE and WRITE_SIZE,
    each scaled by what it reads for a plain copy of one 4*L*L-byte array."""
    nbytes = 4 * L * L
    f_step, f_copy, key = _counter_means(fetch_dir, "FETCH_SIZE", L, kernel)
    w_step, w_copy, _ = _counter_means(write_dir, "WRITE_SIZE", L, kernel)
    f_scale = nbytes / (f_copy * 1024.0)
    w_scale = nbytes / (w_copy * 1024.0)
    fetch_b = f_step * 1024.0 * f_scale
    write_b = w_step * 1024.0 * w_scale
    alg = BYTES_PER_SITE_F32 * L * L
    res = {"kernel": kernel, "L": L, "kernel_hash": kernel_source_hash(), "grid_workgroup": list(key),
           "fetch_kib_per_launch": f_step, "write_kib_per_launch": w_step,
           "copy_fetch_kib": f_copy, "copy_write_kib": w_copy, "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes": fetch_b, "write_bytes": write_b, "bytes_per_launch": fetch_b + write_b,
           "algorithmic_bytes": alg, "traffic_over_algorithmic": (fetch_b + write_b) / alg,
           "commands": commands}
    json.dump(res, open(out_json, "w"), indent=1)
    md = ["# HBM traffic of %s, %dx%d lattice" % (kernel, L, L), "",
          "Commands (from the repository root):", ""] + ["    " + c for c in commands] + [
          "", "| quantity | value |", "|---|---|",
          "| kernel FETCH_SIZE per launch (KiB) | %.0f |" % f_step,
          "| kernel WRITE_SIZE per launch (KiB) | %.0f |" % w_step,
          "| copy of %d B: FETCH_SIZE / WRITE_SIZE (KiB) | %.0f / %.0f |" % (nbytes, f_copy, w_copy),
          "| scale factors fetch / write | %.4f / %.4f |" % (f_scale, w_scale),
          "| scaled fetch + write per launch (MB) | %.1f + %.1f = %.1f |" % (fetch_b / 1e6, write_b / 1e6,
                                                                            (fetch_b + write_b) / 1e6),
          "| algorithmic bytes per launch (MB) | %.1f |" % (alg / 1e6),
          "| traffic / algorithmic | %.3f |" % ((fetch_b + write_b) / alg), ""]
    open(out_md, "w").write("\n".join(md))
    print("\n".join(md))


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F32", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE", "VALUBusy")


def summarize_valu(d, out_json, out_md, L, command, kernel):
    """VALU instructions per launch of the kernel (summed over the device) and
    the VALU busy fraction, from one rocprofv3 --pmc run."""
    import csv
    from collections import defaultdict
    files = _csvs(d, "counter_collection.csv")
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(files[0])):
        if kernel in r["Kernel_Name"] and r.get("Counter_Name") in VALU_COUNTERS:
            vals[(r["Grid_Size"], r["Workgroup_Size"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    key = max(vals, key=lambda k: len(vals[k]["SQ_INSTS_VALU"]))
    mean = {c: sum(v) / len(v) for c, v in vals[key].items()}
    res = {"kernel": kernel, "L": L, "kernel_hash": kernel_source_hash(), "grid_workgroup": list(key),
           "dispatches": len(vals[key]["SQ_INSTS_VALU"]),
           "valu_instructions_per_launch": mean["SQ_INSTS_VALU"],
           "transcendental_f32_per_launch": mean.get("SQ_INSTS_VALU_TRANS_F32"),
           "active_inst_valu_quad_cycles": mean.get("SQ_ACTIVE_INST_VALU"),
           "grbm_gui_active": mean.get("GRBM_GUI_ACTIVE"),
           "valu_busy_percent": mean.get("VALUBusy"),
           "valu_instructions_per_site_update": mean["SQ_INSTS_VALU"] * 64 / (L * L * (2 if "step2" in kernel else 1)),
           "command": command}
    json.dump(res, open(out_json, "w"), indent=1)
    md = ["# VALU work of %s, %dx%d lattice" % (kernel, L, L), "",
          "Command (from the repository root):", "", "    " + command, "",
          "| quantity | value |", "|---|---|",
          "| dispatches averaged | %d |" % res["dispatches"],
          "| SQ_INSTS_VALU per launch (wave instructions) | %.4g |" % res["valu_instructions_per_launch"],
          "| of which FP32 transcendental (SQ_INSTS_VALU_TRANS_F32) | %.4g |" % (res["transcendental_f32_per_launch"] or 0),
          "| lane-instructions per site-update (x 64 / site-updates per launch) | %.1f |"
          % res["valu_instructions_per_site_update"],
          "| SQ_ACTIVE_INST_VALU per launch (quad-cycles) | %.4g |" % (res["active_inst_valu_quad_cycles"] or 0),
          "| GRBM_GUI_ACTIVE per launch | %.4g |" % (res["grbm_gui_active"] or 0),
          "| VALUBusy (%%) | %.1f |" % (res["valu_busy_percent"] or 0), ""]
    open(out_md, "w").write("\n".join(md))
    print("\n".join(md))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--L", type=int, default=4096)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--kernel-steps", type=int, default=1000,
                    help="steps (a multiple of 4) over which each stepping kernel is timed alone")
    ap.add_argument("--only", type=str, default="",
                    help="comma list of extras to run alone (copy, ensemble, quench, adjoint, domains, control, "
                         "si, si_fss, structure); "
                         "prints their JSON and skips the headline measurement")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch rules instead of autotuning (for profiler runs, whose "
                         "serialised dispatches distort the autotuner's timings)")
    ap.add_argument("--launch", type=str, default="",
                    help="rows,waves: fixed launch shape of the step kernel (headline, and the si extra) "
                         "instead of autotuning")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DIR", "OUT_MD", "COMMAND"))
    ap.add_argument("--summarize-traffic", nargs=6,
                    metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON", "OUT_MD", "FETCH_CMD", "WRITE_CMD"))
    ap.add_argument("--summarize-valu", nargs=4, metavar=("DIR", "OUT_JSON", "OUT_MD", "COMMAND"))
    ap.add_argument("--kernel", type=str, default=STEP2_KERNEL,
                    help="kernel name the counter summaries select (default: the two-step pass)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_traffic:
        a = args.summarize_traffic
        summarize_traffic(a[0], a[1], a[2], a[3], args.L, [a[4], a[5]], args.kernel)
        return
    if args.summarize_valu:
        a = args.summarize_valu
        summarize_valu(a[0], a[1], a[2], args.L, a[3], args.kernel)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single MI355X "
              "(sharding across GPUs is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2409_06412_amd as xyl
    from paper_2409_06412_amd import workloads

    assert torch.cuda.is_available(), "no GPU visible"
    fixed = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    if args.only:
        runs = {"copy": lambda: bench_copy(torch),
                "ensemble": lambda: bench_ensemble(torch, xyl, workloads, 200),
                "quench": lambda: bench_quench(torch, xyl, workloads, 100),
                "adjoint": lambda: bench_adjoint(torch, xyl, workloads),
                "domains": lambda: bench_domains(torch, xyl),
                "control": lambda: bench_control_8192(torch, xyl, workloads),
                "si": lambda: bench_si_4096(torch, xyl, workloads, launch=fixed),
                "structure": lambda: bench_structure_factor(torch, xyl, workloads),
                "si_fss": lambda: bench_si_fss(torch, xyl, workloads),
                "fp64": lambda: bench_fp64_4096(torch, xyl, workloads),
                "c1": lambda: bench_c1_temperatures(torch, xyl, workloads)}
        print(json.dumps({k: runs[k]() for k in args.only.split(",")}), flush=True)
        return
    L = args.L
    spec = workloads.large_fp32(0, L)
    stream = torch.cuda.current_stream().cuda_stream
    lat = xyl.Lattice(L, L, dtype="f32", schedule=spec.schedule, seed=spec.seed, replica=spec.replica,
                      stream=stream, **spec.params())
    lat.init_random()
    # one plain device-to-device copy of a 4*L*L-byte array: the reference that
    # the HBM byte counters are scaled by when this run is profiled
    calib = lat.theta_tensor().clone()
    torch.cuda.synchronize()
    del calib
    if fixed:
        lat.set_launch(*fixed)
        launch = lat.launch()
    elif args.no_autotune:
        launch = lat.launch()
    else:
        launch = lat.autotune()
    fusion = lat.fusion()
    log("single-step launch shape (rows per strip, waves per workgroup):", launch,
        "; steps per pass, rows per strip of the two-step pass:", fusion)
    # the warm-up runs the timed path itself (samples and stepping), so that no
    # kernel is loaded or launched for the first time inside the timed region
    if args.warmup:
        lat.step_measured(args.warmup, args.every)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    samples = lat.step_measured(args.steps, args.every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = L * L * args.steps / wall
    log("timed %d steps in %.4f s: %.4g site-updates/s (%d samples)" % (args.steps, wall, value, len(samples)))

    # the stepping kernels timed alone (HIP events on the lattice's stream)
    kern = step_kernels(torch, lat, L, args.kernel_steps)
    lat.close()
    # the practical ceiling of the state's access shape: a plain stream reading
    # two and writing two arrays of L*L floats, ping-ponging like the state
    ceiling = xyl.stream_ceiling(L * L, 100)
    for k in kern.values():
        k["frac_of_stream_ceiling"] = k["algorithmic_GBs"] / ceiling
    two = kern.get("two_step")
    dom = two or kern["single_step"]
    us = dom["avg_kernel_us"]
    hbm = {"algorithmic_bytes_per_launch": BYTES_PER_SITE_F32 * L * L, "achieved_GBs": dom["algorithmic_GBs"],
           "peak_GBs": HBM_PEAK_GBS, "frac": dom["algorithmic_GBs"] / HBM_PEAK_GBS,
           "stream_ceiling_GBs": ceiling, "frac_of_stream_ceiling": dom["algorithmic_GBs"] / ceiling,
           # the rate a one-step-per-pass kernel could reach at 8 TB/s (16 B per
           # site-update), and this kernel's site-update rate over it
           "single_step_roofline_site_updates_per_s": HBM_PEAK_GBS * 1e9 / BYTES_PER_SITE_F32,
           "site_updates_over_single_step_roofline":
               dom["site_updates_per_s"] / (HBM_PEAK_GBS * 1e9 / BYTES_PER_SITE_F32)}
    traffic = load_profile(TRAFFIC_FILE, L, "bytes_per_launch") if two else None
    slots = load_profile(VALU_FILE, L, "active_inst_valu_quad_cycles") if two else None
    if slots:
        # VALU issue slots (one wave64 instruction = 4 cycles of a SIMD; the
        # transcendentals take two) per launch over the launch duration
        achieved = slots / (us * 1e-6) / 1e9
        roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GINST, "unit": "G VALU issue slots/s",
                    "frac": achieved / VALU_PEAK_GINST, "traffic": traffic,
                    "kernel": "k_step2<XY> (two steps per pass)", "avg_kernel_us": us,
                    "valu_issue_slots_per_launch": slots,
                    "valu_instructions_per_launch": load_profile(VALU_FILE, L, "valu_instructions_per_launch"),
                    "hbm": hbm}
    else:
        # no counter summary of the current kernel source: the HBM figure alone
        roofline = {"bound": "hbm", "achieved": dom["algorithmic_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": dom["algorithmic_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                    "kernel": dom["kernel"], "avg_kernel_us": us, "hbm": hbm,
                    "valu_profile": "absent or taken of another kernel source"}
    roofline["single_step_kernel"] = kern["single_step"]
    log("stepping kernels:", json.dumps(kern))
    log("roofline:", json.dumps(roofline))

    extras = {}
    if not args.no_extras:
        extras["ensemble_fss"] = bench_ensemble(torch, xyl, workloads, 200)
        log("ensemble:", extras["ensemble_fss"])
        extras["copy_1GiB"] = bench_copy(torch)
        log("copy:", extras["copy_1GiB"])
        extras["control_8192"] = bench_control_8192(torch, xyl, workloads)
        c = extras["control_8192"]["single_step"]
        c["frac_of_torch_copy"] = c["algorithmic_GBs"] / extras["copy_1GiB"]["GBs_read_plus_write"]
        log("8192^2 control:", extras["control_8192"])
        extras["quench_2048"] = bench_quench(torch, xyl, workloads, 100)
        log("quench:", extras["quench_2048"])
        extras["adjoint_512"] = bench_adjoint(torch, xyl, workloads)
        log("adjoint:", extras["adjoint_512"])
        extras["domains_2048"] = bench_domains(torch, xyl)
        log("domains:", extras["domains_2048"])
        extras["structure_factor_4096"] = bench_structure_factor(torch, xyl, workloads)
        log("structure factor:", extras["structure_factor_4096"])
        extras["si_4096"] = bench_si_4096(torch, xyl, workloads)
        log("si model 4096^2:", extras["si_4096"])
        extras["si_fss"] = bench_si_fss(torch, xyl, workloads)
        log("si model FSS ensemble:", extras["si_fss"])
        extras["fp64_4096"] = bench_fp64_4096(torch, xyl, workloads)
        log("fp64 4096^2:", extras["fp64_4096"])
        extras["c1_temperatures"] = bench_c1_temperatures(torch, xyl, workloads)
        log("4096^2 at eight temperatures:", extras["c1_temperatures"])

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
                   "L": L, "T": spec.schedule[0][1], "seed": spec.seed, "launch": list(launch),
                   "steps_per_pass": fusion[0], "rows_per_strip": fusion[1]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device": device_info(torch),
    }
    # the metric's "% HBM roofline": site-updates/s x 16 B per site-update over
    # 8 TB/s (above 100 when two steps share one pass over the state)
    line["pct_hbm_roofline"] = 100.0 * value * BYTES_PER_SITE_F32 / (HBM_PEAK_GBS * 1e9)
    if "adjoint_512" in extras and "adjoint_over_forward" in extras["adjoint_512"]:
        line["adjoint_over_forward"] = extras["adjoint_512"]["adjoint_over_forward"]
    if "ensemble_fss" in extras:
        line["batched_over_per_replica"] = extras["ensemble_fss"]["speedup"]
    if "copy_1GiB" in extras:
        hbm["frac_of_torch_copy"] = hbm["achieved_GBs"] / extras["copy_1GiB"]["GBs_read_plus_write"]
    line["extras"] = extras
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
