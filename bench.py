#!/usr/bin/env python3
"""Throughput of the 1D3V PIC/MCC step (push + deposit + MCC + Poisson + moments) on one
MI355X, in particle-steps/s, next to the FP64 CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--workload large|production|small|sweep|warmstart|mlp]

The default line is the large argon discharge (3 cm, 4096 cells, 2.5e7 particles per
species, dt = T_rf/4000), the largest single-GPU workload.  One step is one pass of the
whole hot path over every particle of the discharge; the periodic reordering runs inside
the timed steps (a window of K steps holds K / sort_every reorderings when K is a multiple
of sort_every).  Prints one JSON line.  Only one GPU is used; --gpus N > 1 exits with a
message.
"""
import os

# The CPU baseline runs the NumPy oracle on one core: the thread counts are fixed before
# anything imports numpy (the GPU path does not use host threads).
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import platform  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Nominal bytes per particle-step, the method's per-unit figure: the whole particle state
# read (x, vx, vy, vz, id: 20 B) and written (x, vx, vy, vz: 16 B).  The kernel moves less:
# only v_x feels the field, so v_y, v_z are written only after a real collision, and they
# are read only for electrons (the pre-test needs |v|) and for collision candidates.  Its
# minimum is therefore 28 B per electron step (read 20, write x, vx) and 20 B per ion step
# (read x, vx, id, write x, vx); the roofline reports the fraction on both, and the measured
# traffic beside them.
BYTES_PER_PARTICLE_STEP = 36
MIN_BYTES_ELECTRON_STEP = 28
MIN_BYTES_ION_STEP = 20
BYTES_NOTE = ("achieved and frac use the nominal 36 B per particle-step (the whole state read and written); "
              "achieved_min_bytes and frac_min_bytes use the kernel's minimum (28 B per electron step, 20 B per "
              "ion step); traffic is the copy-calibrated FETCH_SIZE + WRITE_SIZE per launch")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak


def workloads_by_name():
    import workloads as W
    return {"production": W.production_helium, "large": W.large_argon, "small": W.small_argon,
            "sweep": W.sweep_argon}


def kernel_source_sha():
    p = os.path.join(ROOT, "paper_1608_04601_amd", "csrc", "pic_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(workload_name, kernel="pass_kernel"):
    """HBM bytes per particle-step of the particle pass from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by what it reads for a plain device copy of
    known size), or None when the summary is absent or was taken on a different kernel
    source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_particle_step"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """The host's CPU model (lscpu's 'Model name', from /proc/cpuinfo) and os.cpu_count()."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(disc, steps, max_particles):
    """The oracle, unchanged, on the same discharge (gas, gap, cells, time step, voltage),
    loaded with at most max_particles per species so that the sample takes seconds: load,
    then `steps` timed steps.  The vectorised oracle's cost per particle-step does not
    depend on the count beyond cache effects, so the rate stands for the full discharge."""
    from oracle import Oracle
    n = min(disc.n_super[0], max_particles)
    sample = disc if n == disc.n_super[0] else disc.replace(n_super=(n, n), capacity=(2 * n, 2 * n))
    o = Oracle(sample)
    ps = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        ps += len(o.sp[0].x) + len(o.sp[1].x)
        o.step()
    dt = time.perf_counter() - t0
    model, ncpu = host_cpu()
    part = "all" if n == disc.n_super[0] else f"{n} of the {disc.n_super[0]}"
    return dict(value=ps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{disc.name}: FP64 NumPy oracle on one thread, {part} particles per species "
                       f"(same gas, gap, cells, time step), {steps} steps after the load, {dt:.1f} s",
                cpu_model=model, host_cpu_count=ncpu)


def copy_ceiling_gbs(torch, mib=1024, reps=5):
    """Bandwidth of a plain device copy of `mib` MiB (read + write), torch events."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def run_sweep(args, B, torch):
    """The batched parameter sweep: every discharge of the sweep advanced by one launch per
    step, whole RF periods replayed from one captured HIP graph each (the timed steps are
    rounded to whole periods).  Also times the batched launch alone, and the same discharges
    advanced one after the other (one launch each per step) for comparison."""
    discs = workloads_by_name()["sweep"]()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    bt = B.Batch(discs, stream=stream.cuda_stream)
    spp = int(round(1.0 / (discs[0].rf_frequency_Hz * discs[0].dt_s)))
    periods = max(1, int(round(args.steps / spp)))
    steps = periods * spp
    try:
        bt.step(args.warmup)
        tuning = bt.autotune(args.tune_steps) if args.tune_steps > 0 else None
        bt.set_graph(spp)
        bt.step(spp)   # captures the period's graph and replays it once
        bt.sync()
        c0 = sum(bt[k].counters()["particle_steps"] for k in range(len(bt)))
        r0 = bt.graph_launches()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        bt.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        bt.sync()
        replays = bt.graph_launches() - r0
        c1 = sum(bt[k].counters()["particle_steps"] for k in range(len(bt)))
        ps = c1 - c0
        value = ps / (ms * 1e-3)
        # duration of the batched launch alone (HIP events around each launch)
        alive = [bt[k].counters()["n_alive"] for k in range(len(bt))]
        units = float(sum(sum(a) for a in alive))
        min_bytes = sum(MIN_BYTES_ELECTRON_STEP * a[0] + MIN_BYTES_ION_STEP * a[1] for a in alive)
        bt.timing(True)
        bt.step(min(args.steps, 50))
        kern_ms, n_launch = bt.timing(False)
        achieved = BYTES_PER_PARTICLE_STEP * units / (kern_ms * 1e-3) / 1e9
        achieved_min = min_bytes / (kern_ms * 1e-3) / 1e9
        bpps = stored_traffic("sweep", "pass_batch_kernel")
        # the same discharges, each advanced alone (one launch per discharge per step)
        bt.sync()
        solo_steps = min(args.steps, 20)
        s0 = sum(bt[k].counters()["particle_steps"] for k in range(len(bt)))
        torch.cuda.synchronize()
        ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev2.record(stream)
        for k in range(len(bt)):
            B.pic_step(bt[k].h, solo_steps)
        ev3.record(stream)
        torch.cuda.synchronize()
        solo_ms = ev2.elapsed_time(ev3)
        s1 = sum(bt[k].counters()["particle_steps"] for k in range(len(bt)))
        solo_value = (s1 - s0) / (solo_ms * 1e-3)
    finally:
        bt.close()
    out = {
        "metric": "particle-steps/s (push+deposit+MCC)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup + spp,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"argon_sweep_{len(discs)}",
            "discharges": len(discs),
            "particles_per_species_initial_total": int(sum(d.n_super[0] for d in discs)),
            "cells_min": int(min(d.n_cells for d in discs)),
            "cells_max": int(max(d.n_cells for d in discs)),
            "alive_particles_mean": ps / steps,
            "steps_per_rf_period": spp,
        },
        "rf_cycles_per_s": periods / (ms * 1e-3),
        "graph": {"steps_per_graph": spp, "replays_timed": replays},
        "tuning": tuning,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if bpps is None else bpps * units,
            "traffic_unit": "B per launch",
            "traffic_GBs": None if bpps is None else bpps * units / (kern_ms * 1e-3) / 1e9,
            "achieved_min_bytes": achieved_min,
            "frac_min_bytes": achieved_min / HBM_PEAK_GBS,
            "kernel": "pass_batch_kernel (fused complete+advance, all discharges)",
            "kernel_ms_mean": kern_ms,
            "launches_timed": n_launch,
            "bytes_per_particle_step": BYTES_PER_PARTICLE_STEP,
            "bytes_note": BYTES_NOTE,
        },
        "solo_sequential": {"value": solo_value, "unit": "particle-steps/s", "steps": solo_steps,
                            "note": "each discharge advanced alone, one launch per discharge per step"},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_warmstart(args, B, torch):
    """RF periods to the periodic steady state, warm (surrogate) against cold (uniform)
    start: the network is trained on the GPU from stored steady states of the batched PIC
    (parameter draws of seeds 1 and 3 to 9), then held-out draws (seed 2) run cold and warm in one batch
    until the steady-state criterion holds (or the period limit)."""
    import numpy as np

    import workloads as W
    from paper_1608_04601_amd import warmstart as WS
    torch.cuda.set_device(0)
    data = WS.load_data()
    keep = WS.training_mask(data)
    t0 = time.time()
    net, norm, loss = WS.train(data["params"][keep], data["profiles"][keep], steps=4000)
    train_s = time.time() - t0
    t1 = time.time()
    if args.ws_target == "production":
        # the production helium discharge at full fidelity (512 cells, 1e6 particles per
        # species, T_rf/2000), storage for 4x its initial count
        disc = W.production_helium().replace(capacity=(4_000_000, 4_000_000))
        rows = [WS.evaluate_discharge(net, norm, disc, 1, args.ws_periods,
                                      log=lambda m: print(m, file=sys.stderr, flush=True))]
    elif args.ws_target == "large":
        # the large argon discharge (4096 cells, T_rf/4000) weighted for --ws-particles
        # particles per species in its periodic state (2.5e7 at full size)
        disc = W.large_argon_periodic(n_periodic=args.ws_particles)
        rows = [WS.evaluate_discharge(net, norm, disc, 0, args.ws_periods,
                                      log=lambda m: print(m, file=sys.stderr, flush=True),
                                      max_seconds=args.ws_seconds, continue_to=args.ws_continue)]
    else:
        params = W.surrogate_params(args.ws_n, 2)
        rows = WS.evaluate(net, norm, params, 2, args.ws_periods,
                           log=lambda m: print(m, file=sys.stderr, flush=True))
    eval_s = time.time() - t1
    sm = WS.summarize(rows, args.ws_periods)
    config = {"workload": disc.name if args.ws_target != "heldout" else f"surrogate_heldout_{args.ws_n}",
              "training_steady_states": int(keep.sum()), "period_limit": args.ws_periods}
    if args.ws_target == "heldout":
        config.update(cells=128, steps_per_rf_period=1000, particles_per_species_initial=20000)
    else:
        config.update(cells=disc.n_cells, steps_per_rf_period=int(round(1.0 / (disc.rf_frequency_Hz * disc.dt_s))),
                      particles_per_species_initial=disc.n_super[0])
        if args.ws_target == "large":
            config.update(particles_per_species_periodic=args.ws_particles, time_limit_s=args.ws_seconds,
                          continue_to_period=args.ws_continue)
    if args.ws_out:
        with open(args.ws_out, "w") as f:
            json.dump(dict(summary=sm, rows=rows), f, indent=1)
    out = {
        "metric": "RF cycles to steady state, warm vs cold",
        "value": sm["warm_periods_mean"],
        "unit": "RF periods (warm start, mean)",
        "n_gpus": 1,
        "higher_is_better": False,
        "cold_periods_mean": sm["cold_periods_mean"],
        "reduction": (sm["cold_periods_mean"] / sm["warm_periods_mean"]) if sm["warm_periods_mean"] else None,
        "vs_baseline": None,
        "dtype": "f32 particles, bf16 network",
        "data": "synthetic",
        "config": config,
        "summary": sm,
        "train_s": train_s,
        "train_loss": loss,
        "evaluate_s": eval_s,
    }
    print(json.dumps(out), flush=True)


def run_mlp(args, B, torch):
    """Throughput of the surrogate network's kernels on the matrix cores (BF16 operands, FP32
    accumulation): the forward pass of 65536 samples (one launch for all layers, activations
    in LDS) and a training step (forward, reverse pass, Adam: layer-by-layer GEMMs with fused
    epilogues) on 8192 samples, 4 -> 3 x 256 -> 640, timed with torch events on the library's
    stream."""
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    dims = [4, 256, 256, 256, 640]
    flop_fwd = 2.0 * sum(dims[i] * dims[i + 1] for i in range(4))   # per sample
    res = {}
    for name, batch, reps in (("forward", 65536, 20), ("train_step", 8192, 20)):
        net = B.Mlp(4, 256, 3, 640, max_batch=batch, seed=1, stream=stream.cuda_stream)
        x = torch.rand(batch, 4, device="cuda") * 2 - 1
        t = torch.rand(batch, 640, device="cuda")
        y = torch.empty(batch, 640, device="cuda")
        run = (lambda: net.forward(x, y)) if name == "forward" else (lambda: net.train_step(x, t, 1e-4))
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flop = flop_fwd * batch * (1 if name == "forward" else 3)   # backward: two GEMMs per layer
        res[name] = {"batch": batch, "ms": ms, "TFLOP_s": flop / (ms * 1e-3) / 1e12}
        net.close()
    # algorithmic bytes of the forward pass per sample: the FP32 input read and the FP32 output
    # written; the activations stay in LDS, and the weights (0.6 MB, read from L2 by every
    # workgroup) are negligible in HBM at this batch
    bytes_fwd = 4 * dims[0] + 4 * dims[4]
    fwd = res["forward"]
    gbs = bytes_fwd * fwd["batch"] / (fwd["ms"] * 1e-3) / 1e9
    ai = flop_fwd / bytes_fwd
    out = {
        "metric": "surrogate network throughput (BF16 MFMA, FP32 accumulate)",
        "value": fwd["TFLOP_s"],
        "unit": "TFLOP/s (forward)",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "mlp_4x256x3x640", "flop_per_sample_forward": flop_fwd,
                   "bytes_per_sample_forward": bytes_fwd, "flop_per_byte": ai},
        # below the ridge (2500 TFLOP/s / 8 TB/s = 312 FLOP/B) the forward pass is bound by HBM
        "roofline": {"bound": "hbm" if ai < MFMA_BF16_PEAK_TFLOPS / HBM_PEAK_GBS * 1e3 else "mfma",
                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "mfma_frac": fwd["TFLOP_s"] / MFMA_BF16_PEAK_TFLOPS},
        "train_step": res["train_step"],
        "forward": fwd,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="large", choices=sorted(workloads_by_name()) + ["warmstart", "mlp"])
    ap.add_argument("--ws-n", type=int, default=16, help="warmstart: held-out discharges")
    ap.add_argument("--ws-periods", type=int, default=1500, help="warmstart: RF period limit")
    ap.add_argument("--ws-out", default=None, help="warmstart: write every discharge's result (JSON)")
    ap.add_argument("--ws-particles", type=int, default=25_000_000,
                    help="warmstart --ws-target large: particles per species in the periodic state")
    ap.add_argument("--ws-seconds", type=float, default=None,
                    help="warmstart --ws-target large: stop the runs after this many seconds")
    ap.add_argument("--ws-continue", type=int, default=None,
                    help="warmstart --ws-target large: keep both runs going to this period after they are "
                         "steady, and compare their final windows there")
    ap.add_argument("--ws-target", default="heldout", choices=("heldout", "production", "large"),
                    help="warmstart: held-out draws of the training family, the production discharge, "
                         "or the large one")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU baseline (0: 3 for the large discharge, else 100)")
    ap.add_argument("--cpu-particles", type=int, default=4_000_000,
                    help="CPU baseline: at most this many particles per species of the same discharge")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch-blocks", type=int, default=0)
    ap.add_argument("--tune-steps", type=int, default=100,
                    help="sweep: steps per autotuning trial before timing (0: keep the default schedule)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this size (5 launches), to calibrate "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE readings against known bytes")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_04601_amd import binding as B

    if args.workload == "warmstart":
        run_warmstart(args, B, torch)
        return
    if args.workload == "mlp":
        run_mlp(args, B, torch)
        return
    if args.workload == "sweep":
        run_sweep(args, B, torch)
        return
    disc = workloads_by_name()[args.workload]()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    d = B.Discharge(disc, stream=stream.cuda_stream, launch_blocks=args.launch_blocks)
    try:
        d.step(args.warmup)
        d.sync()
        c0 = d.counters()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        d.step(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        c1 = d.counters()
        ps = c1["particle_steps"] - c0["particle_steps"]
        value = ps / (ms * 1e-3)

        # kernel duration of the particle pass, HIP events around each launch on its stream
        B.pic_timing(d.h, True)
        k_steps = min(args.steps, 200)
        c2 = d.counters()
        d.step(k_steps)
        kern_ms, n_launch = B.pic_timing(d.h, False)
        c3 = d.counters()
        units = (c3["particle_steps"] - c2["particle_steps"]) / max(k_steps, 1)
        achieved = BYTES_PER_PARTICLE_STEP * units / (kern_ms * 1e-3) / 1e9
        # minimum bytes at the mean of the species counts before and after the timed launches
        min_bytes = sum(b * 0.5 * (c2["n_alive"][s] + c3["n_alive"][s])
                        for s, b in enumerate((MIN_BYTES_ELECTRON_STEP, MIN_BYTES_ION_STEP)))
        achieved_min = min_bytes / (kern_ms * 1e-3) / 1e9
        _, _, dynamic = d.launch_shape()
        kernel = "pass_dyn_kernel" if dynamic else "pass_kernel"
        bpps = stored_traffic(args.workload, kernel)
        traffic = None if bpps is None else bpps * units   # bytes per launch at this launch's size
    finally:
        d.close()
    copy_gbs = copy_ceiling_gbs(torch)
    # reorderings inside the timed window: after every sort_every-th step since the load
    se = disc.sort_every
    sorts_timed = (args.warmup + args.steps) // se - args.warmup // se if se > 0 else 0

    cpu = None
    if not args.no_cpu_baseline:
        steps_cpu = args.cpu_steps or (3 if disc.n_cells >= 4096 else 100)
        cpu = cpu_baseline(disc, steps_cpu, args.cpu_particles)

    spp = disc.steps_per_period
    out = {
        "metric": "particle-steps/s (push+deposit+MCC)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": disc.name,
            "particles_per_species_initial": int(disc.n_super[0]),
            "cells": disc.n_cells,
            "dt_s": disc.dt_s,
            "steps_per_rf_period": spp,
            "sort_every": disc.sort_every,
            "reorderings_timed": sorts_timed,
            "moments_every": disc.moments_every,
            "alive_particles_mean": ps / args.steps,
        },
        "rf_cycles_per_s": (args.steps / (ms * 1e-3)) / spp,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "B per launch",
            "traffic_GBs": None if traffic is None else traffic / (kern_ms * 1e-3) / 1e9,
            "frac_traffic": None if traffic is None else traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "kernel": kernel + " (fused complete+advance" + (", dynamic work distribution)" if dynamic else ")"),
            "kernel_ms_mean": kern_ms,
            "launches_timed": n_launch,
            "achieved_min_bytes": achieved_min,
            "frac_min_bytes": achieved_min / HBM_PEAK_GBS,
            "bytes_per_particle_step": BYTES_PER_PARTICLE_STEP,
            "bytes_note": BYTES_NOTE,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
