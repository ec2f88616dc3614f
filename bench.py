"""Throughput of the per-step update of a plastic network of multi-compartment
neurons on one MI355X.

Workload (default): 2000 ball-and-stick cells with 100-CV dendrites (HH soma
+ 100 passive dendrite CVs, 202,000 CVs), 1600 excitatory / 400 inhibitory,
Bernoulli(0.1) connectivity with 3 ms delays, ~255k plastic (calcium +
tagging-and-capture) E->E synapses and ~146k static ones, 25 x 5 Hz Poisson
inputs per cell, dt = 0.2 ms, seeded synthetic data (no dataset), in the
batched form with mixed precision.  A bench "step" is one time step of the
whole network (event gathering and delivery, currents, cable solve,
mechanisms, plasticity, detection).  Before the warmup the network runs
--settle steps (untimed) from rest into its firing regime.

    python bench.py [--steps 5000] [--warmup 500] [--form batched-mixed]

Prints one JSON line.  value = CV-steps/s of the headline form over the
timed steps; the plain FP64 form and the batched FP64 form run the same
steps for the comparison at equal spikes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# Algorithmic HBM bytes per unit and step (streaming model: state read and
# written once per step, invariants read once), FP64 / mixed.
ALG_BYTES = {
    "cv": (36.0, 36.0),        # V r/w 16, axial 8, C/dt (with g_pas folded) 8, branch-table share 4
    "hh": (48.0, 24.0),        # m, h, n r/w
    "stc": (68.0, 52.0),       # g, c, h, z r/w + CV index 4 (g, c FP32 in the mixed form)
    "static": (20.0, 12.0),    # g r/w + CV index 4
    "cell": (16.0, 16.0),      # p r/w
}


def _alg_bytes_per_launch(form: str, s: dict, steps_per_launch: float) -> float:
    """Algorithmic bytes of one launch of the dominant kernel: the per-unit
    figures of ALG_BYTES times the units one step touches, times the steps
    one launch advances.  The plain form's dominant kernel is the
    synapse-update kernel (one step, synapse units only)."""
    m = 1 if form.endswith("mixed") else 0
    n_stc, n_static = s["n_stc"], s["n_syn"] - s["n_stc"]
    syn = n_stc * ALG_BYTES["stc"][m] + n_static * ALG_BYTES["static"][m]
    if form.startswith("plain"):
        return syn * steps_per_launch
    n_hh = s["n_hh"]
    per_step = (s["n_cv"] * ALG_BYTES["cv"][m] + n_hh * ALG_BYTES["hh"][m] + syn
                + s["n_cells"] * ALG_BYTES["cell"][m])
    return per_step * steps_per_launch


def run_form(net, form, steps, warmup, settle=0, time_kernel=True, plan=None):
    import torch

    from paper_2411_16445_amd import Simulation
    mode, prec = form.split("-")
    t_setup = time.perf_counter()
    sim = Simulation(net, mode=mode, precision={"fp64": "fp64", "mixed": "mixed"}[prec],
                     **(plan if mode == "batched" and plan else {}))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    st = sim.stats()
    st["n_hh"] = sim.n_hh
    retune_s = 0.0
    if settle:
        sim.advance_steps(settle)
        if mode == "batched" and not plan:
            # the plan timed again in the regime the timed steps run in
            t_rt = time.perf_counter()
            sim.retune()
            torch.cuda.synchronize()
            retune_s = time.perf_counter() - t_rt
    sim.advance_steps(warmup)
    sp0 = sim.stats()["spikes"]
    if time_kernel:
        sim.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.advance_steps(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st2 = sim.stats()
    out = dict(form=form, seconds=el, setup_s=t_setup, retune_s=retune_s, ms_per_step=1e3 * el / steps, spikes=st2["spikes"] - sp0,
               cv_steps_per_s=st["n_cv"] * steps / el,
               synapse_updates_per_s=st["n_syn"] * steps / el,
               stc_synapse_updates_per_s=st["n_stc"] * steps / el,
               epoch_steps=st["epoch_steps"], cells_per_block=st2["cells_per_block"],
               block_threads=st2["block_threads"], solver_waves=st2["solver_waves"],
               exchange={1: "kernel", 2: "resident"}.get(st2["exchange"], "-"))
    if time_kernel:
        # launches of the dominant kernel may cover unequal step counts (a
        # resident launch runs up to 256 epochs): the achieved rate is the
        # algorithmic bytes of all timed steps over the summed launch times
        ms, launches, name = sim.kernel_time()
        avg_ms = ms / max(1, launches)
        spl = steps / max(1, launches)
        alg = _alg_bytes_per_launch(form, st, spl)
        alg_step = _alg_bytes_per_launch(form, st, 1.0)
        achieved = alg_step * steps / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out["kernel"] = dict(name=name, launches=launches, avg_us=avg_ms * 1e3,
                             us_per_step=ms * 1e3 / steps, steps_per_launch=spl,
                             alg_bytes_per_launch=alg, alg_bytes_per_step=alg_step,
                             achieved_gbs=achieved, share_of_time=ms / (el * 1e3))
    out["stats"] = st
    sim.close()
    return out


def _oracle_rate(net, budget_s, threaded, min_steps=1):
    """Steps the oracle from the network's start in chunks until budget_s of
    CPU time has passed; returns (CV-steps/s, steps, seconds, spikes)."""
    import oracle
    o = oracle.Oracle(net, threaded=threaded)
    done, el, chunk = 0, 0.0, 1
    while el < budget_s or done < min_steps:
        t0 = time.perf_counter()
        o.run(chunk)
        el += time.perf_counter() - t0
        done += chunk
        if el < 0.25 * budget_s:
            chunk *= 2
    return o.n_cv * done / el, done, el, int(o.spikes()[0].size)


def copy_bandwidth(mib=1024, reps=5):
    """Measured HBM bandwidth of a plain device-to-device copy (bytes read
    plus bytes written over the copy's time, best of reps), the practical
    ceiling beside the 8 TB/s peak.  Runs before any simulation kernel, so a
    profiled run's copy probe (after the timed launches) stays apart."""
    import torch
    x = torch.empty(mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    del x, y
    return 2 * mib * 1024 * 1024 / (best * 1e-3) / 1e9


def cpu_baseline(net, budget_s):
    """The plain FP64 oracle on the host: single-threaded (the oracle as it
    stands) and, as a second figure, its OpenMP build on every host core
    (same expressions and order per value)."""
    rate, steps, el, spikes = _oracle_rate(net, budget_s, threaded=False)
    cores = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    rate_n, steps_n, el_n, _ = _oracle_rate(net, budget_s / 2, threaded=True)
    return dict(value=rate, unit="CV-steps/s", cores=1, kind="oracle",
                sample=f"first {steps} steps ({steps * net['dt']:.1f} ms, {spikes} spikes) of the same network "
                       f"with its inputs, single-threaded plain FP64 C oracle, {el:.1f} s",
                multi_core=dict(value=rate_n, unit="CV-steps/s", cores=cores, kind="oracle (OpenMP build)",
                                sample=f"first {steps_n} steps, {el_n:.1f} s"))


# workloads: name in the JSON line, network builder
WORKLOADS = {"ei2000x21": ("ei-ball-and-stick-2000x21cv", "config2"),
             "ei2000x101": ("ei-ball-and-stick-2000x101cv", "config4"),
             "trees4096": ("uneven-trees-4096x10-300cv", "config3"),
             "large1e5": ("random-trees-1e5x10-60cv-1e7-plastic", "config5"),
             "morpho2000": ("ei-table6-neurons-2000x31cv-sps-prp-diffusion", "stc_morpho_network"),
             "busyring": ("busyring", "busyring"),
             "dpcurve": ("graupner-brunel-dp-curve-41x4000-trials", None)}

DATA = {
    "ei2000x21": "synthetic (seeded E/I network shaped like the paper's 2000-neuron STC network, 20-CV dendrites; "
                 "{settle} untimed settling steps from rest)",
    "ei2000x101": "synthetic (seeded E/I network shaped like the paper's 2000-neuron STC network, 100-CV dendrites; "
                  "{settle} untimed settling steps from rest)",
    "trees4096": "synthetic (seeded random trees of 10-300 CVs with HH somata, 100 plastic synapses per cell; "
                 "{settle} untimed settling steps from rest)",
    "large1e5": "synthetic (seeded random trees of 10-60 CVs, in-degree 100 onto plastic synapses, device Poisson "
                "input; {settle} untimed settling steps from rest)",
    "morpho2000": "synthetic (seeded E/I network of the paper's Table 6 neurons with SPS/PRP diffusion; "
                  "{settle} untimed settling steps from rest)",
    "busyring": "synthetic (seeded busyring of {cells} cells, tree depth {depth}, {kind} synapses on 1000 "
                "zero-weight connections per cell)",
    "dpcurve": "synthetic (Graupner-Brunel pairing protocol trials)",
}

# The paper's own propagation times of the busyring benchmark over 200 ms
# (Table 9, one NVIDIA T1000 GPU; context only, other hardware), seconds:
# (cells, depth) -> (exponential synapses, STDP synapses)
BUSYRING_T1000_S = {(1024, 0): (0.30, 0.78), (1024, 2): (0.41, 1.00), (1024, 10): (2.99, 3.50),
                    (16384, 0): (2.81, 10.44), (16384, 2): (4.15, 12.04), (16384, 10): (40.45, 49.05),
                    (32768, 0): (5.30, 20.47), (32768, 2): (7.78, 23.71), (32768, 10): (80.44, 97.75)}


def dp_curve_bench(args):
    """The Graupner-Brunel DP-curve batch (41 delays x 4000 trials, 60 pairs
    at 1 Hz, dt 0.5 ms) as one launch of pa_gb_trials: synapse-steps/s, and
    the oracle on a sample of trials for the CPU baseline."""
    import numpy as np
    import torch

    import netgen
    from paper_2411_16445_amd import binding as B
    delays = np.repeat(np.linspace(-100.0, 100.0, 41), 4000)
    w0 = np.tile(np.r_[np.zeros(2000), np.ones(2000)], 41)
    d = torch.tensor(delays, dtype=torch.float64, device="cuda")
    w = torch.tensor(w0, dtype=torch.float64, device="cuda")
    steps = int(np.floor((100.0 + 60 * 1000.0) / 0.5))
    for _ in range(max(1, args.warmup and 1)):
        B.gb_trials(netgen.GB_TABLE3, 0.5, d, w, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 1000)
    for k in range(reps):
        wf, _ = B.gb_trials(netgen.GB_TABLE3, 0.5, d, w, seed=1 + k)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    rate = delays.size * steps / el
    cpu = None
    if not args.no_cpu:
        import oracle
        n = 40
        t1 = time.perf_counter()
        oracle.gb_trials(netgen.GB_TABLE3, 0.5, delays[:n], w0[:n], seed=1)
        el_c = time.perf_counter() - t1
        cpu = dict(value=n * steps / el_c, unit="synapse-steps/s", cores=1, kind="oracle",
                   sample=f"{n} of the batch's trials, single-threaded plain FP64 C oracle, {el_c:.1f} s")
    m = wf.cpu().numpy().reshape(41, 4000).mean(1)
    line = {"metric": "Graupner-Brunel DP-curve batch throughput", "value": rate, "unit": "synapse-steps/s",
            "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": el * 1e3 / steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (pairing protocol)",
            "config": {"workload": "graupner-brunel-dp-curve-41x4000-trials", "trials": int(delays.size),
                       "pairs": 60, "dt_ms": 0.5, "parallelism": "single-gpu"},
            "seconds_per_batch": el, "dp_curve_mean_w": [round(float(x), 4) for x in m],
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--settle", type=int, default=1000,
                    help="untimed steps from rest into the firing regime before the warmup")
    ap.add_argument("--form", default=os.environ.get("PA_BENCH_FORM", "batched-mixed"),
                    choices=["plain-fp64", "plain-mixed", "batched-fp64", "batched-mixed"])
    ap.add_argument("--no-compare", action="store_true", help="skip the plain and batched FP64 runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU time of the single-threaded oracle sample (the OpenMP sample takes half)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plan", default="",
                    help="fix the batched form's plan instead of autotuning it: "
                         "CELLS_PER_BLOCK,BLOCK_THREADS,SOLVER_WAVES,EXCHANGE (kernel|resident)")
    ap.add_argument("--workload", default="ei2000x101", choices=sorted(WORKLOADS),
                    help="ei2000x101: the headline network (100-CV dendrites); ei2000x21: 20-CV dendrites; "
                         "trees4096: 4096 random trees of 10-300 CVs; large1e5: 1e5 random trees of 10-60 CVs")
    ap.add_argument("--ring-cells", type=int, default=16384, help="busyring: cells (rings of 4)")
    ap.add_argument("--ring-depth", type=int, default=2, help="busyring: dendritic tree depth")
    ap.add_argument("--ring-stdp", action="store_true", help="busyring: STDP synapses on the random connections")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the runs, copy this many MiB device to device (a plain copy kernel of known "
                         "size that scales rocprofv3's FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "dpcurve":
        dp_curve_bench(args)
        return
    copy_gbs = copy_bandwidth()
    import netgen
    # inputs over everything that runs: settle, warmup, timed steps and the
    # oracle's sample
    t_end = (args.settle + args.warmup + args.steps + 5000) * 0.2
    wname, make = WORKLOADS[args.workload]
    if args.workload == "busyring":
        net = netgen.busyring(n_cells=args.ring_cells, depth=args.ring_depth, stdp=args.ring_stdp,
                              t_end=(args.settle + args.warmup + args.steps + 100) * 0.025)
        wname = net["name"]
    else:
        net = getattr(netgen, make)(t_end=t_end)
    print(f"[bench] network {netgen.summary(net)}", file=sys.stderr, flush=True)
    plan = None
    if args.plan:
        cpb, bt, sw, xm = args.plan.split(",")
        plan = dict(cells_per_block=int(cpb), block_threads=int(bt), solver_waves=int(sw), exchange=xm)
    head = run_form(net, args.form, args.steps, args.warmup, args.settle, plan=plan)
    print(f"[bench] {args.form}: {head['ms_per_step']*1e3:.2f} us/step, {head['spikes']} spikes",
          file=sys.stderr, flush=True)
    ref = bfp = None
    if not args.no_compare and args.form != "plain-fp64":
        ref = run_form(net, "plain-fp64", args.steps, args.warmup, args.settle)
        print(f"[bench] plain-fp64: {ref['ms_per_step']*1e3:.2f} us/step, {ref['spikes']} spikes",
              file=sys.stderr, flush=True)
    if not args.no_compare and args.form == "batched-mixed":
        bfp = run_form(net, "batched-fp64", args.steps, args.warmup, args.settle)
        print(f"[bench] batched-fp64: {bfp['ms_per_step']*1e3:.2f} us/step, {bfp['spikes']} spikes",
              file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(net, args.cpu_seconds)
        print(f"[bench] cpu oracle: {cpu['value']:.3e} CV-steps/s", file=sys.stderr, flush=True)
    if args.copy_probe_mib:
        import torch
        x = torch.ones(args.copy_probe_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    k = head.get("kernel", {})
    from paper_2411_16445_amd.profiling import traffic_for_bench
    traffic, traffic_src = traffic_for_bench(os.path.join(ROOT, "profiles"), k.get("name") or "", args.workload)
    line = {
        "metric": "CV-steps/s + synapse-updates/s, mixed+batched vs plain FP64 at equal spikes",
        "value": head["cv_steps_per_s"],
        "unit": "CV-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.form.endswith("mixed") else "f64",
        "data": DATA[args.workload].format(settle=args.settle, cells=args.ring_cells, depth=args.ring_depth,
                                           kind="STDP" if args.ring_stdp else "exponential"),
        "config": {"workload": wname, "cells": head["stats"]["n_cells"],
                   "cvs": head["stats"]["n_cv"], "synapses": head["stats"]["n_syn"],
                   "stc_synapses": head["stats"]["n_stc"], "dt_ms": net["dt"], "form": args.form,
                   "epoch_steps": head["epoch_steps"], "cells_per_block": head["cells_per_block"],
                   "block_threads": head["block_threads"], "solver_waves": head["solver_waves"],
                   "exchange": head["exchange"], "settle_steps": args.settle, "parallelism": "single-gpu"},
        # setup (network upload, pa_finalize, plan autotuning) apart from
        # the timed propagation, as the paper splits them
        "setup_s": head["setup_s"],
        # the plan timed again after the settling steps (pa_retune)
        "retune_s": head["retune_s"],
        "synapse_updates_per_s": head["synapse_updates_per_s"],
        "stc_synapse_updates_per_s": head["stc_synapse_updates_per_s"],
        "spikes": head["spikes"],
        "roofline": {
            "bound": "hbm", "achieved": k.get("achieved_gbs"), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (k.get("achieved_gbs") or 0) / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic * (k.get("steps_per_launch") or 1),
            "traffic_source": traffic_src,
            "kernel": k.get("name"), "avg_us": k.get("avg_us"), "launches": k.get("launches"),
            "us_per_step": k.get("us_per_step"), "steps_per_launch": k.get("steps_per_launch"),
            "alg_bytes_per_launch": k.get("alg_bytes_per_launch"),
            "alg_bytes_per_step": k.get("alg_bytes_per_step"),
            "kernel_share_of_step_time": k.get("share_of_time"),
            "copy_gbs": copy_gbs,
        },
        "cpu_baseline": cpu,
    }
    if ref is not None:
        line["plain_fp64"] = {"cv_steps_per_s": ref["cv_steps_per_s"], "ms_per_step": ref["ms_per_step"],
                              "spikes": ref["spikes"]}
        line["speedup_vs_plain_fp64"] = ref["seconds"] / head["seconds"]
        if head["spikes"] and ref["spikes"]:
            line["speedup_per_spike"] = (ref["seconds"] / ref["spikes"]) / (head["seconds"] / head["spikes"])
            line["equal_spikes"] = head["spikes"] == ref["spikes"]
    if bfp is not None:
        line["batched_fp64"] = {"cv_steps_per_s": bfp["cv_steps_per_s"], "ms_per_step": bfp["ms_per_step"],
                                "spikes": bfp["spikes"]}
    if args.workload == "busyring":
        # the benchmark's own measure: propagation of 200 ms (8000 steps of 0.025 ms)
        prop = head["ms_per_step"] * 8000 / 1000.0
        paper = BUSYRING_T1000_S.get((args.ring_cells, args.ring_depth))
        line["busyring_200ms_propagation_s"] = prop
        line["paper_t1000_propagation_s"] = None if paper is None else paper[1 if args.ring_stdp else 0]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
