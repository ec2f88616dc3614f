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
    sim = Simulation(net, mode=mode, precision={"fp64": "fp64", "mixed": "mixed"}[prec],
                     **(plan if mode == "batched" and plan else {}))
    st = sim.stats()
    st["n_hh"] = sim.n_hh
    if settle:
        sim.advance_steps(settle)
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
    out = dict(form=form, seconds=el, ms_per_step=1e3 * el / steps, spikes=st2["spikes"] - sp0,
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


def cpu_baseline(net, n_steps):
    import oracle
    o = oracle.Oracle(net)
    t0 = time.perf_counter()
    o.run(n_steps)
    el = time.perf_counter() - t0
    spikes = int(o.spikes()[0].size)
    return dict(value=o.n_cv * n_steps / el, unit="CV-steps/s", cores=1, kind="oracle",
                sample=f"first {n_steps} steps ({n_steps * net['dt']:.0f} ms, {spikes} spikes) of the same "
                       f"network with its inputs, single-threaded plain FP64 C oracle, {el:.1f} s")


# workloads: name in the JSON line, network builder
WORKLOADS = {"ei2000x21": ("ei-ball-and-stick-2000x21cv", "config2"),
             "ei2000x101": ("ei-ball-and-stick-2000x101cv", "config4")}


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
    ap.add_argument("--cpu-steps", type=int, default=1500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plan", default="",
                    help="fix the batched form's plan instead of autotuning it: "
                         "CELLS_PER_BLOCK,BLOCK_THREADS,SOLVER_WAVES,EXCHANGE (kernel|resident)")
    ap.add_argument("--workload", default="ei2000x101", choices=sorted(WORKLOADS),
                    help="ei2000x101: the headline network (100-CV dendrites); ei2000x21: 20-CV dendrites")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the runs, copy this many MiB device to device (a plain copy kernel of known "
                         "size that scales rocprofv3's FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import netgen
    # inputs over everything that runs: settle, warmup, timed steps and the
    # oracle's sample
    t_end = (max(args.settle + args.warmup + args.steps, args.cpu_steps) + 100) * 0.2
    wname, make = WORKLOADS[args.workload]
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
        cpu = cpu_baseline(net, args.cpu_steps)
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
        "data": "synthetic (seeded E/I network shaped like the paper's 2000-neuron STC network; "
                f"{args.settle} untimed settling steps from rest)",
        "config": {"workload": wname, "cells": head["stats"]["n_cells"],
                   "cvs": head["stats"]["n_cv"], "synapses": head["stats"]["n_syn"],
                   "stc_synapses": head["stats"]["n_stc"], "dt_ms": 0.2, "form": args.form,
                   "epoch_steps": head["epoch_steps"], "cells_per_block": head["cells_per_block"],
                   "block_threads": head["block_threads"], "solver_waves": head["solver_waves"],
                   "exchange": head["exchange"], "settle_steps": args.settle, "parallelism": "single-gpu"},
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
