"""Throughput of the per-step update of a plastic network of multi-compartment
neurons on one MI355X.

Workload: 2000 ball-and-stick cells (HH soma + 20 passive dendrite CVs,
42,000 CVs), 1600 excitatory / 400 inhibitory, Bernoulli(0.1) connectivity
with 3 ms delays, ~255k plastic (calcium + tagging-and-capture) E->E
synapses and ~146k static ones, 25 x 5 Hz Poisson inputs per cell, dt = 0.2 ms,
seeded synthetic data (no dataset).  A bench "step" is one time step of the
whole network (delivery, currents, cable solve, mechanisms, plasticity,
detection, and its share of the spike exchange).

    python bench.py [--steps 50000] [--warmup 500] [--form batched-mixed]

Prints one JSON line.  value = CV-steps/s of the headline form over the
timed steps; the plain FP64 form runs the same steps for the comparison at
equal spikes.
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


def _alg_bytes_per_launch(form: str, s: dict, steps_per_launch: float) -> float:
    """Algorithmic HBM bytes of one launch of the dominant kernel.

    plain: the synapse kernel, per step: every synapse reads and writes g and
    reads its decay factor and kind (25 B FP64 / 13 B FP32 g); a plastic
    synapse also reads and writes c, h, z and reads its cell index
    (52 B FP64, 44 B with FP32 c).
    batched: the fused epoch kernel, per step: per CV V r/w + axial + C/dt +
    d0 + g_pas E (48 B); per HH CV 3 gates r/w (48 / 24 B); per synapse as
    above plus its reversal potential and CV index (12 B); per cell p r/w
    and the detector voltage (24 B).
    """
    mixed = form.endswith("mixed")
    n_syn, n_stc, n_cv, n_cells = s["n_syn"], s["n_stc"], s["n_cv"], s["n_cells"]
    syn = 25.0 if not mixed else 13.0
    stc = 52.0 if not mixed else 44.0
    if form.startswith("plain"):
        per_step = n_syn * syn + n_stc * stc
    else:
        gate = 48.0 if not mixed else 24.0
        per_step = (n_cv * 48.0 + n_cells * gate + n_syn * (syn + 12.0) + n_stc * stc
                    + n_cells * 24.0)
    return per_step * steps_per_launch


def run_form(net, form, steps, warmup, time_kernel=True):
    import torch

    from paper_2411_16445_amd import Simulation
    mode, prec = form.split("-")
    sim = Simulation(net, mode=mode, precision={"fp64": "fp64", "mixed": "mixed"}[prec])
    st = sim.stats()
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
               epoch_steps=st["epoch_steps"], cells_per_block=st2["cells_per_block"])
    if time_kernel:
        ms, launches, name = sim.kernel_time()
        avg_ms = ms / max(1, launches)
        spl = steps / max(1, launches)
        alg = _alg_bytes_per_launch(form, st, spl)
        achieved = alg / (avg_ms * 1e-3) / 1e9
        out["kernel"] = dict(name=name, launches=launches, avg_us=avg_ms * 1e3,
                             alg_bytes_per_launch=alg, achieved_gbs=achieved,
                             share_of_time=ms / (el * 1e3))
    out["stats"] = st
    sim.close()
    return out


def cpu_baseline(net, n_steps):
    import oracle
    o = oracle.Oracle(net)
    t0 = time.perf_counter()
    o.run(n_steps)
    el = time.perf_counter() - t0
    return dict(value=o.n_cv * n_steps / el, unit="CV-steps/s", cores=1, kind="oracle",
                sample=f"first {n_steps} steps ({n_steps * net['dt']:.0f} ms) of the same network, "
                       f"single-threaded plain FP64 C oracle, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--form", default=os.environ.get("PA_BENCH_FORM", "batched-mixed"),
                    choices=["plain-fp64", "plain-mixed", "batched-fp64", "batched-mixed"])
    ap.add_argument("--no-compare", action="store_true", help="skip the plain FP64 reference run")
    ap.add_argument("--cpu-steps", type=int, default=1500)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import netgen
    t_end = (args.warmup + args.steps + 10) * 0.2
    net = netgen.config2(t_end=t_end)
    print(f"[bench] network {netgen.summary(net)}", file=sys.stderr, flush=True)
    head = run_form(net, args.form, args.steps, args.warmup)
    print(f"[bench] {args.form}: {head['ms_per_step']*1e3:.2f} us/step, {head['spikes']} spikes",
          file=sys.stderr, flush=True)
    ref = None
    if not args.no_compare and args.form != "plain-fp64":
        ref = run_form(net, "plain-fp64", args.steps, args.warmup)
        print(f"[bench] plain-fp64: {ref['ms_per_step']*1e3:.2f} us/step, {ref['spikes']} spikes",
              file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(net, args.cpu_steps)
        print(f"[bench] cpu oracle: {cpu['value']:.3e} CV-steps/s", file=sys.stderr, flush=True)
    k = head.get("kernel", {})
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
        "data": "synthetic (seeded E/I network shaped like the paper's 2000-neuron STC network)",
        "config": {"workload": "ei-ball-and-stick-2000x21cv", "cells": head["stats"]["n_cells"],
                   "cvs": head["stats"]["n_cv"], "synapses": head["stats"]["n_syn"],
                   "stc_synapses": head["stats"]["n_stc"], "dt_ms": 0.2, "form": args.form,
                   "epoch_steps": head["epoch_steps"], "cells_per_block": head["cells_per_block"],
                   "parallelism": "single-gpu"},
        "synapse_updates_per_s": head["synapse_updates_per_s"],
        "stc_synapse_updates_per_s": head["stc_synapse_updates_per_s"],
        "spikes": head["spikes"],
        "roofline": {
            "bound": "hbm", "achieved": k.get("achieved_gbs"), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": (k.get("achieved_gbs") or 0) / HBM_PEAK_GBS, "traffic": None,
            "kernel": k.get("name"), "avg_us": k.get("avg_us"), "launches": k.get("launches"),
            "alg_bytes_per_launch": k.get("alg_bytes_per_launch"),
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
