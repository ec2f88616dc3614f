"""Writes the oracle fixtures of the long-horizon GPU tests.

Runs the plain FP64 CPU oracle (and nothing else: no value here comes from
the HIP library) on the seeded synthetic networks and stores what the GPU
tests compare against:

  oracle_ei2000x21_10s.npz   the 2000-cell E/I network with 20-CV dendrites
                             over its full 10 s (50,000 steps): the raster in
                             (t*, gid) order, V of every CV and p of every
                             cell at the end, h of every 97th synapse;
  oracle_ei2000x101_1s.npz   the same network with 100-CV dendrites over 1 s
                             (5,000 steps): the raster and V of every 7th CV
                             at the end (for the mixed-precision report).

    python tests/golden/make_fixtures.py [ei2000x21_10s] [ei2000x101_1s]

Each takes minutes on one core.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import netgen  # noqa: E402
import oracle  # noqa: E402

FIXTURES = {
    # name: (network builder, steps, V stride, synapse stride for h)
    "ei2000x21_10s": (lambda: netgen.config2(t_end=10000.0), 50000, 1, 97),
    "ei2000x101_1s": (lambda: netgen.config4(t_end=1000.0), 5000, 7, 0),
}


def path(name):
    return os.path.join(HERE, f"oracle_{name}.npz")


def make(name):
    build, steps, vstride, hstride = FIXTURES[name]
    net = build()
    o = oracle.Oracle(net)
    t0 = time.time()
    done = 0
    while done < steps:
        m = min(5000, steps - done)
        o.run(m)
        done += m
        print(f"[{name}] {done} steps, {o.spikes()[0].size} spikes, {time.time() - t0:.0f} s", flush=True)
    g, st, t = o.spikes()
    out = dict(steps=np.int64(steps), gid=g.astype(np.uint16 if net["n_cells"] < 65536 else np.uint32),
               step=st.astype(np.uint32), t=t, v_stride=np.int64(vstride), V=o.read("V")[::vstride],
               p=o.read("p"))
    if hstride:
        out["h_stride"] = np.int64(hstride)
        out["h"] = o.read("h")[::hstride]
    np.savez_compressed(path(name), **out)
    print(f"[{name}] wrote {path(name)} ({os.path.getsize(path(name)) / 1e6:.2f} MB)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(FIXTURES):
        make(name)
