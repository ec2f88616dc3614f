"""Shared helpers of the GPU parity tests: run the HIP library and the
oracle on the same seeded network and compare them."""
import numpy as np

import oracle
from paper_2411_16445_amd import Simulation

# FP64 voltage bar: |dV| <= 1e-9 max(|V|, 1 mV)
V_RTOL = 1e-9


def run_pair(net, n_steps, chunks=1, **kw):
    o = oracle.Oracle(net)
    s = Simulation(net, **kw)
    per = n_steps // chunks
    done = 0
    for k in range(chunks):
        m = per if k < chunks - 1 else n_steps - done
        o.run(m)
        s.advance_steps(m)
        done += m
    return o, s


def assert_raster_equal(o, s, t_rtol=1e-9):
    """Equal rasters: both sides deliver them in (t*, gid) order; equal
    counts, cells and crossing steps, t* within t_rtol."""
    og, ost, ot = o.spikes()
    sg, sst, stt = s.spikes()
    assert og.size == sg.size, f"spike count oracle {og.size} vs gpu {sg.size}"
    if stt.size > 1:
        assert np.all((np.diff(stt) > 0) | ((np.diff(stt) == 0) & (np.diff(sg) > 0))), "not in (t*, gid) order"
    np.testing.assert_array_equal(sg, og)
    np.testing.assert_array_equal(sst, ost)
    if ot.size:
        np.testing.assert_allclose(stt, ot, rtol=t_rtol, atol=0)
    return og.size


def assert_v_close(vo, vs, rtol=V_RTOL):
    err = np.abs(vs - vo) / np.maximum(np.abs(vo), 1.0)
    assert err.max(initial=0.0) <= rtol, f"max scaled |dV| {err.max():.3e} at {int(err.argmax())}"


def assert_state_close(o, s, rtol=1e-9, atol_h=1e-10):
    assert_v_close(o.read("V"), s.read("V"), rtol)
    for k in ("m", "hh", "n"):
        np.testing.assert_allclose(s.read(k), o.read(k), rtol=rtol, atol=1e-12)
    gs, go = s.read("g"), o.read("g")
    np.testing.assert_allclose(gs, go, rtol=rtol, atol=1e-15 + rtol * np.abs(go).max(initial=0))
    np.testing.assert_allclose(s.read("c"), o.read("c"), rtol=rtol, atol=1e-13)
    np.testing.assert_allclose(s.read("h"), o.read("h"), rtol=rtol, atol=atol_h)
    np.testing.assert_allclose(s.read("z"), o.read("z"), rtol=rtol, atol=1e-12)
    np.testing.assert_allclose(s.read("p"), o.read("p"), rtol=rtol, atol=1e-12)


def assert_routing_equal(o, s):
    oc, osum = o.event_stats()
    sc, ssum = s.event_stats()
    np.testing.assert_array_equal(sc, oc)
    np.testing.assert_array_equal(ssum, osum)
