"""Pins of the oracle's fast-forward mode (the long steps of slow network
dynamics in the 8-h paradigm of Sec. 3.5, with spiking and calcium off):
closed forms of the slow variables under Eqs. 17, 20 and 21 without
calcium, the identity with ordinary steps on a silent network, and the
handling of what is in flight when time jumps."""
import numpy as np
import pytest

import netgen
import oracle

STC = dict(netgen.STC_TABLE5)
H0 = STC["h0"]


def _one_cell(n_syn, dt=0.2, t_end=100.0, trains=()):
    b = netgen._Builder()
    b.add_cell([-1, 0, 1], [20.0, 10.0, 10.0], [20.0, 1.0, 1.0], [netgen.MECH_PAS] * 3)
    sids = [b.add_syn(0, 1 + k % 2, netgen.KIND_STC, 5.0, 0.0) for k in range(n_syn)]
    for sid, times in trains:
        b.add_train(sids[sid], netgen.PORT_G | netgen.PORT_CA, 0.001, times)
    return b.finish("ff", dt, t_end, 1, STC)


def test_early_phase_relaxes_geometrically():
    """Without calcium Eq. 17 reduces to dh/dt = 0.1 (h0 - h) / tau_h: each
    long step multiplies h - h0 by 1 - 0.1 dt_long / tau_h."""
    net = _one_cell(3)
    o = oracle.Oracle(net)
    h = np.array([H0 + 2.0, H0 - 1.5, H0 + 0.3])
    o.write("h", h)
    dl = 1000.0
    for n in (1, 10, 250):
        o.fast_forward(n - (o.step // 5000), dl)
        f = (1.0 - 0.1 * dl / STC["tau_h"]) ** n
        np.testing.assert_allclose(o.read("h") - H0, (h - H0) * f, rtol=1e-12)
    assert o.step == 250 * 5000


def test_protein_and_late_phase_follow_their_products():
    """With S above theta_pro the protein rises as p_max (1 - (1 - a_p)^n)
    (Eq. 21); z of an LTP-tagged synapse follows 1 - z_n = (1 - z_0)
    prod_k (1 - a_z p_k f_int) with the step-start protein p_k (Eq. 20), and
    of an LTD-tagged one z_n + 0.5 = (z_0 + 0.5) prod_k (1 - a_z p_k f_int)."""
    net = _one_cell(2)
    o = oracle.Oracle(net)
    o.write("h", np.array([H0 + 2.5, H0 - 2.0]))   # S = 4.5 > theta_pro, tags of both signs
    o.write("z", np.array([0.1, -0.2]))
    dl, n = 1000.0, 400
    a_p, a_z = dl / STC["tau_p"], dl / STC["tau_z"]
    pk = STC["p_max"] * (1.0 - (1.0 - a_p) ** np.arange(n))     # p at the start of step k
    # S stays above threshold over these steps
    hs = H0 + np.array([2.5, -2.0])[:, None] * (1 - 0.1 * dl / STC["tau_h"]) ** np.arange(n)[None, :]
    assert (np.abs(hs - H0).sum(0) > STC["theta_pro"]).all()
    # the tags hold too
    assert (np.abs(hs - H0) > STC["theta_tag"]).all()
    o.fast_forward(n, dl)
    np.testing.assert_allclose(o.read("p")[0], STC["p_max"] * (1 - (1 - a_p) ** n), rtol=1e-12)
    prod = np.prod(1.0 - a_z * pk * STC["f_int"])
    z = o.read("z")
    np.testing.assert_allclose(1.0 - z[0], 0.9 * prod, rtol=1e-12)
    np.testing.assert_allclose(z[1] + 0.5, 0.3 * prod, rtol=1e-12)


def test_long_steps_of_dt_equal_ordinary_steps_on_a_silent_network():
    """On a network without input or calcium, the ordinary step changes h,
    z and p by exactly the fast-forward formulas (the calcium terms of Eq.
    17 vanish): fast-forward with dt_long = dt gives the same bits."""
    net = _one_cell(5)
    a, b = oracle.Oracle(net), oracle.Oracle(net)
    rng = np.random.default_rng(3)
    h = H0 + rng.uniform(-2.5, 2.5, 5)
    z = rng.uniform(-0.4, 0.9, 5)
    for x in (a, b):
        x.write("h", h)
        x.write("z", z)
        x.write("p", np.array([3.0]))
    a.run(300)
    b.fast_forward(300, 0.2)
    for k in ("h", "z", "p"):
        np.testing.assert_array_equal(a.read(k), b.read(k), err_msg=k)
    assert a.step == b.step == 300


def test_events_in_flight_are_dropped_and_time_moves():
    """Train arrivals before the new time cause nothing; those after arrive
    at their steps; the post-synaptic flag and queued events are gone."""
    times = np.array([1.0, 3.3, 50.1, 1200.3, 1200.5, 1203.9])
    net = _one_cell(1, t_end=2000.0, trains=[(0, times)])
    o = oracle.Oracle(net)
    o.run(10)                     # t = 2 ms: the arrival at 1.0 is delivered, the rest queued
    cnt0, _ = o.event_stats()
    assert cnt0[0, 0] == 1
    o.fast_forward(3, 400.0)      # to t = 1202 ms
    assert o.step == 10 + 3 * 2000
    o.run(150)                    # to t = 1232 ms
    cnt, ssum = o.event_stats()
    # conductance port: arrivals at 1.0 (before) and 1203.9 (after); the
    # calcium port (t + t_cd): only 1203.9 + 18.8 within the run
    assert cnt[0, 0] == 2
    assert ssum[0, 0] == 5 + int(np.floor(1203.9 / 0.2))
    assert cnt[0, 1] == 1
    assert ssum[0, 1] == int(np.floor((1203.9 + STC["t_cd"]) / 0.2))


def test_poisson_source_restarts_after_the_jump():
    """A Poisson source whose next arrival falls inside the jump draws it
    again from the new time (memoryless): its first arrival after the jump
    lies after the new time, and arrivals keep their rate."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    s = b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    b.add_poisson(s, netgen.PORT_G, 0.0001, 200.0)
    net = b.finish("ffp", 0.2, 100.0, 7, STC)
    o = oracle.Oracle(net)
    o.run(50)
    c0, s0 = (x[0, 0] for x in o.event_stats())
    o.fast_forward(10, 1000.0)
    n_new = o.step
    o.run(5000)
    cnt, ssum = (x[0, 0] for x in o.event_stats())
    k = cnt - c0
    assert 150 < k < 260           # 200 Hz over 1 s
    # every arrival after the jump is delivered at or after the new time
    assert ssum - s0 >= k * n_new
