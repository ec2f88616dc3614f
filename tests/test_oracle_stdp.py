"""Pins of the oracle's pair-based STDP synapse (Eqs. 6-8, Table 1)
against the analytic pair rule: for an isolated pair the weight changes by
A_pre e^{-dt/tau_pre} (pre before post) or A_post e^{-|dt|/tau_post} (post
before pre), exactly in its discrete form (traces decaying by e^{-dt/tau}
per step between the delivery step of the presynaptic event and the step
of the post-synaptic hook), and to the time step in the continuous form;
the weight's contribution to the conductance is clipped to [0, w_max]."""
import math

import numpy as np
import pytest

import netgen
import oracle

STC = dict(netgen.STC_TABLE5)
STDP = dict(tau_pre=20.0, tau_post=10.0, a_pre=0.01, a_post=-0.0105, w0=1.0, w_max=10.0)
DT = 0.2


def _pair_net(t_pres, t_clamp, w_conn=0.0, t_end=200.0, stdp=STDP):
    """HH soma with one STDP synapse; presynaptic arrivals from a train of
    connection weight w_conn; the post-synaptic spike from a short
    suprathreshold clamp at t_clamp (None: no post spike)."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH])
    s = b.add_syn(0, 0, 2, 5.0, 0.0)
    if len(t_pres):
        b.add_train(s, netgen.PORT_G, w_conn, np.asarray(t_pres, float))
    if t_clamp is not None:
        b.add_clamp(0, 0, t_clamp, 1.0, 1.0)
    net = b.finish("stdp-pair", DT, t_end, 1, STC)
    net["stdp"] = dict(stdp)
    return net


def _run(net, n=600):
    o = oracle.Oracle(net)
    o.run(n)
    return o


def _post_step(o):
    g, st, _ = o.spikes()
    assert g.size == 1, g.size
    return int(st[0]) + 1        # the hook acts at the start of the step after detection


@pytest.mark.parametrize("t_pre", [3.1, 8.0, 14.9])
def test_pre_before_post_potentiates_by_the_decayed_pre_trace(t_pre):
    o = _run(_pair_net([t_pre], 20.0))
    n_pre = math.floor(t_pre / DT)
    n_hook = _post_step(o)
    assert n_hook > n_pre
    r = math.exp(-DT / STDP["tau_pre"])
    want = STDP["w0"] + STDP["a_pre"] * r ** (n_hook - n_pre)
    np.testing.assert_allclose(o.read("h")[0], want, rtol=1e-13)


@pytest.mark.parametrize("t_pre", [25.3, 31.0, 60.7])
def test_post_before_pre_depresses_by_the_decayed_post_trace(t_pre):
    o = _run(_pair_net([t_pre], 20.0))
    n_pre = math.floor(t_pre / DT)
    n_hook = _post_step(o)
    assert n_pre > n_hook
    r = math.exp(-DT / STDP["tau_post"])
    want = STDP["w0"] + STDP["a_post"] * r ** (n_pre - n_hook)
    np.testing.assert_allclose(o.read("h")[0], want, rtol=1e-13)


def test_stdp_window_matches_the_exponential_pair_rule():
    """The classical window: dw(dt) = A_pre e^{-dt/tau_pre} for dt > 0 and
    A_post e^{dt/tau_post} for dt < 0, within the quantisation of both
    spikes to the step."""
    for dt_pair in (-30.0, -12.0, -4.0, 4.0, 12.0, 30.0):
        o0 = _run(_pair_net([], 40.0))
        t_post = o0.spikes()[2][0]
        o = _run(_pair_net([t_post - dt_pair], 40.0))
        dw = o.read("h")[0] - STDP["w0"]
        if dt_pair > 0:
            want, tau, amp = STDP["a_pre"] * math.exp(-dt_pair / STDP["tau_pre"]), STDP["tau_pre"], STDP["a_pre"]
        else:
            want, tau, amp = STDP["a_post"] * math.exp(dt_pair / STDP["tau_post"]), STDP["tau_post"], STDP["a_post"]
        assert abs(dw - want) <= abs(amp) * (1.0 - math.exp(-3 * DT / tau)), (dt_pair, dw, want)
        assert np.sign(dw) == np.sign(want)


def test_every_pair_counts():
    """Three presynaptic spikes before one postsynaptic spike: the weight
    gains the sum of the three decayed pre-trace jumps (all-to-all pairing
    through the trace)."""
    t_pres = [2.0, 9.4, 15.0]
    o = _run(_pair_net(t_pres, 20.0))
    n_hook = _post_step(o)
    r = math.exp(-DT / STDP["tau_pre"])
    want = STDP["w0"] + sum(STDP["a_pre"] * r ** (n_hook - math.floor(t / DT)) for t in t_pres)
    np.testing.assert_allclose(o.read("h")[0], want, rtol=1e-13)
    # the pre trace itself: three geometric jumps
    n_end = o.step
    np.testing.assert_allclose(o.read("c")[0], sum(STDP["a_pre"] * r ** (n_end - math.floor(t / DT))
                                                   for t in t_pres), rtol=1e-12)


@pytest.mark.parametrize("w_init,a_post,jump", [(3.0, 0.0, 3.0), (25.0, 0.0, 10.0), (-2.0, 0.0, 0.0),
                                                (3.0, -2.0, 3.0)])
def test_conductance_jump_uses_the_clipped_weight(w_init, a_post, jump):
    """A presynaptic spike of connection weight w_conn adds w_conn x
    clip(w, 0, w_max) to the conductance, with the weight before the
    spike's own change by a_post, and the conductance then decays as an
    exponential synapse (tau 5 ms) within the same step."""
    net = _pair_net([1.1], None, w_conn=0.5)
    o = oracle.Oracle(net)
    o.write("h", np.array([w_init]))
    o.write("z", np.array([a_post]))
    o.run(6)                       # delivered at step 5, decayed once
    np.testing.assert_allclose(o.read("g")[0], 0.5 * jump * math.exp(-DT / 5.0), rtol=1e-14)
    r = math.exp(-DT / STDP["tau_post"])
    np.testing.assert_allclose(o.read("h")[0], w_init + a_post * r ** 5, rtol=1e-14)
