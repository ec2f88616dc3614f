"""Pins of the oracle's Graupner-Brunel synapse batch (Sec. 3.3, Eqs.
10-12, Table 3) against facts that do not come from the oracle: the
implicit closed-form solution of the cubic weight dynamics without calcium,
the piecewise-geometric calcium trace of the pairing protocol, the drift of
an isolated pair summed over the steps above each threshold, the variance
of the noise term (Eq. 11), and the shape of the DP curve."""
import math

import numpy as np
import pytest

import netgen
import oracle

GB = dict(netgen.GB_TABLE3)


def _cubic_time(w0, w, a, tau):
    """Time for dw/dt = w (1 - w) (w - a) / tau to go from w0 to w (partial
    fractions of 1 / (w (1 - w) (w - a)))."""
    return tau * (-(1.0 / a) * math.log(w / w0) - (1.0 / (1.0 - a)) * math.log((1.0 - w) / (1.0 - w0))
                  + (1.0 / (a * (1.0 - a))) * math.log((w - a) / (w0 - a)))


@pytest.mark.parametrize("w0", [0.62, 0.35, 0.93, 0.05])
def test_weight_without_calcium_follows_the_cubic_closed_form(w0):
    """No pairs: Eq. 10 reduces to tau_w dw/dt = -w (1 - w) (w_* - w), whose
    solution moves away from w_* towards 0 or 1; the Euler-Maruyama run
    reaches after time T the weight whose closed-form time is T."""
    dt, T = 0.5, 200000.0
    w, _ = oracle.gb_trials(GB, dt, [0.0], [w0], n_pairs=0, t0=T)
    t = _cubic_time(w0, w[0], GB["w_star"], GB["tau_w"])
    assert abs(t - T) < 1e-3 * T, (t, T)
    assert (w[0] - GB["w_star"]) * (w0 - GB["w_star"]) > 0 and abs(w[0] - GB["w_star"]) > abs(w0 - GB["w_star"])


@pytest.mark.parametrize("delay", [-37.3, 0.0, 12.6])
def test_calcium_trace_is_the_sum_of_decayed_jumps(delay):
    """After the protocol the calcium holds every presynaptic jump (delivered
    at floor((t_pre + t_cd) / dt)) and postsynaptic jump (at floor((t_pre +
    delay) / dt)), each decayed by exp(-dt / tau_c) per step since."""
    dt, n_pairs, T, t0 = 0.5, 5, 200.0, 100.0
    _, c = oracle.gb_trials(dict(GB, sigma=0.0), dt, [delay], [0.3], n_pairs=n_pairs, period=T, t0=t0)
    n_end = math.floor((t0 + n_pairs * T) / dt)
    r = math.exp(-dt / GB["tau_c"])
    want = 0.0
    for k in range(n_pairs):
        want += GB["c_pre"] * r ** (n_end - math.floor((t0 + k * T + GB["t_cd"]) / dt))
        want += GB["c_post"] * r ** (n_end - math.floor((t0 + k * T + delay) / dt))
    np.testing.assert_allclose(c[0], want, rtol=1e-12)


def test_isolated_postsynaptic_spike_drift():
    """Near w = 0 the cubic and depression terms vanish, so one pair far
    apart in time changes w by about (dt / tau_w) gamma_p (1 - w) times the
    steps with c > theta_p; those steps follow from the calcium trace of a
    lone postsynaptic jump c_post exp(-k dt / tau_c)."""
    dt = 0.2
    w, _ = oracle.gb_trials(dict(GB, sigma=0.0), dt, [-400.0], [1e-9], n_pairs=1, period=1000.0, t0=500.0)
    # steps with c > theta_p after the post jump (the pre jump, 400 ms
    # later, stays at c_pre = theta_d and crosses neither threshold)
    ah = dt / GB["tau_w"]
    k_p = math.floor(GB["tau_c"] / dt * math.log(GB["c_post"] / GB["theta_p"])) + 1
    k_d = math.floor(GB["tau_c"] / dt * math.log(GB["c_post"] / GB["theta_d"])) + 1
    want = ah * GB["gamma_p"] * k_p
    # what the neglected terms can take off, each at most w_final times:
    # the (1 - w) factor over the k_p steps, depression over the k_d
    # steps, the cubic's slope (at most w_* at small w) over every step
    n_end = math.floor(1500.0 / dt)
    bound = w[0] * ah * (GB["gamma_p"] * k_p + GB["gamma_d"] * k_d + GB["w_star"] * n_end)
    assert want - bound <= w[0] <= want, (w[0], want, bound)
    assert bound < 0.05 * want


def test_noise_term_variance():
    """With both thresholds crossed for the steps after a postsynaptic jump,
    the weight's spread over independent trials is sigma^2 dt / tau_w times
    the summed (Theta_p + Theta_d) of those steps (Eq. 11, variance 1/dt
    white noise); checked at w = w_* where the drift balances."""
    dt, n = 0.5, 4000
    delays = np.full(n, -300.0)
    w, _ = oracle.gb_trials(GB, dt, delays, np.full(n, 0.5), n_pairs=1, period=1000.0, t0=400.0, seed=11)
    k_p = math.floor(GB["tau_c"] / dt * math.log(GB["c_post"] / GB["theta_p"])) + 1
    k_d = math.floor(GB["tau_c"] / dt * math.log(GB["c_post"] / GB["theta_d"])) + 1
    var = GB["sigma"] ** 2 * (dt / GB["tau_w"]) * (k_p + k_d)
    assert abs(np.var(w) / var - 1.0) < 0.08, (np.var(w), var)


def test_dp_curve_shape():
    """The curve of Sec. 3.3 (Fig. 2j, after Graupner and Brunel): pairs with
    the postsynaptic spike shortly after the presynaptic one end above the
    mean of large delays, those with it shortly before end below."""
    dt, trials = 0.5, 200
    delays = np.repeat([-20.0, 15.0, 150.0], trials)
    w0 = np.tile(np.r_[np.zeros(trials // 2), np.ones(trials // 2)], 3)
    w, _ = oracle.gb_trials(GB, dt, delays, w0, n_pairs=60, seed=5)
    m = w.reshape(3, trials).mean(1)
    assert m[0] < m[2] - 0.02 and m[1] > m[2] + 0.01, m
