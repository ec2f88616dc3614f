"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of the paper (or the textbook fact) it checks.
The closed forms here are solutions of the model equations, not restatements
of the oracle's update formulas: a dropped term, a wrong sign, a wrong unit
factor or a transposed index in the oracle makes one of them fail.
"""
import json
import math
import os

import numpy as np
import pytest

import netgen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
STC = dict(netgen.STC_TABLE5)


def _cell_params(**kw):
    p = netgen.DEFAULT_CELL.copy()
    names = ["cm", "ra", "v_init", "g_pas", "e_pas", "gna", "gk", "gl", "ena", "ek", "el"]
    for k, v in kw.items():
        p[names.index(k)] = v
    return p


def _net(builder, stc=None, dt=0.2, t_end=100.0, seed=11):
    return builder.finish("pin", dt, t_end, seed, STC if stc is None else stc)


# ------------------------------------------------------------------ P1
def test_single_passive_cv_backward_euler_decay():
    """A passive isopotential CV relaxes as (V_n - E) = (V0 - E) / (1 + dt/tau)^n
    under backward Euler, tau = c_m / g_pas (cable equation, Eq. 4, without
    the axial term); the continuous e^{-t/tau} holds to O(dt)."""
    b = netgen._Builder()
    cm, gpas, epas, v0 = 1.0, 1e-4, -65.0, -40.0
    b.add_cell([-1], [30.0], [7.0], [netgen.MECH_PAS], params=_cell_params(v_init=v0, g_pas=gpas, e_pas=epas))
    dt = 0.1
    o = oracle.Oracle(_net(b, dt=dt))
    tau = (cm * 1e-6) / gpas * 1e3  # ms
    vs = []
    for _ in range(200):
        o.run(1)
        vs.append(o.read("V")[0])
    n = np.arange(1, 201)
    disc = epas + (v0 - epas) / (1.0 + dt / tau) ** n
    np.testing.assert_allclose(vs, disc, rtol=1e-13, atol=0)
    cont = epas + (v0 - epas) * np.exp(-n * dt / tau)
    # first-order method: global error <= (dt/tau) * t/tau-scale factor
    assert np.max(np.abs(np.array(vs) - cont)) < 0.5 * (dt / tau) * abs(v0 - epas)
    assert np.max(np.abs(np.array(vs) - cont)) > 1e-6  # it is a first-order scheme, not exact


# ------------------------------------------------------------------ P2
def _cable_steady(n_cv, L=1000.0, d=1.0, I0=0.01, Ra=35.4, gpas=1e-4, epas=-65.0):
    b = netgen._Builder()
    parent = np.arange(-1, n_cv - 1)
    b.add_cell(parent, np.full(n_cv, L / n_cv), np.full(n_cv, d), np.zeros(n_cv, np.uint8),
               params=_cell_params(ra=Ra, g_pas=gpas, e_pas=epas, v_init=epas))
    b.add_clamp(0, 0, 0.0, 1e9, I0)
    o = oracle.Oracle(_net(b, dt=0.5))
    o.run(6000)  # 3 s = 300 membrane time constants
    return o.read("V") - epas


def test_passive_cable_steady_state_converges_to_cosh_solution():
    """Sealed-end passive cable with a steady current I0 into its first CV:
    V(x) - E = I0 R_inf cosh((L-x)/lambda) / sinh(L/lambda), lambda =
    sqrt(r R_m / (2 R_a)), R_inf = R_a lambda / (pi r^2) (textbook cable
    theory for Eq. 4).  The finite-volume solution converges at second
    order in the CV length."""
    L, d, I0, Ra, gpas = 1000.0, 1.0, 0.01, 35.4, 1e-4
    r_cm = 0.5 * d * 1e-4
    Rm = 1.0 / gpas                             # ohm cm^2
    lam_cm = math.sqrt(r_cm * Rm / (2 * Ra))
    Rinf = Ra * lam_cm / (math.pi * r_cm ** 2)   # ohm
    L_cm = L * 1e-4
    errs = []
    for n in (8, 16, 32, 64):
        v = _cable_steady(n, L, d, I0, Ra, gpas)
        x_cm = (np.arange(n) + 0.5) * (L_cm / n)
        exact = (I0 * 1e-9) * Rinf * np.cosh((L_cm - x_cm) / lam_cm) / math.sinh(L_cm / lam_cm) * 1e3
        errs.append(np.max(np.abs(v - exact)))
        assert np.max(np.abs(v - exact)) < 0.05 * np.max(exact)
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    for r in ratios:
        assert 3.5 < r < 4.5, (errs, ratios)
    assert abs(lam_cm * 1e4 - 840.0) < 2.0  # ~840 um for d = 1 um


# ------------------------------------------------------------------ P3
def _random_tree_parent(rng, n):
    return np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)], np.int64)


@pytest.mark.parametrize("seed", range(40))
def test_hines_matches_dense_lu_on_random_trees(seed):
    """Hines elimination on a tree (parent[i] < i) equals LAPACK's pivoted LU
    on the same dense symmetric matrix."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 17))
    parent = _random_tree_parent(rng, n)
    U = -rng.uniform(0.1, 5.0, n)
    U[0] = 0.0
    A = np.zeros((n, n))
    for i in range(1, n):
        A[i, parent[i]] = A[parent[i], i] = U[i]
    D = np.abs(A).sum(1) + rng.uniform(0.01, 3.0, n)
    A[np.arange(n), np.arange(n)] = D
    b = rng.normal(size=n)
    x = oracle.hines(parent, U, D, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-12 * np.abs(x).max())


def test_step_solves_assembled_system_exactly():
    """One step of a small network: the new voltages solve the assembled
    symmetric tree system of that step (dense LU), and the matrix is
    symmetric with off-diagonals only between parent and child."""
    net = netgen.tiny(seed=3, n_cells=6, t_end=50.0)
    for k in ("train_dst", "train_ports", "train_w"):
        net[k] = net[k][:0]
    net["train_off"] = net["train_off"][:1]
    net["train_times"] = net["train_times"][:0]
    net["clamp_cell"] = net["clamp_cell"][:0]
    for k in ("clamp_cv", "clamp_t0", "clamp_dur", "clamp_amp"):
        net[k] = net[k][:0]
    o = oracle.Oracle(net)
    rng = np.random.default_rng(0)
    o.write("g", rng.uniform(0, 0.01, o.n_syn))
    o.write("V", rng.uniform(-80, -50, o.n_cv))
    D, U, b = o.assemble()
    o.run(1)
    v = o.read("V")
    off = net["cv_off"]
    for c in range(net["n_cells"]):
        s0, s1 = off[c], off[c + 1]
        n = s1 - s0
        A = np.diag(D[s0:s1])
        for i in range(1, n):
            p = net["parent"][s0 + i]
            A[i, p] = A[p, i] = U[s0 + i]
        np.testing.assert_allclose(v[s0:s1], np.linalg.solve(A, b[s0:s1]), rtol=1e-12)
        # diagonal dominance with equality in the axial part: row sums of the
        # axial matrix vanish, so D - sum|U| is the membrane + capacitive part
        assert np.all(D[s0:s1] > 0)


# ------------------------------------------------------------------ P4
def test_axial_current_conserves_charge():
    """Without membrane currents the axial current only redistributes
    charge: sum_i C_i V_i is invariant (zero column sums of the axial
    matrix, Eq. 4)."""
    rng = np.random.default_rng(5)
    parent, length, diam, mech = netgen.random_tree(rng, 20, 40)
    mech[:] = netgen.MECH_PAS
    b = netgen._Builder()
    b.add_cell(parent, length, diam, mech, params=_cell_params(g_pas=0.0))
    o = oracle.Oracle(_net(b, dt=0.025))
    v0 = rng.uniform(-90, 30, len(parent))
    o.write("V", v0)
    cap = math.pi * diam * length  # capacitance is proportional to the lateral area
    q0 = np.dot(cap, v0)
    for _ in range(5):
        o.run(20)
        q = np.dot(cap, o.read("V"))
        assert abs(q - q0) <= 1e-13 * np.dot(cap, np.abs(v0))
    v = o.read("V")
    assert np.std(v) < np.std(v0)  # it did diffuse


# ------------------------------------------------------------------ P5/P6
def test_hh_steady_state_gates_match_textbook_values():
    g = json.load(open(os.path.join(GOLD, "hh_rest.json")))
    r = oracle.hh_rates(g["v_mV"])
    for (a, bb), key in zip(((r[0], r[1]), (r[2], r[3]), (r[4], r[5])), ("m_inf", "h_inf", "n_inf")):
        assert abs(a / (a + bb) - g[key]) <= g["rel_tol"] * g[key]


def test_hh_alpha_m_removable_singularity():
    """alpha_m = 0.1 (V+40) / (1 - exp(-(V+40)/10)) -> 1 ms^-1 at V = -40."""
    assert oracle.hh_rates(-40.0)[0] == 1.0
    for dv in (1e-12, 1e-9, 1e-6, -1e-9):
        v = -40.0 + dv
        x = (v + 40.0) / 10.0
        expect = 1.0 + x / 2.0 + x * x / 12.0  # series of x / (1 - e^-x)
        assert abs(oracle.hh_rates(v)[0] - expect) < 1e-12
        assert abs(oracle.hh_rates(v - 15.0)[4] - 0.1 * oracle.hh_rates(v)[0]) < 1e-13


def test_gate_exponential_integrator_under_voltage_clamp():
    """With V held fixed (huge capacitance), each gate follows
    x_n = x_inf + (x0 - x_inf) exp(-n dt (alpha + beta))."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH], params=_cell_params(cm=1e15, v_init=-30.0))
    dt = 0.2
    o = oracle.Oracle(_net(b, dt=dt))
    o.write("m", [0.9]); o.write("hh", [0.05]); o.write("n", [0.7])
    x0 = {"m": 0.9, "hh": 0.05, "n": 0.7}
    r = oracle.hh_rates(-30.0)
    o.run(37)
    for k, (a, bb) in zip(("m", "hh", "n"), ((r[0], r[1]), (r[2], r[3]), (r[4], r[5]))):
        xinf = a / (a + bb)
        expect = xinf + (x0[k] - xinf) * math.exp(-37 * dt * (a + bb))
        assert abs(o.read(k)[0] - expect) < 1e-12


def test_hh_soma_rests_and_fires_under_suprathreshold_clamp():
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH])
    b.add_clamp(0, 0, 100.0, 200.0, 0.12)  # ~9.5 uA/cm2, above the repetitive-firing threshold
    o = oracle.Oracle(_net(b, dt=0.025))
    o.run(4000)  # 100 ms at rest
    v_rest = o.read("V")[0]
    assert -65.5 < v_rest < -64.5 and o.spikes()[0].size == 0
    o.run(8000)  # 200 ms of clamp
    gid, step, t = o.spikes()
    assert gid.size >= 5  # repetitive firing
    isi = np.diff(t)
    assert np.all(isi > 5.0)


# ------------------------------------------------------------------ P7
def test_expsyn_single_event_decays_geometrically():
    """One event of weight w at step k0 on an exponential synapse:
    g_k = w r^(k - k0) after the k-th decay, r = exp(-dt / tau)."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    s = b.add_syn(0, 0, netgen.KIND_EXPSYN, 3.0, 0.0)
    w, t_ev, dt = 0.004, 1.03, 0.1
    b.add_train(s, netgen.PORT_G, w, [t_ev])
    o = oracle.Oracle(_net(b, dt=dt))
    k0 = int(math.floor(t_ev / dt))
    o.run(k0)
    assert o.read("g")[0] == 0.0
    r = math.exp(-dt / 3.0)
    for k in range(1, 60):
        o.run(1)
        assert abs(o.read("g")[0] - w * r ** k) <= 1e-14 * w


# ------------------------------------------------------------------ P9
def _ca_synapse(times_ca, c_pre, c_post=0.0, stc=None, extra_post=None):
    stc = dict(STC if stc is None else stc)
    stc["c_pre"], stc["c_post"] = c_pre, c_post
    stc["sigma_pl"] = 0.0
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    s = b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    b.add_train(s, netgen.PORT_CA, 0.0, times_ca)
    return b, stc


def test_calcium_trace_is_piecewise_geometric():
    """Eq. 19 between jumps: c decays by exp(-dt/tau_c) per step; each
    presynaptic arrival adds c_pre at step floor((t + t_c,delay) / dt)."""
    t_pre = np.array([3.3, 10.1, 10.9, 55.0])
    b, stc = _ca_synapse(t_pre, 1.0)
    o = oracle.Oracle(_net(b, stc=stc))
    dt = 0.2
    k_j = np.floor((t_pre + STC["t_cd"]) / dt).astype(int)
    r = math.exp(-dt / STC["tau_c"])
    above = 0
    for k in range(1, 600):
        o.run(1)
        c = o.read("c")[0]
        # after step k-1: jumps delivered at steps <= k-1, then k-1-k_j+1 decays
        expect = sum(1.0 * r ** (k - kj) for kj in k_j if kj <= k - 1)
        assert abs(c - expect) <= 1e-13 * max(1.0, expect)
        above += c > 1.2
    assert above > 0


# ------------------------------------------------------------------ P10
def _affine_runs(h, runs, dt, stc):
    """Compose the closed forms of h <- a h + b over runs of constant
    (Theta_p, Theta_d): h_k = a^k h + b (1 - a^k) / (1 - a)."""
    for thp, thd, k in runs:
        if k == 0:
            continue
        eps = dt / stc["tau_h"]
        a = 1.0 - eps * (0.1 + stc["gamma_p"] * thp + stc["gamma_d"] * thd)
        bb = eps * (0.1 * stc["h0"] + 10.0 * stc["gamma_p"] * thp)
        h = a ** k * h + bb * (1.0 - a ** k) / (1.0 - a)
    return h


def _runs_from_trace(cs, stc):
    runs = []
    for c in cs:
        key = (1.0 if c > stc["theta_p"] else 0.0, 1.0 if c > stc["theta_d"] else 0.0)
        if runs and runs[-1][:2] == key:
            runs[-1] = (key[0], key[1], runs[-1][2] + 1)
        else:
            runs.append((key[0], key[1], 1))
    return runs


@pytest.mark.parametrize("variant", ["table5", "table3_ltp"])
def test_pair_rule_matches_affine_closed_form(variant):
    """Deterministic (sigma_pl = 0) early phase for an isolated pre/post pair
    (Eqs. 17, 19): within each run of constant threshold indicators h obeys
    an affine recurrence with a geometric closed form.  Table 5 amplitudes
    exercise depression only; Table 3's (c_pre = 1, c_post = 2, theta_d = 1,
    theta_p = 1.3) also exercise potentiation."""
    stc = dict(STC)
    stc["sigma_pl"] = 0.0
    if variant == "table3_ltp":
        stc.update(c_pre=1.0, c_post=2.0, theta_d=1.0, theta_p=1.3)
    dt = 0.2
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH])
    s = b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    t_pre = 20.0
    b.add_train(s, netgen.PORT_CA, 0.0, [t_pre])
    b.add_clamp(0, 0, 30.0, 3.0, 0.5)  # one postsynaptic spike near 31 ms
    o = oracle.Oracle(_net(b, stc=stc, dt=dt))
    cs, hs = [], []
    for _ in range(1500):
        # indicators of a step use the calcium after that step's delivery,
        # i.e. c(before decay) = c(after step) / r_c
        o.run(1)
        hs.append(o.read("h")[0])
        cs.append(o.read("c")[0] / math.exp(-dt / stc["tau_c"]))
    gid, step, _ = o.spikes()
    assert gid.size == 1
    k_post = int(step[0]) + 1
    k_pre = int(math.floor((t_pre + stc["t_cd"]) / dt))
    # the calcium trace itself: two jumps, geometric decay
    r = math.exp(-dt / stc["tau_c"])
    expect_c = [sum(a * r ** (k - kj) for a, kj in ((stc["c_pre"], k_pre), (stc["c_post"], k_post)) if kj <= k)
                for k in range(1500)]
    np.testing.assert_allclose(cs, expect_c, rtol=1e-12, atol=1e-15)
    runs = _runs_from_trace(expect_c, stc)
    h_end = _affine_runs(stc["h0"], runs, dt, stc)
    assert abs(hs[-1] - h_end) <= 1e-12 * stc["h0"]
    dh = hs[-1] - stc["h0"]
    if variant == "table5":
        assert dh < 0                       # depression only
    else:
        assert dh > 0 and any(r_[0] for r_ in runs)


def test_pair_rule_continuous_limit():
    """Same pair: the continuous-time change, with times above threshold
    T = tau_c ln(c_peak / theta) per decay segment, agrees to O(dt)."""
    stc = dict(STC)
    stc["sigma_pl"] = 0.0
    stc.update(c_pre=1.0, c_post=2.0, theta_d=1.0, theta_p=1.3)
    b, _ = _ca_synapse([10.0], 1.0)
    # a single presynaptic calcium jump of 2.0 (above theta_p): times above
    # thresholds are tau_c ln(2/1.3) and tau_c ln(2/1.0)
    for dt in (0.2, 0.05):
        st = dict(stc)
        st["c_pre"] = 2.0
        bb = netgen._Builder()
        bb.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
        s = bb.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
        bb.add_train(s, netgen.PORT_CA, 0.0, [10.0])
        o = oracle.Oracle(_net(bb, stc=st, dt=dt))
        o.run(int(round(200.0 / dt)))
        h_num = o.read("h")[0]
        Tp = st["tau_c"] * math.log(2.0 / 1.3)
        Td = st["tau_c"] * math.log(2.0 / 1.0)
        h = st["h0"]
        for thp, T in ((1.0, Tp), (0.0, Td - Tp)):
            lam = (0.1 + st["gamma_p"] * thp + st["gamma_d"]) / st["tau_h"]
            hinf = (0.1 * st["h0"] + 10.0 * st["gamma_p"] * thp) / (0.1 + st["gamma_p"] * thp + st["gamma_d"])
            h = hinf + (h - hinf) * math.exp(-lam * T)
        lam0 = 0.1 / st["tau_h"]
        h = st["h0"] + (h - st["h0"]) * math.exp(-lam0 * (200.0 - 10.0 - st["t_cd"] - Td))
        err = abs(h_num - h)
        assert err < 2.0 * dt * abs(h - st["h0"]) / 10.0 + 1e-9, (dt, h_num, h)


# ------------------------------------------------------------------ P11/P12
def _plastic_cell(h_init, p_init, z_init=0.0, n_syn=1):
    stc = dict(STC)
    stc["sigma_pl"] = 0.0
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    for _ in range(n_syn):
        b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    o = oracle.Oracle(_net(b, stc=stc))
    o.write("h", np.full(n_syn, h_init))
    o.write("p", [p_init])
    o.write("z", np.full(n_syn, z_init))
    return o, stc


def test_prp_rises_to_pmax_under_constant_trigger():
    """Eq. 21 with the trigger on: p_n = p_max (1 - (1 - dt/tau_p)^n), never
    above p_max (Table 5: equilibrium under ongoing synthesis).  For a
    single synapse the sum is |h - h0| of that synapse."""
    o, stc = _plastic_cell(STC["h0"] + 2.2, 0.0)
    a = 0.2 / stc["tau_p"]
    o.run(1000)
    p = o.read("p")[0]
    assert abs(p - stc["p_max"] * (1 - (1 - a) ** 1000)) <= 1e-12 * stc["p_max"]
    o2, _ = _plastic_cell(STC["h0"] - 2.0, 0.0)   # |h - h0| = 2.0 < theta_pro
    o2.run(1000)
    assert o2.read("p")[0] == 0.0
    o3, _ = _plastic_cell(STC["h0"] + 1.2, 0.0, n_syn=2)  # 2 x 1.2 > theta_pro: the sum triggers
    o3.run(10)
    assert o3.read("p")[0] > 0.0
    o4, _ = _plastic_cell(STC["h0"], STC["p_max"])
    o4.write("h", [STC["h0"] + 3.0])
    o4.run(5000)
    assert o4.read("p")[0] <= STC["p_max"]


@pytest.mark.parametrize("sign", [1, -1])
def test_late_phase_converges_with_tag_and_prp(sign):
    """Eq. 20 with p = p_max held (trigger on) and the tag set: LTP tag
    z_n = 1 - (1 - z0)(1 - dt p f_int / tau_z)^n; LTD tag z -> -0.5."""
    o, stc = _plastic_cell(STC["h0"] + sign * 3.0, STC["p_max"], z_init=0.1)
    n = 2000
    o.run(n)
    q = 1 - 0.2 * stc["p_max"] * stc["f_int"] / stc["tau_z"]
    z = o.read("z")[0]
    if sign > 0:
        assert abs(z - (1 - (1 - 0.1) * q ** n)) <= 1e-13
    else:
        assert abs(z - (-0.5 + (0.1 + 0.5) * q ** n)) <= 1e-13
    o5, _ = _plastic_cell(STC["h0"] + 0.5, STC["p_max"], z_init=0.1)  # below tag threshold
    o5.run(100)
    assert o5.read("z")[0] == 0.1


# ------------------------------------------------------------------ P13 noise
def test_threefry_outputs_are_uniform_and_avalanche():
    """Counter-based generator (Sec. 2.3): distinct counters give uniformly
    distributed, independent 64-bit words; flipping one input bit flips
    about half of the output bits."""
    rng = np.random.default_rng(1)
    words = np.array([oracle.threefry([i, 0, 0, 0], [7, 3, 0, 0]) for i in range(4096)]).ravel()
    top = (words >> np.uint64(56)).astype(int)
    hist = np.bincount(top, minlength=256)
    chi2 = ((hist - hist.mean()) ** 2 / hist.mean()).sum()
    assert chi2 < 330  # 255 dof, p ~ 1e-3
    bits = np.unpackbits(words.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.005
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2**63, 4, dtype=np.uint64)
        key = rng.integers(0, 2**63, 4, dtype=np.uint64)
        a = oracle.threefry(ctr, key)
        c2 = ctr.copy()
        c2[int(rng.integers(4))] ^= np.uint64(1) << np.uint64(int(rng.integers(64)))
        bb = oracle.threefry(c2, key)
        flips.append(np.unpackbits((a ^ bb).view(np.uint8)).mean())
    assert abs(np.mean(flips) - 0.5) < 0.02


def test_box_muller_normals_have_unit_moments():
    xs = np.array([oracle.normal(17, s, n) for s in range(500) for n in range(40)])
    assert abs(xs.mean()) < 0.03
    assert abs(xs.var() - 1.0) < 0.04
    assert abs((xs ** 4).mean() - 3.0) < 0.25
    # cos/sin of one Box-Muller pair are uncorrelated
    a = np.array([oracle.normal(5, s, 0) for s in range(3000)])
    b = np.array([oracle.normal(5, s, 1) for s in range(3000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.06


def test_early_phase_noise_increment_statistics():
    """Eq. 18 under Euler-Maruyama with both thresholds crossed: the noise
    part of one step has mean 0 and variance 2 sigma_pl^2 dt / tau_h."""
    n_syn = 4000
    stc = dict(STC)
    nets = []
    for sig in (0.0, stc["sigma_pl"]):
        st = dict(stc)
        st["sigma_pl"] = sig
        b = netgen._Builder()
        b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
        for _ in range(n_syn):
            b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
        nets.append(oracle.Oracle(_net(b, stc=st)))
    rng = np.random.default_rng(2)
    samples = []
    for k in range(12):
        h = rng.uniform(3.0, 5.0, n_syn)
        for o in nets:
            o.write("h", h)
            o.write("c", np.full(n_syn, 50.0))  # above both thresholds
        for o in nets:
            o.run(1)
        samples.append(nets[1].read("h") - nets[0].read("h"))
    x = np.concatenate(samples)
    var = 2 * stc["sigma_pl"] ** 2 * 0.2 / stc["tau_h"]
    z = x / math.sqrt(var)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.04
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-3


# ------------------------------------------------------------------ P8 routing
def test_event_routing_matches_brute_force():
    """Every spike reaches each target synapse of its source through each
    port of the connection at step floor((t* + d)/dt) (conductance) and
    floor((t* + d + t_c,delay)/dt) (calcium) (delays: Sec. 3.8, Eq. 19);
    trains arrive at floor(t/dt).  Multiset of (synapse, port, step) versus
    an enumeration of spikes x connections."""
    net = netgen.tiny(seed=9, n_cells=11, t_end=150.0)
    o = oracle.Oracle(net)
    n_steps = 750
    o.run(n_steps)
    gid, step, ts = o.spikes()
    assert gid.size > 5
    dt, tcd = net["dt"], net["stc"]["t_cd"]
    n_syn = len(net["syn_cell"])
    cnt = np.zeros((n_syn, 2), np.uint64)
    ssum = np.zeros((n_syn, 2), np.uint64)

    def add(s, port, k):
        if k < n_steps:
            cnt[s, port] += np.uint64(1)
            ssum[s, port] += np.uint64(k)
    for g, t in zip(gid, ts):
        for k in np.nonzero(net["conn_src"] == g)[0]:
            te = t + net["conn_d"][k]
            if net["conn_ports"][k] & 1:
                add(net["conn_dst"][k], 0, int(math.floor(te / dt)))
            if net["conn_ports"][k] & 2:
                add(net["conn_dst"][k], 1, int(math.floor((te + tcd) / dt)))
    for tr in range(len(net["train_dst"])):
        for t in net["train_times"][net["train_off"][tr]:net["train_off"][tr + 1]]:
            if net["train_ports"][tr] & 1:
                add(net["train_dst"][tr], 0, int(math.floor(t / dt)))
            if net["train_ports"][tr] & 2:
                add(net["train_dst"][tr], 1, int(math.floor((t + tcd) / dt)))
    c2, s2 = o.event_stats()
    np.testing.assert_array_equal(c2, cnt)
    np.testing.assert_array_equal(s2, ssum)


# ------------------------------------------------------------------ Table 5
def test_table5_constants_and_relations():
    g = json.load(open(os.path.join(GOLD, "table5_stc.json")))
    h0 = 10.0 * 0.5 * g["gamma_p"] / (g["gamma_p"] + g["gamma_d"])
    assert abs(h0 - g["h0_printed_mV"]) < 5e-6
    assert abs(0.5 * h0 - g["theta_pro_printed_mV"]) < 5e-6
    assert abs(0.2 * h0 - g["theta_tag_printed_mV"]) < 5e-7
    assert abs(STC["h0"] - h0) < 1e-12
    assert abs(STC["theta_pro"] - 0.5 * h0) < 1e-12
    assert abs(STC["theta_tag"] - 0.2 * h0) < 1e-12
    for k_json, k in (("tau_c_ms", "tau_c"), ("tau_h_ms", "tau_h"), ("tau_p_ms", "tau_p"),
                      ("tau_z_ms", "tau_z"), ("gamma_p", "gamma_p"), ("gamma_d", "gamma_d"),
                      ("theta_p", "theta_p"), ("theta_d", "theta_d"), ("sigma_pl_mV", "sigma_pl"),
                      ("p_max", "p_max"), ("f_int", "f_int"), ("t_c_delay_ms", "t_cd"),
                      ("c_pre", "c_pre"), ("c_post", "c_post")):
        assert STC[k] == g[k_json], k
    assert netgen.CA_INVIVO == {"c_pre": g["c_pre_in_vivo"], "c_post": g["c_post_in_vivo"]}


# ------------------------------------------------------------------ input errors
def test_oracle_rejects_invalid_networks():
    b = netgen._Builder()
    b.add_cell([-1, 1], [10.0, 10.0], [1.0, 1.0], [1, 0])  # parent[1] = 1 is not < 1
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(_net(b))
    b = netgen._Builder()
    b.add_cell([-1], [10.0], [1.0], [1])
    s = b.add_syn(0, 0, netgen.KIND_EXPSYN)
    b.add_conns([0], [s], netgen.PORT_CA, 0.1, 1.0)  # calcium port on a plain synapse
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(_net(b))
    b = netgen._Builder()
    b.add_cell([-1], [10.0], [1.0], [1])
    s = b.add_syn(0, 0, netgen.KIND_EXPSYN)
    b.add_conns([0], [s], netgen.PORT_G, 0.1, 0.05)  # delay below dt
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(_net(b))


# ------------------------------------------------------------------ Poisson drive
def test_poisson_source_is_a_poisson_process():
    """Counter-based Poisson sources: inter-arrival times are exponential with
    mean 1000/rate ms (KS test), and the arrivals delivered to a synapse over
    T count like Poisson(rate T)."""
    from scipy import stats
    rate = 80.0
    isi = np.array([oracle.poisson_isi(99, 3, j, rate) for j in range(20000)])
    assert stats.kstest(isi, "expon", args=(0, 1000.0 / rate)).pvalue > 1e-3
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    s = b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    b.add_poisson(s, netgen.PORT_G | netgen.PORT_CA, 0.0, rate)
    b.add_poisson(s, netgen.PORT_G, 0.0, 0.0)  # rate 0: silent
    o = oracle.Oracle(_net(b))
    n_steps = 25000  # 5 s
    o.run(n_steps)
    cnt, ssum = o.event_stats()
    lam = rate * 5.0
    assert abs(int(cnt[0, 0]) - lam) < 5 * math.sqrt(lam)
    # calcium events trail the conductance events by t_c,delay (94 steps)
    assert int(cnt[0, 0]) - int(cnt[0, 1]) <= 8


# ------------------------------------------------------------------ Eq. 16 at the conductance port
@pytest.mark.parametrize("h_init,z_init", [(STC["h0"], 1.0), (STC["h0"] + 1.7, 0.0), (STC["h0"] - 0.9, -0.35),
                                           (2.5, 0.6)])
def test_conductance_port_scales_with_total_weight(h_init, z_init):
    """Eq. 16: the total weight of a plastic synapse is w = h + h0 z, h0 its
    baseline; a conductance-port event adds the connection weight times
    w / h0 (reading R10).  So z = 1 at h = h0 doubles the increment of a
    plain synapse, and z = 0 scales it by h / h0."""
    stc = dict(STC)
    stc["sigma_pl"] = 0.0
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    s_stc = b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    s_exp = b.add_syn(0, 0, netgen.KIND_EXPSYN, 5.0, 0.0)
    w = 0.0037
    b.add_train(s_stc, netgen.PORT_G, w, [0.05])   # delivered at step 0
    b.add_train(s_exp, netgen.PORT_G, w, [0.05])
    o = oracle.Oracle(_net(b, stc=stc))
    o.write("h", [h_init, 0.0])
    o.write("z", [z_init, 0.0])
    o.run(1)
    r = math.exp(-0.2 / 5.0)
    g = o.read("g")
    total = h_init + STC["h0"] * z_init
    assert abs(g[0] - w * r * total / STC["h0"]) <= 1e-15 * w
    assert abs(g[1] - w * r) <= 1e-15 * w
    if h_init == STC["h0"] and z_init == 1.0:
        assert abs(g[0] - 2.0 * g[1]) <= 1e-15 * w


# ------------------------------------------------------------------ synaptic conductance in the cable step
@pytest.mark.parametrize("g_syn,e_syn", [(0.002, 0.0), (0.02, -80.0), (0.2, 0.0)])
def test_passive_cv_under_constant_synaptic_conductance(g_syn, e_syn):
    """A passive isopotential CV with a synaptic conductance held constant
    (decay time constant so long that the per-step factor is exactly 1):
    the ohmic current g (V - E) of Sec. 2.4 enters the backward-Euler step
    of Eq. 4 implicitly, so V_n relaxes geometrically toward
    V_inf = (g_pas E_pas + g E) / (g_pas + g) with ratio 1 / (1 + dt/tau_eff),
    tau_eff = C / (g_pas + g).  An explicit (unlinearised) synaptic term, a
    wrong sign or a wrong reversal potential breaks the closed form."""
    cm, gpas_dens, epas, v0, dt = 1.0, 1e-4, -65.0, -70.0, 0.1
    L, d = 30.0, 7.0
    b = netgen._Builder()
    b.add_cell([-1], [L], [d], [netgen.MECH_PAS], params=_cell_params(v_init=v0, g_pas=gpas_dens, e_pas=epas))
    s = b.add_syn(0, 0, netgen.KIND_EXPSYN, 1e300, e_syn)
    b.add_train(s, netgen.PORT_G, g_syn, [0.0])
    o = oracle.Oracle(_net(b, dt=dt))
    area = math.pi * d * L                      # um^2
    C = 1e-5 * cm * area                        # nF
    gpas = 1e-2 * gpas_dens * area              # uS
    v_inf = (gpas * epas + g_syn * e_syn) / (gpas + g_syn)
    q = 1.0 / (1.0 + dt * (gpas + g_syn) / C)
    vs = []
    for _ in range(120):
        o.run(1)
        vs.append(o.read("V")[0])
    n = np.arange(1, 121)
    expect = v_inf + (v0 - v_inf) * q ** n
    np.testing.assert_allclose(vs, expect, rtol=1e-12, atol=1e-12)
    assert o.read("g")[0] == g_syn


# ------------------------------------------------------------------ detection and crossing time
def _passive_clamped(v0, epas, theta, amp, t0=0.0, dur=1e9, dt=0.2, L=20.0, d=20.0):
    b = netgen._Builder()
    b.add_cell([-1], [L], [d], [netgen.MECH_PAS], params=_cell_params(v_init=v0, e_pas=epas))
    if amp != 0.0:
        b.add_clamp(0, 0, t0, dur, amp)
    net = b.finish("pin", dt, 100.0, 11, STC, theta=theta)
    return oracle.Oracle(net)


def test_detector_crossing_step_and_time_on_closed_form_trajectory():
    """A passive CV charged by a steady clamp current I0 follows
    V_n = V_inf + (V_0 - V_inf) / (1 + dt/tau)^n, V_inf = E + I0 / g_pas
    (backward Euler, Eq. 4).  The detector fires in the one step with
    V_n < theta <= V_{n+1}, at the linear interpolation
    t* = t_n + dt (theta - V_n) / (V_{n+1} - V_n) (reading R19), and never
    again while V stays above theta."""
    dt, L, d, cm, gpas_dens, epas, v0, I0, theta = 0.2, 20.0, 20.0, 1.0, 1e-4, -65.0, -65.0, 0.05, -30.0
    o = _passive_clamped(v0, epas, theta, I0, dt=dt, L=L, d=d)
    area = math.pi * d * L
    C, gpas = 1e-5 * cm * area, 1e-2 * gpas_dens * area
    v_inf = epas + I0 / gpas
    q = 1.0 / (1.0 + dt * gpas / C)
    n = np.arange(0, 400)
    v = v_inf + (v0 - v_inf) * q ** n
    k = int(np.nonzero((v[:-1] < theta) & (v[1:] >= theta))[0][0])
    o.run(399)
    gid, step, ts = o.spikes()
    assert gid.size == 1 and int(step[0]) == k
    t_expect = k * dt + dt * (theta - v[k]) / (v[k + 1] - v[k])
    assert abs(ts[0] - t_expect) <= 1e-12 * t_expect
    # the continuous crossing time of the same membrane, to first order in dt
    tau = C / gpas
    t_cont = tau * math.log((v0 - v_inf) / (theta - v_inf))
    assert abs(ts[0] - t_cont) < 0.5 * dt + (dt / tau) * t_cont


def test_detector_threshold_boundaries():
    """The crossing condition is V_n < theta <= V_{n+1}: a voltage that
    starts exactly at theta and rises is not a crossing, and a step that
    lands exactly on theta is one (at t* = t_{n+1})."""
    # starts at theta = 0 and rises toward E = +10 mV: no spike
    o = _passive_clamped(0.0, 10.0, 0.0, 0.0)
    o.run(200)
    assert o.read("V")[0] > 5.0 and o.spikes()[0].size == 0
    # from -10 mV, one clamp step whose charge lands V exactly on theta = 0:
    # b = (C/dt) V_0 + g_pas E_pas + I0 = 0 with E_pas = 0 and I0 = 10 C/dt
    dt, L, d = 0.2, 20.0, 20.0
    cdt = (1e-5 * 1.0 * (math.pi * d * L)) / dt
    o = _passive_clamped(-10.0, 0.0, 0.0, 10.0 * cdt, t0=0.0, dur=0.5 * dt, dt=dt, L=L, d=d)
    o.run(1)
    assert o.read("V")[0] == 0.0
    o.run(50)
    gid, step, ts = o.spikes()
    assert gid.size == 1 and int(step[0]) == 0 and ts[0] == dt


# ------------------------------------------------------------------ HH rates away from rest, resting root
def _hh1952(v):
    """Rate constants (1/ms) in the notation of Hodgkin and Huxley (1952):
    V is the displacement from rest with depolarisation negative, so
    V = -(v - E_rest) for a membrane potential v resting at -65 mV."""
    V = -(v + 65.0)
    am = 0.1 * (V + 25.0) / (math.exp((V + 25.0) / 10.0) - 1.0)
    bm = 4.0 * math.exp(V / 18.0)
    ah = 0.07 * math.exp(V / 20.0)
    bh = 1.0 / (math.exp((V + 30.0) / 10.0) + 1.0)
    an = 0.01 * (V + 10.0) / (math.exp((V + 10.0) / 10.0) - 1.0)
    bn = 0.125 * math.exp(V / 80.0)
    return np.array([am, bm, ah, bh, an, bn])


def test_hh_rates_match_the_1952_formulation_across_voltages():
    """The oracle's rates (written in the modern sign convention with
    exprelr) equal the original paper's expressions over the whole
    physiological range, not only at rest where several exponentials are 1."""
    vs = [v for v in np.linspace(-110.0, 50.0, 97) if min(abs(v + 40.0), abs(v + 55.0)) > 0.5]
    for v in vs:
        np.testing.assert_allclose(oracle.hh_rates(v), _hh1952(v), rtol=2e-13, atol=0)


def test_hh_soma_rests_at_the_root_of_the_steady_state_current():
    """A lone HH CV settles where the membrane current with gates at their
    steady states vanishes (the resting potential of the model, about
    -64.974 mV with these parameters, reading R6).  The discrete step's
    fixed point is that root exactly, so the long-run voltage agrees to
    1e-6 mV with a root found here from the 1952 rate expressions."""
    from scipy.optimize import brentq
    P = netgen.DEFAULT_CELL
    gna, gk, gl, ena, ek, el = P[5], P[6], P[7], P[8], P[9], P[10]

    def i_ss(v):
        am, bm, ah, bh, an, bn = _hh1952(v)
        m, h, n = am / (am + bm), ah / (ah + bh), an / (an + bn)
        return gna * m ** 3 * h * (v - ena) + gk * n ** 4 * (v - ek) + gl * (v - el)

    root = brentq(i_ss, -70.0, -60.0, xtol=1e-13)
    assert abs(root - (-64.974)) < 5e-4
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH])
    o = oracle.Oracle(_net(b, dt=0.2))
    o.run(20000)  # 4 s
    assert abs(o.read("V")[0] - root) < 1e-6


def test_threaded_oracle_build_gives_the_same_bits():
    """The OpenMP build (timing on several host cores) computes every value
    by the same expressions in the same order: identical raster and state."""
    net = netgen.tiny(seed=3, n_cells=13, t_end=100.0)
    a, b = oracle.Oracle(net), oracle.Oracle(net, threaded=True)
    a.run(400)
    b.run(400)
    for x, y in zip(a.spikes(), b.spikes()):
        np.testing.assert_array_equal(x, y)
    for k in ("V", "m", "hh", "n", "g", "c", "h", "z", "p"):
        np.testing.assert_array_equal(a.read(k), b.read(k), err_msg=k)
