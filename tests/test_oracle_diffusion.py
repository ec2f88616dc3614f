"""Pins of the oracle's particle-diffusion model (Eq. 5 of Sec. 2.4; the
SPS / PRP formulation of Sec. 3.6 with the threshold of Eq. 23) against
facts that do not come from the oracle: conservation of the diffused
amount, the exact discrete decay of a cosine mode on a sealed cable, the
two limits of the diffusivity (a well-mixed cell follows the per-cell rule
of Eq. 21; no diffusion keeps each species where it is made), and the
threshold and synthesis scaling of Eq. 23."""
import math

import numpy as np
import pytest

import netgen
import oracle

STC = dict(netgen.STC_TABLE5)


def _vol(net):
    r = 0.5 * net["diam"]
    return math.pi * r * r * net["length"]


def _passive_tree(seed=3, n=40):
    rng = np.random.default_rng(seed)
    parent = [-1] + [int(rng.integers(0, i)) for i in range(1, n)]
    length = rng.uniform(2.0, 15.0, n)
    diam = rng.uniform(0.5, 3.0, n)
    return parent, length, diam


def test_diffusion_conserves_the_amount_of_sps():
    """Without release the axial fluxes only move SPS between CVs: the
    amount sum_i V_i X_i is invariant (sealed ends, Eq. 5 with phi = 0)."""
    b = netgen._Builder()
    for k in range(3):
        parent, length, diam = _passive_tree(seed=k)
        b.add_cell(parent, length, diam, [netgen.MECH_PAS] * len(parent))
    net = b.finish("cons", 0.2, 50.0, 1, STC)
    net = netgen.with_diffusion(net, d_sps=0.7, d_prp=0.0)
    o = oracle.Oracle(net)
    x = np.random.default_rng(4).uniform(0.0, 3.0, o.n_cv)
    o.write("sps", x)
    vol = _vol(net)
    amount0 = np.add.reduceat(vol * x, net["cv_off"][:-1])
    o.run(60)
    y = o.read("sps")
    amount = np.add.reduceat(vol * y, net["cv_off"][:-1])
    np.testing.assert_allclose(amount, amount0, rtol=1e-13, atol=0)
    assert np.abs(y - x).max() > 0.1  # it diffused


@pytest.mark.parametrize("n_cv,mode", [(16, 1), (33, 3)])
def test_cosine_mode_decays_by_the_discrete_eigenvalue(n_cv, mode):
    """On a uniform sealed cable of N CVs of length h the finite-volume
    Laplacian has the eigenvectors cos(pi k (i + 1/2) / N) with eigenvalues
    (2 D / h^2)(1 - cos(pi k / N)); backward Euler multiplies the mode by
    1 / (1 + dt lambda) per step."""
    h, d, D, dt = 2.5, 1.3, 0.9, 0.2
    b = netgen._Builder()
    b.add_cell([-1] + list(range(n_cv - 1)), [h] * n_cv, [d] * n_cv, [netgen.MECH_PAS] * n_cv)
    net = netgen.with_diffusion(b.finish("mode", dt, 50.0, 1, STC), d_sps=D, d_prp=D)
    o = oracle.Oracle(net)
    i = np.arange(n_cv)
    x0 = np.cos(math.pi * mode * (i + 0.5) / n_cv)
    o.write("sps", x0)
    lam = (2.0 * D / h ** 2) * (1.0 - math.cos(math.pi * mode / n_cv))
    g = 1.0 / (1.0 + dt * lam)
    for n in (1, 5, 40):
        o.run(n - (o.step))
        np.testing.assert_allclose(o.read("sps"), g ** n * x0, rtol=0, atol=1e-12)
    # the continuous mode decays as exp(-D (pi k / L)^2 t): the discrete
    # factor approaches it to first order in dt and second order in h
    L = n_cv * h
    cont = math.exp(-D * (math.pi * mode / L) ** 2 * 40 * dt)
    assert abs(g ** 40 - cont) < 0.05 * cont


def _plastic_tiny(d_sps, d_prp, seed=3):
    net = netgen.tiny(seed=seed, n_cells=9, t_end=100.0)
    return net, (netgen.with_diffusion(net, d_sps, d_prp) if d_sps is not None else net)


def _seed_state(net, sims, rng):
    kinds = net["syn_kind"] == 1
    n = len(kinds)
    h0 = STC["h0"]
    h = np.where(kinds, rng.uniform(h0 - 2.5, h0 + 2.5, n), h0)
    z = np.where(kinds, rng.uniform(-0.4, 0.9, n), 0.0)
    c = np.where(kinds, rng.uniform(0.0, 5.0, n), 0.0)
    for s in sims:
        s.write("h", h)
        s.write("z", z)
        s.write("c", c)
    return h


def test_fast_diffusion_reproduces_the_per_cell_rule():
    """With a diffusivity far above the cells' size squared over dt, every
    CV holds the cell's mean concentration: the soma's SPS concentration
    is sum |h - h0| / V_tot, so its test against theta_pro / V_tot (Eq. 23)
    is Eq. 21's test of the sum against theta_pro, and the protein is the
    per-cell p of Eq. 21 in every CV.  Both runs must agree on rasters, h,
    z and p."""
    base, fast = _plastic_tiny(1e7, 1e7)
    a, b = oracle.Oracle(base), oracle.Oracle(fast)
    rng = np.random.default_rng(1)
    h = _seed_state(base, (a, b), rng)
    p = rng.uniform(0.0, 8.0, a.n_cells)
    a.write("p", p)
    vol = _vol(base)
    cv_off = base["cv_off"]
    kinds = base["syn_kind"] == 1
    S = np.zeros(a.n_cells)
    np.add.at(S, base["syn_cell"][kinds], np.abs(h[kinds] - STC["h0"]))
    vtot = np.add.reduceat(vol, cv_off[:-1])
    cell_of_cv = np.repeat(np.arange(a.n_cells), np.diff(cv_off))
    b.write("sps", (S / vtot)[cell_of_cv])
    b.write("prp", p[cell_of_cv])
    # the trigger sums must not sit at the threshold
    assert np.abs(S - STC["theta_pro"]).min() > 1e-6
    for _ in range(4):
        a.run(100)
        b.run(100)
    ga, gb = a.spikes(), b.spikes()
    assert ga[0].size > 5
    for x, y in zip(ga, gb):
        np.testing.assert_array_equal(x, y) if x.dtype != np.float64 else np.testing.assert_allclose(x, y, rtol=1e-12)
    np.testing.assert_allclose(b.read("h"), a.read("h"), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b.read("z"), a.read("z"), rtol=1e-9, atol=1e-12)
    prp = b.read("prp")
    np.testing.assert_allclose(prp, a.read("p")[cell_of_cv], rtol=1e-9, atol=1e-12)
    assert a.read("p").max() > p.max() * 0.5  # the protein moved


def test_without_diffusion_the_species_stay_where_they_are_made():
    """D = 0: each CV's SPS amount V_i X_i is the sum over its plastic
    synapses of |h - h0| (it starts at 0 with h = h0, and each step releases
    the change of |h - h0|); the protein appears only in the soma CV,
    where it follows the single-compartment recurrence with the synthesis
    scaled by V_tot / V_soma."""
    _, net = _plastic_tiny(0.0, 0.0, seed=5)
    o = oracle.Oracle(net)
    rng = np.random.default_rng(2)
    kinds = net["syn_kind"] == 1
    c = np.where(kinds, rng.uniform(1.5, 6.0, len(kinds)), 0.0)
    o.write("c", c)
    o.run(40)
    vol = _vol(net)
    h = o.read("h")
    cv = net["cv_off"][net["syn_cell"]] + net["syn_cv"]
    amount = np.zeros(o.n_cv)
    np.add.at(amount, cv[kinds], np.abs(h[kinds] - STC["h0"]))
    np.testing.assert_allclose(vol * o.read("sps"), amount, rtol=1e-12, atol=1e-14)
    assert amount.max() > 1e-3
    soma = net["cv_off"][:-1] + net["detector"]
    prp = o.read("prp")
    off = np.ones(o.n_cv, bool)
    off[soma] = False
    assert np.all(prp[off] == 0.0)


def test_synthesis_threshold_and_scaling_of_eq23():
    """The soma synthesises while its SPS concentration exceeds
    theta_pro / V_tot (Eq. 23), at the rate that makes the well-mixed cell
    follow Eq. 21: under a constant trigger and fast diffusion every CV
    holds p_max (1 - (1 - dt/tau_p)^n)."""
    b = netgen._Builder()
    parent, length, diam = _passive_tree(seed=9, n=25)
    b.add_cell(parent, length, diam, [netgen.MECH_PAS] * 25, detector=4)
    b.add_cell(parent, length, diam, [netgen.MECH_PAS] * 25, detector=4)
    net0 = b.finish("eq23", 0.2, 50.0, 1, STC)
    vol = _vol(net0)
    vtot = vol[:25].sum()
    thr = STC["theta_pro"] / vtot
    # D = 0 so the soma keeps the written concentration: cell 0 just above
    # the threshold, cell 1 just below
    net = netgen.with_diffusion(net0, 0.0, 0.0)
    o = oracle.Oracle(net)
    x = np.concatenate([np.full(25, thr * (1 + 1e-9)), np.full(25, thr * (1 - 1e-9))])
    o.write("sps", x)
    o.run(1)
    prp = o.read("prp")
    assert prp[4] > 0.0 and prp[25 + 4] == 0.0
    ap = 0.2 / STC["tau_p"]
    np.testing.assert_allclose(prp[4], ap * STC["p_max"] * vtot / vol[4], rtol=1e-13)
    # fast diffusion, a trigger that stays on
    # (the spread a step leaves shrinks as 1/D, about 3e-5 of the mean
    # here; the rounding of the elimination, where V_i is small against
    # dt D A / l, grows with D)
    net = netgen.with_diffusion(net0, 0.0, 1e9)
    o = oracle.Oracle(net)
    o.write("sps", np.full(50, 10.0 * thr))
    n = np.arange(1, 301)
    got = []
    for _ in n:
        o.run(1)
        got.append(o.read("prp")[:25].copy())
    want = STC["p_max"] * (1.0 - (1.0 - ap) ** n)
    np.testing.assert_allclose(np.array(got), np.repeat(want[:, None], 25, 1), rtol=1e-4, atol=0)
    # the amount (volume-weighted mean) carries no spread
    mean = (np.array(got) * vol[None, :25]).sum(1) / vtot
    np.testing.assert_allclose(mean, want, rtol=1e-8, atol=0)
