"""GPU parity: the HIP library against the CPU oracle on the same seeded
networks, through the C ABI.

Bar (FP64 forms): spike rasters identical in count, order (step, gid) and
crossing step; crossing times within 1e-9 relative; delivered-event
multiset per (synapse, port) identical (count and sum of delivery steps);
voltages |dV| <= 1e-9 max(|V|, 1 mV); other state within 1e-9 relative.
Transcendentals (exp, log, sin, cos) differ in the last ulp between the
host C library and the device math library, which is all that separates
the two sides' FP64 arithmetic; the event-driven coupling between cells is
quantised to steps, so these ulps do not reach the rasters.
"""
import numpy as np
import pytest

import netgen
import oracle
from _parity import (assert_raster_equal, assert_routing_equal, assert_state_close,
                     assert_v_close, run_pair)
from paper_2411_16445_amd import PAError, Simulation
from paper_2411_16445_amd import binding as B

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("seed", [3, 7, 11])
def test_tiny_networks_match_oracle(seed, mode):
    net = netgen.tiny(seed=seed, n_cells=13, t_end=200.0)
    _say(f"tiny seed={seed} mode={mode}")
    o, s = run_pair(net, 1000, chunks=3, mode=mode)
    n = assert_raster_equal(o, s)
    assert n > 10
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_single_synapse_config_full_horizon(mode):
    """1 cell, 9 CVs, one plastic synapse at 20 Hz, 10 s (50,000 steps)."""
    net = netgen.config1()
    _say(f"config1 10s mode={mode}")
    o, s = run_pair(net, 50000, chunks=2, mode=mode)
    assert assert_raster_equal(o, s) > 50
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_ei_network_full_size_short_horizon(mode):
    """2000 ball-and-stick cells, ~400k synapses (~255k plastic), 60 ms."""
    net = netgen.config2(t_end=200.0)
    _say(f"config2 full size 300 steps mode={mode}")
    o, s = run_pair(net, 300, chunks=2, mode=mode)
    assert assert_raster_equal(o, s) > 100
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_long_dendrite_network_full_size_short_horizon(mode):
    """The E/I network with 100-CV dendrites (2000 x 101 CVs), 40 ms, FP64:
    long unbranched cells through the elimination at full size."""
    net = netgen.config4(t_end=100.0)
    _say(f"config4 full size 200 steps mode={mode}")
    o, s = run_pair(net, 200, chunks=2, mode=mode)
    assert assert_raster_equal(o, s) > 100
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_uneven_trees_full_size_short_horizon(mode):
    """4096 random trees of 10-300 CVs, 100 plastic sites each, 30 ms."""
    net = netgen.config3(t_end=60.0)
    _say(f"config3 full size 150 steps mode={mode}")
    o, s = run_pair(net, 150, mode=mode)
    assert_raster_equal(o, s)
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_heavy_input_matches_oracle(mode):
    """Several events per cell and step (20 kHz of external arrivals per
    cell): the epoch's events exceed the fused kernel's LDS event buffer, so
    the workgroup's events are gathered into its queue in global memory."""
    net = netgen.tiny(seed=12, n_cells=9, t_end=60.0, ext_rate=20000.0, w_ext=0.0005)
    _say(f"heavy input mode={mode}")
    o, s = run_pair(net, 300, chunks=2, mode=mode)
    assert_raster_equal(o, s)
    assert_routing_equal(o, s)
    assert_state_close(o, s)
    assert s.stats()["events"] > 300 * 9 * 4


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_device_poisson_sources_match_oracle(mode):
    """Poisson drive drawn on the device from the counter-based generator:
    the same arrivals as the oracle's (identical rasters and deliveries)."""
    net = netgen.tiny(seed=14, n_cells=11, t_end=150.0, poisson=True, ext_rate=300.0)
    for k in ("train_dst", "train_ports", "train_w"):
        net[k] = net[k][:0]
    net["train_off"] = net["train_off"][:1]
    net["train_times"] = net["train_times"][:0]
    _say(f"poisson mode={mode}")
    o, s = run_pair(net, 750, chunks=3, mode=mode)
    assert assert_raster_equal(o, s) > 10
    assert_routing_equal(o, s)
    assert_state_close(o, s)


def test_probes_sample_the_oracle_trajectory():
    net = netgen.tiny(seed=5, n_cells=7, t_end=100.0)
    probes = [("V", 0), ("V", int(net["cv_off"][3]) + 1), ("p", 2)]
    stc_syn = int(np.nonzero(net["syn_kind"] == 1)[0][0])
    probes += [("g", stc_syn), ("c", stc_syn), ("h", stc_syn), ("z", stc_syn)]
    _say("probes tiny seed=5")
    s = Simulation(net, probes=probes, probe_stride=3)
    o = oracle.Oracle(net)
    rows = []
    for _ in range(100):
        o.run(3)
        v = o.read("V")
        rows.append([v[0], v[probes[1][1]], o.read("p")[2], o.read("g")[stc_syn],
                     o.read("c")[stc_syn], o.read("h")[stc_syn], o.read("z")[stc_syn]])
    s.advance_steps(150)
    s.advance_steps(150)
    got = s.probes()
    assert got.shape == (100, 7)
    np.testing.assert_allclose(got, np.array(rows), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_probes_with_their_own_strides(mode):
    """Each probe samples after every stride-th step of its own (1, 4, 7,
    10), across advances that end between samples."""
    net = netgen.tiny(seed=5, n_cells=7, t_end=100.0)
    strides = [1, 4, 7, 10]
    probes = [("V", 0, 1), ("V", int(net["cv_off"][3]) + 1, 4), ("p", 2, 7), ("V", 5, 10)]
    _say(f"probe strides mode={mode}")
    s = Simulation(net, mode=mode, probes=probes)
    o = oracle.Oracle(net)
    want = [[] for _ in probes]
    for n in range(1, 141):
        o.run(1)
        for k, (q, i, st) in enumerate(probes):
            if n % st == 0:
                want[k].append(o.read(q)[i])
    for m in (13, 50, 1, 76):
        s.advance_steps(m)
    for k, st in enumerate(strides):
        got = s.probe(k)
        assert got.size == 140 // st
        np.testing.assert_allclose(got, np.array(want[k]), rtol=1e-9, atol=1e-12)


def test_noise_path_matches_bitwise_generator():
    """Both thresholds crossed on many synapses: one step of h carries the
    Threefry + Box-Muller normal; agreement to 1e-12 means the device
    generator produced the same 64-bit words as the oracle's."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    for _ in range(3000):
        b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    net = b.finish("noise", 0.2, 10.0, 123456789, netgen.STC_TABLE5)
    o = oracle.Oracle(net)
    s = Simulation(net)
    rng = np.random.default_rng(0)
    for k in range(6):
        h = rng.uniform(3.0, 5.0, 3000)
        for x in (o, s):
            x.write("h", h)
            x.write("c", np.full(3000, 50.0))
        o.run(1)
        s.advance_steps(1)
        ho, hs = o.read("h"), s.read("h")
        assert np.abs(hs - ho).max() <= 1e-12 * np.abs(ho).max()
        assert np.abs(ho - h).max() > 1e-6  # the noise is there


def test_mixed_noise_of_paired_synapses_matches_single_draws():
    """The mixed form draws the noise of a lane's two synapses in one call in
    256-lane workgroups and with one call per synapse in smaller ones: the
    same bits either way, for synapses above one calcium threshold, both or
    none.  Against the oracle's FP64 normal the FP32 normal and factor stay
    within 5e-3 of the largest increment (a wrong threshold sum is off by
    41 %, a wrong word pair by the whole increment)."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_PAS])
    n = 3000
    for _ in range(n):
        b.add_syn(0, 0, netgen.KIND_STC, 5.0, 0.0)
    net = b.finish("noise", 0.2, 10.0, 123456789, netgen.STC_TABLE5)
    o = oracle.Oracle(net)
    sims = []
    for bt, sw in ((128, 1), (256, 3)):
        s = Simulation(net, mode="batched", precision="mixed", exchange="kernel", cells_per_block=1,
                       block_threads=bt, solver_waves=sw)
        assert s.stats()["block_threads"] == bt
        sims.append(s)
    rng = np.random.default_rng(1)
    for k in range(4):
        _say(f"mixed paired noise step {k}")
        h = rng.uniform(3.0, 5.0, n)
        c = rng.choice([0.5, 2.0, 50.0], n)
        for x in [o] + sims:
            x.write("h", h)
            x.write("c", c)
        o.run(1)
        for s in sims:
            s.advance_steps(1)
        ho = o.read("h")
        h128, h256 = (s.read("h") for s in sims)
        np.testing.assert_array_equal(h128, h256)
        inc = np.abs(ho - h)
        assert np.abs(h256 - ho).max() <= 5e-3 * inc.max()
        drawn = c > 1.2
        assert np.abs(h256 - h)[drawn].min() > 0.0
        assert np.abs(h256 - ho)[~drawn].max() <= 1e-12 * np.abs(ho).max()


def test_gpu_runs_are_deterministic():
    net = netgen.tiny(seed=21, n_cells=17, t_end=150.0)
    _say("determinism tiny seed=21")
    r = []
    for _ in range(2):
        s = Simulation(net)
        s.advance_steps(750)
        r.append((s.spikes(), s.read("V"), s.read("h"), s.read("g")))
    for a, b in zip(r[0][0], r[1][0]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(r[0][1:], r[1][1:]):
        np.testing.assert_array_equal(a, b)


def test_plain_and_batched_forms_are_bitwise_identical():
    net = netgen.tiny(seed=8, n_cells=23, t_end=150.0)
    _say("plain vs batched tiny seed=8")
    out = []
    for mode in ("plain", "batched"):
        s = Simulation(net, mode=mode)
        s.advance_steps(700)
        out.append((s.spikes(), s.read("V"), s.read("h"), s.read("z"), s.read("g"), s.read("c")))
    for a, b in zip(out[0][0], out[1][0]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(out[0][1:], out[1][1:]):
        np.testing.assert_array_equal(a, b)


SHAPES = [
    dict(exchange="kernel", cells_per_block=1, block_threads=64),
    dict(exchange="kernel", cells_per_block=4, block_threads=256, solver_waves=2),
    dict(exchange="resident", cells_per_block=4, block_threads=128, solver_waves=1),
    dict(exchange="resident", cells_per_block=8, block_threads=256, solver_waves=3),
]


def test_workgroup_shapes_and_exchange_modes_are_bitwise_identical():
    """The FP64 batched form gives the same bits whatever the packing, the
    split of wavefront roles and the spike-exchange mode (separate kernel,
    or resident workgroups behind a grid barrier), and the same as the
    plain form."""
    net = netgen.tiny(seed=8, n_cells=23, t_end=150.0)
    ref = Simulation(net, mode="plain")
    ref.advance_steps(700)
    want = (ref.spikes(), [ref.read(k) for k in ("V", "h", "z", "g", "c", "p")], ref.event_stats())
    for shape in SHAPES:
        _say(f"shape {shape}")
        s = Simulation(net, mode="batched", **shape)
        st = s.stats()
        assert st["exchange"] == (2 if shape["exchange"] == "resident" else 1)
        assert st["block_threads"] == shape["block_threads"]
        s.advance_steps(350)
        s.advance_steps(350)
        for a, b in zip(want[0], s.spikes()):
            np.testing.assert_array_equal(a, b)
        for a, k in zip(want[1], ("V", "h", "z", "g", "c", "p")):
            np.testing.assert_array_equal(a, s.read(k), err_msg=k)
        for a, b in zip(want[2], s.event_stats()):
            np.testing.assert_array_equal(a, b)


def test_retune_keeps_the_state_and_the_fp64_bits():
    """pa_retune re-times the plans from the present state and restores it:
    no step advances, the state reads the same, and the FP64 batched form
    continues with the bits of a run that was never retuned (the same bits
    under every plan).  The plain form has no plan to tune."""
    net = netgen.tiny(seed=8, n_cells=23, t_end=150.0)
    _say("retune tiny seed=8")
    ref = Simulation(net, mode="batched")
    ref.advance_steps(700)
    s = Simulation(net, mode="batched")
    s.advance_steps(350)
    before = [s.read(k) for k in ("V", "h", "z", "g", "c", "p")]
    steps = s.stats()["steps"]
    s.retune()
    assert s.stats()["steps"] == steps
    for a, k in zip(before, ("V", "h", "z", "g", "c", "p")):
        np.testing.assert_array_equal(a, s.read(k), err_msg=k)
    s.advance_steps(350)
    for a, b in zip(ref.spikes(), s.spikes()):
        np.testing.assert_array_equal(a, b)
    for k in ("V", "h", "z", "g", "c", "p"):
        np.testing.assert_array_equal(ref.read(k), s.read(k), err_msg=k)
    for a, b in zip(ref.event_stats(), s.event_stats()):
        np.testing.assert_array_equal(a, b)
    m = Simulation(net, mode="batched", precision="mixed")
    m.advance_steps(200)
    vm = m.read("V")
    m.retune()
    np.testing.assert_array_equal(vm, m.read("V"))
    m.advance_steps(100)
    assert np.isfinite(m.read("V")).all()
    # resident plans only: the grid barrier's counts start again with the
    # new plan, whatever its number of workgroups
    r = Simulation(net, mode="batched", exchange="resident", block_threads=128)
    r.advance_steps(350)
    r.retune()
    assert r.stats()["exchange"] == 2
    r.advance_steps(350)
    for a, b in zip(ref.spikes(), r.spikes()):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ref.read("V"), r.read("V"))
    p = Simulation(net, mode="plain")
    with pytest.raises(PAError):
        p.retune()


def test_mixed_exchange_modes_are_bitwise_identical():
    net = netgen.config2(t_end=100.0)
    out = []
    for x in ("kernel", "resident"):
        _say(f"mixed config2 exchange={x}")
        s = Simulation(net, mode="batched", precision="mixed", exchange=x, cells_per_block=2,
                       block_threads=128, solver_waves=1)
        s.advance_steps(280)
        out.append((s.spikes(), s.read("V"), s.read("g"), s.read("c")))
    for a, b in zip(out[0][0], out[1][0]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(out[0][1:], out[1][1:]):
        np.testing.assert_array_equal(a, b)


def _passive_chains(lengths):
    """Unbranched passive cells of the given CV counts (2 um CVs, 1 um
    diameter, a 20 um first CV), each driven by current clamps on its first
    and last CV, no synapses: the mixed form then computes every current in
    FP64 and differs from the FP64 oracle only by how it solves the cable
    systems."""
    b = netgen._Builder()
    for c, n in enumerate(lengths):
        b.add_cell([-1] + list(range(n - 1)), [20.0] + [2.0] * (n - 1), [20.0] + [1.0] * (n - 1),
                   [netgen.MECH_PAS] * n)
        b.add_clamp(c, 0, 0.4 + 0.2 * (c % 3), 4.0, 0.05 + 0.02 * c)
        b.add_clamp(c, n - 1, 1.0, 3.0, -0.01 * (1 + c % 4))
    return b.finish("passive-chains", 0.2, 20.0, 17, netgen.STC_TABLE5)


@pytest.mark.parametrize("shape", [
    dict(cells_per_block=1, block_threads=64),
    dict(cells_per_block=2, block_threads=128, solver_waves=1),
    dict(cells_per_block=3, block_threads=256, solver_waves=2),
    dict(cells_per_block=4, block_threads=256, solver_waves=3),
    dict(cells_per_block=8, block_threads=128, solver_waves=1),
    dict(cells_per_block=12, block_threads=256, solver_waves=2),
    dict(cells_per_block=12, block_threads=64),
])
def test_mixed_chain_solve_matches_oracle(shape):
    """The mixed form's lane solves of unbranched cells (cyclic reduction up
    to 64 CVs a wavefront, the partition method with 2, 3 or 4 CVs a lane
    above, cells sharing a lane's chunk, ragged last chunks; workgroups over
    256 CVs by the same method with a lane's chunk of up to 14 CVs in LDS)
    against the FP64 oracle on passive chains: the voltages agree to the
    FP64 bar."""
    lengths = [101, 130, 1, 2, 65, 64, 37, 255, 3, 90, 129, 5]
    net = _passive_chains(lengths)
    _say(f"mixed passive chains {shape}")
    o = oracle.Oracle(net)
    s = Simulation(net, mode="batched", precision="mixed", exchange="kernel", **shape)
    for _ in range(4):
        o.run(10)
        s.advance_steps(10)
        vo, vs = o.read("V"), s.read("V")
        assert np.all(np.abs(vs - vo) <= 1e-9 * np.maximum(np.abs(vo), 1.0)), np.abs(vs - vo).max()
    assert np.abs(o.read("V") - o.read("V")[0]).max() > 0.1  # the clamps moved V


def test_mixed_written_conductances_reach_the_currents():
    """Mixed form with one decay factor per CV carries the per-CV
    conductance sums as state; conductances written from the host must
    reach them, so the next steps agree with the oracle given the same
    conductances (to the mixed form's rounding)."""
    net = netgen._ei_network("small-ei", 20, 3, 100.0, n_e=16, n_i=4, p=0.3, w_ext=0.004, ext_rate=40.0)
    rng = np.random.default_rng(5)
    for x in ("kernel", "resident"):
        _say(f"mixed small-ei conductance write exchange={x}")
        o = oracle.Oracle(net)
        s = Simulation(net, mode="batched", precision="mixed", exchange=x, cells_per_block=2,
                       block_threads=128, solver_waves=1)
        ref = oracle.Oracle(net)
        for x_ in (o, s, ref):
            x_.advance_steps(30) if x_ is s else x_.run(30)
        g = rng.uniform(0.0, 0.01, o.n_syn)
        o.write("g", g)
        s.write("g", g)
        for _ in range(3):
            o.run(1)
            ref.run(1)
            s.advance_steps(1)
            vo, vs = o.read("V"), s.read("V")
            assert np.abs(vs - vo).max() < 1e-3, np.abs(vs - vo).max()
        # the written conductances moved V
        assert np.abs(o.read("V") - ref.read("V")).max() > 0.1


def test_resident_exchange_matches_oracle_on_ei_network():
    net = netgen.config2(t_end=200.0)
    _say("config2 resident exchange 300 steps")
    o, s = run_pair(net, 300, chunks=2, mode="batched", exchange="resident")
    assert assert_raster_equal(o, s) > 100
    assert_routing_equal(o, s)
    assert_state_close(o, s)


# ------------------------------------------------------------------ edges
def test_edge_cases_empty_and_degenerate():
    """Cells without synapses, a network without connections or trains, a
    single one-CV cell, zero-step advances."""
    b = netgen._Builder()
    b.add_cell([-1], [20.0], [20.0], [netgen.MECH_HH])
    b.add_cell([-1, 0, 1, 1], [20.0, 10.0, 10.0, 10.0], [20.0, 1.0, 1.0, 2.0], [1, 0, 0, 0])
    b.add_clamp(1, 0, 2.0, 5.0, 0.3)
    net = b.finish("edges", 0.1, 50.0, 1, netgen.STC_TABLE5)
    _say("edges")
    for mode in ("plain", "batched"):
        o, s = run_pair(net, 400, chunks=4, mode=mode)
        s.advance_steps(0)
        assert_raster_equal(o, s)
        assert_v_close(o.read("V"), s.read("V"))


def test_advance_time_grid_and_errors():
    net = netgen.tiny(seed=2, n_cells=5, t_end=20.0)
    s = Simulation(net)
    s.advance(10.0)
    assert s.stats()["steps"] == 50
    with pytest.raises(PAError) as e:
        s.advance(10.05)        # off the 0.2 ms grid
    assert e.value.status == B.PA_ERANGE
    with pytest.raises(PAError) as e:
        s.advance(4.0)          # backwards
    assert e.value.status == B.PA_ERANGE
    s.advance(10.0)             # same time: no-op
    s.advance(20.0)
    assert s.stats()["steps"] == 100


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_synchronous_burst_matches_oracle(mode):
    """All 160 cells of an all-to-all network fire in the same step (one
    suprathreshold clamp pulse on every soma), so each cell receives 159
    conductance and 159 calcium events in one step, and again t_c,delay
    later: far beyond a fixed per-step slot; the per-epoch queues hold them
    and the deliveries match the oracle."""
    net = netgen.burst_network(n_cells=160, t_end=60.0)
    _say(f"synchronous burst mode={mode}")
    o, s = run_pair(net, 300, chunks=2, mode=mode)
    assert assert_raster_equal(o, s) >= 160
    assert_routing_equal(o, s)
    assert_state_close(o, s)
    cnt, _ = s.event_stats()
    assert cnt.sum() >= 160 * 159 * 2


def test_non_finite_voltage_is_reported():
    net = netgen.tiny(seed=6, n_cells=4, t_end=10.0)
    s = Simulation(net)
    v = s.read("V")
    v[3] = np.nan
    s.write("V", v)
    _say("nonfinite")
    with pytest.raises(PAError) as e:
        s.advance_steps(5)
    assert e.value.status == B.PA_ENUMERIC


def test_mixed_precision_stays_close_over_short_horizon():
    """Mixed form (FP32 gates, conductances, calcium): a report, not parity.
    Until the first spike the voltage error is FP32 rounding (< 0.01 mV);
    over 40 ms the spike count stays within 25 % of the FP64 oracle's."""
    net = netgen.tiny(seed=3, n_cells=13, t_end=60.0)
    _say("mixed tiny seed=3")
    for mode in ("plain", "batched"):
        o = oracle.Oracle(net)
        s = Simulation(net, precision="mixed", mode=mode)
        checked = 0
        while o.step < 200:
            o.run(1)
            s.advance_steps(1)
            if o.spikes()[0].size:
                break
            assert np.abs(s.read("V") - o.read("V")).max() < 1e-2
            checked += 1
        assert checked >= 5
        o.run(200 - o.step)
        s.advance_steps(200 - s.stats()["steps"])
        no, ns = o.spikes()[0].size, s.spikes()[0].size
        assert abs(ns - no) <= 0.25 * no + 2, (no, ns)
        assert np.all(np.isfinite(s.read("V")))


# ------------------------------------------------- full-size plastic dynamics
def _seed_plastic_state(net, sims, seed=9):
    """The same non-trivial plastic state on every side: h over [h0 - 2.5,
    h0 + 2.5] (tags of both signs), z over [-0.4, 0.9], p over [0, 8] and c
    over [0, 5] (both calcium thresholds crossed) on every plastic synapse."""
    rng = np.random.default_rng(seed)
    kinds = net["syn_kind"] == 1
    n, nc = len(kinds), int(net["n_cells"])
    h0 = net["stc"]["h0"]
    h = np.where(kinds, rng.uniform(h0 - 2.5, h0 + 2.5, n), h0)
    z = np.where(kinds, rng.uniform(-0.4, 0.9, n), 0.0)
    c = np.where(kinds, rng.uniform(0.0, 5.0, n), 0.0)
    p = rng.uniform(0.0, 8.0, nc)
    for x in sims:
        x.write("h", h)
        x.write("z", z)
        x.write("c", c)
        x.write("p", p)
    return h, z


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_ei_network_learning_stimulus_full_size(mode):
    """The 2000-cell E/I network with a learning stimulus on an assembly of
    150 excitatory cells (a somatic current step from 2 ms) and a seeded
    plastic state (tags of both signs, protein, calcium over both
    thresholds), 120 ms at full size: the conductance-port weight of Eq. 16
    with h != h0 and z != 0, the early phase (Eqs. 17-18) on both threshold
    branches with its noise, the late phase (Eq. 20) and the protein (Eq.
    21) all move, and match the oracle."""
    net = netgen.config2(t_end=200.0, stim_n=150, stim_t0=2.0, stim_dur=150.0, stim_amp=0.4)
    _say(f"config2 learning stimulus 600 steps mode={mode}")
    o = oracle.Oracle(net)
    s = Simulation(net, mode=mode)
    h_init, z_init = _seed_plastic_state(net, (o, s))
    for _ in range(3):
        o.run(200)
        s.advance_steps(200)
    assert assert_raster_equal(o, s) > 1000
    assert_routing_equal(o, s)
    assert_state_close(o, s)
    kinds = net["syn_kind"] == 1
    ho, zo, po = o.read("h"), o.read("z"), o.read("p")
    assert np.abs(ho - h_init)[kinds].max() > 0.05      # h moved
    assert np.abs(zo - z_init)[kinds].max() > 1e-6      # z moved
    assert po.max() > 0.0


@pytest.fixture(scope="module")
def large_network_oracle():
    """Config-5 network (1e5 trees of 10-60 CVs, 1e7 plastic synapses, device
    Poisson drive), oracle over 60 steps; computed once for both forms."""
    net = netgen.config5(t_end=20.0)
    _say("config5 oracle 60 steps")
    o = oracle.Oracle(net)
    o.run(60)
    return net, o


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_large_network_full_size_short_horizon(mode, large_network_oracle):
    """1e5 random trees, in-degree 100 through both ports, delays 1-5 ms
    (epochs of 4 steps), device-drawn Poisson input: 12 ms at full size,
    through the start-up burst in which every cell fires."""
    net, o = large_network_oracle
    _say(f"config5 full size 60 steps mode={mode}")
    s = Simulation(net, mode=mode)
    s.advance_steps(25)
    s.advance_steps(35)
    assert assert_raster_equal(o, s) > 1000
    assert_routing_equal(o, s)
    assert_state_close(o, s)


def _fixture(name):
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"oracle_{name}.npz")
    if not os.path.exists(p):
        pytest.skip(f"{p} not written (tests/golden/make_fixtures.py)")
    return np.load(p)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_ei_network_full_horizon_raster(mode):
    """The 2000-cell E/I network over its full 10 s (50,000 steps) against
    the oracle's raster stored by tests/golden/make_fixtures.py: equal
    spikes (count, cells, steps), t* within 1e-9, V and p at the end to the
    FP64 bar, h of every 97th synapse."""
    fx = _fixture("ei2000x21_10s")
    net = netgen.config2(t_end=10000.0)
    _say(f"config2 10 s mode={mode}")
    s = Simulation(net, mode=mode)
    for _ in range(5):
        s.advance_steps(10000)
    g, st, t = s.spikes()
    assert g.size == fx["gid"].size, (g.size, fx["gid"].size)
    np.testing.assert_array_equal(g, fx["gid"].astype(np.int64))
    np.testing.assert_array_equal(st, fx["step"].astype(np.int64))
    np.testing.assert_allclose(t, fx["t"], rtol=1e-9, atol=0)
    assert_v_close(fx["V"], s.read("V")[::int(fx["v_stride"])])
    np.testing.assert_allclose(s.read("p"), fx["p"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(s.read("h")[::int(fx["h_stride"])], fx["h"], rtol=1e-9, atol=1e-10)
