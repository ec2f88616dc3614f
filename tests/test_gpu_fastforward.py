"""GPU parity of fast-forward (the long steps of slow network dynamics of
the 8-h paradigm, Sec. 3.5) against the oracle, and the device state dump:
a run resumed from a dump repeats the original run bit for bit."""
import numpy as np
import pytest

import netgen
import oracle
from _parity import assert_raster_equal, assert_routing_equal, assert_state_close
from paper_2411_16445_amd import PAError, Simulation
from paper_2411_16445_amd import binding as B

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _seed(net, sims, seed=9):
    rng = np.random.default_rng(seed)
    kinds = net["syn_kind"] == 1
    n = len(kinds)
    h0 = net["stc"]["h0"]
    h = np.where(kinds, rng.uniform(h0 - 2.5, h0 + 2.5, n), h0)
    z = np.where(kinds, rng.uniform(-0.4, 0.9, n), 0.0)
    c = np.where(kinds, rng.uniform(0.0, 5.0, n), 0.0)
    p = rng.uniform(0.0, 8.0, int(net["n_cells"]))
    for x in sims:
        x.write("h", h)
        x.write("z", z)
        x.write("c", c)
        x.write("p", p)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_fast_forward_matches_oracle_on_tiny_network(mode):
    """Ordinary steps, a jump of 50 long steps of 100 ms (trains and
    Poisson arrivals inside it dropped), ordinary steps again."""
    net = netgen.tiny(seed=14, n_cells=11, t_end=6000.0, poisson=True, ext_rate=300.0)
    _say(f"fast-forward tiny mode={mode}")
    o = oracle.Oracle(net)
    s = Simulation(net, mode=mode)
    _seed(net, (o, s))
    o.run(300)
    s.advance_steps(300)
    o.fast_forward(50, 100.0)
    s.fast_forward(50, 100.0)
    assert s.stats()["steps"] == o.step == 300 + 50 * 500
    assert_state_close(o, s)
    o.run(400)
    s.advance_steps(400)
    assert assert_raster_equal(o, s) > 10
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_consolidation_protocol_shape_full_size(mode):
    """The 2000-cell E/I network: a learning stimulus on 150 cells (100
    ms), one hour fast-forwarded in long steps of 10 s, then a recall
    stimulus on half of them; rasters and the consolidated state (h, z, p)
    against the oracle."""
    net = netgen.config2(t_end=3601000.0, max_train_t=800.0, stim_n=150, stim_t0=2.0,
                         stim_dur=100.0, stim_amp=0.4)
    _say(f"consolidation protocol mode={mode}")
    o = oracle.Oracle(net)
    s = Simulation(net, mode=mode)
    _seed(net, (o, s), seed=2)
    o.run(600)
    s.advance_steps(600)
    o.fast_forward(360, 10000.0)
    s.fast_forward(360, 10000.0)
    assert_state_close(o, s)
    kinds = net["syn_kind"] == 1
    assert np.abs(o.read("z"))[kinds].max() > 0.05   # the late phase moved
    o.run(300)
    s.advance_steps(300)
    assert_raster_equal(o, s)
    assert_routing_equal(o, s)
    assert_state_close(o, s)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_state_dump_resumes_bit_for_bit(mode):
    """A dump taken into a device tensor after 200 steps, loaded into a new
    simulation of the same network, continues exactly as the original."""
    import torch
    net = netgen.tiny(seed=21, n_cells=17, t_end=300.0)
    _say(f"state dump mode={mode}")
    a = Simulation(net, mode=mode)
    _seed(net, (a,))
    a.advance_steps(200)
    buf = torch.zeros(a.state_size(), dtype=torch.uint8, device="cuda")
    a.save_state(buf)
    n0 = a.spikes()[0].size
    a.advance_steps(500)
    want = [x[n0:] for x in a.spikes()] + [a.read(k) for k in ("V", "g", "c", "h", "z", "p")]
    b = Simulation(net, mode=mode)
    b.load_state(buf)
    assert b.stats()["steps"] == 200
    b.advance_steps(500)
    got = list(b.spikes()) + [b.read(k) for k in ("V", "g", "c", "h", "z", "p")]
    assert want[0].size > 5
    for x, y in zip(want, got):
        np.testing.assert_array_equal(x, y)
    # rewinding the original to the dump repeats it too
    a.load_state(buf)
    a.advance_steps(500)
    np.testing.assert_array_equal(a.read("V"), want[3])
    # a host copy works the same, a dump of another network is refused
    host = buf.cpu().numpy()
    c = Simulation(net, mode=mode)
    c.load_state(host)
    other = Simulation(netgen.tiny(seed=22, n_cells=17, t_end=300.0), mode=mode)
    with pytest.raises(PAError) as e:
        other.load_state(host)
    assert e.value.status == B.PA_EINVAL
