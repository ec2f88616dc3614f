"""Seeded synthetic networks shaped like the paper's workloads.

This module only *generates inputs*: morphologies (parent arrays, lengths,
diameters), synapse placement, connectivity, delays, weights and explicit
presynaptic spike trains.  It holds none of the method's arithmetic (no cable
invariants, no mechanism equations, no event timing); both the CPU oracle and
the HIP library consume the dictionaries it returns.

Network dictionary (all arrays are numpy, C-contiguous):

  cells      n_cells, cv_off[int64 n+1], parent[int32, local index, -1 = root],
             length[f64 um], diam[f64 um], mech[u8: 0 passive, 1 HH],
             detector[int32 local CV], cell_params[f64 n x 11]
             (cm uF/cm2, Ra ohm cm, v_init mV, g_pas S/cm2, e_pas mV,
              gNa, gK, gL S/cm2, ENa, EK, EL mV)
  synapses   syn_cell[int32], syn_cv[int32 local], syn_kind[u8: 0 exp-syn,
             1 STC], syn_tau[f64 ms], syn_erev[f64 mV]
  conns      conn_src[int32 gid], conn_dst[int32 synapse id],
             conn_ports[u8: bit0 conductance, bit1 calcium], conn_w[f64 uS],
             conn_d[f64 ms]
  trains     train_dst, train_ports, train_w, train_off[int64 n+1],
             train_times[f64 ms, sorted within each train]
  clamps     clamp_cell, clamp_cv, clamp_t0, clamp_dur, clamp_amp[nA]
  poisson    pois_dst, pois_ports, pois_w, pois_rate[Hz]: sources whose
             arrivals are drawn by the simulator from the network's seed
  scalars    dt, theta (detector threshold mV), seed, t_end, name, stc{...}
  diffusion  optional {d_sps, d_prp} (um^2/ms): the signal triggering
             protein synthesis and the protein diffuse over each cell's CVs
             instead of the per-cell sum of the plasticity rule

Units: ms, mV, um, nA, uS, nF.  The seed recipe (one master seed, split into
independent substreams for morphology, placement, connectivity, delays and
spike trains) is what makes every workload reproducible on any machine.
"""
from __future__ import annotations

import numpy as np

PORT_G = 1
PORT_CA = 2
KIND_EXPSYN = 0
KIND_STC = 1
MECH_PAS = 0
MECH_HH = 1

# Parameters of the calcium / tagging-and-capture synapse (Table 5 of the
# paper, units ms, mV, umol/l).  h0, theta_pro and theta_tag are the decimal
# values of h0 = 10 mV * 0.5 * gamma_p / (gamma_p + gamma_d), 0.5 h0, 0.2 h0.
STC_TABLE5 = dict(
    tau_c=48.8, tau_h=688400.0, tau_p=3.6e6, tau_z=3.6e6,
    gamma_p=1645.6, gamma_d=313.1, theta_p=3.0, theta_d=1.2,
    sigma_pl=2.90436, p_max=10.0, f_int=0.1, t_cd=18.8,
    h0=4.2007453923521, theta_pro=2.10037269617605, theta_tag=0.840149078470420,
    c_pre=1.0, c_post=0.2758,
)
# in-vivo adjusted calcium amplitudes used for networks (Table 5, parentheses)
CA_INVIVO = dict(c_pre=0.6, c_post=0.1655)

DEFAULT_CELL = np.array([1.0, 35.4, -65.0, 1e-4, -65.0,
                         0.12, 0.036, 0.0003, 50.0, -77.0, -54.3])
N_CELL_PARAMS = 11


def _streams(master: int, n: int):
    ss = np.random.SeedSequence(master)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


class _Builder:
    """Accumulates cells / synapses / connections into flat arrays."""

    def __init__(self):
        self.cv_off = [0]
        self.parent, self.length, self.diam, self.mech = [], [], [], []
        self.detector, self.cell_params = [], []
        self.syn = []      # (cell, cv, kind, tau, erev) added one by one
        self._bulk = []    # bulk synapse arrays
        self._nbulk = 0
        self._chunks = []  # flushed synapse arrays, in id order
        self._nsyn_flushed = 0
        self.conn = []     # arrays appended in chunks
        self.trains = []   # (dst, ports, w, times)
        self.clamps = []
        self.pois = []     # (dst, ports, w, rate)

    @property
    def n_cells(self):
        return len(self.cv_off) - 1

    def add_cell(self, parent, length, diam, mech, detector=0, params=None):
        n = len(parent)
        self.parent.append(np.asarray(parent, np.int32))
        self.length.append(np.asarray(length, np.float64))
        self.diam.append(np.asarray(diam, np.float64))
        self.mech.append(np.asarray(mech, np.uint8))
        self.detector.append(detector)
        self.cell_params.append(DEFAULT_CELL if params is None else np.asarray(params, np.float64))
        self.cv_off.append(self.cv_off[-1] + n)
        return self.n_cells - 1

    def add_syn(self, cell, cv, kind, tau=5.0, erev=0.0):
        if self._bulk:
            self._flush_bulk()
        self.syn.append((cell, cv, kind, tau, erev))
        return self.n_syn - 1

    def add_syns(self, cells, cvs, kind, tau=5.0, erev=0.0):
        """Bulk form of add_syn; returns the new synapse ids."""
        if self.syn:
            self._flush_bulk()
        cells = np.asarray(cells, np.int32)
        n = len(cells)
        first = self.n_syn
        self._bulk.append((cells, np.asarray(cvs, np.int32),
                           np.broadcast_to(np.asarray(kind, np.uint8), (n,)).copy(),
                           np.broadcast_to(np.asarray(tau, np.float64), (n,)).copy(),
                           np.broadcast_to(np.asarray(erev, np.float64), (n,)).copy()))
        self._nbulk += n
        return np.arange(first, first + n, dtype=np.int64)

    @property
    def n_syn(self):
        return self._nsyn_flushed + len(self.syn) + self._nbulk

    def _flush_bulk(self):
        # keep synapse ids in call order: tuples added so far become a chunk
        if self.syn:
            s = self.syn
            self._chunks.append((np.array([x[0] for x in s], np.int32), np.array([x[1] for x in s], np.int32),
                                 np.array([x[2] for x in s], np.uint8), np.array([x[3] for x in s], np.float64),
                                 np.array([x[4] for x in s], np.float64)))
            self._nsyn_flushed += len(s)
            self.syn = []
        if self._bulk:
            self._chunks.extend(self._bulk)
            self._nsyn_flushed += self._nbulk
            self._bulk = []
            self._nbulk = 0

    def add_conns(self, src, dst, ports, w, d):
        src = np.asarray(src, np.int32)
        n = len(src)
        self.conn.append((src, np.asarray(dst, np.int32),
                          np.broadcast_to(np.asarray(ports, np.uint8), (n,)).copy(),
                          np.broadcast_to(np.asarray(w, np.float64), (n,)).copy(),
                          np.broadcast_to(np.asarray(d, np.float64), (n,)).copy()))

    def add_train(self, dst, ports, w, times):
        self.trains.append((dst, ports, w, np.sort(np.asarray(times, np.float64))))

    def add_clamp(self, cell, cv, t0, dur, amp):
        self.clamps.append((cell, cv, t0, dur, amp))

    def add_poisson(self, dst, ports, w, rate_hz):
        dst = np.atleast_1d(np.asarray(dst, np.int64))
        for x in dst:
            self.pois.append((int(x), ports, w, rate_hz))

    def finish(self, name, dt, t_end, seed, stc, theta=-10.0):
        net = dict(name=name, dt=float(dt), t_end=float(t_end), seed=int(seed),
                   theta=float(theta), stc=dict(stc))
        net["n_cells"] = self.n_cells
        net["cv_off"] = np.asarray(self.cv_off, np.int64)
        cat = lambda xs, dt_: (np.concatenate(xs).astype(dt_) if xs else np.zeros(0, dt_))
        net["parent"] = cat(self.parent, np.int32)
        net["length"] = cat(self.length, np.float64)
        net["diam"] = cat(self.diam, np.float64)
        net["mech"] = cat(self.mech, np.uint8)
        net["detector"] = np.asarray(self.detector, np.int32)
        net["cell_params"] = np.ascontiguousarray(np.stack(self.cell_params).astype(np.float64)) \
            if self.cell_params else np.zeros((0, N_CELL_PARAMS))
        self._flush_bulk()
        ch = self._chunks
        for k, (name, t) in enumerate((("syn_cell", np.int32), ("syn_cv", np.int32), ("syn_kind", np.uint8),
                                        ("syn_tau", np.float64), ("syn_erev", np.float64))):
            net[name] = np.concatenate([c[k] for c in ch]).astype(t) if ch else np.zeros(0, t)
        if self.conn:
            c = list(zip(*self.conn))
            net["conn_src"] = np.concatenate(c[0]).astype(np.int32)
            net["conn_dst"] = np.concatenate(c[1]).astype(np.int32)
            net["conn_ports"] = np.concatenate(c[2]).astype(np.uint8)
            net["conn_w"] = np.concatenate(c[3]).astype(np.float64)
            net["conn_d"] = np.concatenate(c[4]).astype(np.float64)
        else:
            for k, t in (("conn_src", np.int32), ("conn_dst", np.int32), ("conn_ports", np.uint8),
                         ("conn_w", np.float64), ("conn_d", np.float64)):
                net[k] = np.zeros(0, t)
        tr = self.trains
        net["train_dst"] = np.array([x[0] for x in tr], np.int32)
        net["train_ports"] = np.array([x[1] for x in tr], np.uint8)
        net["train_w"] = np.array([x[2] for x in tr], np.float64)
        net["train_off"] = np.concatenate([[0], np.cumsum([len(x[3]) for x in tr])]).astype(np.int64)
        net["train_times"] = cat([x[3] for x in tr], np.float64)
        cl = self.clamps
        net["clamp_cell"] = np.array([x[0] for x in cl], np.int32)
        net["clamp_cv"] = np.array([x[1] for x in cl], np.int32)
        net["clamp_t0"] = np.array([x[2] for x in cl], np.float64)
        net["clamp_dur"] = np.array([x[3] for x in cl], np.float64)
        net["clamp_amp"] = np.array([x[4] for x in cl], np.float64)
        po = self.pois
        net["pois_dst"] = np.array([x[0] for x in po], np.int32)
        net["pois_ports"] = np.array([x[1] for x in po], np.uint8)
        net["pois_w"] = np.array([x[2] for x in po], np.float64)
        net["pois_rate"] = np.array([x[3] for x in po], np.float64)
        return net


# ---------------------------------------------------------------- morphologies

def ball_and_stick(n_dend, dend_len=200.0, dend_diam=1.0, soma_diam=20.0):
    """Soma (1 HH CV, cylinder with l = d) + unbranched passive dendrite."""
    parent = np.arange(-1, n_dend, dtype=np.int32)
    length = np.concatenate([[soma_diam], np.full(n_dend, dend_len / n_dend)])
    diam = np.concatenate([[soma_diam], np.full(n_dend, dend_diam)])
    mech = np.concatenate([[MECH_HH], np.full(n_dend, MECH_PAS)]).astype(np.uint8)
    return parent, length, diam, mech


def random_tree(rng, n_min, n_max, soma_diam=20.0, l_rng=(20.0, 150.0),
                d_rng=(0.5, 3.0), cv_len=10.0):
    """Random binary-branching dendrite on an HH soma.

    Draw a target CV count uniformly in [n_min, n_max]; grow from one root
    branch on the soma by splitting a uniformly chosen leaf into two children;
    each branch has a uniform length and diameter and ceil(L / cv_len) CVs; the
    last branch is truncated so the dendrite has exactly the target count.
    CVs are numbered depth-first (pre-order), branch-contiguous, parent < child.
    Returns (parent, length, diam, mech) including the soma as CV 0.
    """
    target = int(rng.integers(n_min, n_max + 1))
    branches = []  # dict(parent_branch, L, d, ncv)
    total = 0

    def new_branch(pb):
        nonlocal total
        L = float(rng.uniform(*l_rng))
        d = float(rng.uniform(*d_rng))
        n = int(np.ceil(L / cv_len))
        if total + n > target:
            n = target - total
        if n <= 0:
            return None
        L = L if n == int(np.ceil(L / cv_len)) else n * cv_len
        branches.append(dict(pb=pb, L=L, d=d, n=n, kids=[]))
        total += n
        return len(branches) - 1

    new_branch(-1)
    leaves = [0]
    while total < target:
        li = int(rng.integers(len(leaves)))
        b = leaves.pop(li)
        for _ in range(2):
            if total >= target:
                break
            k = new_branch(b)
            if k is not None:
                branches[b]["kids"].append(k)
                leaves.append(k)
    parent = [-1]
    length = [soma_diam]
    diam = [soma_diam]

    def emit(bi, pcv):
        br = branches[bi]
        for j in range(br["n"]):
            parent.append(pcv)
            length.append(br["L"] / br["n"])
            diam.append(br["d"])
            pcv = len(parent) - 1
        for k in br["kids"]:
            emit(k, pcv)

    emit(0, 0)
    mech = np.zeros(len(parent), np.uint8)
    mech[0] = MECH_HH
    return (np.asarray(parent, np.int32), np.asarray(length), np.asarray(diam), mech)


def poisson_times(rng, rate_hz, t_end_ms):
    """Homogeneous Poisson arrival times in [0, t_end)."""
    if rate_hz <= 0:
        return np.zeros(0)
    mean_isi = 1000.0 / rate_hz
    n_guess = int(t_end_ms / mean_isi * 1.3 + 20)
    t = np.cumsum(rng.exponential(mean_isi, n_guess))
    while t[-1] < t_end_ms:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(mean_isi, n_guess))])
    return t[t < t_end_ms]


def _merge_trains(rng, n_sources, rate_hz, t_end_ms):
    """Arrivals of n independent Poisson sources onto one synapse: their
    union is a Poisson process of the summed rate, drawn as such."""
    return poisson_times(rng, n_sources * rate_hz, t_end_ms)


# ---------------------------------------------------------------- workloads

def config1(seed=1, t_end=10000.0, w_syn=0.05, rate_hz=20.0, sigma_on=True):
    """1 cell (HH soma + 8-CV passive dendrite, 200 um), one plastic synapse
    (tau 5 ms) on dendrite CV 4 driven by a 20 Hz Poisson train on both its
    conductance and calcium ports."""
    rng_m, rng_t = _streams(seed, 2)
    b = _Builder()
    b.add_cell(*ball_and_stick(8, 200.0, 1.0, 20.0))
    s = b.add_syn(0, 4, KIND_STC, 5.0, 0.0)
    b.add_train(s, PORT_G | PORT_CA, w_syn, poisson_times(rng_t, rate_hz, t_end))
    stc = dict(STC_TABLE5)
    if not sigma_on:
        stc["sigma_pl"] = 0.0
    return b.finish("single-synapse", 0.2, t_end, seed, stc)


def _ei_network(name, n_dend, seed, t_end, n_e=1600, n_i=400, p=0.1, delay=3.0,
                w_ee=0.0003, w_ei=0.0005, w_ie=0.02, w_ii=0.01, w_ext=0.0005,
                n_ext=25, ext_rate=5.0, explicit_trains=True, max_train_t=None,
                stim_n=0, stim_rate=0.0, stim_t0=0.0, stim_dur=0.0, stim_amp=0.0):
    """E/I network of ball-and-stick cells.  A learning stimulus (the shape
    of the assembly-forming protocol of Sec. 3.5): the first stim_n
    excitatory cells receive, on their external synapse, an extra Poisson
    train of stim_rate Hz during [stim_t0, stim_t0 + stim_dur), and a
    somatic current step of stim_amp nA over the same interval."""
    rng_m, rng_c, rng_p, rng_t, rng_s = _streams(seed, 5)
    n = n_e + n_i
    b = _Builder()
    morph = ball_and_stick(n_dend, 200.0, 1.0, 20.0)
    for _ in range(n):
        b.add_cell(*morph)
    # external input: one excitatory exp-syn on the distal CV of every cell
    ext_syn = [b.add_syn(c, n_dend, KIND_EXPSYN, 5.0, 0.0) for c in range(n)]
    # Bernoulli(p) connectivity per ordered pair, no autapses
    conn_src, conn_dst, conn_ports, conn_w = [], [], [], []
    for tgt in range(n):
        src = np.nonzero(rng_c.random(n) < p)[0]
        src = src[src != tgt]
        exc = src[src < n_e]
        inh = src[src >= n_e]
        for s_ in exc:
            cv = int(rng_p.integers(1, n_dend + 1))
            if tgt < n_e:
                sid = b.add_syn(tgt, cv, KIND_STC, 5.0, 0.0)
                conn_src.append(s_); conn_dst.append(sid)
                conn_ports.append(PORT_G | PORT_CA); conn_w.append(w_ee)
            else:
                sid = b.add_syn(tgt, cv, KIND_EXPSYN, 5.0, 0.0)
                conn_src.append(s_); conn_dst.append(sid)
                conn_ports.append(PORT_G); conn_w.append(w_ei)
        for s_ in inh:
            sid = b.add_syn(tgt, 0, KIND_EXPSYN, 5.0, -80.0)
            conn_src.append(s_); conn_dst.append(sid)
            conn_ports.append(PORT_G); conn_w.append(w_ie if tgt < n_e else w_ii)
    b.add_conns(conn_src, conn_dst, conn_ports, conn_w, delay)
    if explicit_trains:
        t_tr = t_end if max_train_t is None else min(t_end, max_train_t)
        for c in range(n):
            times = _merge_trains(rng_t, n_ext, ext_rate, t_tr)
            if c < stim_n:
                extra = stim_t0 + poisson_times(rng_s, stim_rate, min(stim_dur, t_tr - stim_t0))
                times = np.concatenate([times, extra])
            b.add_train(ext_syn[c], PORT_G, w_ext, times)
    if stim_amp:
        for c in range(stim_n):
            b.add_clamp(c, 0, stim_t0, stim_dur, stim_amp)
    stc = dict(STC_TABLE5)
    stc.update(CA_INVIVO)
    net = b.finish(name, 0.2, t_end, seed, stc)
    net["ext_rate_hz"] = n_ext * ext_rate
    return net


def with_diffusion(net, d_sps=1e-2, d_prp=1e-2):
    """The same network with SPS / PRP particle diffusion over every cell
    (diffusivities in um^2/ms; 1e-11 m^2/s = 1e-2 um^2/ms)."""
    out = dict(net)
    out["diffusion"] = dict(d_sps=float(d_sps), d_prp=float(d_prp))
    out["name"] = net["name"] + "-diffusion"
    return out


# Morphologies of the multi-compartment network (Table 6): compartments of
# 1 um, one radius for soma and dendrites, the soma two cylinders with a
# one-compartment middle (protein synthesis, detector), an apical dendrite
# on one end and a basal dendrite on the other.
TABLE6 = dict(small_cell=dict(r=6.0, l_soma=12.0), large_cell=dict(r=12.0, l_soma=24.0),
              small_dendrites=dict(l_apical=12.5, l_basal=5.0),
              large_dendrites=dict(l_apical=25.0, l_basal=10.0))


def stc_neuron(cell="small", dendrites="small", dl=1.0):
    """(parent, length, diam, mech, apical tip, basal tip) of one neuron:
    CV 0 the middle soma compartment, then one soma half and the apical
    dendrite, then the other half and the basal dendrite (depth-first,
    parent < child); HH on the soma, passive dendrites.  Small cells with
    small dendrites have 31 CVs, with large dendrites 48."""
    c = TABLE6[f"{cell}_cell"]
    d = TABLE6[f"{dendrites}_dendrites"]
    half = int(round((c["l_soma"] / 2) / dl))
    parent, length, mech = [-1], [dl], [MECH_HH]

    def chain(start, n, L, m):
        p = start
        for _ in range(n):
            parent.append(p)
            length.append(L / n)
            mech.append(m)
            p = len(parent) - 1
        return p

    end_a = chain(0, half, half * dl, MECH_HH)
    apical = chain(end_a, int(np.ceil(d["l_apical"] / dl)), d["l_apical"], MECH_PAS)
    end_b = chain(0, half, half * dl, MECH_HH)
    basal = chain(end_b, int(np.ceil(d["l_basal"] / dl)), d["l_basal"], MECH_PAS)
    n = len(parent)
    return (np.asarray(parent, np.int32), np.asarray(length), np.full(n, 2.0 * c["r"]),
            np.asarray(mech, np.uint8), apical, basal)


def stc_morpho_network(seed=6, t_end=10000.0, cell="small", dendrites="small", d_sps=1e-2, d_prp=1e-2,
                       n_e=1600, n_i=400, p=0.1, delay=3.0, w_ee=0.0004, w_ei=0.0005, w_ie=0.02,
                       w_ii=0.01, w_ext=0.0006, n_ext=25, ext_rate=5.0, stim_n=0, stim_rate=0.0,
                       stim_t0=0.0, stim_dur=0.0):
    """E/I network of the multi-compartment neurons of Table 6 (Sec. 3.6):
    external input on the apical tip, recurrent excitation on the basal tip
    (plastic E->E through both ports), inhibition on the soma; SPS / PRP
    diffusion with the given diffusivities (um^2/ms)."""
    rng_c, rng_t, rng_s = _streams(seed, 3)
    n = n_e + n_i
    parent, length, diam, mech, apical, basal = stc_neuron(cell, dendrites)
    b = _Builder()
    for _ in range(n):
        b.add_cell(parent, length, diam, mech, detector=0)
    ext_syn = [b.add_syn(c, apical, KIND_EXPSYN, 5.0, 0.0) for c in range(n)]
    conn_src, conn_dst, conn_ports, conn_w = [], [], [], []
    for tgt in range(n):
        src = np.nonzero(rng_c.random(n) < p)[0]
        src = src[src != tgt]
        for s_ in src[src < n_e]:
            plastic = tgt < n_e
            sid = b.add_syn(tgt, basal, KIND_STC if plastic else KIND_EXPSYN, 5.0, 0.0)
            conn_src.append(s_); conn_dst.append(sid)
            conn_ports.append(PORT_G | PORT_CA if plastic else PORT_G)
            conn_w.append(w_ee if plastic else w_ei)
        for s_ in src[src >= n_e]:
            sid = b.add_syn(tgt, 0, KIND_EXPSYN, 5.0, -80.0)
            conn_src.append(s_); conn_dst.append(sid)
            conn_ports.append(PORT_G); conn_w.append(w_ie if tgt < n_e else w_ii)
    b.add_conns(conn_src, conn_dst, conn_ports, conn_w, delay)
    for c in range(n):
        times = _merge_trains(rng_t, n_ext, ext_rate, t_end)
        if c < stim_n:
            extra = stim_t0 + poisson_times(rng_s, stim_rate, min(stim_dur, t_end - stim_t0))
            times = np.concatenate([times, extra])
        b.add_train(ext_syn[c], PORT_G, w_ext, times)
    stc = dict(STC_TABLE5)
    stc.update(CA_INVIVO)
    net = b.finish(f"ei-stc-morpho-{cell}-{dendrites}", 0.2, t_end, seed, stc)
    net["diffusion"] = dict(d_sps=float(d_sps), d_prp=float(d_prp))
    return net


# Graupner-Brunel calcium-based rule (Table 3): time constants in ms,
# weights without unit.
GB_TABLE3 = dict(tau_w=150000.0, w_star=0.5, gamma_p=321.808, gamma_d=200.0, theta_p=1.3, theta_d=1.0,
                 sigma=2.8248, tau_c=20.0, c_pre=1.0, c_post=2.0, t_cd=13.7)

# STDP synapse parameters (Table 1: the classical-window set; Table 7: the
# busyring set), trace amplitudes and weights in uS, time constants in ms.
STDP_TABLE1 = dict(tau_pre=20.0, tau_post=20.0, a_pre=0.01, a_post=-0.0105, w0=1.0, w_max=10.0)
STDP_TABLE7 = dict(tau_pre=10.0, tau_post=10.0, a_pre=0.01, a_post=-0.01, w0=1.0, w_max=10.0)
KIND_STDP = 2


def simple_branchy(rng, depth, soma_diam=20.0, p_split=0.75, cvs=(6, 12), cv_len=10.0, d_rng=(0.5, 1.5)):
    """HH soma and a random passive tree of at most `depth` branch levels
    below the first dendritic branch: every branch above the deepest level
    splits into two children with probability p_split; a branch has a
    uniform number of 10-um CVs in [cvs] and one diameter.  Depth-first,
    parent < child; depth 0 is the soma alone.  Mean sizes: 1, ~44 and
    ~1500 CVs for depths 0, 2 and 10."""
    parent, length, diam = [-1], [soma_diam], [soma_diam]
    if depth > 0:
        def grow(pcv, level):
            n = int(rng.integers(cvs[0], cvs[1] + 1))
            d = float(rng.uniform(*d_rng))
            for _ in range(n):
                parent.append(pcv)
                length.append(cv_len)
                diam.append(d)
                pcv = len(parent) - 1
            if level < depth and rng.random() < p_split:
                grow(pcv, level + 1)
                grow(pcv, level + 1)
        grow(0, 0)
    mech = np.zeros(len(parent), np.uint8)
    mech[0] = MECH_HH
    return np.asarray(parent, np.int32), np.asarray(length), np.asarray(diam), mech


def busyring(n_cells=1024, depth=2, stdp=False, seed=8, ring=4, fanout=1000, delay=5.0, t_end=200.0,
             w_ring=0.05, dt=0.025):
    """The busyring benchmark (Sec. 3.8, Table 7): rings of `ring` cells in
    which each cell excites the next (exp-syn on the soma, tau 2 ms, delay
    5 ms) so that one spike circulates; the first cell of every ring gets a
    single external arrival at t = 0; every cell also makes `fanout`
    connections of weight 0 to synapses of its own on uniformly random
    cells (on a random CV), which load spike transmission and delivery
    without effect -- pair-based STDP synapses in the plasticity variant."""
    rng_m, rng_c = _streams(seed, 2)
    b = _Builder()
    for _ in range(n_cells):
        parent, length, diam, mech = simple_branchy(rng_m, depth)
        b.add_cell(parent, length, diam, mech)
    ring_syn = b.add_syns(np.arange(n_cells), np.zeros(n_cells, np.int32), KIND_EXPSYN, 2.0, 0.0)
    n_ring = n_cells // ring
    src = np.arange(n_ring * ring)
    dst = (src // ring) * ring + (src % ring + 1) % ring
    b.add_conns(src, ring_syn[dst], PORT_G, w_ring, delay)
    # the random zero-weight connections: targets uniform over the cells,
    # each onto a synapse of its own at a uniformly random CV of the target
    tgt = rng_c.integers(0, n_cells, n_cells * fanout)
    ncv = np.diff(np.asarray(b.cv_off))
    cv = (rng_c.random(n_cells * fanout) * ncv[tgt]).astype(np.int32)
    order = np.argsort(tgt, kind="stable")
    sids = b.add_syns(tgt[order], cv[order], KIND_STDP if stdp else KIND_EXPSYN, 2.0, 0.0)
    syn_of = np.empty(n_cells * fanout, np.int64)
    syn_of[order] = sids
    b.add_conns(np.repeat(np.arange(n_cells), fanout), syn_of, PORT_G, 0.0, delay)
    for r in range(n_ring):
        b.add_train(int(ring_syn[r * ring]), PORT_G, 10.0 * w_ring, [0.0])
    net = b.finish(f"busyring-{n_cells}-d{depth}{'-stdp' if stdp else ''}", dt, t_end, seed, STC_TABLE5)
    if stdp:
        net["stdp"] = dict(STDP_TABLE7)
    return net


def config2(seed=2, t_end=10000.0, **kw):
    """2000 ball-and-stick cells (1 soma + 20 dendrite CVs), 1600 E / 400 I,
    p = 0.1, delay 3 ms, E->E plastic, 25 x 5 Hz external Poisson per cell."""
    return _ei_network("ei-ball-and-stick-21cv", 20, seed, t_end, **kw)


def config4(seed=2, t_end=60000.0, **kw):
    """Config-2 network with dendrites of 100 CVs (101 CVs per cell)."""
    return _ei_network("ei-ball-and-stick-101cv", 100, seed, t_end, **kw)


def _tree_network(name, seed, t_end, n_cells, n_min, n_max, sites=100, p=None,
                  indegree=None, delay=3.0, delay_exp=False, w_stc=0.002, w_ext=0.006,
                  n_ext=25, ext_rate=5.0, explicit_trains=True, max_train_t=None):
    rng_m, rng_s, rng_c, rng_d, rng_t = _streams(seed, 5)
    b = _Builder()
    for c in range(n_cells):
        parent, length, diam, mech = random_tree(rng_m, n_min, n_max)
        b.add_cell(parent, length, diam, mech)
    ncv = np.diff(np.asarray(b.cv_off))
    # sites of cell c are synapses c*sites .. c*sites+sites-1
    site_cv = (1 + np.floor(rng_s.random((n_cells, sites)) * (ncv[:, None] - 1))).astype(np.int32)
    b.add_syns(np.repeat(np.arange(n_cells), sites), site_cv.ravel(), KIND_STC, 5.0, 0.0)
    ext_syn = b.add_syns(np.arange(n_cells), ncv - 1, KIND_EXPSYN, 5.0, 0.0)
    src_all, dst_all = [], []
    for tgt in range(n_cells):
        if indegree is not None:
            src = rng_c.integers(0, n_cells - 1, indegree)
            src = src + (src >= tgt)  # uniform over the other cells
        else:
            src = np.nonzero(rng_c.random(n_cells) < p)[0]
            src = src[src != tgt]
        # incoming connection j goes to site j mod sites (round-robin)
        src_all.append(src.astype(np.int32))
        dst_all.append((tgt * sites + np.arange(len(src)) % sites).astype(np.int32))
    src_all = np.concatenate(src_all)
    dst_all = np.concatenate(dst_all)
    nc = len(src_all)
    if delay_exp:
        d = 1.0 + rng_d.exponential(1.0, nc)
        bad = d > 5.0
        while bad.any():
            d[bad] = 1.0 + rng_d.exponential(1.0, int(bad.sum()))
            bad = d > 5.0
    else:
        d = np.full(nc, delay)
    b.add_conns(src_all, dst_all, PORT_G | PORT_CA, w_stc, d)
    if explicit_trains:
        t_tr = t_end if max_train_t is None else min(t_end, max_train_t)
        for c in range(n_cells):
            b.add_train(int(ext_syn[c]), PORT_G, w_ext, _merge_trains(rng_t, n_ext, ext_rate, t_tr))
    else:
        # simulator-drawn Poisson input, one source of the summed rate per cell
        b.add_poisson(ext_syn, PORT_G, w_ext, n_ext * ext_rate)
    stc = dict(STC_TABLE5)
    stc.update(CA_INVIVO)
    net = b.finish(name, 0.2, t_end, seed, stc)
    net["ext_rate_hz"] = n_ext * ext_rate
    return net


def config3(seed=3, t_end=10000.0, **kw):
    """4096 cells with random binary trees of 10-300 dendritic CVs, 100 STC
    sites each, p = 0.02, delay 3 ms."""
    return _tree_network("uneven-trees-4096", seed, t_end, 4096, 10, 300, p=0.02, **kw)


def config5(seed=5, t_end=10000.0, n_cells=100_000, explicit_trains=False, **kw):
    """1e5 cells with random trees of 10-60 dendritic CVs, in-degree exactly
    100 (one source per STC site), delays 1 ms + Exp(1 ms) redrawn above 5 ms;
    external drive drawn by the simulator (one 125 Hz Poisson source per cell)."""
    return _tree_network("large-1e5", seed, t_end, n_cells, 10, 60, indegree=100,
                         delay_exp=True, explicit_trains=explicit_trains, **kw)


def tiny(seed=7, n_cells=13, t_end=200.0, n_min=2, n_max=24, p=0.35, n_static=3,
         clamp=True, dt=0.2, delay_range=(0.6, 4.0), w_ext=0.02, ext_rate=150.0, poisson=False):
    """Small random network exercising every feature: random trees (1-CV
    cells included), mixed synapse kinds, several synapses per CV, random
    delays, two-port connections, explicit trains and current clamps."""
    rng_m, rng_s, rng_c, rng_t = _streams(seed, 4)
    b = _Builder()
    for c in range(n_cells):
        if c % 5 == 4:
            parent, length, diam, mech = (np.array([-1], np.int32), np.array([20.0]),
                                          np.array([20.0]), np.array([MECH_HH], np.uint8))
        else:
            parent, length, diam, mech = random_tree(rng_m, n_min, n_max)
        params = DEFAULT_CELL.copy()
        params[3] *= float(rng_m.uniform(0.5, 2.0))
        b.add_cell(parent, length, diam, mech, detector=0, params=params)
    stc_sites = []
    for c in range(n_cells):
        ncv = b.cv_off[c + 1] - b.cv_off[c]
        for _ in range(int(rng_s.integers(1, 6))):
            stc_sites.append(b.add_syn(c, int(rng_s.integers(0, ncv)), KIND_STC, 5.0, 0.0))
        for _ in range(n_static):
            erev = 0.0 if rng_s.random() < 0.7 else -80.0
            b.add_syn(c, int(rng_s.integers(0, ncv)), KIND_EXPSYN,
                      float(rng_s.uniform(2.0, 8.0)), erev)
    n_syn = len(b.syn)
    kinds = np.array([x[2] for x in b.syn])
    src, dst, ports, w, d = [], [], [], [], []
    for tgt in range(n_cells):
        for s_ in range(n_cells):
            if s_ != tgt and rng_c.random() < p:
                cell_syns = [i for i in range(n_syn) if b.syn[i][0] == tgt]
                sid = int(rng_c.choice(cell_syns))
                src.append(s_); dst.append(sid)
                ports.append(PORT_G | PORT_CA if kinds[sid] == KIND_STC else PORT_G)
                inh = b.syn[sid][4] < -1
                w.append(float(rng_c.uniform(0.002, 0.02)) * (1.0 if not inh else 2.0))
                d.append(float(rng_c.uniform(*delay_range)))
    b.add_conns(src, dst, ports, w, d)
    for c in range(n_cells):
        cell_syns = [i for i in range(n_syn) if b.syn[i][0] == c]
        sid = int(rng_t.choice(cell_syns))
        pr = PORT_G | PORT_CA if kinds[sid] == KIND_STC else PORT_G
        b.add_train(sid, pr, w_ext, poisson_times(rng_t, ext_rate, t_end))
    if poisson:
        for c in range(n_cells):
            cell_syns = [i for i in range(n_syn) if b.syn[i][0] == c]
            sid = int(rng_t.choice(cell_syns))
            pr = PORT_G | PORT_CA if kinds[sid] == KIND_STC else PORT_G
            b.add_poisson(sid, pr, w_ext, ext_rate)
    if clamp:
        b.add_clamp(0, 0, 5.0, 40.0, 0.3)
        b.add_clamp(min(2, n_cells - 1), 0, 60.0, 30.0, 0.25)
    stc = dict(STC_TABLE5)
    stc.update(CA_INVIVO)
    return b.finish("tiny", dt, t_end, seed, stc)


def burst_network(seed=11, n_cells=160, t_end=60.0, n_dend=5, w=0.0004, delay=3.0):
    """All-to-all network whose cells all fire in one step: identical ball-
    and-stick cells, every ordered pair connected through both ports onto a
    plastic synapse of its own on a random dendrite CV, plus a second
    connection from the next cell onto the same synapse (two streams from one
    source into one synapse, equal delivery times); one suprathreshold clamp
    pulse on every soma at 2 ms.  Each cell then receives n_cells - 1 + 1
    conductance events with equal delivery times from different sources in a
    single step, and as many calcium events t_c,delay later."""
    rng_p, = _streams(seed, 1)
    b = _Builder()
    morph = ball_and_stick(n_dend, 100.0, 1.0, 20.0)
    for _ in range(n_cells):
        b.add_cell(*morph)
    src, dst = [], []
    for tgt in range(n_cells):
        for s_ in range(n_cells):
            if s_ == tgt:
                continue
            sid = b.add_syn(tgt, int(rng_p.integers(1, n_dend + 1)), KIND_STC, 5.0, 0.0)
            src.append(s_)
            dst.append(sid)
            if s_ == (tgt + 1) % n_cells:
                src.append(s_)
                dst.append(sid)
    b.add_conns(src, dst, PORT_G | PORT_CA, w, delay)
    for c in range(n_cells):
        b.add_clamp(c, 0, 2.0, 1.0, 2.0)
    stc = dict(STC_TABLE5)
    stc.update(CA_INVIVO)
    return b.finish("burst", 0.2, t_end, seed, stc)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def summary(net):
    """Sizes of a network dictionary."""
    kinds = net["syn_kind"]
    return dict(name=net["name"], cells=int(net["n_cells"]), cvs=int(net["cv_off"][-1]),
                syn=int(len(kinds)), stc=int((kinds == KIND_STC).sum()),
                conns=int(len(net["conn_src"])), trains=int(len(net["train_dst"])),
                train_events=int(len(net["train_times"])), poisson=int(len(net.get("pois_dst", []))))
