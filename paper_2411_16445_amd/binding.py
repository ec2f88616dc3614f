"""Thin ctypes binding of libplasticarbor.so (include/plasticarbor.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  The functions keep the C names (``pa_cells_add`` ...); the
``Simulation`` class strings them together for a network dictionary of the
layout documented in the generator module, and hands the library PyTorch's
current stream and caching allocator when PyTorch sees a GPU.

Loading fails loudly (``ImportError``) if the shared library has not been
built; there is no other execution path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplasticarbor.so")

PA_OK, PA_EINVAL, PA_ESTATE, PA_ENOMEM, PA_EDEVICE, PA_ERANGE, PA_EOVERFLOW, PA_ENUMERIC = \
    0, -1, -2, -3, -4, -5, -6, -7
PA_FP64, PA_MIXED = 0, 1
PA_PLAIN, PA_BATCHED = 0, 1
PA_PORT_G, PA_PORT_CA = 1, 2
PA_PROBE = {"V": 0, "g": 1, "c": 2, "h": 3, "z": 4, "p": 5, "sps": 6, "prp": 7}
PA_STATE = {"V": 0, "m": 1, "hh": 2, "n": 3, "g": 4, "c": 5, "h": 6, "z": 7, "p": 8,
            "evcount": 9, "evstepsum": 10, "sps": 11, "prp": 12}

EXPORTS = [
    "pa_sim_create", "pa_sim_destroy", "pa_set_stream", "pa_set_allocator", "pa_set_diffusion", "pa_set_stdp", "pa_cells_add",
    "pa_synapses_add", "pa_connect", "pa_trains_add", "pa_poisson_add", "pa_clamps_add", "pa_probes_add",
    "pa_finalize", "pa_advance", "pa_advance_steps", "pa_spikes_count", "pa_spikes_read",
    "pa_probe_count", "pa_probe_read", "pa_state_read", "pa_state_read_device", "pa_state_write",
    "pa_stats_get", "pa_retune", "pa_fast_forward", "pa_state_size", "pa_state_save", "pa_state_load",
    "pa_kernel_timing", "pa_kernel_time", "pa_tree_solve", "pa_tree_solve_noalloc", "pa_gb_trials", "pa_last_error",
    "pa_status_str",
]


class pa_config(C.Structure):
    _fields_ = [("dt_ms", C.c_double), ("threshold_mV", C.c_double), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("mode", C.c_int32), ("flags", C.c_uint32),
                ("cells_per_block", C.c_uint32),
                ("block_threads", C.c_uint16), ("solver_waves", C.c_uint16), ("exchange", C.c_uint32)]


STC_FIELDS = ["tau_c", "tau_h", "tau_p", "tau_z", "gamma_p", "gamma_d", "theta_p", "theta_d",
              "sigma_pl", "p_max", "f_int", "t_cd", "h0", "theta_pro", "theta_tag", "c_pre",
              "c_post"]


class pa_stc_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in STC_FIELDS]


class pa_stdp_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("tau_pre", "tau_post", "a_pre", "a_post", "w0", "w_max")]


class pa_gb_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("tau_w", "w_star", "gamma_p", "gamma_d", "theta_p", "theta_d", "sigma",
                                          "tau_c", "c_pre", "c_post", "t_cd")]


class pa_cell_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("cm", "ra", "v_init", "g_pas", "e_pas", "gna", "gk",
                                          "gl", "ena", "ek", "el")]


class pa_stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("n_cells", "n_cv", "n_syn", "n_stc", "n_conn",
                                          "n_trains", "n_probes", "n_poisson", "steps", "spikes",
                                          "events")] + \
        [("epoch_steps", C.c_uint32), ("spike_ring", C.c_uint32), ("queue_events", C.c_uint64),
         ("cells_per_block", C.c_uint32), ("advance_ms", C.c_double), ("device_bytes", C.c_uint64),
         ("block_threads", C.c_uint32), ("solver_waves", C.c_uint32), ("exchange", C.c_uint32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None

# Simulations still open at interpreter exit are destroyed while torch (whose
# caching allocator owns their device memory) is still intact.
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    for sim in list(_LIVE):
        sim.close()


_P = C.c_void_p


def load_library(path: str = None):
    """Loads the in-tree libplasticarbor.so; raises ImportError if it is not
    built."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2411_16445_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname; importing it
    # first makes the library bind to that one, so the process holds a
    # single HIP runtime shared with the torch streams and allocator.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    st = C.c_int32
    sig = {
        "pa_sim_create": (st, [C.POINTER(pa_config), C.POINTER(pa_stc_params), C.POINTER(_P)]),
        "pa_sim_destroy": (None, [_P]),
        "pa_set_stream": (st, [_P, _P]),
        "pa_set_allocator": (st, [_P, ALLOC_FN, FREE_FN, _P]),
        "pa_set_diffusion": (st, [_P, C.c_double, C.c_double]),
        "pa_set_stdp": (st, [_P, C.POINTER(pa_stdp_params)]),
        "pa_cells_add": (st, [_P, C.c_uint32, _P, _P, _P, _P, _P, _P, _P, C.POINTER(C.c_uint32)]),
        "pa_synapses_add": (st, [_P, C.c_uint32, _P, _P, _P, _P, _P, C.POINTER(C.c_uint32)]),
        "pa_connect": (st, [_P, C.c_uint64, _P, _P, _P, _P, _P]),
        "pa_trains_add": (st, [_P, C.c_uint32, _P, _P, _P, _P, _P]),
        "pa_poisson_add": (st, [_P, C.c_uint32, _P, _P, _P, _P]),
        "pa_clamps_add": (st, [_P, C.c_uint32, _P, _P, _P, _P, _P]),
        "pa_probes_add": (st, [_P, C.c_uint32, _P, _P, _P, C.POINTER(C.c_uint32)]),
        "pa_finalize": (st, [_P]),
        "pa_advance": (st, [_P, C.c_double]),
        "pa_advance_steps": (st, [_P, C.c_uint64]),
        "pa_spikes_count": (st, [_P, C.POINTER(C.c_uint64)]),
        "pa_spikes_read": (st, [_P, _P, _P, _P, C.c_uint64, C.POINTER(C.c_uint64)]),
        "pa_probe_count": (st, [_P, C.c_uint32, C.POINTER(C.c_uint64)]),
        "pa_probe_read": (st, [_P, C.c_uint32, _P, C.c_uint64, C.POINTER(C.c_uint64)]),
        "pa_state_read": (st, [_P, C.c_int32, _P, C.c_uint64]),
        "pa_state_read_device": (st, [_P, C.c_int32, _P, C.c_uint64]),
        "pa_state_write": (st, [_P, C.c_int32, _P, C.c_uint64]),
        "pa_stats_get": (st, [_P, C.POINTER(pa_stats)]),
        "pa_retune": (st, [_P]),
        "pa_fast_forward": (st, [_P, C.c_uint64, C.c_double]),
        "pa_state_size": (st, [_P, C.POINTER(C.c_uint64)]),
        "pa_state_save": (st, [_P, _P, C.c_uint64]),
        "pa_state_load": (st, [_P, _P, C.c_uint64]),
        "pa_kernel_timing": (st, [_P, C.c_int32]),
        "pa_kernel_time": (st, [_P, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_char_p)]),
        "pa_tree_solve": (st, [C.c_uint32, C.c_uint64, _P, _P, _P, _P, _P, _P, _P]),
        "pa_tree_solve_noalloc": (st, [C.c_uint32, C.c_uint64, _P, _P, _P, _P, _P, _P, _P]),
        "pa_gb_trials": (st, [C.POINTER(pa_gb_params), C.c_double, C.c_uint64, _P, _P, C.c_uint32, C.c_double,
                              C.c_double, C.c_uint64, _P, _P, _P]),
        "pa_last_error": (C.c_char_p, [_P]),
        "pa_status_str": (C.c_char_p, [C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def gb_trials(params: dict, dt, delays, w0, n_pairs=60, period=1000.0, t0=100.0, seed=1):
    """Graupner-Brunel trials on the device (pa_gb_trials): delays and w0
    are float64 device tensors (or arrays, copied to the device); returns
    the final weights and calcium as device tensors."""
    import torch
    lib = load_library()
    d = torch.as_tensor(delays, dtype=torch.float64, device="cuda").contiguous()
    w = torch.as_tensor(w0, dtype=torch.float64, device="cuda").contiguous()
    out = torch.empty_like(d)
    cout = torch.empty_like(d)
    prm = pa_gb_params(*[float(params[k]) for k, _ in pa_gb_params._fields_])
    st = lib.pa_gb_trials(C.byref(prm), float(dt), d.numel(), C.c_void_p(d.data_ptr()), C.c_void_p(w.data_ptr()),
                          int(n_pairs), float(period), float(t0), int(seed), C.c_void_p(out.data_ptr()),
                          C.c_void_p(cout.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != PA_OK:
        raise PAError(st, lib.pa_status_str(st).decode())
    return out, cout


class PAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def stc_params(d: dict) -> pa_stc_params:
    s = pa_stc_params()
    for k in STC_FIELDS:
        setattr(s, k, float(d[k]))
    return s


class Simulation:
    """A network built through the C ABI from a network dictionary.

    precision: "fp64" | "mixed"; mode: "plain" | "batched".
    probes: list of (quantity, index) or (quantity, index, stride_steps) with
    quantity in V, g, c, h, z, p (and sps, prp per CV with particle
    diffusion, net["diffusion"] = {d_sps, d_prp} in um^2/ms); probe_stride
    is the stride of those without one.
    """

    def __init__(self, net: dict, precision="fp64", mode="plain", probes=(), probe_stride=1,
                 cells_per_block=0, block_threads=0, solver_waves=0, exchange="auto",
                 use_torch=True):
        lib = load_library()
        self._lib = lib
        cfg = pa_config()
        cfg.dt_ms = float(net["dt"])
        cfg.threshold_mV = float(net["theta"])
        cfg.seed = int(net["seed"]) & (2**64 - 1)
        cfg.precision = {"fp64": PA_FP64, "mixed": PA_MIXED}[precision]
        cfg.mode = {"plain": PA_PLAIN, "batched": PA_BATCHED}[mode]
        cfg.flags = 0
        cfg.cells_per_block = int(cells_per_block)
        cfg.block_threads = int(block_threads)
        cfg.solver_waves = int(solver_waves)
        cfg.exchange = {"auto": 0, "kernel": 1, "resident": 2}[exchange]
        stc = stc_params(net["stc"])
        h = _P()
        st = lib.pa_sim_create(C.byref(cfg), C.byref(stc), C.byref(h))
        if st != PA_OK:
            raise PAError(st, "pa_sim_create rejected the configuration")
        self._h = h
        _LIVE.add(self)
        self.dt = cfg.dt_ms
        self._torch_cb = None
        if use_torch:
            self._attach_torch()
        sp = net.get("stdp")
        if sp:
            prm = pa_stdp_params(*[float(sp[k]) for k in ("tau_pre", "tau_post", "a_pre", "a_post", "w0", "w_max")])
            self._check(lib.pa_set_stdp(h, C.byref(prm)))
        self._add_network(net)
        dif = net.get("diffusion")
        if dif:
            self._check(lib.pa_set_diffusion(h, float(dif["d_sps"]), float(dif["d_prp"])))
        if probes:
            what = np.array([PA_PROBE[p[0]] for p in probes], np.int32)
            idx = np.array([int(p[1]) for p in probes], np.uint64)
            stride = np.array([int(p[2]) if len(p) > 2 else int(probe_stride) for p in probes], np.uint32)
            self._check(lib.pa_probes_add(h, len(what), _ptr(what), _ptr(idx), _ptr(stride), None))
        self.n_probes = len(probes)
        self._check(lib.pa_finalize(h))
        s = self.stats()
        self.n_cells, self.n_cv, self.n_syn = s["n_cells"], s["n_cv"], s["n_syn"]
        self.n_hh = int((np.asarray(net["mech"]) == 1).sum())

    # -------------------------------------------------------------- plumbing
    def _attach_torch(self):
        try:
            import torch
        except ImportError:
            return
        if not torch.cuda.is_available():
            return
        dev = torch.cuda.current_device()
        stream = torch.cuda.current_stream(dev)

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except Exception:
                return None

        release = torch.cuda.caching_allocator_delete

        def _free(ptr, ctx):
            try:
                release(ptr)
            except Exception:
                pass  # interpreter shutdown: the process returns the memory

        self._torch_cb = (ALLOC_FN(_alloc), FREE_FN(_free), stream)
        self._check(self._lib.pa_set_stream(self._h, C.c_void_p(stream.cuda_stream)))
        self._check(self._lib.pa_set_allocator(self._h, self._torch_cb[0], self._torch_cb[1], None))

    def _check(self, st):
        if st != PA_OK:
            msg = self._lib.pa_last_error(self._h)
            raise PAError(st, msg.decode() if msg else self._lib.pa_status_str(st).decode())

    def _add_network(self, net):
        lib, h = self._lib, self._h
        n_cells = int(net["n_cells"])
        cv_off = np.ascontiguousarray(net["cv_off"], np.int64)
        cp = net["cell_params"]
        params = (pa_cell_params * max(1, n_cells))()
        for c in range(n_cells):
            params[c] = pa_cell_params(*[float(x) for x in cp[c]])
        arrs = {k: np.ascontiguousarray(net[k], t) for k, t in (
            ("parent", np.int32), ("length", np.float64), ("diam", np.float64),
            ("mech", np.uint8), ("detector", np.int32))}
        self._check(lib.pa_cells_add(h, n_cells, _ptr(cv_off), _ptr(arrs["parent"]),
                                     _ptr(arrs["length"]), _ptr(arrs["diam"]), _ptr(arrs["mech"]),
                                     _ptr(arrs["detector"]), C.cast(params, _P), None))
        sc = np.ascontiguousarray(net["syn_cell"], np.uint32)
        scv = np.ascontiguousarray(net["syn_cv"], np.uint32)
        sk = np.ascontiguousarray(net["syn_kind"], np.uint8)
        stau = np.ascontiguousarray(net["syn_tau"], np.float64)
        serev = np.ascontiguousarray(net["syn_erev"], np.float64)
        self._check(lib.pa_synapses_add(h, len(sc), _ptr(sc), _ptr(scv), _ptr(sk), _ptr(stau),
                                        _ptr(serev), None))
        cs = np.ascontiguousarray(net["conn_src"], np.uint32)
        cd = np.ascontiguousarray(net["conn_dst"], np.uint32)
        cpo = np.ascontiguousarray(net["conn_ports"], np.uint8)
        cw = np.ascontiguousarray(net["conn_w"], np.float64)
        cdl = np.ascontiguousarray(net["conn_d"], np.float64)
        self._check(lib.pa_connect(h, len(cs), _ptr(cs), _ptr(cd), _ptr(cpo), _ptr(cw), _ptr(cdl)))
        td = np.ascontiguousarray(net["train_dst"], np.uint32)
        tp = np.ascontiguousarray(net["train_ports"], np.uint8)
        tw = np.ascontiguousarray(net["train_w"], np.float64)
        to = np.ascontiguousarray(net["train_off"], np.int64)
        tt = np.ascontiguousarray(net["train_times"], np.float64)
        if len(td):
            self._check(lib.pa_trains_add(h, len(td), _ptr(td), _ptr(tp), _ptr(tw), _ptr(to), _ptr(tt)))
        pd = np.ascontiguousarray(net.get("pois_dst", np.zeros(0)), np.uint32)
        if len(pd):
            self._check(lib.pa_poisson_add(
                h, len(pd), _ptr(pd), _ptr(np.ascontiguousarray(net["pois_ports"], np.uint8)),
                _ptr(np.ascontiguousarray(net["pois_w"], np.float64)),
                _ptr(np.ascontiguousarray(net["pois_rate"], np.float64))))
        kc = np.ascontiguousarray(net["clamp_cell"], np.uint32)
        if len(kc):
            self._check(lib.pa_clamps_add(
                h, len(kc), _ptr(kc), _ptr(np.ascontiguousarray(net["clamp_cv"], np.uint32)),
                _ptr(np.ascontiguousarray(net["clamp_t0"], np.float64)),
                _ptr(np.ascontiguousarray(net["clamp_dur"], np.float64)),
                _ptr(np.ascontiguousarray(net["clamp_amp"], np.float64))))

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.pa_sim_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    # -------------------------------------------------------------- running
    def advance(self, t_ms: float):
        self._check(self._lib.pa_advance(self._h, float(t_ms)))

    def advance_steps(self, n: int):
        self._check(self._lib.pa_advance_steps(self._h, int(n)))

    def retune(self):
        """Batched form: choose the plan again from the present state."""
        self._check(self._lib.pa_retune(self._h))

    def fast_forward(self, n_long: int, dt_long: float):
        """n_long long steps of the slow plasticity variables only (spiking
        and calcium off); time moves by n_long * dt_long ms."""
        self._check(self._lib.pa_fast_forward(self._h, int(n_long), float(dt_long)))

    def state_size(self) -> int:
        n = C.c_uint64()
        self._check(self._lib.pa_state_size(self._h, C.byref(n)))
        return n.value

    def save_state(self, buf=None):
        """Dumps the whole mutable state into `buf` (a uint8 device tensor or
        numpy array of state_size() bytes; a new numpy array if None)."""
        if buf is None:
            buf = np.zeros(self.state_size(), np.uint8)
        ptr = buf.data_ptr() if hasattr(buf, "data_ptr") else buf.ctypes.data
        nbytes = buf.numel() * buf.element_size() if hasattr(buf, "data_ptr") else buf.nbytes
        self._check(self._lib.pa_state_save(self._h, C.c_void_p(ptr), int(nbytes)))
        return buf

    def load_state(self, buf):
        ptr = buf.data_ptr() if hasattr(buf, "data_ptr") else buf.ctypes.data
        nbytes = buf.numel() * buf.element_size() if hasattr(buf, "data_ptr") else buf.nbytes
        self._check(self._lib.pa_state_load(self._h, C.c_void_p(ptr), int(nbytes)))

    def spikes(self):
        """The raster, (gid, step, t*) arrays in (t*, gid) order."""
        n = C.c_uint64()
        self._check(self._lib.pa_spikes_count(self._h, C.byref(n)))
        m = n.value
        gid = np.zeros(m, np.uint32)
        step = np.zeros(m, np.uint64)
        t = np.zeros(m, np.float64)
        got = C.c_uint64()
        self._check(self._lib.pa_spikes_read(self._h, _ptr(gid), _ptr(step), _ptr(t), m, C.byref(got)))
        return gid.astype(np.int64), step.astype(np.int64), t

    def probe(self, k: int) -> np.ndarray:
        """Samples of probe k, oldest first."""
        n = C.c_uint64()
        self._check(self._lib.pa_probe_count(self._h, int(k), C.byref(n)))
        out = np.zeros(n.value, np.float64)
        got = C.c_uint64()
        self._check(self._lib.pa_probe_read(self._h, int(k), _ptr(out), out.size, C.byref(got)))
        return out[:got.value]

    def probes(self):
        """Samples of probes with equal strides, shape (samples, probes)."""
        cols = [self.probe(k) for k in range(self.n_probes)]
        return np.stack(cols, axis=1) if cols else np.zeros((0, 0))

    def _size(self, what):
        return {"V": self.n_cv, "m": self.n_hh, "hh": self.n_hh, "n": self.n_hh,
                "p": self.n_cells, "sps": self.n_cv, "prp": self.n_cv}.get(what, self.n_syn)

    def read(self, what: str) -> np.ndarray:
        if what in ("evcount", "evstepsum"):
            out = np.zeros(2 * self.n_syn, np.uint64)
        else:
            out = np.zeros(self._size(what), np.float64)
        self._check(self._lib.pa_state_read(self._h, PA_STATE[what], _ptr(out) or C.c_void_p(1), out.size))
        return out

    def read_into(self, what: str, tensor) -> None:
        """State array `what` into a device tensor (float64, or int64 pairs
        for the event statistics) of the right size, without a host copy."""
        self._check(self._lib.pa_state_read_device(self._h, PA_STATE[what], C.c_void_p(tensor.data_ptr()),
                                                   int(tensor.numel())))

    def write(self, what: str, values):
        a = np.ascontiguousarray(values, np.float64)
        self._check(self._lib.pa_state_write(self._h, PA_STATE[what], _ptr(a) or C.c_void_p(1), a.size))

    def event_stats(self):
        return self.read("evcount").reshape(-1, 2), self.read("evstepsum").reshape(-1, 2)

    def stats(self) -> dict:
        s = pa_stats()
        self._check(self._lib.pa_stats_get(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in pa_stats._fields_}

    def kernel_timing(self, enable=True):
        self._check(self._lib.pa_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_uint64()
        name = C.c_char_p()
        self._check(self._lib.pa_kernel_time(self._h, C.byref(ms), C.byref(n), C.byref(name)))
        return ms.value, n.value, name.value.decode()
