"""Plain FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``oracle.c`` (compiled with gcc,
``-ffp-contract=off``) through ctypes; it shares no code with the HIP
library and imports nothing from it.

    net = netgen.config1(t_end=100.0)
    o = Oracle(net)
    o.run(500)
    v = o.read("V"); spikes = o.spikes()
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
# the same source with OpenMP over the independent per-CV, per-cell and
# per-synapse loops: only for timing the oracle on several host cores
LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

# -O2 without value-changing optimisations: no contraction into FMA, no
# fast-math; the library's results are those of the C source read literally.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (and the OpenMP timing build
    liboracle_omp.so) next to it; returns the path of the first."""
    for path, extra in ((LIB_PATH, []), (LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, SRC_PATH, "-lm"])
            os.replace(tmp, path)
    return LIB_PATH


_D = C.c_double
_I64 = C.c_int64
_P = C.c_void_p


class _Net(C.Structure):
    _fields_ = [("dt", _D), ("theta", _D), ("seed", C.c_uint64)] + \
        [(k, _D) for k in ("tau_c", "tau_h", "tau_p", "tau_z", "gamma_p", "gamma_d", "theta_p",
                           "theta_d", "sigma_pl", "p_max", "f_int", "t_cd", "h0", "theta_pro",
                           "theta_tag", "c_pre", "c_post")] + \
        [("n_cells", _I64), ("cv_off", _P), ("parent", _P), ("length", _P), ("diam", _P),
         ("mech", _P), ("detector", _P), ("cell_params", _P),
         ("n_syn", _I64), ("syn_cell", _P), ("syn_cv", _P), ("syn_kind", _P), ("syn_tau", _P),
         ("syn_erev", _P),
         ("n_conn", _I64), ("conn_src", _P), ("conn_dst", _P), ("conn_ports", _P), ("conn_w", _P),
         ("conn_d", _P),
         ("n_trains", _I64), ("train_dst", _P), ("train_ports", _P), ("train_w", _P),
         ("train_off", _P), ("train_times", _P),
         ("n_clamps", _I64), ("clamp_cell", _P), ("clamp_cv", _P), ("clamp_t0", _P),
         ("clamp_dur", _P), ("clamp_amp", _P),
         ("n_pois", _I64), ("pois_dst", _P), ("pois_ports", _P), ("pois_w", _P), ("pois_rate", _P),
         ("prp_model", _I64), ("d_sps", _D), ("d_prp", _D),
         ("tau_pre", _D), ("tau_post", _D), ("a_pre_amp", _D), ("a_post_amp", _D), ("w0", _D), ("w_max", _D)]


_libs = {}


def _load(threaded: bool = False):
    path = LIB_OMP_PATH if threaded else LIB_PATH
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        lib = C.CDLL(path)
        lib.orc_create.restype = _P
        lib.orc_create.argtypes = [C.POINTER(_Net), C.c_char_p, C.c_int]
        lib.orc_run.restype = C.c_int
        lib.orc_run.argtypes = [_P, _I64]
        lib.orc_fast_forward.restype = C.c_int
        lib.orc_fast_forward.argtypes = [_P, _I64, _D]
        lib.orc_error.restype = C.c_char_p
        lib.orc_error.argtypes = [_P]
        for f in ("orc_step_count", "orc_n_cv", "orc_n_hh", "orc_spike_count"):
            getattr(lib, f).restype = _I64
            getattr(lib, f).argtypes = [_P]
        lib.orc_spikes.argtypes = [_P, _P, _P, _P]
        lib.orc_read.restype = C.c_int
        lib.orc_read.argtypes = [_P, C.c_int, _P]
        lib.orc_write.restype = C.c_int
        lib.orc_write.argtypes = [_P, C.c_int, _P]
        lib.orc_assemble.argtypes = [_P, _P, _P, _P]
        lib.orc_hines.argtypes = [_I64, _P, _P, _P, _P, _P]
        lib.orc_destroy.argtypes = [_P]
        lib.orc_threefry4x64_12.argtypes = [_P, _P, _P]
        lib.orc_normal.restype = _D
        lib.orc_normal.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        lib.orc_hh_rates.argtypes = [_D, _P]
        lib.orc_poisson_isi.restype = _D
        lib.orc_poisson_isi.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, _D]
        _libs[path] = lib
    return _libs[path]


_READ = {"V": 0, "m": 1, "hh": 2, "n": 3, "g": 4, "c": 5, "h": 6, "z": 7, "p": 8, "sps": 11, "prp": 12}

_ARRAYS = {
    "cv_off": np.int64, "parent": np.int32, "length": np.float64, "diam": np.float64,
    "mech": np.uint8, "detector": np.int32, "cell_params": np.float64,
    "syn_cell": np.int32, "syn_cv": np.int32, "syn_kind": np.uint8, "syn_tau": np.float64,
    "syn_erev": np.float64, "conn_src": np.int32, "conn_dst": np.int32, "conn_ports": np.uint8,
    "conn_w": np.float64, "conn_d": np.float64, "train_dst": np.int32, "train_ports": np.uint8,
    "train_w": np.float64, "train_off": np.int64, "train_times": np.float64,
    "clamp_cell": np.int32, "clamp_cv": np.int32, "clamp_t0": np.float64,
    "clamp_dur": np.float64, "clamp_amp": np.float64,
    "pois_dst": np.int32, "pois_ports": np.uint8, "pois_w": np.float64, "pois_rate": np.float64,
}


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle simulation of a netgen network dictionary.  threaded=True
    uses the OpenMP build (same results; for timing on several cores)."""

    def __init__(self, net: dict, threaded: bool = False):
        lib = _load(threaded)
        self._keep = {k: np.ascontiguousarray(net.get(k, np.zeros(0, t)), dtype=t) for k, t in _ARRAYS.items()}
        st = net["stc"]
        s = _Net()
        s.dt, s.theta, s.seed = net["dt"], net["theta"], int(net["seed"]) & (2**64 - 1)
        for k in ("tau_c", "tau_h", "tau_p", "tau_z", "gamma_p", "gamma_d", "theta_p", "theta_d",
                  "sigma_pl", "p_max", "f_int", "t_cd", "h0", "theta_pro", "theta_tag", "c_pre",
                  "c_post"):
            setattr(s, k, float(st[k]))
        for k, a in self._keep.items():
            setattr(s, k, a.ctypes.data)
        s.n_cells = int(net["n_cells"])
        s.n_syn = len(self._keep["syn_cell"])
        s.n_conn = len(self._keep["conn_src"])
        s.n_trains = len(self._keep["train_dst"])
        s.n_clamps = len(self._keep["clamp_cell"])
        s.n_pois = len(self._keep["pois_dst"])
        dif = net.get("diffusion")
        s.prp_model = 1 if dif else 0
        s.d_sps = float(dif["d_sps"]) if dif else 0.0
        s.d_prp = float(dif["d_prp"]) if dif else 0.0
        sp = net.get("stdp") or {}
        s.tau_pre, s.tau_post = float(sp.get("tau_pre", 1.0)), float(sp.get("tau_post", 1.0))
        s.a_pre_amp, s.a_post_amp = float(sp.get("a_pre", 0.0)), float(sp.get("a_post", 0.0))
        s.w0, s.w_max = float(sp.get("w0", 0.0)), float(sp.get("w_max", 0.0))
        self._s = s
        err = C.create_string_buffer(256)
        h = lib.orc_create(C.byref(s), err, 256)
        if not h:
            raise OracleError(err.value.decode())
        self._h = h
        self._lib = lib
        self.n_cells = s.n_cells
        self.n_syn = s.n_syn
        self.n_cv = lib.orc_n_cv(h)
        self.n_hh = lib.orc_n_hh(h)
        self.dt = net["dt"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def step(self) -> int:
        return self._lib.orc_step_count(self._h)

    def run(self, n_steps: int) -> None:
        if self._lib.orc_run(self._h, int(n_steps)) != 0:
            raise OracleError(self._lib.orc_error(self._h).decode())

    def fast_forward(self, n_long: int, dt_long: float) -> None:
        """n_long long steps of the slow plasticity variables only (spiking
        and calcium off); time moves by n_long * dt_long."""
        if self._lib.orc_fast_forward(self._h, int(n_long), float(dt_long)) != 0:
            raise OracleError(self._lib.orc_error(self._h).decode())

    def spikes(self):
        """The raster, (gid, step, t*) arrays in (t*, gid) order."""
        n = self._lib.orc_spike_count(self._h)
        gid = np.zeros(n, np.int64)
        step = np.zeros(n, np.int64)
        t = np.zeros(n, np.float64)
        if n:
            self._lib.orc_spikes(self._h, gid.ctypes.data, step.ctypes.data, t.ctypes.data)
            o = np.lexsort((gid, t))
            gid, step, t = gid[o], step[o], t[o]
        return gid, step, t

    def _size(self, what):
        return {0: self.n_cv, 1: self.n_hh, 2: self.n_hh, 3: self.n_hh, 8: self.n_cells, 11: self.n_cv,
                12: self.n_cv}.get(what, self.n_syn)

    def read(self, what: str) -> np.ndarray:
        code = _READ[what]
        out = np.zeros(self._size(code), np.float64)
        self._lib.orc_read(self._h, code, out.ctypes.data)
        return out

    def write(self, what: str, values) -> None:
        code = _READ[what]
        a = np.ascontiguousarray(values, np.float64)
        assert a.shape == (self._size(code),)
        self._lib.orc_write(self._h, code, a.ctypes.data)

    def event_stats(self):
        """Delivered events per (synapse, port) and the sum of their steps."""
        cnt = np.zeros(2 * self.n_syn, np.uint64)
        ssum = np.zeros(2 * self.n_syn, np.uint64)
        self._lib.orc_read(self._h, 9, cnt.ctypes.data)
        self._lib.orc_read(self._h, 10, ssum.ctypes.data)
        return cnt.reshape(-1, 2), ssum.reshape(-1, 2)

    def assemble(self):
        """(D, U, b) of the cable system at the present state (no time advance)."""
        D = np.zeros(self.n_cv)
        U = np.zeros(self.n_cv)
        b = np.zeros(self.n_cv)
        self._lib.orc_assemble(self._h, D.ctypes.data, U.ctypes.data, b.ctypes.data)
        return D, U, b


def hines(parent, U, D, b):
    """Oracle Hines solve of one tree system (parent[i] < i)."""
    lib = _load()
    parent = np.ascontiguousarray(parent, np.int64)
    U = np.ascontiguousarray(U, np.float64)
    D = np.array(D, np.float64)
    b = np.array(b, np.float64)
    x = np.zeros(len(D))
    lib.orc_hines(len(D), parent.ctypes.data, U.ctypes.data, D.ctypes.data, b.ctypes.data,
                  x.ctypes.data)
    return x


def threefry(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib.orc_threefry4x64_12(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def normal(seed, sid, n):
    return _load().orc_normal(int(seed), int(sid), int(n))


def poisson_isi(seed, k, j, rate_hz):
    return _load().orc_poisson_isi(int(seed), int(k), int(j), float(rate_hz))


class _GB(C.Structure):
    _fields_ = [(k, _D) for k in ("tau_w", "w_star", "gamma_p", "gamma_d", "theta_p", "theta_d", "sigma",
                                   "tau_c", "c_pre", "c_post", "t_cd")]


def gb_trials(params: dict, dt, delays, w0, n_pairs=60, period=1000.0, t0=100.0, seed=1, first_id=0):
    """Final weight and calcium of independent Graupner-Brunel synapses under
    the pairing protocol (one trial per entry of delays / w0; trial k draws
    the noise stream of trial id first_id + k)."""
    lib = _load()
    lib.orc_gb_trials.restype = C.c_int
    lib.orc_gb_trials.argtypes = [C.POINTER(_GB), _D, _I64, _P, _P, _I64, _D, _D, C.c_uint64, C.c_uint64, _P, _P]
    g = _GB(**{k: float(params[k]) for k, _ in _GB._fields_})
    d = np.ascontiguousarray(delays, np.float64)
    w = np.ascontiguousarray(w0, np.float64)
    out = np.zeros(len(d))
    cout = np.zeros(len(d))
    if lib.orc_gb_trials(C.byref(g), float(dt), len(d), d.ctypes.data, w.ctypes.data, int(n_pairs), float(period),
                         float(t0), int(seed), int(first_id), out.ctypes.data, cout.ctypes.data) != 0:
        raise OracleError("invalid Graupner-Brunel parameters")
    return out, cout


def hh_rates(v):
    r = np.zeros(6)
    _load().orc_hh_rates(float(v), r.ctypes.data)
    return r
