"""The C-ABI library: it loads, exports every function include/*.h
declares, and its host-side validation rejects bad input with the
documented status codes (no device needed: nothing here reaches
pa_finalize's device work)."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import netgen
from paper_2411_16445_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(pa_[a-z_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_function():
    lib = B.load_library()
    declared = _declared()
    assert len(declared) >= 20
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(B.EXPORTS)


def _sim(**over):
    lib = B.load_library()
    cfg = B.pa_config(dt_ms=0.2, threshold_mV=-10.0, seed=1, precision=0, mode=0, flags=0)
    for k, v in over.items():
        setattr(cfg, k, v)
    stc = B.stc_params(netgen.STC_TABLE5)
    h = C.c_void_p()
    st = lib.pa_sim_create(C.byref(cfg), C.byref(stc), C.byref(h))
    return lib, st, h


def test_create_validates_configuration():
    lib, st, h = _sim()
    assert st == B.PA_OK and h.value
    lib.pa_sim_destroy(h)
    lib.pa_sim_destroy(None)  # NULL-safe
    for bad in (dict(dt_ms=0.0), dict(dt_ms=float("nan")), dict(precision=7), dict(mode=3),
                dict(flags=1)):
        _, st, _ = _sim(**bad)
        assert st == B.PA_EINVAL, bad
    assert lib.pa_status_str(B.PA_EOVERFLOW) == b"event queue or spike history overflow"


def _add_cells(lib, h, parent, mech=None):
    n = len(parent)
    cv_off = np.array([0, n], np.int64)
    parent = np.array(parent, np.int32)
    length = np.full(n, 10.0)
    diam = np.full(n, 1.0)
    mech = np.zeros(n, np.uint8) if mech is None else np.array(mech, np.uint8)
    det = np.zeros(1, np.int32)
    p = B.pa_cell_params(*netgen.DEFAULT_CELL)
    return lib.pa_cells_add(h, 1, cv_off.ctypes.data, parent.ctypes.data, length.ctypes.data,
                            diam.ctypes.data, mech.ctypes.data, det.ctypes.data, C.byref(p), None)


def test_build_phase_validation():
    lib, st, h = _sim()
    assert _add_cells(lib, h, [-1, 1]) == B.PA_EINVAL          # parent[1] not < 1
    assert b"parent" in lib.pa_last_error(h)
    assert _add_cells(lib, h, [0, 0]) == B.PA_EINVAL           # root must have parent -1
    assert _add_cells(lib, h, [-1, 0, 1, 1]) == B.PA_OK
    gid = np.array([0], np.uint32)
    kind = np.array([1], np.uint8)
    tau = np.array([5.0])
    erev = np.array([0.0])
    bad_cv = np.array([4], np.uint32)
    assert lib.pa_synapses_add(h, 1, gid.ctypes.data, bad_cv.ctypes.data, kind.ctypes.data,
                               tau.ctypes.data, erev.ctypes.data, None) == B.PA_EINVAL
    cv = np.array([3], np.uint32)
    sid = C.c_uint32()
    assert lib.pa_synapses_add(h, 1, gid.ctypes.data, cv.ctypes.data, kind.ctypes.data,
                               tau.ctypes.data, erev.ctypes.data, C.byref(sid)) == B.PA_OK
    exp_kind = np.array([0], np.uint8)
    assert lib.pa_synapses_add(h, 1, gid.ctypes.data, cv.ctypes.data, exp_kind.ctypes.data,
                               tau.ctypes.data, erev.ctypes.data, None) == B.PA_OK  # sid 1
    src = np.array([0], np.uint32)
    w = np.array([0.01])
    for dst, ports, d, expect in ((0, 3, 1.0, B.PA_OK), (0, 3, 0.1, B.PA_EINVAL),  # delay < dt
                                  (1, 2, 1.0, B.PA_EINVAL),  # calcium port on exp-syn
                                  (2, 1, 1.0, B.PA_EINVAL),  # no synapse 2
                                  (1, 0, 1.0, B.PA_EINVAL)):  # no port
        dst_a = np.array([dst], np.uint32)
        pa = np.array([ports], np.uint8)
        da = np.array([d])
        assert lib.pa_connect(h, 1, src.ctypes.data, dst_a.ctypes.data, pa.ctypes.data,
                              w.ctypes.data, da.ctypes.data) == expect, (dst, ports, d)
    off = np.array([0, 2], np.int64)
    times = np.array([3.0, 1.0])  # decreasing
    tdst = np.array([0], np.uint32)
    tp = np.array([3], np.uint8)
    assert lib.pa_trains_add(h, 1, tdst.ctypes.data, tp.ctypes.data, w.ctypes.data,
                             off.ctypes.data, times.ctypes.data) == B.PA_EINVAL
    times = np.array([1.0, 3.0])
    assert lib.pa_trains_add(h, 1, tdst.ctypes.data, tp.ctypes.data, w.ctypes.data,
                             off.ctypes.data, times.ctypes.data) == B.PA_OK
    what = np.array([3], np.int32)  # h of an exp-syn
    idx = np.array([1], np.uint64)
    stride = np.array([1], np.uint32)
    assert lib.pa_probes_add(h, 1, what.ctypes.data, idx.ctypes.data, stride.ctypes.data, None) == B.PA_EINVAL
    what = np.array([0], np.int32)  # V of CV 0, stride 0
    idx = np.array([0], np.uint64)
    stride = np.array([0], np.uint32)
    assert lib.pa_probes_add(h, 1, what.ctypes.data, idx.ctypes.data, stride.ctypes.data, None) == B.PA_EINVAL
    stride = np.array([7], np.uint32)
    first = C.c_uint32()
    assert lib.pa_probes_add(h, 1, what.ctypes.data, idx.ctypes.data, stride.ctypes.data, C.byref(first)) == B.PA_OK
    assert first.value == 0
    assert lib.pa_advance(h, 1.0) == B.PA_ESTATE  # before finalize
    out = np.zeros(4)
    assert lib.pa_state_read(h, 0, out.ctypes.data, 4) == B.PA_ESTATE
    lib.pa_sim_destroy(h)


def test_simulation_class_fails_loudly_without_device(monkeypatch):
    """Without a GPU the product path raises; it never computes on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    net = netgen.tiny(seed=1, n_cells=3, t_end=10.0)
    with pytest.raises(B.PAError) as e:
        B.Simulation(net)
    assert e.value.status == B.PA_EDEVICE
