"""C ABI contract checks that need no GPU: the library loads, exports every
symbol include/psst.h declares, and rejects invalid arguments before any
device call (status INVALID_ARGUMENT with a message), while valid requests
on a machine without a gfx950 device report DEVICE."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1906_03958_amd import psst
from paper_1906_03958_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "psst.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psst_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(psst.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = C.CDLL(psst.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_device_count():
    assert "gfx950" in psst.version()
    assert psst.device_count() >= 0


def _gpu_present():
    return psst.device_count() > 0


def _create_raw(inst, mutate=None, n=None, n_path=None):
    """Call psst_network_create with ctypes structs, optionally mutated."""
    net = inst.net
    keep = []
    vec = {}
    for k in W.PARAM_NAMES:
        a = np.ascontiguousarray(net.params[k], np.float32)
        keep.append(a)
        vec[k] = a.ctypes.data_as(C.POINTER(C.c_float))
    p = psst.NeuronParams(vec["C_m"], vec["g_Na"], vec["g_K"], vec["g_L"], vec["E_Na"],
                          vec["E_K"], vec["E_L"], net.n_pn, net.area_cm2)
    paths = (psst.Pathway * max(1, len(net.pathways)))()
    for q, w in enumerate(net.pathways):
        g = np.ascontiguousarray(w.g_nS, np.float32)
        keep.append(g)
        paths[q] = psst.Pathway(w.type, w.pre_begin, w.pre_end, w.post_begin, w.post_end,
                                g.ctypes.data_as(C.POINTER(C.c_float)), None)
    kin = (psst.Kinetics * 3)()
    for t in range(3):
        kin[t] = psst.Kinetics(*[float(x) for x in net.kinetics[t]])
    if mutate:
        mutate(p, paths, kin, keep)
    h = C.c_void_p()
    st = psst.lib().psst_network_create(C.byref(p), net.n if n is None else n, paths,
                                        len(net.pathways) if n_path is None else n_path, kin,
                                        C.byref(h))
    return st, h


def _expect_invalid(mutate=None, **kw):
    st, h = _create_raw(W.config1(0), mutate, **kw)
    assert st == psst.ERR_INVALID_ARGUMENT, (st, psst.last_error())
    assert not h.value
    assert psst.last_error()


def test_network_create_validation():
    _expect_invalid(n=0)
    _expect_invalid(n_path=-1)
    _expect_invalid(n_path=65)

    def neg_area(p, paths, kin, keep):
        p.area_cm2 = -1.0
    _expect_invalid(neg_area)

    def bad_pn(p, paths, kin, keep):
        p.n_pn = 21
    _expect_invalid(bad_pn)

    def null_vec(p, paths, kin, keep):
        p.g_K = None
    _expect_invalid(null_vec)

    def nan_param(p, paths, kin, keep):
        a = np.full(20, np.nan, np.float32)
        keep.append(a)
        p.E_L = a.ctypes.data_as(C.POINTER(C.c_float))
    _expect_invalid(nan_param)

    def zero_cm(p, paths, kin, keep):
        a = np.zeros(20, np.float32)
        keep.append(a)
        p.C_m = a.ctypes.data_as(C.POINTER(C.c_float))
    _expect_invalid(zero_cm)

    def ach_from_ln(p, paths, kin, keep):
        paths[0].pre_end = 18          # ACh block reaching into LN rows
    _expect_invalid(ach_from_ln)

    def gaba_from_pn(p, paths, kin, keep):
        paths[1].pre_begin = 10
    _expect_invalid(gaba_from_pn)

    def out_of_range(p, paths, kin, keep):
        paths[0].post_end = 21
    _expect_invalid(out_of_range)

    def empty_block(p, paths, kin, keep):
        paths[0].post_end = paths[0].post_begin
    _expect_invalid(empty_block)

    def bad_type(p, paths, kin, keep):
        paths[0].type = 7
    _expect_invalid(bad_type)

    def null_g(p, paths, kin, keep):
        paths[0].g_nS = None
    _expect_invalid(null_g)

    def kp_zero(p, paths, kin, keep):
        kin[0].K_p = 0.0
    _expect_invalid(kp_zero)


def test_overlapping_blocks_and_bad_hill_rejected():
    inst = W.config2(0, t_ms=1.0)

    def overlap(p, paths, kin, keep):
        paths[2].post_begin = 0       # second GABA_A block now overlaps the first
        paths[2].post_end = 30
    st, _ = _create_raw(inst, overlap)
    assert st == psst.ERR_INVALID_ARGUMENT

    def hill(p, paths, kin, keep):
        kin[2].hill_n = 2.5
    st, _ = _create_raw(inst, hill)
    assert st == psst.ERR_INVALID_ARGUMENT


def test_valid_network_without_device_reports_device():
    if _gpu_present():
        pytest.skip("a GPU is present")
    st, h = _create_raw(W.config1(0))
    assert st == psst.ERR_DEVICE and not h.value
    assert "device" in psst.last_error().lower()


def test_null_handles_rejected():
    L = psst.lib()
    assert L.psst_network_destroy(None) == psst.ERR_INVALID_ARGUMENT
    assert L.psst_batch_destroy(None) == psst.ERR_INVALID_ARGUMENT
    assert L.psst_integrate(None, None, None, 0.01, 1, 0, None, None) == psst.ERR_INVALID_ARGUMENT
    assert L.psst_integrate_batch(None, None, None, 0.01, 1, 0, None, None, 0, None) == \
        psst.ERR_INVALID_ARGUMENT
    assert L.psst_adjoint(None, None, 1, None, 0.01, 1, 0, None, None, None, None, None, 0,
                          None) == psst.ERR_INVALID_ARGUMENT
    h = C.c_void_p()
    assert L.psst_batch_create(None, 1, C.byref(h)) == psst.ERR_INVALID_ARGUMENT
    arr = (C.c_void_p * 1)(None)
    assert L.psst_batch_create(arr, 1, C.byref(h)) == psst.ERR_INVALID_ARGUMENT
    assert L.psst_batch_create(arr, 0, C.byref(h)) == psst.ERR_INVALID_ARGUMENT
    nw, nv = C.c_int64(), C.c_int32()
    assert L.psst_state_layout(None, C.byref(nw), C.byref(nv)) == psst.ERR_INVALID_ARGUMENT
    r, s = C.c_int64(), C.c_int64()
    assert L.psst_batch_conductance_bytes(None, C.byref(r), C.byref(s)) == \
        psst.ERR_INVALID_ARGUMENT
    assert L.psst_network_update(None, None, None, None, None, None) == psst.ERR_INVALID_ARGUMENT


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(psst, "_lib", None)
    monkeypatch.setattr(psst, "LIB_PATH", "/nonexistent/libpsst.so")
    with pytest.raises(psst.PsstError):
        psst.lib()
