"""Python binding of libpsst.so: the calls of include/psst.h under the same
names, marshalling arguments only (no arithmetic of the method happens here).

Device buffers are torch tensors on the GPU; the binding passes their
``data_ptr()`` and the current HIP stream.  The library must be built
(``__graft_entry__.build()``); if it is missing every call raises
:class:`PsstError` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsst.so")

OK, ERR_INVALID_ARGUMENT, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NONFINITE, ERR_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARGUMENT", 2: "OUT_OF_MEMORY", 3: "DEVICE",
                4: "NONFINITE", 5: "UNSUPPORTED"}
SYN_ACH, SYN_GABA_A, SYN_GABA_B = 0, 1, 2
N_VARS = 7
WORDS_PER_NEURON = 14

#: every symbol include/psst.h declares
EXPORTS = (
    "psst_last_error", "psst_version", "psst_device_count",
    "psst_network_create", "psst_network_destroy", "psst_state_layout",
    "psst_state_init", "psst_integrate", "psst_network_poll",
    "psst_batch_create", "psst_batch_destroy", "psst_batch_layout",
    "psst_batch_state_init", "psst_integrate_batch", "psst_batch_poll",
    "psst_batch_describe", "psst_adjoint", "psst_network_grad_size",
    "psst_network_set_tableau", "psst_batch_set_tableau", "psst_network_create_storage",
    "psst_integrate_batch_streamed", "psst_batch_conductance_bytes", "psst_adjoint_noalloc",
    "psst_network_update",
)
STORAGE_AUTO, STORAGE_DENSE, STORAGE_SPARSE = 0, 1, 2


class PsstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"psst {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NeuronParams(C.Structure):
    _fields_ = [("C_m", C.POINTER(C.c_float)), ("g_Na", C.POINTER(C.c_float)),
                ("g_K", C.POINTER(C.c_float)), ("g_L", C.POINTER(C.c_float)),
                ("E_Na", C.POINTER(C.c_float)), ("E_K", C.POINTER(C.c_float)),
                ("E_L", C.POINTER(C.c_float)), ("n_pn", C.c_int32),
                ("area_cm2", C.c_float)]


class Pathway(C.Structure):
    _fields_ = [("type", C.c_int32), ("pre_begin", C.c_int32), ("pre_end", C.c_int32),
                ("post_begin", C.c_int32), ("post_end", C.c_int32),
                ("g_nS", C.POINTER(C.c_float)), ("mask", C.POINTER(C.c_uint8))]


class Tableau(C.Structure):
    _fields_ = [("stages", C.c_int32), ("a", (C.c_double * 4) * 4), ("b", C.c_double * 4)]


def _tableau_struct(tab) -> Optional[Tableau]:
    """psst_tableau from dict(a=[[...]] (stages x stages), b=[...]); None -> NULL."""
    if tab is None:
        return None
    b = [float(x) for x in tab["b"]]
    t = Tableau()
    t.stages = len(b)
    for i, row in enumerate(tab["a"]):
        for q, v in enumerate(row):
            t.a[i][q] = float(v)
    for i, v in enumerate(b):
        t.b[i] = v
    return t


class Kinetics(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("alpha", "beta", "E_rev", "V_p", "K_p", "r1", "r2",
                                         "r3", "r4", "K_d", "hill_n")]


class Stimulus(C.Structure):
    _fields_ = [("i_const_nA", C.c_void_p), ("pulse_ptr", C.c_void_p),
                ("on_step", C.c_void_p), ("off_step", C.c_void_p), ("amp_nA", C.c_void_p)]


class Record(C.Structure):
    _fields_ = [("v_out", C.c_void_p), ("stride", C.c_int64), ("capacity", C.c_int64),
                ("spike_count", C.c_void_p), ("spike_t_ms", C.c_void_p),
                ("spike_cap", C.c_int32)]


_lib = None


def lib():
    """Load libpsst.so (raises PsstError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PsstError(ERR_DEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        sig = {
            "psst_last_error": (C.c_char_p, []),
            "psst_version": (C.c_char_p, []),
            "psst_device_count": (i32, []),
            "psst_network_create": (i32, [C.POINTER(NeuronParams), i32, C.POINTER(Pathway), i32,
                                          C.POINTER(Kinetics), C.POINTER(vp)]),
            "psst_network_destroy": (i32, [vp]),
            "psst_state_layout": (i32, [vp, C.POINTER(i64), C.POINTER(i32)]),
            "psst_state_init": (i32, [vp, vp, vp, vp]),
            "psst_integrate": (i32, [vp, vp, C.POINTER(Stimulus), f32, i64, i64,
                                     C.POINTER(Record), vp]),
            "psst_network_poll": (i32, [vp, vp]),
            "psst_batch_create": (i32, [C.POINTER(vp), i32, C.POINTER(vp)]),
            "psst_batch_destroy": (i32, [vp]),
            "psst_batch_layout": (i32, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
            "psst_batch_state_init": (i32, [vp, vp, vp, vp]),
            "psst_integrate_batch": (i32, [vp, vp, C.POINTER(Stimulus), f32, i64, i64,
                                           C.POINTER(Record), vp, i32, vp]),
            "psst_batch_poll": (i32, [vp, vp]),
            "psst_batch_describe": (i32, [vp, C.c_char_p, i32]),
            "psst_adjoint": (i32, [vp, vp, i32, C.POINTER(Stimulus), f32, i64, i64, vp, vp, vp,
                                   vp, vp, i32, vp]),
            "psst_network_grad_size": (i32, [vp, C.POINTER(i64)]),
            "psst_network_set_tableau": (i32, [vp, C.POINTER(Tableau)]),
            "psst_integrate_batch_streamed": (i32, [vp, vp, C.POINTER(Stimulus), f32, i64, i64,
                                                    i64, i64, vp, vp, vp, i32, vp]),
            "psst_network_create_storage": (i32, [C.POINTER(NeuronParams), i32, C.POINTER(Pathway),
                                                  i32, C.POINTER(Kinetics), i32, C.POINTER(vp)]),
            "psst_batch_set_tableau": (i32, [vp, C.POINTER(Tableau)]),
            "psst_batch_conductance_bytes": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
            "psst_adjoint_noalloc": (i32, [vp, vp, i32, C.POINTER(Stimulus), f32, i64, i64, vp,
                                           vp, vp, vp, vp, i32, vp]),
            "psst_network_update": (i32, [vp, vp, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise PsstError(status, lib().psst_last_error().decode())


def last_error() -> str:
    return lib().psst_last_error().decode()


def version() -> str:
    return lib().psst_version().decode()


def device_count() -> int:
    return int(lib().psst_device_count())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


# ---------------------------------------------------------------------------
# networks
# ---------------------------------------------------------------------------

class Network:
    """Owner of a psst_network handle built from a workload description."""

    def __init__(self, handle, n, n_pn, grad_size, desc):
        self.handle = handle
        self.n = n
        self.n_pn = n_pn
        self.grad_size = grad_size
        self.desc = desc

    def close(self):
        if self.handle:
            _check(lib().psst_network_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def network_create(net, storage: Optional[int] = None) -> Network:
    """psst_network_create (or, with a storage choice,
    psst_network_create_storage) from a workload ``Network`` (host arrays)."""
    keep = []
    vecs = {}
    for k in ("C_m", "g_Na", "g_K", "g_L", "E_Na", "E_K", "E_L"):
        a = np.ascontiguousarray(net.params[k], dtype=np.float32)
        keep.append(a)
        vecs[k] = _fptr(a)
    p = NeuronParams(vecs["C_m"], vecs["g_Na"], vecs["g_K"], vecs["g_L"], vecs["E_Na"],
                     vecs["E_K"], vecs["E_L"], int(net.n_pn), float(net.area_cm2))
    paths = (Pathway * max(len(net.pathways), 1))()
    for q, w in enumerate(net.pathways):
        g = np.ascontiguousarray(w.g_nS, dtype=np.float32)
        m = None if w.mask is None else np.ascontiguousarray(w.mask, dtype=np.uint8)
        keep += [g, m]
        paths[q] = Pathway(int(w.type), int(w.pre_begin), int(w.pre_end), int(w.post_begin),
                           int(w.post_end), _fptr(g),
                           None if m is None else m.ctypes.data_as(C.POINTER(C.c_uint8)))
    kin = (Kinetics * 3)()
    kt = np.asarray(net.kinetics, dtype=np.float32)
    for t in range(3):
        kin[t] = Kinetics(*[float(x) for x in kt[t]])
    h = C.c_void_p()
    if storage is None:
        _check(lib().psst_network_create(C.byref(p), int(net.n), paths, len(net.pathways), kin,
                                         C.byref(h)))
    else:
        _check(lib().psst_network_create_storage(C.byref(p), int(net.n), paths,
                                                 len(net.pathways), kin, int(storage),
                                                 C.byref(h)))
    gs = C.c_int64()
    _check(lib().psst_network_grad_size(h, C.byref(gs)))
    return Network(h, int(net.n), int(net.n_pn), int(gs.value), net)


def network_update(net: Network, g=None, g_na=None, g_k=None, g_l=None, stream=None):
    """psst_network_update: new synaptic blocks (device float32 [grad_size],
    grad_g's layout) and intrinsic conductances (device float32 [n] each)
    written into the network's storage in place; None keeps a part."""
    for t, size, name in ((g, net.grad_size, "g"), (g_na, net.n, "g_na"), (g_k, net.n, "g_k"),
                          (g_l, net.n, "g_l")):
        if t is None:
            continue
        if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4
                and t.is_contiguous() and t.numel() == size):
            raise ValueError(f"{name}: a contiguous float32 device tensor of {size} entries")
    _check(lib().psst_network_update(net.handle, _ptr(g), _ptr(g_na), _ptr(g_k), _ptr(g_l),
                                     _stream(stream)))


def network_destroy(net: Network):
    net.close()


def state_layout(net: Network):
    w, v = C.c_int64(), C.c_int32()
    _check(lib().psst_state_layout(net.handle, C.byref(w), C.byref(v)))
    return int(w.value), int(v.value)


def state_init(net: Network, v0, state, stream=None):
    _check(lib().psst_state_init(net.handle, _ptr(v0), _ptr(state), _stream(stream)))


@dataclass
class DeviceStimulus:
    """Packed device stimulus (torch tensors); any member may be None."""
    i_const_nA: object = None
    pulse_ptr: object = None
    on_step: object = None
    off_step: object = None
    amp_nA: object = None

    def c(self):
        return Stimulus(*(None if t is None else t.data_ptr() for t in
                          (self.i_const_nA, self.pulse_ptr, self.on_step, self.off_step,
                           self.amp_nA)))


@dataclass
class DeviceRecord:
    v_out: object = None
    stride: int = 0
    capacity: int = 0
    spike_count: object = None
    spike_t_ms: object = None
    spike_cap: int = 0

    def c(self):
        return Record(None if self.v_out is None else self.v_out.data_ptr(), int(self.stride),
                      int(self.capacity),
                      None if self.spike_count is None else self.spike_count.data_ptr(),
                      None if self.spike_t_ms is None else self.spike_t_ms.data_ptr(),
                      int(self.spike_cap))


def _stim_ref(stim):
    return None if stim is None else C.byref(stim.c())


def _rec_ref(rec):
    return None if rec is None else C.byref(rec.c())


def integrate(net: Network, state, stim: Optional[DeviceStimulus], dt_ms: float, n_steps: int,
              step0: int = 0, rec: Optional[DeviceRecord] = None, stream=None):
    s = None if stim is None else stim.c()
    r = None if rec is None else rec.c()
    _check(lib().psst_integrate(net.handle, _ptr(state), None if s is None else C.byref(s),
                                float(dt_ms), int(n_steps), int(step0),
                                None if r is None else C.byref(r), _stream(stream)))


def network_poll(net: Network, stream=None):
    _check(lib().psst_network_poll(net.handle, _stream(stream)))


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

class Batch:
    def __init__(self, handle, nets):
        self.handle = handle
        self.nets = list(nets)          # keeps the networks alive
        nt, nw = C.c_int64(), C.c_int64()
        offs = (C.c_int64 * (len(nets) + 1))()
        _check(lib().psst_batch_layout(handle, C.byref(nt), C.byref(nw), offs))
        self.n_total = int(nt.value)
        self.n_words = int(nw.value)
        self.offsets = np.array(offs[:], dtype=np.int64)

    def close(self):
        if self.handle:
            _check(lib().psst_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_create(nets: Sequence[Network]) -> Batch:
    arr = (C.c_void_p * len(nets))(*[n.handle.value if isinstance(n.handle, C.c_void_p)
                                     else n.handle for n in nets])
    h = C.c_void_p()
    _check(lib().psst_batch_create(arr, len(nets), C.byref(h)))
    return Batch(h, nets)


def batch_destroy(batch: Batch):
    batch.close()


def batch_layout(batch: Batch):
    return batch.n_total, batch.n_words, batch.offsets.copy()


def batch_state_init(batch: Batch, v0, states, stream=None):
    _check(lib().psst_batch_state_init(batch.handle, _ptr(v0), _ptr(states), _stream(stream)))


def integrate_batch(batch: Batch, states, stim: Optional[DeviceStimulus], dt_ms: float,
                    n_steps: int, step0: int = 0, rec: Optional[DeviceRecord] = None,
                    checkpoints=None, K: int = 0, stream=None):
    s = None if stim is None else stim.c()
    r = None if rec is None else rec.c()
    _check(lib().psst_integrate_batch(batch.handle, _ptr(states),
                                      None if s is None else C.byref(s), float(dt_ms),
                                      int(n_steps), int(step0),
                                      None if r is None else C.byref(r), _ptr(checkpoints),
                                      int(K), _stream(stream)))


def batch_poll(batch: Batch, stream=None):
    _check(lib().psst_batch_poll(batch.handle, _stream(stream)))


def integrate_batch_streamed(batch: Batch, states, stim: Optional[DeviceStimulus],
                             dt_ms: float, n_steps: int, step0: int, chunk_steps: int,
                             rec_stride: int = 0, host_v: Optional[np.ndarray] = None,
                             host_spike_count: Optional[np.ndarray] = None,
                             host_spike_t: Optional[np.ndarray] = None, spike_cap: int = 0,
                             stream=None):
    """psst_integrate_batch_streamed: records land in host numpy arrays
    (host_v float32 [n_steps // rec_stride, n_total], host_spike_count int32
    [n_total], host_spike_t float32 [n_total, spike_cap]), C-contiguous."""
    for a, dt in ((host_v, np.float32), (host_spike_count, np.int32), (host_spike_t, np.float32)):
        if a is not None and (a.dtype != dt or not a.flags.c_contiguous):
            raise PsstError(ERR_INVALID_ARGUMENT, "host arrays must be C-contiguous of the stated dtype")
    s = None if stim is None else stim.c()
    hp = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    _check(lib().psst_integrate_batch_streamed(
        batch.handle, _ptr(states), None if s is None else C.byref(s), float(dt_ms),
        int(n_steps), int(step0), int(chunk_steps), int(rec_stride), hp(host_v),
        hp(host_spike_count), hp(host_spike_t), int(spike_cap), _stream(stream)))


def network_set_tableau(net: Network, tab=None):
    """Explicit Runge-Kutta method of psst_integrate on this network (and of
    batches created from it); tab = dict(a, b) or None for classical RK4."""
    t = _tableau_struct(tab)
    _check(lib().psst_network_set_tableau(net.handle, None if t is None else C.byref(t)))


def batch_set_tableau(batch: Batch, tab=None):
    t = _tableau_struct(tab)
    _check(lib().psst_batch_set_tableau(batch.handle, None if t is None else C.byref(t)))


def batch_describe(batch: Batch) -> str:
    buf = C.create_string_buffer(4096)
    _check(lib().psst_batch_describe(batch.handle, buf, 4096))
    return buf.value.decode()


def batch_conductance_bytes(batch: Batch):
    """(resident, streamed): conductance bytes a forward launch reads once per
    launch and once per stage evaluation."""
    r, s = C.c_int64(), C.c_int64()
    _check(lib().psst_batch_conductance_bytes(batch.handle, C.byref(r), C.byref(s)))
    return int(r.value), int(s.value)


def adjoint(batch: Batch, checkpoints, K: int, stim: Optional[DeviceStimulus], dt_ms: float,
            n_steps: int, step0: int, dL_dV, grad_g, grad_gNa, grad_gK, grad_gL,
            per_instance: bool, stream=None):
    s = None if stim is None else stim.c()
    _check(lib().psst_adjoint(batch.handle, _ptr(checkpoints), int(K),
                              None if s is None else C.byref(s), float(dt_ms), int(n_steps),
                              int(step0), _ptr(dL_dV), _ptr(grad_g), _ptr(grad_gNa),
                              _ptr(grad_gK), _ptr(grad_gL), int(bool(per_instance)),
                              _stream(stream)))


def adjoint_noalloc(batch: Batch, checkpoints, K: int, stim: Optional[DeviceStimulus],
                    dt_ms: float, n_steps: int, step0: int, dL_dV, grad_g, grad_gNa, grad_gK,
                    grad_gL, per_instance: bool, stream=None):
    """psst_adjoint_noalloc: psst_adjoint with the library's fixed scratch array
    instead of an allocated workspace."""
    s = None if stim is None else stim.c()
    _check(lib().psst_adjoint_noalloc(batch.handle, _ptr(checkpoints), int(K),
                                      None if s is None else C.byref(s), float(dt_ms),
                                      int(n_steps), int(step0), _ptr(dL_dV), _ptr(grad_g),
                                      _ptr(grad_gNa), _ptr(grad_gK), _ptr(grad_gL),
                                      int(bool(per_instance)), _stream(stream)))


# ---------------------------------------------------------------------------
# packing helpers (index bookkeeping only)
# ---------------------------------------------------------------------------

def pack_stimulus(stims: List, device) -> DeviceStimulus:
    """Concatenate per-instance workload stimuli into one packed device
    stimulus (pulse pointers shifted by the pulses of earlier instances)."""
    import torch
    ic = np.concatenate([np.asarray(s.i_const_nA, np.float32) for s in stims])
    have_pulses = any(s.pulse_ptr is not None and int(s.pulse_ptr[-1]) > 0 for s in stims)
    out = DeviceStimulus(torch.from_numpy(ic).to(device))
    if have_pulses:
        ptrs, ons, offs, amps = [np.zeros(1, np.int32)], [], [], []
        base = 0
        for s in stims:
            n = len(s.i_const_nA)
            if s.pulse_ptr is None:
                p = np.zeros(n + 1, np.int32)
            else:
                p = np.asarray(s.pulse_ptr, np.int64)
                ons.append(np.asarray(s.on_step, np.int64))
                offs.append(np.asarray(s.off_step, np.int64))
                amps.append(np.asarray(s.amp_nA, np.float32))
            ptrs.append((p[1:] + base).astype(np.int32))
            base += int(p[-1])
        out.pulse_ptr = torch.from_numpy(np.concatenate(ptrs)).to(device)
        out.on_step = torch.from_numpy(np.concatenate(ons)).to(device)
        out.off_step = torch.from_numpy(np.concatenate(offs)).to(device)
        out.amp_nA = torch.from_numpy(np.concatenate(amps)).to(device)
    return out


def state_planes(state, n_total: int):
    """View a state buffer as [7 vars, 2 words, n_total]."""
    return state.view(N_VARS, 2, n_total)
