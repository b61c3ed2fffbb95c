"""FP64 CPU oracle for RK4 integration of coupled Hodgkin-Huxley networks.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its binding) never imports this package, and this package imports nothing from
the product.  Inputs arrive as plain arrays or duck-typed objects with the
generator's field names; every float32 input is widened to float64 exactly.
The step dt is used as given: a caller comparing with a float32 integrator
passes the float32 value of its step.

Functions follow the paper's statement of the method: the initial value problem
and the fourth-order Runge-Kutta step ("Brain simulations as computational
graphs"), structure-of-arrays state with per-neuron parameter vectors (the
vectorisation paragraph), a dense conductance matrix per synapse type
("Circumventing memory constraints", item 1), scan output rows that exclude the
initial value (the tf.scan cumulative-sum example).  The C source lists the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psst_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A separately built copy of the same source (the sanitizer test builds one
# with address and undefined-behaviour checks) is loaded instead when named
# here; it is used as is, never rebuilt.
_LIB_OVERRIDE = os.environ.get("PSST_ORACLE_LIB")

NVAR = 7
VAR_NAMES = ("V", "m", "h", "n", "s", "r", "G")
PARAM_NAMES = ("C_m", "g_Na", "g_K", "g_L", "E_Na", "E_K", "E_L")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _LIB


class _Net(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_pn", C.c_int32),
                ("prm", C.POINTER(C.c_double)),
                ("n_path", C.c_int32),
                ("pinfo", C.POINTER(C.c_int32)),
                ("g", C.POINTER(C.c_double)),
                ("kin", C.POINTER(C.c_double)),
                ("area_cm2", C.c_double)]


class _Stim(C.Structure):
    _fields_ = [("i_const", C.POINTER(C.c_double)),
                ("pulse_ptr", C.POINTER(C.c_int32)),
                ("on_step", C.POINTER(C.c_int64)),
                ("off_step", C.POINTER(C.c_int64)),
                ("amp", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
        dp, ip32, ip64 = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.or_exprel.restype = C.c_double
        L.or_exprel.argtypes = [C.c_double]
        L.or_exprel_d.restype = C.c_double
        L.or_exprel_d.argtypes = [C.c_double]
        L.or_rates.argtypes = [C.c_double, dp]
        L.or_rhs.argtypes = [C.POINTER(_Net), dp, dp, dp]
        L.or_init.argtypes = [C.POINTER(_Net), dp, dp]
        L.or_integrate.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                   C.c_int64, C.c_int64, C.c_int64, C.c_int64, dp,
                                   C.c_int32, ip32, dp]
        L.or_integrate_euler.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                         C.c_int64, C.c_int64, C.c_int64, C.c_int64, dp]
        L.or_integrate_persyn.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                          C.c_int64, C.c_int64, dp]
        L.or_adjoint.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                 C.c_int64, C.c_int64, dp, dp, dp, dp, dp, dp]
        L.or_step_vjp.argtypes = [C.POINTER(_Net), dp, dp, C.c_double, dp, dp]
        L.or_integrate_tab.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                       C.c_int64, C.c_int64, C.c_int64, C.c_int64, dp,
                                       C.c_int32, C.POINTER(C.c_int32), dp, C.c_int32, dp, dp]
        L.or_adjoint_tab.argtypes = [C.POINTER(_Net), dp, C.POINTER(_Stim), C.c_double,
                                     C.c_int64, C.c_int64, dp, dp, dp, dp, dp, dp,
                                     C.c_int32, dp, dp]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).astype(np.float64))


class OracleNet:
    """float64 copy of a network description (keeps the arrays alive)."""

    def __init__(self, net):
        self.n = int(net.n)
        self.n_pn = int(net.n_pn)
        self.prm = np.ascontiguousarray(
            np.stack([_f64(net.params[k]) for k in PARAM_NAMES]))
        self.pinfo = np.ascontiguousarray(np.array(
            [[p.type, p.pre_begin, p.pre_end, p.post_begin, p.post_end]
             for p in net.pathways], dtype=np.int32).reshape(-1, 5))
        blocks = [_f64(p.g_nS).ravel() for p in net.pathways]
        self.g = np.ascontiguousarray(np.concatenate(blocks) if blocks else np.zeros(1))
        self.mask = (np.concatenate([np.asarray(p.mask).ravel() for p in net.pathways])
                     if blocks else np.zeros(1, np.uint8))
        self.block_shapes = [(p.post_end - p.post_begin, p.pre_end - p.pre_begin)
                             for p in net.pathways]
        self.kin = np.ascontiguousarray(_f64(net.kinetics))
        self.area = float(np.float32(net.area_cm2))   # the API takes area as float32
        self.c = _Net(self.n, self.n_pn, _dptr(self.prm), len(net.pathways),
                      self.pinfo.ctypes.data_as(C.POINTER(C.c_int32)),
                      _dptr(self.g), _dptr(self.kin), self.area)

    def with_params(self, prm=None, g=None):
        """Copy with replaced float64 parameter matrix and/or packed g."""
        o = object.__new__(OracleNet)
        o.__dict__.update(self.__dict__)
        o.prm = np.ascontiguousarray(self.prm if prm is None else prm, dtype=np.float64)
        o.g = np.ascontiguousarray(self.g if g is None else g, dtype=np.float64)
        o.c = _Net(o.n, o.n_pn, _dptr(o.prm), self.c.n_path, self.c.pinfo,
                   _dptr(o.g), _dptr(o.kin), o.area)
        return o

    def split_blocks(self, packed):
        out, off = [], 0
        for (a, b) in self.block_shapes:
            out.append(packed[off:off + a * b].reshape(a, b))
            off += a * b
        return out


class OracleStim:
    def __init__(self, stim, n):
        self.i_const = _f64(stim.i_const_nA) if stim.i_const_nA is not None else np.zeros(n)
        self._keep = []
        if stim.pulse_ptr is not None and int(stim.pulse_ptr[-1]) > 0:
            self.ptr = np.ascontiguousarray(stim.pulse_ptr, dtype=np.int32)
            self.on = np.ascontiguousarray(stim.on_step, dtype=np.int64)
            self.off = np.ascontiguousarray(stim.off_step, dtype=np.int64)
            self.amp = _f64(stim.amp_nA)
            self.c = _Stim(_dptr(self.i_const), self.ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                           self.on.ctypes.data_as(C.POINTER(C.c_int64)),
                           self.off.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(self.amp))
        else:
            self.c = _Stim(_dptr(self.i_const), None, None, None, None)


def _as_net(net):
    return net if isinstance(net, OracleNet) else OracleNet(net)


def _as_stim(stim, n):
    return stim if isinstance(stim, OracleStim) else OracleStim(stim, n)


# ---------------------------------------------------------------------------

def exprel(u: float) -> float:
    return lib().or_exprel(float(u))


def rates(V: float) -> np.ndarray:
    out = np.zeros(6)
    lib().or_rates(float(V), _dptr(out))
    return out


def init_state(net, v0) -> np.ndarray:
    """Initial state [7, n]: gates at steady state for V0, synapses at 0."""
    on = _as_net(net)
    y = np.zeros((NVAR, on.n))
    v = _f64(v0)
    lib().or_init(C.byref(on.c), _dptr(v), _dptr(y))
    return y


def rhs(net, y, i_nA) -> np.ndarray:
    on = _as_net(net)
    y = np.ascontiguousarray(y, dtype=np.float64)
    i = np.ascontiguousarray(i_nA, dtype=np.float64)
    f = np.zeros_like(y)
    lib().or_rhs(C.byref(on.c), _dptr(y), _dptr(i), _dptr(f))
    return f


def _tableau(tab):
    """(stages, a[4][4] row-major, b[4]) as float64 arrays from a tableau
    given as dict(a=[[...]], b=[...]) (explicit: a strictly lower triangular)."""
    b = np.asarray(tab["b"], np.float64)
    s = len(b)
    a = np.zeros((4, 4))
    a[:s, :s] = np.asarray(tab["a"], np.float64).reshape(s, s)
    bb = np.zeros(4)
    bb[:s] = b
    return s, np.ascontiguousarray(a.ravel()), bb


def integrate(net, y, stim, dt, n_steps, step0=0, rec_stride=1, rec_cap=None,
              spike_cap=0, euler=False, tableau=None):
    """Advance state y ([7, n] float64, modified in place) by n_steps of RK4
    (or forward Euler, or the explicit method `tableau` = dict(a, b)).

    Returns dict(v=[rows, n] recorded potentials after each stride-th global
    step, spike_count=[n], spike_t=[n, spike_cap] in ms).
    """
    on = _as_net(net)
    st = _as_stim(stim, on.n)
    assert y.dtype == np.float64 and y.flags.c_contiguous and y.shape == (NVAR, on.n)
    if rec_cap is None:
        rec_cap = (step0 + n_steps) // rec_stride - step0 // rec_stride if rec_stride > 0 else 0
    v = np.zeros((max(rec_cap, 1), on.n))
    cnt = np.zeros(on.n, np.int32)
    spk = np.zeros((on.n, max(spike_cap, 1)))
    if tableau is not None:
        s, a, b = _tableau(tableau)
        rc = lib().or_integrate_tab(C.byref(on.c), _dptr(y), C.byref(st.c), float(dt),
                                    int(n_steps), int(step0), int(rec_stride), int(rec_cap),
                                    _dptr(v), int(spike_cap),
                                    cnt.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(spk),
                                    int(s), _dptr(a), _dptr(b))
        if rc != 0:
            raise ValueError("tableau needs 1 to 4 stages")
    elif euler:
        lib().or_integrate_euler(C.byref(on.c), _dptr(y), C.byref(st.c), float(dt),
                                 int(n_steps), int(step0), int(rec_stride), int(rec_cap),
                                 _dptr(v))
    else:
        lib().or_integrate(C.byref(on.c), _dptr(y), C.byref(st.c), float(dt), int(n_steps),
                           int(step0), int(rec_stride), int(rec_cap), _dptr(v),
                           int(spike_cap), cnt.ctypes.data_as(C.POINTER(C.c_int32)),
                           _dptr(spk))
    return dict(v=v[:rec_cap], spike_count=cnt, spike_t=spk[:, :spike_cap])


def integrate_persyn(net, y, stim, dt, n_steps, step0=0):
    """Per-synapse-gate form (first-order synapses only); returns V rows."""
    on = _as_net(net)
    st = _as_stim(stim, on.n)
    v = np.zeros((n_steps, on.n))
    rc = lib().or_integrate_persyn(C.byref(on.c), _dptr(y), C.byref(st.c), float(dt),
                                   int(n_steps), int(step0), _dptr(v))
    if rc != 0:
        raise ValueError("per-synapse form supports first-order synapses only")
    return v


def run(inst, n_steps, dt=0.01, rec_stride=1, spike_cap=0, step0=0, tableau=None):
    """Initial state from inst.v0, then integrate; returns (result, final y)."""
    on = OracleNet(inst.net)
    y = init_state(on, inst.v0)
    res = integrate(on, y, inst.stim, dt, n_steps, step0, rec_stride,
                    spike_cap=spike_cap, tableau=tableau)
    return res, y


def adjoint(net, y0, stim, dt, n_steps, dLdV, step0=0, tableau=None):
    """Discrete adjoint of the RK4 map.  dLdV: [n_steps, n] (dL/dV after each
    step).  Returns dict(g=[packed pathway blocks, nS], g_Na, g_K, g_L [n],
    lambda0 [7, n])."""
    on = _as_net(net)
    st = _as_stim(stim, on.n)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    d = np.ascontiguousarray(dLdV, dtype=np.float64)
    assert d.shape == (n_steps, on.n)
    gg = np.zeros(max(on.g.size, 1))
    gna, gk, gl = np.zeros(on.n), np.zeros(on.n), np.zeros(on.n)
    lam = np.zeros((NVAR, on.n))
    if tableau is None:
        lib().or_adjoint(C.byref(on.c), _dptr(y0), C.byref(st.c), float(dt), int(n_steps),
                         int(step0), _dptr(d), _dptr(gg), _dptr(gna), _dptr(gk), _dptr(gl),
                         _dptr(lam))
    else:
        s, a, b = _tableau(tableau)
        lib().or_adjoint_tab(C.byref(on.c), _dptr(y0), C.byref(st.c), float(dt),
                             int(n_steps), int(step0), _dptr(d), _dptr(gg), _dptr(gna),
                             _dptr(gk), _dptr(gl), _dptr(lam), int(s), _dptr(a), _dptr(b))
    # only existing synapses are parameters: zero where the mask is 0
    g = np.where(on.mask[:on.g.size] != 0, gg[:on.g.size], 0.0)
    return dict(g=g, g_Na=gna, g_K=gk, g_L=gl, lambda0=lam)


def step_vjp(net, yn, i_nA, dt, lam):
    on = _as_net(net)
    yn = np.ascontiguousarray(yn, dtype=np.float64)
    i = np.ascontiguousarray(i_nA, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros_like(lam)
    lib().or_step_vjp(C.byref(on.c), _dptr(yn), _dptr(i), float(dt), _dptr(lam), _dptr(out))
    return out


def run_many(insts, n_steps, dt=0.01, rec_stride=0, spike_cap=0, threads=None, tableau=None):
    """Independent instances in parallel threads (ctypes releases the GIL)."""
    threads = threads or os.cpu_count() or 1

    def one(inst):
        return run(inst, n_steps, dt, rec_stride=rec_stride, spike_cap=spike_cap,
                   tableau=tableau)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, insts))
