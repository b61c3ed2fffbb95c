"""Seeded synthetic workloads: antennal-lobe-shaped Hodgkin-Huxley networks.

This module only draws inputs.  It holds none of the method's arithmetic (no
rate functions, no unit conversion, no integration): both the HIP path and the
FP64 oracle consume the arrays it returns, each doing its own arithmetic.

Every value is rounded to float32 so that the oracle's widening to float64 is
exact and both sides start from identical inputs.  Each quantity of instance
``b`` of workload ``cfg`` comes from its own generator,
``numpy.random.default_rng(SeedSequence([cfg, b, stream]))``, so an instance is
the same whether it is generated alone or inside a batch of thousands.

Units are those of the library's API: mV, ms, nS, nA, uF/cm^2, mS/cm^2.

Network shape (paper, "Brain simulations as computational graphs": state
vector [V, m, n, h] per neuron with per-neuron parameter vectors; "Circumventing
memory constraints": synaptic variables as an n x n matrix): neurons are
ordered projection neurons (PN, excitatory, cholinergic) first, then local
neurons (LN, inhibitory, GABAergic).  A pathway is a dense masked block
``g[post, pre]`` of one synapse type.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

ACH, GABA_A, GABA_B = 0, 1, 2
TYPE_NAMES = {ACH: "ACh", GABA_A: "GABA_A", GABA_B: "GABA_B"}

#: kinetics table columns (one row per synapse type ACh, GABA_A, GABA_B)
KIN_FIELDS = ("alpha", "beta", "E_rev", "V_p", "K_p",
              "r1", "r2", "r3", "r4", "K_d", "hill_n")

# Textbook squid-axon values in the -65 mV convention (Hodgkin & Huxley 1952);
# the paper names the parameters C_m, g_K, ..., E_L but prints no values.
HH_DEFAULTS = dict(C_m=1.0, g_Na=120.0, g_K=36.0, g_L=0.3,
                   E_Na=50.0, E_K=-77.0, E_L=-54.387)
PARAM_NAMES = ("C_m", "g_Na", "g_K", "g_L", "E_Na", "E_K", "E_L")

# First-order transmitter kinetics and two-variable G-protein kinetics.  The
# paper is silent on these; the values are free parameters in the range of
# published kinetic synapse models.  E_rev of ACh (0 mV) and fast GABA (-70 mV)
# are the workload's stated reversal potentials.
DEFAULT_KINETICS = np.array([
    # alpha  beta   E_rev  V_p  K_p  r1   r2      r3   r4     K_d    n
    [10.0,  0.2,    0.0,  2.0, 5.0, 0.0, 0.0,    0.0, 0.0,    1.0,  1.0],  # ACh
    [10.0,  0.16, -70.0,  2.0, 5.0, 0.0, 0.0,    0.0, 0.0,    1.0,  1.0],  # GABA_A
    [0.0,   0.0,  -95.0,  2.0, 5.0, 0.5, 0.0013, 0.1, 0.033, 100.0, 4.0],  # GABA_B
], dtype=np.float32)

AREA_CM2 = 1e-4   # single-compartment membrane area used for nS/nA -> densities

DT_MS = 0.01


def _f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def rng_for(cfg: int, instance: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, instance, stream]))


# streams
S_SIZE, S_MASK, S_G, S_STIM, S_V0, S_JITTER, S_PULSE = range(7)


@dataclass
class Pathway:
    type: int
    pre_begin: int
    pre_end: int
    post_begin: int
    post_end: int
    g_nS: np.ndarray          # float32 [post x pre], zero where mask == 0
    mask: np.ndarray          # uint8  [post x pre]

    @property
    def shape(self):
        return (self.post_end - self.post_begin, self.pre_end - self.pre_begin)


@dataclass
class Network:
    n: int
    n_pn: int
    params: dict              # name -> float32 [n]
    pathways: List[Pathway]
    kinetics: np.ndarray = field(default_factory=lambda: DEFAULT_KINETICS.copy())
    area_cm2: float = AREA_CM2

    @property
    def n_ln(self) -> int:
        return self.n - self.n_pn

    @property
    def cell_type(self) -> np.ndarray:
        t = np.zeros(self.n, dtype=np.uint8)
        t[self.n_pn:] = 1
        return t

    @property
    def has_gabab(self) -> bool:
        return any(p.type == GABA_B for p in self.pathways)

    def param_matrix(self) -> np.ndarray:
        return np.stack([self.params[k] for k in PARAM_NAMES]).astype(np.float32)


@dataclass
class Stimulus:
    """Injected current in nA: a constant per neuron plus per-neuron pulses.

    Pulses are grouped by neuron (CSR): neuron i owns pulses
    ``pulse_ptr[i]:pulse_ptr[i+1]``; a pulse is on for global steps
    ``on_step <= g < off_step``.
    """
    i_const_nA: np.ndarray            # float32 [n]
    pulse_ptr: Optional[np.ndarray] = None   # int32 [n+1]
    on_step: Optional[np.ndarray] = None     # int64 [P]
    off_step: Optional[np.ndarray] = None    # int64 [P]
    amp_nA: Optional[np.ndarray] = None      # float32 [P]

    @property
    def n_pulses(self) -> int:
        return 0 if self.pulse_ptr is None else int(self.pulse_ptr[-1])


@dataclass
class Instance:
    net: Network
    v0: np.ndarray                    # float32 [n]
    stim: Stimulus


def hh_params(n: int) -> dict:
    return {k: np.full(n, v, dtype=np.float32) for k, v in HH_DEFAULTS.items()}


def _bernoulli_block(rng_mask, rng_g, shape, p, g_max, no_autapse_offset=None,
                     scale=1.0):
    """Dense masked block: mask ~ Bernoulli(p), g ~ U(0, g_max) * scale."""
    mask = (rng_mask.random(shape) < p).astype(np.uint8)
    if no_autapse_offset is not None:
        # block rows are post (post_begin + r), columns pre (pre_begin + c);
        # the autapse sits where post index == pre index.
        r0, c0 = no_autapse_offset
        rows = np.arange(shape[0]) + r0
        cols = rows - c0
        ok = (cols >= 0) & (cols < shape[1])
        mask[rows[ok] - r0, cols[ok]] = 0
    g = rng_g.uniform(0.0, g_max, shape) * scale
    g = np.where(mask != 0, g, 0.0)
    return _f32(g), mask


def all_pairs_network(cfg: int, instance: int, n_pn: int, n_ln: int,
                      g_max: float = 0.5, p: float = 0.5,
                      g_scale: float = 1.0) -> Network:
    """Every ordered pair i != j is a Bernoulli(p) candidate; the presynaptic
    cell type sets the synapse (PN -> ACh, LN -> fast GABA)."""
    n = n_pn + n_ln
    rm = rng_for(cfg, instance, S_MASK)
    rg = rng_for(cfg, instance, S_G)
    paths = []
    g, m = _bernoulli_block(rm, rg, (n, n_pn), p, g_max, (0, 0), g_scale)
    paths.append(Pathway(ACH, 0, n_pn, 0, n, g, m))
    g, m = _bernoulli_block(rm, rg, (n, n_ln), p, g_max, (0, n_pn), g_scale)
    paths.append(Pathway(GABA_A, n_pn, n, 0, n, g, m))
    return Network(n, n_pn, hh_params(n), paths)


def _const_stim(cfg, instance, n, lo=0.0, hi=2.0) -> Stimulus:
    r = rng_for(cfg, instance, S_STIM)
    return Stimulus(_f32(r.uniform(lo, hi, n)))


def _v0(cfg, instance, n) -> np.ndarray:
    return _f32(rng_for(cfg, instance, S_V0).uniform(-70.0, -60.0, n))


def sized_instance(instance: int, n_pn: int, n_ln: int) -> Instance:
    """A network of any size built with the config-1 recipe (all ordered
    pairs Bernoulli(0.5), g ~ U(0, 0.5) nS, I ~ U(0, 2) nA, V0 ~ U(-70, -60)
    mV), seeded by (9, instance): sizes at the kernels' boundaries.  A cell
    type with no neurons contributes no pathway."""
    cfg = 9
    net = all_pairs_network(cfg, instance, n_pn, n_ln)
    net.pathways = [w for w in net.pathways if w.pre_end > w.pre_begin and w.post_end > w.post_begin]
    return Instance(net, _v0(cfg, instance, net.n), _const_stim(cfg, instance, net.n))


def sized_instance_slow(instance: int, n_pn: int, n_ln: int) -> Instance:
    """sized_instance with slow GABA added: every LN -> any pair is also a
    Bernoulli(0.5) candidate for a G-protein synapse, g ~ U(0, 0.5) nS (its
    own mask and values; seeded by (10, instance))."""
    base = sized_instance(instance, n_pn, n_ln)
    n = n_pn + n_ln
    if n_ln > 0:
        rm = rng_for(10, instance, S_MASK)
        rg = rng_for(10, instance, S_G)
        g, m = _bernoulli_block(rm, rg, (n, n_ln), 0.5, 0.5, (0, n_pn))
        base.net.pathways.append(Pathway(GABA_B, n_pn, n, 0, n, g, m))
    return base


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def config1(seed: int = 0) -> Instance:
    """20 neurons (15 PN, 5 LN), ACh + fast GABA, Bernoulli(0.5), g ~ U(0,0.5) nS,
    constant current U(0,2) nA, V0 ~ U(-70,-60) mV; 100 ms at dt = 0.01 ms."""
    cfg = 1
    net = all_pairs_network(cfg, seed, 15, 5)
    return Instance(net, _v0(cfg, seed, net.n), _const_stim(cfg, seed, net.n))


CONFIG1_STEPS = 10_000


def config2(seed: int = 0, t_ms: float = 1000.0) -> Instance:
    """Antennal-lobe-shaped network: 90 PN + 30 LN.

    Pathways (each Bernoulli(0.5), g ~ U(0, 0.5) nS): PN->LN cholinergic;
    LN->PN and LN->LN fast GABA; LN->PN and LN->LN slow GABA (G-protein).
    Stimulus: a random 33% of the neurons (40 of 120) receive a train of
    100 ms current pulses (100 ms on, 100 ms off, from t = 0 to the end of the
    run) with a per-neuron amplitude U(1, 10) nA.
    """
    cfg = 2
    n_pn, n_ln = 90, 30
    n = n_pn + n_ln
    rm = rng_for(cfg, seed, S_MASK)
    rg = rng_for(cfg, seed, S_G)
    paths = []
    g, m = _bernoulli_block(rm, rg, (n_ln, n_pn), 0.5, 0.5)
    paths.append(Pathway(ACH, 0, n_pn, n_pn, n, g, m))
    for typ in (GABA_A, GABA_B):
        g, m = _bernoulli_block(rm, rg, (n_pn, n_ln), 0.5, 0.5)
        paths.append(Pathway(typ, n_pn, n, 0, n_pn, g, m))
        g, m = _bernoulli_block(rm, rg, (n_ln, n_ln), 0.5, 0.5, (0, 0))
        paths.append(Pathway(typ, n_pn, n, n_pn, n, g, m))
    net = Network(n, n_pn, hh_params(n), paths)
    rs = rng_for(cfg, seed, S_PULSE)
    chosen = np.sort(rs.choice(n, size=40, replace=False))
    amp = _f32(rs.uniform(1.0, 10.0, 40))
    period = int(round(100.0 / DT_MS))
    n_steps = int(round(t_ms / DT_MS))
    ptr = np.zeros(n + 1, dtype=np.int32)
    ons, offs, amps = [], [], []
    k = 0
    for i in range(n):
        if k < len(chosen) and chosen[k] == i:
            for s in range(0, n_steps, 2 * period):
                ons.append(s)
                offs.append(min(s + period, n_steps))
                amps.append(amp[k])
            k += 1
        ptr[i + 1] = len(ons)
    stim = Stimulus(np.zeros(n, dtype=np.float32), ptr,
                    np.asarray(ons, dtype=np.int64),
                    np.asarray(offs, dtype=np.int64),
                    _f32(amps))
    return Instance(net, _v0(cfg, seed, n), stim)


CONFIG2_STEPS = 100_000


def config3_size(b: int) -> int:
    """Size of batched instance b: N = 4k, k ~ U{15..120} (60..480 neurons,
    PN:LN = 3:1)."""
    k = int(rng_for(3, b, S_SIZE).integers(15, 121))
    return 4 * k


def config3_instance(b: int) -> Instance:
    """Instance b of the batched workload: the config-1 recipe at its own size,
    with one conductance jitter x_b ~ LogNormal(0, 0.1) scaling all its g."""
    cfg = 3
    n = config3_size(b)
    k = n // 4
    x = float(rng_for(cfg, b, S_JITTER).lognormal(0.0, 0.1))
    net = all_pairs_network(cfg, b, 3 * k, k, g_scale=x)
    return Instance(net, _v0(cfg, b, n), _const_stim(cfg, b, n))


def config3(n_instances: int = 4096, first: int = 0) -> List[Instance]:
    return [config3_instance(b) for b in range(first, first + n_instances)]


def config3_sparse_instance(b: int, p: float = 0.1) -> Instance:
    """Instance b of the sparse batched workload: the batched recipe's size,
    jitter, stimulus and V0 with connection probability p and g ~ U(0, 0.25 /
    p) nS, so the expected conductance onto a neuron matches the p = 0.5
    recipe (its own generator streams: workload id 6)."""
    cfg = 6
    n = config3_size(b)
    k = n // 4
    x = float(rng_for(cfg, b, S_JITTER).lognormal(0.0, 0.1))
    net = all_pairs_network(cfg, b, 3 * k, k, g_max=0.25 / p, p=p, g_scale=x)
    return Instance(net, _v0(cfg, b, n), _const_stim(cfg, b, n))


def config3_sparse(n_instances: int = 4096, p: float = 0.1, first: int = 0) -> List[Instance]:
    return [config3_sparse_instance(b, p) for b in range(first, first + n_instances)]


def config3_uncoupled(n_instances: int = 4096, first: int = 0) -> List[Instance]:
    """The batched workload with every synapse removed (independent neurons,
    the compute-only counterpart): instance b keeps its size, neuron
    parameters, stimulus and V0."""
    cfg = 3
    out = []
    for b in range(first, first + n_instances):
        n = config3_size(b)
        net = Network(n, 3 * (n // 4), hh_params(n), [])
        out.append(Instance(net, _v0(cfg, b, n), _const_stim(cfg, b, n)))
    return out


# Butcher tableaux of explicit Runge-Kutta methods (a strictly lower
# triangular, rows = stages; b = weights) and their classical orders.  Inputs
# for both the library and the oracle, like the kinetic constants.
TABLEAUX = {
    "euler": dict(a=[[0.0]], b=[1.0]),
    "midpoint": dict(a=[[0.0, 0.0], [0.5, 0.0]], b=[0.0, 1.0]),
    "heun": dict(a=[[0.0, 0.0], [1.0, 0.0]], b=[0.5, 0.5]),
    "ralston": dict(a=[[0.0, 0.0], [2.0 / 3.0, 0.0]], b=[0.25, 0.75]),
    "kutta3": dict(a=[[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [-1.0, 2.0, 0.0]],
                   b=[1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0]),
    "ssprk3": dict(a=[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.0]],
                   b=[1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0]),
    "rk4": dict(a=[[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0],
                   [0.0, 0.0, 1.0, 0.0]],
                b=[1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]),
    "rk38": dict(a=[[0.0, 0.0, 0.0, 0.0], [1.0 / 3.0, 0.0, 0.0, 0.0],
                    [-1.0 / 3.0, 1.0, 0.0, 0.0], [1.0, -1.0, 1.0, 0.0]],
                 b=[0.125, 0.375, 0.375, 0.125]),
}
TABLEAU_ORDER = {"euler": 1, "midpoint": 2, "heun": 2, "ralston": 2, "kutta3": 3,
                 "ssprk3": 3, "rk4": 4, "rk38": 4}


CONFIG3_INSTANCES = 4096
CONFIG3_STEPS = 50_000


def config4_network(n_pn: int = 12288, n_ln: int = 4096, chunk_rows: int = 1024,
                    p: float = 0.5, g_max: float = 0.1) -> Network:
    """Large network: Bernoulli(p) mask, g ~ U(0, g_max) nS, no autapses
    (default: the dense p = 0.5, g_max = 0.1 network).

    Generated in row chunks so the float64 temporaries stay small; each chunk
    has its own generator (stream id offset by the chunk index); a density
    other than 0.5 draws from workload id 12."""
    cfg = 4 if p == 0.5 else 12
    n = n_pn + n_ln
    g_ach = np.empty((n, n_pn), np.float32)
    m_ach = np.empty((n, n_pn), np.uint8)
    g_gab = np.empty((n, n_ln), np.float32)
    m_gab = np.empty((n, n_ln), np.uint8)
    for c, r0 in enumerate(range(0, n, chunk_rows)):
        r1 = min(n, r0 + chunk_rows)
        rm = rng_for(cfg, 0, 100 + 2 * c)
        rg = rng_for(cfg, 0, 101 + 2 * c)
        g, m = _bernoulli_block(rm, rg, (r1 - r0, n_pn), p, g_max, (r0, 0))
        g_ach[r0:r1], m_ach[r0:r1] = g, m
        g, m = _bernoulli_block(rm, rg, (r1 - r0, n_ln), p, g_max, (r0, n_pn))
        g_gab[r0:r1], m_gab[r0:r1] = g, m
    paths = [Pathway(ACH, 0, n_pn, 0, n, g_ach, m_ach),
             Pathway(GABA_A, n_pn, n, 0, n, g_gab, m_gab)]
    return Network(n, n_pn, hh_params(n), paths)


def trial_inputs(cfg: int, n: int, n_trials: int, first: int = 0):
    """Per-trial constant current U(0,2) nA and V0 ~ U(-70,-60) mV, [B, n]."""
    i = np.stack([_const_stim(cfg, 1000 + t, n).i_const_nA
                  for t in range(first, first + n_trials)])
    v = np.stack([_v0(cfg, 1000 + t, n) for t in range(first, first + n_trials)])
    return i, v


CONFIG4_TRIALS = 64
CONFIG4_STEPS = 20_000


def config5(n_trials: int = 256, first_trial: int = 0):
    """Adjoint workload: trials of the 120-neuron config-1 physics network
    (90 PN + 30 LN, all pairs Bernoulli(0.5), ACh + fast GABA).

    Returns ``(net_hidden, net_eval, i_nA [B,n], v0 [B,n])``: ``net_hidden``
    holds the hidden conductances g* that generate the target traces,
    ``net_eval`` the point g = g* * x (x ~ LogNormal(0, 0.1) per synapse and per
    neuron for g_Na, g_K, g_L) at which gradients are evaluated.
    """
    cfg = 5
    hidden = all_pairs_network(cfg, 0, 90, 30)
    rj = rng_for(cfg, 0, S_JITTER)
    paths = []
    for p in hidden.pathways:
        x = rj.lognormal(0.0, 0.1, p.g_nS.shape)
        g = _f32(np.where(p.mask != 0, p.g_nS.astype(np.float64) * x, 0.0))
        paths.append(Pathway(p.type, p.pre_begin, p.pre_end, p.post_begin,
                             p.post_end, g, p.mask.copy()))
    params = {k: v.copy() for k, v in hidden.params.items()}
    for k in ("g_Na", "g_K", "g_L"):
        params[k] = _f32(params[k].astype(np.float64) *
                         rj.lognormal(0.0, 0.1, hidden.n))
    ev = Network(hidden.n, hidden.n_pn, params, paths)
    i, v = trial_inputs(cfg, hidden.n, n_trials, first_trial)
    return hidden, ev, i, v


CONFIG5_TRIALS = 256
CONFIG5_STEPS = 20_000
CONFIG5_CHECKPOINT = 100


def single_neuron(i_nA: float = 0.0, params: Optional[dict] = None,
                  v0: float = -65.0) -> Instance:
    """One uncoupled neuron (pins and edge cases)."""
    pr = hh_params(1)
    if params:
        for k, v in params.items():
            pr[k] = _f32([v])
    net = Network(1, 1, pr, [])
    return Instance(net, _f32([v0]), Stimulus(_f32([i_nA])))


def uncoupled(i_nA: np.ndarray, v0: np.ndarray, params: Optional[dict] = None
              ) -> Instance:
    """n independent neurons (no pathways), e.g. a current sweep."""
    n = len(i_nA)
    pr = hh_params(n)
    if params:
        for k, v in params.items():
            pr[k] = _f32(np.broadcast_to(v, (n,)))
    return Instance(Network(n, n, pr, []), _f32(v0), Stimulus(_f32(i_nA)))
