"""GPU checks against facts that need no oracle run, through the C ABI:

- transmitter release at the logistic's special values: a presynaptic cell
  clamped at V_p releases at T = 1/2 exactly (at V_p +- K_p ln 3: 3/4, 1/4),
  so its gate follows the RK4 amplification polynomial of a linear ODE
  (closed form, no exponential in the expectation);
- gating variables stay in [0, 1] after every step of coupled networks (the
  exact ODE keeps them there; float32 storage is allowed 1e-6), on the
  per-instance path (a ragged batch including the 120-neuron network with
  slow GABA and pulse trains) and on the per-stage matrix-core path.
"""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R
from tests._pins import (RELEASE_VK, clamped_release_network, gate_closed_form,
                         release_points, slow_gaba_half_closed_form)

pytestmark = pytest.mark.gpu

GATE_SLACK = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _stepwise(inst, dt, n_steps, batched):
    """State after each of n_steps one-step calls, [n_steps, 7, n] float64."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    net = psst.network_create(inst.net)
    n = inst.net.n
    st = torch.zeros(14 * n, dtype=torch.float32, device=dev)
    v0 = torch.from_numpy(inst.v0).to(dev)
    stim = psst.pack_stimulus([inst.stim], dev)
    batch = psst.batch_create([net]) if batched else None
    if batched:
        psst.batch_state_init(batch, v0, st)
    else:
        psst.state_init(net, v0, st)
    out = []
    for s in range(n_steps):
        if batched:
            psst.integrate_batch(batch, st, stim, dt, 1, s)
        else:
            psst.integrate(net, st, stim, dt, 1, s)
        out.append(R.state_value(st.view(7, 2, n).cpu().numpy()))
    if batched:
        psst.batch_poll(batch)
    else:
        psst.network_poll(net)
    return np.array(out)


@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("syn_type", [W.ACH, W.GABA_A])
def test_release_special_values_on_gpu(syn_type, batched):
    for v, T, dT in release_points(syn_type):
        inst, k = clamped_release_network(v, syn_type)
        a, b = k[0], k[1]
        dt = R.step_f32(1.5 / (a * T + b))          # the library takes dt as float32
        ys = _stepwise(inst, dt, 6, batched)
        assert np.all(ys[:, 0, 0] == float(np.float32(v)))     # the clamp holds
        expect = gate_closed_form(a, b, T, dt, 6)
        err = float(np.abs(ys[:, 4, 0] - expect).max())
        _say(f"  type {syn_type} V={v:.4f} T={T}: max |s - closed form| = {err:.2e}")
        # float32-pair storage keeps 48 bits; dT is the clamp voltage's rounding
        assert err <= 1e-12 + 4.0 * dT


@pytest.mark.parametrize("batched", [False, True])
def test_release_slow_gaba_at_half_on_gpu(batched):
    inst, k = clamped_release_network(RELEASE_VK[W.GABA_B][0], W.GABA_B)
    ys = _stepwise(inst, 2.0, 4, batched)
    expect = slow_gaba_half_closed_form(k, 2.0, 4)
    err = float(np.abs(ys[:, 5:7, 0] - expect).max())
    _say(f"  slow GABA at T_B = 1/2: max |(r, G) - closed form| = {err:.2e}")
    assert err <= 1e-12


def _check_bounds(ck, final, nt, kin, gabab_rows):
    """ck: [rows, 14 * nt] checkpoints (state before each step), final: the
    state after the last step.  m, h, n, s in [0, 1]; r in [0, 1] and G in [0,
    r3 / r4] on slow-GABA rows (G' = r3 r - r4 G with r <= 1); 1e-6 slack for
    float32 storage.  Returns the worst excursion found."""
    allst = np.concatenate([ck, final[None, :]], axis=0).reshape(-1, 7, 2, nt)
    y = allst[:, :, 0, :].astype(np.float64) + allst[:, :, 1, :].astype(np.float64)
    assert np.all(np.isfinite(y))
    gates = y[:, 1:5, :]
    worst = max(float(-gates.min()), float(gates.max() - 1.0))
    assert gates.min() >= -GATE_SLACK and gates.max() <= 1.0 + GATE_SLACK
    if gabab_rows.any():
        r = y[:, 5, gabab_rows]
        G = y[:, 6, gabab_rows]
        gmax = float(kin[2, 7]) / float(kin[2, 8])
        assert r.min() >= -GATE_SLACK and r.max() <= 1.0 + GATE_SLACK
        assert G.min() >= -GATE_SLACK and G.max() <= gmax + GATE_SLACK
        assert r.max() > 1e-3                      # the slow pathway was active
    return worst, y


def test_gates_stay_in_unit_interval_every_step_per_instance_path():
    """Every step of 30 ms of a ragged coupled batch: the 120-neuron network
    with fast and slow GABA and pulse trains, and three batched-recipe
    instances (68, 308 and 480 neurons, the largest of the batch recipe)."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    insts = [W.config2(0, t_ms=30.0)] + [W.config3_instance(b) for b in (5, 900, 158)]
    _say("  sizes", [i.net.n for i in insts])
    nets = [psst.network_create(i.net) for i in insts]
    batch = psst.batch_create(nets)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    n = 3000
    ck = torch.zeros((n, 14 * nt), dtype=torch.float32, device=dev)
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    st0 = st.clone()
    psst.integrate_batch(batch, st, stim, 0.01, n, 0, psst.DeviceRecord(None, 0, 0, cnt), ck, 1)
    psst.batch_poll(batch)
    gb = np.zeros(nt, bool)
    a, b = batch.offsets[0], batch.offsets[1]
    gb[a + insts[0].net.n_pn:b] = True            # LN rows of the slow-GABA network
    worst, y = _check_bounds(ck.cpu().numpy(), st.cpu().numpy(), nt, insts[0].net.kinetics, gb)
    spikes = int(cnt.sum())
    _say(f"  {n + 1} states x {nt} neurons: worst gate excursion {worst:.2e}, {spikes} spikes")
    assert spikes > 100                            # gates swung through action potentials
    assert np.array_equal(ck[0].cpu().numpy(), st0.cpu().numpy())   # row 0: initial state


def _slow_gaba_large_network(n_pn=1536, n_ln=512):
    """AL-shaped network above the per-workgroup limit: PN -> LN cholinergic,
    LN -> all fast and slow GABA, each Bernoulli(0.5), g ~ U(0, 0.05) nS;
    constant drive U(0, 2) nA plus a 5 ms pulse of U(1, 10) nA to every
    neuron."""
    rm = W.rng_for(46, 0, W.S_MASK)
    rg = W.rng_for(46, 0, W.S_G)
    n = n_pn + n_ln
    paths = []
    g_, m_ = W._bernoulli_block(rm, rg, (n_ln, n_pn), 0.5, 0.05)
    paths.append(W.Pathway(W.ACH, 0, n_pn, n_pn, n, g_, m_))
    for typ in (W.GABA_A, W.GABA_B):
        g_, m_ = W._bernoulli_block(rm, rg, (n_pn, n_ln), 0.5, 0.05)
        paths.append(W.Pathway(typ, n_pn, n, 0, n_pn, g_, m_))
        g_, m_ = W._bernoulli_block(rm, rg, (n_ln, n_ln), 0.5, 0.05, (0, 0))
        paths.append(W.Pathway(typ, n_pn, n, n_pn, n, g_, m_))
    return W.Network(n, n_pn, W.hh_params(n), paths)


@pytest.mark.parametrize("sparse", [False, True], ids=["dense", "sparse"])
def test_gates_stay_in_unit_interval_every_step_per_stage_path(sparse):
    """Every step of 5 ms of a 2048-neuron network with slow GABA x 4 trials
    on the per-stage path, matrix-core or sparse storage (one-step calls; the
    state after each is copied aside on the device)."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    net = _slow_gaba_large_network()
    T = 4
    i_nA, v0 = W.trial_inputs(46, net.n, T)
    amp = W.rng_for(46, 0, W.S_PULSE).uniform(1.0, 10.0, net.n * T).astype(np.float32)
    h = psst.network_create(net, storage=psst.STORAGE_SPARSE if sparse else None)
    batch = psst.batch_create([h] * T)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), st)
    td = lambda a: torch.from_numpy(a).to(dev)
    stim = psst.DeviceStimulus(td(i_nA.ravel()), td(np.arange(nt + 1, dtype=np.int32)),
                               td(np.zeros(nt, np.int64)), td(np.full(nt, 500, np.int64)),
                               td(amp))
    n = 500
    hist = torch.zeros((n, 14 * nt), dtype=torch.float32, device=dev)
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    hist[0].copy_(st)
    for s in range(n):
        psst.integrate_batch(batch, st, stim, 0.01, 1, s, psst.DeviceRecord(None, 0, 0, cnt))
        if s + 1 < n:
            hist[s + 1].copy_(st)
    psst.batch_poll(batch)
    gb = np.zeros(nt, bool)
    for t in range(T):
        gb[t * net.n + net.n_pn:(t + 1) * net.n] = True
    worst, _ = _check_bounds(hist.cpu().numpy(), st.cpu().numpy(), nt, net.kinetics, gb)
    spikes = int(cnt.sum())
    _say(f"  {n + 1} states x {nt} neurons: worst gate excursion {worst:.2e}, {spikes} spikes")
    assert spikes > 100
