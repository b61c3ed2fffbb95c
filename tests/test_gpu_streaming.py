"""Long runs streamed to host memory (psst_integrate_batch_streamed): the
host arrays drained chunk by chunk match the FP64 oracle (max |dV| <= 1e-3
mV over 50 ms, spike times within 0.05 ms) on a ragged per-instance batch and
on a batch of a large network (per-stage path); the records equal those of
one psst_integrate_batch call bit for bit (V rows, spike counts and times,
final state), for a ragged last chunk and a spike cap that drops spikes;
argument checks."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(insts):
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    nets = [psst.network_create(i.net) for i in insts]
    batch = psst.batch_create(nets)
    nt = batch.n_total
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, v0, st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    return psst, torch, dev, nets, batch, nt, st, stim


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_streamed_ragged_batch_matches_oracle_50ms():
    """A ragged batch (the 120-neuron network with slow GABA and pulse trains,
    and instances of 68, 124, 192 and 480 neurons) streamed to host memory
    over 50 ms in chunks of 700 steps (ragged last chunk), V every 10 steps:
    the host rows against the FP64 oracle, max |dV| <= 1e-3 mV, and every
    spike paired within 0.05 ms."""
    insts = [W.config2(0, t_ms=50.0)] + [W.config3_instance(b) for b in (5, 77, 3, 158)]
    n, chunk, stride, cap = 5000, 700, 10, 64
    psst, torch, dev, nets, batch, nt, st, stim = _setup(insts)
    _say("  streamed ragged batch, sizes", [i.net.n for i in insts])
    hv = np.full((n // stride, nt), np.nan, np.float32)
    hc = np.zeros(nt, np.int32)
    hs = np.zeros((nt, cap), np.float32)
    psst.integrate_batch_streamed(batch, st, stim, 0.01, n, 0, chunk, stride, hv, hc, hs, cap)
    o = R.oracle_run(insts, n, rec_stride=stride, spike_cap=cap)
    dv = float(np.abs(hv.astype(np.float64) - o["v"]).max())
    bad, worst, total = R.spike_match(hc, hs, o["spike_count"], o["spike_t"], 50.0)
    _say(f"  max|dV| {dv:.2e} mV over 50 ms; {total} spikes, {bad} count mismatches, "
         f"worst dt {worst:.2e} ms")
    assert dv <= 1e-3
    assert bad == 0 and worst <= 0.05 and total > 100
    y = R.state_value(st.view(7, 2, nt).cpu().numpy())
    assert np.abs(y[0] - o["state"][0]).max() <= 1e-3


def test_streamed_per_stage_batch_matches_oracle():
    """A 2048-neuron network x 8 trials (per-stage matrix-core path) streamed
    over 600 steps in chunks of 128 (ragged last chunk), V every 4 steps: two
    trials' host rows against the FP64 oracle (max |dV| <= 1e-3 mV, spike
    counts equal)."""
    from paper_1906_03958_amd import psst
    import torch
    dev = torch.device("cuda:0")
    net = W.all_pairs_network(40, 0, 1536, 512, g_max=0.1)
    T = 8
    i_nA, v0 = W.trial_inputs(40, net.n, T)
    insts = [W.Instance(net, v0[t], W.Stimulus(i_nA[t])) for t in range(T)]
    h = psst.network_create(net)
    batch = psst.batch_create([h] * T)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), st)
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    n, chunk, stride, cap = 600, 128, 4, 16
    hv = np.full((n // stride, nt), np.nan, np.float32)
    hc = np.zeros(nt, np.int32)
    hs = np.zeros((nt, cap), np.float32)
    psst.integrate_batch_streamed(batch, st, stim, 0.01, n, 0, chunk, stride, hv, hc, hs, cap)
    pick = [0, 7]
    o = R.oracle_run([insts[t] for t in pick], n, rec_stride=stride, spike_cap=cap, threads=2)
    for k, t in enumerate(pick):
        a, b = t * net.n, (t + 1) * net.n
        oa, ob = k * net.n, (k + 1) * net.n
        dv = float(np.abs(hv[:, a:b].astype(np.float64) - o["v"][:, oa:ob]).max())
        _say(f"  trial {t}: max|dV| {dv:.2e} mV over {n} steps, "
             f"{int(o['spike_count'][oa:ob].sum())} spikes")
        assert dv <= 1e-3
        np.testing.assert_array_equal(hc[a:b], o["spike_count"][oa:ob])
        bad, worst, total = R.spike_match(hc[a:b], hs[a:b], o["spike_count"][oa:ob],
                                          o["spike_t"][oa:ob], n * 0.01)
        assert bad == 0 and worst <= 0.05


@pytest.mark.parametrize("chunk,stride,cap", [(96, 4, 8), (250, 1, 1), (1000, 10, 16)])
def test_streamed_equals_one_call_bitwise(chunk, stride, cap):
    insts = [W.config3_instance(b) for b in (3, 77, 140)] + [W.config2(0, t_ms=20.0)]
    n, step0 = 1000, 40
    psst, torch, dev, nets, batch, nt, st, stim = _setup(insts)
    # one call, records on the device
    st1 = st.clone()
    rows = (step0 + n) // stride - step0 // stride
    v = torch.zeros((rows, nt), dtype=torch.float32, device=dev)
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    spk = torch.zeros((nt, cap), dtype=torch.float32, device=dev)
    psst.integrate_batch(batch, st1, stim, 0.01, n, step0,
                         psst.DeviceRecord(v, stride, rows, cnt, spk, cap))
    psst.batch_poll(batch)
    # streamed to host
    hv = np.zeros((n // stride, nt), np.float32)
    hc = np.zeros(nt, np.int32)
    hs = np.zeros((nt, cap), np.float32)
    psst.integrate_batch_streamed(batch, st, stim, 0.01, n, step0, chunk, stride, hv, hc, hs, cap)
    np.testing.assert_array_equal(hv, v.cpu().numpy())
    np.testing.assert_array_equal(hc, cnt.cpu().numpy())
    np.testing.assert_array_equal(hs, spk.cpu().numpy())
    np.testing.assert_array_equal(st.cpu().numpy(), st1.cpu().numpy())
    if cap == 1:
        assert hc.max() > cap      # the cap dropped spikes and the counts kept them


def test_streamed_argument_checks():
    insts = [W.config1(0)]
    psst, torch, dev, nets, batch, nt, st, stim = _setup(insts)
    hv = np.zeros((10, nt), np.float32)
    for chunk, stride, step0 in ((30, 4, 0), (32, 4, 2), (0, 1, 0)):
        with pytest.raises(psst.PsstError) as e:
            psst.integrate_batch_streamed(batch, st, stim, 0.01, 40, step0, chunk, stride, hv)
        assert e.value.status == psst.ERR_INVALID_ARGUMENT


def test_streamed_per_stage_path_equals_one_call_bitwise():
    """A large shared network (2048 neurons x 8 trials, the per-stage MFMA
    path) streamed in chunks of 64 steps (ragged last chunk) equals one call
    with device records bit for bit."""
    net = W.all_pairs_network(45, 0, 1536, 512, g_max=0.1)
    i_nA, v0 = W.trial_inputs(45, net.n, 8)
    insts = [W.Instance(net, v0[t], W.Stimulus(i_nA[t])) for t in range(8)]
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    h = psst.network_create(net)
    batch = psst.batch_create([h] * 8)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), st)
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    n, stride, cap, chunk = 300, 4, 8, 64
    st1 = st.clone()
    rows = n // stride
    v = torch.zeros((rows, nt), dtype=torch.float32, device=dev)
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    spk = torch.zeros((nt, cap), dtype=torch.float32, device=dev)
    psst.integrate_batch(batch, st1, stim, 0.01, n, 0,
                         psst.DeviceRecord(v, stride, rows, cnt, spk, cap))
    psst.batch_poll(batch)
    hv = np.zeros((rows, nt), np.float32)
    hc = np.zeros(nt, np.int32)
    hs = np.zeros((nt, cap), np.float32)
    psst.integrate_batch_streamed(batch, st, stim, 0.01, n, 0, chunk, stride, hv, hc, hs, cap)
    np.testing.assert_array_equal(hv, v.cpu().numpy())
    np.testing.assert_array_equal(hc, cnt.cpu().numpy())
    np.testing.assert_array_equal(hs, spk.cpu().numpy())
    np.testing.assert_array_equal(st.cpu().numpy(), st1.cpu().numpy())
    assert hc.sum() > 0
