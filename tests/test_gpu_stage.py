"""GPU parity of the per-stage path (networks above 1024 neurons, shared by
many trials; float32 matrix-core GEMM for the synaptic product) against the
FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _trials(net, cfg, n_trials, first=0):
    i_nA, v0 = W.trial_inputs(cfg, net.n, n_trials, first)
    return [W.Instance(net, v0[t], W.Stimulus(i_nA[t])) for t in range(n_trials)]


def _gpu_trials(net, insts, n_steps, rec_stride=1, spike_cap=0):
    """One shared network, len(insts) trials, one psst_batch."""
    from paper_1906_03958_amd import psst
    h = psst.network_create(net)
    return R.gpu_run(insts, n_steps, rec_stride=rec_stride, spike_cap=spike_cap,
                     nets=[h] * len(insts))


def test_stage_path_2048_neurons_8_trials():
    net = W.all_pairs_network(40, 0, 1536, 512, g_max=0.1)
    insts = _trials(net, 40, 8)
    n = 300
    _say("stage path: 2048 neurons x 8 trials,", n, "steps")
    g = _gpu_trials(net, insts, n, rec_stride=1, spike_cap=16)
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=16)
    dv = np.abs(g["v"] - o["v"]).max()
    _say("  max|dV|", dv)
    assert dv <= 1e-3
    np.testing.assert_array_equal(g["spike_count"], o["spike_count"])
    y = R.state_value(g["state"])
    assert np.abs(y[1:5] - o["state"][1:5]).max() < 1e-5


def test_stage_path_50ms_parity_and_spikes():
    """The literal forward gate on the per-stage path: max |dV| <= 1e-3 mV
    over 0-50 ms and spike times within 0.05 ms, 2048 neurons, two of eight
    trials followed by the oracle (float32 matrix-core sums, the path's
    largest error source, accumulate over 5000 steps)."""
    net = W.all_pairs_network(40, 0, 1536, 512, g_max=0.1)
    insts = _trials(net, 40, 8)
    n = 5000
    _say("stage path: 2048 neurons x 8 trials, 50 ms")
    g = _gpu_trials(net, insts, n, rec_stride=1, spike_cap=64)
    pick = [0, 7]
    o = R.oracle_run([insts[t] for t in pick], n, rec_stride=1, spike_cap=64, threads=2)
    for k, t in enumerate(pick):
        a, b = t * net.n, (t + 1) * net.n
        oa, ob = k * net.n, (k + 1) * net.n
        dv = np.abs(g["v"][:, a:b].astype(np.float64) - o["v"][:, oa:ob]).max()
        bad, worst, total = R.spike_match(g["spike_count"][a:b], g["spike_t"][a:b],
                                          o["spike_count"][oa:ob], o["spike_t"][oa:ob], 50.0)
        _say(f"  trial {t}: max|dV| 0-50 ms {dv:.2e} mV, spikes {total}, count mismatches "
             f"{bad}, worst dt {worst:.2e} ms")
        assert dv <= 1e-3, (t, dv)
        assert bad == 0 and worst <= 0.05 and total > 0


def test_stage_path_slow_gaba_and_pulses():
    # an AL-shaped network above the per-workgroup limit: 900 PN + 300 LN with
    # cholinergic, fast-GABA and slow-GABA pathways and pulse stimuli
    base = W.config2(3, t_ms=10.0)
    rm = W.rng_for(41, 0, W.S_MASK)
    rg = W.rng_for(41, 0, W.S_G)
    n_pn, n_ln = 900, 300
    n = n_pn + n_ln
    paths = []
    g_, m_ = W._bernoulli_block(rm, rg, (n_ln, n_pn), 0.5, 0.05)
    paths.append(W.Pathway(W.ACH, 0, n_pn, n_pn, n, g_, m_))
    for typ in (W.GABA_A, W.GABA_B):
        g_, m_ = W._bernoulli_block(rm, rg, (n_pn, n_ln), 0.5, 0.05)
        paths.append(W.Pathway(typ, n_pn, n, 0, n_pn, g_, m_))
        g_, m_ = W._bernoulli_block(rm, rg, (n_ln, n_ln), 0.5, 0.05, (0, 0))
        paths.append(W.Pathway(typ, n_pn, n, n_pn, n, g_, m_))
    net = W.Network(n, n_pn, W.hh_params(n), paths)
    del base
    rs = W.rng_for(41, 0, W.S_PULSE)
    amp = rs.uniform(1.0, 10.0, n).astype(np.float32)
    on = np.zeros(n, np.int64)
    off = np.full(n, 500, np.int64)
    stim = W.Stimulus(np.zeros(n, np.float32), np.arange(n + 1, dtype=np.int32), on, off, amp)
    v0 = W.rng_for(41, 0, W.S_V0).uniform(-70, -60, n).astype(np.float32)
    insts = [W.Instance(net, v0, stim), W.Instance(net, v0[::-1].copy(), stim)]
    steps = 800
    _say("stage path with slow GABA: 1200 neurons x 2 trials,", steps, "steps")
    g = _gpu_trials(net, insts, steps, rec_stride=1, spike_cap=16)
    o = R.oracle_run(insts, steps, rec_stride=1, spike_cap=16)
    dv = np.abs(g["v"] - o["v"]).max()
    _say("  max|dV|", dv, "spikes", int(o["spike_count"].sum()))
    assert dv <= 1e-3
    assert o["spike_count"].sum() > 0
    np.testing.assert_array_equal(g["spike_count"], o["spike_count"])
    y = R.state_value(g["state"])
    assert np.abs(y[5:7] - o["state"][5:7]).max() < 1e-6


def test_stage_path_single_network_integrate_and_chunking():
    from paper_1906_03958_amd import psst
    net = W.all_pairs_network(42, 0, 1200, 400, g_max=0.1)
    inst = _trials(net, 42, 1)[0]
    n = 400
    h = psst.network_create(net)
    g1 = R.gpu_run([inst], n, rec_stride=1, batched=False, nets=[h])
    g2 = R.gpu_run([inst], n, rec_stride=1, batched=False, nets=[h], chunks=[150, 250])
    np.testing.assert_array_equal(g1["state"], g2["state"])
    np.testing.assert_array_equal(g1["v"], g2["v"])
    o = R.oracle_run([inst], n, rec_stride=1)
    dv = np.abs(g1["v"] - o["v"]).max()
    _say("single 1600-neuron network: max|dV|", dv)
    assert dv <= 1e-3


def test_config4_full_size_sampled_trials():
    # the full 16384-neuron network, 64 trials on the GPU; the oracle follows
    # two of the trials for 100 steps (about a minute of oracle time each)
    from paper_1906_03958_amd import psst
    import torch
    net = W.config4_network()
    insts = _trials(net, 4, W.CONFIG4_TRIALS)
    steps = 100
    _say("config4: 16384 neurons x 64 trials,", steps, "steps")
    h = psst.network_create(net)
    g = R.gpu_run(insts, steps, rec_stride=1, nets=[h] * len(insts))
    del h
    torch.cuda.empty_cache()
    pick = [0, 37]
    o = R.oracle_run([insts[t] for t in pick], steps, rec_stride=1, threads=2)
    n = net.n
    for k, t in enumerate(pick):
        gv = g["v"][:, t * n:(t + 1) * n]
        ov = o["v"][:, k * n:(k + 1) * n]
        dv = np.abs(gv - ov).max()
        _say(f"  trial {t}: max|dV| over {steps} steps = {dv:.3e}")
        assert dv <= 1e-3


def test_stage_path_ragged_tiles():
    # 1025 neurons (770 PN + 255 LN): one neuron past the per-workgroup limit,
    # a last 64-row tile holding one real row, K blocks padded (770 -> 896,
    # 255 -> 256); 70 trials: a second 64-trial tile holding 6.  The oracle
    # follows trials at both tiles' edges.
    net = W.all_pairs_network(43, 0, 770, 255, g_max=0.1)
    insts = _trials(net, 43, 70)
    n = 150
    _say("stage path, ragged tiles: 1025 neurons x 70 trials,", n, "steps")
    g = _gpu_trials(net, insts, n, rec_stride=1, spike_cap=16)
    picks = [0, 63, 64, 69]
    o = R.oracle_run([insts[t] for t in picks], n, rec_stride=1, spike_cap=16)
    for k, t in enumerate(picks):
        a = t * net.n
        dv = np.abs(g["v"][:, a:a + net.n].astype(np.float64)
                    - o["v"][:, k * net.n:(k + 1) * net.n]).max()
        _say(f"  trial {t}: max|dV| {dv:.2e} mV")
        assert dv <= 1e-3, (t, dv)
        np.testing.assert_array_equal(g["spike_count"][a:a + net.n],
                                      o["spike_count"][k * net.n:(k + 1) * net.n])


def test_stage_path_trial_invariance_bitwise():
    """A trial's trajectory on the per-stage path does not depend on the
    other trials of its batch: 70 trials (64-trial tiles, the second one
    ragged) vs ten of them alone (16-trial tiles) vs the same ten in reverse
    order, bit for bit."""
    net = W.all_pairs_network(44, 0, 816, 272, g_max=0.1)
    insts = _trials(net, 44, 70)
    n = 100
    a = _gpu_trials(net, insts, n, rec_stride=1, spike_cap=8)
    sub = list(range(60, 70))
    b = _gpu_trials(net, [insts[t] for t in sub], n, rec_stride=1, spike_cap=8)
    c = _gpu_trials(net, [insts[t] for t in sub[::-1]], n, rec_stride=1, spike_cap=8)
    m = net.n
    for k, t in enumerate(sub):
        ka = slice(t * m, (t + 1) * m)
        kb = slice(k * m, (k + 1) * m)
        kc = slice((len(sub) - 1 - k) * m, (len(sub) - k) * m)
        np.testing.assert_array_equal(a["v"][:, ka], b["v"][:, kb])
        np.testing.assert_array_equal(a["v"][:, ka], c["v"][:, kc])
        np.testing.assert_array_equal(a["state"][:, :, ka], b["state"][:, :, kb])
        np.testing.assert_array_equal(a["spike_t"][ka], c["spike_t"][kc])
    _say("  per-stage path: 10 trials bitwise equal in batches of 70, 10 and 10 reversed")


def test_stage_path_reports_a_blow_up():
    """The per-stage path flags non-finite states too (dt = 5 ms, 1100
    neurons x 2 trials); the poll clears the flag."""
    from paper_1906_03958_amd import psst
    import torch
    dev = torch.device("cuda:0")
    net = W.all_pairs_network(46, 0, 825, 275, g_max=0.1)
    insts = _trials(net, 46, 2)
    h = psst.network_create(net)
    batch = psst.batch_create([h, h])
    st = torch.zeros(14 * batch.n_total, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    psst.integrate_batch(batch, st, stim, 5.0, 50, 0)
    with pytest.raises(psst.PsstError) as e:
        psst.batch_poll(batch)
    assert e.value.status == psst.ERR_NONFINITE
    psst.batch_poll(batch)


def test_stage_path_strided_records_across_chunks():
    """Records every 7th step on the per-stage path, the run split at step 10
    (not a multiple of the stride): the rows are exactly the stride-1 run's
    rows at steps 7, 14, ..., 35, and the state is the same bit for bit."""
    net = W.all_pairs_network(47, 0, 780, 260, g_max=0.1)
    insts = _trials(net, 47, 3)
    from paper_1906_03958_amd import psst
    h = psst.network_create(net)
    a = R.gpu_run(insts, 35, rec_stride=1, nets=[h] * 3)
    b = R.gpu_run(insts, 35, rec_stride=7, nets=[h] * 3, chunks=[10, 25])
    assert b["v"].shape[0] == 5
    np.testing.assert_array_equal(b["v"], a["v"][6::7])
    np.testing.assert_array_equal(b["state"], a["state"])
