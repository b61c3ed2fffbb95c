"""Sparse storage of networks above 1024 neurons (the per-stage path's
synapse buckets) against the FP64 oracle through the C ABI: a 2048-neuron
network at p = 0.1, ragged row and trial tiles with slow GABA and pulse
trains, explicit methods other than RK4 (also on a full 64-trial tile),
sparse storage forced on a p = 0.5 network next to its dense (matrix-core)
form, and trial invariance."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R

pytestmark = pytest.mark.gpu

DV_TOL = 1e-3


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


def _run(net, insts, n_steps, storage="sparse", rec_stride=1, spike_cap=16, tableau=None):
    from paper_1906_03958_amd import psst
    h = psst.network_create(net, storage={"sparse": psst.STORAGE_SPARSE,
                                          "dense": psst.STORAGE_DENSE, None: None}[storage])
    if tableau is not None:
        psst.network_set_tableau(h, tableau)
    desc = psst.batch_describe(psst.batch_create([h] * len(insts)))
    g = R.gpu_run(insts, n_steps, rec_stride=rec_stride, spike_cap=spike_cap,
                  nets=[h] * len(insts))
    return g, desc


def _check(g, o, net, picks, n_steps):
    for k, t in enumerate(picks):
        a = t * net.n
        dv = np.abs(g["v"][:, a:a + net.n].astype(np.float64)
                    - o["v"][:, k * net.n:(k + 1) * net.n]).max()
        bad, worst, total = R.spike_match(g["spike_count"][a:a + net.n],
                                          g["spike_t"][a:a + net.n],
                                          o["spike_count"][k * net.n:(k + 1) * net.n],
                                          o["spike_t"][k * net.n:(k + 1) * net.n],
                                          n_steps * 0.01)
        _say(f"  trial {t}: max|dV| {dv:.2e} mV, spikes {total}, worst dt {worst:.2e} ms")
        assert dv <= DV_TOL, (t, dv)
        assert bad == 0 and worst <= 0.05


def test_sparse_large_network_against_oracle():
    """2048 neurons (1536 PN + 512 LN), p = 0.1 with g ~ U(0, 0.5) nS (the
    expected input of the p = 0.5, U(0, 0.1) network), 8 trials, 30 ms,
    against the oracle and bit for bit against the same network under AUTO
    storage, which keeps a network of this size dense."""
    net = W.all_pairs_network(48, 0, 1536, 512, g_max=0.5, p=0.1)
    insts = _trials(net, 48, 8)
    n = 3000
    g, desc = _run(net, insts, n)
    _say("sparse per-stage:", desc)
    assert "sparse" in desc
    a, adesc = _run(net, insts, n, storage=None)
    assert "sparse" not in adesc and "MFMA" in adesc, adesc
    np.testing.assert_array_equal(g["v"], a["v"])
    np.testing.assert_array_equal(g["spike_t"], a["spike_t"])
    picks = [0, 7]
    o = R.oracle_run([insts[t] for t in picks], n, rec_stride=1, spike_cap=16, threads=2)
    _check(g, o, net, picks, n)


def _slow_net(cfg, n_pn, n_ln, p):
    """all_pairs_network at density p plus a slow-GABA pathway LN -> all, its
    own Bernoulli(p) mask and U(0, 0.5) nS values (seeded numpy)."""
    net = W.all_pairs_network(cfg, 0, n_pn, n_ln, g_max=0.5, p=p)
    n = n_pn + n_ln
    rng = np.random.default_rng(cfg)
    m = (rng.random((n, n_ln)) < p).astype(np.uint8)
    for k in range(n_ln):
        m[n_pn + k, k] = 0                       # no autapse
    g = np.where(m != 0, rng.uniform(0.0, 0.5, (n, n_ln)), 0.0).astype(np.float32)
    net.pathways.append(W.Pathway(W.GABA_B, n_pn, n, 0, n, g, m))
    return net


def test_sparse_large_slow_gaba_pulses_ragged_tiles():
    """1025 neurons (770 PN + 255 LN, one real row in the last 64-row block,
    padded column blocks) with slow GABA at p = 0.1, pulse trains on top of
    the constant currents, 70 trials (a ragged second 64-trial tile); trials
    at both tiles' edges against the oracle."""
    net = _slow_net(49, 770, 255, 0.1)
    insts = _trials(net, 49, 70)
    for t, inst in enumerate(insts):
        ptr = np.zeros(net.n + 1, np.int32)
        on, off, amp = [], [], []
        for i in range(0, net.n, 37):
            on.append(50 + t), off.append(120 + t), amp.append(1.5)
            ptr[i + 1:] += 1
        inst.stim = W.Stimulus(inst.stim.i_const_nA, ptr, np.array(on, np.int64),
                               np.array(off, np.int64), np.array(amp, np.float32))
    n = 400
    g, desc = _run(net, insts, n)
    _say("sparse per-stage, slow GABA, ragged:", desc)
    assert "sparse" in desc
    picks = [0, 63, 64, 69]
    o = R.oracle_run([insts[t] for t in picks], n, rec_stride=1, spike_cap=16, threads=4)
    _check(g, o, net, picks, n)


def test_sparse_large_tableau():
    """Heun's method on the sparse per-stage path against the oracle's run of
    the same tableau."""
    tab = W.TABLEAUX["heun"]
    net = W.all_pairs_network(50, 0, 825, 275, g_max=0.5, p=0.1)
    insts = _trials(net, 50, 3)
    n = 300
    g, desc = _run(net, insts, n, tableau=tab)
    assert "sparse" in desc and "2 launches per step" in desc
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=16, tableau=tab)
    _check(g, o, net, [0, 1, 2], n)


def test_sparse_large_tableau_full_trial_tile():
    """The 3/8 rule on the sparse per-stage path with 20 trials (one 64-trial
    tile: the eight-wavefront general-tableau kernel): two trials against the
    oracle's run of the same tableau, and every trial bit for bit against
    dense storage of the network."""
    tab = W.TABLEAUX["rk38"]
    net = W.all_pairs_network(58, 0, 840, 280, g_max=0.5, p=0.1)
    insts = _trials(net, 58, 20)
    n = 300
    s, ds = _run(net, insts, n, tableau=tab)
    d, dd = _run(net, insts, n, storage="dense", tableau=tab)
    assert "sparse" in ds and "tile 64 x 64" in ds and "4 launches per step" in ds, ds
    assert "sparse" not in dd, dd
    np.testing.assert_array_equal(s["v"], d["v"])
    np.testing.assert_array_equal(s["state"], d["state"])
    picks = [0, 19]
    o = R.oracle_run([insts[t] for t in picks], n, rec_stride=1, spike_cap=16, threads=2,
                     tableau=tab)
    _check(s, o, net, picks, n)


def test_sparse_forced_on_a_dense_network():
    """Sparse storage asked for on a p = 0.5 network of 1100 neurons: the
    sparse path and the matrix-core path both match the oracle, and each
    other bit for bit (the sparse path builds the same conductance tiles in
    LDS that dense storage loads)."""
    from paper_1906_03958_amd import psst
    net = W.all_pairs_network(51, 0, 825, 275, g_max=0.1)
    insts = _trials(net, 51, 2)
    n = 300
    s, ds = _run(net, insts, n)
    d, dd = _run(net, insts, n, storage=None)
    assert "sparse" in ds and "MFMA" in dd
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=16)
    _check(s, o, net, [0, 1], n)
    _check(d, o, net, [0, 1], n)
    np.testing.assert_array_equal(s["v"], d["v"])
    np.testing.assert_array_equal(s["state"], d["state"])
    np.testing.assert_array_equal(s["spike_t"], d["spike_t"])


def test_sparse_large_trial_invariance_bitwise():
    """A trial's trajectory does not depend on the other trials of its batch:
    70 trials vs ten of them alone vs the same ten reversed, bit for bit."""
    net = W.all_pairs_network(52, 0, 816, 272, g_max=0.5, p=0.1)
    insts = _trials(net, 52, 70)
    n = 100
    a, _ = _run(net, insts, n, spike_cap=8)
    sub = list(range(60, 70))
    b, _ = _run(net, [insts[t] for t in sub], n, spike_cap=8)
    c, _ = _run(net, [insts[t] for t in sub[::-1]], n, spike_cap=8)
    m = net.n
    for k, t in enumerate(sub):
        ka = slice(t * m, (t + 1) * m)
        kb = slice(k * m, (k + 1) * m)
        kc = slice((len(sub) - 1 - k) * m, (len(sub) - k) * m)
        np.testing.assert_array_equal(a["v"][:, ka], b["v"][:, kb])
        np.testing.assert_array_equal(a["v"][:, ka], c["v"][:, kc])
        np.testing.assert_array_equal(a["state"][:, :, ka], b["state"][:, :, kb])
