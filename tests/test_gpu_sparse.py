"""Sparse conductance storage on the per-instance path
(psst_network_create_storage): the same fixed summation order as dense
storage, so sparse and dense runs of one network agree bit for bit; parity
of the sparse workload (p = 0.1) with the FP64 oracle; the adjoint of
sparse storage (bitwise the dense one, and against the oracle); storage
validation."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R

pytestmark = pytest.mark.gpu

DV_TOL = 1e-3
SPIKE_TOL = 0.05


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sample(k):
    sizes = np.array([W.config3_size(b) for b in range(256)])
    order = np.argsort(sizes, kind="stable")
    return [int(b) for b in order[np.linspace(0, 255, k).astype(int)]]


def _nets(insts, storage):
    from paper_1906_03958_amd import psst
    return [psst.network_create(i.net, storage=storage) for i in insts]


def test_sparse_equals_dense_bitwise():
    from paper_1906_03958_amd import psst
    insts = [W.config3_sparse_instance(b) for b in _sample(5)] + \
        [W.config3_instance(b) for b in _sample(3)] + [W.config2(0, t_ms=20.0)]
    _say("sizes", [i.net.n for i in insts])
    for batched in (True, False):
        d = R.gpu_run(insts, 400, rec_stride=1, spike_cap=16, batched=batched,
                      nets=_nets(insts, psst.STORAGE_DENSE))
        s = R.gpu_run(insts, 400, rec_stride=1, spike_cap=16, batched=batched,
                      nets=_nets(insts, psst.STORAGE_SPARSE))
        np.testing.assert_array_equal(d["state"], s["state"])
        np.testing.assert_array_equal(d["v"], s["v"])
        np.testing.assert_array_equal(d["spike_count"], s["spike_count"])
        np.testing.assert_array_equal(d["spike_t"], s["spike_t"])
    # a batch mixing storages gives each instance its own result
    mixed = [psst.network_create(i.net, storage=(psst.STORAGE_SPARSE if k % 2 else
                                                 psst.STORAGE_DENSE))
             for k, i in enumerate(insts)]
    m = R.gpu_run(insts, 400, rec_stride=1, spike_cap=16, nets=mixed)
    np.testing.assert_array_equal(d["state"], m["state"])


def test_sparse_workload_parity_and_spikes():
    insts = [W.config3_sparse_instance(b) for b in _sample(10)]
    n = 5000
    g = R.gpu_run(insts, n, rec_stride=10, spike_cap=32)        # AUTO: sparse at p = 0.1
    o = R.oracle_run(insts, n, rec_stride=10, spike_cap=32)
    dv = np.abs(g["v"] - o["v"]).max()
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], 50.0)
    _say(f"sparse p=0.1: max|dV| {dv:.2e} mV, {total} spikes, worst {worst:.2e} ms")
    assert dv <= DV_TOL
    assert bad == 0 and worst <= SPIKE_TOL


def test_storage_validation():
    import torch
    from paper_1906_03958_amd import psst
    inst = W.config1(0)
    with pytest.raises(psst.PsstError) as e:
        psst.network_create(inst.net, storage=7)
    assert e.value.status == psst.ERR_INVALID_ARGUMENT
    # above 1024 neurons sparse storage takes the per-stage path's buckets
    big = W.config4_network(n_pn=1536, n_ln=512)
    h = psst.network_create(big, storage=psst.STORAGE_SPARSE)
    assert "sparse" in psst.batch_describe(psst.batch_create([h]))


def _adjoint(insts, nets, n_steps, K, dl):
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    batch = psst.batch_create(nets)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    ck = torch.zeros(((n_steps + K - 1) // K, 14 * nt), dtype=torch.float32, device=dev)
    psst.integrate_batch(batch, st, stim, 0.01, n_steps, 0, None, ck, K)
    gg = torch.zeros(sum(h.grad_size for h in nets), dtype=torch.float32, device=dev)
    gna = torch.zeros(nt, dtype=torch.float32, device=dev)
    gk, gl = torch.zeros_like(gna), torch.zeros_like(gna)
    psst.adjoint(batch, ck, K, stim, 0.01, n_steps, 0, torch.from_numpy(dl).to(dev), gg, gna,
                 gk, gl, per_instance=True)
    psst.batch_poll(batch)
    return [x.cpu().numpy() for x in (gg, gna, gk, gl)]


def test_sparse_adjoint_equals_dense_bitwise_and_oracle():
    """The adjoint of sparsely stored networks (p = 0.1 instances of 60-480
    neurons and the 120-neuron network with slow GABA): the recomputed
    forward is bitwise the dense one and the transposed products read the
    same dense rows, so the gradients equal the dense-storage ones bit for
    bit; one instance against the oracle's reverse sweep."""
    import oracle
    from paper_1906_03958_amd import psst
    insts = [W.config3_sparse_instance(b) for b in _sample(4)] + [W.config2(1, t_ms=10.0)]
    n_steps, K = 150, 40
    nt = sum(i.net.n for i in insts)
    dl = (np.random.default_rng(21).standard_normal((n_steps, nt)) * 1e-3).astype(np.float32)
    _say("sparse adjoint: sizes", [i.net.n for i in insts])
    d = _adjoint(insts, _nets(insts, psst.STORAGE_DENSE), n_steps, K, dl)
    s = _adjoint(insts, _nets(insts, psst.STORAGE_SPARSE), n_steps, K, dl)
    for a, b in zip(d, s):
        np.testing.assert_array_equal(a, b)
    k = len(insts) - 1                          # the slow-GABA network
    inst = insts[k]
    off = nt - inst.net.n
    on = oracle.OracleNet(inst.net)
    ref = oracle.adjoint(on, oracle.init_state(on, inst.v0), inst.stim, R.DT, n_steps,
                         dl[:, off:].astype(np.float64))
    gsz = sum(int(p.g_nS.size) for p in inst.net.pathways)
    got = {"g": s[0][-gsz:], "g_Na": s[1][off:], "g_K": s[2][off:], "g_L": s[3][off:]}
    for key, v in got.items():
        r = np.asarray(ref[key], np.float64)
        nrm = np.linalg.norm(v - r) / np.linalg.norm(r)
        _say(f"  {key}: norm rel err {nrm:.2e}")
        assert nrm <= 1e-3, (key, nrm)


def test_sparse_at_the_per_instance_limit():
    """Sparse rows at the largest per-instance network, 1024 neurons
    (768 PN + 256 LN, p = 0.1): bitwise the dense result (plain and batched)
    and within the forward gate of the oracle over 3 ms."""
    from paper_1906_03958_amd import psst
    net = W.all_pairs_network(45, 0, 768, 256, p=0.1)
    i_nA, v0 = W.trial_inputs(45, net.n, 1)
    inst = W.Instance(net, v0[0], W.Stimulus(i_nA[0]))
    n = 300
    for batched in (True, False):
        d = R.gpu_run([inst], n, rec_stride=1, spike_cap=16, batched=batched,
                      nets=_nets([inst], psst.STORAGE_DENSE))
        s = R.gpu_run([inst], n, rec_stride=1, spike_cap=16, batched=batched,
                      nets=_nets([inst], psst.STORAGE_SPARSE))
        np.testing.assert_array_equal(d["state"], s["state"])
        np.testing.assert_array_equal(d["v"], s["v"])
    o = R.oracle_run([inst], n, rec_stride=1, spike_cap=16)
    dv = float(np.abs(s["v"] - o["v"]).max())
    _say(f"  sparse 1024 neurons: max|dV| {dv:.2e} mV")
    assert dv <= DV_TOL
    np.testing.assert_array_equal(s["spike_count"], o["spike_count"])
