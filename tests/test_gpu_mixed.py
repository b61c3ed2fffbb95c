"""Ragged batches that mix networks above 1024 neurons (per-stage path) with
smaller ones (per-instance kernels): every instance against the FP64 oracle,
and bit for bit against the same instances run in batches of their own
kind; pulses, strided records and resumed calls; dense and sparse large
networks; what the per-stage path does not offer (checkpoints, adjoint) is
refused with UNSUPPORTED."""
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


def _trial(net, cfg, t):
    i_nA, v0 = W.trial_inputs(cfg, net.n, 1, t)
    return W.Instance(net, v0[0], W.Stimulus(i_nA[0]))


def _mixed():
    """[small, large x2 (one run), small with pulses, large sparse, small]."""
    big = W.all_pairs_network(53, 0, 825, 275, g_max=0.1)
    sparse = W.all_pairs_network(54, 0, 780, 260, g_max=0.5, p=0.1)
    insts = [W.config3_instance(11), _trial(big, 53, 0), _trial(big, 53, 1),
             W.config2(0, t_ms=20.0), _trial(sparse, 54, 0), W.config3_instance(3000)]
    return insts


def _nets(insts):
    """Device networks, one per distinct network; sparse storage for every
    network above 1024 neurons at density 0.25 or less."""
    from paper_1906_03958_amd import psst
    made = {}
    out = []
    for inst in insts:
        key = id(inst.net)
        if key not in made:
            dens = (sum(int(np.count_nonzero(w.mask)) for w in inst.net.pathways)
                    / max(1, sum(w.mask.size for w in inst.net.pathways)))
            sparse = inst.net.n > 1024 and dens <= 0.25
            made[key] = psst.network_create(inst.net,
                                            storage=psst.STORAGE_SPARSE if sparse else None)
        out.append(made[key])
    return out


def test_mixed_batch_against_oracle_and_own_kind_bitwise():
    from paper_1906_03958_amd import psst
    insts = _mixed()
    nets = _nets(insts)
    desc = psst.batch_describe(psst.batch_create(nets))
    _say("sizes", [i.net.n for i in insts], "\n ", desc)
    assert "per-stage fp32 MFMA" in desc and "per-stage sparse" in desc
    n = 400
    g = R.gpu_run(insts, n, rec_stride=2, spike_cap=16, nets=nets, chunks=[150, 250])
    o = R.oracle_run(insts, n, rec_stride=2, spike_cap=16, threads=6)
    offs = g["offsets"]
    for k, inst in enumerate(insts):
        a, b = offs[k], offs[k + 1]
        dv = np.abs(g["v"][:, a:b].astype(np.float64) - o["v"][:, a:b]).max()
        bad, worst, total = R.spike_match(g["spike_count"][a:b], g["spike_t"][a:b],
                                          o["spike_count"][a:b], o["spike_t"][a:b], n * 0.01)
        _say(f"  instance {k} (n={inst.net.n}): max|dV| {dv:.2e} mV, spikes {total}")
        assert dv <= 1e-3 and bad == 0 and worst <= 0.05
    # the small instances alone, and the large network's two trials alone
    small = [0, 3, 5]
    s = R.gpu_run([insts[k] for k in small], n, rec_stride=2, spike_cap=16,
                  nets=[nets[k] for k in small])
    for j, k in enumerate(small):
        a, b = offs[k], offs[k + 1]
        c, d = s["offsets"][j], s["offsets"][j + 1]
        np.testing.assert_array_equal(g["v"][:, a:b], s["v"][:, c:d])
        np.testing.assert_array_equal(g["state"][:, :, a:b], s["state"][:, :, c:d])
    L = R.gpu_run(insts[1:3], n, rec_stride=2, spike_cap=16, nets=nets[1:3])
    a, b = offs[1], offs[3]
    np.testing.assert_array_equal(g["v"][:, a:b], L["v"])
    np.testing.assert_array_equal(g["spike_t"][a:b], L["spike_t"])
    np.testing.assert_array_equal(g["state"][:, :, a:b], L["state"])


def test_mixed_batch_tableau_and_description():
    """An explicit method set on a mixed batch reaches its per-stage
    sub-batches (the description follows), and the run matches the oracle's
    run of that tableau."""
    from paper_1906_03958_amd import psst
    tab = W.TABLEAUX["heun"]
    insts = _mixed()
    nets = _nets(insts)
    batch = psst.batch_create(nets)
    assert "4 launches per step" in psst.batch_describe(batch)
    psst.batch_set_tableau(batch, tab)
    d = psst.batch_describe(batch)
    assert "2 launches per step" in d and "4 launches per step" not in d, d
    for h in nets:
        psst.network_set_tableau(h, tab)
    n = 200
    g = R.gpu_run(insts, n, rec_stride=1, spike_cap=16, nets=nets)
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=16, threads=6, tableau=tab)
    dv = np.abs(g["v"].astype(np.float64) - o["v"]).max()
    _say(f"  mixed batch, Heun: max|dV| {dv:.2e} mV")
    assert dv <= 1e-3
    np.testing.assert_array_equal(g["spike_count"], o["spike_count"])


def test_non_contiguous_runs_and_edge_networks():
    """One large network in two separate runs (two sub-batches), a sparse
    large network of projection neurons only (one synapse class) and one
    whose fast-GABA pathway has no synapse at all, between small instances:
    every instance against the oracle."""
    import copy
    from paper_1906_03958_amd import psst
    big = W.all_pairs_network(55, 0, 825, 275, g_max=0.1)
    pn_only = W.all_pairs_network(56, 0, 1030, 0, g_max=0.5, p=0.1)
    pn_only.pathways = [w for w in pn_only.pathways if w.pre_end > w.pre_begin]
    empty_gaba = W.all_pairs_network(57, 0, 780, 260, g_max=0.5, p=0.1)
    empty_gaba = copy.deepcopy(empty_gaba)
    w = empty_gaba.pathways[1]
    w.mask[:] = 0
    w.g_nS[:] = 0.0
    insts = [_trial(big, 55, 0), W.config3_instance(7), _trial(big, 55, 1),
             _trial(pn_only, 56, 0), _trial(empty_gaba, 57, 0), W.config3_instance(8)]
    made = {}
    nets = []
    for inst in insts:
        if id(inst.net) not in made:
            sparse = inst.net is not big and inst.net.n > 1024
            made[id(inst.net)] = psst.network_create(
                inst.net, storage=psst.STORAGE_SPARSE if sparse else None)
        nets.append(made[id(inst.net)])
    desc = psst.batch_describe(psst.batch_create(nets))
    _say(" ", desc)
    assert desc.count("per-stage fp32 MFMA") == 2 and desc.count("per-stage sparse") == 2
    n = 200
    g = R.gpu_run(insts, n, rec_stride=1, spike_cap=16, nets=nets)
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=16, threads=6)
    offs = g["offsets"]
    for k, inst in enumerate(insts):
        a, b = offs[k], offs[k + 1]
        dv = np.abs(g["v"][:, a:b].astype(np.float64) - o["v"][:, a:b]).max()
        _say(f"  instance {k} (n={inst.net.n}): max|dV| {dv:.2e} mV")
        assert dv <= 1e-3
        np.testing.assert_array_equal(g["spike_count"][a:b], o["spike_count"][a:b])


def test_only_large_networks_of_different_kinds():
    """No per-instance instance at all: two different large networks."""
    insts = _mixed()
    picks = [1, 4]
    sub = [insts[k] for k in picks]
    n = 200
    g = R.gpu_run(sub, n, rec_stride=1, spike_cap=16, nets=_nets(sub))
    o = R.oracle_run(sub, n, rec_stride=1, spike_cap=16, threads=2)
    dv = np.abs(g["v"].astype(np.float64) - o["v"]).max()
    _say(f"  two large networks: max|dV| {dv:.2e} mV")
    assert dv <= 1e-3
    np.testing.assert_array_equal(g["spike_count"], o["spike_count"])


def test_mixed_batch_refuses_checkpoints_and_adjoint():
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    insts = _mixed()
    nets = _nets(insts)
    batch = psst.batch_create(nets)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    ck = torch.zeros((2, 14 * nt), dtype=torch.float32, device=dev)
    with pytest.raises(psst.PsstError) as e:
        psst.integrate_batch(batch, st, stim, 0.01, 20, 0, None, ck, 10)
    assert e.value.status == psst.ERR_UNSUPPORTED
    gs = sum(h.grad_size for h in nets)
    gg = torch.zeros(gs, dtype=torch.float32, device=dev)
    gv = [torch.zeros(nt, dtype=torch.float32, device=dev) for _ in range(3)]
    dl = torch.zeros((20, nt), dtype=torch.float32, device=dev)
    with pytest.raises(psst.PsstError) as e:
        psst.adjoint(batch, ck, 10, stim, 0.01, 20, 0, dl, gg, *gv, per_instance=True)
    assert e.value.status == psst.ERR_UNSUPPORTED


def test_mixed_batch_streamed_equals_one_call():
    """The mixed batch's records drained to host memory in chunks equal one
    on-device call bit for bit."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    insts = _mixed()
    nets = _nets(insts)
    n, chunk = 120, 40
    one = R.gpu_run(insts, n, rec_stride=4, spike_cap=8, nets=nets)
    batch = psst.batch_create(nets)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    hv = np.zeros((n // 4, nt), np.float32)
    hc = np.zeros(nt, np.int32)
    hs = np.zeros((nt, 8), np.float32)
    psst.integrate_batch_streamed(batch, st, stim, 0.01, n, 0, chunk, 4, hv, hc, hs, 8)
    np.testing.assert_array_equal(hv, one["v"])
    np.testing.assert_array_equal(hc, one["spike_count"])
    np.testing.assert_array_equal(hs, one["spike_t"])
    np.testing.assert_array_equal(st.view(7, 2, nt).cpu().numpy(), one["state"])
