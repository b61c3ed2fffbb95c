"""General explicit Runge-Kutta tableaux on the GPU (psst_network_set_tableau,
psst_batch_set_tableau): the same discrete map as the FP64 oracle run with
the same tableau -- forward parity (max |dV| <= 1e-3 mV over the first
50 ms, spike times within 0.05 ms), bitwise invariances (batched = plain,
chunking, batch order), the per-stage path of large networks, the discrete adjoint against the oracle's tableau
adjoint, classical RK4 given as a tableau = the default path bit for bit,
and the validation of the tableau rules."""
import sys

import numpy as np
import pytest

import oracle
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


def _c3_sample(k):
    sizes = np.array([W.config3_size(b) for b in range(256)])
    order = np.argsort(sizes, kind="stable")
    return [int(b) for b in order[np.linspace(0, 255, k).astype(int)]]


@pytest.mark.parametrize("name", ["euler", "midpoint", "heun", "ralston", "kutta3", "ssprk3",
                                  "rk38"])
def test_tableau_forward_parity(name):
    tab = W.TABLEAUX[name]
    insts = [W.config1(0), W.config2(0, t_ms=60.0)] + \
        [W.config3_instance(b) for b in _c3_sample(4)]
    n = 5000
    _say(f"{name}: sizes {[i.net.n for i in insts]}")
    g = R.gpu_run(insts, n, rec_stride=10, spike_cap=32, tableau=tab)
    o = R.oracle_run(insts, n, rec_stride=10, spike_cap=32, tableau=tab)
    dv = np.abs(g["v"] - o["v"]).max()
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], 50.0)
    _say(f"  max|dV| {dv:.2e} mV, spikes {total}, count mismatches {bad}, worst dt {worst:.2e} ms")
    assert dv <= DV_TOL
    assert bad == 0 and worst <= SPIKE_TOL


def test_tableau_batched_equals_plain_chunked_and_order_invariant_bitwise():
    tab = W.TABLEAUX["ssprk3"]
    insts = [W.config3_instance(b) for b in _c3_sample(6)] + [W.config2(0, t_ms=5.0)]
    a = R.gpu_run(insts, 300, rec_stride=1, spike_cap=8, batched=True, tableau=tab)
    p = R.gpu_run(insts, 300, rec_stride=1, spike_cap=8, batched=False, tableau=tab)
    np.testing.assert_array_equal(a["state"], p["state"])
    np.testing.assert_array_equal(a["v"], p["v"])
    c = R.gpu_run(insts, 300, rec_stride=1, spike_cap=8, batched=True, tableau=tab,
                  chunks=[100, 37, 163])
    np.testing.assert_array_equal(a["state"], c["state"])
    np.testing.assert_array_equal(a["v"], c["v"])
    perm = np.random.default_rng(1).permutation(len(insts))
    d = R.gpu_run([insts[k] for k in perm], 300, rec_stride=1, spike_cap=8, batched=True,
                  tableau=tab)
    for new, old in enumerate(perm):
        a0, a1 = a["offsets"][old], a["offsets"][old + 1]
        d0, d1 = d["offsets"][new], d["offsets"][new + 1]
        np.testing.assert_array_equal(a["state"][:, :, a0:a1], d["state"][:, :, d0:d1])


def test_rk4_tableau_is_the_default_path_bitwise():
    insts = [W.config3_instance(b) for b in _c3_sample(3)]
    a = R.gpu_run(insts, 200, rec_stride=1)
    b = R.gpu_run(insts, 200, rec_stride=1, tableau=W.TABLEAUX["rk4"])
    np.testing.assert_array_equal(a["state"], b["state"])
    np.testing.assert_array_equal(a["v"], b["v"])


def test_batch_set_tableau_switches_method():
    import torch
    from paper_1906_03958_amd import psst
    insts = [W.config3_instance(b) for b in _c3_sample(3)]
    ref = R.gpu_run(insts, 100, rec_stride=0, tableau=W.TABLEAUX["kutta3"])
    nets = [psst.network_create(i.net) for i in insts]
    batch = psst.batch_create(nets)                  # RK4 networks
    dev = torch.device("cuda:0")
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    psst.integrate_batch(batch, st, stim, 0.01, 1, 0)      # builds the RK4 graph
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    psst.batch_set_tableau(batch, W.TABLEAUX["kutta3"])
    psst.integrate_batch(batch, st, stim, 0.01, 100, 0)
    psst.batch_poll(batch)
    np.testing.assert_array_equal(st.view(7, 2, nt).cpu().numpy(), ref["state"])


def test_tableau_validation():
    from paper_1906_03958_amd import psst
    net = psst.network_create(W.config1(0).net)
    bad = [
        dict(a=[], b=[]),                                         # 0 stages
        dict(a=[[0.0] * 5] * 5, b=[0.2] * 5),                     # 5 stages
        dict(a=[[0.0, 1.0], [0.5, 0.0]], b=[0.5, 0.5]),           # implicit entry
        dict(a=[[0.0, 0.0], [float("nan"), 0.0]], b=[0.5, 0.5]),  # not finite
    ]
    for tab in bad:
        with pytest.raises(psst.PsstError) as e:
            if len(tab["b"]) in (0, 5):
                t = psst.Tableau()
                t.stages = len(tab["b"])
                import ctypes as C
                psst._check(psst.lib().psst_network_set_tableau(net.handle, C.byref(t)))
            else:
                psst.network_set_tableau(net, tab)
        assert e.value.status == psst.ERR_INVALID_ARGUMENT
    t = psst.Tableau()                                            # unused stage's weight
    t.stages = 2
    t.a[1][0] = 1.0
    t.b[0] = t.b[1] = 0.5
    t.b[2] = 0.1
    import ctypes as C
    with pytest.raises(psst.PsstError) as e:
        psst._check(psst.lib().psst_network_set_tableau(net.handle, C.byref(t)))
    assert e.value.status == psst.ERR_INVALID_ARGUMENT
    # mixing methods in one batch
    n2 = psst.network_create(W.config1(1).net)
    psst.network_set_tableau(n2, W.TABLEAUX["heun"])
    with pytest.raises(psst.PsstError) as e:
        psst.batch_create([net, n2])
    assert e.value.status == psst.ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("name", ["ssprk3", "rk38", "heun"])
def test_tableau_adjoint_matches_oracle(name):
    import torch
    from paper_1906_03958_amd import psst
    tab = W.TABLEAUX[name]
    B, n_steps, K = 3, 250, 80
    hidden, ev, i_nA, v0 = W.config5(B)
    dev = torch.device("cuda:0")
    net = psst.network_create(ev)
    psst.network_set_tableau(net, tab)
    batch = psst.batch_create([net] * B)
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), st)
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    ck = torch.zeros(((n_steps + K - 1) // K, 14 * nt), dtype=torch.float32, device=dev)
    psst.integrate_batch(batch, st, stim, 0.01, n_steps, 0, None, ck, K)
    psst.batch_poll(batch)
    dl = (np.random.default_rng(11).standard_normal((n_steps, nt)) * 1e-3).astype(np.float32)
    gs = net.grad_size
    gg = torch.zeros(B * gs, dtype=torch.float32, device=dev)
    gna = torch.zeros(nt, dtype=torch.float32, device=dev)
    gk, gl = torch.zeros_like(gna), torch.zeros_like(gna)
    _say(f"adjoint {name}: {B} trials x {ev.n} neurons, {n_steps} steps, K={K}")
    psst.adjoint(batch, ck, K, stim, 0.01, n_steps, 0, torch.from_numpy(dl).to(dev), gg, gna,
                 gk, gl, per_instance=True)
    psst.batch_poll(batch)
    on = oracle.OracleNet(ev)
    gg = gg.cpu().numpy().reshape(B, gs)
    for t in range(B):
        y0 = oracle.init_state(on, v0[t])
        ref = oracle.adjoint(on, y0, W.Stimulus(i_nA[t]), R.DT, n_steps,
                             dl[:, t * ev.n:(t + 1) * ev.n].astype(np.float64), tableau=tab)
        for key, got in (("g", gg[t]), ("g_Na", gna.cpu().numpy()[t * ev.n:(t + 1) * ev.n]),
                         ("g_K", gk.cpu().numpy()[t * ev.n:(t + 1) * ev.n]),
                         ("g_L", gl.cpu().numpy()[t * ev.n:(t + 1) * ev.n])):
            r = np.asarray(ref[key], np.float64)
            nrm = np.linalg.norm(got - r) / np.linalg.norm(r)
            _say(f"  trial {t} {key}: norm rel err {nrm:.2e}")
            assert nrm <= 1e-3, (name, t, key, nrm)


def test_tableau_adjoint_after_rk4_on_the_same_batch():
    """A method with fewer stages than RK4, differentiated on a batch whose
    workspace still holds an RK4 adjoint's stage records: the stages the
    method lacks must add nothing to dL/dg (against the oracle's adjoint of
    the same method)."""
    import torch
    from paper_1906_03958_amd import psst
    B, n_steps, K = 2, 160, 40
    hidden, ev, i_nA, v0 = W.config5(B)
    dev = torch.device("cuda:0")
    net = psst.network_create(ev)
    batch = psst.batch_create([net] * B)
    nt = batch.n_total
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel()).to(dev))
    dl = (np.random.default_rng(12).standard_normal((n_steps, nt)) * 1e-3).astype(np.float32)
    gs = net.grad_size
    outs = {}
    for name in ("rk4", "heun"):
        if name != "rk4":
            psst.batch_set_tableau(batch, W.TABLEAUX[name])
        st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
        psst.batch_state_init(batch, torch.from_numpy(v0.ravel()).to(dev), st)
        ck = torch.zeros(((n_steps + K - 1) // K, 14 * nt), dtype=torch.float32, device=dev)
        psst.integrate_batch(batch, st, stim, 0.01, n_steps, 0, None, ck, K)
        gg = torch.zeros(B * gs, dtype=torch.float32, device=dev)
        gna = torch.zeros(nt, dtype=torch.float32, device=dev)
        gk, gl = torch.zeros_like(gna), torch.zeros_like(gna)
        _say(f"adjoint {name} on the shared batch: {B} trials x {ev.n} neurons, {n_steps} steps")
        psst.adjoint(batch, ck, K, stim, 0.01, n_steps, 0, torch.from_numpy(dl).to(dev), gg,
                     gna, gk, gl, per_instance=True)
        psst.batch_poll(batch)
        outs[name] = gg.cpu().numpy().reshape(B, gs)
    on = oracle.OracleNet(ev)
    for t in range(B):
        y0 = oracle.init_state(on, v0[t])
        ref = np.asarray(oracle.adjoint(on, y0, W.Stimulus(i_nA[t]), R.DT, n_steps,
                                        dl[:, t * ev.n:(t + 1) * ev.n].astype(np.float64),
                                        tableau=W.TABLEAUX["heun"])["g"], np.float64)
        nrm = np.linalg.norm(outs["heun"][t] - ref) / np.linalg.norm(ref)
        _say(f"  trial {t} g: norm rel err {nrm:.2e}")
        assert nrm <= 1e-3, (t, nrm)


def _big_trials(n_trials):
    net = W.all_pairs_network(44, 0, 1536, 512, g_max=0.1)
    i_nA, v0 = W.trial_inputs(44, net.n, n_trials)
    return net, [W.Instance(net, v0[t], W.Stimulus(i_nA[t])) for t in range(n_trials)]


@pytest.mark.parametrize("name", ["euler", "heun", "kutta3", "rk38"])
def test_tableau_on_the_per_stage_path(name):
    """2048 neurons shared by 20 trials (one 64-trial GEMM tile), one launch
    per stage of the method: oracle parity on two trials and on trial 0 run
    alone through psst_integrate (a 16-trial tile), chunking bit for bit."""
    from paper_1906_03958_amd import psst
    tab = W.TABLEAUX[name]
    net, insts = _big_trials(20)
    h = psst.network_create(net)
    psst.network_set_tableau(h, tab)
    n = 200
    _say(f"per-stage path, {name}: 2048 neurons x 20 trials, {n} steps")
    g = R.gpu_run(insts, n, rec_stride=1, spike_cap=16, nets=[h] * 20)
    c = R.gpu_run(insts, n, rec_stride=1, spike_cap=16, nets=[h] * 20, chunks=[70, 130])
    np.testing.assert_array_equal(g["state"], c["state"])
    np.testing.assert_array_equal(g["v"], c["v"])
    o = R.oracle_run(insts[:2], n, rec_stride=1, spike_cap=16, tableau=tab)
    dv = np.abs(g["v"][:, :2 * net.n].astype(np.float64) - o["v"]).max()
    _say(f"  max|dV| {dv:.2e} mV")
    assert dv <= DV_TOL
    np.testing.assert_array_equal(g["spike_count"][:2 * net.n], o["spike_count"])
    # trial 0 alone through psst_integrate (a one-trial stage batch)
    p = R.gpu_run(insts[:1], n, rec_stride=1, batched=False, nets=[h])
    dv1 = np.abs(p["v"].astype(np.float64) - o["v"][:, :net.n]).max()
    _say(f"  plain call, trial 0: max|dV| {dv1:.2e} mV")
    assert dv1 <= DV_TOL


def test_per_stage_batch_switches_method():
    """A large-network batch switched RK4 -> Heun -> RK4 with
    psst_batch_set_tableau gives the bits of batches built with each method."""
    import torch
    from paper_1906_03958_amd import psst
    net, insts = _big_trials(8)
    n = 60
    ref = {}
    for name in ("rk4", "heun"):
        h = psst.network_create(net)
        if name != "rk4":
            psst.network_set_tableau(h, W.TABLEAUX[name])
        ref[name] = R.gpu_run(insts, n, rec_stride=0, nets=[h] * 8)["state"]
    h = psst.network_create(net)
    batch = psst.batch_create([h] * 8)
    dev = torch.device("cuda:0")
    nt = batch.n_total
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    for name, tab in (("rk4", None), ("heun", W.TABLEAUX["heun"]), ("rk4", None)):
        psst.batch_set_tableau(batch, tab)
        st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
        psst.batch_state_init(batch, v0, st)
        psst.integrate_batch(batch, st, stim, 0.01, n, 0)
        psst.batch_poll(batch)
        _say(f"  switched to {name}: {psst.batch_describe(batch)}")
        np.testing.assert_array_equal(st.view(7, 2, nt).cpu().numpy(), ref[name])
