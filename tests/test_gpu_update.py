"""In-place conductance updates (psst_network_update): a network created
with one set of values and then given another runs, integrates and
differentiates bit for bit as a network created with the new values -- in
every storage (dense with and without slow GABA, lane-group size, sparse
rows with and without the dense copy, the per-stage layout of a network
above 1024 neurons, dense and sparse) and through batches created before the update; values
where the network has no synapse are ignored; parity of an updated network
with the FP64 oracle; the autograd Function reusing its network."""
import copy
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


def _revalued(inst, seed):
    """The instance with new synaptic and intrinsic conductances (same masks):
    each synapse scaled by U(0.5, 1.5), g_Na, g_K, g_L by U(0.8, 1.2)."""
    rng = np.random.default_rng(seed)
    out = copy.deepcopy(inst)
    for p in out.net.pathways:
        x = rng.uniform(0.5, 1.5, p.g_nS.shape)
        p.g_nS = np.where(p.mask != 0, p.g_nS * x, 0.0).astype(np.float32)
    for k in ("g_Na", "g_K", "g_L"):
        out.net.params[k] = (out.net.params[k] * rng.uniform(0.8, 1.2, out.net.n)).astype(np.float32)
    return out


def _update_tensors(net, dev, junk=7.0):
    """Device tensors of a network's values in the update's layout; entries
    with no synapse carry junk (the update must ignore them)."""
    import torch
    g = np.concatenate([np.where(p.mask != 0, p.g_nS, np.float32(junk)).reshape(-1)
                        for p in net.pathways]).astype(np.float32)
    vec = [torch.from_numpy(np.ascontiguousarray(net.params[k], np.float32)).to(dev)
           for k in ("g_Na", "g_K", "g_L")]
    return [torch.from_numpy(g).to(dev)] + vec


def _run_batch(batch, inst, n_trials, n_steps, dev):
    import torch
    from paper_1906_03958_amd import psst
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    v0 = np.concatenate([inst.v0] * n_trials)
    psst.batch_state_init(batch, torch.from_numpy(v0).to(dev), st)
    v = torch.zeros((n_steps, nt), dtype=torch.float32, device=dev)
    stim = psst.pack_stimulus([inst.stim] * n_trials, dev)
    psst.integrate_batch(batch, st, stim, 0.01, n_steps, 0, psst.DeviceRecord(v, 1, n_steps))
    psst.batch_poll(batch)
    return v.cpu().numpy(), st.cpu().numpy()


CASES = [
    ("lane-group size, slow GABA", lambda: W.sized_instance_slow(3, 90, 30), None),
    ("dense 400 neurons", lambda: W.sized_instance(4, 300, 100), None),
    ("sparse rows + dense copy", lambda: W.config3_sparse_instance(17), "sparse"),
    ("sparse rows only (n > 512)", lambda: W.sized_instance(5, 450, 150), "sparse"),
    ("per-stage layout, 1200 neurons", lambda: W.sized_instance(6, 900, 300), None),
    ("per-stage sparse buckets, 1200 neurons", lambda: W.sized_instance(9, 900, 300), "sparse"),
]


@pytest.mark.parametrize("name,make,storage", CASES, ids=[c[0] for c in CASES])
def test_update_equals_create_bitwise(name, make, storage):
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    inst1 = make()
    inst2 = _revalued(inst1, 11)
    st = psst.STORAGE_SPARSE if storage == "sparse" else None
    _say(f"case {name}: n = {inst1.net.n}")
    a = psst.network_create(inst1.net, storage=st)
    before = psst.batch_create([a, a])           # created before the update
    psst.network_update(a, *_update_tensors(inst2.net, dev))
    b = psst.network_create(inst2.net, storage=st)
    n_steps = 200
    va, sa = _run_batch(before, inst2, 2, n_steps, dev)
    vb, sb = _run_batch(psst.batch_create([b, b]), inst2, 2, n_steps, dev)
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(sa, sb)
    # the plain form on the updated network itself
    pa = R.gpu_run([inst2], n_steps, batched=False, nets=[a])
    pb = R.gpu_run([inst2], n_steps, batched=False, nets=[b])
    np.testing.assert_array_equal(pa["v"], pb["v"])
    np.testing.assert_array_equal(pa["state"], pb["state"])
    # and it moved: the first values give another trajectory
    p1 = R.gpu_run([inst1], n_steps, batched=False)
    assert not np.array_equal(p1["v"], pa["v"])


def test_partial_update_keeps_the_rest():
    """NULL parts are kept: only g_L changed equals a network created with
    only g_L changed; then only the synapses."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    inst1 = W.sized_instance(8, 150, 50)
    inst2 = _revalued(inst1, 12)
    only_gl = copy.deepcopy(inst1)
    only_gl.net.params["g_L"] = inst2.net.params["g_L"]
    a = psst.network_create(inst1.net)
    g, gna, gk, gl = _update_tensors(inst2.net, dev)
    psst.network_update(a, None, None, None, gl)
    ra = R.gpu_run([only_gl], 200, batched=False, nets=[a])
    rb = R.gpu_run([only_gl], 200, batched=False)
    np.testing.assert_array_equal(ra["v"], rb["v"])
    syn_too = copy.deepcopy(only_gl)
    syn_too.net.pathways = inst2.net.pathways
    psst.network_update(a, g)
    ra = R.gpu_run([syn_too], 200, batched=False, nets=[a])
    rb = R.gpu_run([syn_too], 200, batched=False)
    np.testing.assert_array_equal(ra["v"], rb["v"])


def test_updated_network_against_oracle():
    """Parity: a network updated to new values, integrated over 50 ms in a
    batch, against the FP64 oracle run of those values."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    inst1 = W.sized_instance_slow(21, 60, 20)
    inst2 = _revalued(inst1, 13)
    a = psst.network_create(inst1.net)
    psst.network_update(a, *_update_tensors(inst2.net, dev))
    n_steps = 5000
    g = R.gpu_run([inst2], n_steps, rec_stride=10, spike_cap=64, nets=[a])
    o = R.oracle_run([inst2], n_steps, rec_stride=10, spike_cap=64)
    dv = float(np.abs(g["v"] - o["v"]).max())
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], n_steps * 0.01)
    _say(f"updated network vs oracle: max|dV| = {dv:.3e} mV, spikes {total}, worst dt {worst}")
    assert dv <= 1e-3 and bad == 0 and worst <= 0.05


def test_adjoint_after_update_equals_created_bitwise():
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    hidden, ev, i_nA, v0 = W.config5(4)
    B, T, K = 4, 300, 50
    a = psst.network_create(hidden)
    batch_a = psst.batch_create([a] * B)
    psst.network_update(a, *_update_tensors(ev, dev))
    b = psst.network_create(ev)
    batch_b = psst.batch_create([b] * B)
    stim = psst.DeviceStimulus(torch.from_numpy(i_nA.ravel().astype(np.float32)).to(dev))
    dld = torch.from_numpy((np.random.default_rng(3).standard_normal((T, B * ev.n)) * 1e-3)
                           .astype(np.float32)).to(dev)
    outs = []
    for batch, net in ((batch_a, a), (batch_b, b)):
        nt = batch.n_total
        st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
        psst.batch_state_init(batch, torch.from_numpy(v0.ravel().astype(np.float32)).to(dev), st)
        ck = torch.zeros((T // K, 14 * nt), dtype=torch.float32, device=dev)
        psst.integrate_batch(batch, st, stim, 0.01, T, 0, None, ck, K)
        gg = torch.zeros(net.grad_size * B, dtype=torch.float32, device=dev)
        gv = [torch.zeros(nt, dtype=torch.float32, device=dev) for _ in range(3)]
        psst.adjoint(batch, ck, K, stim, 0.01, T, 0, dld, gg, *gv, per_instance=True)
        psst.batch_poll(batch)
        outs.append([ck.cpu().numpy(), gg.cpu().numpy()] + [x.cpu().numpy() for x in gv])
    for x, y in zip(*outs):
        np.testing.assert_array_equal(x, y)


def test_autograd_reuses_its_network():
    """Repeated calls of the autograd Function keep at most two networks (one
    held by a live graph, one updated in place) and each call's trace equals
    that of a fresh simulation at the same values."""
    import torch
    from paper_1906_03958_amd.autograd import TraceSimulation
    hidden, ev, i_nA, v0 = W.config5(2)
    sim = TraceSimulation(ev, i_nA, v0, 0.01, 150, K=50)
    g0 = sim.pack([p.g_nS for p in ev.pathways])
    gna = torch.as_tensor(ev.params["g_Na"]).clone()
    gk = torch.as_tensor(ev.params["g_K"]).clone()
    gl = torch.as_tensor(ev.params["g_L"]).clone()
    rng = np.random.default_rng(4)
    loss = None
    for it in range(4):
        g = (g0 * torch.from_numpy(rng.uniform(0.7, 1.3, g0.shape).astype(np.float32))
             ).requires_grad_(True)
        v = sim(g, gna, gk, gl)
        fresh = TraceSimulation(ev, i_nA, v0, 0.01, 150, K=50)
        with torch.no_grad():
            vf = fresh(g, gna, gk, gl)
        assert torch.equal(v, vf), it
        loss = (v.double() ** 2).mean()
        loss.backward()
        assert len(sim._slots) <= 2, len(sim._slots)
