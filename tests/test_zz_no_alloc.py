"""psst_adjoint_noalloc (the adjoint for callers that cannot allocate) through
the C ABI against psst_adjoint on the same batch and inputs: two calls in a
row, the second on a smaller input (fewer instances, fewer steps, another
K), each bit for bit equal to psst_adjoint (same kernels, same summation
order; the scratch array keeps the first call's contents, which must not
leak into the second); a call with no steps gives zero gradients; a request
above the scratch array's 64 MiB is refused before any device work."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _forward(psst, torch, dev, batch, insts, T, K):
    nt = batch.n_total
    st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    psst.batch_state_init(batch, v0, st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    ck = torch.zeros(((T + K - 1) // K, 14 * nt), dtype=torch.float32, device=dev)
    psst.integrate_batch(batch, st, stim, 0.01, T, 0, None, ck, K)
    psst.batch_poll(batch)
    return stim, ck


def _grads(psst, torch, dev, fn, batch, nets, ck, K, stim, T, dl, per_instance):
    gsize = sum(n.grad_size for n in nets) if per_instance else nets[0].grad_size
    nn = batch.n_total if per_instance else nets[0].n
    # outputs start as NaN: every entry must be written by the call
    gg = torch.full((max(gsize, 1),), float("nan"), dtype=torch.float32, device=dev)
    gna = torch.full((nn,), float("nan"), dtype=torch.float32, device=dev)
    gk, gl = gna.clone(), gna.clone()
    fn(batch, ck, K, stim, 0.01, T, 0, dl, gg, gna, gk, gl, per_instance=per_instance)
    psst.batch_poll(batch)
    return [t.cpu().numpy() for t in (gg, gna, gk, gl)]


def _compare(psst, torch, dev, insts, nets, T, K, per_instance, seed):
    batch = psst.batch_create(nets)
    stim, ck = _forward(psst, torch, dev, batch, insts, T, K)
    rng = np.random.default_rng(seed)
    dl = torch.from_numpy((rng.standard_normal((T, batch.n_total)) * 1e-3)
                          .astype(np.float32)).to(dev)
    ref = _grads(psst, torch, dev, psst.adjoint, batch, nets, ck, K, stim, T, dl, per_instance)
    got = _grads(psst, torch, dev, psst.adjoint_noalloc, batch, nets, ck, K, stim, T, dl,
                 per_instance)
    for name, a, b in zip(("g", "g_Na", "g_K", "g_L"), got, ref):
        assert np.all(np.isfinite(b)), name
        np.testing.assert_array_equal(a, b, err_msg=name)
    _say(f"  {len(nets)} instances, {T} steps, K={K}: bitwise equal, |dL/dg| = "
         f"{float(np.linalg.norm(ref[0])):.3e}")
    return batch, stim, ck, dl


def test_noalloc_adjoint_equals_adjoint_two_calls():
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    # first call: a ragged batch with slow GABA and pulse trains, per instance
    insts = [W.config2(0, t_ms=3.0), W.config3_instance(5), W.config3_instance(77),
             W.config1(0)]
    nets = [psst.network_create(i.net) for i in insts]
    _say("  first call: sizes", [i.net.n for i in insts])
    _compare(psst, torch, dev, insts, nets, 300, 50, True, 1)
    # second call, smaller: two trials of one 20-neuron network, summed
    net = W.config1(1).net
    i_nA, v0 = W.trial_inputs(1, net.n, 2)
    insts2 = [W.Instance(net, v0[t], W.Stimulus(i_nA[t])) for t in range(2)]
    h = psst.network_create(net)
    batch, stim, ck, dl = _compare(psst, torch, dev, insts2, [h, h], 120, 40, False, 2)
    # no steps: zero gradients (the accumulators still hold the last call's)
    got = _grads(psst, torch, dev, psst.adjoint_noalloc, batch, [h, h], ck, 40, stim, 0, dl,
                 False)
    for a in got:
        assert np.all(a == 0.0)


def test_noalloc_adjoint_refuses_requests_above_its_scratch():
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    hidden, ev, i_nA, v0 = W.config5(64)
    net = psst.network_create(ev)
    batch = psst.batch_create([net] * 64)
    nt = batch.n_total
    K, T = 100, 200
    # 64 trials x 120 neurons x K = 100 need 480 * 120 * 100 * 64 B = 369 MB
    ck = torch.zeros((T // K, 14 * nt), dtype=torch.float32, device=dev)
    dl = torch.zeros((T, nt), dtype=torch.float32, device=dev)
    gg = torch.zeros(net.grad_size, dtype=torch.float32, device=dev)
    gn = torch.zeros(net.n, dtype=torch.float32, device=dev)
    with pytest.raises(psst.PsstError) as e:
        psst.adjoint_noalloc(batch, ck, K, None, 0.01, T, 0, dl, gg, gn, gn, gn,
                             per_instance=False)
    assert e.value.status == psst.ERR_INVALID_ARGUMENT
    assert "scratch" in str(e.value)
    _say("  refused:", str(e.value)[:120])
