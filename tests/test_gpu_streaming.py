"""Long runs streamed to host memory (psst_integrate_batch_streamed): the
records drained chunk by chunk through two alternating buffer sets equal
those of one psst_integrate_batch call bit for bit (V rows, spike counts and
times, final state), for a ragged last chunk and a spike cap that drops
spikes; argument checks."""
import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W

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
