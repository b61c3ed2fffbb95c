"""Register-held conductance columns (the batch variant that keeps the leading
columns of every chunk of a streamed network in registers, then LDS, then
global memory) against the same launch shape without them, through the C ABI:
the column-order fma sequence is unchanged, so trajectories, records, spikes,
states and adjoint gradients must agree bit for bit -- across chunk counts per
column group of 1 to 6 (with and without slow GABA), with no conductances in
LDS at all, and across resumed calls; the tuned batch meets the oracle gate;
the byte accounting moves exactly the register columns from streamed to
resident."""
import os
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import psst
from paper_1906_03958_amd import workloads as W
from tests import _runs as R

pytestmark = pytest.mark.gpu

DV_TOL = 1e-3        # mV, 0-50 ms
SPIKE_TOL = 0.05     # ms

RR = "256x2r48"      # 256 threads x 2 neurons, 48 register slots per thread
NO_RR = "256x2"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class _env:
    """Set (value) or clear (None) environment variables for the library's
    next calls."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        for k, v in self.kv.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = str(v)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _chunks_per_group(n, n_pn, slow, bs=256):
    """Chunks of 64 columns per column group of four-row threads (ld / 4
    threads per group) -- what sets the register columns per chunk."""
    ld = (n + 3) & ~3
    nch = -(-n_pn // 64) + -(-(n - n_pn) // 64) * (2 if slow else 1)
    ncg = bs // (ld // 4)
    return -(-nch // ncg)


# (n_pn, n_ln, slow GABA): chunk counts per column group 1 .. 6, an all-LN
# network, the 512-neuron limit of 256 x 2 and sizes at chunk edges
_SIZES = [(192, 64, False), (195, 65, False), (255, 85, False), (258, 86, False),
          (360, 120, False), (180, 60, True), (270, 90, True), (384, 128, True),
          (0, 300, False), (321, 127, False), (256, 96, False), (256, 256, True)]


def _insts():
    out = []
    for k, (n_pn, n_ln, slow) in enumerate(_SIZES):
        gen = W.sized_instance_slow if slow else W.sized_instance
        out.append(gen(800 + k, n_pn, n_ln))
    return out


def _run(insts, n, shape, lds_g=None, **kw):
    with _env(PSST_WG_SHAPE=shape, PSST_LDS_G=lds_g):
        return R.gpu_run(insts, n, **kw)


def _equal(a, b):
    np.testing.assert_array_equal(a["state"], b["state"])
    np.testing.assert_array_equal(a["v"], b["v"])
    np.testing.assert_array_equal(a["spike_count"], b["spike_count"])
    np.testing.assert_array_equal(a["spike_t"], b["spike_t"])


def _describe(insts, shape):
    nets = [psst.network_create(i.net) for i in insts]
    with _env(PSST_WG_SHAPE=shape):
        return psst.batch_describe(psst.batch_create(nets))


def test_register_columns_bitwise():
    insts = _insts()
    kcs = [_chunks_per_group(i.net.n, i.net.n_pn, i.net.has_gabab) for i in insts]
    _say("sizes", [i.net.n for i in insts], "chunks per column group", kcs)
    assert set(range(1, 7)) <= set(kcs)
    # the two runs take the variants they are meant to compare
    d_rr, d_no = _describe(insts, RR), _describe(insts, NO_RR)
    _say(d_rr, d_no)
    assert "256 thr x 2 neurons, 48 register slots" in d_rr
    assert "256 thr x 2 neurons, lds" in d_no
    n = 300
    base = _run(insts, n, NO_RR, rec_stride=1, spike_cap=8)
    rr = _run(insts, n, RR, rec_stride=1, spike_cap=8)
    _equal(rr, base)
    # no conductances in LDS: registers, then global memory
    rr0 = _run(insts, n, RR, lds_g=0, rec_stride=1, spike_cap=8)
    _equal(rr0, base)
    # resumed calls, strided records
    rc = _run(insts, n, RR, rec_stride=3, spike_cap=8, chunks=[100, 41, 159])
    b3 = _run(insts, n, NO_RR, rec_stride=3, spike_cap=8)
    _equal(rc, b3)


def test_register_columns_describe_and_bytes():
    torch, dev = R.torch_dev()
    insts = _insts()
    nets = [psst.network_create(i.net) for i in insts]
    out = {}
    for shape in (RR, NO_RR):
        with _env(PSST_WG_SHAPE=shape):
            b = psst.batch_create(nets)
        out[shape] = (psst.batch_describe(b), psst.batch_conductance_bytes(b))
        _say(shape, out[shape])
    assert "48 register slots" in out[RR][0]
    assert "register slots" not in out[NO_RR][0]
    (res_r, str_r), (res_n, str_n) = out[RR][1], out[NO_RR][1]
    # every conductance is counted once: resident or streamed
    assert res_r + str_r == res_n + str_n
    assert str_r < str_n and res_r > res_n


def test_tuned_batch_with_register_columns_meets_the_oracle_gate():
    insts = [_insts()[k] for k in (1, 3, 4, 6, 7)]
    n = 5000                            # 50 ms
    with _env(PSST_WG_SHAPE=None, PSST_TUNE=None, PSST_RR=None):
        nets = [psst.network_create(i.net) for i in insts]
        b = psst.batch_create(nets)
        _say("tuned:", psst.batch_describe(b))
        g = R.gpu_run(insts, n, rec_stride=10, spike_cap=32, nets=nets)
    # the forced register variant over the same horizon, for the record
    f = _run(insts, n, RR, rec_stride=10, spike_cap=32)
    o = R.oracle_run(insts, n, rec_stride=10, spike_cap=32)
    for name, r in (("tuned", g), ("register columns", f)):
        dv = np.abs(r["v"] - o["v"]).max()
        bad, worst, total = R.spike_match(r["spike_count"], r["spike_t"], o["spike_count"],
                                          o["spike_t"], 50.0)
        _say(f"  {name}: max|dV| {dv:.3e} mV, spikes {total} matched, worst {worst:.2e} ms")
        assert dv <= DV_TOL
        assert bad == 0 and worst <= SPIKE_TOL


def test_adjoint_recomputation_with_register_columns_bitwise():
    # the adjoint recomputes each segment with the batch's own forward
    # kernels: gradients through the register-column variant equal those
    # through the same shape without it
    torch, dev = R.torch_dev()
    insts = [_insts()[k] for k in (3, 6)]
    T, K = 120, 40
    grads = {}
    for shape in (RR, NO_RR):
        with _env(PSST_WG_SHAPE=shape):
            nets = [psst.network_create(i.net) for i in insts]
            b = psst.batch_create(nets)
        nt = b.n_total
        st = torch.zeros(14 * nt, dtype=torch.float32, device=dev)
        v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
        psst.batch_state_init(b, v0, st)
        stim = psst.pack_stimulus([i.stim for i in insts], dev)
        ck = torch.zeros((T // K, 14 * nt), dtype=torch.float32, device=dev)
        psst.integrate_batch(b, st, stim, 0.01, T, 0, None, ck, K)
        dl = (np.random.default_rng(3).standard_normal((T, nt)) * 1e-3).astype(np.float32)
        gsz = sum(h.grad_size for h in nets)
        gg = torch.zeros(gsz, dtype=torch.float32, device=dev)
        gna = torch.zeros(nt, dtype=torch.float32, device=dev)
        gk, gl = torch.zeros_like(gna), torch.zeros_like(gna)
        psst.adjoint(b, ck, K, stim, 0.01, T, 0, torch.from_numpy(dl).to(dev), gg, gna, gk, gl,
                     per_instance=True)
        psst.batch_poll(b)
        grads[shape] = [x.cpu().numpy() for x in (gg, gna, gk, gl)]
        _say(shape, psst.batch_describe(b), "|g| =", float(np.linalg.norm(grads[shape][0])))
    for x, y in zip(grads[RR], grads[NO_RR]):
        np.testing.assert_array_equal(x, y)


def test_tuning_table_is_written_on_request(tmp_path):
    # a batch whose classes are not in the process's tuning cache (register
    # columns switched off makes a new key) is tuned, and PSST_TUNE_WRITE=1
    # writes the cache to the table named by PSST_TUNE_FILE
    path = tmp_path / "table.txt"
    insts = [_insts()[k] for k in (0, 4)]
    nets = [psst.network_create(i.net) for i in insts]
    with _env(PSST_WG_SHAPE=None, PSST_TUNE=None, PSST_RR="0", PSST_TUNE_WRITE="1",
              PSST_TUNE_FILE=str(path)):
        b = psst.batch_create(nets)
    _say(psst.batch_describe(b))
    lines = [ln.split() for ln in open(path) if ln.startswith("class ")]
    assert any(int(t[7]) == 0 for t in lines)          # an entry with register columns off
    assert all(int(t[10]) == 0 for t in lines if int(t[7]) == 0)
