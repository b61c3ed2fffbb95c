"""The lane-group kernel (small dense networks, conductances held in
registers) against the LDS-resident per-instance kernels, through the C ABI:
the same fma sequence in the same order, so trajectories, records, spikes and
final states must be equal bit for bit -- plain and batched, resumed calls,
an explicit tableau, ragged sizes at the mapping's edges (chunk boundaries at
64 columns, the 128-row limit, four chunks with slow GABA, no PN), and a batch
mixing eligible and ineligible networks; plus the oracle gate on the
120-neuron network with slow GABA."""
import os
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


class _env:
    """Set environment variables for the library's next calls."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update({k: str(v) for k, v in self.kv.items()})

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _insts():
    out = [W.config1(0), W.config2(0, t_ms=30.0)]
    for k, (n_pn, n_ln) in enumerate([(48, 16), (63, 1), (64, 1), (65, 19), (96, 32),
                                      (0, 40), (120, 8), (2, 1)]):
        out.append(W.sized_instance(700 + k, n_pn, n_ln))
    return out


def _both(insts, n, batched, **kw):
    a = R.gpu_run(insts, n, batched=batched, **kw)
    with _env(PSST_LG=0):
        b = R.gpu_run(insts, n, batched=batched, **kw)
    return a, b


def _equal(a, b):
    for key in ("v", "spike_count", "spike_t", "state"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_lane_group_kernel_is_used_for_small_dense_networks():
    from paper_1906_03958_amd import psst
    insts = _insts() + [W.config3_instance(158)]          # one 480-neuron network too
    nets = [psst.network_create(i.net) for i in insts]
    d = psst.batch_describe(psst.batch_create(nets))
    _say("  ", d)
    assert "lane-group" in d and d.count("[") == 2
    with _env(PSST_LG=0):
        d0 = psst.batch_describe(psst.batch_create(nets))
    assert "lane-group" not in d0


@pytest.mark.parametrize("batched", [True, False])
def test_lane_group_equals_lds_kernels_bitwise(batched):
    insts = _insts()
    a, b = _both(insts, 1500, batched, rec_stride=1, spike_cap=16)
    _equal(a, b)
    assert a["spike_count"].sum() > 50
    _say(f"  {len(insts)} networks, 1500 steps, {int(a['spike_count'].sum())} spikes: equal")


def test_lane_group_resumed_calls_and_strided_records_bitwise():
    insts = _insts()[:4]
    a = R.gpu_run(insts, 900, rec_stride=7, spike_cap=8, chunks=[1, 300, 599])
    with _env(PSST_LG=0):
        b = R.gpu_run(insts, 900, rec_stride=7, spike_cap=8)
    _equal(a, b)


def test_lane_group_tableau_bitwise():
    insts = _insts()[:5]
    for name in ("heun", "kutta3", "rk38"):
        a, b = _both(insts, 400, True, rec_stride=1, tableau=W.TABLEAUX[name])
        _equal(a, b)


def test_lane_group_mixed_batch_bitwise_and_oracle():
    insts = [W.config2(0, t_ms=50.0), W.config3_instance(158), W.config3_instance(3),
             W.config1(1)]
    a, b = _both(insts, 5000, True, rec_stride=10, spike_cap=64)
    _equal(a, b)
    o = R.oracle_run(insts, 5000, rec_stride=10, spike_cap=64)
    dv = float(np.abs(a["v"] - o["v"]).max())
    bad, worst, total = R.spike_match(a["spike_count"], a["spike_t"], o["spike_count"],
                                      o["spike_t"], 50.0)
    _say(f"  mixed batch: max|dV| {dv:.2e} mV over 50 ms, {total} spikes, worst dt {worst:.1e}")
    assert dv <= 1e-3 and bad == 0 and worst <= 0.05
