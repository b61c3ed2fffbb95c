"""Sparse conductance storage on the per-instance path
(psst_network_create_storage): the same fixed summation order as dense
storage, so sparse and dense runs of one network agree bit for bit; parity
of the sparse workload (p = 0.1) with the FP64 oracle; storage validation."""
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
    big = W.config4_network(n_pn=1536, n_ln=512)
    with pytest.raises(psst.PsstError) as e:
        psst.network_create(big, storage=psst.STORAGE_SPARSE)
    assert e.value.status == psst.ERR_UNSUPPORTED
    # the adjoint does not take sparse storage
    net = psst.network_create(inst.net, storage=psst.STORAGE_SPARSE)
    batch = psst.batch_create([net])
    dev = torch.device("cuda:0")
    ck = torch.zeros((1, 14 * inst.net.n), dtype=torch.float32, device=dev)
    dl = torch.zeros((10, inst.net.n), dtype=torch.float32, device=dev)
    g = torch.zeros(max(net.grad_size, 1), dtype=torch.float32, device=dev)
    a = torch.zeros(inst.net.n, dtype=torch.float32, device=dev)
    with pytest.raises(psst.PsstError) as e:
        psst.adjoint(batch, ck, 10, None, 0.01, 10, 0, dl, g, a, a.clone(), a.clone(),
                     per_instance=True)
    assert e.value.status == psst.ERR_UNSUPPORTED
