"""The seeded input generator: deterministic, float32 throughout, and the
recipe the benchmarks state (sizes, cell-type ratio, connection density,
value ranges)."""
import numpy as np

from paper_1906_03958_amd import workloads as W


def _arrays(inst):
    out = [inst.v0, inst.stim.i_const_nA]
    out += [np.asarray(v) for v in inst.net.params.values()]
    out += [p.g_nS for p in inst.net.pathways]
    return out


def test_seeded_and_float32():
    a, b = W.config3_instance(17), W.config3_instance(17)
    for x, y in zip(_arrays(a), _arrays(b)):
        assert x.dtype == np.float32
        np.testing.assert_array_equal(x, y)
    c = W.config3_instance(18)
    assert not np.array_equal(a.v0[:8], c.v0[:8])


def test_batched_workload_recipe():
    sizes = np.array([W.config3_size(b) for b in range(4096)])
    assert sizes.min() >= 60 and sizes.max() <= 480 and np.all(sizes % 4 == 0)
    assert abs(sizes.mean() - 270) < 5                      # E[N] of 4 U{15..120}
    assert abs((sizes.astype(np.float64) ** 2).mean() - 87_880) < 0.03 * 87_880
    inst = W.config3_instance(5)
    n = inst.net.n
    assert inst.net.n_pn == 3 * n // 4                      # PN:LN = 3:1
    assert inst.v0.min() >= -70 and inst.v0.max() <= -60
    i = inst.stim.i_const_nA
    assert i.min() >= 0 and i.max() <= 2
    masks = [np.asarray(p.mask) for p in inst.net.pathways]
    present = sum(int(m.sum()) for m in masks)
    pairs = n * (n - 1)
    assert abs(present / pairs - 0.5) < 0.05                # Bernoulli(0.5) over i != j
    for p in inst.net.pathways:                             # no autapses
        for r in range(p.post_end - p.post_begin):
            j = p.post_begin + r - p.pre_begin
            if 0 <= j < p.pre_end - p.pre_begin:
                assert p.mask[r, j] == 0
