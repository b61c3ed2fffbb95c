"""GPU parity of the forward RK4 path against the FP64 oracle (calls go
through the C ABI).  Tolerances are the stated ones: max |dV| <= 1e-3 mV over
the first 50 ms, spike times within 0.05 ms over 200 ms, population firing
rates within 2 % for long chaotic runs; bitwise identity for chunking, batch
composition and order."""
import sys

import numpy as np
import pytest

from paper_1906_03958_amd import workloads as W
from tests import _runs as R
from tests._floor import conditioning_floor

pytestmark = pytest.mark.gpu

DV_TOL = 1e-3        # mV, first 50 ms
SPIKE_TOL = 0.05     # ms, first 200 ms
RATE_TOL = 0.02      # relative, population rates


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_03958_amd import psst
    assert psst.device_count() >= 1


def test_state_init_matches_oracle():
    import oracle
    inst = W.config1(0)
    g = R.gpu_run([inst], 0, rec_stride=0)
    y = R.state_value(g["state"])
    yo = oracle.init_state(inst.net, inst.v0)
    np.testing.assert_allclose(y, yo, rtol=0, atol=1e-13)


def test_steady_state_gates_over_a_voltage_grid():
    """The rate functions through the initial state x_inf(V0) = a / (a + b)
    on a dense grid of V0 over [-150, 100] mV plus the removable
    singularities of a_m (-40 mV) and a_n (-55 mV), exactly and a little off
    them on both sides of where the kernels switch from the series of
    u / (1 - e^-u) to the quotient: every gate within 1e-13 of the oracle."""
    import oracle
    grid = np.arange(-150.0, 100.0 + 1e-9, 1.25)
    sing = []
    for vs in (-40.0, -55.0):
        for d in (0.0, 1e-6, 1e-3, 0.1, 0.49, 0.5, 0.51, 1.0):
            sing += [vs - d, vs + d]
    v0 = np.unique(np.concatenate([grid, sing])).astype(np.float32)
    inst = W.uncoupled(np.zeros(len(v0)), v0)
    g = R.gpu_run([inst], 0, rec_stride=0)
    y = R.state_value(g["state"])
    yo = oracle.init_state(inst.net, inst.v0)
    err = np.abs(y[1:4] - yo[1:4]).max()
    _say(f"  {len(v0)} voltages: max |x_inf gpu - oracle| = {err:.2e}")
    assert err <= 1e-13


def test_config1_parity_50ms_and_spikes_100ms():
    for seed in (0, 1):
        inst = W.config1(seed)
        _say("config1 seed", seed)
        g = R.gpu_run([inst], W.CONFIG1_STEPS, rec_stride=1, spike_cap=64, batched=False)
        o = R.oracle_run([inst], W.CONFIG1_STEPS, rec_stride=1, spike_cap=64)
        dv = np.abs(g["v"][:5000] - o["v"][:5000]).max()
        _say("  max|dV| 0-50 ms", dv)
        # reported beside the gate: each neuron's error against the oracle's
        # own change under one float32 ulp of that neuron's inputs, plus the
        # half ulp lost in recording V as float32
        floor = conditioning_floor(inst, 5000)
        dvi = np.abs(g["v"][:5000] - o["v"][:5000]).max(axis=0)
        half = 0.5 * np.spacing(np.abs(o["v"][:5000]).astype(np.float32)).max(axis=0)
        _say(f"  per neuron: max|dV| / (floor + half ulp) {np.max(dvi / (floor + half)):.2f}, "
             f"neurons above {int((dvi > floor + half).sum())} of {len(floor)}, "
             f"floor median {np.median(floor):.2e} max {floor.max():.2e}")
        assert dv <= DV_TOL
        bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                          o["spike_t"], 100.0)
        _say("  spikes", total, "count mismatches", bad, "max|dt|", worst)
        assert bad == 0 and worst <= SPIKE_TOL and total > 0


def test_config2_parity():
    inst = W.config2(0)
    n = 20_000                         # 200 ms
    _say("config2 200 ms")
    g = R.gpu_run([inst], n, rec_stride=1, spike_cap=256, batched=False)
    o = R.oracle_run([inst], n, rec_stride=1, spike_cap=256)
    dv = np.abs(g["v"][:5000] - o["v"][:5000]).max()
    _say("  max|dV| 0-50 ms", dv)
    assert dv <= DV_TOL
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], 200.0)
    _say("  spikes", total, "mismatch", bad, "max|dt|", worst)
    assert total > 0 and bad == 0 and worst <= SPIKE_TOL
    # slow-GABA variables follow too
    y = R.state_value(g["state"])
    assert np.abs(y[5:7, 90:] - o["state"][5:7, 90:]).max() < 1e-6


@pytest.mark.parametrize("which", ["pn", "ln"])
def test_config2_full_second_rates(which):
    if which == "ln":
        pytest.skip("rates checked for both populations in the 'pn' case")
    inst = W.config2(0)
    n = W.CONFIG2_STEPS                 # 1 s
    _say("config2 1 s")
    g = R.gpu_run([inst], n, rec_stride=0, spike_cap=1, batched=False)
    o = R.oracle_run([inst], n, rec_stride=0, spike_cap=1)
    for name, sl in (("PN", slice(0, 90)), ("LN", slice(90, 120))):
        rg = g["spike_count"][sl].mean()
        ro = o["spike_count"][sl].mean()
        _say(f"  {name} mean spikes/neuron gpu {rg:.3f} oracle {ro:.3f}")
        assert ro > 0 and abs(rg - ro) <= RATE_TOL * ro


def test_chunked_equals_unchunked_bitwise():
    insts = [W.config2(0, t_ms=30.0), W.config3_instance(7)]
    a = R.gpu_run(insts, 3000, rec_stride=7, spike_cap=16)
    b = R.gpu_run(insts, 3000, rec_stride=7, spike_cap=16, chunks=[1000, 333, 1667])
    np.testing.assert_array_equal(a["state"], b["state"])
    np.testing.assert_array_equal(a["v"], b["v"])
    np.testing.assert_array_equal(a["spike_count"], b["spike_count"])
    np.testing.assert_array_equal(a["spike_t"], b["spike_t"])


def _c3_sample(k):
    # instances spread over the size range (ranked by size)
    sizes = np.array([W.config3_size(b) for b in range(256)])
    order = np.argsort(sizes, kind="stable")
    pick = order[np.linspace(0, 255, k).astype(int)]
    return [int(b) for b in pick]


def test_batch_equals_plain_and_is_order_invariant_bitwise():
    ids = _c3_sample(10)
    insts = [W.config3_instance(b) for b in ids]
    _say("sizes", [i.net.n for i in insts])
    a = R.gpu_run(insts, 400, rec_stride=1, spike_cap=8, batched=True)
    p = R.gpu_run(insts, 400, rec_stride=1, spike_cap=8, batched=False)
    np.testing.assert_array_equal(a["state"], p["state"])
    np.testing.assert_array_equal(a["v"], p["v"])
    perm = np.random.default_rng(0).permutation(len(insts))
    c = R.gpu_run([insts[k] for k in perm], 400, rec_stride=1, spike_cap=8, batched=True)
    for new, old in enumerate(perm):
        a0, a1 = a["offsets"][old], a["offsets"][old + 1]
        c0, c1 = c["offsets"][new], c["offsets"][new + 1]
        np.testing.assert_array_equal(a["state"][:, :, a0:a1], c["state"][:, :, c0:c1])
        np.testing.assert_array_equal(a["v"][:, a0:a1], c["v"][:, c0:c1])


def test_lds_resident_equals_streamed_bitwise(monkeypatch):
    # small instances keep their whole conductance matrix in LDS and form
    # the chunk partials one row per thread; with PSST_LDS_G=0 every matrix
    # streams from global memory through the four-rows-per-thread form.  The
    # summation order is the same, so the trajectories agree bit for bit
    # (the slow-GABA network covers the second matrix).
    ids = _c3_sample(8)
    insts = [W.config3_instance(b) for b in ids] + [W.config2(0, t_ms=10.0)]
    _say("sizes", [i.net.n for i in insts])
    for batched in (True, False):
        monkeypatch.delenv("PSST_LDS_G", raising=False)
        a = R.gpu_run(insts, 300, rec_stride=1, spike_cap=8, batched=batched)
        monkeypatch.setenv("PSST_LDS_G", "0")
        b = R.gpu_run(insts, 300, rec_stride=1, spike_cap=8, batched=batched)
        np.testing.assert_array_equal(a["state"], b["state"])
        np.testing.assert_array_equal(a["v"], b["v"])
        np.testing.assert_array_equal(a["spike_t"], b["spike_t"])
    monkeypatch.delenv("PSST_LDS_G", raising=False)


def test_config3_sampled_parity():
    ids = _c3_sample(12)
    insts = [W.config3_instance(b) for b in ids]
    n = 5000                            # 50 ms
    _say("config3 sample sizes", [i.net.n for i in insts])
    g = R.gpu_run(insts, n, rec_stride=10, spike_cap=32)
    o = R.oracle_run(insts, n, rec_stride=10, spike_cap=32)
    dv = np.abs(g["v"] - o["v"]).max(axis=0)
    _say("  max|dV|", dv.max(), "neurons over tol", int((dv > DV_TOL).sum()), "of", len(dv))
    assert dv.max() <= DV_TOL
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], 50.0)
    assert bad == 0 and worst <= SPIKE_TOL


def _thresholds():
    """Oracle single-spike threshold and repetitive-firing onset (nA) on a
    fine current grid, 500 ms steps from rest."""
    import oracle
    grid1 = np.linspace(0.220, 0.225, 41)
    grid2 = np.linspace(0.625, 0.630, 41)
    I = np.concatenate([grid1, grid2])
    res, _ = oracle.run(W.uncoupled(I, np.full(len(I), -65.0)), 50_000, dt=R.DT,
                        rec_stride=0, spike_cap=128)
    c = res["spike_count"]
    late = np.array([(res["spike_t"][k, :c[k]] > 250.0).sum() for k in range(len(I))])
    t1 = grid1[np.argmax(c[:41] > 0)]
    t2 = grid2[np.argmax(late[41:] >= 2)]
    return float(t1), float(t2)


def test_uncoupled_rest_rheobase_and_gate_bounds():
    t1, t2 = _thresholds()
    _say("oracle thresholds (nA)", t1, t2)
    I = np.array([0.0, t1 * 0.995, t1 * 1.005, t2 * 0.995, t2 * 1.005, 1.0])
    inst = W.uncoupled(I, np.full(len(I), -65.0))
    g = R.gpu_run([inst], 50_000, rec_stride=100, spike_cap=128, batched=False)
    o = R.oracle_run([inst], 50_000, rec_stride=100, spike_cap=128)
    np.testing.assert_array_equal(g["spike_count"], o["spike_count"])
    late_g = [(g["spike_t"][k, :g["spike_count"][k]] > 250).sum() for k in range(len(I))]
    late_o = [(o["spike_t"][k, :o["spike_count"][k]] > 250).sum() for k in range(len(I))]
    assert late_g == late_o
    assert o["spike_count"][1] == 0 and o["spike_count"][2] >= 1
    assert late_o[3] < 2 and late_o[4] >= 2
    assert abs(g["v"][-1, 0] - o["v"][-1, 0]) < 1e-3        # resting potential
    y = R.state_value(g["state"])
    assert y[1:4].min() >= -1e-6 and y[1:4].max() <= 1 + 1e-6


@pytest.mark.parametrize("batched", [False, True], ids=["plain", "batched"])
def test_compensated_state_against_closed_form(batched):
    """The float32 (value, compensation) state over many tiny steps.
    Passive membranes (g_Na = g_K = 0, no synapses) obey a linear ODE, so RK4
    gives V_n = V_inf + R(z)^n (V0 - V_inf) exactly, R(z) = 1 + z + z^2/2 +
    z^3/6 + z^4/24, z = -g_L dt / C.  At dt = 5e-5 ms each step changes V by
    a few hundred float32 ulps at most, so a float32 state without its
    compensation word drifts by far more than the gate over 200000 steps
    (shown below on the CPU); the pair must stay within 1e-7 mV."""
    I = np.array([0.0, 0.5, 1.5, 3.0])
    v0 = np.array([-70.0, -80.0, -65.0, -40.0])
    inst = W.uncoupled(I, v0, params=dict(g_Na=0.0, g_K=0.0, g_L=0.3))
    n_steps, stride, dt = 200_000, 1000, 5e-5
    g = R.gpu_run([inst], n_steps, dt=dt, rec_stride=stride, batched=batched)
    p = {k: np.asarray(v, np.float64) for k, v in inst.net.params.items()}
    ci = 1e-3 / float(np.float32(W.AREA_CM2))
    dt32 = float(np.float32(dt))             # the library takes dt as float32
    z = -p["g_L"] * dt32 / p["C_m"]
    Rz = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    vinf = p["E_L"] + ci * inst.stim.i_const_nA.astype(np.float64) / p["g_L"]
    x0 = inst.v0.astype(np.float64)
    n = np.arange(stride, n_steps + 1, stride)[:, None]
    expect = vinf + Rz ** n * (x0 - vinf)
    v_end = R.state_value(g["state"])[0]
    err_pair = float(np.abs(v_end - expect[-1]).max())
    rec = g["v"].astype(np.float64)
    ulp = np.spacing(np.abs(expect).astype(np.float32)).astype(np.float64)
    err_rec = float((np.abs(rec - expect) / ulp).max())
    # the same recursion with a plain float32 state: the increment is formed
    # exactly in float64, then the sum is rounded to float32 every step
    v32 = inst.v0.astype(np.float32)
    rm1 = Rz - 1
    for _ in range(n_steps):
        v32 = (v32.astype(np.float64) + rm1 * (v32.astype(np.float64) - vinf)).astype(np.float32)
    err_f32 = float(np.abs(v32.astype(np.float64) - expect[-1]).max())
    _say(f"  {'batched' if batched else 'plain'}: |V - closed form| at 10 ms: pair "
         f"{err_pair:.2e} mV, recorded rows {err_rec:.2f} ulp; float32 state without "
         f"compensation {err_f32:.2e} mV")
    assert err_pair <= 1e-7
    assert err_rec <= 0.55                      # the recorded float32 is the rounded pair
    assert err_f32 > 1e3 * 1e-7                 # the gate would catch a dropped compensation


@pytest.mark.parametrize("batched", [False, True], ids=["plain", "batched"])
def test_spike_time_on_a_passive_crossing(batched):
    """Spike detection against a closed form: a passive membrane driven to
    V_inf > 0 crosses 0 mV once, between V_n = V_inf + R(z)^n (V0 - V_inf)
    and V_{n+1}; the spike time is (n + (0 - V_n) / (V_{n+1} - V_n)) dt, stored
    as float32.  A neuron settling below 0 mV records none."""
    I = np.array([3.0, 1.0])
    inst = W.uncoupled(I, np.full(2, -65.0), params=dict(g_Na=0.0, g_K=0.0, g_L=0.3))
    N = 600
    g = R.gpu_run([inst], N, rec_stride=0, spike_cap=4, batched=batched)
    p = {k: np.asarray(v, np.float64) for k, v in inst.net.params.items()}
    ci = 1e-3 / float(np.float32(W.AREA_CM2))
    dt = R.DT
    z = -p["g_L"][0] * dt / p["C_m"][0]
    vinf = p["E_L"][0] + ci * float(np.float32(I[0])) / p["g_L"][0]
    v = vinf + (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** np.arange(N + 1) * (-65.0 - vinf)
    n = int(np.argmax(v >= 0.0)) - 1
    t = (n + (0.0 - v[n]) / (v[n + 1] - v[n])) * dt
    _say(f"  spike at {g['spike_t'][0, 0]:.7f} ms, closed form {t:.7f} ms")
    assert list(g["spike_count"]) == [1, 0]
    assert abs(float(g["spike_t"][0, 0]) - t) <= 0.5 * np.spacing(np.float32(t)) + 1e-9


def test_edge_cases():
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    inst = W.single_neuron(0.5)
    net = psst.network_create(inst.net)
    st = torch.zeros(14, dtype=torch.float32, device=dev)
    psst.state_init(net, torch.from_numpy(inst.v0).to(dev), st)
    before = st.clone()
    psst.integrate(net, st, None, 0.01, 0)          # n_steps = 0: no-op
    torch.cuda.synchronize()
    assert torch.equal(st, before)
    with pytest.raises(psst.PsstError) as e:
        psst.integrate(net, st, None, -0.01, 10)
    assert e.value.status == psst.ERR_INVALID_ARGUMENT
    # a blow-up is reported, not hidden: dt = 5 ms is far beyond stability
    psst.integrate(net, st, psst.pack_stimulus([inst.stim], dev), 5.0, 200)
    with pytest.raises(psst.PsstError) as e:
        psst.network_poll(net)
    assert e.value.status == psst.ERR_NONFINITE
    psst.network_poll(net)                           # flag was cleared


def test_ragged_extremes_parity_and_batch_equals_plain():
    """Sizes at the kernels' boundaries in one ragged batch: a lone neuron
    (no synapses), 63/64/65 and 127/129 neurons around the 64-column chunk
    edges, 202/203 around the whole-matrix-in-LDS limit, and 1024, the
    largest network of the per-instance kernel (mostly streamed).  Oracle
    parity over 3 ms (max |dV| <= 1e-3 mV) and batch = plain bit for bit."""
    sizes = [(1, 0), (48, 15), (48, 16), (49, 16), (96, 31), (97, 32), (152, 50), (152, 51),
             (768, 256)]
    insts = [W.sized_instance(k, a, b) for k, (a, b) in enumerate(sizes)]
    n = 300
    _say(f"ragged extremes: sizes {[i.net.n for i in insts]}, {n} steps")
    g = R.gpu_run(insts, n, rec_stride=1, spike_cap=8)
    p = R.gpu_run(insts, n, rec_stride=1, spike_cap=8, batched=False)
    np.testing.assert_array_equal(g["state"], p["state"])
    np.testing.assert_array_equal(g["v"], p["v"])
    o = R.oracle_run(insts, n, rec_stride=1, spike_cap=8)
    offs = np.concatenate([[0], np.cumsum([i.net.n for i in insts])])
    for k, inst in enumerate(insts):
        a, b = offs[k], offs[k + 1]
        dv = np.abs(g["v"][:, a:b].astype(np.float64) - o["v"][:, a:b]).max()
        _say(f"  n={inst.net.n}: max|dV| {dv:.2e} mV")
        assert dv <= 1e-3, (inst.net.n, dv)
    bad, worst, total = R.spike_match(g["spike_count"], g["spike_t"], o["spike_count"],
                                      o["spike_t"], 3.0)
    assert bad == 0 and worst <= 0.05, (bad, worst, total)


def test_config3_full_batch_sampled_parity():
    """The whole 4096-network batch in the launch configuration the benchmark
    times (one batch, tuned launch shape, records on the device): 50 ms with V
    every 25 steps and spikes, then 32 instances stratified by size against the
    oracle, each run on its own: max |dV| <= 1e-3 mV, spikes matched."""
    insts = W.config3(4096)
    n = 5000
    _say("config3 full batch: 4096 networks,", sum(i.net.n for i in insts), "neurons,", n, "steps")
    g = R.gpu_run(insts, n, rec_stride=25, spike_cap=16)
    sizes = np.array([i.net.n for i in insts])
    order = np.argsort(sizes, kind="stable")
    pick = [int(b) for b in order[np.linspace(0, len(sizes) - 1, 32).astype(int)]]
    o = R.oracle_run([insts[b] for b in pick], n, rec_stride=25, spike_cap=16)
    offs = g["offsets"]
    cols = np.concatenate([np.arange(offs[b], offs[b + 1]) for b in pick])
    dv = np.abs(g["v"][:, cols].astype(np.float64) - o["v"]).max()
    _say(f"  sampled instances {sorted(sizes[pick].tolist())[:3]}...: max|dV| {dv:.2e} mV")
    assert dv <= DV_TOL
    bad, worst, total = R.spike_match(g["spike_count"][cols], g["spike_t"][cols],
                                      o["spike_count"], o["spike_t"], 50.0)
    _say(f"  spikes {total}, count mismatches {bad}, worst dt {worst:.2e} ms")
    assert bad == 0 and worst <= SPIKE_TOL


def test_config3_full_horizon_rates():
    """The batched workload's whole horizon, 500 ms (50,000 steps), for all
    4096 networks in one batch; the runs are chaotic, so the comparison is the
    population firing rate (PN and LN pooled over 16 instances stratified by
    size) against the oracle, within 2 %."""
    insts = W.config3(4096)
    n = 50_000
    _say("config3 full horizon: 4096 networks, 500 ms")
    g = R.gpu_run(insts, n, rec_stride=0, spike_cap=1)
    sizes = np.array([i.net.n for i in insts])
    order = np.argsort(sizes, kind="stable")
    pick = [int(b) for b in order[np.linspace(0, len(sizes) - 1, 16).astype(int)]]
    o = R.oracle_run([insts[b] for b in pick], n, rec_stride=0, spike_cap=1)
    offs = g["offsets"]
    gp = gl = op = ol = 0.0
    npn = nln = 0
    k = 0
    for b in pick:
        net = insts[b].net
        c = g["spike_count"][offs[b]:offs[b + 1]]
        oc = o["spike_count"][k:k + net.n]
        gp += c[:net.n_pn].sum(); op += oc[:net.n_pn].sum(); npn += net.n_pn
        gl += c[net.n_pn:].sum(); ol += oc[net.n_pn:].sum(); nln += net.n - net.n_pn
        k += net.n
    for name, a, r, m in (("PN", gp, op, npn), ("LN", gl, ol, nln)):
        _say(f"  {name}: {a / m / 0.5:.2f} Hz on the GPU, {r / m / 0.5:.2f} Hz in the oracle")
        assert r > 0 and abs(a - r) <= RATE_TOL * r


def test_readme_example_runs():
    """The README's minimal-use snippet, executed as written, integrates the
    20-neuron network within the forward gate of the oracle."""
    import os
    import oracle
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "README.md")).read()
    lines = []
    for line in text.split("## Minimal use from Python", 1)[1].splitlines()[1:]:
        if line.strip() and not line.startswith("    "):
            break                                   # end of the indented block
        lines.append(line[4:])
    code = "\n".join(lines)
    assert "integrate_batch" in code
    ns = {}
    exec(compile(code, "README.md", "exec"), ns)
    v = ns["v"].cpu().numpy()
    ref, _ = oracle.run(ns["inst"], 1000, dt=R.DT)
    dv = float(np.abs(v - ref["v"]).max())
    _say(f"  README example: max|dV| vs oracle {dv:.2e} mV")
    assert dv <= DV_TOL


def test_batch_reports_a_blow_up():
    """A batch driven far beyond stability (dt = 5 ms) reports non-finite
    states through psst_batch_poll, which then clears the flag."""
    import torch
    from paper_1906_03958_amd import psst
    dev = torch.device("cuda:0")
    insts = [W.config3_instance(b) for b in (1, 2)]
    nets = [psst.network_create(i.net) for i in insts]
    batch = psst.batch_create(nets)
    st = torch.zeros(14 * batch.n_total, dtype=torch.float32, device=dev)
    psst.batch_state_init(batch, torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev),
                          st)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    psst.integrate_batch(batch, st, stim, 5.0, 200, 0)
    with pytest.raises(psst.PsstError) as e:
        psst.batch_poll(batch)
    assert e.value.status == psst.ERR_NONFINITE
    psst.batch_poll(batch)                           # flag was cleared
