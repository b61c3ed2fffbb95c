"""Test helpers: run workload instances through the HIP library and the oracle
on identical inputs and return numpy results.  The GPU side goes through the
C ABI binding only; the oracle side through the oracle package only."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1906_03958_amd import psst


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def gpu_run(insts, n_steps, dt=0.01, rec_stride=1, spike_cap=0, batched=True,
            chunks=None, nets=None, state=None, return_state=False, tableau=None):
    """Integrate instances on the GPU.  batched=True: one psst_batch of all
    instances; False: one psst_integrate per instance.  chunks: list of step
    counts summing to n_steps (resumed calls).  Returns dict with v [rows, NT],
    spike_count [NT], spike_t [NT, cap], state [7, 2, NT], offsets."""
    torch, dev = torch_dev()
    if nets is None:
        nets = [psst.network_create(i.net) for i in insts]
        if tableau is not None:
            for h in nets:
                psst.network_set_tableau(h, tableau)
    sizes = np.array([i.net.n for i in insts])
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    nt = int(offs[-1])
    v0 = torch.from_numpy(np.concatenate([i.v0 for i in insts])).to(dev)
    stim = psst.pack_stimulus([i.stim for i in insts], dev)
    rows = n_steps // rec_stride if rec_stride else 0
    vout = torch.zeros((max(rows, 1), nt), dtype=torch.float32, device=dev)
    cnt = torch.zeros(nt, dtype=torch.int32, device=dev)
    spk = torch.zeros((nt, max(spike_cap, 1)), dtype=torch.float32, device=dev)
    chunks = chunks or [n_steps]
    assert sum(chunks) == n_steps
    if batched:
        batch = psst.batch_create(nets)
        assert batch.n_total == nt
        st = torch.zeros(14 * nt, dtype=torch.float32, device=dev) if state is None else state
        if state is None:
            psst.batch_state_init(batch, v0, st)
        s0 = 0
        for c in chunks:
            row0 = s0 // rec_stride if rec_stride else 0
            rec = psst.DeviceRecord(vout[row0:] if rec_stride else None, rec_stride,
                                    rows - row0, cnt, spk, spike_cap)
            psst.integrate_batch(batch, st, stim, dt, c, s0, rec)
            s0 += c
        psst.batch_poll(batch)
        torch.cuda.synchronize()
        stv = st.view(7, 2, nt).cpu().numpy()
    else:
        stv = np.zeros((7, 2, nt), np.float32)
        for k, (inst, net) in enumerate(zip(insts, nets)):
            a, b = offs[k], offs[k + 1]
            n = b - a
            st = torch.zeros(14 * n, dtype=torch.float32, device=dev)
            psst.state_init(net, v0[a:b].contiguous(), st)
            s1 = psst.pack_stimulus([inst.stim], dev)
            vloc = torch.zeros((max(rows, 1), n), dtype=torch.float32, device=dev)
            cl = torch.zeros(n, dtype=torch.int32, device=dev)
            sl = torch.zeros((n, max(spike_cap, 1)), dtype=torch.float32, device=dev)
            s0 = 0
            for c in chunks:
                row0 = s0 // rec_stride if rec_stride else 0
                rec = psst.DeviceRecord(vloc[row0:] if rec_stride else None, rec_stride,
                                        rows - row0, cl, sl, spike_cap)
                psst.integrate(net, st, s1, dt, c, s0, rec)
                s0 += c
            psst.network_poll(net)
            vout[:, a:b] = vloc
            cnt[a:b] = cl
            spk[a:b] = sl
            stv[:, :, a:b] = st.view(7, 2, n).cpu().numpy()
    torch.cuda.synchronize()
    out = dict(v=vout[:rows].cpu().numpy(), spike_count=cnt.cpu().numpy(),
               spike_t=spk[:, :spike_cap].cpu().numpy(), state=stv, offsets=offs)
    return out


# The library takes the step as float32 (dt_ms in the C ABI); the oracle is
# handed that same value, so both integrate the same discrete map.
DT = float(np.float32(0.01))


def step_f32(dt):
    return float(np.float32(dt))


def oracle_run(insts, n_steps, dt=0.01, rec_stride=1, spike_cap=0, threads=None, tableau=None):
    res = oracle.run_many(insts, n_steps, dt=step_f32(dt), rec_stride=rec_stride, spike_cap=spike_cap,
                          threads=threads, tableau=tableau)
    v = np.concatenate([r[0]["v"] for r in res], axis=1) if rec_stride else None
    cnt = np.concatenate([r[0]["spike_count"] for r in res])
    spk = np.concatenate([r[0]["spike_t"] for r in res], axis=0)
    y = np.concatenate([r[1] for r in res], axis=1)
    return dict(v=v, spike_count=cnt, spike_t=spk, state=y)


def state_value(stv):
    """float64 value of a [7, 2, NT] float32 pair state."""
    return stv[:, 0, :].astype(np.float64) + stv[:, 1, :].astype(np.float64)


def spike_match(gc, gt, oc, ot, t_max, tol=0.05):
    """Spikes before t_max: equal counts per neuron, paired in order, max |dt|.
    Returns (n_count_mismatch, max_abs_dt, n_spikes)."""
    bad, worst, total = 0, 0.0, 0
    for i in range(len(gc)):
        a = gt[i, :gc[i]]
        b = ot[i, :oc[i]]
        a = a[a < t_max]
        b = b[b < t_max]
        if len(a) != len(b):
            bad += 1
            continue
        total += len(a)
        if len(a):
            worst = max(worst, float(np.abs(a.astype(np.float64) - b).max()))
    return bad, worst, total

