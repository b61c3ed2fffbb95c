"""torch.autograd.Function over the C ABI: a batch of stimulus trials of one
network, its recorded membrane-potential traces as a differentiable function
of the synaptic conductances (per pathway block, nS) and the intrinsic
conductances g_Na, g_K, g_L (mS/cm^2).

forward  -> psst_integrate_batch with checkpoints every K steps, V every step
backward -> psst_adjoint (discrete adjoint of the RK4 map, or of the explicit
            method given as a tableau, summed over trials)

The network and its batch are created on the first call and kept: later
calls write the new conductances into them in place (psst_network_update).
A network whose values an autograd graph may still differentiate is not
overwritten; a call made while one is held takes another network (created
once, then reused alike).

All arithmetic happens in the HIP library; this module only marshals tensors.
"""
from __future__ import annotations

import copy
from typing import List

import numpy as np
import torch

from . import psst


class _Slot:
    """A network of the simulation's trials and its batch; held while an
    autograd context that read its values is alive."""

    def __init__(self, net, batch):
        self.net, self.batch, self.held = net, batch, False


class _Lease:
    """Holds a slot for the lifetime of the autograd context it is stored on."""

    def __init__(self, slot):
        self.slot = slot
        slot.held = True

    def __del__(self):
        self.slot.held = False


class TraceSimulation:
    """Trials of one network.  net: a workload Network (its g values are
    replaced by the tensors passed to __call__); i_nA, v0: [B, n] arrays."""

    def __init__(self, net, i_nA, v0, dt: float, n_steps: int, K: int = 100,
                 device: str = "cuda:0", tableau=None):
        self.template = net
        self.tableau = tableau          # explicit method (dict(a, b)); None: classical RK4
        self.dev = torch.device(device)
        self.B = int(i_nA.shape[0])
        self.n = int(net.n)
        self.dt = float(dt)
        self.n_steps = int(n_steps)
        self.K = int(K)
        self.shapes = [tuple(p.g_nS.shape) for p in net.pathways]
        self.stim = psst.DeviceStimulus(
            torch.from_numpy(np.ascontiguousarray(i_nA, np.float32).ravel()).to(self.dev))
        self.v0 = torch.from_numpy(np.ascontiguousarray(v0, np.float32).ravel()).to(self.dev)
        self._slots: List[_Slot] = []

    def pack(self, blocks: List) -> torch.Tensor:
        return torch.cat([torch.as_tensor(b, dtype=torch.float32).reshape(-1) for b in blocks])

    def build(self, g_flat: torch.Tensor, g_na, g_k, g_l):
        net = copy.copy(self.template)
        flat = g_flat.detach().to("cpu", torch.float32).numpy()
        paths, off = [], 0
        for p, (a, b) in zip(self.template.pathways, self.shapes):
            q = copy.copy(p)
            q.g_nS = flat[off:off + a * b].reshape(a, b).copy()
            off += a * b
            paths.append(q)
        net.pathways = paths
        net.params = dict(self.template.params)
        for k, t in (("g_Na", g_na), ("g_K", g_k), ("g_L", g_l)):
            net.params[k] = t.detach().to("cpu", torch.float32).numpy().copy()
        return net

    def _dev32(self, t) -> torch.Tensor:
        return t.detach().to(self.dev, torch.float32).contiguous()

    def acquire(self, g_flat, g_na, g_k, g_l) -> _Slot:
        """A network holding these values, and its batch: a free kept one with
        the values written in place, else a new one."""
        for slot in self._slots:
            if not slot.held:
                psst.network_update(slot.net, self._dev32(g_flat), self._dev32(g_na),
                                    self._dev32(g_k), self._dev32(g_l))
                return slot
        net = psst.network_create(self.build(g_flat, g_na, g_k, g_l))
        if self.tableau is not None:
            psst.network_set_tableau(net, self.tableau)
        slot = _Slot(net, psst.batch_create([net] * self.B))
        self._slots.append(slot)
        return slot

    def __call__(self, g_flat, g_na, g_k, g_l) -> torch.Tensor:
        return PsstTraceFn.apply(self, g_flat, g_na, g_k, g_l)


class PsstTraceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: TraceSimulation, g_flat, g_na, g_k, g_l):
        slot = sim.acquire(g_flat, g_na, g_k, g_l)
        net, batch = slot.net, slot.batch
        nt = batch.n_total
        states = torch.zeros(14 * nt, dtype=torch.float32, device=sim.dev)
        psst.batch_state_init(batch, sim.v0, states)
        v = torch.empty((sim.n_steps, nt), dtype=torch.float32, device=sim.dev)
        n_ck = (sim.n_steps + sim.K - 1) // sim.K
        ckpt = torch.empty((max(n_ck, 1), 14 * nt), dtype=torch.float32, device=sim.dev)
        psst.integrate_batch(batch, states, sim.stim, sim.dt, sim.n_steps, 0,
                             psst.DeviceRecord(v, 1, sim.n_steps), ckpt, sim.K)
        psst.batch_poll(batch)
        ctx.sim = sim
        ctx.net, ctx.batch, ctx.ckpt = net, batch, ckpt
        ctx.lease = _Lease(slot)
        ctx.devs = (g_flat.device, g_na.device, g_k.device, g_l.device)
        return v

    @staticmethod
    def backward(ctx, dLdV):
        sim, batch = ctx.sim, ctx.batch
        dLdV = dLdV.to(torch.float32).contiguous()
        gg = torch.empty(ctx.net.grad_size, dtype=torch.float32, device=sim.dev)
        gna = torch.empty(sim.n, dtype=torch.float32, device=sim.dev)
        gk = torch.empty_like(gna)
        gl = torch.empty_like(gna)
        psst.adjoint(batch, ctx.ckpt, sim.K, sim.stim, sim.dt, sim.n_steps, 0, dLdV, gg, gna,
                     gk, gl, per_instance=False)
        psst.batch_poll(batch)
        d = ctx.devs
        return None, gg.to(d[0]), gna.to(d[1]), gk.to(d[2]), gl.to(d[3])
