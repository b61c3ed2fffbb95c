"""Conditioning floor of the FP64 oracle (test infrastructure; oracle and
input generators only)."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_1906_03958_amd import workloads as W


def conditioning_floor(inst, n_steps, dt=0.01):
    """Per-neuron conditioning floor of the FP64 oracle: for each neuron i,
    max over the run of |V_i(perturbed) - V_i(reference)| when neuron i's own
    inputs (V0_i and its constant current) move up by one float32 ulp.  The
    float32 inputs of the GPU path are exact, but a discrepancy of this size
    in neuron i is indistinguishable from a one-ulp change of its inputs.
    The step is taken as the float32 value the library integrates with."""
    dt = float(np.float32(dt))
    ref = oracle.run(inst, n_steps, dt, rec_stride=1)[0]["v"]
    insts = []
    for i in range(inst.net.n):
        v0 = inst.v0.copy()
        v0[i] = np.nextafter(v0[i], np.float32(np.inf))
        cur = inst.stim.i_const_nA.copy()
        cur[i] = np.nextafter(cur[i], np.float32(np.inf))
        insts.append(W.Instance(inst.net, v0, dataclasses.replace(inst.stim, i_const_nA=cur)))
    res = oracle.run_many(insts, n_steps, dt=dt, rec_stride=1)
    return np.array([np.abs(res[i][0]["v"][:, i] - ref[:, i]).max() for i in range(inst.net.n)])
